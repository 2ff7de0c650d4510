"""CPU oracle for the colour-coding dynamic program -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never loads it.

It wraps ``oracle.c`` (plain C, written from the paper of Malik, Suchy and
Valla, arXiv 1908.11248) through ctypes:

* ``color_of``, ``color_array`` -- splitmix64 random colouring (Sec. 2.1)
* ``brute_count``      -- count of colourful mappings by backtracking (the
                          definition: Sec. 1 problem statement, colourful copy)
* ``brute_enum``       -- lexicographically first mappings (same definition)
* ``build_td``         -- exact-width nice tree decomposition (Sec. 3, Sec. 1.2)
* ``treewidth``        -- exact treewidth (Sec. 3)
* ``validate_td``      -- nice tree decomposition checker (Sec. 1.2)
* ``dp_count``         -- the DP over the nice TD with counts (Sec. 3.1)
* ``dp_count_range``   -- the same, for mappings with Phi(0) in a range
* ``dp_enumerate``     -- reconstruction R(x, M) (Sec. 4)
* ``vertex_sets``      -- distinct vertex sets of the mappings (Sec. 5.2)
* ``repetitions``, ``search`` -- the repetition driver (Sec. 2.1, Sec. 5.2)

Every function here is pinned by tests in ``tests/test_oracle_*.py`` against
brute force, closed forms and invariants (see the module docstrings there).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        lib.orc_splitmix64.restype = u64
        lib.orc_splitmix64.argtypes = [u64]
        lib.orc_color_of.restype = ctypes.c_int
        lib.orc_color_of.argtypes = [u64, i64, i64, i32]
        lib.orc_color_array.restype = None
        lib.orc_color_array.argtypes = [u64, i64, i32, i32, P]
        lib.orc_brute_count.restype = ctypes.c_int
        lib.orc_brute_count.argtypes = [i32, P, P, i32, i32, P, P, i32, P]
        lib.orc_brute_enum.restype = ctypes.c_int
        lib.orc_brute_enum.argtypes = [i32, P, P, i32, i32, P, P, u64, P, P]
        lib.orc_build_td.restype = ctypes.c_int
        lib.orc_build_td.argtypes = [i32, i32, P, P, i32, P, P]
        lib.orc_treewidth.restype = ctypes.c_int
        lib.orc_treewidth.argtypes = [i32, i32, P, P]
        lib.orc_validate_td.restype = ctypes.c_int
        lib.orc_validate_td.argtypes = [i32, i32, P, P, i32]
        lib.orc_count.restype = ctypes.c_int
        lib.orc_count.argtypes = [i32, P, P, i32, i32, P, i32, P, P, i32, i32, P, P, P, P]
        lib.orc_count_range.restype = ctypes.c_int
        lib.orc_count_range.argtypes = [i32, P, P, i32, i32, P, i32, P, P, i32, i32, i32, i32, P, P, P]
        lib.orc_enumerate.restype = ctypes.c_int
        lib.orc_enumerate.argtypes = [i32, P, P, i32, i32, P, i32, P, P, i32, i32, u64, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


def _graph(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    return int(g.n), rp, col


def _pattern(pat):
    nF = int(pat.n)
    e = np.ascontiguousarray(np.asarray(pat.edges, dtype=np.int32).reshape(-1, 2))
    if e.size == 0:
        e = np.zeros((1, 2), dtype=np.int32)
        return nF, 0, e
    return nF, int(e.shape[0]), e


def splitmix64(x: int) -> int:
    return int(_load().orc_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def color_of(seed: int, b: int, v: int, k: int) -> int:
    return int(_load().orc_color_of(seed & (2**64 - 1), b, v, k))


def color_array(seed: int, b: int, n: int, k: int) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=np.uint8)
    _load().orc_color_array(seed & (2**64 - 1), b, n, k, _p(out))
    return out[:n]


def brute_count(g, pat, colors, fix0: int = -1) -> int:
    n, rp, col = _graph(g)
    nF, mF, e = _pattern(pat)
    colors = np.ascontiguousarray(colors, dtype=np.uint8)
    out = np.zeros(1, dtype=np.uint64)
    _check(_load().orc_brute_count(n, _p(rp), _p(col), nF, mF, _p(e), _p(colors), fix0, _p(out)),
           "brute_count")
    return int(out[0])


def brute_enum(g, pat, colors, cap: int) -> np.ndarray:
    n, rp, col = _graph(g)
    nF, mF, e = _pattern(pat)
    colors = np.ascontiguousarray(colors, dtype=np.uint8)
    rows = np.empty((max(cap, 1), nF), dtype=np.int32)
    nr = np.zeros(1, dtype=np.uint64)
    _check(_load().orc_brute_enum(n, _p(rp), _p(col), nF, mF, _p(e), _p(colors), cap, _p(rows),
                                  _p(nr)), "brute_enum")
    return rows[: int(nr[0])].copy()


def build_td(pat):
    """Returns (td int32 array, width)."""
    nF, mF, e = _pattern(pat)
    cap = 1 + 5 * 4096
    td = np.zeros(cap, dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    w = np.zeros(1, dtype=np.int32)
    _check(_load().orc_build_td(nF, mF, _p(e), _p(td), cap, _p(ln), _p(w)), "build_td")
    return td[: int(ln[0])].copy(), int(w[0])


def treewidth(pat) -> int:
    nF, mF, e = _pattern(pat)
    w = np.zeros(1, dtype=np.int32)
    _check(_load().orc_treewidth(nF, mF, _p(e), _p(w)), "treewidth")
    return int(w[0])


def validate_td(pat, td) -> int:
    """0 when td is a valid nice tree decomposition of pat, else a rule code."""
    nF, mF, e = _pattern(pat)
    td = np.ascontiguousarray(td, dtype=np.int32)
    return int(_load().orc_validate_td(nF, mF, _p(e), _p(td), int(td.size)))


def _opts(degmask, distbound):
    return (1 if degmask else 0) | (0 if distbound else 2)


def dp_count(g, pat, k, colors, td=None, degmask=True, per_root_vertex=False, sizes=False, distbound=True):
    """Count of colourful mappings by the DP.  Returns a dict with 'count',
    'overflow' and optionally 'per_root_vertex' (np.uint64[n]) and 'sizes'.
    degmask / distbound switch the degree mask and the distance bound of
    Sec. 3.2 (both prune entries that cannot complete; counts are the same)."""
    n, rp, col = _graph(g)
    nF, mF, e = _pattern(pat)
    if td is None:
        td, _ = build_td(pat)
    td = np.ascontiguousarray(td, dtype=np.int32)
    colors = np.ascontiguousarray(colors, dtype=np.uint8)
    cnt = np.zeros(1, dtype=np.uint64)
    ovf = np.zeros(1, dtype=np.uint8)
    prv = np.zeros(max(n, 1), dtype=np.uint64) if per_root_vertex else None
    sz = np.zeros(int(td[0]), dtype=np.int64) if sizes else None
    rc = _load().orc_count(n, _p(rp), _p(col), nF, mF, _p(e), k, _p(colors), _p(td), int(td.size),
                           _opts(degmask, distbound), _p(cnt), _p(ovf),
                           _p(prv) if prv is not None else None,
                           _p(sz) if sz is not None else None)
    _check(rc, "dp_count")
    out = {"count": int(cnt[0]), "overflow": bool(ovf[0])}
    if prv is not None:
        out["per_root_vertex"] = prv[:n]
    if sz is not None:
        out["sizes"] = sz
    return out


def dp_count_range(g, pat, k, colors, lo, hi, td=None, degmask=True, sizes=False, distbound=True):
    """dp_count restricted to the mappings with Phi(0) in [lo, hi)."""
    n, rp, col = _graph(g)
    nF, mF, e = _pattern(pat)
    if td is None:
        td, _ = build_td(pat)
    td = np.ascontiguousarray(td, dtype=np.int32)
    colors = np.ascontiguousarray(colors, dtype=np.uint8)
    cnt = np.zeros(1, dtype=np.uint64)
    ovf = np.zeros(1, dtype=np.uint8)
    sz = np.zeros(int(td[0]), dtype=np.int64) if sizes else None
    rc = _load().orc_count_range(n, _p(rp), _p(col), nF, mF, _p(e), k, _p(colors), _p(td), int(td.size),
                                 _opts(degmask, distbound), int(lo), int(hi), _p(cnt), _p(ovf),
                                 _p(sz) if sz is not None else None)
    _check(rc, "dp_count_range")
    out = {"count": int(cnt[0]), "overflow": bool(ovf[0])}
    if sz is not None:
        out["sizes"] = sz
    return out


def dp_enumerate(g, pat, k, colors, cap, td=None, degmask=True, distbound=True):
    """(rows int32[min(total,cap), nF] lexicographically sorted, total)."""
    n, rp, col = _graph(g)
    nF, mF, e = _pattern(pat)
    if td is None:
        td, _ = build_td(pat)
    td = np.ascontiguousarray(td, dtype=np.int32)
    colors = np.ascontiguousarray(colors, dtype=np.uint8)
    # rows buffer bounded by the true total, found with a count first
    total = dp_count(g, pat, k, colors, td=td, degmask=degmask, distbound=distbound)["count"]
    m = min(total, cap)
    rows = np.empty((max(m, 1), nF), dtype=np.int32)
    nr = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.uint64)
    rc = _load().orc_enumerate(n, _p(rp), _p(col), nF, mF, _p(e), k, _p(colors), _p(td),
                               int(td.size), _opts(degmask, distbound), cap, _p(rows), _p(nr), _p(tot))
    _check(rc, "dp_enumerate")
    return rows[: int(nr[0])].copy(), int(tot[0])


def vertex_sets(g, pat, k, colors):
    """Distinct vertex sets of the colourful mappings (the paper's second
    counting mode, Sec. 5.2): sorted tuples, in lexicographic order."""
    rows, _ = dp_enumerate(g, pat, k, colors, 2**62)
    return sorted({tuple(sorted(int(x) for x in r)) for r in rows})


def repetitions(n_f, eps):
    """Colourings the randomised algorithm runs for error bound eps (Sec. 2.1):
    each run reveals a fixed occurrence with probability at least e^{-n_F},
    so ceil(e^{n_F} ln(1/eps)) runs miss it with probability at most eps."""
    import math

    return int(math.ceil(math.exp(n_f) * math.log(1.0 / eps)))


def search(g, pat, eps, seed, max_solutions, distinct_sets=False):
    """The repetition driver step by step: colourings b = 0, 1, ... of the
    seed (k = n_F colours) until repetitions(n_F, eps) are done or at least
    max_solutions distinct solutions are known; each colouring adds its first
    max_solutions mappings (or their sorted vertex sets).  Returns (the
    lexicographically first min(found, max_solutions) solutions, colourings
    run)."""
    k = pat.n
    planned = repetitions(pat.n, eps)
    found = set()
    run = 0
    while run < planned and len(found) < max_solutions:
        col = color_array(seed, run, g.n, k)
        run += 1
        rows, _ = dp_enumerate(g, pat, k, col, max_solutions)
        for r in rows:
            t = tuple(int(x) for x in r)
            found.add(tuple(sorted(t)) if distinct_sets else t)
    return sorted(found)[:max_solutions], run
