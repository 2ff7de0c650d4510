"""Python binding of libccgpu (the colour-coding DP on MI355X / gfx950).

Argument marshalling only: every step of the DP runs in the HIP library
behind the C ABI of ``include/ccgpu.h``.  The functions carry the ABI's names
without the ``cc_`` prefix.  Importing this module does not load the library;
the first call does, and it raises ``LibraryMissing`` when ``libccgpu.so``
has not been built (``python -m paper_1908_11248_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccgpu.so")

CC_OK = 0
CC_EINVAL = -1
CC_ERANGE = -2
CC_ENOMEM = -3
CC_EDEVICE = -4
CC_ECANCELLED = -5
CC_GRAPH_CANONICALIZE = 1
CC_NO_DEGREE_MASK = 1
CC_SPARSE_TABLES = 2
CC_CLASSIC_EXPAND = 4

# every symbol the header declares (checked by the CPU tests)
EXPORTS = [
    "cc_last_error", "cc_context_create", "cc_context_destroy", "cc_load_graph", "cc_graph_free",
    "cc_graph_num_vertices", "cc_color", "cc_color_explicit", "cc_coloring_download", "cc_coloring_free",
    "cc_build_decomposition", "cc_decomp_export", "cc_decomp_import", "cc_decomp_width", "cc_decomp_free",
    "cc_count", "cc_count_by_vertex", "cc_enumerate", "cc_last_table_sizes", "cc_count_batch",
    "cc_profile_enable", "cc_profile_filter", "cc_profile_read", "cc_decomp_describe",
    "cc_set_batch_lanes", "cc_tune_batch", "cc_set_table_budget",
    "cc_server_start", "cc_server_submit", "cc_server_poll", "cc_server_wait", "cc_server_stop",
    "cc_count_noalloc", "cc_count_range", "cc_last_chunk_count", "cc_estimate_memory", "cc_vertex_sets",
    "cc_search", "cc_plan_create", "cc_plan_count", "cc_plan_destroy", "cc_get_schedule", "cc_set_schedule",
]


class LibraryMissing(RuntimeError):
    pass


class CcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing("libccgpu.so is not built: run python -m paper_1908_11248_amd.build")
        # One HIP runtime per process: torch ships its own libamdhip64 (same
        # soname), which it loads by file name.  Loaded first, it also serves
        # this library; loaded second, a second runtime would start that sees
        # no devices.  So torch, when installed, is imported before the
        # library is opened.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I32, U32, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "cc_last_error": (ctypes.c_char_p, []),
            "cc_context_create": (ctypes.c_int, [ctypes.c_int, P, SZ, P, PP]),
            "cc_context_destroy": (ctypes.c_int, [P]),
            "cc_load_graph": (ctypes.c_int, [P, I32, P, P, U32, PP]),
            "cc_graph_free": (None, [P]),
            "cc_graph_num_vertices": (I32, [P]),
            "cc_color": (ctypes.c_int, [P, P, I32, U64, I32, PP]),
            "cc_color_explicit": (ctypes.c_int, [P, P, I32, I32, P, PP]),
            "cc_coloring_download": (ctypes.c_int, [P, I32, P]),
            "cc_coloring_free": (None, [P]),
            "cc_build_decomposition": (ctypes.c_int, [I32, I32, P, U32, PP]),
            "cc_decomp_export": (ctypes.c_int, [P, P, SZ, ctypes.POINTER(SZ)]),
            "cc_decomp_import": (ctypes.c_int, [I32, I32, P, P, SZ, PP]),
            "cc_decomp_width": (I32, [P]),
            "cc_decomp_free": (None, [P]),
            "cc_count": (ctypes.c_int, [P, P, P, P, U32, P, P]),
            "cc_count_noalloc": (ctypes.c_int, [P, P, P, P, U32, P, P]),
            "cc_count_range": (ctypes.c_int, [P, P, P, P, U32, I32, I32, P, P]),
            "cc_last_chunk_count": (I32, [P]),
            "cc_estimate_memory": (ctypes.c_int, [P, P, I32, I32, P, P]),
            "cc_vertex_sets": (ctypes.c_int, [P, P, P, I32, P, U64, P, P, P]),
            "cc_search": (ctypes.c_int, [P, P, P, P, P, P, P, P]),
            "cc_plan_create": (ctypes.c_int, [P, P, P, I32, I32, U32, PP]),
            "cc_plan_count": (ctypes.c_int, [P, U64, P, P]),
            "cc_plan_destroy": (ctypes.c_int, [P]),
            "cc_get_schedule": (ctypes.c_int, [P, P]),
            "cc_set_schedule": (ctypes.c_int, [P, P]),
            "cc_count_by_vertex": (ctypes.c_int, [P, P, P, I32, P, U32, P, P, P]),
            "cc_enumerate": (ctypes.c_int, [P, P, P, I32, P, U64, P, P, P]),
            "cc_last_table_sizes": (ctypes.c_int, [P, P, SZ, ctypes.POINTER(SZ)]),
            "cc_count_batch": (ctypes.c_int, [P, P, I32, P, U32, P, P]),
            "cc_profile_enable": (ctypes.c_int, [P, ctypes.c_int]),
            "cc_profile_filter": (ctypes.c_int, [P, ctypes.c_char_p, U32]),
            "cc_profile_read": (ctypes.c_int, [P, P, SZ, ctypes.POINTER(SZ)]),
            "cc_decomp_describe": (ctypes.c_int, [P, P, SZ, ctypes.POINTER(SZ)]),
            "cc_set_batch_lanes": (ctypes.c_int, [P, I32]),
            "cc_tune_batch": (ctypes.c_int, [P, P, I32, P, U32, P]),
            "cc_set_table_budget": (ctypes.c_int, [P, U64]),
            "cc_server_start": (ctypes.c_int, [P, P, P, PP]),
            "cc_server_submit": (ctypes.c_int, [P, P, I32, U64, I32, P]),
            "cc_server_poll": (ctypes.c_int, [P, U64, P, P, P]),
            "cc_server_wait": (ctypes.c_int, [P, U64, P, P, P]),
            "cc_server_stop": (ctypes.c_int, [P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != CC_OK:
        raise CcError(rc, lib().cc_last_error().decode())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Handle:
    _free = None

    def __init__(self, ptr):
        self.ptr = ptr

    def close(self):
        if self.ptr:
            getattr(lib(), self._free)(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph(_Handle):
    _free = "cc_graph_free"

    def __init__(self, ptr, ctx):
        super().__init__(ptr)
        self.ctx = ctx  # keep the context alive

    @property
    def n(self) -> int:
        return int(lib().cc_graph_num_vertices(self.ptr))


class Coloring(_Handle):
    _free = "cc_coloring_free"

    def __init__(self, ptr, ctx, k, num):
        super().__init__(ptr)
        self.ctx = ctx
        self.k = k
        self.num = num

    def download(self, b: int, n: int) -> np.ndarray:
        out = np.empty(max(n, 1), dtype=np.uint8)
        _check(lib().cc_coloring_download(self.ptr, b, _p(out)))
        return out[:n]


class Decomp(_Handle):
    _free = "cc_decomp_free"

    def __init__(self, ptr, n_F):
        super().__init__(ptr)
        self.n_F = n_F

    @property
    def width(self) -> int:
        return int(lib().cc_decomp_width(self.ptr))

    def describe(self) -> str:
        ln = ctypes.c_size_t(0)
        lib().cc_decomp_describe(self.ptr, None, 0, ctypes.byref(ln))
        buf = ctypes.create_string_buffer(ln.value)
        _check(lib().cc_decomp_describe(self.ptr, buf, ln.value, ctypes.byref(ln)))
        return buf.value.decode()

    def export(self) -> np.ndarray:
        ln = ctypes.c_size_t(0)
        rc = lib().cc_decomp_export(self.ptr, None, 0, ctypes.byref(ln))
        buf = np.zeros(ln.value, dtype=np.int32)
        _check(lib().cc_decomp_export(self.ptr, _p(buf), buf.size, ctypes.byref(ln)))
        return buf


class _Schedule(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("entry_factor", ctypes.c_int32), ("sort_above_k", ctypes.c_int32),
                ("group_min", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_double)]


def _stream_handle(stream):
    """A raw hipStream_t from None, an int, or an object with .cuda_stream
    (torch.cuda.Stream)."""
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream)) or None


class Context(_Handle):
    """A library context on one device.

    ``arena`` optionally supplies the DP arena as caller-owned device memory:
    any object with ``data_ptr()`` and ``numel()`` (a contiguous torch uint8
    tensor on the context's device, say) -- the context keeps a reference to
    it.  ``stream`` is a raw hipStream_t or a torch.cuda.Stream."""
    _free = None

    def __init__(self, device: int = 0, arena_bytes: int = 0, stream=None, arena=None):
        out = ctypes.c_void_p()
        ptr = None
        if arena is not None:
            ptr = int(arena.data_ptr())
            arena_bytes = int(arena.numel()) * int(getattr(arena, "element_size", lambda: 1)())
        self._arena = arena
        self._stream = stream
        _check(lib().cc_context_create(device, ptr, arena_bytes, _stream_handle(stream), ctypes.byref(out)))
        super().__init__(out.value)

    def close(self):
        if self.ptr:
            lib().cc_context_destroy(self.ptr)
            self.ptr = None
        self._arena = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def profile_enable(self, on: bool = True):
        _check(lib().cc_profile_enable(self.ptr, 1 if on else 0))

    def profile_filter(self, name=None, every=1):
        """Record only the kernel statistic `name`, one launch in `every`
        (None: every kernel)."""
        _check(lib().cc_profile_filter(self.ptr, name.encode() if name else None, int(every)))

    def profile_read(self):
        """{kernel name: (launches, total_ms, algo_bytes)}"""
        arr = (KernelStat * 256)()
        n = ctypes.c_size_t(0)
        _check(lib().cc_profile_read(self.ptr, ctypes.cast(arr, ctypes.c_void_p), 256, ctypes.byref(n)))
        out = {}
        for i in range(min(n.value, 256)):
            out[arr[i].name.decode()] = (int(arr[i].launches), float(arr[i].total_ms), float(arr[i].algo_bytes))
        return out

    def set_batch_lanes(self, lanes: int):
        _check(lib().cc_set_batch_lanes(self.ptr, lanes))

    def schedule(self) -> dict:
        s = _Schedule()
        _check(lib().cc_get_schedule(self.ptr, ctypes.byref(s)))
        return {"lanes": s.lanes, "entry_factor": s.entry_factor, "sort_above_k": s.sort_above_k,
                "group_min": s.group_min}

    def set_schedule(self, lanes: int = 0, entry_factor: int = 3, sort_above_k: int = 12, group_min: int = 2):
        s = _Schedule(lanes, entry_factor, sort_above_k, group_min)
        _check(lib().cc_set_schedule(self.ptr, ctypes.byref(s)))

    def set_table_budget(self, max_entries: int):
        _check(lib().cc_set_table_budget(self.ptr, max_entries))

    def last_chunk_count(self) -> int:
        return int(lib().cc_last_chunk_count(self.ptr))

    def last_table_sizes(self) -> np.ndarray:
        n = ctypes.c_size_t(0)
        buf = np.zeros(4096, dtype=np.int64)
        _check(lib().cc_last_table_sizes(self.ptr, _p(buf), buf.size, ctypes.byref(n)))
        return buf[: n.value].copy()


def _edges(edges) -> Tuple[int, np.ndarray]:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    if e.size == 0:
        return 0, np.zeros((1, 2), dtype=np.int32)
    return int(e.shape[0]), e


def load_graph(ctx: Context, n: int, row_ptr, col, flags: int = 0) -> Graph:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib().cc_load_graph(ctx.ptr, n, _p(rp), _p(cl), flags, ctypes.byref(out)))
    return Graph(out.value, ctx)


def color(ctx: Context, g: Graph, k: int, seed: int, num_colorings: int) -> Coloring:
    out = ctypes.c_void_p()
    _check(lib().cc_color(ctx.ptr, g.ptr, k, seed & (2**64 - 1), num_colorings, ctypes.byref(out)))
    return Coloring(out.value, ctx, k, num_colorings)


def color_explicit(ctx: Context, g: Graph, k: int, colors) -> Coloring:
    c = np.ascontiguousarray(colors, dtype=np.uint8)
    num = 1 if c.ndim == 1 else int(c.shape[0])
    out = ctypes.c_void_p()
    _check(lib().cc_color_explicit(ctx.ptr, g.ptr, k, num, _p(c), ctypes.byref(out)))
    return Coloring(out.value, ctx, k, num)


def build_decomposition(n_F: int, edges, flags: int = 0) -> Decomp:
    m, e = _edges(edges)
    out = ctypes.c_void_p()
    _check(lib().cc_build_decomposition(n_F, m, _p(e), flags, ctypes.byref(out)))
    return Decomp(out.value, n_F)


def decomp_import(n_F: int, edges, td) -> Decomp:
    m, e = _edges(edges)
    buf = np.ascontiguousarray(td, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(lib().cc_decomp_import(n_F, m, _p(e), _p(buf), buf.size, ctypes.byref(out)))
    return Decomp(out.value, n_F)


def count(ctx: Context, g: Graph, c: Coloring, d: Decomp, flags: int = 0):
    """(counts uint64[num_colorings], overflow bool[num_colorings])"""
    counts = np.zeros(c.num, dtype=np.uint64)
    ovf = np.zeros(c.num, dtype=np.uint8)
    _check(lib().cc_count(ctx.ptr, g.ptr, c.ptr, d.ptr, flags, _p(counts), _p(ovf)))
    return counts, ovf.astype(bool)


def vertex_sets(ctx: Context, g: Graph, c: Coloring, b: int, d: Decomp, cap: int):
    """(distinct vertex sets int32[n_sets, n_F] sorted, n_mappings) of colouring b."""
    sets = np.zeros((max(cap, 1), d.n_F), dtype=np.int32)
    ns = np.zeros(1, dtype=np.uint64)
    nm = np.zeros(1, dtype=np.uint64)
    _check(lib().cc_vertex_sets(ctx.ptr, g.ptr, c.ptr, b, d.ptr, cap, _p(sets), _p(ns), _p(nm)))
    return sets[: int(ns[0])].copy(), int(nm[0])


CC_SEARCH_DISTINCT_SETS = 1


class SearchOpts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("seed", ctypes.c_uint64), ("batch", ctypes.c_int32),
                ("max_solutions", ctypes.c_uint64), ("flags", ctypes.c_uint32)]


def search(ctx: Context, g: Graph, d: Decomp, eps: float, seed: int, max_solutions: int, batch: int = 16,
           distinct_sets: bool = False):
    """Repetition driver: (solutions int32[m, n_F], colourings run, colourings planned)."""
    opts = SearchOpts(eps, seed & (2**64 - 1), batch, max_solutions, CC_SEARCH_DISTINCT_SETS if distinct_sets else 0)
    rows = np.zeros((max_solutions, d.n_F), dtype=np.int32)
    nr = ctypes.c_uint64(0)
    run = ctypes.c_uint64(0)
    planned = ctypes.c_uint64(0)
    _check(lib().cc_search(ctx.ptr, g.ptr, d.ptr, ctypes.byref(opts), _p(rows), ctypes.byref(nr), ctypes.byref(run),
                           ctypes.byref(planned)))
    return rows[: nr.value].copy(), run.value, planned.value


class Plan(_Handle):
    """A count captured into a HIP graph (cc_plan_*): replay with new seeds."""
    _free = "cc_plan_destroy"

    def __init__(self, ctx: Context, g: Graph, d: Decomp, k: int, num_colorings: int, flags: int = 0):
        out = ctypes.c_void_p()
        _check(lib().cc_plan_create(ctx.ptr, g.ptr, d.ptr, k, num_colorings, flags, ctypes.byref(out)))
        super().__init__(out.value)
        self.ctx, self.g, self.d, self.num = ctx, g, d, num_colorings

    def count(self, seed: int):
        counts = np.zeros(self.num, dtype=np.uint64)
        ovf = np.zeros(self.num, dtype=np.uint8)
        _check(lib().cc_plan_count(self.ptr, seed & (2**64 - 1), _p(counts), _p(ovf)))
        return counts, ovf.astype(bool)


def estimate_memory(g: Graph, d: Decomp, k: int, num_colorings: int):
    """(estimated peak arena bytes, estimated sum of |D_x|) of a count."""
    pk = ctypes.c_double(0)
    en = ctypes.c_double(0)
    _check(lib().cc_estimate_memory(g.ptr, d.ptr, k, num_colorings, ctypes.byref(pk), ctypes.byref(en)))
    return pk.value, en.value


def count_range(ctx: Context, g: Graph, c: Coloring, d: Decomp, lo: int, hi: int, flags: int = 0):
    """Counts of the mappings with Phi(0) in [lo, hi): (counts, overflow)."""
    counts = np.zeros(c.num, dtype=np.uint64)
    ovf = np.zeros(c.num, dtype=np.uint8)
    _check(lib().cc_count_range(ctx.ptr, g.ptr, c.ptr, d.ptr, flags, int(lo), int(hi), _p(counts), _p(ovf)))
    return counts, ovf.astype(bool)


def count_noalloc(ctx: Context, g: Graph, c: Coloring, d: Decomp, flags: int = 0):
    """count() through cc_count_noalloc (the library's fixed device scratch;
    no device allocation).  (counts, overflow)"""
    counts = np.zeros(c.num, dtype=np.uint64)
    ovf = np.zeros(c.num, dtype=np.uint8)
    _check(lib().cc_count_noalloc(ctx.ptr, g.ptr, c.ptr, d.ptr, flags, _p(counts), _p(ovf)))
    return counts, ovf.astype(bool)


def count_by_vertex(ctx: Context, g: Graph, c: Coloring, b: int, d: Decomp, flags: int = 0):
    """(per_vertex uint64[n], count, overflow)"""
    pv = np.zeros(max(g.n, 1), dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    ovf = np.zeros(1, dtype=np.uint8)
    _check(lib().cc_count_by_vertex(ctx.ptr, g.ptr, c.ptr, b, d.ptr, flags, _p(pv), _p(cnt), _p(ovf)))
    return pv[: g.n], int(cnt[0]), bool(ovf[0])


def enumerate(ctx: Context, g: Graph, c: Coloring, b: int, d: Decomp, cap: int):  # noqa: A001
    """(rows int32[min(total, cap), n_F] lexicographically sorted, total)"""
    rows = np.zeros((max(cap, 1), d.n_F), dtype=np.int32)
    nr = np.zeros(1, dtype=np.uint64)
    tot = np.zeros(1, dtype=np.uint64)
    _check(lib().cc_enumerate(ctx.ptr, g.ptr, c.ptr, b, d.ptr, cap, _p(rows), _p(nr), _p(tot)))
    return rows[: int(nr[0])].copy(), int(tot[0])


class _Q(ctypes.Structure):
    _fields_ = [("decomp", ctypes.c_void_p), ("coloring", ctypes.c_void_p)]


def _query_array(queries):
    nq = len(queries)
    arr = (_Q * max(nq, 1))()
    for i in range(nq):
        arr[i].decomp = queries[i][0].ptr
        arr[i].coloring = queries[i][1].ptr
    return arr


def tune_batch(ctx: Context, g: Graph, queries, flags: int = 0) -> int:
    """Times the batch with 1, 2, 4 and 8 lanes; keeps and returns the best."""
    best = ctypes.c_int32(0)
    arr = _query_array(queries)
    _check(lib().cc_tune_batch(ctx.ptr, g.ptr, len(queries), ctypes.cast(arr, ctypes.c_void_p), flags,
                               ctypes.byref(best)))
    return best.value


def count_batch(ctx: Context, g: Graph, queries: Sequence[Tuple[Decomp, Coloring]], flags: int = 0):
    """Counts of many (decomposition, colouring) queries: list of (counts, overflow)."""
    nq = len(queries)
    arr = (_Q * max(nq, 1))()
    total = 0
    for i in range(nq):
        d, c = queries[i]
        arr[i].decomp = d.ptr
        arr[i].coloring = c.ptr
        total += c.num
    counts = np.zeros(max(total, 1), dtype=np.uint64)
    ovf = np.zeros(max(total, 1), dtype=np.uint8)
    _check(lib().cc_count_batch(ctx.ptr, g.ptr, nq, ctypes.cast(arr, ctypes.c_void_p), flags, _p(counts), _p(ovf)))
    out = []
    off = 0
    for d, c in queries:
        out.append((counts[off:off + c.num].copy(), ovf[off:off + c.num].astype(bool)))
        off += c.num
    return out


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("mem_budget", ctypes.c_size_t), ("max_entries", ctypes.c_uint64),
                ("max_heavy", ctypes.c_int32), ("tail_factor", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("requeued", ctypes.c_uint64), ("wall_s", ctypes.c_double), ("qps", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class Server:
    """Request loop over a resident graph (cc_server_*)."""

    def __init__(self, ctx: Context, g: Graph, max_inflight: int = 4, mem_budget: int = 0, max_entries: int = 0,
                 max_heavy: int = 1, tail_factor: float = 0.0):
        self.ctx, self.g = ctx, g
        opts = ServerOpts(max_inflight, mem_budget, max_entries, max_heavy, tail_factor)
        out = ctypes.c_void_p()
        _check(lib().cc_server_start(ctx.ptr, g.ptr, ctypes.byref(opts), ctypes.byref(out)))
        self.ptr = out.value
        self._keep = {}

    def submit(self, d: Decomp, k: int, seed: int, num_colorings: int) -> int:
        t = ctypes.c_uint64(0)
        _check(lib().cc_server_submit(self.ptr, d.ptr, k, seed & (2**64 - 1), num_colorings, ctypes.byref(t)))
        self._keep[t.value] = (d, num_colorings)
        return t.value

    def _res(self, fn, ticket):
        d, nc = self._keep[ticket]
        counts = np.zeros(nc, dtype=np.uint64)
        ovf = np.zeros(nc, dtype=np.uint8)
        st = ctypes.c_int32(0)
        _check(fn(self.ptr, ticket, _p(counts), _p(ovf), ctypes.byref(st)))
        return st.value, counts, ovf.astype(bool)

    def poll(self, ticket: int):
        """(state, counts, overflow): state 0 pending, 1 done, < 0 error code."""
        return self._res(lib().cc_server_poll, ticket)

    def wait(self, ticket: int):
        return self._res(lib().cc_server_wait, ticket)

    def stop(self) -> dict:
        st = ServerStats()
        _check(lib().cc_server_stop(self.ptr, ctypes.byref(st)))
        self.ptr = None
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}
