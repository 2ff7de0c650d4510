"""The C-ABI boundary on the GPU: caller-owned arena and stream (torch as
device-memory plumbing), the graph loader's validation and canonicalisation
branches, and the size limits (CC_ERANGE) of colourings and served queries.

Counts are compared with the oracle on the same inputs.
"""
import sys

import numpy as np
import pytest

import oracle as O
import paper_1908_11248_amd as cc
from paper_1908_11248_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_counts(g, pat, k, seed, B):
    return [O.dp_count(g, pat, k, O.color_array(seed, b, g.n, k))["count"] for b in range(B)]


def test_torch_arena_and_stream():
    import torch

    say("boundary: torch arena + stream")
    arena = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.Stream()
    g = W.er_pairs(200, 0.05, W.workload(1).seed)
    pats = [W.path(5), W.cycle(5), W.pattern_B(), W.random_tree(8, 3)]
    with cc.Context(0, stream=stream, arena=arena) as ctx:
        G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
        for pat in pats:
            C = cc.color(ctx, G, pat.n, 99, 3)
            D = cc.build_decomposition(pat.n, pat.edges)
            counts, _ = cc.count(ctx, G, C, D)
            assert [int(x) for x in counts] == _oracle_counts(g, pat, pat.n, 99, 3), pat.name
    # the arena is still the caller's: it can be written after the context is gone
    arena.fill_(1)
    torch.cuda.synchronize()
    assert int(arena[:16].sum()) == 16


def test_caller_arena_misaligned_or_too_small():
    import torch

    say("boundary: bad arenas")
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(cc.CcError) as e:
        cc.Context(0, arena=buf[1:])
    assert e.value.code == cc.CC_EINVAL
    with pytest.raises(cc.CcError) as e:
        cc.Context(0, arena=buf[:1024])
    assert e.value.code == cc.CC_EINVAL


def test_arena_too_small_for_the_tables_is_enomem():
    import torch

    say("boundary: small arena")
    arena = torch.empty(64 << 10, dtype=torch.uint8, device="cuda:0")
    g = W.er_pairs(400, 0.05, 5)
    with cc.Context(0, arena=arena) as ctx:
        G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
        C = cc.color(ctx, G, 6, 1, 8)
        D = cc.build_decomposition(6, W.cycle(6).edges)
        with pytest.raises(cc.CcError) as e:
            cc.count(ctx, G, C, D)
        assert e.value.code == cc.CC_ENOMEM


def _raw_csr(n, pairs):
    """CSR of exactly the given directed pairs, in the given order."""
    rows = [[] for _ in range(n)]
    for a, b in pairs:
        rows[a].append(b)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in r], dtype=np.int32)
    return rp, col


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0, arena_bytes=1 << 30)
    yield c
    c.close()


def test_load_graph_rejects_malformed_and_canonicalizes(ctx):
    say("boundary: cc_load_graph branches")
    g = W.er_pairs(60, 0.15, 21)
    src, dst = W.edge_list(g)
    pairs = list(zip(src.tolist(), dst.tolist()))
    cases = {
        "one direction only": pairs,
        "self-loop": pairs + [(b, a) for a, b in pairs] + [(3, 3)],
        "duplicate": pairs + [(b, a) for a, b in pairs] + [pairs[0]],
        "unsorted rows": [(b, a) for a, b in pairs][::-1] + pairs[::-1],
    }
    pat = W.cycle(4)
    D = cc.build_decomposition(pat.n, pat.edges)
    want = _oracle_counts(g, pat, 4, 5, 2)
    for name, pr in cases.items():
        rp, col = _raw_csr(g.n, pr)
        with pytest.raises(cc.CcError) as e:
            cc.load_graph(ctx, g.n, rp, col)
        assert e.value.code == cc.CC_EINVAL, name
        G = cc.load_graph(ctx, g.n, rp, col, cc.CC_GRAPH_CANONICALIZE)
        C = cc.color(ctx, G, 4, 5, 2)
        counts, _ = cc.count(ctx, G, C, D)
        assert [int(x) for x in counts] == want, name
    # out-of-range ids and a bad row_ptr stay errors even with the flag
    rp, col = _raw_csr(g.n, pairs + [(b, a) for a, b in pairs])
    bad = col.copy()
    bad[0] = g.n
    for flags in (0, cc.CC_GRAPH_CANONICALIZE):
        with pytest.raises(cc.CcError) as e:
            cc.load_graph(ctx, g.n, rp, bad, flags)
        assert e.value.code == cc.CC_EINVAL
        rp2 = rp.copy()
        rp2[0] = 1
        with pytest.raises(cc.CcError) as e:
            cc.load_graph(ctx, g.n, rp2, col, flags)
        assert e.value.code == cc.CC_EINVAL


def test_size_limits_are_erange(ctx):
    say("boundary: CC_ERANGE limits")
    g = W.er_pairs(30, 0.2, 2)
    G = cc.load_graph(ctx, g.n, g.row_ptr, g.col)
    for k in (0, 17, 33):
        with pytest.raises(cc.CcError) as e:
            cc.color(ctx, G, k, 1, 1)
        assert e.value.code == cc.CC_ERANGE
        with pytest.raises(cc.CcError) as e:
            cc.color_explicit(ctx, G, k, np.zeros(g.n, dtype=np.uint8))
        assert e.value.code == cc.CC_ERANGE
    D = cc.build_decomposition(6, W.cycle(6).edges)
    C = cc.color(ctx, G, 5, 1, 1)
    with pytest.raises(cc.CcError) as e:  # fewer colours than pattern vertices
        cc.count(ctx, G, C, D)
    assert e.value.code == cc.CC_ERANGE
    srv = cc.Server(ctx, G, max_inflight=1)
    try:
        for k in (5, 17):
            with pytest.raises(cc.CcError) as e:
                srv.submit(D, k, 1, 1)
            assert e.value.code == cc.CC_ERANGE
    finally:
        srv.stop()
