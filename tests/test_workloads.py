"""Generators: determinism and CSR hygiene (simple, symmetric, sorted rows)."""
import numpy as np
import pytest

from paper_1908_11248_amd import workloads as W


def check_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(src != col)  # no loops
    for v in range(0, g.n, max(1, g.n // 500)):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)  # sorted, no duplicates
    a = src.astype(np.int64) * g.n + col
    b = col.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(a), np.sort(b))  # symmetric


@pytest.mark.parametrize("make", [lambda: W.er_pairs(200, 0.05, 1), lambda: W.er_skip(3000, 8 / 2999, 2),
                                  lambda: W.rgg(4000, 10, 3), lambda: W.barabasi_albert(3000, 5, 4),
                                  lambda: W.chung_lu(20000, 2.5, 10, 5)])
def test_generators_deterministic_and_simple(make):
    g1, g2 = make(), make()
    assert np.array_equal(g1.row_ptr, g2.row_ptr) and np.array_equal(g1.col, g2.col)
    check_csr(g1)


def test_mean_degrees_near_targets():
    assert abs(W.er_skip(20000, 8 / 19999, 1).degrees().mean() - 8) < 0.3
    assert abs(W.rgg(20000, 10, 1).degrees().mean() - 10) < 0.6
    assert abs(W.barabasi_albert(5000, 5, 1).degrees().mean() - 10) < 0.1
    g = W.chung_lu(50000, 2.5, 10, 1)
    assert abs(g.degrees().mean() - 10) < 1.0


def test_patterns():
    for n in range(5, 11):
        t = W.random_tree(n, n)
        assert len(t.edges) == n - 1
        p = W.partial_3tree(n, n)
        assert len(p.edges) >= n - 1
    assert len(W.ladder(4).edges) == 10
