"""Pins of the CCSS forest (Sec. III) and of the memoised STTSV over it
(Alg. 4): node, root and convolution counts against closed forms worked out
by hand for the substructures of Sec. IV-C (one edge, a nested chain, a
sunflower), and the STTSV against the plain definition (Alg. 2 oracle)."""
import random

import numpy as np
import pytest

from oracle import ccss_ref as cr
from oracle import sttsv_ref as sr


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int64)
    return eptr, eidx


@pytest.mark.parametrize("k", range(2, 10))
def test_single_edge_counts(k):
    # paths e \ u_j: the prefixes (u_1..u_l), l <= k-1, are shared; removing
    # u_j (2 <= j <= k-1) adds k-j nodes; removing u_1 starts a second tree of
    # k-1 nodes:  (k-1) + (k-1)(k-2)/2 + (k-1) = (k-1)(k+2)/2 nodes, 2 roots
    eptr, eidx = _csr([tuple(range(10, 10 + k))[::-1]])      # unsorted input
    c = cr.counts(cr.build_forest(eptr, eidx, 20))
    assert c["nodes"] == (k - 1) * (k + 2) // 2
    assert c["roots"] == 2
    assert c["convolutions"] == (k * k + k - 6) // 2
    assert c["leaves"] == k


@pytest.mark.parametrize("sizes", [(2, 3), (3, 5, 6), (2, 4, 7, 9), (5,)])
def test_nested_chain_counts(sizes):
    # e_i = the first k_i vertices: every prefix of a path of a smaller edge is
    # a prefix of a path of the largest one, so the forest is the largest
    # edge's: (K-1)(K+2)/2 nodes, 2 roots; special leaves sum k_i
    K = max(sizes)
    eptr, eidx = _csr([tuple(range(k)) for k in sizes])
    c = cr.counts(cr.build_forest(eptr, eidx, K))
    assert c["nodes"] == (K - 1) * (K + 2) // 2 and c["roots"] == 2
    assert c["leaves"] == sum(sizes)


@pytest.mark.parametrize("m,t,s", [(1, 2, 2), (3, 2, 3), (4, 3, 1), (5, 4, 4), (2, 6, 2)])
def test_sunflower_counts(m, t, s):
    # m edges of size k = t + s sharing the kernel {0..t-1} (first in the
    # order), disjoint petals of size s.  Kernel-only prefixes are shared:
    # t + t(t-1)/2 nodes; every edge adds t s nodes (kernel vertex removed,
    # then its petal) and the trie of its petal's paths under the whole
    # kernel, (s-1)(s+2)/2 nodes; 2 roots (t >= 2)
    edges = [tuple(range(t)) + tuple(range(t + i * s, t + (i + 1) * s)) for i in range(m)]
    eptr, eidx = _csr(edges)
    c = cr.counts(cr.build_forest(eptr, eidx, t + m * s))
    assert c["nodes"] == t + t * (t - 1) // 2 + m * (t * s + (s - 1) * (s + 2) // 2)
    assert c["roots"] == 2
    assert c["leaves"] == m * (t + s)


def test_key_order_changes_sharing_not_results():
    rng = np.random.default_rng(3)
    n, m, r = 40, 120, 7
    sizes = rng.integers(1, 8, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    eptr, eidx = _csr(edges)
    x = rng.uniform(0.05, 1.0, n)
    ref = sr.sttsv(eptr, eidx, n, r, x)
    for key in (None, rng.permutation(n)):
        f = cr.build_forest(eptr, eidx, n, key)
        # levels in increasing (parent, key) order, parents valid
        for depth, (v, p) in enumerate(f["levels"]):
            kk = (p if depth else np.zeros_like(p)) * n + (np.arange(n) if key is None else key)[v]
            assert np.all(np.diff(kk) > 0)
        y = cr.sttsv_alg4(eptr, eidx, n, r, x, forest=f)
        np.testing.assert_allclose(y, ref, rtol=2e-14)


@pytest.mark.parametrize("seed", range(4))
def test_alg4_matches_definition(seed):
    rng = random.Random(500 + seed)
    r = rng.choice([3, 5, 9, 25, 50])
    n = rng.randint(max(r, 10), 60)
    m = rng.randint(20, 120)
    edges = [tuple(rng.sample(range(n), rng.randint(1, min(r, 9)))) for _ in range(m)]
    # shared structure: a sunflower and a nested chain on top of random edges
    edges += [(0, 1, 3 + i)[:min(r, 3)] for i in range(5)] + [tuple(range(k)) for k in (2, 4, 6) if k <= r]
    eptr, eidx = _csr(edges)
    x = np.array([rng.uniform(1e-3, 1.0) for _ in range(n)])
    w = np.array([rng.uniform(0.1, 4.0) for _ in edges])
    np.testing.assert_allclose(cr.sttsv_alg4(eptr, eidx, n, r, x), sr.sttsv(eptr, eidx, n, r, x), rtol=1e-13)
    np.testing.assert_allclose(cr.sttsv_alg4(eptr, eidx, n, r, x, w=w), sr.sttsv(eptr, eidx, n, r, x, w=w),
                               rtol=1e-13)


def test_sharing_only_removes_convolutions():
    # Edges on disjoint vertex sets share no prefix: the forest is the union
    # of the single-edge forests.  Overlapping edges can only share nodes.
    rng = np.random.default_rng(9)
    ks = rng.integers(2, 9, size=20)
    off = np.concatenate([[0], np.cumsum(ks)])
    eptr, eidx = _csr([tuple(range(off[i], off[i + 1])) for i in range(len(ks))])
    c = cr.counts(cr.build_forest(eptr, eidx, int(off[-1])))
    assert c["convolutions"] == sum((k * k + k - 6) // 2 for k in ks)
    edges = [tuple(rng.choice(12, size=k, replace=False)) for k in ks]
    eptr, eidx = _csr(edges)
    c = cr.counts(cr.build_forest(eptr, eidx, 12))
    assert c["convolutions"] < sum((k * k + k - 6) // 2 for k in ks)
