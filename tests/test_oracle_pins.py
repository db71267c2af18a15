"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check is an independent
route to the same number (enumeration of tensor entries, a closed form, an
invariant stated in Sec. II, a textbook special case).
"""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import blowup as bl
from oracle import sttsv_ref as sr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int32)
    return eptr, eidx


def _random_hypergraph(rng, n, m, r, kmin=1):
    edges = []
    for _ in range(m):
        k = rng.randint(kmin, min(r, n))
        edges.append(tuple(rng.sample(range(n), k)))
    return edges


def _read_fig1():
    edges, deg, vals, betas, order = [], None, {}, {}, None
    with open(os.path.join(GOLDEN, "fig1_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tag, *rest = line.split()
            if tag == "edge":
                edges.append(tuple(int(v) - 1 for v in rest))
            elif tag == "order":
                order = int(rest[0])
            elif tag == "degrees":
                deg = [int(v) for v in rest]
            elif tag == "value":
                vals[int(rest[0])] = Fraction(rest[1])
            elif tag == "beta":
                betas[int(rest[0])] = int(rest[1])
    return edges, order, deg, vals, betas


# ---------------------------------------------------------------- definitions

def test_stirling_table_small():
    # S(n,k) values of the textbook table
    assert [bl.stirling2(4, k) for k in range(5)] == [0, 1, 7, 6, 1]
    assert [bl.stirling2(5, k) for k in range(6)] == [0, 1, 15, 25, 10, 1]
    assert bl.stirling2(10, 3) == 9330
    # sum_k S(n,k) = Bell number
    assert sum(bl.stirling2(8, k) for k in range(9)) == 4140


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6])
def test_beta_size_counts_covering_tuples(r):
    # footnote of Sec. II: |beta(e)| = |e|! S(N,|e|) -- counted by brute force
    for k in range(1, r + 1):
        assert len(bl.beta_tuples(range(k), r)) == bl.beta_size(r, k)


def test_fig1_worked_example():
    edges, N, deg, vals, betas = _read_fig1()
    n = 8
    for e in edges:
        k = len(e)
        assert len(bl.beta_tuples(e, N)) == betas[k]
        assert bl.blowup_value(N, k) == vals[k]
    B = bl.blowup_entries(edges, N)
    # every entry belongs to exactly one edge; total mass = sum_e w(e)
    assert sum(B.values()) == sum(len(e) for e in edges)
    assert len(B) == sum(betas[len(e)] for e in edges)
    # symmetry: value unchanged under any permutation of an index tuple
    for t, v in list(B.items())[:200]:
        assert B[tuple(reversed(t))] == v
    one = [Fraction(1)] * n
    # Sec. II: B 1^(N-1) = d
    assert bl.ttsv1_from_entries(B, n, N, one) == [Fraction(d) for d in deg]
    assert bl.aay_exact(edges, n, N, one) == [Fraction(d) for d in deg]
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, N, np.ones(n))
    np.testing.assert_allclose(y, deg, rtol=1e-15)


def test_uniform_blowup_is_adjacency_tensor():
    # Sec. II: for a uniform hypergraph the blowup tensor is the adjacency
    # tensor, value w(e)/N! at each of the N! permutations of the edge.
    e = (0, 2, 3)
    B = bl.blowup_entries([e], 3)
    assert len(B) == 6
    assert set(B.values()) == {Fraction(3, 6)}


# ------------------------------------------------- AAY vs independent routes

@pytest.mark.parametrize("seed", range(6))
def test_aay_exact_equals_entry_enumeration(seed):
    rng = random.Random(seed)
    r = rng.randint(2, 5)
    n = rng.randint(r, 8)
    edges = _random_hypergraph(rng, n, rng.randint(1, 6), r)
    x = [Fraction(rng.randint(1, 9), rng.randint(1, 9)) for _ in range(n)]
    B = bl.blowup_entries(edges, r)
    assert bl.aay_exact(edges, n, r, x) == bl.ttsv1_from_entries(B, n, r, x)


@pytest.mark.parametrize("seed", range(6))
def test_inclusion_exclusion_equals_aay(seed):
    rng = random.Random(100 + seed)
    r = rng.randint(2, 9)
    n = rng.randint(r, 12)
    edges = _random_hypergraph(rng, n, rng.randint(1, 5), min(r, 6))
    x = [Fraction(rng.randint(-5, 9), rng.randint(1, 7)) for _ in range(n)]
    assert bl.aay_exact(edges, n, r, x) == bl.inclusion_exclusion_sttsv(edges, n, r, x)


@pytest.mark.parametrize("seed", range(5))
def test_fp64_oracle_matches_exact(seed):
    rng = random.Random(200 + seed)
    r = rng.randint(2, 7)
    n = rng.randint(r, 10)
    edges = _random_hypergraph(rng, n, rng.randint(2, 12), r)
    xf = np.array([rng.uniform(0.01, 1.0) for _ in range(n)])
    exact = bl.inclusion_exclusion_sttsv(edges, n, r, [Fraction(v) for v in xf])
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, xf)
    for v in range(n):
        ev = float(exact[v])
        assert abs(y[v] - ev) <= 1e-14 * abs(ev) + 1e-300


@pytest.mark.parametrize("r", [2, 3, 5, 12, 25, 50])
def test_degree_invariant_all_orders(r):
    # Sec. II: with w(e)=|e|, B 1^(r-1) = d, for every tensor order r >= max|e|
    rng = np.random.default_rng(r)
    n, m = 60, 200
    sizes = rng.integers(1, min(r, 9) + 1, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    eptr, eidx = _csr(edges)
    d = np.bincount(eidx, minlength=n)
    y = sr.sttsv(eptr, eidx, n, r, np.ones(n))
    np.testing.assert_allclose(y, d, rtol=2e-14)


def _contraction_closed_form(edges, r, x):
    # B x^r = sum_e w(e)/|beta(e)| * sum_{S subset e} (-1)^{|e|-|S|} (sum_S x)^r
    tot = Fraction(0)
    for e in edges:
        k = len(e)
        inner = Fraction(0)
        for mask in range(1 << k):
            s = sum((x[e[j]] for j in range(k) if mask >> j & 1), Fraction(0))
            inner += (-1) ** (k - bin(mask).count("1")) * s ** r
        tot += bl.blowup_value(r, k) * inner
    return tot


def test_full_contraction_identity_tiny():
    rng = random.Random(7)
    r, n = 4, 6
    edges = _random_hypergraph(rng, n, 5, r)
    x = [Fraction(rng.randint(1, 5), rng.randint(1, 5)) for _ in range(n)]
    B = bl.blowup_entries(edges, r)
    assert bl.full_contraction_from_entries(B, r, x) == _contraction_closed_form(edges, r, x)


@pytest.mark.parametrize("r", [3, 6, 11])
def test_xTy_equals_full_contraction(r):
    # x^T (B x^(r-1)) = B x^r
    rng = random.Random(r)
    n = 14
    edges = _random_hypergraph(rng, n, 25, min(r, 7))
    xf = np.array([rng.uniform(0.1, 1.0) for _ in range(n)])
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, xf)
    lhs = math.fsum((xf * y).tolist())
    rhs = float(_contraction_closed_form(edges, r, [Fraction(v) for v in xf]))
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


def test_uniform_reduction():
    # all edges of size r: y_v = sum_{e containing v} prod_{u in e, u != v} x_u
    rng = np.random.default_rng(3)
    n, m, r = 40, 150, 5
    edges = [tuple(rng.choice(n, size=r, replace=False)) for _ in range(m)]
    x = rng.uniform(0.1, 1.0, n)
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, x)
    ref = np.zeros(n)
    for e in edges:
        for v in e:
            ref[v] += np.prod([x[u] for u in e if u != v])
    np.testing.assert_allclose(y, ref, rtol=1e-13)


def test_graph_case_is_adjacency_matvec():
    # r = 2 and all edges of size 2: B is the adjacency matrix, y = A x
    rng = np.random.default_rng(4)
    n, m = 50, 300
    edges = [tuple(rng.choice(n, size=2, replace=False)) for _ in range(m)]
    x = rng.uniform(-1.0, 1.0, n)
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, 2, x)
    i = np.array([e[0] for e in edges] + [e[1] for e in edges])
    j = np.array([e[1] for e in edges] + [e[0] for e in edges])
    A = sp.coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n)).tocsr()
    np.testing.assert_allclose(y, A @ x, rtol=1e-14, atol=1e-14)


def test_size_one_edges():
    # a size-1 edge {v}: beta = {(v,...,v)}, value 1, so y_v += x_v^(r-1)
    eptr, eidx = _csr([(0,), (1,), (0, 1)])
    x = np.array([0.5, 2.0])
    r = 4
    y = sr.sttsv(eptr, eidx, 2, r, x)
    B = bl.blowup_entries([(0,), (1,), (0, 1)], r)
    ref = bl.ttsv1_from_entries(B, 2, r, [Fraction(v) for v in x])
    np.testing.assert_allclose(y, [float(v) for v in ref], rtol=1e-15)


def test_homogeneity_and_equivariance():
    rng = np.random.default_rng(5)
    n, m, r = 80, 300, 7
    sizes = rng.integers(2, 7, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    x = rng.uniform(0.05, 1.0, n)
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, x)
    # Eq. (2) is homogeneous of degree r-1 in x
    y3 = sr.sttsv(eptr, eidx, n, r, 3.0 * x)
    np.testing.assert_allclose(y3, 3.0 ** (r - 1) * y, rtol=1e-13)
    # relabelling vertices permutes y the same way
    p = rng.permutation(n)
    edges_p = [tuple(p[v] for v in e) for e in edges]
    xp = np.empty(n)
    xp[p] = x
    ep, ei = _csr(edges_p)
    yp = sr.sttsv(ep, ei, n, r, xp)
    np.testing.assert_allclose(yp[p], y, rtol=1e-14)
    # edge order and member order do not matter
    order = rng.permutation(m)
    edges_o = [tuple(rng.permutation(list(edges[i]))) for i in order]
    eo, io = _csr(edges_o)
    np.testing.assert_allclose(sr.sttsv(eo, io, n, r, x), y, rtol=1e-14)


def test_sampled_nodes_match_full():
    rng = np.random.default_rng(6)
    n, m, r = 300, 1500, 9
    sizes = rng.integers(1, 8, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    x = rng.uniform(0.0, 1.0, n)
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, x)
    nodes = rng.choice(n, size=40, replace=False)
    np.testing.assert_array_equal(sr.sttsv_at(eptr, eidx, n, r, x, nodes), y[nodes])


def test_weight_table_exact():
    # w(e)/|beta(e)| (r-1)! rounded once; k = r gives exactly 1
    for r in (2, 5, 25, 50, 64):
        assert sr.weight_fp64(r, r) == 1.0
        for k in range(1, r + 1):
            w = sr.weight_exact(r, k)
            assert w == Fraction(k * math.factorial(r - 1), math.factorial(k) * bl.stirling2(r, k))
            assert sr.weight_fp64(r, k) == float(w)


def test_validation_errors():
    with pytest.raises(ValueError):
        sr.sttsv(*_csr([(0, 0, 1)]), 3, 3, np.ones(3))      # repeated vertex
    with pytest.raises(ValueError):
        sr.sttsv(*_csr([(0, 1, 2, 3)]), 4, 3, np.ones(4))   # |e| > r
    with pytest.raises(ValueError):
        sr.sttsv(*_csr([(0, 5)]), 4, 3, np.ones(4))         # id out of range


# ------------------------------------------------- edge-weighted H = (V, E, w)

@pytest.mark.parametrize("seed", range(4))
def test_weighted_oracle_matches_entry_enumeration(seed):
    # Sec. II defines B for an edge-weighted H: every blowup of e carries
    # w(e)/|beta(e)|.  Listing the entries with random weights, in exact
    # rationals, and evaluating Eq. (2) must give the FP64 oracle's y.
    rng = random.Random(300 + seed)
    r = rng.randint(2, 5)
    n = rng.randint(r, 8)
    edges = _random_hypergraph(rng, n, rng.randint(2, 7), r)
    w = np.array([rng.uniform(0.1, 5.0) for _ in edges])
    xf = np.array([rng.uniform(0.05, 1.0) for _ in range(n)])
    B = bl.blowup_entries(edges, r, weights=[Fraction(v) for v in w])
    exact = bl.ttsv1_from_entries(B, n, r, [Fraction(v) for v in xf])
    eptr, eidx = _csr(edges)
    y = sr.sttsv(eptr, eidx, n, r, xf, w=w)
    for v in range(n):
        assert abs(y[v] - float(exact[v])) <= 1e-14 * abs(float(exact[v])) + 1e-300
    # the paper's default w(e) = |e| is the weighted case with w = sizes
    np.testing.assert_array_equal(sr.sttsv(eptr, eidx, n, r, xf, w=np.diff(eptr).astype(float)),
                                  sr.sttsv(eptr, eidx, n, r, xf))


@pytest.mark.parametrize("r", [3, 7, 25])
def test_weighted_ones_give_weighted_degree(r):
    # B 1^(r-1) = sum over e containing v of w(e)/|e|: each row of the
    # blowups of e holds |beta(e)|/|e| entries of value w(e)/|beta(e)|
    rng = np.random.default_rng(40 + r)
    n, m = 50, 160
    sizes = rng.integers(1, min(r, 8) + 1, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    eptr, eidx = _csr(edges)
    w = rng.uniform(0.01, 10.0, size=m)
    edge_of = np.repeat(np.arange(m), sizes)
    expect = np.bincount(eidx, weights=(w / sizes)[edge_of], minlength=n)
    y = sr.sttsv(eptr, eidx, n, r, np.ones(n), w=w)
    np.testing.assert_allclose(y, expect, rtol=2e-14)


def test_weight_validation():
    eptr, eidx = _csr([(0, 1), (1, 2)])
    for bad in ([1.0, 0.0], [1.0, -2.0], [1.0, np.inf], [1.0, np.nan], [1.0]):
        with pytest.raises(ValueError):
            sr.sttsv(eptr, eidx, 3, 3, np.ones(3), w=np.array(bad))
