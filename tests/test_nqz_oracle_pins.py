"""Pins of the NQZ oracle (Alg. 1) against closed forms."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import blowup as bl
from oracle import nqz_ref
from oracle import sttsv_ref as sr


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int32)
    return eptr, eidx


def _cyclic_intervals(n, sizes):
    return [tuple((s + j) % n for j in range(k)) for k in sizes for s in range(n)]


def test_regular_hypergraph_uniform_vector():
    # every vertex lies in k intervals of size k for k = 2..5: degree 14.
    # A regular hypergraph has x = 1/n and lambda = degree (B 1 = d, Sec. II).
    n, r = 23, 5
    eptr, eidx = _csr(_cyclic_intervals(n, [2, 3, 4, 5]))
    out = nqz_ref.nqz(eptr, eidx, n, r, tol=1e-12)
    assert out["iterations"] == 1
    np.testing.assert_allclose(out["x"], 1.0 / n, rtol=1e-14)
    assert abs(out["lambda_min"] - 14.0) < 1e-12 and abs(out["lambda_max"] - 14.0) < 1e-12


def test_first_iterate_is_degree_root():
    # from y = 1/n, z = B y^(r-1) = d / n^(r-1), so x_1 = d^(1/(r-1)) / ||.||_1
    rng = np.random.default_rng(1)
    n, m, r = 50, 200, 6
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in rng.integers(2, 7, size=m)]
    eptr, eidx = _csr(edges)
    d = np.bincount(eidx, minlength=n).astype(float)
    out = nqz_ref.nqz(eptr, eidx, n, r, tol=0.0, max_iter=1, history=True)
    w = d ** (1.0 / (r - 1))
    np.testing.assert_allclose(out["xs"][0], w / w.sum(), rtol=1e-14)


def test_graph_case_perron_vector():
    # r = 2: B = A, NQZ is the power method; a connected non-bipartite graph
    # gives the Perron vector and the spectral radius.
    rng = np.random.default_rng(2)
    n = 40
    edges = {(i, (i + 1) % n) for i in range(n)} | {(0, 2)}          # odd cycle -> aperiodic
    while len(edges) < 90:
        a, b = rng.choice(n, size=2, replace=False)
        edges.add((min(a, b), max(a, b)))
    edges = sorted(edges)
    eptr, eidx = _csr(edges)
    out = nqz_ref.nqz(eptr, eidx, n, 2, tol=1e-13, max_iter=5000)
    assert out["converged"]
    i = np.array([e[0] for e in edges] + [e[1] for e in edges])
    j = np.array([e[1] for e in edges] + [e[0] for e in edges])
    A = sp.coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n)).toarray()
    w, V = np.linalg.eigh(A)
    v = np.abs(V[:, -1])
    np.testing.assert_allclose(out["x"], v / v.sum(), rtol=1e-9)
    assert abs(out["lambda_max"] - w[-1]) < 1e-10 * w[-1]


def _ie_term(e, v, r, x):
    # inclusion-exclusion closed form of one term (floats; small edges only)
    others = [u for u in e if u != v]
    k = len(e)
    tot = 0.0
    for mask in range(1 << len(others)):
        s = x[v] + sum(x[u] for j, u in enumerate(others) if mask >> j & 1)
        tot += (-1) ** (k - 1 - bin(mask).count("1")) * s ** (r - 1)
    return float(bl.blowup_value(r, k)) * tot


def test_sunflower_fixed_point():
    # p petals {0} U P_i, |e| = k, core vertex 0.  By symmetry x = (a, b, ..., b);
    # with b = 1 the eigen-equation reduces to one scalar equation in a,
    # solved here by bisection on closed-form terms.
    p, k, r = 7, 4, 5
    edges = [(0,) + tuple(1 + i * (k - 1) + j for j in range(k - 1)) for i in range(p)]
    n = 1 + p * (k - 1)
    e0 = edges[0]

    def f(a):
        x = {u: (a if u == 0 else 1.0) for u in e0}
        lam_core = p * _ie_term(e0, 0, r, x) / a ** (r - 1)
        lam_petal = _ie_term(e0, e0[1], r, x)
        return lam_core - lam_petal
    lo, hi = 1e-3, 1e3
    assert f(lo) * f(hi) < 0
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if f(lo) * f(mid) <= 0:
            hi = mid
        else:
            lo = mid
    a = math.sqrt(lo * hi)
    xref = np.ones(n)
    xref[0] = a
    xref /= xref.sum()
    eptr, eidx = _csr(edges)
    out = nqz_ref.nqz(eptr, eidx, n, r, tol=1e-13, max_iter=2000)
    assert out["converged"]
    np.testing.assert_allclose(out["x"], xref, rtol=1e-10)


def test_shift_changes_ratios_not_vector():
    # the shift adds alpha to every ratio; the fixed point is the same vector
    rng = np.random.default_rng(3)
    n, r = 30, 4
    edges = _cyclic_intervals(n, [2, 3]) + [tuple(rng.choice(n, size=3, replace=False)) for _ in range(20)]
    eptr, eidx = _csr(edges)
    a = nqz_ref.nqz(eptr, eidx, n, r, tol=1e-12, max_iter=3000)
    b = nqz_ref.nqz(eptr, eidx, n, r, tol=1e-12, max_iter=3000, alpha=2.0)
    assert a["converged"] and b["converged"]
    np.testing.assert_allclose(a["x"], b["x"], rtol=1e-9)
    assert abs(a["lambda_max"] - b["lambda_max"]) < 1e-9 * a["lambda_max"]
