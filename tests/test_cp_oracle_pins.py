"""Pins of the symmetric CP oracle: ||B||^2 and the objective against sums
over every listed tensor entry (exact rationals / dense arrays), the
gradient against central differences of that pinned objective, the graph
case r = 2 against a library eigendecomposition, and the descent itself."""
import itertools
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import blowup as bl
from oracle import cp_ref


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int64)
    return eptr, eidx


def _tiny(seed, n=5, r=4, m=6):
    rng = random.Random(seed)
    edges = [tuple(rng.sample(range(n), rng.randint(1, min(r, n)))) for _ in range(m)]
    w = [rng.uniform(0.2, 3.0) for _ in edges]
    return edges, w


@pytest.mark.parametrize("seed", range(3))
def test_norm2_is_sum_of_squared_entries(seed):
    edges, w = _tiny(seed)
    r = 4
    eptr, eidx = _csr(edges + edges[:2])          # a repeated edge adds to the same entries
    w = w + w[:2]
    edges = edges + edges[:2]
    for weights in (None, w):
        B = bl.blowup_entries(edges, r, weights=None if weights is None else [Fraction(v) for v in weights])
        exact = float(sum(v * v for v in B.values()))
        got = cp_ref.norm2(eptr, eidx, 5, r, None if weights is None else np.array(weights))
        assert abs(got - exact) <= 1e-15 * exact


@pytest.mark.parametrize("seed", range(3))
def test_objective_against_dense_tensor(seed):
    edges, w = _tiny(10 + seed)
    n, r, R = 5, 4, 3
    rng = np.random.default_rng(seed)
    lam = rng.normal(size=R)
    A = rng.normal(size=(n, R))
    B = np.zeros((n,) * r)
    for t, v in bl.blowup_entries(edges, r, weights=[Fraction(x) for x in w]).items():
        B[t] = float(v)
    M = B.copy()
    for l in range(R):
        outer = A[:, l]
        for _ in range(r - 1):
            outer = np.multiply.outer(outer, A[:, l])
        M -= lam[l] * outer
    eptr, eidx = _csr(edges)
    f, _, _ = cp_ref.objective_grad(eptr, eidx, n, r, lam, A, w=np.array(w))
    assert abs(f - float(np.sum(M * M))) <= 1e-12 * max(1.0, float(np.sum(B * B)))


def test_gradient_against_central_differences():
    edges, w = _tiny(20, n=6, r=5, m=8)
    n, r, R = 6, 5, 2
    rng = np.random.default_rng(4)
    lam = rng.normal(size=R)
    A = rng.normal(size=(n, R)) * 0.5
    eptr, eidx = _csr(edges)
    f, dl, dA = cp_ref.objective_grad(eptr, eidx, n, r, lam, A)
    h = 1e-6
    for l in range(R):
        lp, lm = lam.copy(), lam.copy()
        lp[l] += h
        lm[l] -= h
        fd = (cp_ref.objective_grad(eptr, eidx, n, r, lp, A)[0] - cp_ref.objective_grad(eptr, eidx, n, r, lm, A)[0]) / (2 * h)
        assert abs(fd - dl[l]) <= 1e-6 * max(1.0, abs(fd))
    for v, l in itertools.product(range(n), range(R)):
        Ap, Am = A.copy(), A.copy()
        Ap[v, l] += h
        Am[v, l] -= h
        fd = (cp_ref.objective_grad(eptr, eidx, n, r, lam, Ap)[0] - cp_ref.objective_grad(eptr, eidx, n, r, lam, Am)[0]) / (2 * h)
        assert abs(fd - dA[v, l]) <= 1e-6 * max(1.0, abs(fd))


def test_graph_case_eigendecomposition_is_exact():
    # r = 2: B is the adjacency matrix; its eigendecomposition is an exact
    # symmetric CP of rank n: zero objective and zero gradient
    rng = np.random.default_rng(7)
    n = 9
    edges = sorted({tuple(sorted(rng.choice(n, size=2, replace=False))) for _ in range(20)})
    eptr, eidx = _csr(edges)
    Adj = np.zeros((n, n))
    for a, b in edges:
        Adj[a, b] = Adj[b, a] = 1.0
    ev, V = np.linalg.eigh(Adj)
    f, dl, dA = cp_ref.objective_grad(eptr, eidx, n, 2, ev, V)
    assert abs(f) <= 1e-12 * len(edges)
    assert np.max(np.abs(dl)) <= 1e-12 and np.max(np.abs(dA)) <= 1e-12


def test_descent_decreases_objective():
    rng = np.random.default_rng(11)
    n, m, r, R = 40, 120, 4, 3
    sizes = rng.integers(2, 5, size=m)
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in sizes]
    eptr, eidx = _csr(edges)
    lam0 = np.ones(R)
    A0 = rng.uniform(0.1, 1.0, size=(n, R)) / np.sqrt(n)
    _, _, info = cp_ref.gradient_descent(eptr, eidx, n, r, lam0, A0, iters=15, step=1.0, history=True)
    fs = info["fs"]
    assert all(b <= a for a, b in zip(fs, fs[1:]))
    assert fs[-1] < fs[0] - 1.0 and fs[-1] > 0.0
