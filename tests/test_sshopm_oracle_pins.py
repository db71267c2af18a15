"""Pins of the SS-HOPM and full-contraction oracle against closed forms,
brute-force blowup entries and a library eigensolver."""
import math
import random
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from oracle import blowup as bl
from oracle import sshopm_ref
from oracle import sttsv_ref as sr


def _csr(edges):
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int32)
    return eptr, eidx


def test_contraction_equals_entry_enumeration():
    # B x^r summed over every blowup entry (exact rationals) for a tiny
    # non-uniform hypergraph, n <= 8, r <= 5
    rng = random.Random(3)
    n, r = 7, 5
    edges = []
    while len(edges) < 6:
        k = rng.randint(1, r)
        e = tuple(sorted(rng.sample(range(n), k)))
        edges.append(e)
    x = [rng.uniform(0.1, 1.0) for _ in range(n)]
    B = bl.blowup_entries(edges, r)
    exact = float(bl.full_contraction_from_entries(B, r, [Fraction(v) for v in x]))
    eptr, eidx = _csr(edges)
    got = sshopm_ref.contract(eptr, eidx, n, r, np.array(x))
    assert abs(got - exact) <= 1e-14 * abs(exact)


def test_graph_case_is_perron_eigenpair():
    # r = 2: B = A, Z-eigenpairs are eigenpairs of A; from a positive start
    # the shifted power method reaches the Perron pair (spectral radius).
    rng = np.random.default_rng(5)
    n = 30
    edges = {(i, (i + 1) % n) for i in range(n)}                     # even cycle: bipartite
    while len(edges) < 70:
        a, b = rng.choice(n, size=2, replace=False)
        edges.add((min(a, b), max(a, b)))
    edges = sorted(edges)
    eptr, eidx = _csr(edges)
    x, info = sshopm_ref.sshopm(eptr, eidx, n, 2, np.ones(n), alpha=1.0, tol=1e-15, max_iter=20000)
    i = np.array([e[0] for e in edges] + [e[1] for e in edges])
    j = np.array([e[1] for e in edges] + [e[0] for e in edges])
    A = sp.coo_matrix((np.ones(len(i)), (i, j)), shape=(n, n)).toarray()
    w, V = np.linalg.eigh(A)
    v = np.abs(V[:, -1])
    assert abs(info["lambda_"] - w[-1]) <= 1e-12 * w[-1]
    np.testing.assert_allclose(x, v / np.linalg.norm(v), rtol=1e-6)


def test_regular_hypergraph_fixed_point():
    # every vertex in k cyclic intervals of size k for k = 2..5 (degree 14);
    # B 1^(r-1) = d 1 (Sec. II), so x = 1/sqrt(n) gives B x^(r-1) = d n^(-(r-1)/2) 1
    # = lambda x with lambda = d n^(-(r-2)/2), and the method stays there.
    n, r = 19, 5
    edges = [tuple((s + j) % n for j in range(k)) for k in (2, 3, 4, 5) for s in range(n)]
    eptr, eidx = _csr(edges)
    x, info = sshopm_ref.sshopm(eptr, eidx, n, r, np.ones(n), alpha=0.5, tol=1e-14)
    lam = 14.0 * n ** (-(r - 2) / 2)
    assert info["iterations"] == 1 and info["converged"]
    assert abs(info["lambda_"] - lam) <= 1e-14 * lam
    np.testing.assert_allclose(x, 1.0 / math.sqrt(n), rtol=1e-14)
    assert info["residual"] <= 1e-14 * lam


def test_converged_pair_is_a_z_eigenpair():
    # random non-uniform hypergraph: at convergence ||x|| = 1, B x^(r-1) = lambda x
    # to the tolerance, and lambda = B x^r by the entry-free contraction
    rng = np.random.default_rng(9)
    n, m, r = 60, 300, 6
    edges = [tuple(rng.choice(n, size=k, replace=False)) for k in rng.integers(1, r + 1, size=m)]
    eptr, eidx = _csr(edges)
    x, info = sshopm_ref.sshopm(eptr, eidx, n, r, rng.random(n) + 0.1, alpha=1.0, tol=1e-15, max_iter=5000)
    assert info["converged"]
    assert abs(np.linalg.norm(x) - 1.0) < 1e-14
    y = sr.sttsv(eptr, eidx, n, r, x)
    assert np.linalg.norm(y - info["lambda_"] * x) <= 1e-6 * info["lambda_"]
    assert abs(sshopm_ref.contract(eptr, eidx, n, r, x) - info["lambda_"]) <= 1e-13 * info["lambda_"]
    # lambda_k never decreases (convex shift; Kolda and Mayo's monotonicity)
    _, hinfo = sshopm_ref.sshopm(eptr, eidx, n, r, rng.random(n) + 0.1, alpha=float(r), tol=0.0,
                                 max_iter=40, history=True)
    lams = [lam for _, lam in hinfo["history"]]
    assert all(b >= a * (1 - 1e-14) for a, b in zip(lams, lams[1:]))


def _exact_sshopm(edges, n, r, x0, alpha, K):
    """SS-HOPM with every blowup entry listed (Sec. II) and 80-digit decimal
    arithmetic (square roots included): the iterates x_0..x_K, exact far
    beyond FP64."""
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 80
        B = {t: Decimal(v.numerator) / Decimal(v.denominator) for t, v in bl.blowup_entries(edges, r).items()}

        def ttsv(x):
            y = [Decimal(0)] * n
            for t, val in B.items():
                p = val
                for i in t[1:]:
                    p *= x[i]
                y[t[0]] += p
            return y

        x = [Decimal(float(v)) for v in x0]
        nr = sum(v * v for v in x).sqrt()
        x = [v / nr for v in x]
        a = Decimal(float(alpha))
        hist = [[float(v) for v in x]]
        y = ttsv(x)
        for _ in range(K):
            w = [y[i] + a * x[i] for i in range(n)]
            nr = sum(v * v for v in w).sqrt()
            x = [v / nr for v in w]
            y = ttsv(x)
            hist.append([float(v) for v in x])
    return hist


def test_sshopm_matches_exact_iteration():
    # r = 5, n = 8: the FP64 oracle's iterates against the exact iteration.
    # Every entry of x_K keeps a relative error of a few ulps; the bound that
    # holds in general grows like (r-1)^K (each entry of B x^(r-1) is a sum of
    # positive products of r-1 entries, so relative errors can be multiplied
    # by r-1 per update), and the observed errors stay far inside it here.
    r, n, K = 5, 8, 5
    u = 2.0 ** -53
    worst = []
    for seed in range(4):
        rng = random.Random(seed)
        edges = [tuple(sorted(rng.sample(range(n), rng.randint(2, r)))) for _ in range(10)]
        x0 = np.array([rng.uniform(0.05, 1.0) for _ in range(n)])
        eptr, eidx = _csr(edges)
        for alpha in (0.0, 0.5):
            _, h = sshopm_ref.sshopm(eptr, eidx, n, r, x0, alpha=alpha, tol=0.0, max_iter=K, history=True)
            ex = _exact_sshopm(edges, n, r, x0, alpha, K)
            for k in range(K + 1):
                xe = np.array(ex[k])
                rel = float(np.max(np.abs(h["history"][k][0] - xe) / np.abs(xe)))
                assert rel <= 64 * u * (r - 1) ** k, (seed, alpha, k, rel)
                assert rel <= 1e-14, (seed, alpha, k, rel)
                worst.append(rel)
    assert max(worst) > 0.0


def test_sshopm_rounding_spread_stays_small_on_large_entries():
    # Two correct FP64 runs that differ only by rounding (the start vector
    # moved by one ulp per entry) on the GPU parity cases: after K updates the
    # entries at or above 1e-6 of the largest agree to 1e-13 relative, while
    # far smaller entries (fed by (r-1)-th powers of small entries) may drift
    # further apart relatively -- the reason the GPU test checks those on the
    # unit vector's scale instead.
    from paper_2311_08595_amd import workloads as wl
    small_drift = 0.0
    for seed, n, m, r, kmin, kmax in [(31, 400, 2001, 5, 1, 5), (32, 700, 2501, 12, 2, 12)]:
        g = np.random.default_rng(seed)
        sizes = g.integers(kmin, kmax + 1, size=m)
        eptr, eidx = wl.uniform_members(g, n, sizes)
        x0 = wl.uniform_x(g, n)
        for shift in (0.0, 2.0):
            alpha = shift * sshopm_ref.contract(eptr, eidx, n, r, x0 / np.linalg.norm(x0))
            _, a = sshopm_ref.sshopm(eptr, eidx, n, r, x0, alpha=alpha, tol=0.0, max_iter=12, history=True)
            xp = x0 * (1.0 + np.random.default_rng(5).choice([-1.0, 1.0], n) * 2.0 ** -52)
            _, b = sshopm_ref.sshopm(eptr, eidx, n, r, xp, alpha=alpha, tol=0.0, max_iter=12, history=True)
            for K in (1, 3, 5, 12):
                xa, xb = a["history"][K][0], b["history"][K][0]
                big = np.abs(xa) >= 1e-6 * np.max(np.abs(xa))
                assert np.max(np.abs(xa[big] - xb[big]) / np.abs(xa[big])) <= 1e-13, (seed, shift, K)
                assert np.max(np.abs(xa - xb)) <= 1e-13
                tiny = ~big & (xa > 1e-250)
                if tiny.any():
                    small_drift = max(small_drift, float(np.max(np.abs(xa[tiny] - xb[tiny]) / xa[tiny])))
    assert small_drift > 1e-13
