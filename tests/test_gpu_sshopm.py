"""GPU parity of the full contraction and the shifted power method
(``sttsv_contract``, ``zeigvec_sshopm``) against the CPU oracle.

Tolerances: contraction, lambda at every iterate, and every entry of the
first iterate 1e-12 relative (FP64 series, all terms non-negative; entries
below 1e-200 absolutely).  Later iterates: every entry at or above 1e-6 of the
largest 1e-12 relative, the rest 1e-12 on the unit vector's scale -- an entry
fed by (r-1)-th powers of other small entries carries r-1 times their relative
error, so rounding differences between two correct runs can grow like
(r-1)^K there; the oracle tests pin the iteration against exact arithmetic
and measure that drift (tests/test_sshopm_oracle_pins.py).  Converged pairs:
lambda 1e-10, x 1e-6 absolute (the two runs may stop one update apart).
"""
import sys

import numpy as np
import pytest

from oracle import sshopm_ref
from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed(seed, n, m, r, kmin, kmax):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m)
    eptr, eidx = wl.uniform_members(rng, n, sizes)
    return eptr, eidx, wl.uniform_x(rng, n)


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _close(a, b, rtol):
    """|a - b| <= rtol |b| entrywise, entries of a unit vector below 1e-200
    (products there can underflow differently) checked absolutely."""
    return bool(np.all(np.abs(a - b) <= rtol * np.abs(b) + 1e-200))


CASES = [("r5", 31, 400, 2001, 5, 1, 5), ("r12", 32, 700, 2501, 12, 2, 12), ("r25", 33, 1500, 3001, 25, 1, 25)]


@pytest.mark.parametrize("name,seed,n,m,r,kmin,kmax", CASES)
def test_contract_matches_oracle(torch_cuda, name, seed, n, m, r, kmin, kmax):
    import paper_2311_08595_amd as st
    _say(f"[contract] {name}")
    eptr, eidx, x = _mixed(seed, n, m, r, kmin, kmax)
    ref = sshopm_ref.contract(eptr, eidx, n, r, x)
    with st.Plan(eptr, eidx, n, r) as plan:
        xd = torch_cuda.tensor(x, dtype=torch_cuda.float64, device="cuda")
        v1, y = plan.contract(xd)
        v2, _ = plan.contract(xd)
        y = y.cpu().numpy()
    assert abs(v1 - ref) <= 1e-12 * abs(ref)
    assert v1 == v2
    yr = sr.sttsv(eptr, eidx, n, r, x)
    nz = yr != 0
    assert _rel(y[nz], yr[nz]) <= 1e-12


@pytest.mark.parametrize("shift", [0.0, 2.0])
@pytest.mark.parametrize("name,seed,n,m,r,kmin,kmax", CASES)
def test_sshopm_iterates_match_oracle(torch_cuda, name, seed, n, m, r, kmin, kmax, shift):
    """After exactly K updates (tol = 0) x and lambda match the oracle's K-th
    iterate.  alpha = shift * lambda_0 (the shift has to be on the scale of
    B x^r, which is ~ d n^(-(r-2)/2) for unit x)."""
    import paper_2311_08595_amd as st
    _say(f"[sshopm] iterates {name} shift {shift}")
    eptr, eidx, x0 = _mixed(seed, n, m, r, kmin, kmax)
    alpha = shift * sshopm_ref.contract(eptr, eidx, n, r, x0 / np.linalg.norm(x0))
    _, hist = sshopm_ref.sshopm(eptr, eidx, n, r, x0, alpha=alpha, tol=0.0, max_iter=12, history=True)
    with st.Plan(eptr, eidx, n, r) as plan:
        x0d = torch_cuda.tensor(x0, dtype=torch_cuda.float64, device="cuda")
        for K in (0, 1, 3, 5, 12):
            xk, info = plan.zeig_sshopm(x0d, alpha=alpha, tol=0.0, max_iter=K, raise_on_notconv=False)
            xr, lr = hist["history"][K]
            xk = xk.cpu().numpy()
            assert info["iterations"] == K
            bad = np.abs(xk - xr) > 1e-12 * np.abs(xr) + 1e-200
            _say(f"  K={K}: lambda rel err {abs(info['lambda_'] - lr) / lr:.2e}, "
                 f"max abs err {np.max(np.abs(xk - xr)):.2e}, entries off {int(bad.sum())}"
                 + (f" (e.g. {xk[bad][:3]} vs {xr[bad][:3]})" if bad.any() else ""))
            assert abs(info["lambda_"] - lr) <= 1e-12 * lr
            if K <= 1:
                assert not bad.any()
            else:
                big = np.abs(xr) >= 1e-6 * np.max(np.abs(xr))
                assert not bad[big].any(), np.flatnonzero(bad & big)[:5]
                assert np.max(np.abs(xk - xr)) <= 1e-12


def test_sshopm_converges_to_oracle_pair(torch_cuda):
    import paper_2311_08595_amd as st
    n, m, r = 800, 4001, 8
    eptr, eidx, x0 = _mixed(41, n, m, r, 2, 8)
    alpha = sshopm_ref.contract(eptr, eidx, n, r, x0 / np.linalg.norm(x0))
    xr, ir = sshopm_ref.sshopm(eptr, eidx, n, r, x0, alpha=alpha, tol=1e-14, max_iter=2000)
    assert ir["converged"]
    with st.Plan(eptr, eidx, n, r) as plan:
        xg, ig = plan.zeig_sshopm(torch_cuda.tensor(x0, dtype=torch_cuda.float64, device="cuda"),
                                  alpha=alpha, tol=1e-14, max_iter=2000)
        xg = xg.cpu().numpy()
    _say(f"[sshopm] converged: {ig['iterations']} vs {ir['iterations']} updates, residual {ig['residual']:.2e}")
    assert ig["converged"]
    assert abs(ig["lambda_"] - ir["lambda_"]) <= 1e-10 * ir["lambda_"]
    assert float(np.max(np.abs(xg - xr))) <= 1e-6
    assert abs(np.linalg.norm(xg) - 1.0) <= 1e-13
    assert ig["residual"] <= 1e-5 * ig["lambda_"]


def test_sshopm_regular_and_graph_cases(torch_cuda):
    import paper_2311_08595_amd as st
    # regular hypergraph: 1/sqrt(n) is a fixed point, lambda = d n^(-(r-2)/2)
    n, r = 19, 5
    edges = [tuple((s + j) % n for j in range(k)) for k in (2, 3, 4, 5) for s in range(n)]
    eptr = np.zeros(len(edges) + 1, dtype=np.int64)
    eptr[1:] = np.cumsum([len(e) for e in edges])
    eidx = np.array([v for e in edges for v in e], dtype=np.int32)
    with st.Plan(eptr, eidx, n, r) as plan:
        x, info = plan.zeig_sshopm(None, alpha=0.5, tol=1e-14)
        x = x.cpu().numpy()
    lam = 14.0 * n ** (-(r - 2) / 2)
    assert info["iterations"] == 1
    assert abs(info["lambda_"] - lam) <= 1e-14 * lam
    np.testing.assert_allclose(x, 1.0 / np.sqrt(n), rtol=1e-14)


def test_sshopm_errors(torch_cuda):
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import _lib
    eptr, eidx, _ = _mixed(5, 50, 120, 4, 1, 4)
    with st.Plan(eptr, eidx, 50, 4) as plan:
        with pytest.raises(Exception):
            plan.zeig_sshopm(None, alpha=-1.0)
        z = torch_cuda.zeros(50, dtype=torch_cuda.float64, device="cuda")
        with pytest.raises(Exception):
            plan.zeig_sshopm(z, alpha=1.0)          # zero start: ENUMERIC, nothing launched after the norm
        _, info = plan.zeig_sshopm(None, alpha=1.0, tol=0.0, max_iter=3, raise_on_notconv=False)
        assert info["status"] == _lib.STTSV_ENOTCONV and info["iterations"] == 3


def test_sshopm_graph_reuse_across_calls_and_retune(torch_cuda):
    """The K-update graph is captured once per plan with the shift and the
    tolerance in the device control block: calls with other shifts, stopping
    rules and start vectors on one plan, and a call after autotuning (which
    drops the graph), give bit for bit what a fresh plan gives."""
    import paper_2311_08595_amd as st
    _say("[sshopm] graph reuse")
    eptr, eidx, x0 = _mixed(11, 300, 1500, 6, 1, 6)
    n, r = 300, 6
    lam0 = sshopm_ref.contract(eptr, eidx, n, r, x0 / np.linalg.norm(x0))
    calls = [(2.0 * lam0, 0.0, 5, True), (0.0, 0.0, 11, True), (lam0, 1e-12, 400, False), (3.0 * lam0, 0.0, 1, True)]

    def run(plan, alpha, tol, k, from_x0):
        x0d = torch_cuda.tensor(x0, dtype=torch_cuda.float64, device="cuda")
        x, info = plan.zeig_sshopm(x0d if from_x0 else None, alpha=alpha, tol=tol, max_iter=k,
                                   raise_on_notconv=False)
        assert np.array_equal(x0d.cpu().numpy(), x0)          # the start vector is not written
        return x.cpu().numpy().tobytes(), info["lambda_"], info["iterations"]

    fresh = []
    for c in calls:
        with st.Plan(eptr, eidx, n, r) as plan:
            fresh.append(run(plan, *c))
    with st.Plan(eptr, eidx, n, r) as plan:
        for c, want in zip(calls, fresh):
            assert run(plan, *c) == want
        plan.autotune(torch_cuda.tensor(x0, dtype=torch_cuda.float64, device="cuda"), reps=1)
        for c, want in zip(calls, fresh):
            assert run(plan, *c) == want
