"""GPU parity of the NAIVE baseline (Alg. 3, ``sttsv_apply_naive``) against
the CPU oracle, and against the memoised path on the paper's synthetic sets
S1-S4 (n=2500, m=25000, sizes 5, 10, ..., N_k, r = N_k).

Tolerance: max relative error per vertex 1e-12 (FP64, all terms
non-negative); naive vs memoised 2e-12 (each within 1e-12 of the exact value).
"""
import sys

import numpy as np
import pytest

from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(y, ref):
    den = np.where(ref != 0, np.abs(ref), 1.0)
    return float(np.max(np.abs(y - ref) / den)) if len(ref) else 0.0


def _mixed(seed, n, m, r, kmin, kmax):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m)
    eptr, eidx = wl.uniform_members(rng, n, sizes)
    return eptr, eidx, wl.uniform_x(rng, n)


# every size 1..r present (size-1 edges included), several 64-thread tiles per
# bucket with ragged tails; r covers every series capacity 8, 16, ..., 64
CASES = [
    ("r5", 11, 400, 3001, 5, 1, 5),
    ("r12", 12, 600, 2503, 12, 1, 12),
    ("r25", 13, 2000, 4007, 25, 1, 25),
    ("r33_r_above_max_size", 14, 1500, 3001, 33, 1, 20),
    ("r41", 15, 2000, 2003, 41, 1, 41),
    ("r50", 16, 3000, 2501, 50, 1, 50),
    ("r57", 17, 3000, 1999, 57, 1, 57),
    ("r64", 18, 3000, 2003, 64, 1, 64),
]


@pytest.mark.parametrize("name,seed,n,m,r,kmin,kmax", CASES)
def test_naive_matches_oracle(torch_cuda, name, seed, n, m, r, kmin, kmax):
    import paper_2311_08595_amd as st
    _say(f"[naive] {name}")
    eptr, eidx, x = _mixed(seed, n, m, r, kmin, kmax)
    ref = sr.sttsv(eptr, eidx, n, r, x)
    with st.Plan(eptr, eidx, n, r) as plan:
        xd = torch_cuda.tensor(x, dtype=torch_cuda.float64, device="cuda")
        y1 = plan.apply_naive(xd)
        y2 = plan.apply_naive(xd)
        torch_cuda.cuda.synchronize()
        y1, y2 = y1.cpu().numpy(), y2.cpu().numpy()
    err = _relerr(y1, ref)
    _say(f"  max rel err {err:.3e}")
    assert err <= TOL
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))   # reproducible bit for bit
    assert np.all(y1[ref == 0] == 0)


@pytest.mark.parametrize("nk", [30, 40, 50, 60])
def test_paper_synthetic_naive_vs_memoised(torch_cuda, nk):
    """S1-S4 at full size: the naive and memoised FP64 paths agree on every
    vertex, and both match the oracle on sampled vertices."""
    import paper_2311_08595_amd as st
    d = wl.paper_synthetic(nk)
    _say(f"[naive] {d['name']}")
    n, r = d["n"], d["r"]
    with st.Plan(d["eptr"], d["eidx"], n, r) as plan:
        xd = torch_cuda.tensor(d["x"], dtype=torch_cuda.float64, device="cuda")
        yn = plan.apply_naive(xd).cpu().numpy()
        ym = plan.apply(xd, precision="fp64").cpu().numpy()
    assert _relerr(yn, ym) <= 2 * TOL
    nodes = np.random.default_rng(nk).choice(n, 16, replace=False)
    ref = sr.sttsv_at(d["eptr"], d["eidx"], n, r, d["x"], nodes)
    e_naive, e_memo = _relerr(yn[nodes], ref), _relerr(ym[nodes], ref)
    _say(f"  sampled: naive {e_naive:.3e}, memoised {e_memo:.3e}")
    assert e_naive <= TOL and e_memo <= TOL


def test_naive_batched_plan(torch_cuda):
    """A batched plan (graphs of different r in one plan): each graph's block
    of y matches its own oracle."""
    import paper_2311_08595_amd as st
    shapes = [(300, 1501, 4), (500, 2003, 17), (700, 1203, 40)]
    descs, xs = [], []
    for g, (n, m, r) in enumerate(shapes):
        eptr, eidx, x = _mixed(21 + g, n, m, r, 1, r)
        descs.append((eptr, eidx, n, r))
        xs.append(x)
    with st.Plan.batch(descs) as plan:
        xd = torch_cuda.tensor(np.concatenate(xs), dtype=torch_cuda.float64, device="cuda")
        y = plan.apply_naive(xd).cpu().numpy()
    off = 0
    for (eptr, eidx, n, r), x in zip(descs, xs):
        ref = sr.sttsv(eptr, eidx, n, r, x)
        assert _relerr(y[off:off + n], ref) <= TOL
        off += n


def test_naive_edge_cases(torch_cuda):
    """One edge of size r (window 1), the graph case r=2 with isolated
    vertices (exact zeros), size-1 edges, x with zeros."""
    import paper_2311_08595_amd as st

    def run(eptr, eidx, n, r, x):
        with st.Plan(np.asarray(eptr, dtype=np.int64), np.asarray(eidx, dtype=np.int32), n, r) as plan:
            xd = torch_cuda.tensor(np.asarray(x, dtype=np.float64), device="cuda")
            return plan.apply_naive(xd).cpu().numpy()

    y = run([0, 4], [0, 1, 2, 3], 4, 4, [0.5, 2.0, 3.0, 0.25])
    np.testing.assert_allclose(y, [2 * 3 * 0.25, 0.5 * 3 * 0.25, 0.5 * 2 * 0.25, 0.5 * 2 * 3], rtol=1e-15)
    y = run([0, 2, 4, 6, 8], [0, 1, 1, 2, 2, 0, 0, 1], 5, 2, [1.0, 2.0, 3.0, 4.0, 5.0])
    np.testing.assert_array_equal(y, [2 * 2.0 + 3.0, 2 * 1.0 + 3.0, 1.0 + 2.0, 0.0, 0.0])
    y = run([0, 1, 2, 3], [0, 1, 1], 2, 6, [1.5, 0.5])
    np.testing.assert_allclose(y, [1.5 ** 5, 2 * 0.5 ** 5], rtol=1e-15)
    n, r = 50, 6
    eptr, eidx = [0, 3, 5, 6], [0, 4, 9, 4, 7, 20]
    x = np.linspace(0.0, 1.0, n)
    ref = sr.sttsv(np.array(eptr), np.array(eidx), n, r, x)
    y = run(eptr, eidx, n, r, x)
    assert _relerr(y, ref) <= TOL
    assert np.all(y[ref == 0] == 0)
