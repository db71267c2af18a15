"""Edge-weighted hypergraphs H = (V, E, w) (Sec. II; Alg. 2 takes w as
input) on the GPU against the CPU oracle: every blowup of e carries
w(e)/|beta(e)|.  Tolerances as for the unweighted path: FP64 series 1e-12,
FP32 series 1e-5 relative per vertex."""
import sys

import numpy as np
import pytest

from oracle import nqz_ref, sshopm_ref
from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(y, ref):
    den = np.where(ref != 0, np.abs(ref), 1.0)
    return float(np.max(np.abs(y - ref) / den)) if len(ref) else 0.0


def _weighted(seed, n, m, r, kmin, kmax):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m)
    eptr, eidx = wl.uniform_members(rng, n, sizes)
    x = wl.uniform_x(rng, n)
    w = np.exp(rng.uniform(np.log(0.05), np.log(20.0), size=m))
    return eptr, eidx, x, w


CASES = [("r5", 61, 400, 3001, 5, 1, 5), ("r25", 62, 2000, 6007, 25, 1, 25), ("r50", 63, 3000, 5003, 50, 1, 50)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "naive"])
@pytest.mark.parametrize("name,seed,n,m,r,kmin,kmax", CASES)
def test_weighted_apply_matches_oracle(prec, name, seed, n, m, r, kmin, kmax):
    import torch
    import paper_2311_08595_amd as st
    _say(f"[weighted apply] {name} {prec}")
    eptr, eidx, x, w = _weighted(seed, n, m, r, kmin, kmax)
    ref = sr.sttsv(eptr, eidx, n, r, x, w=w)
    with st.Plan(eptr, eidx, n, r, weights=w) as plan:
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        y = (plan.apply_naive(xd) if prec == "naive" else plan.apply(xd, precision=prec)).cpu().numpy()
    err = _relerr(y, ref)
    _say(f"  max rel err {err:.3e}")
    assert err <= TOL["fp64" if prec == "naive" else prec]


def test_weights_equal_to_sizes_give_the_default():
    import torch
    import paper_2311_08595_amd as st
    eptr, eidx, x, _ = _weighted(64, 500, 4001, 9, 1, 9)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    with st.Plan(eptr, eidx, 500, 9) as a, st.Plan(eptr, eidx, 500, 9, weights=np.diff(eptr).astype(float)) as b:
        ya, yb = a.apply(xd).cpu().numpy(), b.apply(xd).cpu().numpy()
    assert _relerr(yb, ya) <= 4e-16


def test_weighted_batch_equals_single_plans():
    import torch
    import paper_2311_08595_amd as st
    g0 = _weighted(65, 300, 2000, 7, 1, 7)
    g1 = _weighted(66, 500, 3000, 12, 2, 12)
    x = np.concatenate([g0[2], g1[2]])
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    with st.Plan.batch([(g0[0], g0[1], 300, 7, g0[3]), (g1[0], g1[1], 500, 12)]) as pb:
        yb = pb.apply(xd).cpu().numpy()
    with st.Plan(g0[0], g0[1], 300, 7, weights=g0[3]) as p0, st.Plan(g1[0], g1[1], 500, 12) as p1:
        y0 = p0.apply(xd[:300].contiguous()).cpu().numpy()
        y1 = p1.apply(xd[300:].contiguous()).cpu().numpy()
    assert yb[:300].tobytes() == y0.tobytes() and yb[300:].tobytes() == y1.tobytes()
    assert _relerr(y0, sr.sttsv(g0[0], g0[1], 300, 7, g0[2], w=g0[3])) <= 1e-12


def test_weighted_solve_and_contraction_match_oracle():
    import torch
    import paper_2311_08595_amd as st
    w0 = wl.zipf_powerlaw(seed=67, n=3000, m=15000, kmax=12)
    eptr, eidx, n, _ = wl.largest_component(w0["eptr"], w0["eidx"], w0["n"])
    r = 12
    w = np.exp(np.random.default_rng(68).uniform(np.log(0.1), np.log(10.0), size=len(eptr) - 1))
    ref = nqz_ref.nqz(eptr, eidx, n, r, tol=0.0, max_iter=4, history=True, w=w)
    x = np.random.default_rng(69).uniform(0.1, 1.0, n)
    with st.Plan(eptr, eidx, n, r, weights=w) as plan:
        for t in (1, 4):
            xs, info = plan.solve(tol=1e-300, max_iter=t, raise_on_notconv=False)
            err = float(np.max(np.abs(xs.cpu().numpy() - ref["xs"][t - 1]) / ref["xs"][t - 1]))
            _say(f"[weighted solve] iterate {t}: max rel err {err:.2e}")
            assert info["iterations"] == t and err <= 1e-12
        v, _ = plan.contract(torch.tensor(x, dtype=torch.float64, device="cuda"))
    c = sshopm_ref.contract(eptr, eidx, n, r, x, w=w)
    assert abs(v - c) <= 1e-12 * abs(c)
