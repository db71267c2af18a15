"""Full-size workloads through the same launch sequence the benchmark times,
checked against the oracle on sampled vertices (the oracle sums each sampled
vertex's edge terms one by one) and by properties that hold at any size.

Samples: the highest-degree vertices (the hub's list spans several reduction
levels), random vertices, and isolated vertices (y = 0 exactly).
"""
import sys

import numpy as np
import pytest

from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(y, ref):
    den = np.where(ref != 0, np.abs(ref), 1.0)
    return float(np.max(np.abs(y - ref) / den))


def _sample(deg, seed, count=48, top=4):
    rng = np.random.default_rng(seed)
    hubs = np.argsort(-deg, kind="stable")[:top]
    rnd = rng.choice(len(deg), size=count, replace=False)
    iso = np.flatnonzero(deg == 0)[:2]
    return np.unique(np.concatenate([hubs, rnd, iso]))


def _check_apply(w, seed):
    import torch
    import paper_2311_08595_amd as st
    n, r = w["n"], w["r"]
    deg = np.bincount(w["eidx"], minlength=n)
    nodes = _sample(deg, seed)
    _say(f"  oracle on {len(nodes)} sampled vertices (max degree {deg[nodes].max()})")
    ref = sr.sttsv_at(w["eptr"], w["eidx"], n, r, w["x"], nodes)
    with st.Plan(w["eptr"], w["eidx"], n, r) as plan:
        xd = torch.tensor(w["x"], dtype=torch.float64, device="cuda")
        for prec in ("fp64", "fp32"):
            y = plan.apply(xd, precision=prec).cpu().numpy()
            err = _relerr(y[nodes], ref)
            _say(f"  {prec}: max rel err {err:.2e}")
            assert err <= TOL[prec], (prec, err)
            iso = nodes[deg[nodes] == 0]
            assert np.all(y[iso] == 0.0)


def test_zipf_full_size_sampled():
    # n = 1e6, m = 5e6, sizes ~ k^-2.5 on [2, 25], r = 25, Zipf(1.0) membership
    _say("[fullsize] zipf n=1e6 m=5e6 r=25")
    _check_apply(wl.zipf_powerlaw(), seed=1)


def test_heavy_tail_full_size_sampled():
    # n = 2e5, m = 2e6, 99 % of sizes geometric on [2, 8], 1 % uniform on [9, 50], r = 50
    _say("[fullsize] heavy tail n=2e5 m=2e6 r=50")
    _check_apply(wl.heavy_tail(), seed=2)


def test_batched_full_size_sampled():
    # 256 graphs, n log-uniform in [1e3, 1e5], m = 5n, r in {3..12}, one plan;
    # every 32nd graph checked on sampled vertices
    import torch
    import paper_2311_08595_amd as st
    _say("[fullsize] batched 256 graphs")
    gs, xs = [], []
    for g in range(256):
        w = wl.batch_graph(g)
        gs.append((w["eptr"], w["eidx"], w["n"], w["r"]))
        xs.append(w["x"])
    with st.Plan.batch(gs) as pb:
        x = torch.tensor(np.concatenate(xs), dtype=torch.float64, device="cuda")
        y = pb.apply(x).cpu().numpy()
        offs = [pb.graph_info(g)["voff"] for g in range(len(gs))]
    for g in range(0, 256, 32):
        eptr, eidx, n, r = gs[g]
        deg = np.bincount(eidx, minlength=n)
        nodes = _sample(deg, seed=g, count=16, top=2)
        ref = sr.sttsv_at(eptr, eidx, n, r, xs[g], nodes)
        err = _relerr(y[offs[g] + nodes], ref)
        assert err <= TOL["fp64"], (g, err)


def test_zipf_full_size_solve_is_an_eigenvector():
    # Alg. 1 to 1e-8 on the largest component of the benchmark hypergraph:
    # at sampled vertices the oracle's (B x^(r-1))_v / x_v^(r-1) lies within
    # the solver's [lambda_min, lambda_max] (up to rounding), which is 1e-8 wide
    import torch
    import paper_2311_08595_amd as st
    _say("[fullsize] solve on the zipf LCC")
    w = wl.zipf_powerlaw()
    eptr, eidx, n, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
    r = w["r"]
    with st.Plan(eptr, eidx, n, r) as plan:
        x, info = plan.solve(tol=1e-8)
    assert info["converged"]
    x = x.cpu().numpy()
    assert np.all(x > 0) and abs(x.sum() - 1.0) < 1e-12
    xs = x / x.max()                       # Eq. (2) is homogeneous: scale to avoid underflow
    deg = np.bincount(eidx, minlength=n)
    nodes = _sample(deg, seed=3, count=32, top=4)
    yv = sr.sttsv_at(eptr, eidx, n, r, xs, nodes)
    lam = yv / xs[nodes] ** (r - 1)
    lo, hi = info["lambda_min"], info["lambda_max"]
    _say(f"  lambda in [{lo:.12e}, {hi:.12e}], sampled [{lam.min():.12e}, {lam.max():.12e}]")
    assert (hi - lo) / lo < 1e-8
    assert lam.min() >= lo * (1 - 1e-10) and lam.max() <= hi * (1 + 1e-10)
