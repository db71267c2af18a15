"""Batched plans: many hypergraphs of different n, m and r in one plan."""
import sys

import numpy as np
import pytest

from oracle import nqz_ref
from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _graphs(count, seed=0, lcc=True):
    out = []
    for g in range(count):
        w = wl.batch_graph(g, base_seed=900 + seed, lo=2.3, hi=3.3)
        eptr, eidx, n = w["eptr"], w["eidx"], w["n"]
        if lcc:
            eptr, eidx, n, _ = wl.largest_component(eptr, eidx, n)
        out.append((eptr, eidx, n, w["r"]))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_apply_bitwise_equals_single(prec):
    import torch
    import paper_2311_08595_amd as st
    gs = _graphs(7, seed=1, lcc=False)
    # add a graph with size-1 edges and one of order 2 (graph case)
    gs.append((np.array([0, 1, 3, 5, 6], np.int64), np.array([0, 0, 1, 1, 2, 3], np.int32), 4, 4))
    gs.append((np.array([0, 2, 4, 6], np.int64), np.array([0, 1, 1, 2, 2, 0], np.int32), 3, 2))
    rng = np.random.default_rng(3)
    xs = [1.0 - rng.random(g[2]) for g in gs]
    xcat = torch.tensor(np.concatenate(xs), dtype=torch.float64, device="cuda")
    with st.Plan.batch(gs) as pb:
        yb = pb.apply(xcat, precision=prec).cpu().numpy()
        offs = [pb.graph_info(g)["voff"] for g in range(len(gs))]
    for g, (eptr, eidx, n, r) in enumerate(gs):
        with st.Plan(eptr, eidx, n, r) as p1:
            y1 = p1.apply(torch.tensor(xs[g], dtype=torch.float64, device="cuda"), precision=prec).cpu().numpy()
        assert yb[offs[g]:offs[g] + n].tobytes() == y1.tobytes(), g
        ref = sr.sttsv(eptr, eidx, n, r, xs[g])
        tol = 1e-12 if prec == "fp64" else 1e-5
        assert np.max(np.abs(y1 - ref) / np.where(ref != 0, np.abs(ref), 1)) <= tol


def test_batch_flags_keep_bits():
    # prefix reuse (runs never cross graphs: they share their first two
    # vertices) and the one-stream launch order leave every bit of y alone
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import _lib
    gs = []
    for g in range(5):
        w = wl.zipf_powerlaw(seed=70 + g, n=40000, m=200000)
        gs.append((w["eptr"], w["eidx"], w["n"], w["r"]))
    rng = np.random.default_rng(9)
    x = torch.tensor(1.0 - rng.random(sum(g[2] for g in gs)), dtype=torch.float64, device="cuda")
    out = {}
    for flags in (0, _lib.FLAG_PREFIX_REUSE, _lib.FLAG_ONE_STREAM):
        with st.Plan.batch(gs, flags=flags) as pb:
            if flags == _lib.FLAG_PREFIX_REUSE:
                assert np.any(pb.query(_lib.Q_BUCKET_RUNS) > 0)
            if flags == 0:
                assert pb.info()["lanes"] > 1
            out[flags] = pb.apply(x).cpu().numpy().tobytes()
    assert out[0] == out[_lib.FLAG_PREFIX_REUSE] == out[_lib.FLAG_ONE_STREAM]


@pytest.mark.parametrize("schedule", ["fp64", "fp32_fp64"])
def test_batch_solve_matches_single_and_oracle(schedule):
    import torch
    import paper_2311_08595_amd as st
    gs = _graphs(6, seed=2)
    with st.Plan.batch(gs) as pb:
        xb, infos = pb.solve_batch(tol=1e-10, schedule=schedule)
        xb = xb.cpu().numpy()
        offs = [pb.graph_info(g)["voff"] for g in range(len(gs))]
    iters = [i["iterations"] for i in infos]
    _say(f"  per-graph iterations {iters}")
    for g, (eptr, eidx, n, r) in enumerate(gs):
        with st.Plan(eptr, eidx, n, r) as p1:
            x1, i1 = p1.solve(tol=1e-10, schedule=schedule)
        x1 = x1.cpu().numpy()
        assert infos[g]["converged"] and infos[g]["iterations"] == i1["iterations"], (g, infos[g], i1)
        assert xb[offs[g]:offs[g] + n].tobytes() == x1.tobytes(), g
        if schedule == "fp64" and g < 3:
            o = nqz_ref.nqz(eptr, eidx, n, r, tol=1e-10)
            assert o["iterations"] == i1["iterations"]
            np.testing.assert_allclose(x1, o["x"], rtol=1e-11)


def test_batch_warm_start_and_masking():
    import torch
    import paper_2311_08595_amd as st
    gs = _graphs(4, seed=3)
    # warm start graph 0 at its converged vector: it stops after one
    # iteration while the others keep going; its slice must stay frozen
    with st.Plan.batch(gs) as pb:
        x_plain, inf_plain = pb.solve_batch(tol=1e-11)
        x0 = x_plain.clone()
        n0 = gs[0][2]
        x0[n0:] = 1.0
        xw, inf_w = pb.solve_batch(tol=1e-10, x0=x0)
    assert inf_w[0]["iterations"] <= 2 < max(i["iterations"] for i in inf_w[1:])
    np.testing.assert_allclose(xw[:n0].cpu().numpy(), x_plain[:n0].cpu().numpy(), rtol=1e-9)
