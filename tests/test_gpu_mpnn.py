"""Warm-start network on the GPU against the FP64 oracle (oracle/mpnn_ref.py).

The oracle is run with the same bfloat16 roundings the kernels make, so the
remaining differences come from FP32 accumulation and from the bf16 roundings
that an FP32-vs-FP64 difference can flip.  Every score, the loss and every
gradient entry is checked against its own bound, carried through the network
by ``mpnn_bounds`` (FP32 summation lengths, bf16 rounding intervals, ReLU
masks that can flip), and every stage of the forward and backward pass is
then checked entry by entry against the oracle's arithmetic on the GPU's own
inputs of that stage (``mpnn_bounds.stage_checks``).
"""
import numpy as np
import pytest

import mpnn_bounds as mb
from oracle import mpnn_ref as mr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu

KF, HID = 16, 64


def to_gpu_params(p):
    W0 = np.zeros((KF, HID))
    W0[:4] = p["W0"]
    parts = [W0, p["b0"], p["W1"], p["b1"], p["W2"], p["b2"], p["wout"], p["bout"]]
    return np.concatenate([np.asarray(a).ravel() for a in parts]).astype(np.float32)


def from_gpu_vec(v):
    v = np.asarray(v, dtype=np.float64)
    o = 0
    out = {}
    for name, shp in [("W0", (KF, HID)), ("b0", (HID,)), ("W1", (2 * HID, HID)), ("b1", (HID,)),
                      ("W2", (2 * HID, HID)), ("b2", (HID,)), ("wout", (HID,)), ("bout", (1,))]:
        size = int(np.prod(shp))
        out[name] = v[o:o + size].reshape(shp)
        o += size
    out["W0pad"] = out["W0"][4:]
    out["W0"] = out["W0"][:4]
    return out


def _graph(seed=4, n=400, m=1600, r=9):
    w = wl.zipf_powerlaw(seed=seed, n=n, m=m, kmax=r)
    e, i, nl, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
    return e, i, nl, r


def test_forward_and_gradients_match_oracle():
    import torch
    from paper_2311_08595_amd.warmstart import MpnnGraph, WarmStartNet
    e, i, n, r = _graph()
    rng = np.random.default_rng(1)
    p = {k: rng.normal(0, 0.2, shp) for k, shp in mr.PARAM_SHAPES}
    # round the weights to what FP32 storage holds, as the GPU sees them
    p = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    xs = np.exp(rng.normal(0, 0.4, n))
    xs /= xs.sum()
    g_ref = mr.Graph(e, i, n, r)
    s_ref, cache = mr.forward(p, g_ref, bf=True)
    L_ref, ds = mr.loss(s_ref, xs)
    gr = mr.backward(p, g_ref, cache, ds, bf=True)

    fb = mb.forward_bounds(p, g_ref)
    np.testing.assert_allclose(fb["s"], s_ref, rtol=1e-13, atol=1e-13)   # the bound model follows the oracle
    bb = mb.backward_bounds(p, g_ref, fb, xs)

    net = WarmStartNet(params=to_gpu_params(p))
    g = MpnnGraph(e, i, n, r)
    s = net.scores(g).cpu().numpy().astype(np.float64)
    es = np.abs(s - s_ref)
    print("scores: max err %.2e, max err / bound %.3f" % (es.max(), np.max(es / fb["es"])), flush=True)
    assert np.all(es <= fb["es"]), np.flatnonzero(es > fb["es"])[:5]
    L = net.loss_grad(g, torch.tensor(xs, dtype=torch.float64, device="cuda"))
    assert abs(L - L_ref) <= bb["loss"], (L, L_ref, bb["loss"])
    G = from_gpu_vec(net.grads())
    q = {name: net.query(g, name) for name in net.QUERY}
    for stage, err, ratio in mb.stage_checks(p, g_ref, q, G, xs):
        print("%-14s max err %.2e, max err / bound %.3f" % (stage, err, ratio), flush=True)
    assert np.all(G["W0pad"] == 0.0)


def test_training_reduces_loss_and_warm_start_is_valid():
    import torch
    from paper_2311_08595_amd import Plan
    from paper_2311_08595_amd.warmstart import MpnnGraph, WarmStartNet, train
    data = []
    for s in range(6):
        e, i, n, r = _graph(seed=40 + s, n=1500, m=6000, r=12)
        with Plan(e, i, n, r) as p:
            x, _ = p.solve(tol=1e-9)
        data.append((MpnnGraph(e, i, n, r), x, 0))
    net = WarmStartNet(seed=3)
    before = np.mean([net.loss_grad(g, x) for g, x, _ in data])
    hist = train(net, data, epochs=6, lr=3e-3)
    after = np.mean([net.loss_grad(g, x) for g, x, _ in data])
    assert after < 0.7 * before, (before, after, hist)
    g, x, _ = data[0]
    x0 = net.warm_start(g).cpu().numpy()
    assert np.all(x0 > 0) and abs(x0.sum() - 1.0) < 1e-12
    s = net.scores(g).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(x0, mr.warm_start(s), rtol=1e-6)
    # deterministic: same data, same seed -> same weights
    net2 = WarmStartNet(seed=3)
    train(net2, data, epochs=6, lr=3e-3)
    assert net.params().tobytes() == net2.params().tobytes()


def test_trained_network_gains_over_plain_and_degree_start():
    # held-out graphs of the training recipe (seeds outside the training set):
    # iterations to 1e-8 from the learned start vs the uniform start of
    # Alg. 1 and the degree start d^(1/(r-1))
    import os
    import torch
    from paper_2311_08595_amd import Plan
    from paper_2311_08595_amd.warmstart import DEFAULT_WEIGHTS, MpnnGraph, WarmStartNet
    assert os.path.exists(DEFAULT_WEIGHTS)
    net = WarmStartNet.load(DEFAULT_WEIGHTS)
    its = {"uniform": [], "degree": [], "net": []}
    for i in range(6):
        w = wl.warmstart_train_graph(i, base_seed=90_000)
        e, idx, n, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
        r = w["r"]
        with Plan(e, idx, n, r) as p:
            _, a = p.solve(tol=1e-8)
            d = np.bincount(idx, minlength=n).astype(np.float64)
            _, b = p.solve(tol=1e-8, x0=torch.tensor(d ** (1.0 / (r - 1)), dtype=torch.float64, device="cuda"))
            x0 = net.warm_start(MpnnGraph(e, idx, n, r))
            x, c = p.solve(tol=1e-8, x0=x0)
            xr, _ = p.solve(tol=1e-8)
        assert a["converged"] and b["converged"] and c["converged"]
        np.testing.assert_allclose(x.cpu().numpy(), xr.cpu().numpy(), rtol=1e-6)
        its["uniform"].append(a["iterations"])
        its["degree"].append(b["iterations"])
        its["net"].append(c["iterations"])
    print(its, flush=True)
    assert np.mean(its["net"]) < np.mean(its["degree"]) < np.mean(its["uniform"])
