"""Per-entry error bounds for the warm-start network on the GPU against the
FP64 oracle run with the same bfloat16 roundings (``bf=True``).

Test infrastructure.  The kernels compute in FP32 where the oracle computes in
FP64, and round the inputs of every dense product to bfloat16 as the oracle
does.  Two effects separate them:

* FP32 rounding.  A sum of n terms (products included, any order) is off by at
  most gamma_n * sum|terms|, gamma_n = n u / (1 - n u), u = 2^-24; a product or
  a quotient by a rounded reciprocal adds 2u relative.
* bfloat16 roundings.  A value known to within e rounds to the same bfloat16
  number as the oracle's when every value within e does; otherwise the two
  rounded values differ by at most the spread of the rounded interval ends
  (rounding is monotone).  ReLU masks can differ where |Z| <= e_Z.

The bound of every quantity is carried through the network in the order the
kernels compute it, so each GPU entry is checked against its own bound.
"""
import numpy as np

from oracle import mpnn_ref as mr

U = 2.0 ** -24
HD = mr.H


def gam(n):
    n = np.asarray(n, dtype=np.float64)
    return n * U / (1.0 - n * U)


def bf16_spread(pre, e):
    """Largest |bf16(v) - bf16(pre)| over |v - pre| <= e (0 when all round alike)."""
    mid = mr.bf16(pre)
    return np.maximum(np.abs(mr.bf16(pre - e) - mid), np.abs(mr.bf16(pre + e) - mid))


def _edge_sum(g, A):      # sum over the members of each edge: (n,H) -> (m,H)
    return g.edge_mean(A) * g.sizes[:, None]


def _vertex_sum(g, A):    # sum over the edges of each vertex: (m,H) -> (n,H)
    return g.node_mean(A) * np.maximum(g.deg, 1)[:, None]


def forward_bounds(p, g):
    """Bounds on the scores and the intermediate values the backward pass
    needs.  ``p``: parameters holding FP32 values (as the GPU stores them)."""
    k = g.sizes[:, None]
    d = np.maximum(g.deg, 1)[:, None]
    b = {}
    F = g.F
    eF = 1e-14 * np.abs(F)                    # features: FP64 logs and quotients on both sides
    X0 = mr.bf16(F)
    eX0 = bf16_spread(F, eF)
    W0 = mr.bf16(p["W0"])
    # 16 padded feature columns + bias
    eZ = gam(17) * (np.abs(X0) @ np.abs(W0) + np.abs(p["b0"])) + eX0 @ np.abs(W0)
    Hc = np.maximum(X0 @ W0 + p["b0"], 0.0)
    b["X0"], b["eX0"], b["Z0"], b["eZ0"] = X0, eX0, X0 @ W0 + p["b0"], eZ
    eH = eZ
    for l in (1, 2):
        eXL = bf16_spread(Hc, eH)
        # vertex -> edge mean: |e| - 1 adds, then a product by the rounded 1/|e|
        E = g.edge_mean(Hc)
        eE = (gam(k - 1) * _edge_sum(g, np.abs(Hc)) + _edge_sum(g, eH)) / k * (1 + 2 * U) + 2 * U * np.abs(E)
        # edge -> vertex mean: d - 1 adds (any tree), product by the rounded 1/d
        A = g.node_mean(E)
        eA = (gam(d - 1) * _vertex_sum(g, np.abs(E)) + _vertex_sum(g, eE)) / d * (1 + 2 * U) + 2 * U * np.abs(A)
        eXR = bf16_spread(A, eA)
        X = mr.bf16(np.concatenate([Hc, A], axis=1))
        eX = np.concatenate([eXL, eXR], axis=1)
        W = mr.bf16(p["W%d" % l])
        Z = X @ W + p["b%d" % l]
        eZ = gam(2 * HD + 1) * (np.abs(X) @ np.abs(W) + np.abs(p["b%d" % l])) + eX @ np.abs(W)
        b["X%d" % l], b["eX%d" % l], b["Z%d" % l], b["eZ%d" % l] = X, eX, Z, eZ
        Hc, eH = np.maximum(Z, 0.0), eZ
    b["H2"], b["eH2"] = Hc, eH
    s = Hc @ p["wout"] + p["bout"][0]
    es = gam(HD + 1) * (np.abs(Hc) @ np.abs(p["wout"]) + abs(p["bout"][0])) + eH @ np.abs(p["wout"])
    b["s"], b["es"] = s, es
    return b


def backward_bounds(p, g, b, x_star):
    """Bounds on the loss and on every gradient (dict keyed like the
    parameters, plus "loss")."""
    n = g.n
    k = g.sizes[:, None]
    s, es = b["s"], b["es"]
    t = np.log(x_star)
    et = 2 * U * np.abs(t)
    sm, tm = s.mean(), t.mean()
    esm = (gam(n) * np.abs(s).sum() + es.sum()) / n + 2 * U * abs(sm)
    etm = (gam(n) * np.abs(t).sum() + et.sum()) / n + 2 * U * abs(tm)
    u = (s - sm) - (t - tm)
    eu = es + esm + et + etm + 3 * U * (np.abs(s) + abs(sm) + np.abs(t) + abs(tm))
    ds = 2.0 * u / n
    eds = 2.0 / n * eu + U * np.abs(ds)
    out = {}
    out["loss"] = (2 * np.abs(u) @ eu + (eu * eu).sum() + gam(2 * n) * (u * u).sum()) / n \
        + 2 * U * float(np.mean(u * u))
    H2, eH2 = b["H2"], b["eH2"]
    out["wout"] = gam(n + 1) * (np.abs(H2).T @ np.abs(ds)) + eH2.T @ np.abs(ds) + np.abs(H2).T @ eds + eH2.T @ eds
    out["bout"] = np.array([gam(n) * np.abs(ds).sum() + eds.sum()])
    dH = np.outer(ds, p["wout"])
    edH = np.outer(eds, np.abs(p["wout"])) + U * np.abs(dH)
    for l in (2, 1):
        Z, eZ = b["Z%d" % l], b["eZ%d" % l]
        X, eX = b["X%d" % l], b["eX%d" % l]
        on = Z > 0
        maybe = np.abs(Z) <= eZ
        dZ = dH * on
        edZ = np.where(maybe, np.abs(dH) + edH, np.where(on, edH, 0.0))
        aX, adZ = np.abs(X), np.abs(dZ)
        out["W%d" % l] = gam(n + 1) * (aX.T @ adZ) + eX.T @ adZ + aX.T @ edZ + eX.T @ edZ
        out["b%d" % l] = gam(n) * adZ.sum(axis=0) + edZ.sum(axis=0)
        dZb = mr.bf16(dZ)
        edZb = bf16_spread(dZ, edZ)
        W = mr.bf16(p["W%d" % l])
        dX = dZb @ W.T
        edX = gam(HD) * (np.abs(dZb) @ np.abs(W).T) + edZb @ np.abs(W).T
        dHp, edHp = dX[:, :HD], edX[:, :HD]
        dA, edA = dX[:, HD:], edX[:, HD:]
        # dE_e = sum over members of dA_v / d_v (rounded 1/d_v, product, adds)
        dE = g.node_mean_T(dA)
        edE = gam(k + 1) * g.node_mean_T(np.abs(dA)) + g.node_mean_T(edA) * (1 + 2 * U)
        # dH_v += sum over edges of dE_e / |e| (rounded 1/|e|, product, adds)
        acc = g.edge_mean_T(dE)
        dvec = np.maximum(g.deg, 1)[:, None]
        eacc = gam(dvec + 1) * g.edge_mean_T(np.abs(dE)) + g.edge_mean_T(edE) * (1 + 2 * U)
        dH = dHp + acc
        edH = edHp + eacc + U * np.abs(dH)
    Z0, eZ0 = b["Z0"], b["eZ0"]
    on = Z0 > 0
    maybe = np.abs(Z0) <= eZ0
    dZ = dH * on
    edZ = np.where(maybe, np.abs(dH) + edH, np.where(on, edH, 0.0))
    aX, eX, adZ = np.abs(b["X0"]), b["eX0"], np.abs(dZ)
    out["W0"] = gam(n + 1) * (aX.T @ adZ) + eX.T @ adZ + aX.T @ edZ + eX.T @ edZ
    out["b0"] = gam(n) * adZ.sum(axis=0) + edZ.sum(axis=0)
    return out


def _close(name, got, ref, bound, report):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    ratio = float(np.max(err / np.maximum(bound, 1e-300))) if err.size else 0.0
    report.append((name, float(err.max()) if err.size else 0.0, ratio))
    bad = np.argwhere(err > bound)
    assert bad.size == 0, (name, bad[:5], got[tuple(bad[0])], ref[tuple(bad[0])], bound[tuple(bad[0])])


def stage_checks(p, g, q, G, x_star):
    """Check every stage of one forward + loss_grad call on the GPU against
    the oracle's arithmetic applied to the GPU's own inputs of that stage
    (``q``: the intermediates from the network's query call, ``G``: its
    gradients), each entry within the FP32 rounding bound of that stage.
    Returns [(stage, max error, max error / bound)]."""
    rep = []
    k = g.sizes[:, None]
    d = np.maximum(g.deg, 1)[:, None]
    n = g.n
    X0 = q["X0"][:, :4].astype(np.float64)
    assert np.all(q["X0"][:, 4:] == 0.0)
    _close("X0", X0, mr.bf16(g.F), bf16_spread(g.F, 1e-14 * np.abs(g.F)), rep)
    # dense layer 0
    W = mr.bf16(p["W0"])
    _close("Z0", q["Z0"], X0 @ W + p["b0"], gam(17) * (np.abs(X0) @ np.abs(W) + np.abs(p["b0"])), rep)
    Zs = [q["Z0"].astype(np.float64)]
    for l in (1, 2):
        Hc = np.maximum(Zs[-1], 0.0)
        X = q["X%d" % l].astype(np.float64)
        # left half: the previous layer's H, rounded to bf16 (bit for bit)
        assert np.array_equal(X[:, :HD], mr.bf16(Hc)), "X%d left half" % l
        # right half: vertex mean of edge means of the GPU's H, rounded to bf16
        E = g.edge_mean(Hc)
        eE = gam(k - 1) * _edge_sum(g, np.abs(Hc)) / k * (1 + 2 * U) + 2 * U * np.abs(E)
        A = g.node_mean(E)
        eA = (gam(d - 1) * _vertex_sum(g, np.abs(E)) + _vertex_sum(g, eE)) / d * (1 + 2 * U) + 2 * U * np.abs(A)
        _close("X%d mean half" % l, X[:, HD:], mr.bf16(A), bf16_spread(A, eA), rep)
        W = mr.bf16(p["W%d" % l])
        _close("Z%d" % l, q["Z%d" % l], X @ W + p["b%d" % l],
               gam(2 * HD + 1) * (np.abs(X) @ np.abs(W) + np.abs(p["b%d" % l])), rep)
        Zs.append(q["Z%d" % l].astype(np.float64))
    H2 = np.maximum(Zs[2], 0.0)
    s = q["s"].astype(np.float64)
    _close("s", s, H2 @ p["wout"] + p["bout"][0],
           gam(HD + 1) * (np.abs(H2) @ np.abs(p["wout"]) + abs(p["bout"][0])), rep)
    # loss gradient ds from the GPU's scores
    t = np.log(x_star)
    sm, tm = s.mean(), t.mean()
    esm = gam(n) * np.abs(s).sum() / n + 2 * U * abs(sm)
    etm = (gam(n) * np.abs(t).sum() + 2 * U * np.abs(t).sum()) / n + 2 * U * abs(tm)
    u = (s - sm) - (t - tm)
    eu = esm + 2 * U * np.abs(t) + etm + 3 * U * (np.abs(s) + abs(sm) + np.abs(t) + abs(tm))
    ds_ref = 2.0 * u / n
    ds = q["ds"].astype(np.float64)
    _close("ds", ds, ds_ref, 2.0 / n * eu + U * np.abs(ds_ref), rep)
    # output layer gradients from the GPU's ds
    _close("grad wout", G["wout"], H2.T @ ds, gam(n + 1) * (np.abs(H2).T @ np.abs(ds)), rep)
    _close("grad bout", G["bout"], np.array([ds.sum()]), np.array([gam(n) * np.abs(ds).sum()]), rep)
    # dH2 = ds wout is one FP32 product per entry: reproduced exactly
    dH = (q["ds"][:, None] * np.asarray(p["wout"], np.float32)[None, :]).astype(np.float64)
    edH = np.zeros_like(dH)
    for l in (2, 1):
        on = Zs[l] > 0
        dZ = dH * on
        edZ = edH * on
        X = q["X%d" % l].astype(np.float64)
        _close("grad W%d" % l, G["W%d" % l], X.T @ dZ,
               gam(n + 1) * (np.abs(X).T @ np.abs(dZ)) + np.abs(X).T @ edZ, rep)
        _close("grad b%d" % l, G["b%d" % l], dZ.sum(axis=0), gam(n) * np.abs(dZ).sum(axis=0) + edZ.sum(axis=0), rep)
        W = mr.bf16(p["W%d" % l])
        dZb = mr.bf16(dZ)
        edZb = bf16_spread(dZ, edZ)
        dX = dZb @ W.T
        edX = gam(HD) * (np.abs(dZb) @ np.abs(W).T) + edZb @ np.abs(W).T
        dHp, edHp = dX[:, :HD], edX[:, :HD]
        dA, edA = dX[:, HD:], edX[:, HD:]
        if l == 1:
            # the GPU's layer-1 dA and dE are kept: check them and continue from them
            _close("dA1", q["dA1"], dA, edA, rep)
            dA, edA = q["dA1"].astype(np.float64), np.zeros_like(dA)
        dE = g.node_mean_T(dA)
        edE = gam(k + 1) * g.node_mean_T(np.abs(dA)) + g.node_mean_T(edA) * (1 + 2 * U)
        if l == 1:
            _close("dE1", q["dE1"], dE, edE, rep)
            dE, edE = q["dE1"].astype(np.float64), np.zeros_like(dE)
        acc = g.edge_mean_T(dE)
        eacc = gam(d + 1) * g.edge_mean_T(np.abs(dE)) + g.edge_mean_T(edE) * (1 + 2 * U)
        dH = dHp + acc
        edH = edHp + eacc + U * np.abs(dH)
    _close("dH0", q["dH0"], dH, edH, rep)
    dH0 = q["dH0"].astype(np.float64)
    assert np.array_equal(q["dZ0"].astype(np.float64), dH0 * (Zs[0] > 0)), "dZ0 = dH0 [Z0 > 0]"
    dZ = q["dZ0"].astype(np.float64)
    _close("grad W0", G["W0"], X0.T @ dZ, gam(n + 1) * (np.abs(X0).T @ np.abs(dZ)), rep)
    _close("grad b0", G["b0"], dZ.sum(axis=0), gam(n) * np.abs(dZ).sum(axis=0), rep)
    return rep
