"""FP64 oracle of the warm-start message-passing network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper names hypergraph learning only as future work (Sec. VI); the
network is this library's own component.  Definition (hidden width H = 64):

features of vertex v (d_v = degree, E(v) = edges containing v):
    f0 = log(1 + d_v)
    f1 = mean_{e in E(v)} log|e|
    f2 = log(d_v) / (r - 1)
    f3 = log(1 + sum_{e in E(v)} (|e| - 1))
layers:
    H0 = relu(F W0 + b0)                                   (4 -> 64)
    for l = 1, 2:
        Ed_e = (1/|e|) sum_{v in e} H_{l-1, v}             (vertex -> edge mean)
        A_v  = (1/d_v) sum_{e in E(v)} Ed_e               (edge -> vertex mean)
        H_l  = relu([H_{l-1}, A] W_l + b_l)                (128 -> 64)
    s_v = H2_v . w_out + b_out                             (score ~ log x_v)
loss against the converged centrality x*:
    u = (s - mean s) - (t - mean t),  t = log x*,   L = mean(u^2)
warm start:  x0 = exp(s - max s) / sum(exp(s - max s)).

``bf16=True`` rounds, as the GPU kernels do, the inputs of every dense
product (features, [H, A], the weights, and dZ in the input-gradient
product) to bfloat16 (round to nearest even from float32); everything else
is FP64 here.  Gradients are by hand (checked against central differences
in the tests).
"""
import math

import numpy as np

H = 64
PARAM_SHAPES = [("W0", (4, H)), ("b0", (H,)), ("W1", (2 * H, H)), ("b1", (H,)),
                ("W2", (2 * H, H)), ("b2", (H,)), ("wout", (H,)), ("bout", (1,))]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), through float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(eptr, eidx, n, r):
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    sizes = np.diff(eptr).astype(np.float64)
    edge_of = np.repeat(np.arange(len(sizes)), np.diff(eptr))
    d = np.bincount(eidx, minlength=n).astype(np.float64)
    slog = np.bincount(eidx, weights=np.log(sizes)[edge_of], minlength=n)
    sco = np.bincount(eidx, weights=(sizes - 1.0)[edge_of], minlength=n)
    F = np.zeros((n, 4))
    F[:, 0] = np.log1p(d)
    F[:, 1] = np.where(d > 0, slog / np.maximum(d, 1), 0.0)
    F[:, 2] = np.where(d > 0, np.log(np.maximum(d, 1)) / (r - 1), 0.0)
    F[:, 3] = np.log1p(sco)
    return F


class Graph:
    def __init__(self, eptr, eidx, n, r):
        self.eptr = np.asarray(eptr, dtype=np.int64)
        self.eidx = np.asarray(eidx, dtype=np.int64)
        self.n, self.r = n, r
        self.m = len(self.eptr) - 1
        self.sizes = np.diff(self.eptr).astype(np.float64)
        self.edge_of = np.repeat(np.arange(self.m), np.diff(self.eptr))
        self.deg = np.bincount(self.eidx, minlength=n).astype(np.float64)
        self.F = features(eptr, eidx, n, r)

    def edge_mean(self, Hv):          # (n,H) -> (m,H)
        out = np.zeros((self.m, Hv.shape[1]))
        np.add.at(out, self.edge_of, Hv[self.eidx])
        return out / self.sizes[:, None]

    def node_mean(self, Ee):          # (m,H) -> (n,H)
        out = np.zeros((self.n, Ee.shape[1]))
        np.add.at(out, self.eidx, Ee[self.edge_of])
        return out / np.maximum(self.deg, 1)[:, None]

    def edge_mean_T(self, dE):        # adjoint of edge_mean
        out = np.zeros((self.n, dE.shape[1]))
        np.add.at(out, self.eidx, (dE / self.sizes[:, None])[self.edge_of])
        return out

    def node_mean_T(self, dA):        # adjoint of node_mean
        out = np.zeros((self.m, dA.shape[1]))
        np.add.at(out, self.edge_of, (dA / np.maximum(self.deg, 1)[:, None])[self.eidx])
        return out


def unpack(vec):
    p, o = {}, 0
    for name, shp in PARAM_SHAPES:
        size = int(np.prod(shp))
        p[name] = np.asarray(vec[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    return p


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def forward(p, g, bf=False):
    rnd = bf16 if bf else (lambda a: a)
    c = {}
    X0 = rnd(g.F)
    Z0 = X0 @ rnd(p["W0"]) + p["b0"]
    Hc = np.maximum(Z0, 0.0)
    c["X0"], c["Z0"] = X0, Z0
    for l in (1, 2):
        Ed = g.edge_mean(Hc)
        A = g.node_mean(Ed)
        X = rnd(np.concatenate([Hc, A], axis=1))
        Z = X @ rnd(p["W%d" % l]) + p["b%d" % l]
        c["X%d" % l], c["Z%d" % l] = X, Z
        Hc = np.maximum(Z, 0.0)
    c["H2"] = Hc
    s = Hc @ p["wout"] + p["bout"][0]
    return s, c


def loss(s, x_star):
    t = np.log(x_star)
    u = (s - s.mean()) - (t - t.mean())
    n = len(s)
    return float(np.mean(u * u)), 2.0 * u / n


def backward(p, g, c, ds, bf=False, trace=None):
    """Gradients of the loss given dL/ds.  ``trace`` (a dict, optional)
    receives dA and dEd of layer 1 and dH, dZ of layer 0."""
    rnd = bf16 if bf else (lambda a: a)
    gr = {}
    gr["wout"] = c["H2"].T @ ds
    gr["bout"] = np.array([ds.sum()])
    dH = np.outer(ds, p["wout"])
    for l in (2, 1):
        dZ = dH * (c["Z%d" % l] > 0)
        gr["W%d" % l] = c["X%d" % l].T @ dZ
        gr["b%d" % l] = dZ.sum(axis=0)
        dX = rnd(dZ) @ rnd(p["W%d" % l]).T
        dHprev, dA = dX[:, :H], dX[:, H:]
        dE = g.node_mean_T(dA)
        dH = dHprev + g.edge_mean_T(dE)
        if trace is not None and l == 1:
            trace["dA1"], trace["dE1"] = dA, dE
    dZ0 = dH * (c["Z0"] > 0)
    if trace is not None:
        trace["dH0"], trace["dZ0"] = dH, dZ0
    gr["W0"] = c["X0"].T @ dZ0
    gr["b0"] = dZ0.sum(axis=0)
    return gr


def warm_start(s):
    e = np.exp(s - s.max())
    return e / math.fsum(e.tolist())
