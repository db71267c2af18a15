"""Learned warm start for the H-eigenvector solve.

A small hypergraph message-passing network (HIP kernels behind
``sttsv_mpnn_*``; see include/sttsv.h for its definition) is trained on
centrality vectors that the plain FP64 solver computes, and predicts a start
vector x0 for Alg. 1.  This module only orchestrates: data preparation,
the epoch loop, saving and loading weights.  Every arithmetic step runs on
the GPU.

    python -m paper_2311_08595_amd.warmstart train --graphs 2000 --out weights.npz
"""
import argparse
import ctypes
import os
import sys
import time

import numpy as np

from . import _lib
from . import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "warmstart_weights.npz")
HID = _lib.MPNN_HIDDEN
KF = 16


def init_params(seed=0):
    """Glorot-uniform weights, zero biases, packed in the library's order
    (W0 16x64 with rows 4..15 zero, b0, W1 128x64, b1, W2 128x64, b2,
    w_out, b_out)."""
    rng = np.random.default_rng(seed)

    def glorot(fi, fo):
        lim = np.sqrt(6.0 / (fi + fo))
        return rng.uniform(-lim, lim, size=(fi, fo))
    W0 = np.zeros((KF, HID))
    W0[:4] = glorot(4, HID)
    parts = [W0, np.zeros(HID), glorot(2 * HID, HID), np.zeros(HID), glorot(2 * HID, HID), np.zeros(HID),
             glorot(HID, 1)[:, 0], np.zeros(1)]
    vec = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert vec.size == _lib.MPNN_NPARAM
    return vec


class MpnnGraph:
    """Device copy of one hypergraph for the network."""

    def __init__(self, eptr, eidx, n, r):
        lib = _lib.load()
        self._lib = lib
        eptr = np.ascontiguousarray(eptr, dtype=np.int64)
        eidx = np.ascontiguousarray(eidx, dtype=np.int32)
        self.n, self.r, self.m = int(n), int(r), len(eptr) - 1
        h = ctypes.c_void_p()
        _lib.check(lib.sttsv_mpnn_graph(eptr.ctypes.data, eidx.ctypes.data, self.m, self.n, self.r,
                                        ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sttsv_mpnn_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WarmStartNet:
    """The network: FP32 master weights, Adam state, BF16 copies on the GPU."""

    def __init__(self, params=None, seed=0):
        lib = _lib.load()
        self._lib = lib
        p = np.ascontiguousarray(init_params(seed) if params is None else params, dtype=np.float32)
        if p.size != _lib.MPNN_NPARAM:
            raise ValueError("expected %d parameters" % _lib.MPNN_NPARAM)
        h = ctypes.c_void_p()
        _lib.check(lib.sttsv_mpnn_create(p.ctypes.data, ctypes.byref(h)))
        self._h = h

    def params(self):
        out = np.empty(_lib.MPNN_NPARAM, dtype=np.float32)
        _lib.check(self._lib.sttsv_mpnn_params(self._h, out.ctypes.data, None))
        return out

    def grads(self):
        out = np.empty(_lib.MPNN_NPARAM, dtype=np.float32)
        _lib.check(self._lib.sttsv_mpnn_params(self._h, None, out.ctypes.data))
        return out

    def scores(self, g):
        import torch
        s = torch.empty(g.n, dtype=torch.float32, device="cuda")
        _lib.check(self._lib.sttsv_mpnn_forward(self._h, g._h, ctypes.c_void_p(s.data_ptr())))
        return s

    def loss_grad(self, g, x_star):
        loss = ctypes.c_float()
        _lib.check(self._lib.sttsv_mpnn_loss_grad(self._h, g._h, ctypes.c_void_p(x_star.data_ptr()),
                                                  ctypes.byref(loss)))
        return loss.value

    QUERY = {"X0": (11, 16), "Z0": (0, 64), "Z1": (1, 64), "Z2": (2, 64), "X1": (3, 128), "X2": (4, 128),
             "s": (5, 0), "ds": (6, 0), "dZ0": (7, 64), "dA1": (8, 64), "dE1": (9, 64), "dH0": (10, 64)}

    def query(self, g, name):
        """Host copy (float32) of an intermediate value of the last forward /
        loss_grad call on graph ``g`` (names in QUERY)."""
        what, cols = self.QUERY[name]
        rows = g.m if name == "dE1" else g.n
        out = np.empty(rows * cols if cols else rows, dtype=np.float32)
        _lib.check(self._lib.sttsv_mpnn_query(self._h, g._h, what, out.ctypes.data, out.size))
        return out.reshape(rows, cols) if cols else out

    def step(self, g, x_star, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        loss = self.loss_grad(g, x_star)
        _lib.check(self._lib.sttsv_mpnn_adam(self._h, lr, beta1, beta2, eps))
        return loss

    def warm_start(self, g, out=None):
        import torch
        if out is None:
            out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        _lib.check(self._lib.sttsv_mpnn_warm_start(self._h, g._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def save(self, path, **meta):
        np.savez(path, params=self.params(), **{k: np.asarray(v) for k, v in meta.items()})

    @classmethod
    def load(cls, path=DEFAULT_WEIGHTS):
        with np.load(path, allow_pickle=False) as z:
            return cls(params=z["params"])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sttsv_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def training_set(count, n=10_000, base_seed=50_000, tol=1e-8, log=None):
    """``count`` graphs of the Zipf / power-law recipe at n vertices (their
    largest component), each with its converged centrality from the plain
    FP64 solve (uniform start) as target."""
    import torch
    from . import Plan
    data = []
    for i in range(count):
        w = wl.warmstart_train_graph(i, n=n, base_seed=base_seed)
        eptr, eidx, nl, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
        with Plan(eptr, eidx, nl, w["r"]) as p:
            x, info = p.solve(tol=tol)
        data.append((MpnnGraph(eptr, eidx, nl, w["r"]), x, info["iterations"]))
        if log and (i + 1) % 200 == 0:
            log("[warmstart] prepared %d/%d graphs" % (i + 1, count))
    torch.cuda.synchronize()
    return data


def train(net, data, epochs=8, lr=2e-3, log=None, seed=0):
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(data))
        tot = 0.0
        lr_ep = lr * (0.5 ** (ep // 3))
        for j in order:
            g, x, _ = data[j]
            tot += net.step(g, x, lr=lr_ep)
        hist.append(tot / len(data))
        if log:
            log("[warmstart] epoch %d loss %.5f" % (ep, hist[-1]))
    return hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd")
    t = sub.add_parser("train")
    t.add_argument("--graphs", type=int, default=2000)
    t.add_argument("--n", type=int, default=10_000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args(argv)
    if a.cmd != "train":
        ap.print_help()
        return 2

    def log(msg):
        print(msg, flush=True)
    t0 = time.perf_counter()
    data = training_set(a.graphs, n=a.n, log=log)
    prep = time.perf_counter() - t0
    net = WarmStartNet(seed=a.seed)
    t0 = time.perf_counter()
    hist = train(net, data, epochs=a.epochs, lr=a.lr, log=log, seed=a.seed)
    tr = time.perf_counter() - t0
    net.save(a.out, loss_history=np.array(hist), graphs=a.graphs, n=a.n, epochs=a.epochs,
             prepare_s=prep, train_s=tr)
    log("[warmstart] saved %s (prepare %.1f s, train %.1f s)" % (a.out, prep, tr))
    return 0


if __name__ == "__main__":
    sys.exit(main())
