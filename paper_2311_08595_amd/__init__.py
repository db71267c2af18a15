"""STTSV on the blowup adjacency tensor of a hypergraph, and H-eigenvector
centrality by the NQZ iteration, on AMD MI355X (gfx950).

The computation runs in ``libsttsv.so`` (HIP kernels behind a C ABI,
``include/sttsv.h``); this package only marshals arguments.  PyTorch is used
for device memory and streams.

    import torch, paper_2311_08595_amd as st
    plan = st.Plan(eptr, eidx, n, r)                   # host CSR (numpy)
    y = plan.apply(x)                                  # x: cuda float64 tensor
    x, info = plan.solve(tol=1e-8)                     # H-eigenvector (Alg. 1)
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import SttsvError, STTSV_MAX_ORDER  # noqa: F401

__all__ = ["Plan", "SttsvError", "load"]

load = _lib.load


def _dev_ptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous cuda float64 tensor of length %d" % (name, n))
    return ctypes.c_void_p(t.data_ptr())


def _opts(precision, flags, stream):
    import torch
    if stream is None and torch.cuda.is_available():
        stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    return _lib.SttsvOpts(_lib.PREC[precision], int(flags), sptr), stream


def _info_dict(info, rc):
    return dict(iterations=info.iterations, iters_fp32=info.iters_fp32, iters_fp64=info.iters_fp64,
                converged=bool(info.converged), lambda_min=info.lambda_min,
                lambda_max=info.lambda_max, criterion=info.criterion, status=rc)


class Plan:
    """Execution plan of one hypergraph (``sttsv_plan``), or of several
    (``Plan.batch`` -> ``sttsv_plan_batch``)."""

    def __init__(self, eptr, eidx, n, r, precision="fp64", stream=None, flags=0, weights=None, _graphs=None):
        """``weights``: optional w(e) per input edge (finite, > 0) of the
        edge-weighted hypergraph H = (V, E, w); default w(e) = |e|."""
        lib = _lib.load()
        self._lib = lib
        opts, self.stream = _opts(precision, flags, stream)
        h = ctypes.c_void_p()
        if _graphs is None:
            eptr = np.ascontiguousarray(eptr, dtype=np.int64)
            eidx = np.ascontiguousarray(eidx, dtype=np.int32)
            self.n, self.r, self.m = int(n), int(r), len(eptr) - 1
            if weights is not None:
                weights = np.ascontiguousarray(weights, dtype=np.float64)
                if weights.shape != (self.m,):
                    raise ValueError("weights must hold one value per edge")
                opts.edge_weights = weights.ctypes.data
            _lib.check(lib.sttsv_plan(eptr.ctypes.data, eidx.ctypes.data, self.m, self.n, self.r,
                                      ctypes.byref(opts), ctypes.byref(h)))
            self.graphs = 1
        else:
            keep = []
            descs = (_lib.GraphDesc * len(_graphs))()
            for g, gr in enumerate(_graphs):
                ep, ei, ng, rg = gr[:4]
                wg = gr[4] if len(gr) > 4 else None
                ep = np.ascontiguousarray(ep, dtype=np.int64)
                ei = np.ascontiguousarray(ei, dtype=np.int32)
                if wg is not None:
                    wg = np.ascontiguousarray(wg, dtype=np.float64)
                    if wg.shape != (len(ep) - 1,):
                        raise ValueError("weights of graph %d must hold one value per edge" % g)
                keep.append((ep, ei, wg))
                descs[g] = _lib.GraphDesc(ep.ctypes.data, ei.ctypes.data, len(ep) - 1, int(ng), int(rg),
                                          None if wg is None else wg.ctypes.data)
            _lib.check(lib.sttsv_plan_batch(len(_graphs), descs, ctypes.byref(opts), ctypes.byref(h)))
            self.n = sum(int(g[2]) for g in _graphs)
            self.m = sum(len(g[0]) - 1 for g in _graphs)
            self.r = max(int(g[3]) for g in _graphs)
            self.graphs = len(_graphs)
        self._h = h
        self.precision = precision

    @classmethod
    def batch(cls, graphs, precision="fp64", stream=None, flags=0):
        """One plan over many hypergraphs: ``graphs`` = [(eptr, eidx, n, r[, w]), ...].
        Vectors are the concatenation of the per-graph vectors in graph order."""
        return cls(None, None, None, None, precision, stream, flags, _graphs=list(graphs))

    def graph_info(self, g):
        gi = _lib.GraphInfo()
        _lib.check(self._lib.sttsv_plan_graph_info(self._h, int(g), ctypes.byref(gi)))
        return dict(m=gi.m, n=gi.n, r=gi.r, voff=gi.voff, connected=bool(gi.connected))

    def solve_batch(self, tol=1e-8, x0=None, out=None, max_iter=500, check_every=8, schedule="fp64",
                    use_graph=True, shift=0.0, switch_tol=1e-4, raise_on_notconv=True):
        """Alg. 1 for every graph of the plan at once.  Returns (x, [info per graph])."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        op = _dev_ptr(out, self.n, "out")
        x0p = None if x0 is None else _dev_ptr(x0, self.n, "x0")
        o = _lib.SolveOpts(max_iter, check_every, _lib.SCHEDULE[schedule], 1 if use_graph else 0,
                           float(shift), float(switch_tol))
        infos = (_lib.SolveInfo * self.graphs)()
        rc = self._lib.heigvec_solve_batch(self._h, x0p, float(tol), ctypes.byref(o), op, infos)
        res = [_info_dict(infos[g], rc) for g in range(self.graphs)]
        if rc != _lib.STTSV_OK and (rc != _lib.STTSV_ENOTCONV or raise_on_notconv):
            _lib.check(rc)
        return out, res

    # ------------------------------------------------------------ compute
    def apply(self, x, y=None, precision=None):
        """y = B x^(r-1) (TTSV1, Eq. (2)) on the GPU; returns y."""
        import torch
        xp = _dev_ptr(x, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        yp = _dev_ptr(y, self.n, "y")
        prec = _lib.PREC[precision or self.precision]
        _lib.check(self._lib.sttsv_apply_prec(self._h, xp, yp, prec))
        return y

    def apply_naive(self, x, y=None):
        """y = B x^(r-1) by Alg. 3 (no memoisation, FP64): the comparison
        baseline for apply; returns y."""
        import torch
        xp = _dev_ptr(x, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        yp = _dev_ptr(y, self.n, "y")
        _lib.check(self._lib.sttsv_apply_naive(self._h, xp, yp))
        return y

    def contract(self, x, y=None, noalloc=False):
        """B x^r (full contraction); y receives B x^(r-1).  Returns (value, y).
        ``noalloc``: the allocation-free entry point (static scratch)."""
        import torch
        xp = _dev_ptr(x, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        yp = _dev_ptr(y, self.n, "y")
        out = ctypes.c_double()
        fn = self._lib.sttsv_contract_noalloc if noalloc else self._lib.sttsv_contract
        _lib.check(fn(self._h, xp, yp, ctypes.byref(out)))
        return out.value, y

    def ccss_build(self):
        """Build the CCSS forest (Sec. III) on the device; returns its sizes."""
        ci = _lib.CcssInfo()
        _lib.check(self._lib.sttsv_ccss_build(self._h, ctypes.byref(ci)))
        return dict(levels=ci.levels, nodes=ci.nodes, roots=ci.roots, convolutions=ci.convolutions,
                    leaves=ci.leaves, device_bytes=ci.device_bytes, build_ms=ci.build_ms)

    def apply_ccss(self, x, y=None):
        """y = B x^(r-1) by Alg. 4 over the CCSS forest (FP64); returns y."""
        import torch
        xp = _dev_ptr(x, self.n, "x")
        if y is None:
            y = torch.empty_like(x)
        yp = _dev_ptr(y, self.n, "y")
        _lib.check(self._lib.sttsv_apply_ccss(self._h, xp, yp))
        return y

    def ccss_query(self, what, count):
        out = np.empty(count, dtype=np.int64)
        _lib.check(self._lib.sttsv_plan_query(self._h, what, out.ctypes.data, count))
        return out

    def _cp_args(self, A, lam):
        import torch
        if not isinstance(A, torch.Tensor) or A.dim() != 2 or A.shape[1] != self.n:
            raise ValueError("A must be an R x n tensor (row l = a_l)")
        R = A.shape[0]
        return R, _dev_ptr(A.view(-1), R * self.n, "A"), _dev_ptr(lam, R, "lambda")

    def cp_objective_grad(self, A, lam):
        """Symmetric CP objective f(lambda, A) and its gradient (Sec. I):
        A is R x n on the device (row l = a_l).  Returns (f, dA, dlambda)."""
        import torch
        R, ap, lp = self._cp_args(A, lam)
        dA = torch.empty_like(A)
        dl = torch.empty_like(lam)
        f = ctypes.c_double()
        _lib.check(self._lib.sttsv_cp_objective_grad(self._h, R, ap, lp, ctypes.byref(f),
                                                     _dev_ptr(dA.view(-1), R * self.n, "dA"),
                                                     _dev_ptr(dl, R, "dlambda")))
        return f.value, dA, dl

    def cp_descent(self, A, lam, iters, step=1.0):
        """Armijo gradient descent on the symmetric CP objective, in place on
        (A, lam); returns the info dict."""
        R, ap, lp = self._cp_args(A, lam)
        info = _lib.CpInfo()
        _lib.check(self._lib.sym_cp_descent(self._h, R, ap, lp, int(iters), float(step), ctypes.byref(info)))
        return dict(iterations=info.iterations, halvings=info.halvings, f0=info.f0, f=info.f, norm2=info.norm2)

    def zeig_sshopm(self, x0=None, alpha=1.0, tol=1e-12, max_iter=500, out=None, raise_on_notconv=True):
        """Z-eigenpair by the shifted power method (SS-HOPM, convex shift
        alpha >= 0).  Returns (x, info dict); x has 2-norm 1."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        op = _dev_ptr(out, self.n, "out")
        x0p = None if x0 is None else _dev_ptr(x0, self.n, "x0")
        info = _lib.ZeigInfo()
        rc = self._lib.zeigvec_sshopm(self._h, x0p, float(alpha), float(tol), int(max_iter), op,
                                      ctypes.byref(info))
        if rc != _lib.STTSV_OK and (rc != _lib.STTSV_ENOTCONV or raise_on_notconv):
            _lib.check(rc)
        return out, dict(iterations=info.iterations, converged=bool(info.converged), lambda_=info.lambda_,
                         residual=info.residual, status=rc)

    def solve(self, tol=1e-8, x0=None, out=None, max_iter=500, check_every=8, schedule="fp64",
              use_graph=True, shift=0.0, switch_tol=1e-4, raise_on_notconv=True):
        """NQZ iteration (Alg. 1).  Returns (x, info dict); x has l1 norm 1."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        op = _dev_ptr(out, self.n, "out")
        x0p = None if x0 is None else _dev_ptr(x0, self.n, "x0")
        o = _lib.SolveOpts(max_iter, check_every, _lib.SCHEDULE[schedule], 1 if use_graph else 0,
                           float(shift), float(switch_tol))
        info = _lib.SolveInfo()
        rc = self._lib.heigvec_solve_ex(self._h, x0p, float(tol), ctypes.byref(o), op, ctypes.byref(info))
        d = _info_dict(info, rc)
        if rc != _lib.STTSV_OK and (rc != _lib.STTSV_ENOTCONV or raise_on_notconv):
            _lib.check(rc)
        return out, d

    def autotune(self, x, reps=5, cache_path=None):
        """Pick the fastest bitwise-equivalent kernel variants per bucket
        (``sttsv_plan_autotune``); returns the number of decisions."""
        xp = _dev_ptr(x, self.n, "x")
        n = ctypes.c_int32()
        cp = cache_path.encode() if cache_path else None
        _lib.check(self._lib.sttsv_plan_autotune(self._h, xp, int(reps), cp, ctypes.byref(n)))
        return n.value

    # ------------------------------------------------------- introspection
    def info(self):
        pi = _lib.PlanInfo()
        _lib.check(self._lib.sttsv_plan_get_info(self._h, ctypes.byref(pi)))
        return dict(m=pi.m, nnz=pi.nnz, n=pi.n, r=pi.r, nbuckets=pi.nbuckets,
                    connected=bool(pi.connected), device_bytes=pi.device_bytes, graphs=pi.graphs,
                    lanes=pi.lanes)

    def query(self, what):
        inf = self.info()
        sizes = {_lib.Q_PERM: inf["m"], _lib.Q_MEM: inf["nnz"], _lib.Q_BUCKET_K: inf["nbuckets"],
                 _lib.Q_BUCKET_M: inf["nbuckets"], _lib.Q_TPTR: inf["n"] + 1,
                 _lib.Q_TSLOT: inf["nnz"], _lib.Q_BUCKET_R: inf["nbuckets"],
                 _lib.Q_BUCKET_RUNS: inf["nbuckets"], _lib.Q_BUCKET_LANES: inf["nbuckets"],
                 _lib.Q_BUCKET_STACK: inf["nbuckets"],
                 _lib.Q_CONTRIB: inf["nnz"]}
        if what in (_lib.Q_WEIGHTS, _lib.Q_SCALE_EXP):
            sizes[what] = self.graph_info(0)["r"] + 1
        cnt = sizes[what]
        out = np.empty(cnt, dtype=np.float64 if what in (_lib.Q_WEIGHTS, _lib.Q_CONTRIB) else np.int64)
        _lib.check(self._lib.sttsv_plan_query(self._h, what, out.ctypes.data, cnt))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sttsv_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
