"""Alg. 1 (NQZ) for H-eigenvector centrality, on top of the FP64 STTSV oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Alg. 1, step by step:
    y = (1/n) 1;  z = TTSV1(H, y)
    repeat
        x = z^[1/(r-1)] / || z^[1/(r-1)] ||_1
        z = TTSV1(H, x)
        lambda_min = min(z ./ x^[r-1]);  lambda_max = max(z ./ x^[r-1])
    until (lambda_max - lambda_min) / lambda_min < tau
    return x

Readings taken:
* The optional shift ``alpha`` (default 0, i.e. Alg. 1 as printed) replaces
  z by z + alpha x^[r-1] after each TTSV1, which shifts every ratio by alpha;
  the reported lambda bounds have alpha taken off again.
* x^[r-1] can underflow FP64 for large r and n (x ~ 1/n), so the ratio
  z_v / x_v^(r-1) is evaluated on x/max(x): both TTSV1(x) and x^[r-1] are
  homogeneous of degree r-1, so the ratio is unchanged.
* One pass of the repeat loop is one iteration; the returned x is the one
  whose z met the test (the loop's last x).
"""
import math

import numpy as np

from .sttsv_ref import sttsv


def _l1_normalise(w):
    return w / math.fsum(w.tolist())


def nqz(eptr, eidx, n, r, tol, max_iter=200, x0=None, alpha=0.0, history=False,
        apply=None, w=None):
    """Run Alg. 1.  Returns dict(x, lambda_min, lambda_max, criterion,
    iterations, converged[, xs, crits]).  ``x0`` replaces the uniform start
    y = 1/n (a warm start); ``apply`` replaces the STTSV oracle (used only to
    time the loop structure); ``w``: per-edge weights (default w(e) = |e|)."""
    if apply is None:
        weights = w

        def apply(v):
            return sttsv(eptr, eidx, n, r, v, weights)
    y = np.full(n, 1.0 / n) if x0 is None else np.asarray(x0, dtype=np.float64)
    yt = y / y.max()                        # scale of the first z is irrelevant too
    z = apply(yt)
    if alpha:
        z = z + alpha * yt ** (r - 1)
    xs, crits = [], []
    it = 0
    while True:
        w = z ** (1.0 / (r - 1))
        x = _l1_normalise(w)
        xm = x.max()
        xt = x / xm
        zt = apply(xt)                      # TTSV1(x) / max(x)^(r-1)
        pw = xt ** (r - 1)
        if alpha:
            zt = zt + alpha * pw
        lam = zt / pw
        lmin, lmax = float(lam.min()), float(lam.max())
        crit = (lmax - lmin) / lmin
        it += 1
        if history:
            xs.append(x.copy())
            crits.append(crit)
        z = zt                              # scale of z is irrelevant to the next x
        if crit < tol or it >= max_iter:
            break
    out = dict(x=x, lambda_min=lmin - alpha, lambda_max=lmax - alpha,
               criterion=crit, iterations=it, converged=bool(crit < tol))
    if history:
        out["xs"] = xs
        out["crits"] = crits
    return out
