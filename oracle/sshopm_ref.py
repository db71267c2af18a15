"""The shifted power method for Z-eigenpairs of the blowup tensor, and the
full contraction B x^r, on top of the FP64 STTSV oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper names the shifted power method for tensor eigenpairs as one of the
algorithms whose bottleneck is STTSV (Sec. I, citing Kolda and Mayo's
SS-HOPM).  A Z-eigenpair of the symmetric order-r tensor B is (lambda, x) with
B x^(r-1) = lambda x and ||x||_2 = 1; then lambda = B x^r = x . (B x^(r-1)).
SS-HOPM, convex form (shift alpha >= 0), step by step:

    x_0 = x0 / ||x0||_2;  y_0 = B x_0^(r-1);  lambda_0 = x_0 . y_0
    repeat for k = 0, 1, ...
        w = y_k + alpha x_k;   x_{k+1} = w / ||w||_2
        y_{k+1} = B x_{k+1}^(r-1);   lambda_{k+1} = x_{k+1} . y_{k+1}
    until |lambda_{k+1} - lambda_k| <= tol |lambda_{k+1}|

Readings taken:
* The stopping rule is relative to |lambda| (the method's papers state an
  absolute one; the blowup tensor's eigenvalues span many orders of
  magnitude with r and n).
* One pass of the loop is one iteration; the returned pair is the last
  (x_{k+1}, lambda_{k+1}).  ``residual`` is ||y - lambda x||_2 there.
* tol = 0 means "run max_iter updates" (no early stop even where lambda
  repeats exactly), so runs can be compared iterate by iterate.

Parity pins (tests/test_sshopm_oracle_pins.py): the graph case r = 2 gives the
Perron eigenpair of the adjacency matrix; on a regular hypergraph the
normalised all-ones vector is a fixed point with lambda = d n^(-(r-2)/2);
lambda = B x^r equals the blowup entries summed against x^r by brute force.
"""
import math

import numpy as np

from .sttsv_ref import sttsv


def contract(eptr, eidx, n, r, x, w=None):
    """B x^r = sum_v x_v (B x^(r-1))_v, summed with math.fsum."""
    y = sttsv(eptr, eidx, n, r, x, w)
    return math.fsum((np.asarray(x, dtype=np.float64) * y).tolist())


def _norm2(w):
    return math.sqrt(math.fsum((w * w).tolist()))


def sshopm(eptr, eidx, n, r, x0, alpha=1.0, tol=1e-12, max_iter=500, history=False):
    """SS-HOPM (convex shift alpha >= 0).  Returns (x, info); info holds
    iterations, lambda, residual, converged and, with history=True, the
    list of (x_k, lambda_k) for k = 0..iterations."""
    if alpha < 0:
        raise ValueError("alpha must be >= 0 (convex SS-HOPM)")
    x = np.asarray(x0, dtype=np.float64)
    x = x / _norm2(x)
    y = sttsv(eptr, eidx, n, r, x)
    lam = math.fsum((x * y).tolist())
    hist = [(x.copy(), lam)]
    converged = False
    it = 0
    while it < max_iter:
        w = y + alpha * x
        x = w / _norm2(w)
        y = sttsv(eptr, eidx, n, r, x)
        lam_new = math.fsum((x * y).tolist())
        it += 1
        if history:
            hist.append((x.copy(), lam_new))
        done = tol > 0 and abs(lam_new - lam) <= tol * abs(lam_new)
        lam = lam_new
        if done:
            converged = True
            break
    res = _norm2(y - lam * x)
    info = dict(iterations=it, lambda_=lam, residual=res, converged=converged)
    if history:
        info["history"] = hist
    return x, info
