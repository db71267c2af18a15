"""Symmetric CP decomposition of the blowup tensor by gradient descent, the
second STTSV consumer Sec. I names (symmetric CP decomposition), on top of
the FP64 STTSV oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Model: B ~ sum_l lambda_l a_l^(o r) (R symmetric rank-one terms, a_l in R^n).
Objective, with <.,.> the entrywise inner product of order-r tensors:
    f(lambda, A) = ||B||^2 - 2 sum_l lambda_l B a_l^r
                   + sum_{l,m} lambda_l lambda_m (a_l . a_m)^r
where B a^r = a . (B a^(r-1)) (one STTSV) and
    ||B||^2 = sum over the blowup entries of their squares
            = sum_e |beta(e)| (w(e)/|beta(e)|)^2 = sum_e w(e)^2 / |beta(e)|
(edges on the same vertex set first add their weights: their blowups are
the same entries).
Gradient:
    df/dlambda_l = -2 B a_l^r + 2 sum_m lambda_m (a_l . a_m)^r
    df/da_l      = -2 r lambda_l B a_l^(r-1)
                   + 2 r lambda_l sum_m lambda_m (a_l . a_m)^(r-1) a_m
(R STTSVs per evaluation: the bottleneck Sec. I points at).

Optimizer (the paper names the decomposition, not a method; a plain one is
taken): gradient descent on (lambda, A) with Armijo backtracking.  Iteration:
g = grad f at (lambda, A); t = step; while
f((lambda, A) - t g) > f(lambda, A) - 1e-4 t ||g||^2 and fewer than 40
halvings: t = t / 2; accept the step; the next trial step is 2 t.
"""
import math
from fractions import Fraction

import numpy as np

from .blowup import beta_size
from .sttsv_ref import sttsv, validate_weights


def norm2(eptr, eidx, n, r, w=None):
    """||B||^2 = sum over distinct vertex sets S of W_S^2 / |beta(S)|, where
    W_S adds up the weights of the edges on S (a repeated edge adds its
    value to the same entries); exact rationals rounded once."""
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    sizes = np.diff(eptr)
    w = validate_weights(w, len(sizes))
    acc = {}
    for q, k in enumerate(sizes.tolist()):
        S = tuple(sorted(eidx[eptr[q]:eptr[q + 1]].tolist()))
        acc[S] = acc.get(S, Fraction(0)) + (Fraction(k) if w is None else Fraction(float(w[q])))
    tot = sum((W * W / beta_size(r, len(S)) for S, W in acc.items()), Fraction(0))
    return tot.numerator / tot.denominator


def objective_grad(eptr, eidx, n, r, lam, A, w=None, nb2=None):
    """(f, dlambda, dA) at (lam, A); A is n x R (column l = a_l)."""
    lam = np.asarray(lam, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    R = A.shape[1]
    Y = np.column_stack([sttsv(eptr, eidx, n, r, A[:, l], w) for l in range(R)])
    c = np.array([math.fsum((A[:, l] * Y[:, l]).tolist()) for l in range(R)])          # B a_l^r
    G = np.array([[math.fsum((A[:, l] * A[:, m]).tolist()) for m in range(R)] for l in range(R)])
    if nb2 is None:
        nb2 = norm2(eptr, eidx, n, r, w)
    Gr = G ** r
    f = nb2 - 2.0 * float(lam @ c) + float(lam @ Gr @ lam)
    dlam = -2.0 * c + 2.0 * Gr @ lam
    C = G ** (r - 1) * lam[None, :]                                                     # C_lm = lam_m G_lm^(r-1)
    dA = 2.0 * r * lam[None, :] * (-Y + A @ C.T)
    return f, dlam, dA


def gradient_descent(eptr, eidx, n, r, lam0, A0, iters, step, w=None, history=False):
    """The Armijo gradient descent above; returns (lam, A, info)."""
    lam = np.asarray(lam0, dtype=np.float64).copy()
    A = np.asarray(A0, dtype=np.float64).copy()
    nb2 = norm2(eptr, eidx, n, r, w)
    f, dl, dA = objective_grad(eptr, eidx, n, r, lam, A, w, nb2)
    fs = [f]
    halvings = []
    t = step
    for _ in range(iters):
        gg = math.fsum((dl * dl).tolist()) + math.fsum((dA * dA).ravel().tolist())
        h = 0
        while True:
            lt, At = lam - t * dl, A - t * dA
            ft, dlt, dAt = objective_grad(eptr, eidx, n, r, lt, At, w, nb2)
            if ft <= f - 1e-4 * t * gg or h >= 40:
                break
            t *= 0.5
            h += 1
        lam, A, f, dl, dA = lt, At, ft, dlt, dAt
        fs.append(f)
        halvings.append(h)
        t *= 2.0
    info = dict(f=f, norm2=nb2)
    if history:
        info["fs"] = fs
        info["halvings"] = halvings
    return lam, A, info
