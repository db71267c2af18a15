"""FP64 oracle for STTSV on the blowup tensor: the AAY computation of Alg. 2.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For every edge e (k = |e|) and every member v of e, Alg. 2 adds to s_v
    w(e)/|beta(e)| * (r-1)! * [E_r(x_v) * conv_{u in e\\v} Ebar_r(x_u)][r-1]
with w(e) = |e| (Sec. II), |beta(e)| = k! S(r,k) (footnote in Sec. II),
E_r(c) = [1, c, c^2/2!, ..., c^(r-1)/(r-1)!] and Ebar_r(c) = E_r(c) with its
constant term set to 0 (Sec. II-A).  The oracle does exactly that, in the
ordinary power-series basis, with a full-length (degrees 0..r-1) truncated
convolution per factor, vectorised over the edges of one size.

Two choices that change no value beyond rounding:
* each edge's term is a homogeneous polynomial of degree r-1 in that edge's
  x values (Eq. (2)), so the edge's x values are divided by s_e = max |x_u|
  over the edge before the series are formed and the term is multiplied by
  s_e^(r-1) afterwards; this keeps x^a/a! away from underflow when r is large;
* the terms of a vertex are summed with math.fsum (correctly rounded sum).

The weight w(e)/|beta(e)| * (r-1)! is formed from exact integers and rounded
to FP64 once.  Edge weights other than the paper's w(e) = |e| (the hypergraph
H = (V, E, w) of Sec. II is edge-weighted, and Alg. 2 takes w as input) are
passed as one positive FP64 value per input edge; the weight factor is then
formed exactly from that value and rounded once.
"""
import math
from fractions import Fraction

import numpy as np

from .blowup import beta_size


def weight_exact(r: int, k: int) -> Fraction:
    """w(e)/|beta(e)| * (r-1)! with w(e) = |e| = k (Sec. II and Alg. 2)."""
    return Fraction(k * math.factorial(r - 1), beta_size(r, k))


def weight_fp64(r: int, k: int) -> float:
    w = weight_exact(r, k)
    return w.numerator / w.denominator  # int/int true division rounds once


def edge_weight_fp64(r: int, k: int, w: float) -> float:
    """w(e)/|beta(e)| * (r-1)! for an edge of size k with weight w (an FP64
    value), formed exactly and rounded once."""
    f = Fraction(w) * Fraction(math.factorial(r - 1), beta_size(r, k))
    return f.numerator / f.denominator


def validate_weights(w, m):
    """Edge weights: one finite, positive FP64 value per edge (or None)."""
    if w is None:
        return None
    w = np.asarray(w, dtype=np.float64)
    if w.shape != (m,) or not np.all(np.isfinite(w)) or np.any(w <= 0):
        raise ValueError("edge weights must be m finite positive values")
    return w


def validate(eptr, eidx, n, r):
    """Input checks the oracle relies on; mirrors the problem statement
    (Sec. II): E is a set system of non-empty vertex subsets of size <= r."""
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    if n < 1 or r < 2:
        raise ValueError("need n >= 1 and r >= 2")
    if eptr[0] != 0 or eptr[-1] != len(eidx) or np.any(np.diff(eptr) < 1):
        raise ValueError("bad edge pointer array")
    if len(eidx) and (eidx.min() < 0 or eidx.max() >= n):
        raise ValueError("vertex id out of range")
    sizes = np.diff(eptr)
    if sizes.max(initial=0) > r:
        raise ValueError("edge larger than r")
    for k in np.unique(sizes):
        rows = np.flatnonzero(sizes == k)
        M = eidx[eptr[rows][:, None] + np.arange(k)[None, :]]
        Ms = np.sort(M, axis=1)
        if k > 1 and np.any(Ms[:, 1:] == Ms[:, :-1]):
            raise ValueError("repeated vertex inside an edge")
    return eptr, eidx


def _edge_terms(M, x, r, k, chunk=1 << 15, members=None, wts=None):
    """Terms of Alg. 2 for a block of edges of size k.

    M: (m_k, k) member ids.  Returns (m_k, k) FP64 terms, column p being the
    term of member M[:, p].  ``members`` limits the work to those columns
    (the others are left undefined).  ``wts``: per-row weight factors
    w(e)/|beta(e)| (r-1)! (default: the factor of w(e) = |e|)."""
    wk = weight_fp64(r, k)
    inv_fact = np.array([1.0 / math.factorial(a) for a in range(r)])
    out = np.empty(M.shape, dtype=np.float64)
    for c0 in range(0, M.shape[0], chunk):
        Mc = M[c0:c0 + chunk]
        xs = x[Mc]                                   # (b, k)
        s = np.max(np.abs(xs), axis=1)
        s = np.where(s > 0, s, 1.0)
        xt = xs / s[:, None]
        # powers xt^a / a!  (b, k, r)
        a = np.arange(r)
        E = xt[:, :, None] ** a[None, None, :] * inv_fact[None, None, :]
        Eb = E.copy()
        Eb[:, :, 0] = 0.0
        scale = s ** (r - 1)
        for p in (range(k) if members is None else members):
            c = E[:, p, :].copy()                    # E_r(x_v)
            for q in range(k):
                if q == p:
                    continue
                eb = Eb[:, q, :]
                nc = np.zeros_like(c)
                # truncated convolution: nc[d] = sum_{j=1..d} eb[j] c[d-j]
                for j in range(1, r):
                    nc[:, j:] += eb[:, j:j + 1] * c[:, :r - j]
                c = nc
            wrow = wk if wts is None else wts[c0:c0 + chunk]
            out[c0:c0 + chunk, p] = wrow * c[:, r - 1] * scale
    return out


def _row_weights(w, rows, r, k):
    if w is None:
        return None
    return np.array([edge_weight_fp64(r, k, float(v)) for v in w[rows]])


def incidence_terms(eptr, eidx, n, r, x, w=None):
    """All (vertex, term) pairs of Alg. 2, one per incidence, in input order
    (edge by edge, member by member).  ``w``: per-edge weights or None
    (w(e) = |e|)."""
    eptr, eidx = validate(eptr, eidx, n, r)
    w = validate_weights(w, len(eptr) - 1)
    x = np.asarray(x, dtype=np.float64)
    sizes = np.diff(eptr)
    terms = np.empty(len(eidx), dtype=np.float64)
    for k in np.unique(sizes):
        rows = np.flatnonzero(sizes == k)
        pos = eptr[rows][:, None] + np.arange(k)[None, :]
        M = eidx[pos]
        terms[pos.ravel()] = _edge_terms(M, x, r, int(k), wts=_row_weights(w, rows, r, int(k))).ravel()
    return eidx, terms


def sttsv(eptr, eidx, n, r, x, w=None):
    """y = B x^(r-1) (TTSV1, Eq. (2)) for the blowup tensor B, by Alg. 2.
    Each y_v is the correctly rounded sum of its FP64 terms.  ``w``: per-edge
    weights of H = (V, E, w) (default w(e) = |e|, Sec. II)."""
    verts, terms = incidence_terms(eptr, eidx, n, r, x, w)
    order = np.argsort(verts, kind="stable")
    vs = verts[order]
    ts = terms[order]
    bounds = np.searchsorted(vs, np.arange(n + 1))
    y = np.zeros(n, dtype=np.float64)
    for v in range(n):
        a, b = bounds[v], bounds[v + 1]
        if b > a:
            y[v] = math.fsum(ts[a:b].tolist())
    return y


def sttsv_at(eptr, eidx, n, r, x, nodes, w=None):
    """y_v for a list of vertices only: each requested y_v is the fsum of
    the terms of the edges that contain v.  Used to check full-size runs on
    sampled outputs.

    Only the requested members' terms are formed: each (edge, requested
    member) pair becomes a row with that member first and the others after
    it in their original order, and column 0 of that row is computed.  The
    factors of a term are then multiplied in the same order as in ``sttsv``,
    so every term, and every y_v, is bitwise the same as there."""
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    x = np.asarray(x, dtype=np.float64)
    w = validate_weights(w, len(eptr) - 1)
    nodes = np.asarray(nodes, dtype=np.int64)
    want = np.zeros(n, dtype=bool)
    want[nodes] = True
    edge_of = np.repeat(np.arange(len(eptr) - 1), np.diff(eptr))
    hit = np.unique(edge_of[want[eidx]])
    sizes = np.diff(eptr)[hit]
    acc = {int(v): [] for v in nodes}
    for k in np.unique(sizes):
        k = int(k)
        rows = hit[sizes == k]
        M = eidx[eptr[rows][:, None] + np.arange(k)[None, :]]
        er, ep = np.nonzero(want[M])                 # (edge row, member position) pairs
        # column order per pair: the member itself, then the others in order
        rest = np.arange(k)[None, :].repeat(len(ep), axis=0)
        rest = rest[rest != ep[:, None]].reshape(len(ep), k - 1)
        Mp = np.take_along_axis(M[er], np.concatenate([ep[:, None], rest], axis=1), axis=1)
        T = _edge_terms(Mp, x, r, k, members=(0,), wts=_row_weights(w, rows[er], r, k))[:, 0]
        for v, t in zip(Mp[:, 0].tolist(), T.tolist()):
            acc[v].append(t)
    return np.array([math.fsum(acc[int(v)]) for v in nodes])
