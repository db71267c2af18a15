"""Exact-rational definitions of the blowup tensor and TTSV1.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything here is written straight from the definitions in Sec. II of the
paper, in Python integers and ``fractions.Fraction``; it is meant for tiny
hypergraphs (n <= 8, r <= 5) where every tensor entry can be listed.

Reading taken (the set definition of beta(e) in Sec. II only asks that every
vertex of e appear in the tuple; the footnote's count |e|! S(N, |e|) is the
number of surjections onto e, so the tuple's entries must also lie in e):
    beta(e) = { (i_1..i_r) in e^r : {i_1..i_r} = e }.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial


@lru_cache(maxsize=None)
def stirling2(n: int, k: int) -> int:
    """Stirling number of the second kind S(n, k) (footnote in Sec. II), by
    the recurrence S(n,k) = k S(n-1,k) + S(n-1,k-1)."""
    if n == 0 and k == 0:
        return 1
    if n == 0 or k == 0:
        return 0
    if k > n:
        return 0
    return k * stirling2(n - 1, k) + stirling2(n - 1, k - 1)


def beta_size(r: int, k: int) -> int:
    """|beta(e)| for |e| = k in an order-r blowup tensor: k! S(r, k)
    (footnote in Sec. II)."""
    return factorial(k) * stirling2(r, k)


def blowup_value(r: int, k: int, w=None) -> Fraction:
    """Value of every entry of beta(e): w(e)/|beta(e)|, with the paper's
    weight w(e) = |e| (Sec. II) unless ``w`` is given."""
    if w is None:
        w = k
    return Fraction(w, beta_size(r, k))


def beta_tuples(edge, r: int):
    """All r-tuples over the vertices of ``edge`` whose entry set is exactly
    the edge (the blowups of the edge, Sec. II)."""
    e = tuple(edge)
    es = set(e)
    return [t for t in product(e, repeat=r) if set(t) == es]


def blowup_entries(edges, r: int, weights=None) -> dict:
    """Every non-zero of the order-r blowup tensor, listed one by one:
    {index tuple: Fraction}.  Distinct edges give disjoint beta(e); a repeated
    edge (multiset input) adds its value again.  ``weights``: w(e) per edge
    (exact numbers, e.g. Fractions of FP64 values), default w(e) = |e|."""
    B = {}
    for q, e in enumerate(edges):
        k = len(e)
        if k > r:
            raise ValueError("edge larger than the tensor order")
        val = blowup_value(r, k, None if weights is None else Fraction(weights[q]))
        for t in beta_tuples(e, r):
            B[t] = B.get(t, Fraction(0)) + val
    return B


def ttsv1_from_entries(B: dict, n: int, r: int, x) -> list:
    """TTSV1 by its index definition, Eq. (2):
    y_{i1} = sum_{i2..ir} B_{i1..ir} prod_{j>=2} x_{ij}, summed over the
    listed non-zeros.  ``x`` entries may be Fractions (exact) or floats."""
    y = [Fraction(0)] * n if isinstance(x[0], Fraction) else [0.0] * n
    for t, val in B.items():
        p = val
        for i in t[1:]:
            p = p * x[i]
        y[t[0]] = y[t[0]] + p
    return y


def full_contraction_from_entries(B: dict, r: int, x):
    """B x^r = sum over all entries of B_i prod_j x_{ij}."""
    s = Fraction(0)
    for t, val in B.items():
        p = val
        for i in t:
            p = p * x[i]
        s += p
    return s


def _E(c, r):
    """E_N(c) of Sec. II-A: [1, c, c^2/2!, ..., c^(r-1)/(r-1)!]."""
    return [c ** a / factorial(a) for a in range(r)]


def _Ebar(c, r):
    """Ebar_N(c) of Sec. II-A: E_N(c) with its constant term set to 0."""
    v = _E(c, r)
    v[0] = 0 * v[0]
    return v


def _conv_trunc(a, b, r):
    """(a * b)[k] = sum_{i<=k} a_i b_{k-i}, kept for degrees 0..r-1
    (Sec. II-A; the paper's 'length N+1' is read as degrees 0..N-1)."""
    return [sum(a[i] * b[kk - i] for i in range(kk + 1)) for kk in range(r)]


def aay_exact(edges, n: int, r: int, x) -> list:
    """Alg. 2 (AAY implicit TTSV1) in exact arithmetic, written out as
    printed: for every vertex v and every edge e containing v,
        c += w(e)/|beta(e)| * (r-1)! * (E(x_v) * conv_{u in e\\v} Ebar(x_u))[r-1]
    with w(e) = |e|.  ``x`` entries should be Fractions."""
    y = [Fraction(0)] * n
    for e in edges:
        k = len(e)
        wgt = blowup_value(r, k) * factorial(r - 1)
        for v in e:
            c = _E(x[v], r)
            for u in e:
                if u != v:
                    c = _conv_trunc(c, _Ebar(x[u], r), r)
            y[v] += wgt * c[r - 1]
    return y


def inclusion_exclusion_term(e, v, r: int, x) -> Fraction:
    """Closed form of one (edge, vertex) term, independent of the series
    arithmetic.  Counting the (r-1)-tuples over e that cover e\\{v} by
    inclusion-exclusion over the vertices left out gives
        (r-1)! [t^(r-1)] e^{x_v t} prod_{u != v} (e^{x_u t} - 1)
          = sum_{S subset e\\v} (-1)^{|e|-1-|S|} (x_v + sum_{u in S} x_u)^(r-1),
    and the term is w(e)/|beta(e)| times that."""
    others = [u for u in e if u != v]
    k = len(e)
    tot = Fraction(0)
    for mask in range(1 << len(others)):
        s = x[v]
        cnt = 0
        for j, u in enumerate(others):
            if mask >> j & 1:
                s = s + x[u]
                cnt += 1
        sign = -1 if (k - 1 - cnt) % 2 else 1
        tot += sign * s ** (r - 1)
    return blowup_value(r, k) * tot


def inclusion_exclusion_sttsv(edges, n: int, r: int, x) -> list:
    y = [Fraction(0)] * n
    for e in edges:
        for v in e:
            y[v] += inclusion_exclusion_term(e, v, r, x)
    return y
