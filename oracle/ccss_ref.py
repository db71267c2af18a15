"""The Compound CSS forest (Sec. III) and the memoised STTSV over it (Alg. 4,
Sec. IV-B), in FP64, written from the paper's definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Forest.  Every edge e of size k >= 2 is listed in increasing order of a
vertex key (the paper's in-order listing uses the vertex index; any order can
be passed).  For every member u of e the sorted sequence e \\ {u} (length
k - 1) is a root-to-level-(k-1) path of the forest, and the pair (e, u) is a
special leaf owned by the node that ends the path.  The forest is the trie of
all these paths: a node is a distinct prefix, its level is the prefix length,
roots are level-1 nodes.  Nodes of a level are numbered in increasing (parent
number, vertex key) order; that numbering is what ``build_forest`` returns and
what a device construction must reproduce.  Only paths that end in a special
leaf are ever created, which is the paper's trimming.  Size-1 edges own no
path; their term is w(e) x_u^(r-1) (the blowup of {u} is one entry).

Memoised STTSV (Alg. 4).  The workspace of a node is the truncated
convolution (degrees 0..r-1) of Ebar(x_v) over the vertices v of its path,
obtained from its parent's by one more convolution (the forest edge), and the
term of a special leaf (e, u) owned by it is
    w(e)/|beta(e)| (r-1)! sum_a x_u^a / a! * workspace[r - 1 - a]
(the dot product of the leaf's coefficients with the workspace column).  The
order of the traversal does not change any value (a node's workspace depends
only on its path), so the levels are processed one after another here.

Scaling (exact by homogeneity, Eq. (2)): the workspace coefficient of degree d
is homogeneous of degree d in the path's x, so each node keeps it for the x
divided by s = max |x| over its path, and a leaf rescales it to its edge's
s_e = max(s, |x_u|) by (s / s_e)^d.  This keeps x^a/a! away from underflow for
large r, as the per-edge scaling of the plain oracle does.

Readings (the paper's counts in Sec. IV-C are stated for this forest):
* A node is a distinct prefix; "convolutions" are forest edges, i.e. nodes
  minus roots (Sec. IV-C: one less than the number of nodes, per tree).
* For one edge of size k >= 2 that gives (k-1)(k+2)/2 nodes on 2 roots, hence
  (k^2 + k - 6)/2 convolutions; the paper prints (k^2 - k)/2 for the single
  edge, while its nested-chain count reduces to (k^2 + k - 2)/2 -- our node
  count -- for a chain of one edge.  The pins use our counts, derived by hand.
  With them, one edge needs fewer than half of Alg. 3's k(k-1) convolutions
  only for k <= 3; the saving the paper measures comes from prefixes shared
  between edges, which the trie merges.
* The in-order listing may use any vertex order; the library lists members by
  degree rank (a relabelling of the vertices), which shares more prefixes.
"""
import math

import numpy as np

from .sttsv_ref import edge_weight_fp64, validate, validate_weights, weight_fp64


def build_forest(eptr, eidx, n, key=None):
    """The CCSS forest of a hypergraph.  ``key``: sort key of every vertex
    (default: the vertex index).  Returns dict(levels=[(vertex, parent), ...]
    per level 1, 2, ... (parent indexes the previous level, -1 at level 1),
    leaf_node=int64[nnz] (node, at level |e| - 1, owning the special leaf of
    every incidence in input order; -1 for size-1 edges), member=int64[nnz]
    (the incidence's vertex), edge=int64[nnz])."""
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    key = np.arange(n, dtype=np.int64) if key is None else np.asarray(key, dtype=np.int64)
    m = len(eptr) - 1
    sizes = np.diff(eptr)
    edge_of = np.repeat(np.arange(m), sizes)
    # every edge's members in increasing key order
    order = np.lexsort((key[eidx], edge_of))
    mem = eidx[order]
    start = np.repeat(eptr[:-1], sizes)
    pos = np.arange(len(eidx)) - start            # position of the incidence's member in its sorted edge
    klen = sizes[edge_of]
    node = np.full(len(eidx), -1, dtype=np.int64)  # current node of every path (one path per incidence)
    levels = []
    depth = 0
    while True:
        act = np.flatnonzero(klen - 1 > depth)      # paths of length > depth
        if act.size == 0:
            break
        j = pos[act]
        elem = mem[start[act] + np.where(depth < j, depth, depth + 1)]   # member number depth of e \ u
        parent = node[act] if depth > 0 else np.zeros(act.size, dtype=np.int64)
        kk = parent * np.int64(n) + key[elem]
        uniq, first, inv = np.unique(kk, return_index=True, return_inverse=True)
        node[act] = inv
        levels.append((elem[first], (parent[first] if depth > 0 else np.full(len(uniq), -1, dtype=np.int64))))
        depth += 1
    leaf = np.full(len(eidx), -1, dtype=np.int64)
    leaf[order] = np.where(klen >= 2, node, -1)     # back to input incidence order
    return dict(levels=levels, leaf_node=leaf, member=eidx.copy(), edge=edge_of)


def counts(forest):
    """Nodes, roots, convolutions (= forest edges) and special leaves."""
    nodes = sum(len(v) for v, _ in forest["levels"])
    roots = len(forest["levels"][0][0]) if forest["levels"] else 0
    leaves = int(np.sum(forest["leaf_node"] >= 0))
    return dict(nodes=nodes, roots=roots, convolutions=nodes - roots, leaves=leaves)


def sttsv_alg4(eptr, eidx, n, r, x, forest=None, key=None, w=None):
    """y = B x^(r-1) by Alg. 4 over the CCSS forest (FP64, ordinary basis,
    full-length workspaces); per-vertex sums with math.fsum."""
    eptr, eidx = validate(eptr, eidx, n, r)
    w = validate_weights(w, len(eptr) - 1)
    x = np.asarray(x, dtype=np.float64)
    if forest is None:
        forest = build_forest(eptr, eidx, n, key)
    inv_fact = np.array([1.0 / math.factorial(a) for a in range(r)])
    deg = np.arange(r)
    work, scale = [], []                         # per level: (N, r) workspace on x / s, and s
    for depth, (vert, par) in enumerate(forest["levels"]):
        xv = x[vert]
        if depth == 0:
            s = np.abs(xv)
            Wp = np.zeros((len(vert), r))
            Wp[:, 0] = 1.0                       # empty path: the constant 1
            sp = s
        else:
            sp = scale[-1][par]
            s = np.maximum(sp, np.abs(xv))
            Wp = work[-1][par] * (np.where(s > 0, sp / np.where(s > 0, s, 1.0), 1.0)[:, None] ** deg[None, :])
        s = np.where(s > 0, s, 1.0)
        z = xv / s
        Eb = z[:, None] ** deg[None, :] * inv_fact[None, :]
        Eb[:, 0] = 0.0                           # Ebar: constant term dropped
        Wn = np.zeros_like(Wp)
        for a in range(1, r):                    # truncated convolution Wp * Ebar(z)
            Wn[:, a:] += Eb[:, a:a + 1] * Wp[:, :r - a]
        work.append(Wn)
        scale.append(s)
    sizes = np.diff(eptr)
    edge_of = forest["edge"]
    terms = np.empty(len(eidx))
    for q in range(len(eidx)):
        e = edge_of[q]
        k = int(sizes[e])
        u = eidx[q]
        if k == 1:                               # the single blowup entry of {u}, value w(e)
            terms[q] = (1.0 if w is None else float(w[e])) * x[u] ** (r - 1)
            continue
        wk = weight_fp64(r, k) if w is None else edge_weight_fp64(r, k, float(w[e]))
        nd = forest["leaf_node"][q]
        Wq, sq = work[k - 2][nd], scale[k - 2][nd]
        se = max(sq, abs(x[u]))
        Wr = Wq * (sq / se) ** deg
        zu = x[u] / se
        coefs = zu ** deg * inv_fact              # E(x_u) on the edge's scale
        terms[q] = wk * se ** (r - 1) * float(np.dot(coefs, Wr[::-1]))
    y = np.zeros(n)
    order = np.argsort(eidx, kind="stable")
    bounds = np.searchsorted(eidx[order], np.arange(n + 1))
    for v in range(n):
        a, b = bounds[v], bounds[v + 1]
        if b > a:
            y[v] = math.fsum(terms[order[a:b]].tolist())
    return y
