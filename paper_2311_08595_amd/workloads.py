"""Seeded synthetic hypergraph workloads.

This module generates inputs only (edge lists and vectors); it holds none of
the STTSV / NQZ arithmetic.  Both the HIP path and the CPU oracle are fed
from here.

Hypergraphs are returned as a CSR pair: ``eptr`` (int64, m+1) and ``eidx``
(int32, nnz) with 0-based vertex ids; edge i is eidx[eptr[i]:eptr[i+1]].

Recipes (seeded numpy PCG64):
* ``uniform_sizes``       sizes uniform on {kmin..kmax}
* ``powerlaw_sizes``      P(k) proportional to k^-a on [kmin, kmax]
* ``geometric_mix_sizes`` with prob 1-q a truncated geometric P(k) ~ (1-p)^(k-kmin)
                          on [kmin, kmax], with prob q uniform on [tlo, thi]
* ``uniform_members``     members uniform over V, without replacement in an edge
* ``zipf_members``        sequential draws with P(rank j) ~ 1/j^s, a repeat
                          inside an edge is redrawn; rank -> vertex id through
                          a seeded random permutation
"""
import numpy as np


def uniform_sizes(rng, m, kmin, kmax):
    return rng.integers(kmin, kmax + 1, size=m)


def powerlaw_sizes(rng, m, a, kmin, kmax):
    ks = np.arange(kmin, kmax + 1)
    p = ks.astype(np.float64) ** (-a)
    p /= p.sum()
    return rng.choice(ks, size=m, p=p)


def geometric_mix_sizes(rng, m, p, kmin, kmax, q, tlo, thi):
    ks = np.arange(kmin, kmax + 1)
    w = (1.0 - p) ** (ks - kmin)
    w /= w.sum()
    body = rng.choice(ks, size=m, p=w)
    tail = rng.integers(tlo, thi + 1, size=m)
    use_tail = rng.random(m) < q
    return np.where(use_tail, tail, body)


def _fill_without_repeats(rng, sizes, draw):
    """Members for every edge: ``draw(rng, count)`` gives vertex ids; rows with
    a repeated vertex are redrawn until none is left."""
    m = len(sizes)
    eptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(sizes, out=eptr[1:])
    eidx = np.empty(int(eptr[-1]), dtype=np.int32)
    for k in np.unique(sizes):
        rows = np.flatnonzero(sizes == k)
        M = draw(rng, (len(rows), k))
        if k > 1:
            while True:
                S = np.sort(M, axis=1)
                bad = np.flatnonzero(np.any(S[:, 1:] == S[:, :-1], axis=1))
                if bad.size == 0:
                    break
                M[bad] = draw(rng, (bad.size, k))
        eidx[(eptr[rows][:, None] + np.arange(k)[None, :]).ravel()] = M.ravel()
    return eptr, eidx


def uniform_members(rng, n, sizes):
    if np.max(sizes) > n:
        raise ValueError("edge larger than the vertex set")
    return _fill_without_repeats(rng, sizes, lambda g, shp: g.integers(0, n, size=shp))


def zipf_members(rng, n, sizes, s=1.0):
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    ids = rng.permutation(n).astype(np.int64)        # rank -> vertex id

    def draw(g, shp):
        u = g.random(size=shp)
        rk = np.minimum(np.searchsorted(cdf, u, side="right"), n - 1)
        return ids[rk]
    return _fill_without_repeats(rng, sizes, draw)


def uniform_x(rng, n):
    """x uniform on (0, 1]."""
    return 1.0 - rng.random(n)


def largest_component(eptr, eidx, n):
    """Restrict a hypergraph to its largest connected component (vertices
    joined through shared edges), relabelled densely in increasing old id.
    Returns (eptr, eidx, n_lcc, old_ids)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    m = len(eptr) - 1
    sizes = np.diff(eptr)
    edge_of = np.repeat(np.arange(m), sizes)
    # bipartite vertex-edge incidence graph
    rows = np.concatenate([eidx.astype(np.int64), n + edge_of])
    cols = np.concatenate([n + edge_of, eidx.astype(np.int64)])
    g = sp.coo_matrix((np.ones(len(rows), np.int8), (rows, cols)), shape=(n + m, n + m)).tocsr()
    ncomp, lab = connected_components(g, directed=False)
    vlab = lab[:n]
    deg = np.bincount(eidx, minlength=n)
    counts = np.bincount(vlab[deg > 0], minlength=ncomp)
    big = int(np.argmax(counts))
    keep_v = (vlab == big) & (deg > 0)
    old_ids = np.flatnonzero(keep_v)
    new_id = np.full(n, -1, dtype=np.int64)
    new_id[old_ids] = np.arange(len(old_ids))
    keep_e = lab[n:] == big
    ke = np.flatnonzero(keep_e)
    ks = sizes[ke]
    neptr = np.zeros(len(ke) + 1, dtype=np.int64)
    np.cumsum(ks, out=neptr[1:])
    src = (np.repeat(eptr[ke], ks) + (np.arange(neptr[-1]) - np.repeat(neptr[:-1], ks)))
    neidx = new_id[eidx[src]].astype(np.int32)
    return neptr, neidx, len(old_ids), old_ids


# ---------------------------------------------------------------------------
# The named workloads (sizes and laws as specified for each benchmark case)
# ---------------------------------------------------------------------------

def small_uniform(seed=1, n=1000, m=5000, kmin=2, kmax=5):
    """n=1000, m=5000, sizes uniform on {2..5} (order r=5), members uniform
    without replacement, x uniform on (0,1]."""
    rng = np.random.default_rng(seed)
    sizes = uniform_sizes(rng, m, kmin, kmax)
    eptr, eidx = uniform_members(rng, n, sizes)
    x = uniform_x(rng, n)
    return dict(eptr=eptr, eidx=eidx, n=n, r=kmax, x=x, name="uniform-n1e3-m5e3-r5")


def zipf_powerlaw(seed=2, n=1_000_000, m=5_000_000, a=2.5, kmin=2, kmax=25, s=1.0):
    """n=1e6, m=5e6, sizes P(k) ~ k^-2.5 on [2,25] (r=25), Zipf(1.0)
    membership, x uniform on (0,1]."""
    rng = np.random.default_rng(seed)
    sizes = powerlaw_sizes(rng, m, a, kmin, kmax)
    eptr, eidx = zipf_members(rng, n, sizes, s)
    x = uniform_x(rng, n)
    return dict(eptr=eptr, eidx=eidx, n=n, r=kmax, x=x,
                name=f"zipf-n{n:.0e}-m{m:.0e}-r{kmax}".replace("+0", ""))


def heavy_tail(seed=3, n=200_000, m=2_000_000, p=0.4, r=50):
    """n=2e5, m=2e6, sizes: w.p. 0.99 truncated geometric (p=0.4) on [2,8],
    w.p. 0.01 uniform on [9,50]; order r=50; uniform membership."""
    rng = np.random.default_rng(seed)
    sizes = geometric_mix_sizes(rng, m, p, 2, 8, 0.01, 9, 50)
    eptr, eidx = uniform_members(rng, n, sizes)
    x = uniform_x(rng, n)
    return dict(eptr=eptr, eidx=eidx, n=n, r=r, x=x,
                name=f"heavytail-n{n:.0e}-m{m:.0e}-r{r}".replace("+0", ""))


def batch_graph(g, base_seed=4000, lo=3.0, hi=5.0, a=2.5):
    """Graph g of the batched workload: n = round(10^U(3,5)), m = 5n,
    r uniform on {3..12}, sizes P(k) ~ k^-2.5 on [2, r], uniform membership."""
    rng = np.random.default_rng(base_seed + g)
    n = int(round(10 ** rng.uniform(lo, hi)))
    r = int(rng.integers(3, 13))
    m = 5 * n
    sizes = powerlaw_sizes(rng, m, a, 2, r)
    eptr, eidx = uniform_members(rng, n, sizes)
    x = uniform_x(rng, n)
    return dict(eptr=eptr, eidx=eidx, n=n, r=r, x=x, name=f"batch-g{g}")


def warmstart_train_graph(i, n=10_000, base_seed=50_000):
    """Training graph i of the warm-start net: the Zipf/power-law recipe at
    n=1e4 (m=5e4, r=25)."""
    return zipf_powerlaw(seed=base_seed + i, n=n, m=5 * n)


def paper_synthetic(nk, seed=None, n=2500, m=25000):
    """The paper's synthetic sets S1-S4 (Sec. V, dataset table: n=2500,
    m=25000, rank N_k = 30, 40, 50, 60): the union of 5-, 10-, ..., N_k-uniform
    hypergraphs holding about the same number of edges each (m/(N_k/5), the
    remainder spread one edge each over the first sizes), members uniform
    without replacement; order r = N_k; x uniform on (0,1]."""
    if nk % 5 != 0 or nk < 5:
        raise ValueError("N_k must be a positive multiple of 5")
    rng = np.random.default_rng(6000 + nk if seed is None else seed)
    ks = np.arange(5, nk + 1, 5)
    per = np.full(len(ks), m // len(ks))
    per[: m - per.sum()] += 1
    sizes = rng.permutation(np.repeat(ks, per))
    eptr, eidx = uniform_members(rng, n, sizes)
    x = uniform_x(rng, n)
    return dict(eptr=eptr, eidx=eidx, n=n, r=nk, x=x, name=f"synthetic-S{nk // 10 - 2}-n{n}-m{m}-r{nk}")

