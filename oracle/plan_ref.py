"""Reference construction of the canonical plan layout (bit-exact check).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The layout is this library's own format (the paper's CCSS forest, Sec. III,
is prior art for it: edges are kept as sorted vertex sequences, Sec. II-B,
and grouped by size, the levels L_k of Sec. III).  Definition:

1. deg(v) = number of edges containing v.
2. Vertex order: vertices sorted by (deg descending, id ascending);
   rank(v) = position in that order.  Hubs come first, so edges that share
   hubs share sorted prefixes (the shared-prefix structure CCSS exploits).
3. Every edge lists its members by increasing rank.
4. Canonical edge order: by (size k, member-rank sequence lexicographically,
   input edge index).  ``perm[c]`` is the input index of canonical edge c.
5. Size buckets: the canonical order is a run of buckets of increasing k;
   bucket k holds m_k edges.
6. Member slots: slot_off(k) = sum_{k' < k} k' m_k'.  Member j (in rank
   order) of the i-th edge of bucket k sits at slot slot_off(k) + j m_k + i
   (structure-of-arrays, so consecutive edges are consecutive slots).
   ``mem[slot]`` is the member's original vertex id.
7. Node-major incidence: for every vertex v, the slots holding v ordered by
   canonical edge index; ``tptr`` (n+1) and ``tslot`` (nnz).

Written with numpy sorts only, independently of the C++ planner.
"""
import numpy as np


def canonical_plan(eptr, eidx, n):
    eptr = np.asarray(eptr, dtype=np.int64)
    eidx = np.asarray(eidx, dtype=np.int64)
    m = len(eptr) - 1
    sizes = np.diff(eptr)
    deg = np.bincount(eidx, minlength=n)
    order = np.lexsort((np.arange(n), -deg))        # primary: -deg, then id
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)

    ks = np.unique(sizes)
    perm_parts, mem_parts, bucket_k, bucket_m = [], [], [], []
    for k in ks:
        rows = np.flatnonzero(sizes == k)
        M = eidx[eptr[rows][:, None] + np.arange(k)[None, :]]
        R = rank[M]
        srt = np.argsort(R, axis=1, kind="stable")
        R = np.take_along_axis(R, srt, axis=1)
        M = np.take_along_axis(M, srt, axis=1)
        # lexsort: last key is primary -> (rows, R[:, k-1], ..., R[:, 0])
        keys = [rows] + [R[:, j] for j in range(k - 1, -1, -1)]
        o = np.lexsort(keys)
        perm_parts.append(rows[o])
        mem_parts.append(M[o].T.ravel())            # SoA: j-major
        bucket_k.append(int(k))
        bucket_m.append(len(rows))
    perm = np.concatenate(perm_parts) if perm_parts else np.zeros(0, np.int64)
    mem = np.concatenate(mem_parts) if mem_parts else np.zeros(0, np.int64)

    # node-major incidence lists in canonical edge order
    slot_edge = np.empty(len(mem), dtype=np.int64)   # canonical edge of each slot
    off = 0
    ebase = 0
    for k, mk in zip(bucket_k, bucket_m):
        i = np.arange(mk)
        for j in range(k):
            slot_edge[off + j * mk: off + (j + 1) * mk] = ebase + i
        off += k * mk
        ebase += mk
    o = np.lexsort((slot_edge, mem))                 # by vertex, then canonical edge
    tslot = o.astype(np.int64)
    tptr = np.concatenate([[0], np.cumsum(np.bincount(mem, minlength=n))])
    return dict(perm=perm, mem=mem, bucket_k=np.array(bucket_k, np.int64),
                bucket_m=np.array(bucket_m, np.int64), tptr=tptr, tslot=tslot,
                rank=rank)
