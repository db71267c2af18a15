"""Host-side checks of the seeded generators and of the canonical-plan reference."""
import numpy as np

from oracle import plan_ref
from paper_2311_08595_amd import workloads as wl


def _check_csr(eptr, eidx, n, r):
    sizes = np.diff(eptr)
    assert sizes.min() >= 1 and sizes.max() <= r
    assert eidx.min() >= 0 and eidx.max() < n
    for k in np.unique(sizes):
        rows = np.flatnonzero(sizes == k)
        M = np.sort(eidx[eptr[rows][:, None] + np.arange(k)], axis=1)
        assert not np.any(M[:, 1:] == M[:, :-1])


def test_small_uniform_recipe():
    w = wl.small_uniform()
    assert w["n"] == 1000 and len(w["eptr"]) == 5001 and w["r"] == 5
    _check_csr(w["eptr"], w["eidx"], w["n"], w["r"])
    sizes = np.diff(w["eptr"])
    assert set(np.unique(sizes)) == {2, 3, 4, 5}
    assert (w["x"] > 0).all() and (w["x"] <= 1).all()
    w2 = wl.small_uniform()
    np.testing.assert_array_equal(w["eidx"], w2["eidx"])      # seeded


def test_scaled_down_recipes():
    w = wl.zipf_powerlaw(seed=9, n=20000, m=100000)
    _check_csr(w["eptr"], w["eidx"], w["n"], w["r"])
    sizes = np.diff(w["eptr"])
    frac2 = np.mean(sizes == 2)
    assert 0.5 < frac2 < 0.58                   # 2^-2.5 / sum_k k^-2.5 ~ 0.54
    deg = np.bincount(w["eidx"], minlength=w["n"])
    assert deg.max() > 50 * deg.mean()          # Zipf hubs
    h = wl.heavy_tail(seed=9, n=20000, m=100000)
    _check_csr(h["eptr"], h["eidx"], h["n"], h["r"])
    hs = np.diff(h["eptr"])
    assert 0.005 < np.mean(hs > 8) < 0.015


def test_largest_component():
    eptr = np.array([0, 2, 4, 6, 8], dtype=np.int64)
    eidx = np.array([0, 1, 1, 2, 5, 6, 6, 7], dtype=np.int32)   # {0,1,2} and {5,6,7}; 3,4 isolated
    e2, i2, n2, old = wl.largest_component(eptr, eidx, 8)
    assert n2 == 3 and list(old) == [0, 1, 2]
    assert list(e2) == [0, 2, 4] and sorted(i2.tolist()) == [0, 1, 1, 2]


def test_plan_reference_invariants():
    w = wl.zipf_powerlaw(seed=11, n=3000, m=9000, kmax=9)
    eptr, eidx, n = w["eptr"], w["eidx"], w["n"]
    p = plan_ref.canonical_plan(eptr, eidx, n)
    m = len(eptr) - 1
    assert sorted(p["perm"].tolist()) == list(range(m))
    deg = np.bincount(eidx, minlength=n)
    # rank order: degree descending, id ascending
    order = np.argsort(p["rank"])
    assert np.all(np.diff(deg[order]) <= 0)
    off = 0
    c = 0
    prev = None
    for k, mk in zip(p["bucket_k"], p["bucket_m"]):
        for i in range(mk):
            members = [int(p["mem"][off + j * mk + i]) for j in range(k)]
            src = p["perm"][c]
            assert sorted(members) == sorted(eidx[eptr[src]:eptr[src + 1]].tolist())
            ranks = [int(p["rank"][v]) for v in members]
            assert ranks == sorted(ranks)
            key = (k, ranks, src)
            if prev is not None:
                assert prev < key
            prev = key
            c += 1
        off += k * mk
    for v in range(0, n, 37):
        slots = p["tslot"][p["tptr"][v]:p["tptr"][v + 1]]
        assert np.all(p["mem"][slots] == v)
        assert len(slots) == deg[v]


def test_paper_synthetic_recipe():
    """S1-S4 (n=2500, m=25000, ranks 30..60): only multiples of 5 up to N_k,
    equal edge counts per size (within one), no repeated member, r = N_k."""
    for nk in (30, 40, 50, 60):
        d = wl.paper_synthetic(nk)
        sizes = np.diff(d["eptr"])
        assert d["n"] == 2500 and len(sizes) == 25000 and d["r"] == nk
        ks, counts = np.unique(sizes, return_counts=True)
        assert list(ks) == list(range(5, nk + 1, 5))
        assert counts.max() - counts.min() <= 1 and counts.sum() == 25000
        for e in range(0, len(sizes), 997):
            mem = d["eidx"][d["eptr"][e]:d["eptr"][e + 1]]
            assert len(set(mem.tolist())) == len(mem)
        assert d["eidx"].min() >= 0 and d["eidx"].max() < 2500
        assert np.all(d["x"] > 0) and np.all(d["x"] <= 1)
    a, b = wl.paper_synthetic(40), wl.paper_synthetic(40)
    assert np.array_equal(a["eidx"], b["eidx"]) and np.array_equal(a["x"], b["x"])
