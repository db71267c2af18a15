"""The CCSS forest built on the GPU (Sec. III) against the oracle's forest,
node for node, and Alg. 4's memoised STTSV over it against the Alg. 2 oracle
(FP64 series: 1e-12 relative per vertex)."""
import sys

import numpy as np
import pytest

from oracle import ccss_ref as cr
from oracle import plan_ref
from oracle import sttsv_ref as sr
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relerr(y, ref):
    den = np.where(ref != 0, np.abs(ref), 1.0)
    return float(np.max(np.abs(y - ref) / den)) if len(ref) else 0.0


def _mixed(seed, n, m, r, kmin, kmax, extra=()):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m)
    eptr, eidx = wl.uniform_members(rng, n, sizes)
    if extra:
        eptr = np.concatenate([eptr, eptr[-1] + np.cumsum([len(e) for e in extra])])
        eidx = np.concatenate([eidx, np.array([v for e in extra for v in e], dtype=np.int32)])
    return eptr, eidx, wl.uniform_x(rng, n)


def _canonical_slot_edges(ref):
    out = np.empty(len(ref["mem"]), dtype=np.int64)
    off = ebase = 0
    for k, mk in zip(ref["bucket_k"], ref["bucket_m"]):
        for j in range(k):
            out[off + j * mk: off + (j + 1) * mk] = ebase + np.arange(mk)
        off += k * mk
        ebase += mk
    return out


def test_forest_matches_oracle_node_for_node():
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import _lib
    # random edges plus a sunflower and a nested chain (shared prefixes)
    extra = [(0, 1, 2, 10 + i) for i in range(6)] + [tuple(range(k)) for k in (2, 4, 7)]
    eptr, eidx, x = _mixed(81, 300, 2500, 9, 1, 9, extra)
    n = 300
    ref = plan_ref.canonical_plan(eptr, eidx, n)
    f = cr.build_forest(eptr, eidx, n, key=ref["rank"])
    c = cr.counts(f)
    with st.Plan(eptr, eidx, n, 9) as plan:
        info = plan.ccss_build()
        _say(f"[ccss] {info}")
        assert (info["levels"], info["nodes"], info["roots"], info["leaves"]) == \
            (len(f["levels"]), c["nodes"], c["roots"], c["leaves"])
        nl = plan.ccss_query(_lib.Q_CCSS_LEVEL_N, info["levels"])
        assert nl.tolist() == [len(v) for v, _ in f["levels"]]
        np.testing.assert_array_equal(plan.ccss_query(_lib.Q_CCSS_VERT, info["nodes"]),
                                      np.concatenate([v for v, _ in f["levels"]]))
        np.testing.assert_array_equal(plan.ccss_query(_lib.Q_CCSS_PARENT, info["nodes"]),
                                      np.concatenate([p for _, p in f["levels"]]))
        leaf = plan.ccss_query(_lib.Q_CCSS_LEAF, len(eidx))
    # the special leaf of every (edge, member) pair sits at the same node
    own = {(int(e), int(v)): int(q) for e, v, q in zip(f["edge"], f["member"], f["leaf_node"])}
    edges = ref["perm"][_canonical_slot_edges(ref)]
    want = np.array([own[(int(e), int(v))] for e, v in zip(edges, ref["mem"])])
    np.testing.assert_array_equal(leaf, want)


CASES = [("r5_all_sizes", 82, 400, 3001, 5, 1, 5), ("r12", 83, 700, 4001, 12, 1, 12),
         ("r25", 84, 2000, 6007, 25, 1, 25), ("r50", 85, 3000, 5003, 50, 1, 50), ("r64", 86, 3000, 3001, 64, 1, 64)]


@pytest.mark.parametrize("name,seed,n,m,r,kmin,kmax", CASES)
def test_alg4_apply_matches_oracle(name, seed, n, m, r, kmin, kmax):
    import torch
    import paper_2311_08595_amd as st
    _say(f"[ccss apply] {name}")
    extra = [(0, 1, 2, 3 + i)[:min(4, r)] for i in range(8)] + [tuple(range(k)) for k in (2, 5, 8) if k <= r]
    eptr, eidx, x = _mixed(seed, n, m, r, kmin, kmax, extra)
    ref = sr.sttsv(eptr, eidx, n, r, x)
    with st.Plan(eptr, eidx, n, r) as plan:
        plan.ccss_build()
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        y1 = plan.apply_ccss(xd).cpu().numpy()
        y2 = plan.apply_ccss(xd).cpu().numpy()
    err = _relerr(y1, ref)
    _say(f"  max rel err {err:.3e}")
    assert err <= 1e-12
    assert y1.tobytes() == y2.tobytes()


def test_alg4_zipf_weighted_and_against_ccss_oracle():
    import torch
    import paper_2311_08595_amd as st
    w = wl.zipf_powerlaw(seed=87, n=20000, m=60000)
    n, r = w["n"], w["r"]
    wts = np.random.default_rng(88).uniform(0.2, 5.0, size=len(w["eptr"]) - 1)
    ref = sr.sttsv(w["eptr"], w["eidx"], n, r, w["x"], w=wts)
    with st.Plan(w["eptr"], w["eidx"], n, r, weights=wts) as plan:
        info = plan.ccss_build()
        y = plan.apply_ccss(torch.tensor(w["x"], dtype=torch.float64, device="cuda")).cpu().numpy()
    err = _relerr(y, ref)
    _say(f"[ccss] zipf n=2e4 weighted: {info['nodes']} nodes, max rel err {err:.3e}")
    assert err <= 1e-12
    # the oracle's own Alg. 4 on a smaller Zipf graph, same forest order
    w2 = wl.zipf_powerlaw(seed=89, n=2000, m=6000, kmax=12)
    rk = plan_ref.canonical_plan(w2["eptr"], w2["eidx"], w2["n"])["rank"]
    y_or = cr.sttsv_alg4(w2["eptr"], w2["eidx"], w2["n"], 12, w2["x"], key=rk)
    with st.Plan(w2["eptr"], w2["eidx"], w2["n"], 12) as plan:
        plan.ccss_build()
        y2 = plan.apply_ccss(torch.tensor(w2["x"], dtype=torch.float64, device="cuda")).cpu().numpy()
    assert _relerr(y2, y_or) <= 1e-12


def test_ccss_errors():
    import torch
    import paper_2311_08595_amd as st
    from paper_2311_08595_amd import SttsvError, _lib
    eptr, eidx, x = _mixed(90, 50, 100, 4, 1, 4)
    with st.Plan(eptr, eidx, 50, 4) as plan:
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        with pytest.raises(SttsvError) as e:
            plan.apply_ccss(xd)                       # no forest yet
        assert e.value.code == _lib.STTSV_EINVAL
    with st.Plan.batch([(eptr, eidx, 50, 4), (eptr, eidx, 50, 4)]) as pb:
        with pytest.raises(SttsvError) as e:
            pb.ccss_build()
        assert e.value.code == _lib.STTSV_ENOTSUP
