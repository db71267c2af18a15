"""Pins of the warm-start network oracle: its hand-written backward against
central finite differences (FP64), and the bfloat16 rounding helper."""
import numpy as np

from oracle import mpnn_ref as mr
from paper_2311_08595_amd import workloads as wl


def _small():
    w = wl.zipf_powerlaw(seed=3, n=60, m=150, kmax=6)
    e, i, n, _ = wl.largest_component(w["eptr"], w["eidx"], w["n"])
    return mr.Graph(e, i, n, 6)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, 3.14159, -2.5e-3])
    r = mr.bf16(vals)
    assert r[0] == 1.0
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7          # above the halfway point
    assert abs(r[4] - 3.14159) < 3.14159 * 2 ** -8
    # every result is exactly representable in 8 mantissa bits
    m, _ = np.frexp(r[r != 0])
    assert np.all((m * 2 ** 8) == np.round(m * 2 ** 8))


def test_features_by_hand():
    eptr = np.array([0, 2, 5, 7])
    eidx = np.array([0, 1, 1, 2, 3, 0, 3])
    F = mr.features(eptr, eidx, 4, 5)
    # vertex 0: edges {0,1} and {0,3}: d=2, sizes 2,2
    np.testing.assert_allclose(F[0], [np.log(3), np.log(2), np.log(2) / 4, np.log(3)])
    # vertex 2: edge {1,2,3}: d=1
    np.testing.assert_allclose(F[2], [np.log(2), np.log(3), 0.0, np.log(3)])


def test_backward_matches_finite_differences():
    g = _small()
    rng = np.random.default_rng(0)
    p = {k: rng.normal(0, 0.3, shp) for k, shp in mr.PARAM_SHAPES}
    xs = np.exp(rng.normal(0, 0.5, g.n))
    xs /= xs.sum()
    s, c = mr.forward(p, g)
    L, ds = mr.loss(s, xs)
    gr = mr.backward(p, g, c, ds)
    vec = mr.pack(p)
    gvec = mr.pack(gr)
    h = 1e-6
    for idx in rng.choice(len(vec), size=40, replace=False):
        vp, vm = vec.copy(), vec.copy()
        vp[idx] += h
        vm[idx] -= h
        Lp = mr.loss(mr.forward(mr.unpack(vp), g)[0], xs)[0]
        Lm = mr.loss(mr.forward(mr.unpack(vm), g)[0], xs)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gvec[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, gvec[idx])


def test_warm_start_is_positive_and_normalised():
    s = np.array([0.0, -1.0, 700.0, 699.0])
    x = mr.warm_start(s)
    assert np.all(x > 0) and abs(x.sum() - 1) < 1e-15


def test_forward_by_hand():
    # Four vertices, edges {0,1}, {1,2,3}, {0,3} (degrees 2, 2, 1, 2), a
    # feature column of 1, 2, 3, 4 and dyadic weights that route a few hidden
    # units; every value below was worked out by hand:
    #   H0_v = [v+1, relu(-(v+1)) = 0, 1/2, 0...]
    #   layer 1 (unit 0): edge means 3/2, 3, 5/2; vertex means A = 2, 9/4, 3, 11/4
    #   H1_v = [v+1, 2 A_v, relu(v+1 - A_v)] = [1,4,0], [2,9/2,0], [3,6,0], [4,11/2,5/4]
    #   layer 2: edge means of unit 1: 17/4, 16/3, 19/4; of unit 2: 0, 5/12, 5/8
    #            vertex means A2_1 = 9/2, 115/24, 16/3, 121/24; A2_2 = 5/16, 5/24, 5/12, 25/48
    #   H2_v = [relu(A2_1 - H1_0), relu(2 H1_2 - 4 A2_2), A2_2 + 1/8]
    #   s_v = H2_0 + 2 H2_1 - H2_2 + 1/4 = 53/16, 65/24, 49/24, 71/48
    # A vertex->edge or edge->vertex mean over the wrong count, or [A, H] in
    # place of [H, A], changes every score.
    eptr = np.array([0, 2, 5, 7])
    eidx = np.array([0, 1, 1, 2, 3, 0, 3])
    g = mr.Graph(eptr, eidx, 4, 5)
    g.F = np.zeros((4, 4))
    g.F[:, 0] = [1.0, 2.0, 3.0, 4.0]
    H = mr.H
    p = {k: np.zeros(shp) for k, shp in mr.PARAM_SHAPES}
    p["W0"][0, 0], p["W0"][0, 1], p["b0"][2] = 1.0, -1.0, 0.5
    p["W1"][0, 0], p["W1"][H, 1] = 1.0, 2.0
    p["W1"][0, 2], p["W1"][H, 2] = 1.0, -1.0
    p["b1"][3] = -0.25
    p["W2"][H + 1, 0], p["W2"][0, 0] = 1.0, -1.0
    p["W2"][2, 1], p["W2"][H + 2, 1] = 2.0, -4.0
    p["W2"][H + 2, 2], p["b2"][2] = 1.0, 0.125
    p["wout"][:3] = [1.0, 2.0, -1.0]
    p["bout"][0] = 0.25
    s, c = mr.forward(p, g)
    expect = np.array([53 / 16, 65 / 24, 49 / 24, 71 / 48])
    np.testing.assert_allclose(s, expect, rtol=4e-15, atol=0)
    np.testing.assert_allclose(c["H2"][:, :3], [[7 / 2, 0, 7 / 16], [67 / 24, 0, 1 / 3],
                                                [7 / 3, 0, 13 / 24], [25 / 24, 5 / 12, 31 / 48]],
                               rtol=4e-15, atol=0)
    # the loss is the mean square of the centred difference of s and log x*
    xs = np.exp(expect - 1.0)
    L, ds = mr.loss(s, xs)
    assert abs(L) <= 1e-30 and np.all(np.abs(ds) <= 1e-15)
    L, _ = mr.loss(s, np.exp(np.array([1.0, 0.0, 0.0, 0.0])))
    u = (s - s.mean()) - (np.array([1.0, 0, 0, 0]) - 0.25)
    assert abs(L - np.mean(u * u)) <= 1e-15


def test_stage_checks_follow_the_oracle():
    # the per-stage checks of the GPU test, fed the oracle's own intermediate
    # values, must reproduce the oracle's gradients (so they restate the
    # oracle's backward, stage by stage) and find no error
    import mpnn_bounds as mb
    g = _small()
    rng = np.random.default_rng(2)
    p = {k: np.asarray(rng.normal(0, 0.3, shp), np.float32).astype(np.float64) for k, shp in mr.PARAM_SHAPES}
    xs = np.exp(rng.normal(0, 0.5, g.n))
    xs /= xs.sum()
    s, c = mr.forward(p, g, bf=True)
    _, ds = mr.loss(s, xs)
    tr = {}
    gr = mr.backward(p, g, c, ds, bf=True, trace=tr)
    X0 = np.zeros((g.n, 16))
    X0[:, :4] = c["X0"]
    q = {"X0": X0, "Z0": c["Z0"], "Z1": c["Z1"], "Z2": c["Z2"], "X1": c["X1"], "X2": c["X2"],
         "s": s, "ds": ds}
    q.update(tr)
    for stage, err, ratio in mb.stage_checks(p, g, q, gr, xs):
        assert ratio <= 1e-3, (stage, err, ratio)
