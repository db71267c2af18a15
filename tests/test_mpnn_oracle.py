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
