"""Pins of three oracle helpers that the filters build on: the uniform-reuse
remap (Sec. 2.2 eq. uniform-sample-reuse), the FIS nearest-texel lookup
(Sec. 4.2) and the positivised Keys pick (Sec. 2.2 "Positivization")."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("filt", ["LINEAR", "BSPLINE3"])
def test_reuse_rescales_the_uniform_into_its_bin(orc, filt):
    """For u in bin j of the inverse-CDF pick, the reused uniform is
    (u - C_{j-1}) / (C_j - C_{j-1}) (C the cumulative weights), below 1,
    increasing in u, and uniform over the bin's lattice points."""
    f = getattr(orc, filt)
    rng = np.random.default_rng(4)
    for t in (0.0, 0.13, 0.5, 0.77, 0.999):
        t = float(np.float32(t))
        w = np.asarray(orc.axis_weights64(f, t), np.float64)
        w = w[:2] if filt == "LINEAR" else w
        C = np.concatenate([[0.0], np.cumsum(w)])
        for j in range(len(w)):
            if w[j] < 1e-6:
                continue
            us = np.sort(C[j] + (rng.random(400) * 0.998 + 0.001) * w[j])
            us = np.floor(us * 2 ** 24) / 2 ** 24
            r = np.array([orc.reuse(f, t, float(u), j) for u in us])
            assert np.all(r >= 0.0) and np.all(r < 1.0)
            assert np.all(np.diff(r) >= 0)
            assert np.allclose(r, (us - C[j]) / w[j], atol=4e-6 / w[j] + 1e-6)
            assert abs(r.mean() - 0.5) < 0.1


def test_fis_nearest_is_the_cell_containing_the_offset_point():
    """The FIS lookup takes the texel whose cell [k - 1/2, k + 1/2) holds
    t + d (texel centres at integers, t the fractional position)."""
    import oracle as orc
    rng = np.random.default_rng(5)
    n = 0
    for _ in range(20000):
        t = float(np.float32(rng.random()))
        d = float(np.float32(rng.uniform(-4, 4)))
        x = t + 0.5 + d
        if abs(x - round(x)) < 1e-5:
            continue                     # binary32 rounding decides exact ties
        k = orc.fis_nearest(t, d)
        assert k - 0.5 <= t + d < k + 0.5, (t, d, k)
        assert k == math.floor(x)
        n += 1
    assert n > 19000


def test_keys_picks_respect_the_sign_sets(orc):
    """Every positive draw of the positivised Keys estimator lands on a
    product weight > 0 and every negative draw on one < 0."""
    rng = np.random.default_rng(6)
    for _ in range(3000):
        tx, ty = (float(np.float32(x)) for x in rng.random(2))
        u = (np.floor(rng.random(6) * 2 ** 24) / 2 ** 24).astype(np.float32)
        off, has_neg = orc.keys_pick(tx, ty, u)
        wx = np.asarray(orc.axis_weights64(orc.KEYS3, tx))
        wy = np.asarray(orc.axis_weights64(orc.KEYS3, ty))
        assert wx[off[0] + 1] * wy[off[1] + 1] > 0
        if has_neg:
            assert wx[off[2] + 1] * wy[off[3] + 1] < 0
