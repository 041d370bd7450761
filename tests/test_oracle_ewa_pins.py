"""Pins of the oracle's EWA filter and its stochastic form (Sec. 4.1: a MIP
level from the ellipse's extent, all EWA weights, one texel drawn from their
distribution; the EWA kernel of Greene and Heckbert) against numpy's
singular value decomposition and matrix inverse in FP64, libm, exact
enumeration of the 24-bit uniforms and closed cases."""
import math

import numpy as np
import pytest

from paper_2407_06107_amd import inputs

U24 = 2.0 ** -24


def test_weight_function(orc):
    """Truncated Gaussian e^(-2 r^2) - e^(-2): libm values inside the
    ellipse, zero on and outside it, decreasing in r^2."""
    r2 = np.concatenate([np.linspace(0.0, 0.999, 1001), [1.0 - 2 ** -24]]).astype(np.float32)
    w = np.array([orc.ewa_gauss(float(x)) for x in r2])
    ref = np.exp(-2.0 * r2.astype(np.float64)) - math.exp(-2.0)
    assert np.all(np.abs(w - ref) <= 2.0 ** -22)
    assert np.all(np.diff(w) <= 0) and w[0] > 0.86
    for x in (1.0, 1.5, 100.0, float("inf")):
        assert orc.ewa_gauss(x) == 0.0


def _jacobian(q, w, h):
    """Footprint Jacobian in level-0 texels: columns d(s,t)/dx, d(s,t)/dy."""
    q = np.asarray(q, np.float64)
    return np.array([[w * q[2], w * q[4]], [h * q[3], h * q[5]]])


def _random_queries(rng, n, spread=2.0):
    ang = rng.uniform(0, 2 * np.pi, size=(n, 2))
    mag = 10.0 ** rng.uniform(-1.5, spread, size=(n, 2)) / 64
    q = np.zeros((n, 6), np.float32)
    q[:, 0], q[:, 1] = rng.random(n), rng.random(n)
    q[:, 2], q[:, 3] = mag[:, 0] * np.cos(ang[:, 0]), mag[:, 0] * np.sin(ang[:, 0])
    q[:, 4], q[:, 5] = mag[:, 1] * np.cos(ang[:, 1]), mag[:, 1] * np.sin(ang[:, 1])
    return q


@pytest.mark.parametrize("wh", [(64, 64), (256, 32)])
def test_frame_is_the_jacobian_covariance(orc, wh):
    """Within the anisotropy limit the frame is S = J J^T (numpy, FP64) and
    the level of detail is log2 of J's smaller singular value, clamped at 0;
    beyond it the clamped S keeps J J^T's eigenvectors and its larger
    eigenvalue, and its smaller eigenvalue becomes (s1 / amax)^2, with
    lod = log2(s1 / amax)."""
    w, h = wh
    rng = np.random.default_rng(7)
    q = _random_queries(rng, 400)
    for amax in (1, 4, 16, 64):
        for qq in q:
            lod, sss, stt, sst, det = orc.ewa_frame(qq, w, h, amax).astype(np.float64)
            J = _jacobian(qq, w, h)
            S = J @ J.T
            lam, vec = np.linalg.eigh(S)
            s1, s2 = np.sqrt(lam[1]), np.sqrt(max(lam[0], 0.0))
            Sc = np.array([[sss, sst], [sst, stt]])
            scale = lam[1]
            if s2 * amax >= s1 * (1 + 1e-5):
                assert np.allclose(Sc, S, rtol=0, atol=2e-6 * scale)
                assert abs(det - lam[0] * lam[1]) <= 2e-5 * lam[1] ** 2
                minor = s2
            elif s2 * amax <= s1 * (1 - 1e-5):
                minor = s1 / amax
                target = vec @ np.diag([minor ** 2, lam[1]]) @ vec.T
                assert np.allclose(Sc, target, rtol=0, atol=2e-6 * scale), (amax, Sc, target)
                assert abs(det - lam[1] * minor ** 2) <= 2e-5 * lam[1] ** 2
            else:
                continue   # on the limit: either branch
            ref = max(0.0, math.log2(minor)) if minor > 0 else 0.0
            assert abs(lod - ref) <= 3e-6 * max(1.0, ref), (lod, ref)


def _pyr(N=64):
    tex = inputs.texture_uniform(N, seed=12)
    lv = inputs.mip_chain(tex)
    buf, offs = inputs.pack_levels(lv)
    return lv, buf, offs


QUERIES = [
    [0.3, 0.6, 3.0 / 64, 1.0 / 64, -0.5 / 64, 1.5 / 64],     # tilted ellipse, ratio ~2
    [0.71, 0.22, 6.0 / 64, 0.0, 0.0, 1.0 / 64],              # axis-aligned, ratio 6
    [0.5, 0.5, 0.5 / 64, 0.5 / 64, -0.5 / 64, 0.5 / 64],     # small, rotated 45 degrees
    [0.12, 0.93, 20.0 / 64, 3.0 / 64, -0.2 / 64, 1.2 / 64],  # beyond the anisotropy limit 8
    [0.45, 0.35, 2.0 / 64, 2.0 / 64, 2.1 / 64, 1.9 / 64],    # nearly parallel derivatives
]


def _levels(orc, q, L=7, w=64, h=64, amax=8):
    lod = orc.ewa_lod(q, w, h, amax)
    fl = int(math.floor(lod))
    return sorted({min(fl, L - 1), min(fl + 1, L - 1)})


@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_weights_are_the_gaussian_of_the_inverse_covariance(orc, qi):
    """At a level, the oracle's normalised weights equal the truncated
    Gaussian of r^2 = d^T (S_l + I)^-1 d computed by numpy in FP64 from the
    frame scaled to the level (S_l = D S D, D = diag(W_l / W, H_l / H)),
    and every cell of positive FP64 weight lies in the oracle's box."""
    q = np.array(QUERIES[qi], np.float32)
    lod, sss, stt, sst, _ = orc.ewa_frame(q, 64, 64, 8).astype(np.float64)
    for level in _levels(orc, q):
        n = 64 >> level
        Dl = np.diag([n / 64, n / 64])
        V = Dl @ np.array([[sss, sst], [sst, stt]]) @ Dl + np.eye(2)
        Vi = np.linalg.inv(V)
        s, t = float(q[0]) * n - 0.5, float(q[1]) * n - 0.5
        s0, s1, t0, t1 = orc.ewa_box(64, 64, 7, q, level)
        R = 40
        ref = np.zeros((2 * R + 1, 2 * R + 1))
        for j, it in enumerate(range(int(t) - R, int(t) + R + 1)):
            for i, is_ in enumerate(range(int(s) - R, int(s) + R + 1)):
                d = np.array([is_ - s, it - t])
                r2 = d @ Vi @ d
                ref[j, i] = math.exp(-2 * r2) - math.exp(-2) if r2 < 1 else 0.0
        jj, ii = np.nonzero(ref > 1e-6)
        assert (ii + int(s) - R).min() >= s0 and (ii + int(s) - R).max() <= s1
        assert (jj + int(t) - R).min() >= t0 and (jj + int(t) - R).max() <= t1
        P = orc.ewa_weights(64, 64, 7, q, level)
        P = P.reshape(t1 - t0 + 1, s1 - s0 + 1)
        sub = ref[t0 - (int(t) - R):t1 - (int(t) - R) + 1, s0 - (int(s) - R):s1 - (int(s) - R) + 1]
        sub = sub / sub.sum()
        assert np.max(np.abs(P - sub)) <= 2e-5 * sub.max(), np.max(np.abs(P - sub))


@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_pick_pmf_by_enumeration(orc, qi):
    """The inverse-CDF pick (Sec. 2.2, sampling arrays) takes cell i with
    probability w_i / sum w: all 2^24 uniforms run through it, and each
    probability is within (n + 4) 2^-24 of the normalised weight (a
    threshold u W and a running sum each round once, and the FP64 weight
    total differs from the binary32 one by at most n ulp)."""
    q = np.array(QUERIES[qi], np.float32)
    for level in _levels(orc, q):
        P, box = orc.ewa_pick_pmf(64, 64, 7, q, level)
        W = orc.ewa_weights(64, 64, 7, q, level).reshape(P.shape)
        n = int((W > 0).sum())
        assert abs(P.sum() - 1.0) < 1e-12
        assert np.all(P[W == 0] == 0)
        assert np.max(np.abs(P - W)) <= (n + 4) * U24, (level, n, np.max(np.abs(P - W)) / U24)


def test_four_equal_weights_exact(orc):
    """A zero footprint centred between four texel centres: V = I, each of
    the four cells at r^2 = 1/2 has the same weight and is picked with
    probability 1/4 up to two lattice points."""
    q = np.array([32.0 / 64, 17.0 / 64, 0.0, 0.0, 0.0, 0.0], np.float32)
    P, box = orc.ewa_pick_pmf(64, 64, 7, q, 0)
    W = orc.ewa_weights(64, 64, 7, q, 0).reshape(P.shape)
    pos = W > 0
    assert pos.sum() == 4 and np.allclose(W[pos], 0.25, rtol=0, atol=1e-7)
    assert np.all(np.abs(P[pos] - W[pos]) <= 2 * U24)


def test_zero_footprint_reads_the_centre_texel(orc):
    """Zero derivatives: the ellipse is the unit disk in level-0 texels, so a
    query at a texel centre has one positive weight — the texel itself."""
    lv, buf, offs = _pyr()
    ot = orc.Tex2D(buf, 64, 64, len(lv), orc.RGBA32F, offs, orc.REPEAT, orc.MIP_LINEAR)
    iy, ix = np.meshgrid(np.arange(0, 64, 7), np.arange(0, 64, 5), indexing="ij")
    q = np.zeros((ix.size, 6), np.float32)
    q[:, 0] = (ix.ravel() + 0.5) / 64
    q[:, 1] = (iy.ravel() + 0.5) / 64
    for m in (orc.BEFORE, orc.AFTER):
        out = orc.filter2d_aniso(ot, q, orc.EWA, m, amax=8)
        assert np.allclose(out, lv[0][iy.ravel(), ix.ravel()], rtol=0, atol=1e-12)
    S, taps = orc.filter2d_aniso(ot, q, orc.EWA, orc.STOCHASTIC, spp=8, seed=2, amax=8, taps=True)
    assert np.all(taps[..., 0] == 0) and np.all(taps[..., 1] == ix.ravel()[:, None])


def test_after_is_the_level_blend_of_normalised_weights(orc):
    """The deterministic EWA after shading is the definition written out:
    (1-f) times the weight-normalised sum of shaded texels on level
    floor(lod) plus f times that on the next level; and the stochastic
    estimator's exact expectation (enumerated pick probabilities, 24-bit
    level probability) is within the pick's rounding of it."""
    lv, buf, offs = _pyr()
    ot = orc.Tex2D(buf, 64, 64, len(lv), orc.RGBA32F, offs, orc.REPEAT, orc.MIP_LINEAR)
    g = orc.ggx_params()
    for qv in QUERIES[:3] + QUERIES[4:]:
        q = np.array(qv, np.float32)
        A = orc.filter2d_aniso(ot, q[None], orc.EWA, orc.AFTER, shade=1, amax=8)[0]
        lc = np.float32(min(orc.ewa_lod(q, 64, 64), 6.0))
        fl = int(math.floor(lc))
        f = float(np.float32(lc - np.float32(fl)))
        c = math.ceil(float(np.float32(1.0) - np.float32(f)) * 2 ** 24)
        p1 = (2 ** 24 - c) / 2 ** 24                   # P(u24 >= 1 - f)
        D = np.zeros(3)
        E = np.zeros(3)
        drift = 0.0
        for level, pd, pe in ((fl, 1 - f, 1 - p1), (min(fl + 1, 6), f, p1)):
            P, (s0, s1, t0, t1) = orc.ewa_pick_pmf(64, 64, 7, q, level)
            W = orc.ewa_weights(64, 64, 7, q, level).reshape(P.shape)
            n = 64 >> level
            vals = np.zeros(P.shape + (3,))
            for yy in range(t0, t1 + 1):
                for xx in range(s0, s1 + 1):
                    vals[yy - t0, xx - s0] = orc.shade_ggx(g, lv[level][yy % n, xx % n].astype(np.float64))
            D += pd * np.einsum("ij,ijc->c", W, vals)
            E += pe * np.einsum("ij,ijc->c", P, vals)
            drift += pe * np.abs(P - W).sum() * np.abs(vals).max()
        assert np.max(np.abs(D - A)) <= 1e-12 * max(1.0, np.abs(A).max()), (D, A)
        assert np.max(np.abs(E - A)) <= drift + abs(p1 - f) * 2 * np.abs(A).max() + 1e-12


def test_lod_uses_the_minor_axis(orc):
    """For orthogonal derivative vectors the singular values are their
    lengths, so the EWA level equals the anisotropic filter's level of
    detail: log2 of the shorter axis in level-0 texels after the anisotropy
    limit, clamped at 0; a degenerate (line) footprint takes longer/amax."""
    for k in (0, 1, 3):
        q = np.array([0.4, 0.4, 2.0 ** k * 4 / 64, 0.0, 0.0, 2.0 ** k / 64], np.float32)
        assert orc.ewa_lod(q, 64, 64) == k
        q = np.array([0.4, 0.4, 0.0, 2.0 ** k / 64, -(2.0 ** k) * 4 / 64, 0.0], np.float32)   # axes swapped
        assert orc.ewa_lod(q, 64, 64) == k
        q = np.array([0.4, 0.4, 2.0 ** k / 256, 0.0, 0.0, 2.0 ** k * 2 / 32], np.float32)   # 256 x 32 texels
        assert orc.ewa_lod(q, 256, 32) == k
    q = np.array([0.4, 0.4, 32.0 / 64, 0.0, 0.0, 1.0 / 64], np.float32)
    assert orc.ewa_lod(q, 64, 64, amax=8) == 2.0 and orc.ewa_lod(q, 64, 64, amax=64) == 0.0
    assert orc.ewa_lod(np.array([0.4, 0.4, 32.0 / 64, 0, 0, 0], np.float32), 64, 64, amax=8) == 2.0
    assert orc.ewa_lod(np.zeros(6, np.float32), 64, 64) == 0.0
    assert orc.ewa_lod(np.array([0.4, 0.4, 0.1 / 64, 0, 0, 0.2 / 64], np.float32), 64, 64) == 0.0
    for qv in ([0.3, 0.6, 3.0 / 64, 1.0 / 64, -1.0 / 64, 3.0 / 64], [0.71, 0.22, 6.0 / 64, 0.0, 0.0, 1.0 / 64]):
        q = np.array(qv, np.float32)
        lam, _, _ = orc.aniso_lod(64, 64, q[2:], 8)
        assert abs(orc.ewa_lod(q, 64, 64) - max(lam, 0.0)) <= 2e-6


@pytest.mark.parametrize("wh", [(64, 64), (256, 32), (16, 128), (8, 1), (2048, 2048)])
@pytest.mark.parametrize("amax", [1, 4, 16])
def test_bounding_box_is_bounded(orc, wh, amax):
    """On a complete pyramid, at the levels a sample can read, the ellipse's
    box has at most (4 r_x amax + 3) x (4 r_y amax + 3) cells,
    r_x = max(W, H)/W, r_y = max(W, H)/H: the box's half-width along s is
    sqrt(V_ss) <= sqrt(s1^2 + 1), the major axis s1 is at most amax times
    the minor, and the minor is below 2 texels at level floor(lod) (one
    axis of a non-square texture stops shrinking at 1 texel, r times
    longer).  Footprints of 1e-7 to 1e34 uv units, nearly parallel and
    degenerate derivatives included."""
    w, h = wh
    L = int(math.floor(math.log2(max(w, h)))) + 1
    rx, ry = max(w, h) / w, max(w, h) / h
    bx, by = 4 * rx * amax + 3, 4 * ry * amax + 3
    rng = np.random.default_rng(amax * 7 + w)
    for _ in range(3000):
        mag = 10.0 ** rng.uniform(-7, 3 if rng.random() < 0.8 else 34, size=2)
        ang = rng.uniform(0, 2 * np.pi, size=2)
        if rng.random() < 0.3:
            ang[1] = ang[0] + rng.normal(0, 0.01)          # nearly parallel axes
        q = np.array([rng.random(), rng.random(), mag[0] * np.cos(ang[0]), mag[0] * np.sin(ang[0]),
                      mag[1] * np.cos(ang[1]), mag[1] * np.sin(ang[1])], np.float32)
        if rng.random() < 0.1:
            q[4:6] = 0
        lod = orc.ewa_lod(q, w, h, amax)
        if lod > L - 1:
            continue
        fl = int(math.floor(lod))
        for l in {fl, min(fl + 1, L - 1)}:
            s0, s1, t0, t1 = orc.ewa_box(w, h, L, q, l, amax)
            assert 1 <= s1 - s0 + 1 <= bx and 1 <= t1 - t0 + 1 <= by, (q, l, (s0, s1, t0, t1))


def test_huge_footprints_read_the_last_level(orc):
    """Footprints whose squares would overflow binary32 are beyond every
    level: the frame reports an infinite level of detail."""
    for m in (1e12, 1e30, 3e38):
        q = np.array([0.3, 0.3, m, 0.0, 0.0, m], np.float32)
        assert orc.ewa_lod(q, 64, 64) == math.inf


def test_stochastic_mean_within_five_sigma(orc):
    lv, buf, offs = _pyr()
    ot = orc.Tex2D(buf, 64, 64, len(lv), orc.RGBA32F, offs, orc.REPEAT, orc.MIP_LINEAR)
    q = inputs.plane_queries_aniso(40, 30)
    q = q[::20]
    A = orc.filter2d_aniso(ot, q, orc.EWA, orc.AFTER, shade=1, amax=8)
    spp = 4096
    S = orc.filter2d_aniso(ot, q, orc.EWA, orc.STOCHASTIC, spp=spp, seed=5, shade=1, amax=8)
    assert np.all(np.abs(S - A) <= 5 * 1.0 / math.sqrt(spp))


def test_footprint_wider_than_the_texture(orc):
    lv, buf, offs = _pyr()
    ot = orc.Tex2D(buf, 64, 64, len(lv), orc.RGBA32F, offs, orc.REPEAT, orc.MIP_LINEAR)
    q = np.array([[0.3, 0.3, 3.0, 0.0, 0.0, 2.0]], np.float32)       # 128+ texels per pixel on a 64^2 texture
    for m in (orc.AFTER, orc.BEFORE):
        assert np.allclose(orc.filter2d_aniso(ot, q, orc.EWA, m, amax=8), lv[-1][0, 0], atol=1e-12)
    _, taps = orc.filter2d_aniso(ot, q, orc.EWA, orc.STOCHASTIC, spp=3, amax=8, taps=True)
    assert np.all(taps[0] == [len(lv) - 1, 0, 0])
