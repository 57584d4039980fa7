"""Pins of the oracle's sample specification (Sec. 3.2 Eq. ao-direction-pdf,
Sec. 3.3 Eq. shadow-light-pdf): distributions and moments fixed by the
mathematics, not by re-typing the sampler."""
import numpy as np
import pytest

import oracle
import workloads as w


def _grid_gbuffer(n, normal, origin=(3.0, 1.0, -2.0)):
    gb = w.plane_gbuffer(n, n, 0.01, origin=origin, prim=7)
    gb.nrm[:] = np.asarray(normal, np.float32)
    return gb


def test_pcg4d_uniform_and_decorrelated():
    # 2^16 consecutive counters; each output's top 24 bits must look uniform
    # (chi-square over 64 bins) and the four outputs must be uncorrelated.
    n = 1 << 16
    out = np.array([oracle.pcg4d(i & 255, i >> 8, 3, 12345) for i in range(n)], dtype=np.uint64)
    u = (out >> 8).astype(np.float64) / (1 << 24)
    for c in range(4):
        hist = np.bincount((u[:, c] * 64).astype(int), minlength=64)
        chi2 = ((hist - n / 64) ** 2 / (n / 64)).sum()
        assert chi2 < 120, chi2  # 63 dof; p ~ 1e-5
    cc = np.corrcoef(u.T)
    assert np.abs(cc - np.eye(4)).max() < 0.02
    # different seeds give different streams
    a = oracle.pcg4d(1, 2, 3, 4)
    b = oracle.pcg4d(1, 2, 3, 5)
    assert not np.array_equal(a, b)


# pcg4d as Jarzynski and Olano (JCGT 2020) define it, evaluated here in numpy
# uint32 arithmetic (wrapping products and sums): a multiply-add step per
# word, a round of cross products v0 += v1 v3, v1 += v2 v0, v2 += v0 v1,
# v3 += v1 v2, an xor with each word's upper half, and the cross products
# again.
_M, _C = np.uint32(1664525), np.uint32(1013904223)


def _np_pcg4d(v):
    v = np.array(v, dtype=np.uint32, copy=True)
    with np.errstate(over="ignore"):
        v = v * _M + _C

        def cross(v):
            v[0] += v[1] * v[3]
            v[1] += v[2] * v[0]
            v[2] += v[0] * v[1]
            v[3] += v[1] * v[2]

        cross(v)
        v ^= v >> np.uint32(16)
        cross(v)
    return v


def _np_pcg4d_inverse(v):
    # each step of the hash is invertible: the cross products are undone in
    # reverse order, the half-word xor is its own inverse, and the
    # multiply-add is undone with the inverse of the odd multiplier mod 2^32
    v = np.array(v, dtype=np.uint32, copy=True)
    minv = np.uint32(pow(1664525, -1, 1 << 32))
    with np.errstate(over="ignore"):

        def uncross(v):
            v[3] -= v[1] * v[2]
            v[2] -= v[0] * v[1]
            v[1] -= v[2] * v[0]
            v[0] -= v[1] * v[3]

        uncross(v)
        v ^= v >> np.uint32(16)
        uncross(v)
        v = (v - _C) * minv
    return v


def test_pcg4d_known_answers():
    # known-answer vectors: the oracle's hash against the independent numpy
    # evaluation of the published definition, on edge and random counters
    rng = np.random.default_rng(20)
    ins = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 0, 0, 1), (0xFFFFFFFF,) * 4, (1919, 1079, 0, 0x9E3779B9),
           (12, 34, 56, 78)]
    ins += [tuple(int(x) for x in row) for row in rng.integers(0, 1 << 32, (500, 4), dtype=np.uint64)]
    ref = _np_pcg4d(np.array(ins, dtype=np.uint64).astype(np.uint32).T)
    got = np.array([oracle.pcg4d(*v) for v in ins], dtype=np.uint32).T
    assert np.array_equal(got, ref)
    # and the hash is a bijection of (Z / 2^32)^4: the numpy inverse undoes it
    back = _np_pcg4d_inverse(got)
    assert np.array_equal(back, np.array(ins, dtype=np.uint64).astype(np.uint32).T)


def test_pcg4d_avalanche():
    # flipping one low input bit (the pixel, sample and seed counters live
    # there) flips each output bit with probability ~1/2.  (Flips of the top
    # input bits diffuse less -- a product moves a change in bit b only to
    # bits >= b until the half-word xor -- so they are not asserted.)
    rng = np.random.default_rng(21)
    base = rng.integers(0, 1 << 32, (4, 256), dtype=np.uint64).astype(np.uint32)
    h0 = np.array([oracle.pcg4d(*base[:, i]) for i in range(base.shape[1])], dtype=np.uint32)
    rates = []
    for word in range(4):
        for bit in (0, 4, 8, 12, 16):
            b = base.copy()
            b[word] ^= np.uint32(1 << bit)
            h1 = np.array([oracle.pcg4d(*b[:, i]) for i in range(b.shape[1])], dtype=np.uint32)
            flips = np.unpackbits((h0 ^ h1).view(np.uint8)).mean()
            rates.append(flips)
    assert 0.45 < min(rates) and max(rates) < 0.55, rates


@pytest.mark.parametrize("normal", [(0.0, 1.0, 0.0), (0.0, 0.0, -1.0), (0.0, 0.0, 1.0),
                                    (0.48, -0.6, 0.64), (-0.8, 0.0, -0.6)])
def test_cosine_hemisphere_moments(normal):
    n = np.asarray(normal, np.float64)
    gb = _grid_gbuffer(256, normal)
    p = oracle.params("ao", "none", seed=99, sample=5)
    o, d, kind = oracle.samples(gb, p)
    assert (kind == 0).all()
    d = d.reshape(-1, 3).astype(np.float64)
    N = d.shape[0]
    # unit length to FP32 rounding
    assert np.abs(np.linalg.norm(d, axis=1) - 1.0).max() < 1e-6
    c = d @ n
    assert c.min() >= 0.0
    # cosine-weighted hemisphere: cos(theta) = sqrt(1 - r^2) with r^2 ~ U[0,1],
    # so E[cos] = 2/3, E[cos^2] = 1/2, Var[cos] = 1/18
    assert abs(c.mean() - 2 / 3) < 4 * np.sqrt(1 / 18 / N)
    assert abs((c ** 2).mean() - 0.5) < 4 * np.sqrt(1 / 12 / N)
    # tangential components have zero mean and E[(w.t)^2] = 1/4 for any unit t perpendicular to n
    t = np.cross(n, [0.3, 0.7, 0.2])
    t /= np.linalg.norm(t)
    b = np.cross(n, t)
    for e in (t, b):
        x = d @ e
        assert abs(x.mean()) < 4 * np.sqrt(0.25 / N)
        assert abs((x ** 2).mean() - 0.25) < 4 * np.sqrt(0.05 / N)
    # CDF of cos^2 = 1 - r^2 is uniform: Kolmogorov-Smirnov
    q = np.sort(c ** 2)
    ks = np.abs(q - (np.arange(N) + 0.5) / N).max()
    assert ks < 1.95 / np.sqrt(N)


def test_receiver_offset_spec():
    gb = _grid_gbuffer(16, (0.0, 1.0, 0.0), origin=(-40.0, 2.5, 7.0))
    p = oracle.params("ao", "none")
    o, d, kind = oracle.samples(gb, p)
    x = gb.pos.astype(np.float64)
    eps = (1.0 + np.abs(x).max(axis=-1)) * 2.0 ** -16
    off = o.astype(np.float64) - x
    # o_y = x_y + eps rounded once to FP32: within half an ulp of o_y
    ulp = np.spacing(np.abs(o[..., 1])).astype(np.float64)
    assert (np.abs(off[..., 1] - eps) <= 0.5 * ulp + 1e-12).all()
    assert np.abs(off[..., [0, 2]]).max() == 0.0


def test_light_points_uniform_on_rectangle():
    light = w.RectLight(np.array([0.5, 10.0, -1.0], np.float32), np.array([2.0, 0.0, 0.0], np.float32),
                        np.array([0.0, 0.0, 0.5], np.float32))
    gb = _grid_gbuffer(200, (0.0, 1.0, 0.0), origin=(0.0, 0.0, 0.0))
    p = oracle.params("shadow", "none", light=light, seed=4)
    o, d, kind = oracle.samples(gb, p)
    assert (kind == 0).all()
    y = (o.astype(np.float64) + d.astype(np.float64)).reshape(-1, 3)
    N = y.shape[0]
    a = (y[:, 0] - 0.5) / 2.0
    b = (y[:, 2] + 1.0) / 0.5
    assert np.abs(y[:, 1] - 10.0).max() < 1e-5
    assert np.abs(a).max() <= 0.5 + 1e-6 and np.abs(b).max() <= 0.5 + 1e-6
    # mean at the centre, per-axis variance |e|^2 / 12
    assert abs(y[:, 0].mean() - 0.5) < 4 * np.sqrt(4 / 12 / N)
    assert abs(y[:, 2].mean() + 1.0) < 4 * np.sqrt(0.25 / 12 / N)
    assert abs(y[:, 0].var() - 4 / 12) < 0.02 * 4 / 12
    assert abs(y[:, 2].var() - 0.25 / 12) < 0.02 * 0.25 / 12


def test_light_sampler_reproduces_rectangle_form_factor():
    # E_y[Area cos_x cos_y / (pi d^2)] over uniform light points equals the
    # point-to-rectangle form factor (Lambert's polygon formula).
    import scenes
    light = w.RectLight(np.array([0.0, 1.5, 0.0], np.float32), np.array([1.0, 0.0, 0.0], np.float32),
                        np.array([0.0, 0.0, 1.0], np.float32))
    gb = _grid_gbuffer(256, (0.0, 1.0, 0.0), origin=(0.0, 0.0, 0.0))
    gb.pos[:] = 0.0  # one receiver at the origin, 65536 independent counters
    p = oracle.params("shadow", "none", light=light, seed=11)
    o, d, kind = oracle.samples(gb, p)
    v = d.reshape(-1, 3).astype(np.float64)
    dist2 = (v ** 2).sum(1)
    dd = np.sqrt(dist2)
    cos_x = v[:, 1] / dd
    cos_y = v[:, 1] / dd  # light faces down, n_y = (0,-1,0)
    est = 1.0 * cos_x * cos_y / (np.pi * dist2)
    corners = [(-0.5, 1.5, -0.5), (0.5, 1.5, -0.5), (0.5, 1.5, 0.5), (-0.5, 1.5, 0.5)]
    ff = scenes.lambert_polygon_ff((0, 0, 0), (0, 1, 0), corners)
    assert abs(est.mean() - ff) < 4 * est.std() / np.sqrt(est.size)


def test_shadow_samples_self_blocked_and_unlit():
    light = w.terrain_light()
    # receiver facing straight down: every light point is behind its tangent plane
    gb = _grid_gbuffer(8, (0.0, -1.0, 0.0), origin=(0.0, 0.0, 12.0))
    p = oracle.params("shadow", "none", light=light)
    _, _, kind = oracle.samples(gb, p)
    assert (kind == 1).all()
    # receiver above the light (behind its emitting face), facing up
    gb = _grid_gbuffer(8, (0.0, 1.0, 0.0), origin=(0.0, 20.0, 12.0))
    _, _, kind = oracle.samples(gb, p)
    assert (kind == 1).all()
    # background pixels are never sampled
    gb = _grid_gbuffer(8, (0.0, 1.0, 0.0))
    gb.prim[:] = 0xFFFFFFFF
    _, _, kind = oracle.samples(gb, p)
    assert (kind == 2).all()
