"""Pins of the FP64 softmax-blend oracle (paper, Section 3.2, Algorithm 2):
limits with closed forms, invariances, and finite differences."""
import numpy as np
import pytest
from scipy.special import softmax as sp_softmax

import oracle


def frags(seed, N=2, H=3, W=4, K=5, C=3, empty_frac=0.3):
    rng = np.random.default_rng(seed)
    p2f = rng.integers(0, 100, (N, H, W, K))
    p2f[rng.uniform(size=p2f.shape) < empty_frac] = -1
    zbuf = rng.uniform(1.0, 3.0, p2f.shape)
    dists = rng.uniform(-2e-3, 1e-3, p2f.shape)
    colors = rng.uniform(0, 1, p2f.shape + (C,))
    return p2f, zbuf, dists, colors


ARGS = dict(sigma=1e-3, gamma=0.1, znear=1.0, zfar=100.0)


def test_single_face_gives_its_color():
    p2f, z, d, c = frags(1, K=4, empty_frac=0.0)
    p2f[..., 1:] = -1
    img = oracle.softmax_blend(p2f, z, d, c, **ARGS)
    np.testing.assert_allclose(img, c[..., 0, :], rtol=1e-15, atol=0)


def test_empty_pixels_are_zero_and_empty_slots_ignored():
    p2f, z, d, c = frags(2)
    p2f[0, 0, 0] = -1
    img = oracle.softmax_blend(p2f, z, d, c, **ARGS)
    assert (img[0, 0, 0] == 0).all()
    # garbage in empty slots changes nothing
    z2, d2, c2 = z.copy(), d.copy(), c.copy()
    e = p2f < 0
    z2[e], d2[e] = -7.0, 123.0
    c2[e] = 9.0
    np.testing.assert_array_equal(oracle.softmax_blend(p2f, z2, d2, c2, **ARGS), img)


def test_invariances():
    p2f, z, d, c = frags(3)
    img = oracle.softmax_blend(p2f, z, d, c, **ARGS)
    # a common depth shift of a pixel's faces cancels in the normalised weights
    np.testing.assert_allclose(oracle.softmax_blend(p2f, z + 0.37, d, c, **ARGS), img, rtol=1e-12, atol=1e-14)
    # the slot order does not matter
    perm = np.random.default_rng(0).permutation(p2f.shape[-1])
    np.testing.assert_allclose(oracle.softmax_blend(p2f[..., perm], z[..., perm], d[..., perm], c[..., perm, :],
                                                    **ARGS), img, rtol=1e-12, atol=1e-14)
    # a convex combination of the face colors
    valid = p2f >= 0
    lo = np.where(valid[..., None], c, np.inf).min(-2)
    hi = np.where(valid[..., None], c, -np.inf).max(-2)
    has = valid.any(-1)
    assert ((img[has] >= lo[has] - 1e-12) & (img[has] <= hi[has] + 1e-12)).all()


def test_limits():
    p2f, z, d, c = frags(4, empty_frac=0.0)
    # gamma -> 0: the face nearest the camera (largest zinv = smallest z) wins
    img = oracle.softmax_blend(p2f, z, d, c, sigma=1e-3, gamma=1e-9, znear=1.0, zfar=100.0)
    near = np.argmin(z, axis=-1)
    np.testing.assert_allclose(img, np.take_along_axis(c, near[..., None, None], -2)[..., 0, :], atol=1e-12)
    # sigma -> 0 with every pixel inside its faces: weights are a softmax of zinv / gamma
    din = -np.abs(d) - 1e-3
    gamma = 0.05
    img = oracle.softmax_blend(p2f, z, din, c, sigma=1e-9, gamma=gamma, znear=1.0, zfar=100.0)
    w = sp_softmax((100.0 - z) / 99.0 / gamma, axis=-1)
    np.testing.assert_allclose(img, (w[..., None] * c).sum(-2), rtol=1e-12, atol=1e-14)
    # gamma -> infinity: weights proportional to the sigmoid probabilities
    img = oracle.softmax_blend(p2f, z, d, c, sigma=1e-3, gamma=1e12, znear=1.0, zfar=100.0)
    pr = 1.0 / (1.0 + np.exp(d / 1e-3))
    np.testing.assert_allclose(img, (pr[..., None] * c).sum(-2) / pr.sum(-1)[..., None], rtol=1e-9)


@pytest.mark.parametrize("which", ["zbuf", "dists", "colors"])
def test_backward_fd(which):
    p2f, z, d, c = frags(5)
    g = np.random.default_rng(6).standard_normal(p2f.shape[:-1] + (c.shape[-1],))
    gz, gd, gc = oracle.softmax_blend_backward(p2f, z, d, c, **ARGS, grad_image=g)
    x, ana = dict(zbuf=(z, gz), dists=(d, gd), colors=(c, gc))[which]
    h = dict(zbuf=1e-6, dists=1e-9, colors=1e-6)[which]
    rng = np.random.default_rng(7)
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        args = dict(zbuf=z, dists=d, colors=c)
        args[which] = xp
        fp = (oracle.softmax_blend(p2f, args["zbuf"], args["dists"], args["colors"], **ARGS) * g).sum()
        args[which] = xm
        fm = (oracle.softmax_blend(p2f, args["zbuf"], args["dists"], args["colors"], **ARGS) * g).sum()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - ana[idx]) <= 1e-6 * max(1.0, abs(fd)), (which, idx, fd, ana[idx])
    if which != "colors":
        assert (ana[p2f < 0] == 0).all()
