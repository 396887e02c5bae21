"""Pins of the oracle's analytic backward and of the blend oracle by central
finite differences of their forward maps (FP64)."""
import numpy as np
import pytest

import oracle
from paper_2007_08501_amd import meshgen

from test_oracle_pins import sphere_batch, random_soup


def fixed_loss(verts, faces, image_size, p2f, gz, gb, gd):
    z, b, d, _ = oracle.fragments_fixed(verts, faces, image_size, p2f)
    valid = p2f >= 0
    return (np.where(valid, z, 0) * gz).sum() + (np.where(valid[..., None], b, 0) * gb).sum() + \
        (np.where(valid, d, 0) * gd).sum()


def _fd_case(v, f, fi, nf, image_size, blur, K, seed, coords=None, h=1e-7):
    o = oracle.rasterize(v, f, fi, nf, image_size, blur, K)
    p2f = o["p2f"]
    rng = np.random.default_rng(seed)
    gz = rng.standard_normal(p2f.shape)
    gb = rng.standard_normal(p2f.shape + (3,))
    gd = rng.standard_normal(p2f.shape)
    # slots whose nearest edge is (nearly) tied have a kink in dists: drop grad_dists there
    _, _, _, tie = oracle.fragments_fixed(v, f, image_size, p2f)
    gd = np.where(tie.astype(bool), 0.0, gd)
    g = oracle.backward(v, f, image_size, p2f, gz, gb, gd)
    vv = np.asarray(v, dtype=np.float64)
    if coords is None:
        coords = [(i, j) for i in range(vv.shape[0]) for j in range(3)]
    err = 0.0
    scale = np.abs(g).max()
    for (i, j) in coords:
        vp = vv.copy()
        vp[i, j] += h
        vm = vv.copy()
        vm[i, j] -= h
        fd = (fixed_loss(vp, f, image_size, p2f, gz, gb, gd) - fixed_loss(vm, f, image_size, p2f, gz, gb, gd)) / (2 * h)
        err = max(err, abs(fd - g[i, j]))
    return err, scale


def test_fd_single_triangle_all_coords():
    v = np.array([[-0.7, -0.6, 1.0], [0.8, -0.5, 2.0], [-0.4, 0.9, 3.0]])
    f = np.array([[0, 1, 2]])
    err, scale = _fd_case(v, f, [0], [1], (12, 12), 0.05, 1, seed=1)
    assert err <= 1e-6 * scale


def test_fd_soup_all_coords():
    rng = np.random.default_rng(11)
    v, f, fi, nf = random_soup(rng, n_meshes=2, faces_per=(4, 9))
    err, scale = _fd_case(v.astype(np.float64), f, fi, nf, (16, 16), 1e-2, 4, seed=2)
    assert err <= 1e-6 * scale


def test_fd_sphere_sampled_coords():
    v, f, fi, nf = sphere_batch([2, 2], seed=12)
    rng = np.random.default_rng(3)
    coords = [(int(i), int(j)) for i, j in zip(rng.integers(0, v.shape[0], 40), rng.integers(0, 3, 40))]
    err, scale = _fd_case(v.astype(np.float64), f, fi, nf, (32, 32), 2e-3, 4, seed=3, coords=coords)
    assert err <= 1e-6 * scale


def test_free_selection_fd_on_unambiguous_pixels():
    # Away from decision margins the selection is locally constant, so the
    # derivative of the full (re-selecting) forward equals the analytic one.
    v, f, fi, nf = sphere_batch([2], seed=13)
    v = v.astype(np.float64)
    H = W = 24
    o = oracle.rasterize(v, f, fi, nf, (H, W), 2e-3, 3)
    rng = np.random.default_rng(4)
    gz = rng.standard_normal(o["p2f"].shape)
    keep = (o["amb"] == 0)[..., None]
    gz = gz * keep
    g = oracle.backward(v, f, (H, W), o["p2f"], grad_zbuf=gz)
    h = 1e-8
    for i, j in [(int(a), int(b)) for a, b in zip(rng.integers(0, v.shape[0], 25), rng.integers(0, 3, 25))]:
        vals = []
        for s in (1, -1):
            vp = v.copy()
            vp[i, j] += s * h
            op = oracle.rasterize(vp, f, fi, nf, (H, W), 2e-3, 3)
            same = (op["p2f"] == o["p2f"]).all(-1, keepdims=True) | ~keep
            assert same.all()
            vals.append((np.where(op["p2f"] >= 0, op["zbuf"], 0) * gz).sum())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-5 * max(1.0, np.abs(g).max())


def test_grad_z_sum_invariant():
    # sum_v dL/dz_v = sum over valid slots of grad_zbuf, since sum_i w_i = 1 and
    # only zbuf depends on z
    v, f, fi, nf = sphere_batch([2, 3], seed=14)
    o = oracle.rasterize(v, f, fi, nf, (32, 32), 1e-3, 4)
    rng = np.random.default_rng(5)
    gz = rng.standard_normal(o["p2f"].shape)
    gb = rng.standard_normal(o["p2f"].shape + (3,))
    gd = rng.standard_normal(o["p2f"].shape)
    g = oracle.backward(v, f, (32, 32), o["p2f"], gz, gb, gd)
    assert abs(g[:, 2].sum() - gz[o["p2f"] >= 0].sum()) < 1e-9 * max(1.0, np.abs(gz).sum())
    # a constant grad_bary (c, c, c) has zero effect: sum_i w_i is constant
    gc = np.ones(o["p2f"].shape + (3,)) * 0.7
    g0 = oracle.backward(v, f, (32, 32), o["p2f"], grad_bary=gc)
    assert np.abs(g0).max() < 1e-9


# ---------------------------------------------------------------- blend oracle
SIG = 1e-4


def test_blend_special_cases():
    p2f = np.array([[[[0, -1, -1], [-1, -1, -1], [3, 4, -1]]]])
    d = np.array([[[[-2e-4, -1.0, -1.0], [-1.0, -1.0, -1.0], [1e-4, -1e-4, -1.0]]]])
    a = oracle.silhouette_blend(p2f, d, SIG)
    s = lambda x: 1.0 / (1.0 + np.exp(-x))
    assert a[0, 0, 0] == pytest.approx(s(2.0), abs=1e-15)         # K=1: the logistic itself
    assert a[0, 0, 1] == 0.0                                        # empty pixel is transparent
    p1, p2 = s(-1.0), s(1.0)
    assert a[0, 0, 2] == pytest.approx(1 - (1 - p1) * (1 - p2), abs=1e-15)


def test_blend_backward_fd():
    rng = np.random.default_rng(6)
    shp = (2, 3, 4, 6)
    p2f = np.where(rng.random(shp) < 0.8, 1, -1)
    p2f = np.where(np.cumsum(p2f < 0, -1) > 0, -1, p2f)  # valid prefix
    d = rng.normal(0.0, 2e-4, size=shp)
    ga = rng.standard_normal(shp[:3])
    g = oracle.silhouette_blend_backward(p2f, d, SIG, ga)
    h = 1e-10
    for idx in np.ndindex(*shp):
        dp = d.copy()
        dp[idx] += h
        dm = d.copy()
        dm[idx] -= h
        fd = ((oracle.silhouette_blend(p2f, dp, SIG) - oracle.silhouette_blend(p2f, dm, SIG)) * ga).sum() / (2 * h)
        assert abs(fd - g[idx]) <= 1e-5 * max(1.0, abs(g).max())


def test_iou_loss_cases():
    S = np.zeros((2, 4, 4))
    S[0, :2] = 1.0
    S[1, 1:3, 1:3] = 0.5
    assert oracle.iou_loss(S, S) == pytest.approx(np.mean([0.0, 1 - 2.0 / 6.0]))  # (.25*4)/(4*(1-.25))
    T = np.zeros_like(S)
    T[:, 2:] = 1.0
    assert oracle.iou_loss(S[:1], T[:1]) == pytest.approx(1.0)


def test_backward_pixel_list_matches_full():
    v, f, fi, nf = sphere_batch([2, 3], seed=15)
    H = W = 24
    o = oracle.rasterize(v, f, fi, nf, (H, W), 1e-3, 3)
    rng = np.random.default_rng(7)
    gz = rng.standard_normal(o["p2f"].shape)
    gb = rng.standard_normal(o["p2f"].shape + (3,))
    gd = rng.standard_normal(o["p2f"].shape)
    pix = np.sort(rng.choice(2 * H * W, 300, replace=False))
    keep = np.zeros(2 * H * W, bool)
    keep[pix] = True
    keep = keep.reshape(2, H, W, 1)
    full = oracle.backward(v, f, (H, W), np.where(keep, o["p2f"], -1), gz, gb, gd)
    flat = lambda a: a.reshape((2 * H * W,) + a.shape[3:])[pix]
    part = oracle.backward(v, f, (H, W), flat(o["p2f"]), flat(gz), flat(gb), flat(gd), pixels=pix, N=2)
    np.testing.assert_allclose(part, full, rtol=1e-12, atol=1e-12)


def test_fragments_fixed_pixel_list_matches_full():
    v, f, fi, nf = sphere_batch([2, 3], seed=16)
    H = W = 20
    o = oracle.rasterize(v, f, fi, nf, (H, W), 1e-3, 4)
    full = oracle.fragments_fixed(v, f, (H, W), o["p2f"])
    pix = np.sort(np.random.default_rng(3).choice(2 * H * W, 250, replace=False))
    rows = o["p2f"].reshape(2 * H * W, 4)[pix]
    part = oracle.fragments_fixed(v, f, (H, W), rows, pixels=pix)
    for a, b in zip(full, part):
        np.testing.assert_array_equal(a.reshape((2 * H * W,) + a.shape[3:])[pix], b)
    # the frozen-selection values are those of the free forward at the same slots
    np.testing.assert_allclose(part[0], o["zbuf"].reshape(2 * H * W, 4)[pix], rtol=0, atol=1e-12)


def _tiny_fit(seed=11):
    prob = meshgen.silhouette_fit_problem(level=1, n_views=3, seed=seed)
    return prob


def test_silfit_gradient_matches_frozen_selection_fd():
    """The fitting loss's analytic gradient (fixed selection) against central
    differences of the frozen-selection loss, every coordinate of a level-1
    template in three 24x24 views."""
    from oracle import silfit
    prob = _tiny_fit()
    H, K, blur, sigma = 24, 8, 5e-3, 2e-3
    target = silfit.target_silhouettes(prob.target, prob.rotations, prob.faces, H, K, blur, sigma)
    off = np.random.default_rng(4).standard_normal(prob.base.shape) * 0.01
    loss, g, p2f = silfit.loss_and_grad(prob.base, prob.rotations, prob.faces, off, target, H, K, blur, sigma)
    assert 0.0 < loss < 1.0
    h = 1e-6
    fd = np.zeros_like(g)
    for i in range(g.shape[0]):
        for c in range(3):
            e = np.zeros_like(off)
            e[i, c] = h
            lp = silfit.frozen_loss(prob.base, prob.rotations, prob.faces, off + e, target, H, p2f, sigma)
            lm = silfit.frozen_loss(prob.base, prob.rotations, prob.faces, off - e, target, H, p2f, sigma)
            fd[i, c] = (lp - lm) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 0
    # the analytic side sees FP32 vertices (as the rasterizer does), the FD side FP64 ones
    np.testing.assert_allclose(g, fd, rtol=0, atol=2e-4 * scale)


def test_iou_grad_fd_and_zero_loss_at_target():
    from oracle import silfit
    rng = np.random.default_rng(9)
    S = rng.uniform(0, 1, (2, 5, 6))
    T = rng.uniform(0, 1, (2, 5, 6))
    g = silfit.iou_loss_grad(S, T)
    h = 1e-7
    for idx in [(0, 1, 2), (1, 4, 5), (0, 0, 0)]:
        e = np.zeros_like(S)
        e[idx] = h
        fd = (oracle.iou_loss(S + e, T) - oracle.iou_loss(S - e, T)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(fd))
    # a binary silhouette that equals its target has IoU 1 and loss 0, and is a stationary point
    B = (rng.uniform(0, 1, (2, 5, 6)) > 0.5).astype(np.float64)
    assert oracle.iou_loss(B, B) == 0.0
