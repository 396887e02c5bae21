"""Pins of the FP64 point-cloud oracle (paper, Section 3.3): hand-computed
cases, exact symmetries, invariants, finite differences for the backward,
and closed forms and finite differences for Alpha and Norm compositing."""
import numpy as np
import pytest

import oracle
from paper_2007_08501_amd import meshgen


def cloud(pts):
    pts = np.asarray(pts, np.float64)
    return pts, np.array([0]), np.array([pts.shape[0]])


def test_single_point_hand_case():
    # 8x8 image: pixel pitch 0.25 in NDC; pixel (r, c) centre (1 - (2c+1)/8, 1 - (2r+1)/8)
    x, y = 1 - 7 / 8, 1 - 5 / 8                   # centre of pixel (2, 3)
    p, fi, n = cloud([[x, y, 2.5]])
    o = oracle.rasterize_points(p, fi, n, (8, 8), 0.3, 2)
    cov = o["idx"][0, :, :, 0] >= 0
    # covered: the pixel itself and its four edge neighbours (distance 0.25 < 0.3), not the diagonals (0.354)
    expect = np.zeros((8, 8), bool)
    for r, c in [(2, 3), (1, 3), (3, 3), (2, 2), (2, 4)]:
        expect[r, c] = True
    np.testing.assert_array_equal(cov, expect)
    assert o["dists"][0, 2, 3, 0] == 0.0 and o["dists"][0, 2, 4, 0] == 0.0625
    assert o["zbuf"][0, 2, 3, 0] == 2.5 and o["idx"][0, 2, 3, 1] == -1 and o["zbuf"][0, 2, 3, 1] == -1
    # radius exactly the neighbour distance: strict test drops them and flags the pixel
    o = oracle.rasterize_points(p, fi, n, (8, 8), 0.25, 1)
    assert (o["idx"][0, :, :, 0] >= 0).sum() == 1
    assert o["amb"][0, 2, 4] & 1


def test_depth_order_ties_and_behind_camera():
    x, y = 1 - 7 / 8, 1 - 5 / 8
    p, fi, n = cloud([[x, y, 3.0], [x, y, 1.0], [x, y, 1.0], [x, y, -0.5], [x, y, 0.0]])
    o = oracle.rasterize_points(p, fi, n, (8, 8), 0.1, 5)
    assert list(o["idx"][0, 2, 3]) == [4, 1, 2, 0, -1]   # z = 0 counts, z < 0 does not; equal z by index
    assert o["amb"][0, 2, 3] & 2 and o["amb"][0, 2, 3] & 4
    o1 = oracle.rasterize_points(p, fi, n, (8, 8), 0.1, 1)
    assert o1["idx"][0, 2, 3, 0] == 4


def test_exact_symmetries():
    rng = np.random.default_rng(3)
    # dyadic coordinates so that shifting by a whole pixel is exact
    pts = np.round(rng.uniform(-0.8, 0.8, (60, 3)) * 64) / 64
    pts[:, 2] = np.abs(pts[:, 2]) + 1.0
    p, fi, n = cloud(pts)
    o = oracle.rasterize_points(p, fi, n, (16, 16), 0.15, 4)
    # one pixel is 2/16 in NDC; +x is to the left, so x + 1/8 moves everything one column left
    q = p.copy()
    q[:, 0] += 0.125
    o2 = oracle.rasterize_points(q, fi, n, (16, 16), 0.15, 4)
    np.testing.assert_array_equal(o2["idx"][0, :, :-1], o["idx"][0, :, 1:])
    np.testing.assert_array_equal(o2["dists"][0, :, :-1], o["dists"][0, :, 1:])
    # mirror x -> -x reverses the columns
    m = p.copy()
    m[:, 0] = -m[:, 0]
    o3 = oracle.rasterize_points(m, fi, n, (16, 16), 0.15, 4)
    np.testing.assert_array_equal(o3["idx"][0, :, ::-1], o["idx"][0])


def test_invariants_and_clouds():
    b = meshgen.make_points_config(2, image_override=24)
    o = oracle.rasterize_points(b.points, b.first_idx, b.num_points, b.image_size, b.radius, b.points_per_pixel)
    idx, z, d = o["idx"], o["zbuf"], o["dists"]
    valid = idx >= 0
    assert valid.any()
    assert not (valid[..., 1:] & ~valid[..., :-1]).any()
    both = valid[..., 1:] & valid[..., :-1]
    assert (np.diff(z, axis=-1)[both] >= 0).all()
    assert (d[valid] < b.radius ** 2).all() and (d[valid] >= 0).all()
    lo = b.first_idx[:, None, None, None]
    hi = lo + b.num_points[:, None, None, None]
    assert (((idx >= lo) & (idx < hi)) | ~valid).all()
    # pixel list mode gives the same rows
    pix = np.array([0, 5, 24 * 24 + 7, 3 * 24 * 24 + 100])
    r = oracle.rasterize_points(b.points, b.first_idx, b.num_points, b.image_size, b.radius, b.points_per_pixel,
                                pixels=pix)
    np.testing.assert_array_equal(r["idx"], idx.reshape(-1, idx.shape[-1])[pix])


def test_backward_fd():
    b = meshgen.make_points_config(1, image_override=20)
    o = oracle.rasterize_points(b.points, b.first_idx, b.num_points, b.image_size, b.radius, b.points_per_pixel)
    rng = np.random.default_rng(1)
    gz = rng.standard_normal(o["idx"].shape)
    gd = rng.standard_normal(o["idx"].shape)
    g = oracle.points_backward(b.points, b.image_size, o["idx"], gz, gd)
    P = np.asarray(b.points, np.float64)
    H, W = b.image_size
    r, c = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    px = (1 - (2 * c + 1) / W)[None, ..., None]
    py = (1 - (2 * r + 1) / H)[None, ..., None]
    valid = o["idx"] >= 0

    def loss(Q):
        q = Q[np.where(valid, o["idx"], 0)]
        d2 = (q[..., 0] - px) ** 2 + (q[..., 1] - py) ** 2
        return float((np.where(valid, gz * q[..., 2] + gd * d2, 0.0)).sum())

    h = 1e-6
    for pi in rng.choice(np.unique(o["idx"][valid]), 10, replace=False):
        for k in range(3):
            Qp, Qm = P.copy(), P.copy()
            Qp[pi, k] += h
            Qm[pi, k] -= h
            fd = (loss(Qp) - loss(Qm)) / (2 * h)
            assert abs(fd - g[pi, k]) < 1e-6 * max(1.0, abs(fd)), (pi, k, fd, g[pi, k])


def comp_case(seed=0, K=5, D=3):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 30, (2, 3, 4, K))
    cut = rng.integers(0, K + 1, (2, 3, 4))
    idx = np.where(np.arange(K) < cut[..., None], idx, -1)   # valid slots form a prefix
    a = rng.uniform(0, 1, idx.shape)
    f = rng.uniform(0, 1, (30, D))
    return idx, a, f


def test_compositing_closed_forms():
    idx, a, f = comp_case()
    # an opaque first point hides everything behind it
    a2 = a.copy()
    a2[..., 0] = 1.0
    out = oracle.alpha_composite(idx, a2, f)
    has = idx[..., 0] >= 0
    np.testing.assert_allclose(out[has], f[idx[..., 0][has]], rtol=0, atol=1e-15)
    # equal opacities and features: alpha gives f (1 - (1-a)^n) over n points, norm gives f
    K = 6
    idx2 = np.tile(np.arange(K), (1, 1, 1, 1))
    same = np.full((7, 2), 0.3)
    for n_valid in range(1, K + 1):
        ix = np.where(np.arange(K) < n_valid, idx2, -1)
        aa = np.full(ix.shape, 0.4)
        np.testing.assert_allclose(oracle.alpha_composite(ix, aa, same)[0, 0, 0], 0.3 * (1 - 0.6 ** n_valid),
                                   rtol=1e-14)
        np.testing.assert_allclose(oracle.norm_composite(ix, aa, same)[0, 0, 0], 0.3, rtol=1e-14)
    # norm ignores the slot order; empty pixels are 0 under both
    perm = np.array([2, 0, 4, 1, 3])
    full = np.tile(np.arange(5), (1, 1, 1, 1))
    aa = np.random.default_rng(2).uniform(0, 1, full.shape)
    np.testing.assert_allclose(oracle.norm_composite(full[..., perm], aa[..., perm], f),
                               oracle.norm_composite(full, aa, f), rtol=1e-14)
    empty = np.full((1, 1, 1, 3), -1)
    assert (oracle.alpha_composite(empty, np.ones(empty.shape), f) == 0).all()
    assert (oracle.norm_composite(empty, np.ones(empty.shape), f) == 0).all()


@pytest.mark.parametrize("mode", ["alpha", "norm"])
def test_compositing_backward_fd(mode):
    idx, a, f = comp_case(seed=4)
    g = np.random.default_rng(5).standard_normal(idx.shape[:-1] + (f.shape[1],))
    fwd = dict(alpha=oracle.alpha_composite, norm=oracle.norm_composite)[mode]
    bwd = dict(alpha=oracle.alpha_composite_backward, norm=oracle.norm_composite_backward)[mode]
    ga, gf = bwd(idx, a, f, g)
    h = 1e-7
    rng = np.random.default_rng(6)
    for _ in range(20):
        i = tuple(rng.integers(0, s) for s in a.shape)
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = ((fwd(idx, ap, f) - fwd(idx, am, f)) * g).sum() / (2 * h)
        assert abs(fd - ga[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, ga[i])
    for _ in range(10):
        i = (rng.integers(0, f.shape[0]), rng.integers(0, f.shape[1]))
        fp, fm = f.copy(), f.copy()
        fp[i] += h
        fm[i] -= h
        fd = ((fwd(idx, a, fp) - fwd(idx, a, fm)) * g).sum() / (2 * h)
        assert abs(fd - gf[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, gf[i])


def test_splat_alpha_closed_form():
    idx = np.array([[3, 7, -1]])
    r = 0.25
    d = np.array([[0.0, r * r / 4, 0.5]])
    a = oracle.splat_alpha(idx, d, r)
    # opaque at the point, 3/4 at half the radius (d = r^2 / 4), nothing for an empty slot
    np.testing.assert_allclose(a, [[1.0, 0.75, 0.0]], rtol=0, atol=1e-15)
    # zero at the rim and linear in d in between
    np.testing.assert_allclose(oracle.splat_alpha([[0]], [[r * r]], r), [[0.0]], atol=1e-15)
    ds = np.linspace(0, r * r, 9)[None, :]
    assert np.allclose(np.diff(oracle.splat_alpha(np.zeros_like(ds, int), ds, r)), -1 / 8)
