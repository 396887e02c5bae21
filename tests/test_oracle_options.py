"""Pins of the oracle's rasterizer options (perspective-correct and clipped
barycentrics, back-face culling): hand-computed cases, invariants that hold
on closed convex meshes, and central finite differences of the
frozen-selection map for the backward under every combination."""
import numpy as np
import pytest

import oracle
from paper_2007_08501_amd import meshgen

from test_oracle_pins import sphere_batch

PC, CL, CU = oracle.PERSPECTIVE_CORRECT, oracle.CLIP_BARYCENTRIC, oracle.CULL_BACKFACES


def one(v, f, size, blur, K, options, pixels=None):
    v = np.asarray(v, np.float64)
    f = np.asarray(f, np.int64)
    return oracle.rasterize(v, f, [0], [f.shape[0]], size, blur, K, pixels=pixels, options=options)


TRI = np.array([[0.9, -0.8, 1.0], [-0.9, -0.8, 2.0], [0.0, 0.9, 4.0]])


def test_perspective_hand_case():
    H = W = 16
    raw = one(TRI, [[0, 1, 2]], (H, W), 0.0, 1, 0)
    per = one(TRI, [[0, 1, 2]], (H, W), 0.0, 1, PC)
    inside = raw["p2f"][0, ..., 0] >= 0
    assert inside.sum() > 50
    np.testing.assert_array_equal(per["p2f"], raw["p2f"])
    w = raw["bary"][0][inside][:, 0, :]
    u = w / TRI[:, 2]
    D = u.sum(-1, keepdims=True)
    np.testing.assert_allclose(per["bary"][0][inside][:, 0, :], u / D, rtol=1e-13, atol=1e-15)
    # the corrected depth is the harmonic interpolation 1 / sum_i (w_i / z_i)
    np.testing.assert_allclose(per["zbuf"][0][inside][:, 0], 1.0 / D[:, 0], rtol=1e-13)
    # distances are geometric and unchanged
    np.testing.assert_array_equal(per["dists"], raw["dists"])


def test_perspective_is_identity_at_equal_depths_and_needs_positive_depths():
    t = TRI.copy()
    t[:, 2] = 2.5
    raw = one(t, [[0, 1, 2]], (12, 12), 0.01, 1, 0)
    per = one(t, [[0, 1, 2]], (12, 12), 0.01, 1, PC)
    np.testing.assert_array_equal(per["p2f"], raw["p2f"])
    np.testing.assert_allclose(per["bary"], raw["bary"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(per["zbuf"], raw["zbuf"], rtol=1e-14)
    # a vertex at z <= 0: the face never counts under the correction
    t[1, 2] = 0.0
    assert (one(t, [[0, 1, 2]], (12, 12), 0.01, 1, PC)["p2f"] < 0).all()
    assert (one(t, [[0, 1, 2]], (12, 12), 0.01, 1, 0)["p2f"] >= 0).any()


def test_clip_hand_case():
    H = W = 16
    blur = 0.04
    raw = one(TRI, [[0, 1, 2]], (H, W), blur, 1, 0)
    cl = one(TRI, [[0, 1, 2]], (H, W), blur, 1, CL)
    np.testing.assert_array_equal(cl["p2f"], raw["p2f"])
    hit = raw["p2f"][0, ..., 0] >= 0
    w = raw["bary"][0][hit][:, 0, :]
    outside = (w <= 0).any(-1)
    assert outside.sum() > 5 and (~outside).sum() > 50
    m = np.maximum(w, 0)
    wc = m / m.sum(-1, keepdims=True)
    np.testing.assert_allclose(cl["bary"][0][hit][:, 0, :], wc, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(cl["zbuf"][0][hit][:, 0], wc @ TRI[:, 2], rtol=1e-13)
    # inside pixels keep their barycentrics (up to the renormalisation's
    # rounding); outside ones lie on the triangle
    np.testing.assert_allclose(cl["bary"][0][hit][~outside], raw["bary"][0][hit][~outside], rtol=0, atol=1e-15)
    assert (cl["bary"][0][hit] >= 0).all()


def test_cull_hand_case():
    # the same triangle in both windings: E < 0 for (0, 1, 2) (anticlockwise as displayed, +x to the left)
    f = [[0, 1, 2], [0, 2, 1]]
    E = (TRI[1, 0] - TRI[0, 0]) * (TRI[2, 1] - TRI[0, 1]) - (TRI[1, 1] - TRI[0, 1]) * (TRI[2, 0] - TRI[0, 0])
    assert E < 0
    both = one(TRI, f, (12, 12), 0.0, 2, 0)
    cu = one(TRI, f, (12, 12), 0.0, 2, CU)
    cov = both["p2f"][0, ..., 0] >= 0
    assert cov.sum() > 20
    assert (both["p2f"][0][cov][:, 1] >= 0).all()          # both windings without culling
    assert (cu["p2f"][0][cov][:, 0] == 0).all() and (cu["p2f"][0][cov][:, 1] == -1).all()


def test_cull_keeps_the_visible_surface_of_a_convex_mesh():
    # closed outward-facing convex spheres (no noise, no blur): the nearest
    # face covering a pixel faces the camera, so K = 1 is the same with and
    # without culling, and culling removes about half the faces from deeper
    # slots
    rng = np.random.default_rng(21)
    meshes = []
    for L in (3, 2):
        u, fl = meshgen.icosphere(L)
        meshes.append((meshgen.transform_mesh(u, rot=meshgen.random_rotation(rng), ndc_scale=0.8,
                                              offset=rng.uniform(-0.2, 0.2, 2), dz=2.0), fl))
    v, f, fi, nf, _, _ = meshgen.pack(meshes)
    a = oracle.rasterize(v, f, fi, nf, (32, 32), 0.0, 1)
    b = oracle.rasterize(v, f, fi, nf, (32, 32), 0.0, 1, options=CU)
    ok = (a["amb"] == 0) & (b["amb"] == 0)
    assert ok.sum() > 500
    np.testing.assert_array_equal(a["p2f"][ok], b["p2f"][ok])
    a4 = oracle.rasterize(v, f, fi, nf, (32, 32), 0.0, 4)
    b4 = oracle.rasterize(v, f, fi, nf, (32, 32), 0.0, 4, options=CU)
    assert (b4["p2f"] >= 0).sum() < 0.8 * (a4["p2f"] >= 0).sum()
    # every kept face has E < 0
    vv = np.asarray(v, np.float64)
    sel = b4["p2f"][b4["p2f"] >= 0]
    P = vv[np.asarray(f)[sel]]
    E = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
    assert (E < 0).all()


def _fd(options, seed):
    v, f, fi, nf = sphere_batch([2], seed=30 + seed)
    v = np.asarray(v, np.float64)
    size = (20, 20)
    blur = 4e-3
    o = oracle.rasterize(v, f, fi, nf, size, blur, 3, options=options)
    p2f = o["p2f"]
    rng = np.random.default_rng(seed)
    gz = rng.standard_normal(p2f.shape)
    gb = rng.standard_normal(p2f.shape + (3,))
    gd = rng.standard_normal(p2f.shape)
    _, wraw, _, tie = oracle.fragments_fixed(v, f, size, p2f)
    gd = np.where(tie.astype(bool), 0.0, gd)
    # clipping has a kink where a barycentric crosses 0: leave those slots out
    near0 = (np.abs(wraw) < 1e-4).any(-1) & (p2f >= 0)
    gz = np.where(near0, 0.0, gz)
    gb = np.where(near0[..., None], 0.0, gb)
    gd = np.where(near0, 0.0, gd)
    g = oracle.backward(v, f, size, p2f, gz, gb, gd, options=options)

    def loss(vv):
        z, b, d, _ = oracle.fragments_fixed(vv, f, size, p2f, options=options)
        val = p2f >= 0
        return (np.where(val, z, 0) * gz).sum() + (np.where(val[..., None], b, 0) * gb).sum() + \
            (np.where(val, d, 0) * gd).sum()

    h = 1e-7
    err = 0.0
    coords = [(int(i), int(j)) for i, j in zip(rng.integers(0, v.shape[0], 40), rng.integers(0, 3, 40))]
    for i, j in coords:
        vp, vm = v.copy(), v.copy()
        vp[i, j] += h
        vm[i, j] -= h
        err = max(err, abs((loss(vp) - loss(vm)) / (2 * h) - g[i, j]))
    return err, np.abs(g).max()


@pytest.mark.parametrize("options", [PC, CL, CU, PC | CL, PC | CL | CU])
def test_backward_fd_with_options(options):
    err, scale = _fd(options, seed=options % 17)
    assert scale > 0
    assert err <= 1e-6 * scale, (err, scale)
