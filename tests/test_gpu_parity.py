"""GPU parity: the HIP rasterizer (through the C ABI) against the FP64 oracle.

Small cases are compared in full; the full-size workloads are compared on
seeded pixel samples (forward, and backward over the oracle's selection on
those pixels), plus size-independent invariants.  The oracle never takes an
input produced by the GPU.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
from paper_2007_08501_amd import _lib, meshgen
from paper_2007_08501_amd.raster import empty_fragments, round_up

from _util import (bin_capacity, compare_fwd, compare_grad, frag_numpy, invariants_torch, log, run_bwd, run_fwd,
                   threads, tie_masked_grads, to_dev)

pytestmark = pytest.mark.gpu


def oracle_full(b, K=None):
    return oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                            K or b.faces_per_pixel, nthreads=threads())


def small_cfg(i, **kw):
    return meshgen.make_config(i, **kw)


# ----------------------------------------------------------------- forward

def test_cfg1_naive_vs_oracle():
    b = meshgen.make_config(1)
    log("cfg1 naive", b.image_size, b.faces.shape)
    out, _ = run_fwd(b, 0)
    o = oracle_full(b)
    st = compare_fwd(frag_numpy(out), o, b, "cfg1")
    log("cfg1", st)
    assert st["slots"] > 1000


@pytest.mark.parametrize("bs", [8, 16, 24, 32, 64])
def test_binned_equals_naive_bitwise(bs):
    b = meshgen.make_config(2, n_override=3, level_override=3, image_override=72)
    log("binned==naive", bs)
    d = to_dev(b)
    naive, _ = run_fwd(b, 0, dev_inputs=d)
    for sched in (0, 1):
        binned, _ = run_fwd(b, bs, sched=sched, dev_inputs=d)
        for x, y in zip(naive, binned):
            assert torch.equal(x, y)


def test_reduced_cfg2_vs_oracle_ragged():
    # 3 meshes at level 3, a 72x88 image: ragged against 8-pixel tiles and 32-pixel bins
    b = meshgen.make_config(2, n_override=3, level_override=3)
    b.image_size = (72, 88)
    log("cfg2 reduced ragged")
    out, _ = run_fwd(b, 32)
    o = oracle_full(b)
    st = compare_fwd(frag_numpy(out), o, b, "cfg2-reduced")
    log(st)


def test_reduced_cfg3_heterogeneous_vs_oracle():
    b = meshgen.make_config(3, n_override=6, level_override=4, image_override=96)
    log("cfg3 reduced", b.levels)
    for bs, sched in ((0, 0), (16, 1), (24, 0)):
        out, _ = run_fwd(b, bs, sched=sched)
        o = oracle_full(b)
        st = compare_fwd(frag_numpy(out), o, b, f"cfg3-reduced bs{bs}")
        log(bs, sched, st)


def test_reduced_cfg5_K50_vs_oracle():
    b = meshgen.make_config(5, n_override=3, level_override=3, image_override=48)
    log("cfg5 reduced K=50")
    out, _ = run_fwd(b, 16)
    o = oracle_full(b)
    st = compare_fwd(frag_numpy(out), o, b, "cfg5-reduced")
    log(st)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 7, 8, 12, 16, 20, 32, 33, 64])
def test_every_K_bucket(K):
    b = meshgen.make_config(2, n_override=2, level_override=3, image_override=40)
    b.blur_radius = float(np.float32(3e-3))
    out, _ = run_fwd(b, 8, K=K)
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius, K,
                         nthreads=threads())
    compare_fwd(frag_numpy(out), o, b, f"K={K}")


def test_batch_equals_per_mesh_bitwise():
    b = meshgen.make_config(3, n_override=5, level_override=4, image_override=64)
    out, _ = run_fwd(b, 16)
    for n in range(b.N):
        fs = b.faces[b.first_idx[n]:b.first_idx[n] + b.num_faces[n]]
        one = meshgen.Batch(name="one", verts=b.verts, faces=np.ascontiguousarray(fs), first_idx=np.array([0]),
                            num_faces=np.array([fs.shape[0]]), verts_first_idx=np.array([0]),
                            num_verts=np.array([b.verts.shape[0]]), image_size=b.image_size,
                            faces_per_pixel=b.faces_per_pixel, blur_radius=b.blur_radius, bin_size=16,
                            max_faces_per_bin=None)
        o1, _ = run_fwd(one, 16)
        p = o1.pix_to_face[0]
        exp = torch.where(p >= 0, p + int(b.first_idx[n]), p)
        assert torch.equal(out.pix_to_face[n], exp)
        for x, y in zip(out[1:], o1[1:]):
            assert torch.equal(x[n], y[0])


def test_forward_deterministic():
    b = meshgen.make_config(2, n_override=4, level_override=4, image_override=128)
    d = to_dev(b)
    ref, _ = run_fwd(b, 16, sched=1, dev_inputs=d)
    for _ in range(5):
        again, _ = run_fwd(b, 16, sched=1, dev_inputs=d)
        for x, y in zip(ref, again):
            assert torch.equal(x, y)


# ----------------------------------------------------------------- full-size samples

def sampled_check(i, bs, n_pix=1500, seed=0, sched=1, M=None):
    b = meshgen.make_config(i)
    log(f"cfg{i} full size", b.image_size, b.faces.shape, "bs", bs, "M", M, "sched", sched)
    d = to_dev(b)
    out, _ = run_fwd(b, bs, M=M, sched=sched, dev_inputs=d)
    torch.cuda.synchronize()
    invariants_torch(out, d[2], d[3], b.blur_radius)
    N, (H, W) = b.N, b.image_size
    # seeded uniform pixel sample (the meshes cover most of every image)
    pix = np.unique(np.random.default_rng(seed).integers(0, N * H * W, n_pix))
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                         b.faces_per_pixel, pixels=pix, nthreads=threads())
    st = compare_fwd(frag_numpy(out, pix), o, b, f"cfg{i}-sampled", pixels=pix)
    log(st)
    return b, d, out, pix, o


def full_backward_check(b, d, out, pix, o, bins):
    """Backward at full size in the launch configuration.  Parity: both sides
    take the oracle's selection on the sampled pixels (every other pixel
    empty).  At full density: the bin-major passes against the per-face pass
    on the GPU's own selection, and additivity over a split of the pixels."""
    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    gz, gb, gd = meshgen.upstream_grads(b)
    rows = lambda a: a.reshape((N * H * W,) + a.shape[3:])[pix]
    gz, gb, gd = tie_masked_grads(b, o["p2f"], gz, gb, gd, pixels=pix)
    p2f = np.full((N * H * W, K), -1, np.int32)
    p2f[pix] = o["p2f"]
    p2f = p2f.reshape(N, H, W, K)
    ref = oracle.backward(b.verts, b.faces, b.image_size, o["p2f"], rows(gz), rows(gb), rows(gd),
                          nthreads=threads(), pixels=pix, N=N)
    p2f_dev = torch.from_numpy(p2f).cuda()
    for bs in bins:
        gv = run_bwd(b, p2f_dev, gz, gb, gd, dev_inputs=d, bs=bs).cpu().numpy()
        log(f"{b.name} bs{bs} sampled grad rel err", compare_grad(gv, ref, f"{b.name} bs{bs}"))
    # dense selection: every slot of the forward, all passes must agree
    gz_t, gb_t, gd_t = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    dense = [run_bwd(b, out.pix_to_face, gz_t, gb_t, gd_t, dev_inputs=d, bs=bs) for bs in bins]
    scale = float(dense[0].abs().max())
    for bs, g in zip(bins[1:], dense[1:]):
        torch.testing.assert_close(g, dense[0], rtol=0, atol=2e-5 * scale, msg=f"dense bs{bs} vs bs{bins[0]}")
    half = torch.zeros(N, H, W, 1, dtype=torch.bool, device="cuda")
    half[:, ::2] = True
    empty = torch.full_like(out.pix_to_face, -1)
    a = run_bwd(b, torch.where(half, out.pix_to_face, empty), gz_t, gb_t, gd_t, dev_inputs=d, bs=bins[-1])
    c = run_bwd(b, torch.where(half, empty, out.pix_to_face), gz_t, gb_t, gd_t, dev_inputs=d, bs=bins[-1])
    torch.testing.assert_close(a + c, dense[-1], rtol=0, atol=2e-5 * scale, msg="additivity over pixel halves")


def test_cfg2_full_size_sampled_and_backward():
    full_backward_check(*sampled_check(2, 32), bins=(0, 8, 16))


def test_cfg3_full_size_sampled_and_backward():
    full_backward_check(*sampled_check(3, 16), bins=(0, 8, 16))


def test_cfg4_full_size_sampled_and_backward():
    full_backward_check(*sampled_check(4, 16, n_pix=800), bins=(0, 8, 16))


def test_cfg4_bench_launch_config_sampled():
    """Config 4 in the launch configuration the benchmark times (8-pixel
    bins, capacity rounded up to 32 from the exact count, grid scheduler) on
    8,192 seeded pixels: exact ids on unflagged pixels, a correct answer by
    the oracle's candidates on every flagged one, values within tolerance;
    the fraction flagged per ambiguity bit is logged."""
    b = meshgen.make_config(4)
    M = round_up(bin_capacity(b, 8), 32)
    b, d, out, pix, o = sampled_check(4, 8, n_pix=8192, seed=77, sched=0, M=M)
    assert pix.size >= 8000


# ----------------------------------------------------------------- backward

@pytest.mark.parametrize("bs", [0, 8, 16, 32])
@pytest.mark.parametrize("which", ["zbuf", "bary", "dists", "all"])
def test_backward_vs_oracle_small(which, bs):
    b = meshgen.make_config(2, n_override=3, level_override=3, image_override=64)
    # both sides take the oracle's selection
    p2f = oracle_full(b)["p2f"]
    gz, gb, gd = meshgen.upstream_grads(b)
    gz, gb, gd = tie_masked_grads(b, p2f, gz, gb, gd)
    sel = dict(zbuf=(gz, None, None), bary=(None, gb, None), dists=(None, None, gd), all=(gz, gb, gd))[which]
    gv = run_bwd(b, torch.from_numpy(p2f.astype(np.int32)).cuda(), *sel, bs=bs).cpu().numpy()
    ref = oracle.backward(b.verts, b.faces, b.image_size, p2f, *sel, nthreads=threads())
    compare_grad(gv, ref, which)


@pytest.mark.parametrize("bs", [0, 8, 16])
def test_backward_tiny_upstream_gradients(bs):
    """Upstream gradients of a mean over every slot of a large image (about
    1e-8 each, as for config 4's 67 M slots): the binned sums carry no
    absolute rounding grid, so the result keeps the relative tolerance."""
    b = meshgen.make_config(2, n_override=3, level_override=3, image_override=64)
    p2f = oracle_full(b)["p2f"]
    gz, gb, gd = meshgen.upstream_grads(b)
    gz, gb, gd = tie_masked_grads(b, p2f, gz, gb, gd)
    scale = np.float32(1.5e-8)
    gz, gb, gd = gz * scale, gb * scale, gd * scale
    gv = run_bwd(b, torch.from_numpy(p2f.astype(np.int32)).cuda(), gz, gb, gd, bs=bs).cpu().numpy()
    ref = oracle.backward(b.verts, b.faces, b.image_size, p2f, gz, gb, gd, nthreads=threads())
    log(f"bs{bs} tiny-gradient rel err", compare_grad(gv, ref, f"tiny upstream bs{bs}"))


def crowded_batch(F, seed, size=16, blur=1e-3, K=16):
    """F independent tiny triangles (about half a pixel across) scattered over
    a size x size image: an 8x8 bin's slots name far more distinct faces
    than one LDS chunk holds (about 300 at F = 1500, 700 at F = 4000)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, (F, 1, 2))
    xy = (c + rng.normal(0, 0.06, (F, 3, 2))).reshape(-1, 2)
    v = np.concatenate([xy, rng.uniform(1, 5, (3 * F, 1))], 1).astype(np.float32)
    f = np.arange(3 * F, dtype=np.int32).reshape(F, 3)
    return meshgen.Batch(name="crowd", verts=v, faces=f, first_idx=np.array([0]), num_faces=np.array([F]),
                         verts_first_idx=np.array([0]), num_verts=np.array([3 * F]), image_size=(size, size),
                         faces_per_pixel=K, blur_radius=blur, bin_size=8, max_faces_per_bin=None)


@pytest.mark.parametrize("F", [300, 1500, 4000])
def test_backward_crowded_bins(F):
    """Bins whose slots name more faces than an LDS chunk (and, at F = 4000,
    than the hash table) take the listed way through the bin; both ways
    match the oracle and the per-face form."""
    b = crowded_batch(F, seed=F)
    p2f = oracle_full(b)["p2f"]
    named = [len(np.unique(x[x >= 0])) for x in
             p2f.reshape(2, 8, 2, 8, -1).transpose(0, 2, 1, 3, 4).reshape(4, -1)]
    log(f"F={F}: distinct faces per bin {named}")
    gz, gb, gd = meshgen.upstream_grads(b)
    gz, gb, gd = tie_masked_grads(b, p2f, gz, gb, gd)
    t = torch.from_numpy(p2f.astype(np.int32)).cuda()
    ref = oracle.backward(b.verts, b.faces, b.image_size, p2f, gz, gb, gd, nthreads=threads())
    g8 = run_bwd(b, t, gz, gb, gd, bs=8).cpu().numpy()
    g0 = run_bwd(b, t, gz, gb, gd, bs=0).cpu().numpy()
    compare_grad(g8, ref, f"crowded F={F} bins of 8")
    compare_grad(g0, ref, f"crowded F={F} per face")


@pytest.mark.parametrize("bs", [0, 8])
def test_backward_ignores_slots_no_face_of_the_image_can_fill(bs):
    """Slot ids the forward cannot produce -- out of [0, F), a face of
    another image, a degenerate face -- contribute nothing: the gradient
    equals the one with those slots emptied."""
    b = meshgen.make_config(2, n_override=3, level_override=3, image_override=64)
    v = b.verts.copy()
    f = b.faces.copy()
    dead = int(b.first_idx[0])  # face 0 of image 0 made degenerate (never counts)
    f[dead, 1] = f[dead, 0]
    f[dead, 2] = f[dead, 0]
    b.verts, b.faces = v, f
    d = to_dev(b)
    out, _ = run_fwd(b, 8, dev_inputs=d)
    p2f = out.pix_to_face.clone()
    filled = (p2f >= 0).nonzero()
    sel = filled[torch.randperm(filled.shape[0], generator=torch.Generator().manual_seed(3))[:600].to(p2f.device)]
    F = b.faces.shape[0]
    bad = torch.empty(sel.shape[0], dtype=torch.int32, device=p2f.device)
    third = sel.shape[0] // 3
    bad[:third] = F + 5                                                  # out of range
    img = sel[third:2 * third, 0]                                       # a face of the next image
    bad[third:2 * third] = torch.from_numpy(b.first_idx).to(p2f.device)[(img + 1) % 3].int()
    bad[2 * third:] = dead                                              # the degenerate face
    corrupt = p2f.clone()
    corrupt[sel[:, 0], sel[:, 1], sel[:, 2], sel[:, 3]] = bad
    clean = p2f.clone()
    clean[sel[:, 0], sel[:, 1], sel[:, 2], sel[:, 3]] = -1
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    g_bad = run_bwd(b, corrupt, gz, gb, gd, dev_inputs=d, bs=bs)
    g_ref = run_bwd(b, clean, gz, gb, gd, dev_inputs=d, bs=bs)
    torch.testing.assert_close(g_bad, g_ref, rtol=0, atol=1e-6 * float(g_ref.abs().max()))


def test_backward_hand_case():
    # triangle T, pixel (2,2) of a 4x4 image; hand-derived gradients
    v = np.array([[-1.0, -1.0, 1.0], [1.0, -1.0, 2.0], [-1.0, 1.0, 3.0]], np.float32)
    f = np.array([[0, 1, 2]], np.int32)
    b = meshgen.Batch(name="T", verts=v, faces=f, first_idx=np.array([0]), num_faces=np.array([1]),
                      verts_first_idx=np.array([0]), num_verts=np.array([3]), image_size=(4, 4), faces_per_pixel=1,
                      blur_radius=0.0, bin_size=0, max_faces_per_bin=None)
    out, _ = run_fwd(b, 0)
    p2f = out.pix_to_face.clone()
    p2f[:] = -1
    p2f[0, 2, 2, 0] = 0
    one = torch.zeros((1, 4, 4, 1), device="cuda")
    one[0, 2, 2, 0] = 1
    for bs in (0, 8):
        g = run_bwd(b, p2f, None, None, one, bs=bs).cpu().numpy()
        np.testing.assert_allclose(g, [[0, 0, 0], [-0.25, -0.25, 0], [-0.25, -0.25, 0]], atol=1e-6)
        g = run_bwd(b, p2f, one, None, None, bs=bs).cpu().numpy()
        np.testing.assert_allclose(g, [[-0.125, -0.25, 0.25], [-0.1875, -0.375, 0.375], [-0.1875, -0.375, 0.375]],
                                   atol=1e-6)


def test_autograd_matches_abi():
    from paper_2007_08501_amd.raster import RasterSettings, rasterize_meshes
    b = meshgen.make_config(2, n_override=2, level_override=3, image_override=48)
    v, f, fi, nf = to_dev(b)
    vv = v.clone().requires_grad_(True)
    frags = rasterize_meshes(vv, f, fi, nf, RasterSettings(48, b.blur_radius, b.faces_per_pixel, bin_size=16))
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    loss = (frags.zbuf * gz).sum() + (frags.bary * gb).sum() + (frags.dists * gd).sum()
    loss.backward()
    direct = run_bwd(b, frags.pix_to_face, gz, gb, gd, bs=16)
    # float atomics accumulate in a different order on each call
    scale = float(direct.abs().max())
    torch.testing.assert_close(vv.grad, direct, rtol=0, atol=1e-5 * scale)


def test_binning_large_faces_past_the_hash_table():
    """600 large triangles over a 256x256 image in 8-pixel bins: a binning
    workgroup's 256 faces touch more distinct bins than its LDS table holds,
    so appends take the direct global path; the binned forward still equals
    the single-pass one bitwise, the recorded largest count is exact (it
    fits as the capacity, one less overflows)."""
    rng = np.random.default_rng(7)
    F = 600
    c = rng.uniform(-0.8, 0.8, (F, 1, 2))
    xy = (c + rng.normal(0, 0.35, (F, 3, 2))).reshape(-1, 2)
    v = np.concatenate([xy, rng.uniform(1, 5, (3 * F, 1))], 1).astype(np.float32)
    b = meshgen.Batch(name="large", verts=v, faces=np.arange(3 * F, dtype=np.int32).reshape(F, 3),
                      first_idx=np.array([0]), num_faces=np.array([F]), verts_first_idx=np.array([0]),
                      num_verts=np.array([3 * F]), image_size=(256, 256), faces_per_pixel=8, blur_radius=1e-4,
                      bin_size=8, max_faces_per_bin=None)
    d = to_dev(b)
    naive, _ = run_fwd(b, 0, dev_inputs=d)
    mx = bin_capacity(b, 8, d)
    log("largest bin count", mx)
    assert mx > 100
    binned, _ = run_fwd(b, 8, M=mx, dev_inputs=d)
    for x, y in zip(naive, binned):
        assert torch.equal(x, y)
    _, ws = run_fwd(b, 8, M=mx - 1, dev_inputs=d, check=False)
    st, got = _lib.rast_query_status(ws)
    assert st == _lib.RAST_EOVERFLOW and got == mx, (_lib.status_string(st), got, mx)


# ----------------------------------------------------------------- edge cases

def test_empty_and_offscreen_meshes():
    b = meshgen.make_config(2, n_override=3, level_override=2, image_override=32)
    v = b.verts.copy()
    # mesh 1 moved far off screen; mesh 2 given zero faces
    s1 = slice(int(b.verts_first_idx[1]), int(b.verts_first_idx[1] + b.num_verts[1]))
    v[s1, 0] += 5.0
    b.verts = v
    b.num_faces = b.num_faces.copy()
    b.num_faces[2] = 0
    for bs in (0, 8, 32):
        out, _ = run_fwd(b, bs)
        assert (out.pix_to_face[1:] == -1).all()
        assert (out.pix_to_face[0] >= 0).any()
        o = oracle_full(b)
        compare_fwd(frag_numpy(out), o, b, f"empty bs{bs}")


def test_bin_larger_than_image_and_K_above_hits():
    b = meshgen.make_config(1)
    b.blur_radius = float(np.float32(1e-3))
    out, _ = run_fwd(b, 128, K=12)   # one bin covers the whole 64x64 image
    o = oracle_full(b, K=12)
    compare_fwd(frag_numpy(out), o, b, "bin>image")
    assert (out.pix_to_face[..., -1] == -1).any() and (out.pix_to_face[..., 0] >= 0).any()


def test_degenerate_and_behind_camera_faces():
    v = np.array([
        [-0.5, -0.5, 1.0], [0.5, -0.5, 1.0], [0.0, 0.5, 1.0],
        [-0.9, 0.0, 0.5], [0.9, 0.0, 0.5], [0.0, 0.0, 0.5],
        [-0.5, -0.5, -1.0], [0.5, -0.5, -1.0], [0.0, 0.5, -1.0],
        [-0.2, -0.2, -0.5], [0.6, -0.2, 0.5], [-0.2, 0.6, 0.5],   # crosses z = 0
    ], np.float32)
    f = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]], np.int32)
    b = meshgen.Batch(name="deg", verts=v, faces=f, first_idx=np.array([0]), num_faces=np.array([4]),
                      verts_first_idx=np.array([0]), num_verts=np.array([12]), image_size=(24, 24),
                      faces_per_pixel=3, blur_radius=float(np.float32(1e-2)), bin_size=8, max_faces_per_bin=None)
    for bs in (0, 8):
        out, _ = run_fwd(b, bs)
        o = oracle_full(b)
        compare_fwd(frag_numpy(out), o, b, f"degenerate bs{bs}", verts=v, faces=f)
        assert not (out.pix_to_face == 1).any() and not (out.pix_to_face == 2).any()


def test_overflow_is_reported_not_truncated():
    b = meshgen.make_config(2, n_override=2, level_override=3, image_override=64)
    out, ws = run_fwd(b, 32, M=1, check=False)
    st, mx = _lib.rast_query_status(ws)
    assert st == _lib.RAST_EOVERFLOW and mx > 1


def test_bad_mesh_ranges_reported():
    b = meshgen.make_config(2, n_override=2, level_override=2, image_override=32)
    b.first_idx = np.array([0, 100], np.int64)  # overlaps mesh 0's range
    out, ws = run_fwd(b, 0, check=False)
    st, _ = _lib.rast_query_status(ws)
    assert st == _lib.RAST_EMESH


def test_zero_faces_total():
    v = np.zeros((3, 3), np.float32)
    f = np.zeros((0, 3), np.int32)
    b = meshgen.Batch(name="nil", verts=v, faces=f, first_idx=np.array([0, 0]), num_faces=np.array([0, 0]),
                      verts_first_idx=np.array([0, 0]), num_verts=np.array([3, 0]), image_size=(16, 16),
                      faces_per_pixel=2, blur_radius=0.0, bin_size=8, max_faces_per_bin=None)
    for bs in (0, 8):
        out, _ = run_fwd(b, bs, M=4)
        assert (out.pix_to_face == -1).all() and (out.zbuf == -1).all()


def test_zero_depth_faces_order_by_id():
    # coplanar copies of one triangle at z = +0 and -0: every key has a zero
    # depth, so a covered pixel lists the copies in face-id order, on both the
    # binned and the single-pass path, and agrees with the oracle
    tri = np.array([[0.8, -0.7, 0.0], [-0.8, -0.7, 0.0], [0.0, 0.8, 0.0]], np.float32)
    neg = tri.copy()
    neg[:, 2] = -0.0
    copies = 6
    v = np.concatenate([tri, neg, tri, neg, tri, neg]).astype(np.float32)
    f = (np.arange(copies)[:, None] * 3 + np.arange(3)[None, :]).astype(np.int32)
    b = meshgen.Batch(name="z0", verts=v, faces=f, first_idx=np.array([0]), num_faces=np.array([copies]),
                      verts_first_idx=np.array([0]), num_verts=np.array([v.shape[0]]), image_size=(16, 16),
                      faces_per_pixel=8, blur_radius=0.0, bin_size=8, max_faces_per_bin=None)
    o = oracle_full(b)
    covered = o["p2f"][0, ..., 0] >= 0
    assert covered.sum() > 40
    want = np.array(list(range(copies)) + [-1] * (8 - copies))
    assert (o["p2f"][0][covered] == want).all()
    for bs in (0, 8):
        out, _ = run_fwd(b, bs)
        g = frag_numpy(out)
        np.testing.assert_array_equal(g["p2f"][0][covered], np.broadcast_to(want, (int(covered.sum()), 8)))
        np.testing.assert_array_equal(g["p2f"].astype(np.int64), o["p2f"])
        assert (g["zbuf"][0][covered][:, :copies] == 0).all()


# ----------------------------------------------------------------- blend

def test_silhouette_blend_vs_oracle():
    # both sides blend the oracle's fragments (dists rounded to f32 once)
    b = meshgen.make_config(5, n_override=4, level_override=3, image_override=64)
    o = oracle_full(b)
    p2f, dn = o["p2f"], o["dists"].astype(np.float32)
    p2f_t, dn_t = torch.from_numpy(p2f.astype(np.int32)).cuda(), torch.from_numpy(dn).cuda()
    sig = meshgen.SIL_SIGMA
    alpha = torch.empty(dn_t.shape[:-1], device="cuda")
    _lib.silhouette_blend_fwd(p2f_t, dn_t, sig, alpha)
    ref = oracle.silhouette_blend(p2f, dn.astype(np.float64), sig)
    assert np.abs(alpha.cpu().numpy() - ref).max() < 1e-5
    ga_np = np.random.default_rng(7).standard_normal(alpha.shape).astype(np.float32)
    ga = torch.from_numpy(ga_np).cuda()
    gd = torch.empty_like(dn_t)
    _lib.silhouette_blend_bwd(p2f_t, dn_t, ga, sig, gd)
    refg = oracle.silhouette_blend_backward(p2f, dn.astype(np.float64), sig, ga_np)
    compare_grad(gd.cpu().numpy(), refg, "blend")


# ----------------------------------------------------------------- graphs

def test_graph_replay_matches_eager():
    from paper_2007_08501_amd.graph import GraphRunner
    b = meshgen.make_config(3, n_override=6, level_override=4, image_override=128)
    v, f, fi, nf = to_dev(b)
    _, ws0 = run_fwd(b, 16, check=True, dev_inputs=(v, f, fi, nf))
    st, mx = _lib.rast_query_status(ws0)
    gr = GraphRunner(v, f, fi, nf, 128, 128, b.blur_radius, 8, 16, 2 * mx + 64, sched=1)
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    gr.set_grads(gz, gb, gd)
    gr.step_eager()
    torch.cuda.synchronize()
    ref = [t.clone() for t in gr.out]
    ref_g = gr.grad_verts.clone()
    gr.capture()
    for it in range(4):
        # unrelated eager work between replays
        gr.out.pix_to_face.fill_(7)
        gr.grad_verts.fill_(3.0)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        for x, y in zip(ref, gr.out):
            assert torch.equal(x, y), f"replay {it}"
        # float atomics: summation order differs between runs
        torch.testing.assert_close(gr.grad_verts, ref_g, rtol=0, atol=1e-5 * float(ref_g.abs().max()))
        assert gr.status()[0] == _lib.RAST_OK
    # new vertex positions flow through the captured graph
    gr.set_verts(v * 0.9)
    gr.replay()
    torch.cuda.synchronize()
    b2 = meshgen.make_config(3, n_override=6, level_override=4, image_override=128)
    b2.verts = (b.verts * np.float32(0.9)).astype(np.float32)
    e, _ = run_fwd(b2, 16, M=2 * mx + 64, sched=1)
    for x, y in zip(e, gr.out):
        assert torch.equal(x, y)


# ----------------------------------------------------------------- backward reusing the forward's bins

def test_backward_reuse_matches_rebuild_and_checks_signature():
    b = meshgen.make_config(3, n_override=5, level_override=4, image_override=96)
    d = to_dev(b)
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    for bs in (8, 16):
        out, ws = run_fwd(b, bs, dev_inputs=d)
        M = bin_capacity(b, bs, d)
        fresh = run_bwd(b, out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=bs, M=M)
        out, ws = run_fwd(b, bs, M=M, dev_inputs=d)
        reused = run_bwd(b, out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=bs, M=M,
                         flags=_lib.RAST_BWD_REUSE_FORWARD, ws=ws)
        torch.testing.assert_close(reused, fresh, rtol=0, atol=1e-5 * float(fresh.abs().max()))
        # a second reuse of the same workspace is still valid (nothing rebuilt it)
        again = run_bwd(b, out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=bs, M=M,
                        flags=_lib.RAST_BWD_REUSE_FORWARD, ws=ws)
        torch.testing.assert_close(again, fresh, rtol=0, atol=1e-5 * float(fresh.abs().max()))
        # another blur radius than the forward's: refused, gradients left zero
        b2 = copy.copy(b)
        b2.blur_radius = b.blur_radius * 2
        bad = run_bwd(b2, out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=bs, M=M,
                      flags=_lib.RAST_BWD_REUSE_FORWARD, ws=ws, check=False)
        st, _ = _lib.rast_query_status(ws)
        assert st == _lib.RAST_EREUSE and not bad.any()
        # a counting pass in between clears the forward's signature
        out, ws = run_fwd(b, bs, M=M, dev_inputs=d)
        v, f, fi, nf = d
        H, W = b.image_size
        _lib.rast_bin_count(v, f, fi, nf, H, W, b.blur_radius, bs, ws)
        run_bwd(b, out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=bs, M=M, flags=_lib.RAST_BWD_REUSE_FORWARD, ws=ws,
                check=False)
        st, _ = _lib.rast_query_status(ws)
        assert st == _lib.RAST_EREUSE


# ----------------------------------------------------------------- softmax blend (Algorithm 2)

@pytest.mark.parametrize("C", [3, 6])
def test_softmax_blend_vs_oracle(C):
    from paper_2007_08501_amd.raster import softmax_blend
    # the oracle's fragments of a reduced textured-render batch, random per-slot colours
    b = meshgen.make_config(3, n_override=4, level_override=3, image_override=48)
    o = oracle_full(b)
    p2f, z, d = o["p2f"], o["zbuf"].astype(np.float32), o["dists"].astype(np.float32)
    rng = np.random.default_rng(C)
    col = rng.uniform(0, 1, p2f.shape + (C,)).astype(np.float32)
    gimg = rng.standard_normal(p2f.shape[:-1] + (C,)).astype(np.float32)
    prm = dict(sigma=1e-4, gamma=1e-4, znear=1.0, zfar=100.0)
    ref = oracle.softmax_blend(p2f, z.astype(np.float64), d.astype(np.float64), col.astype(np.float64), **prm)
    rgz, rgd, rgc = oracle.softmax_blend_backward(p2f, z.astype(np.float64), d.astype(np.float64),
                                                  col.astype(np.float64), **prm, grad_image=gimg)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    zt, dt, ct = t(z).requires_grad_(True), t(d).requires_grad_(True), t(col).requires_grad_(True)
    img = softmax_blend(t(p2f.astype(np.int32)), zt, dt, ct, **prm)
    assert np.abs(img.detach().cpu().numpy() - ref).max() < 1e-5
    (img * t(gimg)).sum().backward()
    compare_grad(zt.grad.cpu().numpy(), rgz, "softmax zbuf")
    compare_grad(dt.grad.cpu().numpy(), rgd, "softmax dists")
    compare_grad(ct.grad.cpu().numpy(), rgc, "softmax colors")


def test_unaligned_outputs_match_aligned():
    """Outputs that are not 16-byte aligned take the general store path; the
    fragments must be identical to those of aligned outputs."""
    b = meshgen.make_config(2, n_override=2, level_override=3, image_override=40)
    d = to_dev(b)
    ref, _ = run_fwd(b, 8, dev_inputs=d)
    v, f, fi, nf = d
    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    M = bin_capacity(b, 8, d)

    def shifted(shape, dtype):
        n = int(np.prod(shape))
        return torch.empty(n + 1, dtype=dtype, device="cuda")[1:].view(shape)

    p2f = shifted((N, H, W, K), torch.int32)
    zb = shifted((N, H, W, K), torch.float32)
    ba = shifted((N, H, W, K, 3), torch.float32)
    di = shifted((N, H, W, K), torch.float32)
    assert p2f.data_ptr() % 16 != 0
    ws = _lib.alloc_workspace(_lib.rast_workspace_size(N, H, W, f.shape[0], 8, M), v.device)
    _lib.rasterize_meshes_fwd(v, f, fi, nf, H, W, b.blur_radius, K, 8, M, 0, p2f, zb, ba, di, ws)
    torch.cuda.synchronize()
    for x, y in zip(ref, (p2f, zb, ba, di)):
        assert torch.equal(x, y)
