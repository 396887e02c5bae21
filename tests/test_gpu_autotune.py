"""The scheduling layer on the GPU: the autotuner's choice, its cache, the
recount that keeps a cached capacity correct when the vertices change, and
the heterogeneous configuration in its stated form (autotuned bins,
persistent most-loaded-first scheduler, forward+backward replayed from one
HIP graph), each against the FP64 oracle.

The paper times batches of heterogeneous meshes, where its two-pass
rasterizer gains most (Section 3.2, "Performance"; Appendix A); the bin
parameters of that form come from the autotuner, which the paper does not
have.
"""
import numpy as np
import pytest
import torch

import oracle
from _util import (compare_fwd, compare_grad, frag_numpy, invariants_torch, log, run_bwd, threads,
                   tie_masked_grads, to_dev)
from paper_2007_08501_amd import _lib, autotune, meshgen
from paper_2007_08501_amd.graph import GraphRunner
from paper_2007_08501_amd.raster import RasterSettings, count_max_faces_per_bin, rasterize_meshes

pytestmark = pytest.mark.gpu


def reduced_cfg3():
    # six heterogeneous meshes (levels drawn from {2..5}), 128x128, K = 8
    return meshgen.make_config(3, n_override=6, image_override=128)


def oracle_fwd(b, K=None):
    return oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                            K or b.faces_per_pixel, nthreads=threads())


def test_autotune_choice_is_cached_per_signature(monkeypatch):
    b = reduced_cfg3()
    v, f, fi, nf = to_dev(b)
    H, W = b.image_size
    K = b.faces_per_pixel
    ch = autotune.autotune(v, f, fi, nf, H, W, b.blur_radius, K, reps=1, force=True)
    log("choice", ch)
    assert ch.bin_size == 0 or (ch.bin_size % _lib.RAST_TILE == 0 and ch.bin_size in autotune.DEFAULT_BIN_SIZES)
    if ch.bin_size > 0:
        # the capacity is the exact largest bin count rounded up to 32
        mx = count_max_faces_per_bin(v, f, fi, nf, H, W, b.blur_radius, ch.bin_size)
        assert ch.max_faces_per_bin >= mx and ch.max_faces_per_bin % 32 == 0 and ch.max_faces_per_bin - mx < 32
    assert ch.sched in (_lib.RAST_SCHED_GRID, _lib.RAST_SCHED_PERSISTENT)
    assert np.isfinite(ch.ms) and ch.ms > 0

    # a second call with the same signature is answered from the cache: no candidate is timed
    def no_timing(*a, **k):
        raise AssertionError("the cached choice was not used")

    monkeypatch.setattr(autotune, "_time_step", no_timing)
    assert autotune.autotune(v, f, fi, nf, H, W, b.blur_radius, K) is ch
    # moved vertices with the same statistics share the signature (the recount covers them)
    assert autotune.autotune(v * 0.5, f, fi, nf, H, W, b.blur_radius, K) is ch
    # another K, image size or blur radius is another problem
    sig = autotune.signature(v, f, fi, nf, H, W, b.blur_radius, K)
    assert autotune.signature(v, f, fi, nf, H, W, b.blur_radius, K + 1) != sig
    assert autotune.signature(v, f, fi, nf, H, W // 2, b.blur_radius, K) != sig
    assert autotune.signature(v, f, fi, nf, H, W, 2 * b.blur_radius, K) != sig


def test_rasterize_autotuned_vs_oracle_forward_and_backward():
    b = reduced_cfg3()
    v, f, fi, nf = to_dev(b)
    vg = v.clone().requires_grad_(True)
    s = RasterSettings(image_size=b.image_size, blur_radius=b.blur_radius, faces_per_pixel=b.faces_per_pixel,
                       bin_size=None)
    frags = rasterize_meshes(vg, f, fi, nf, s)
    invariants_torch(frags, fi, nf, b.blur_radius)
    o = oracle_fwd(b)
    st = compare_fwd(frag_numpy(frags), o, b, "autotuned reduced cfg3")
    log(st)
    # backward through autograd (the forward's workspace reused), against the
    # oracle's analytic backward on the GPU's own selection; distance
    # gradients of slots whose two nearest edges tie are zeroed on both sides
    gz, gb, gd = meshgen.upstream_grads(b)
    p2f = frags.pix_to_face.detach().cpu().numpy()
    gz, gb, gd = tie_masked_grads(b, p2f, gz, gb, gd)
    t = lambda a: torch.from_numpy(a).cuda()
    loss = (frags.zbuf * t(gz)).sum() + (frags.bary * t(gb)).sum() + (frags.dists * t(gd)).sum()
    g, = torch.autograd.grad(loss, vg)
    ref = oracle.backward(b.verts, b.faces, b.image_size, p2f, gz, gb, gd, nthreads=threads())
    log("autotuned backward rel err", compare_grad(g.cpu().numpy(), ref, "autotuned backward"))


def test_cached_capacity_too_small_is_recounted():
    """A cached choice whose capacity no longer fits (the cache is keyed on
    the batch's statistics, not on its vertices): the forward reports the
    overflow, the front end recounts and rasterizes again, and the result is
    the oracle's."""
    b = reduced_cfg3()
    v, f, fi, nf = to_dev(b)
    H, W = b.image_size
    K = b.faces_per_pixel
    bs = 16
    mx = count_max_faces_per_bin(v, f, fi, nf, H, W, b.blur_radius, bs)
    assert mx > 32, mx
    key = autotune.signature(v, f, fi, nf, H, W, b.blur_radius, K) + "|bwd"
    saved = dict(autotune._cache)
    try:
        autotune._cache[key] = autotune.Choice(bs, 32, _lib.RAST_SCHED_PERSISTENT, 1.0)
        # the stale capacity overflows when used directly ...
        s_fixed = RasterSettings(image_size=b.image_size, blur_radius=b.blur_radius, faces_per_pixel=K, bin_size=bs,
                                 max_faces_per_bin=32)
        with pytest.raises(Exception, match="max_faces_per_bin"):
            rasterize_meshes(v, f, fi, nf, s_fixed)
        # ... and the autotuned front end recovers from it
        vg = v.clone().requires_grad_(True)
        s = RasterSettings(image_size=b.image_size, blur_radius=b.blur_radius, faces_per_pixel=K, bin_size=None)
        frags = rasterize_meshes(vg, f, fi, nf, s)
        o = oracle_fwd(b)
        log(compare_fwd(frag_numpy(frags), o, b, "recounted capacity"))
        gz = meshgen.upstream_grads(b)[0]
        g, = torch.autograd.grad((frags.zbuf * torch.from_numpy(gz).cuda()).sum(), vg)
        ref = oracle.backward(b.verts, b.faces, b.image_size, frags.pix_to_face.cpu().numpy(), grad_zbuf=gz,
                              nthreads=threads())
        compare_grad(g.cpu().numpy(), ref, "recounted capacity backward")
    finally:
        autotune._cache.clear()
        autotune._cache.update(saved)


def test_cfg3_full_size_autotuned_persistent_graph():
    """Config 3 at full size (32 heterogeneous meshes, 512x512, K = 8) in
    its stated form: autotuned bin size and capacity, the persistent
    scheduler, forward+backward captured in one HIP graph and replayed.
    Every replay equals the eager step; the fragments match the oracle on a
    seeded sample of 8,192 pixels (validity checked on flagged ones); the
    dense gradient equals the single-pass backward's on the same selection,
    and the backward in the graph's bin parameters matches the oracle's on
    the sampled pixels."""
    b = meshgen.make_config(3)
    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    d = to_dev(b)
    v, f, fi, nf = d
    ch = autotune.autotune(v, f, fi, nf, H, W, b.blur_radius, K, reps=1, force=True)
    log("cfg3 autotuned", ch)
    bs = ch.bin_size if ch.bin_size > 0 else 16
    M = ch.max_faces_per_bin if ch.bin_size > 0 else count_max_faces_per_bin(v, f, fi, nf, H, W, b.blur_radius, bs)
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    gr = GraphRunner(v, f, fi, nf, H, W, b.blur_radius, K, bs, M, sched=_lib.RAST_SCHED_PERSISTENT)
    gr.set_grads(gz, gb, gd)
    gr.step_eager()
    torch.cuda.synchronize()
    eager = [x.clone() for x in gr.out] + [gr.grad_verts.clone()]
    gr.capture(warmup=1)
    for rep in range(3):
        gr.replay()
        torch.cuda.synchronize()
        st, mx = gr.status()
        assert st == _lib.RAST_OK, (_lib.status_string(st), mx)
        for x, y in zip(eager[:4], gr.out):
            assert torch.equal(x, y), f"replay {rep}: fragments differ from the eager step"
        torch.testing.assert_close(gr.grad_verts, eager[4], rtol=0,
                                   atol=1e-6 * float(eager[4].abs().max()), msg=f"replay {rep}: grad_verts")
    invariants_torch(gr.out, fi, nf, b.blur_radius)
    pix = np.unique(np.random.default_rng(33).integers(0, N * H * W, 8192))
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius, K, pixels=pix,
                         nthreads=threads())
    st = compare_fwd(frag_numpy(gr.out, pix), o, b, "cfg3 graph", pixels=pix)
    log("cfg3 graph sampled", st)
    # dense selection: the graph's gradient against the single-pass backward (another kernel path)
    ref_sp = run_bwd(b, gr.out.pix_to_face, gz, gb, gd, dev_inputs=d, bs=0)
    torch.testing.assert_close(gr.grad_verts, ref_sp, rtol=0, atol=2e-5 * float(ref_sp.abs().max()),
                               msg="graph backward vs single-pass backward")
    # oracle parity of the backward in the graph's bin parameters on the sampled pixels
    gz_n, gb_n, gd_n = meshgen.upstream_grads(b)
    gz_n, gb_n, gd_n = tie_masked_grads(b, o["p2f"], gz_n, gb_n, gd_n, pixels=pix)
    p2f = np.full((N * H * W, K), -1, np.int32)
    p2f[pix] = o["p2f"]
    rows = lambda a: a.reshape((N * H * W,) + a.shape[3:])[pix]
    ref = oracle.backward(b.verts, b.faces, (H, W), o["p2f"], rows(gz_n), rows(gb_n), rows(gd_n),
                          nthreads=threads(), pixels=pix, N=N)
    g = run_bwd(b, torch.from_numpy(p2f.reshape(N, H, W, K)).cuda(), gz_n, gb_n, gd_n, dev_inputs=d, bs=bs, M=M)
    log("cfg3 graph-config backward rel err", compare_grad(g.cpu().numpy(), ref, "cfg3 sampled backward"))
