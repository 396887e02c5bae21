"""GPU parity of the rasterizer options (perspective-correct and clipped
barycentrics, back-face culling) against the FP64 oracle under the same
options, forward and backward, single-pass and binned, through the C ABI and
through the autograd wrapper.  Tolerances as in test_gpu_parity."""
import numpy as np
import pytest
import torch

import oracle
from paper_2007_08501_amd import _lib, meshgen

from _util import compare_fwd, compare_grad, frag_numpy, log, run_bwd, run_fwd, threads, tie_masked_grads, to_dev

pytestmark = pytest.mark.gpu

PC, CL, CU = _lib.RAST_PERSPECTIVE_CORRECT, _lib.RAST_CLIP_BARYCENTRIC, _lib.RAST_CULL_BACKFACES
COMBOS = [PC, CL, CU, PC | CL, PC | CL | CU]


def small():
    # blur 1e-4: pixels outside faces within the blur radius exercise the clipping
    return meshgen.make_config(2, n_override=3, level_override=3, image_override=64)


@pytest.mark.parametrize("bs", [0, 8, 16])
@pytest.mark.parametrize("opts", COMBOS)
def test_options_forward_vs_oracle(opts, bs):
    b = small()
    log("options fwd", hex(opts), "bs", bs)
    out, _ = run_fwd(b, bs, options=opts)
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                         b.faces_per_pixel, nthreads=threads(), options=opts)
    st = compare_fwd(frag_numpy(out), o, b, f"opts {opts:#x} bs {bs}", options=opts)
    assert st["slots"] > 1000
    p2f = out.pix_to_face.cpu().numpy()
    if opts & CL:
        bary = out.bary.cpu().numpy()[p2f >= 0]
        assert (bary >= 0).all()
    if opts & CU:
        v = b.verts.astype(np.float64)
        P = v[b.faces[p2f[p2f >= 0]]]
        E = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
        assert (E < 0).all()


def masked_grads(b, p2f, opts):
    gz, gb, gd = meshgen.upstream_grads(b)
    gz, gb, gd = tie_masked_grads(b, p2f, gz, gb, gd)
    if opts & CL:
        # clipping has a kink where a barycentric crosses 0: slots within
        # rounding of it get no upstream gradient on either side
        _, wraw, _, _ = oracle.fragments_fixed(b.verts, b.faces, b.image_size, p2f, nthreads=threads())
        near0 = (np.abs(wraw) < 1e-5).any(-1) & (p2f >= 0)
        gz = np.where(near0, np.float32(0), gz).astype(np.float32)
        gb = np.where(near0[..., None], np.float32(0), gb).astype(np.float32)
    return gz, gb, gd


@pytest.mark.parametrize("bs", [0, 8])
@pytest.mark.parametrize("opts", COMBOS)
def test_options_backward_vs_oracle(opts, bs):
    b = small()
    log("options bwd", hex(opts), "bs", bs)
    # both sides take the oracle's selection
    p2f = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                           b.faces_per_pixel, nthreads=threads(), options=opts)["p2f"]
    gz, gb, gd = masked_grads(b, p2f, opts)
    gv = run_bwd(b, torch.from_numpy(p2f.astype(np.int32)).cuda(), gz, gb, gd, bs=bs, flags=opts).cpu().numpy()
    ref = oracle.backward(b.verts, b.faces, b.image_size, p2f, gz, gb, gd, nthreads=threads(), options=opts)
    compare_grad(gv, ref, f"opts {opts:#x} bs {bs}")


@pytest.mark.parametrize("opts", [PC | CL | CU, PC])
def test_options_reuse_and_autograd(opts):
    from paper_2007_08501_amd.raster import RasterSettings, rasterize_meshes
    b = small()
    H, W = b.image_size
    v, f, fi, nf = to_dev(b)
    out, ws = run_fwd(b, 16, options=opts)
    gz, gb, gd = [torch.from_numpy(x).cuda() for x in meshgen.upstream_grads(b)]
    reuse = run_bwd(b, out.pix_to_face, gz, gb, gd, bs=16, flags=opts | _lib.RAST_BWD_REUSE_FORWARD, ws=ws)
    fresh = run_bwd(b, out.pix_to_face, gz, gb, gd, bs=16, flags=opts)
    scale = float(fresh.abs().max())
    torch.testing.assert_close(reuse, fresh, rtol=0, atol=1e-5 * scale)
    # a reusing backward that names other options than the forward's is refused
    bad = run_bwd(b, out.pix_to_face, gz, gb, gd, bs=16, flags=(opts ^ CU) | _lib.RAST_BWD_REUSE_FORWARD, ws=ws,
                  check=False)
    assert _lib.rast_query_status(ws)[0] == _lib.RAST_EREUSE and (bad == 0).all()
    vv = v.clone().requires_grad_(True)
    s = RasterSettings((H, W), b.blur_radius, b.faces_per_pixel, bin_size=16, perspective_correct=bool(opts & PC),
                       clip_barycentric_coords=bool(opts & CL), cull_backfaces=bool(opts & CU))
    frags = rasterize_meshes(vv, f, fi, nf, s)
    assert torch.equal(frags.pix_to_face, out.pix_to_face)
    ((frags.zbuf * gz).sum() + (frags.bary * gb).sum() + (frags.dists * gd).sum()).backward()
    torch.testing.assert_close(vv.grad, fresh, rtol=0, atol=1e-5 * scale)
