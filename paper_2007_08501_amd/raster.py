"""PyTorch front end of the HIP rasterizer: autograd Functions over the C ABI.

    frags = rasterize_meshes(verts, faces, first_idx, num_faces, settings)
    alpha = silhouette_blend(frags.pix_to_face, frags.dists, sigma)

PyTorch provides device memory and the stream; every computation runs in
librast.so.  Differentiable in ``verts`` (rasterizer) and ``dists`` (blend).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import NamedTuple, Optional, Tuple, Union

import torch

from . import _lib


@dataclass
class RasterSettings:
    """image_size: int or (H, W).  blur_radius: squared NDC distance.
    bin_size: 0 = single pass over every face of the mesh; a multiple of 8 =
    two passes with bins of that many pixels; None = pick with the autotuner.
    max_faces_per_bin: None = exact value from a counting pass.
    sched: 0 = grid launch, 1 = persistent most-loaded-first scheduler.
    check: read the device status after the forward (synchronises) and
    recover from a bin overflow by recounting when max_faces_per_bin is None.
    perspective_correct / clip_barycentric_coords / cull_backfaces: the
    rasterizer options (see RAST_PERSPECTIVE_CORRECT etc. in rast.h).
    """

    image_size: Union[int, Tuple[int, int]]
    blur_radius: float = 0.0
    faces_per_pixel: int = 1
    bin_size: Optional[int] = None
    max_faces_per_bin: Optional[int] = None
    sched: int = _lib.RAST_SCHED_GRID
    check: bool = True
    perspective_correct: bool = False
    clip_barycentric_coords: bool = False
    cull_backfaces: bool = False

    @property
    def options(self) -> int:
        return ((_lib.RAST_PERSPECTIVE_CORRECT if self.perspective_correct else 0)
                | (_lib.RAST_CLIP_BARYCENTRIC if self.clip_barycentric_coords else 0)
                | (_lib.RAST_CULL_BACKFACES if self.cull_backfaces else 0))

    @property
    def hw(self):
        if isinstance(self.image_size, int):
            return self.image_size, self.image_size
        return tuple(self.image_size)


class Fragments(NamedTuple):
    pix_to_face: torch.Tensor  # (N,H,W,K) int32
    zbuf: torch.Tensor         # (N,H,W,K) f32
    bary: torch.Tensor         # (N,H,W,K,3) f32
    dists: torch.Tensor        # (N,H,W,K) f32


class BinOverflow(RuntimeError):
    pass


_ws = {}


def workspace(device, nbytes: int) -> torch.Tensor:
    """A per-device scratch buffer of at least nbytes (grown on demand)."""
    key = torch.device(device).index
    t = _ws.get(key)
    if t is None or t.numel() < nbytes:
        t = _lib.alloc_workspace(int(nbytes * 1.25) + 4096, device)
        _ws[key] = t
    return t


def count_max_faces_per_bin(verts, faces, first_idx, num_faces, H, W, blur_radius, bin_size) -> int:
    """Largest bin count for this bin size (runs the counting pass; synchronises)."""
    N = first_idx.shape[0]
    ws = workspace(verts.device, _lib.rast_workspace_size(N, H, W, faces.shape[0], bin_size, 1))
    _lib.rast_bin_count(verts, faces, first_idx, num_faces, H, W, blur_radius, bin_size, ws)
    st, mx = _lib.rast_query_status(ws)
    if st != _lib.RAST_OK:
        raise _lib.RastError("rast_bin_count", st, _lib.status_string(st))
    return mx


def round_up(x: int, m: int) -> int:
    return max(m, (x + m - 1) // m * m)


def forward_into(verts, faces, first_idx, num_faces, H, W, blur_radius, K, bin_size, M, sched, out, ws, options=0):
    """Raw forward into preallocated outputs (no status read)."""
    _lib.rasterize_meshes_fwd(verts, faces, first_idx, num_faces, H, W, blur_radius, K, bin_size, M, sched,
                              out.pix_to_face, out.zbuf, out.bary, out.dists, ws, options)


def empty_fragments(N, H, W, K, device) -> Fragments:
    return Fragments(
        torch.empty((N, H, W, K), dtype=torch.int32, device=device),
        torch.empty((N, H, W, K), dtype=torch.float32, device=device),
        torch.empty((N, H, W, K, 3), dtype=torch.float32, device=device),
        torch.empty((N, H, W, K), dtype=torch.float32, device=device),
    )


class _RasterizeMeshes(torch.autograd.Function):
    @staticmethod
    def forward(ctx, verts, faces, first_idx, num_faces, H, W, blur, K, bs, M, sched, check, options):
        N = first_idx.shape[0]
        out = empty_fragments(N, H, W, K, verts.device)
        vd = verts.detach().contiguous()
        # a workspace of this call's own: its backward reuses the face records and bins
        ws = _lib.alloc_workspace(_lib.rast_workspace_size(N, H, W, faces.shape[0], bs, M), verts.device)
        forward_into(vd, faces, first_idx, num_faces, H, W, blur, K, bs, M, sched, out, ws, options)
        if check:
            st, mx = _lib.rast_query_status(ws)
            if st == _lib.RAST_EOVERFLOW:
                raise BinOverflow(f"a bin received {mx} faces > max_faces_per_bin={M}")
            if st != _lib.RAST_OK:
                raise _lib.RastError("rasterize_meshes_fwd", st, _lib.status_string(st))
        ctx.save_for_backward(vd, faces, first_idx, num_faces, out.pix_to_face)
        ctx.mark_non_differentiable(out.pix_to_face)
        ctx.dims = (N, H, W, K)
        ctx.blur = blur
        ctx.bins = (bs, M)
        ctx.options = options
        ctx.ws = ws
        return out.pix_to_face, out.zbuf, out.bary, out.dists

    @staticmethod
    def backward(ctx, _g_p2f, g_zbuf, g_bary, g_dists):
        verts, faces, first_idx, num_faces, p2f = ctx.saved_tensors
        N, H, W, K = ctx.dims

        def prep(g):
            return None if g is None else g.contiguous().to(torch.float32)

        grad_verts = torch.empty_like(verts)
        bs, M = ctx.bins
        # the saved vertices cannot have changed (autograd checks their version),
        # so the forward's face records and bins are still valid
        _lib.rasterize_meshes_bwd(verts, faces, first_idx, num_faces, H, W, ctx.blur, K, bs, M,
                                  _lib.RAST_BWD_REUSE_FORWARD | ctx.options, p2f, prep(g_zbuf), prep(g_bary),
                                  prep(g_dists), grad_verts, ctx.ws)
        ctx.ws = None
        return (grad_verts,) + (None,) * 12


def rasterize_meshes(verts, faces, first_idx, num_faces, settings: RasterSettings) -> Fragments:
    """Fragments of the K nearest faces per pixel for a packed mesh batch.

    verts (V,3) f32 device tensor (may require grad); faces (F,3) int32;
    first_idx/num_faces (N,) int64 on the same device.
    """
    H, W = settings.hw
    K = int(settings.faces_per_pixel)
    bs = settings.bin_size
    M = settings.max_faces_per_bin
    if faces.dtype != torch.int32:
        faces = faces.to(torch.int32)
    faces = faces.contiguous()
    if bs is None:
        from .autotune import autotune
        choice = autotune(verts.detach(), faces, first_idx, num_faces, H, W, settings.blur_radius, K)
        bs, M, sched = choice.bin_size, choice.max_faces_per_bin, choice.sched
    else:
        sched = settings.sched
    # a capacity the caller did not fix is recounted when a bin overflows (the
    # autotuner's comes from a cache keyed on the batch's statistics, not on
    # these vertices)
    auto_M = bs > 0 and settings.max_faces_per_bin is None
    if bs > 0 and M is None:
        M = round_up(count_max_faces_per_bin(verts.detach(), faces, first_idx, num_faces, H, W,
                                             settings.blur_radius, bs), 32)
    try:
        res = _RasterizeMeshes.apply(verts, faces, first_idx, num_faces, H, W, float(settings.blur_radius), K,
                                     int(bs), int(M or 0), int(sched), bool(settings.check), settings.options)
    except BinOverflow:
        if not auto_M:
            raise
        M = round_up(count_max_faces_per_bin(verts.detach(), faces, first_idx, num_faces, H, W,
                                             settings.blur_radius, bs), 32)
        res = _RasterizeMeshes.apply(verts, faces, first_idx, num_faces, H, W, float(settings.blur_radius), K,
                                     int(bs), int(M), int(sched), bool(settings.check), settings.options)
    return Fragments(*res)


class _SilhouetteBlend(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pix_to_face, dists, sigma):
        d = dists.detach().contiguous()
        alpha = torch.empty(d.shape[:-1], dtype=torch.float32, device=d.device)
        _lib.silhouette_blend_fwd(pix_to_face, d, sigma, alpha)
        ctx.save_for_backward(pix_to_face, d)
        ctx.sigma = sigma
        return alpha

    @staticmethod
    def backward(ctx, grad_alpha):
        p2f, d = ctx.saved_tensors
        gd = torch.empty_like(d)
        _lib.silhouette_blend_bwd(p2f, d, grad_alpha.contiguous().to(torch.float32), ctx.sigma, gd)
        return None, gd, None


def silhouette_blend(pix_to_face, dists, sigma: float):
    """Algorithm 1 of the paper: alpha = 1 - prod_k (1 - sigmoid(-dists_k / sigma)),
    with empty slots (pix_to_face == -1) left out.  Differentiable in dists."""
    return _SilhouetteBlend.apply(pix_to_face.contiguous(), dists, float(sigma))


class _SoftmaxBlend(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pix_to_face, zbuf, dists, colors, sigma, gamma, znear, zfar):
        z = zbuf.detach().contiguous()
        d = dists.detach().contiguous()
        c = colors.detach().contiguous().to(torch.float32)
        img = torch.empty(d.shape[:-1] + (c.shape[-1],), dtype=torch.float32, device=d.device)
        _lib.softmax_blend_fwd(pix_to_face, z, d, c, sigma, gamma, znear, zfar, img)
        ctx.save_for_backward(pix_to_face, z, d, c)
        ctx.params = (sigma, gamma, znear, zfar)
        return img

    @staticmethod
    def backward(ctx, grad_image):
        p2f, z, d, c = ctx.saved_tensors
        need_z, need_d, need_c = ctx.needs_input_grad[1:4]
        gz = torch.empty_like(z) if need_z else None
        gd = torch.empty_like(d) if need_d else None
        gc = torch.empty_like(c) if need_c else None
        _lib.softmax_blend_bwd(p2f, z, d, c, *ctx.params, grad_image.contiguous().to(torch.float32), gz, gd, gc)
        return None, gz, gd, gc, None, None, None, None


def softmax_blend(pix_to_face, zbuf, dists, colors, sigma: float, gamma: float, znear: float, zfar: float):
    """Algorithm 2 of the paper: image = sum_k w_k colors_k / sum_k w_k with
    w_k = sigmoid(-dists_k / sigma) exp((zinv_k - max zinv) / gamma),
    zinv = (zfar - zbuf) / (zfar - znear); empty slots are left out.
    colors (..., K, C) with C <= 8.  Differentiable in zbuf, dists and colors."""
    return _SoftmaxBlend.apply(pix_to_face.contiguous(), zbuf, dists, colors, float(sigma), float(gamma), float(znear),
                               float(zfar))
