"""PyTorch front end of the HIP point-cloud renderer (paper, Section 3.3).

    frags = rasterize_points(points, first_idx, num_points, settings)
    image = splat_composite(frags.idx, frags.dists, features, settings.radius)   # Alpha
    image = splat_composite(..., norm=True)                                       # Norm

rasterize_points is differentiable in ``points``; the compositing functions
in their opacities (or squared distances) and in ``features``.  Every
computation runs in librast.so; this module allocates outputs and marshals
arguments.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import NamedTuple, Optional, Tuple, Union

import torch

from . import _lib


@dataclass
class PointsRasterSettings:
    """image_size: int or (H, W).  radius: disc radius in NDC units.
    check: read the device status after the forward (synchronises) and raise
    on inconsistent cloud ranges."""

    image_size: Union[int, Tuple[int, int]]
    radius: float = 0.01
    points_per_pixel: int = 8
    check: bool = True

    @property
    def hw(self):
        if isinstance(self.image_size, int):
            return self.image_size, self.image_size
        return tuple(self.image_size)


class PointFragments(NamedTuple):
    idx: torch.Tensor    # (N,H,W,K) int32, -1 for empty slots
    zbuf: torch.Tensor   # (N,H,W,K) f32
    dists: torch.Tensor  # (N,H,W,K) f32, squared xy distance to the pixel centre


def _status_check(ws):
    st, _ = _lib.rast_query_status(ws)
    if st != _lib.RAST_OK:
        raise _lib.RastError("rasterize_points", st, _lib.status_string(st))


class _RasterizePoints(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, first_idx, num_points, H, W, radius, K, check):
        dev = points.device
        N = first_idx.shape[0]
        ws = _lib.alloc_workspace(_lib.rast_points_workspace_size(N, H, W, points.shape[0]), dev)
        idx = torch.empty((N, H, W, K), dtype=torch.int32, device=dev)
        zbuf = torch.empty((N, H, W, K), dtype=torch.float32, device=dev)
        dists = torch.empty_like(zbuf)
        _lib.rasterize_points_fwd(points, first_idx, num_points, H, W, radius, K, idx, zbuf, dists, ws)
        if check:
            _status_check(ws)
        ctx.save_for_backward(points, first_idx, num_points, idx)
        ctx.ws = ws
        ctx.args = (H, W, radius, K)
        ctx.mark_non_differentiable(idx)
        return idx, zbuf, dists

    @staticmethod
    def backward(ctx, _g_idx, g_zbuf, g_dists):
        points, first_idx, num_points, idx = ctx.saved_tensors
        H, W, radius, K = ctx.args
        gz = None if g_zbuf is None else g_zbuf.contiguous()
        gd = None if g_dists is None else g_dists.contiguous()
        grad = torch.empty_like(points)
        # the forward's workspace still holds the sorted points of this call
        _lib.rasterize_points_bwd(points, first_idx, num_points, H, W, radius, K, _lib.RAST_BWD_REUSE_FORWARD, idx,
                                  gz, gd, grad, ctx.ws)
        return grad, None, None, None, None, None, None, None


def rasterize_points(points: torch.Tensor, first_idx: torch.Tensor, num_points: torch.Tensor,
                     settings: PointsRasterSettings) -> PointFragments:
    """K nearest points along z per pixel for a packed heterogeneous batch:
    points (P,3) f32 on the device, first_idx / num_points (N,) int64."""
    H, W = settings.hw
    pts = points.contiguous()
    idx, zbuf, dists = _RasterizePoints.apply(pts, first_idx.contiguous(), num_points.contiguous(), int(H), int(W),
                                              float(settings.radius), int(settings.points_per_pixel),
                                              bool(settings.check))
    return PointFragments(idx, zbuf, dists)


class _Composite(torch.autograd.Function):
    @staticmethod
    def forward(ctx, idx, weights, features, mode, radius, num_points):
        D = features.shape[1] if features is not None else 1
        image = torch.empty(tuple(idx.shape[:-1]) + (D,), dtype=torch.float32, device=idx.device)
        _lib.points_composite_fwd(idx, weights, features, mode, radius, image, num_points)
        ctx.save_for_backward(idx, weights, features)
        ctx.mode = mode
        ctx.radius = radius
        ctx.num_points = num_points
        return image

    @staticmethod
    def backward(ctx, g_image):
        idx, weights, features = ctx.saved_tensors
        gw = torch.empty_like(weights)
        gf = torch.empty_like(features) if (features is not None and ctx.needs_input_grad[2]) else None
        _lib.points_composite_bwd(idx, weights, features, ctx.mode, ctx.radius, g_image.contiguous(), gw, gf,
                                  ctx.num_points)
        return None, gw, gf, None, None, None


def _composite(idx, weights, features, mode, radius, num_points):
    if features is None and num_points is None:
        raise ValueError("without features, give num_points (the ids must be below it)")
    f = None if features is None else features.contiguous()
    n = int(num_points) if num_points is not None else int(f.shape[0])
    return _Composite.apply(idx.contiguous(), weights.contiguous(), f, int(mode), float(radius), n)


def alpha_composite(idx: torch.Tensor, alphas: torch.Tensor, features: Optional[torch.Tensor] = None,
                    num_points: Optional[int] = None) -> torch.Tensor:
    """sum_k alpha_k prod_{j<k} (1 - alpha_j) f_{idx_k}: idx/alphas (...,K), features (P,D) -> (...,D).
    features None: every feature is 1 (a silhouette, (...,1)); num_points then bounds the ids."""
    return _composite(idx, alphas, features, _lib.RAST_COMPOSITE_ALPHA, 0.0, num_points)


def norm_composite(idx: torch.Tensor, alphas: torch.Tensor, features: Optional[torch.Tensor] = None,
                   num_points: Optional[int] = None) -> torch.Tensor:
    """sum_k alpha_k f_{idx_k} / sum_k alpha_k (0 where the sum is <= 0)."""
    return _composite(idx, alphas, features, _lib.RAST_COMPOSITE_NORM, 0.0, num_points)


def splat_composite(idx: torch.Tensor, dists: torch.Tensor, features: Optional[torch.Tensor], radius: float,
                    norm: bool = False, num_points: Optional[int] = None) -> torch.Tensor:
    """Compositing of splats whose opacity falls from 1 at the point to 0 at
    the disc's rim, alpha = 1 - d / radius^2, formed inside the kernel from
    the rasterizer's squared distances d (differentiable in dists).  features
    None: a silhouette (every feature 1)."""
    mode = (_lib.RAST_COMPOSITE_NORM if norm else _lib.RAST_COMPOSITE_ALPHA) | _lib.RAST_COMPOSITE_FROM_DISTS
    return _composite(idx, dists, features, mode, radius, num_points)
