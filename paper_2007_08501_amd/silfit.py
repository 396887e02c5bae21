"""Differentiable silhouette fitting on the GPU rasterizer.

The mesh-fitting experiment of the paper (Section 3.2 Algorithm 1 for the
soft silhouette, Appendix B for the IoU loss): per-vertex offsets of a
template mesh are optimised with Adam so that the soft silhouettes of the
offset mesh, seen from several views in one packed batch, match those of a
target shape.  Every view of one step is one rasterizer launch (the views
are the meshes of a packed batch); the blend is the library's kernel; the
view transform, the IoU loss and Adam are a handful of torch elementwise
operations.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import meshgen
from .raster import RasterSettings, rasterize_meshes, silhouette_blend


def iou_loss(alpha: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean over views of 1 - sum(S T) / sum(S + T - S T); alpha/target (n,H,W)."""
    n = alpha.shape[0]
    inter = (alpha * target).reshape(n, -1).sum(1)
    union = (alpha + target - alpha * target).reshape(n, -1).sum(1)
    return (1.0 - inter / union).mean()


@dataclass
class FitResult:
    losses: List[float] = field(default_factory=list)
    offsets: Optional[torch.Tensor] = None
    grad0: Optional[torch.Tensor] = None


class SilhouetteFit:
    """The fitting problem on one device: template, views, target silhouettes."""

    def __init__(self, problem: meshgen.SilhouetteFitProblem, image_size: int = 128, faces_per_pixel: int = 50,
                 blur_radius: float = meshgen.SIL_BLUR, sigma: float = meshgen.SIL_SIGMA,
                 bin_size: Optional[int] = None, device="cuda"):
        self.problem = problem
        self.device = torch.device(device)
        self.n = problem.n_views
        self.sigma = float(sigma)
        self.settings = RasterSettings(image_size=image_size, blur_radius=float(np.float32(blur_radius)),
                                       faces_per_pixel=faces_per_pixel, bin_size=bin_size)
        dev = self.device
        self.base = torch.from_numpy(problem.base.astype(np.float32)).to(dev)
        self.rot = torch.from_numpy(problem.rotations.astype(np.float32)).to(dev)
        V = problem.base.shape[0]
        f = problem.faces.astype(np.int64)
        F = f.shape[0]
        self.faces = torch.from_numpy(np.concatenate([f + v * V for v in range(self.n)]).astype(np.int32)).to(dev)
        self.first_idx = torch.arange(self.n, dtype=torch.int64, device=dev) * F
        self.num_faces = torch.full((self.n,), F, dtype=torch.int64, device=dev)
        self.scale = torch.tensor([problem.ndc_scale, problem.ndc_scale, 1.0], device=dev)
        self.shift = torch.tensor([0.0, 0.0, problem.dz], device=dev)
        with torch.no_grad():
            tgt = torch.from_numpy(problem.target.astype(np.float32)).to(dev)
            self.target = self.render(self.view_verts(tgt, torch.zeros_like(tgt)))

    def view_verts(self, base: torch.Tensor, offsets: torch.Tensor) -> torch.Tensor:
        """Packed (n*V, 3) view-space vertices of base + offsets."""
        u = base + offsets                                   # (V,3)
        vv = torch.matmul(self.rot, u.t().contiguous())      # (n,3,V)
        vv = vv.transpose(1, 2) * self.scale + self.shift    # (n,V,3)
        return vv.reshape(-1, 3).contiguous()

    def render(self, verts: torch.Tensor) -> torch.Tensor:
        frags = rasterize_meshes(verts, self.faces, self.first_idx, self.num_faces, self.settings)
        return silhouette_blend(frags.pix_to_face, frags.dists, self.sigma)

    def loss(self, offsets: torch.Tensor) -> torch.Tensor:
        return iou_loss(self.render(self.view_verts(self.base, offsets)), self.target)

    def run(self, steps: int = 50, lr: float = 1e-3) -> FitResult:
        offsets = torch.zeros_like(self.base, requires_grad=True)
        opt = torch.optim.Adam([offsets], lr=lr)
        res = FitResult()
        for it in range(steps):
            opt.zero_grad(set_to_none=True)
            loss = self.loss(offsets)
            loss.backward()
            if it == 0:
                res.grad0 = offsets.grad.detach().clone()
            res.losses.append(float(loss.detach()))
            opt.step()
        res.offsets = offsets.detach()
        return res
