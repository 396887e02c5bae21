"""hipGraph capture of a whole forward+backward rasterization step.

The runner owns static device buffers (vertex positions, fragments, upstream
gradients, vertex gradients and one workspace, whose face records and bins the
backward reuses from the forward), captures one forward and one backward call
of the C ABI into a HIP graph through torch.cuda.graph, and replays it.  Inputs are updated in place with ``set_verts`` / ``set_grads``
between replays; the device status (bin overflow) is read after a replay,
never inside the graph.  Every kernel in the captured calls clears its
counters with a fill kernel, so a replay needs no memset node.
"""
from __future__ import annotations

import torch

from . import _lib
from .raster import empty_fragments


class GraphRunner:
    def __init__(self, verts, faces, first_idx, num_faces, H, W, blur, K, bin_size, max_faces_per_bin,
                 sched=_lib.RAST_SCHED_GRID, backward=True, options=0):
        dev = verts.device
        self.device = dev
        self.options = int(options)
        self.dims = (first_idx.shape[0], H, W, K)
        self.args = (float(blur), int(bin_size), int(max_faces_per_bin or 0), int(sched))
        self.verts = verts.detach().clone().contiguous()
        self.faces = faces.to(torch.int32).contiguous()
        self.first_idx = first_idx.contiguous()
        self.num_faces = num_faces.contiguous()
        N = self.dims[0]
        self.out = empty_fragments(N, H, W, K, dev)
        self.ws = torch.empty(_lib.rast_workspace_size(N, H, W, self.faces.shape[0], bin_size, max_faces_per_bin),
                              dtype=torch.uint8, device=dev)
        self.backward = backward
        if backward:
            self.grad_zbuf = torch.zeros((N, H, W, K), device=dev)
            self.grad_bary = torch.zeros((N, H, W, K, 3), device=dev)
            self.grad_dists = torch.zeros((N, H, W, K), device=dev)
            self.grad_verts = torch.empty_like(self.verts)
        self.graph = None

    def set_verts(self, verts):
        self.verts.copy_(verts)

    def set_grads(self, gz, gb, gd):
        self.grad_zbuf.copy_(gz)
        self.grad_bary.copy_(gb)
        self.grad_dists.copy_(gd)

    def step_eager(self):
        N, H, W, K = self.dims
        blur, bs, M, sched = self.args
        _lib.rasterize_meshes_fwd(self.verts, self.faces, self.first_idx, self.num_faces, H, W, blur, K, bs, M, sched,
                                  self.out.pix_to_face, self.out.zbuf, self.out.bary, self.out.dists, self.ws,
                                  self.options)
        if self.backward:
            # the backward reuses the forward's face records and bins in the same workspace
            _lib.rasterize_meshes_bwd(self.verts, self.faces, self.first_idx, self.num_faces, H, W, blur, K, bs, M,
                                      _lib.RAST_BWD_REUSE_FORWARD | self.options,
                                      self.out.pix_to_face, self.grad_zbuf, self.grad_bary, self.grad_dists,
                                      self.grad_verts, self.ws)

    def capture(self, warmup: int = 2):
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step_eager()
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step_eager()
        torch.cuda.synchronize(self.device)
        return self

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def status(self):
        """(status, max_bin_count) of the last forward; synchronises."""
        return _lib.rast_query_status(self.ws)


class PointsGraphRunner:
    """hipGraph of one point-cloud render step: rasterize, composite the
    splats (Alpha or Norm, opacity 1 - d / r^2), composite backward, rasterize
    backward reusing the forward's sorted points.  Static buffers as for
    GraphRunner; ``features`` (P,D) and the upstream image gradient are set
    with ``set_features`` / ``set_grad_image``; ``silhouette`` renders with
    every feature 1 and no feature table."""

    def __init__(self, points, first_idx, num_points, H, W, radius, K, D=1, norm=False, feature_grad=False,
                 silhouette=False):
        dev = points.device
        self.device = dev
        N, P = first_idx.shape[0], points.shape[0]
        self.dims = (N, H, W, K, D)
        self.radius = float(radius)
        self.mode = ((_lib.RAST_COMPOSITE_NORM if norm else _lib.RAST_COMPOSITE_ALPHA)
                     | _lib.RAST_COMPOSITE_FROM_DISTS)
        self.points = points.detach().clone().contiguous()
        self.first_idx = first_idx.contiguous()
        self.num_points = num_points.contiguous()
        self.idx = torch.empty((N, H, W, K), dtype=torch.int32, device=dev)
        self.zbuf = torch.empty((N, H, W, K), dtype=torch.float32, device=dev)
        self.dists = torch.empty_like(self.zbuf)
        # silhouette: no feature table, every feature is 1
        self.features = None if silhouette else torch.ones((P, D), dtype=torch.float32, device=dev)
        self.image = torch.empty((N, H, W, 1 if silhouette else D), dtype=torch.float32, device=dev)
        self.grad_image = torch.zeros_like(self.image)
        self.grad_dists = torch.empty_like(self.zbuf)
        self.grad_features = torch.empty_like(self.features) if (feature_grad and not silhouette) else None
        self.grad_points = torch.empty_like(self.points)
        self.ws = torch.empty(_lib.rast_points_workspace_size(N, H, W, P), dtype=torch.uint8, device=dev)
        self.graph = None

    def set_features(self, f):
        self.features.copy_(f)

    def set_grad_image(self, g):
        self.grad_image.copy_(g)

    def forward_eager(self):
        N, H, W, K, D = self.dims
        _lib.rasterize_points_fwd(self.points, self.first_idx, self.num_points, H, W, self.radius, K, self.idx,
                                  self.zbuf, self.dists, self.ws)
        _lib.points_composite_fwd(self.idx, self.dists, self.features, self.mode, self.radius, self.image,
                                  self.points.shape[0])

    def backward_eager(self):
        N, H, W, K, D = self.dims
        _lib.points_composite_bwd(self.idx, self.dists, self.features, self.mode, self.radius, self.grad_image,
                                  self.grad_dists, self.grad_features, self.points.shape[0])
        _lib.rasterize_points_bwd(self.points, self.first_idx, self.num_points, H, W, self.radius, K,
                                  _lib.RAST_BWD_REUSE_FORWARD, self.idx, None, self.grad_dists, self.grad_points,
                                  self.ws)

    def step_eager(self):
        self.forward_eager()
        self.backward_eager()

    def capture(self, warmup: int = 2):
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step_eager()
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.step_eager()
        torch.cuda.synchronize(self.device)
        return self

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def status(self):
        return _lib.rast_query_status(self.ws)
