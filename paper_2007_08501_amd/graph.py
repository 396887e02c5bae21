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
                 sched=_lib.RAST_SCHED_GRID, backward=True):
        dev = verts.device
        self.device = dev
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
                                  self.out.pix_to_face, self.out.zbuf, self.out.bary, self.out.dists, self.ws)
        if self.backward:
            # the backward reuses the forward's face records and bins in the same workspace
            _lib.rasterize_meshes_bwd(self.verts, self.faces, self.first_idx, self.num_faces, H, W, blur, K, bs, M,
                                      _lib.RAST_BWD_REUSE_FORWARD,
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
