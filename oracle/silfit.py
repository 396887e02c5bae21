"""FP64 oracle of the silhouette-fitting loss and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss of the mesh-fitting experiment: per-vertex offsets o (V,3) move a
template mesh; view v renders the vertices R_v (base + o), with x and y
scaled by s and z shifted by dz, into an H x H image; the K nearest faces
per pixel (paper, Section 3.2) give signed distances, the silhouette blend
(Algorithm 1) gives alpha, and the loss is the mean over views of
1 - IoU(alpha_v, target_v) (Appendix B).

The gradient with respect to o holds the face selection fixed: the selection
is piecewise constant in o, and the gradient is that of the frozen-selection
map (oracle.fragments_fixed), chained through the blend, the IoU and the
view transform:
    dL/dalpha_v = -(T_v U_v - I_v (1 - T_v)) / (U_v^2 n_views),
    with I_v = sum alpha T, U_v = sum (alpha + T - alpha T);
    dL/do = sum_v R_v^T diag(s, s, 1) dL/dverts_v.
"""
from __future__ import annotations

import numpy as np

from . import backward, fragments_fixed, rasterize
from .blend import iou_loss, silhouette_blend, silhouette_blend_backward


def view_vertices(base, rotations, offsets, ndc_scale, dz):
    """(n_views, V, 3) FP64 vertices of each view."""
    u = np.asarray(base, np.float64) + np.asarray(offsets, np.float64)
    out = np.stack([u @ np.asarray(R, np.float64).T for R in rotations])
    out[..., :2] *= ndc_scale
    out[..., 2] += dz
    return out


def pack_views(view_verts, faces):
    """Packed (n*V,3) vertices, (n*F,3) faces with global vertex ids, mesh ranges."""
    n, V, _ = view_verts.shape
    f = np.asarray(faces, np.int64)
    F = f.shape[0]
    verts = view_verts.reshape(n * V, 3)
    faces_p = np.concatenate([f + v * V for v in range(n)])
    first = np.arange(n, dtype=np.int64) * F
    nf = np.full(n, F, dtype=np.int64)
    return verts, faces_p, first, nf


def iou_loss_grad(alpha, target):
    """d(mean_v (1 - IoU_v)) / d alpha, FP64 (n,H,W)."""
    S = np.asarray(alpha, np.float64)
    T = np.asarray(target, np.float64)
    n = S.shape[0]
    I = (S * T).reshape(n, -1).sum(1)[:, None, None]
    U = (S + T - S * T).reshape(n, -1).sum(1)[:, None, None]
    return -(T * U - I * (1.0 - T)) / (U * U) / n


def loss_and_grad(base, rotations, faces, offsets, target, image_size, K, blur, sigma, ndc_scale=0.8, dz=2.0,
                  nthreads=None):
    """(loss, dloss/doffsets (V,3), selection p2f) at the given offsets."""
    vv = view_vertices(base, rotations, offsets, ndc_scale, dz)
    verts, faces_p, first, nf = pack_views(vv, faces)
    # the vertices the rasterizer sees are FP32
    verts32 = verts.astype(np.float32)
    o = rasterize(verts32, faces_p, first, nf, (image_size, image_size), blur, K, nthreads=nthreads)
    alpha = silhouette_blend(o["p2f"], o["dists"], sigma)
    loss = iou_loss(alpha, target)
    g_alpha = iou_loss_grad(alpha, target)
    g_d = silhouette_blend_backward(o["p2f"], o["dists"], sigma, g_alpha)
    g_verts = backward(verts32, faces_p, (image_size, image_size), o["p2f"], grad_dists=g_d, nthreads=nthreads)
    n, V = vv.shape[:2]
    g_view = g_verts.reshape(n, V, 3).copy()
    g_view[..., :2] *= ndc_scale
    g_off = np.zeros((V, 3))
    for v in range(n):
        g_off += g_view[v] @ np.asarray(rotations[v], np.float64)
    return loss, g_off, o["p2f"]


def frozen_loss(base, rotations, faces, offsets, target, image_size, p2f, sigma, ndc_scale=0.8, dz=2.0,
                nthreads=None):
    """The loss with the face selection p2f held fixed (FP64 throughout)."""
    vv = view_vertices(base, rotations, offsets, ndc_scale, dz)
    verts, faces_p, _, _ = pack_views(vv, faces)
    _, _, dists, _ = fragments_fixed(verts, faces_p, (image_size, image_size), p2f, nthreads=nthreads)
    return iou_loss(silhouette_blend(p2f, dists, sigma), target)


def target_silhouettes(target_verts, rotations, faces, image_size, K, blur, sigma, ndc_scale=0.8, dz=2.0,
                       nthreads=None):
    """alpha of the target shape in every view (the fit's goal)."""
    vv = view_vertices(target_verts, rotations, np.zeros_like(target_verts), ndc_scale, dz)
    verts, faces_p, first, nf = pack_views(vv, faces)
    o = rasterize(verts.astype(np.float32), faces_p, first, nf, (image_size, image_size), blur, K,
                  nthreads=nthreads)
    return silhouette_blend(o["p2f"], o["dists"], sigma)
