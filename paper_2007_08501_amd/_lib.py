"""ctypes binding of librast.so (the C ABI in include/rast.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
library.  There is no fallback of any kind -- if the library is missing or
cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAST_LIB_PATH names another build of the same sources (the sanitized host
# build of the CPU checks); by default the in-tree librast.so
LIB_PATH = os.environ.get("RAST_LIB_PATH") or os.path.join(_HERE, "librast.so")

RAST_OK = 0
RAST_EINVAL = -1
RAST_EWORKSPACE = -2
RAST_EHIP = -3
RAST_EOVERFLOW = -4
RAST_EMESH = -5
RAST_EREUSE = -6
RAST_ESCRATCH = -7
RAST_STATIC_SCRATCH_BYTES = 64 << 20
RAST_BWD_REUSE_FORWARD = 1
RAST_KMAX = 64
RAST_TILE = 8
RAST_MAX_BIN = 512
RAST_SCHED_GRID = 0
RAST_SCHED_PERSISTENT = 1
RAST_PERSPECTIVE_CORRECT = 0x100
RAST_CLIP_BARYCENTRIC = 0x200
RAST_CULL_BACKFACES = 0x400

_lock = threading.Lock()
_lib = None


class RastError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn}: {msg} (status {code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing; build it with "
                               "`python -m paper_2007_08501_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        cf = ctypes.c_float
        sz = ctypes.c_size_t
        L.rast_workspace_size.argtypes = [ci, ci, ci, i64, ci, ci, ctypes.POINTER(sz)]
        L.rasterize_meshes_fwd.argtypes = [P, i64, P, i64, P, P, ci, ci, ci, cf, ci, ci, ci, ci, ci, P, P, P, P, P, sz, P]
        L.rasterize_meshes_fwd_static.argtypes = [P, i64, P, i64, P, P, ci, ci, ci, cf, ci, ci, ci, ci, ci, P, P, P, P,
                                                  P, P]
        L.rasterize_meshes_bwd.argtypes = [P, i64, P, i64, P, P, ci, ci, ci, cf, ci, ci, ci, ci, P, P, P, P, P, P, sz, P]
        L.rast_bin_count.argtypes = [P, i64, P, i64, P, P, ci, ci, ci, cf, ci, P, sz, P]
        L.rast_query_status.argtypes = [P, ctypes.POINTER(ci), ctypes.POINTER(ci), P]
        L.rast_status_string.argtypes = [ci]
        L.rast_status_string.restype = ctypes.c_char_p
        L.rast_set_kernel_events.argtypes = [ci, P, P]
        L.silhouette_blend_fwd.argtypes = [P, P, i64, ci, cf, P, P]
        L.silhouette_blend_bwd.argtypes = [P, P, P, i64, ci, cf, P, P]
        L.softmax_blend_fwd.argtypes = [P, P, P, P, i64, ci, ci, cf, cf, cf, cf, P, P]
        L.softmax_blend_bwd.argtypes = [P, P, P, P, i64, ci, ci, cf, cf, cf, cf, P, P, P, P, P]
        L.rast_points_workspace_size.argtypes = [ci, ci, ci, i64, ctypes.POINTER(sz)]
        L.rasterize_points_fwd.argtypes = [P, i64, P, P, ci, ci, ci, cf, ci, P, P, P, P, sz, P]
        L.rasterize_points_bwd.argtypes = [P, i64, P, P, ci, ci, ci, cf, ci, ci, P, P, P, P, P, sz, P]
        L.points_composite_fwd.argtypes = [P, P, P, i64, i64, ci, ci, ci, cf, P, P]
        L.points_composite_bwd.argtypes = [P, P, P, i64, i64, ci, ci, ci, cf, P, P, P, P]
        for fn in ("rast_workspace_size", "rasterize_meshes_fwd", "rasterize_meshes_fwd_static", "rasterize_meshes_bwd",
                   "rast_bin_count",
                   "rast_query_status", "silhouette_blend_fwd", "silhouette_blend_bwd", "rast_set_kernel_events",
                   "softmax_blend_fwd", "softmax_blend_bwd", "rast_points_workspace_size", "rasterize_points_fwd",
                   "rasterize_points_bwd", "points_composite_fwd", "points_composite_bwd"):
            getattr(L, fn).restype = ci
        _lib = L
        return L


EXPORTS = ("rast_workspace_size", "rasterize_meshes_fwd", "rasterize_meshes_fwd_static", "rasterize_meshes_bwd",
           "rast_bin_count",
           "rast_query_status", "rast_status_string", "silhouette_blend_fwd", "silhouette_blend_bwd",
           "rast_set_kernel_events", "softmax_blend_fwd", "softmax_blend_bwd", "rast_points_workspace_size",
           "rasterize_points_fwd", "rasterize_points_bwd", "points_composite_fwd", "points_composite_bwd")
RAST_KERNEL_FINE = 0
RAST_KERNEL_BWD = 1
RAST_KERNEL_POINTS_FINE = 2
RAST_KERNEL_POINTS_BWD = 3
RAST_POINTS_MAX = 1 << 30
RAST_POINTS_MAX_SIDE = 16384
RAST_POINTS_MAX_RADIUS = 2.0
RAST_COMPOSITE_ALPHA = 0
RAST_COMPOSITE_NORM = 1
RAST_COMPOSITE_FROM_DISTS = 2
RAST_COMPOSITE_DMAX = 8


def status_string(code: int) -> str:
    return lib().rast_status_string(int(code)).decode()


def _check(fn: str, rc: int):
    if rc != RAST_OK:
        raise RastError(fn, rc, status_string(rc))


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require(t, name, dtype, device=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def rast_workspace_size(N, H, W, F, bin_size, max_faces_per_bin) -> int:
    out = ctypes.c_size_t(0)
    _check("rast_workspace_size",
           lib().rast_workspace_size(int(N), int(H), int(W), int(F), int(bin_size), int(max_faces_per_bin or 0),
                                     ctypes.byref(out)))
    return int(out.value)


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    """Device bytes for a workspace (torch allocations are 256-byte aligned)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _mesh_shapes(verts, faces, first_idx, num_faces):
    """Shapes of the packed mesh inputs; returns N."""
    if verts.dim() != 2 or verts.shape[1] != 3:
        raise ValueError(f"verts must be (V,3), got {tuple(verts.shape)}")
    if faces.dim() != 2 or faces.shape[1] != 3:
        raise ValueError(f"faces must be (F,3), got {tuple(faces.shape)}")
    if first_idx.dim() != 1 or tuple(num_faces.shape) != tuple(first_idx.shape):
        raise ValueError("mesh_to_face_first_idx and num_faces_per_mesh must be (N,) each")
    return first_idx.shape[0]


def rasterize_meshes_fwd(verts, faces, first_idx, num_faces, H, W, blur_radius, K, bin_size, max_faces_per_bin,
                         sched, pix_to_face, zbuf, bary, dists, workspace, options=0):
    dev = verts.device
    _require(verts, "verts", torch.float32, dev)
    _require(faces, "faces", torch.int32, dev)
    _require(first_idx, "mesh_to_face_first_idx", torch.int64, dev)
    _require(num_faces, "num_faces_per_mesh", torch.int64, dev)
    for t, n, d in ((pix_to_face, "pix_to_face", torch.int32), (zbuf, "zbuf", torch.float32),
                    (bary, "bary", torch.float32), (dists, "dists", torch.float32), (workspace, "workspace", torch.uint8)):
        _require(t, n, d, dev)
    N = _mesh_shapes(verts, faces, first_idx, num_faces)
    shp = (N, int(H), int(W), int(K))
    _same_shape("N,H,W,K", shp, (pix_to_face, "pix_to_face"), (zbuf, "zbuf"), (dists, "dists"))
    _same_shape("N,H,W,K", shp + (3,), (bary, "bary"))
    rc = lib().rasterize_meshes_fwd(_p(verts), verts.shape[0], _p(faces), faces.shape[0], _p(first_idx),
                                    _p(num_faces), int(N), int(H), int(W), float(blur_radius), int(K), int(bin_size),
                                    int(max_faces_per_bin or 0), int(sched), int(options), _p(pix_to_face), _p(zbuf),
                                    _p(bary), _p(dists), _p(workspace), workspace.numel(), _stream(dev))
    _check("rasterize_meshes_fwd", rc)


def rasterize_meshes_fwd_static(verts, faces, first_idx, num_faces, H, W, blur_radius, K, bin_size,
                                max_faces_per_bin, sched, pix_to_face, zbuf, bary, dists, status_out, options=0):
    """The forward on the library's static scratch (no workspace argument);
    status_out: int32 device tensor of 2 (device status, largest bin count) or None."""
    dev = verts.device
    _require(verts, "verts", torch.float32, dev)
    _require(faces, "faces", torch.int32, dev)
    _require(first_idx, "mesh_to_face_first_idx", torch.int64, dev)
    _require(num_faces, "num_faces_per_mesh", torch.int64, dev)
    for t, n, d in ((pix_to_face, "pix_to_face", torch.int32), (zbuf, "zbuf", torch.float32),
                    (bary, "bary", torch.float32), (dists, "dists", torch.float32),
                    (status_out, "status_out", torch.int32)):
        _require(t, n, d, dev)
    if status_out is not None and status_out.numel() < 2:
        raise ValueError("status_out must hold 2 int32")
    N = _mesh_shapes(verts, faces, first_idx, num_faces)
    shp = (N, int(H), int(W), int(K))
    _same_shape("N,H,W,K", shp, (pix_to_face, "pix_to_face"), (zbuf, "zbuf"), (dists, "dists"))
    _same_shape("N,H,W,K", shp + (3,), (bary, "bary"))
    rc = lib().rasterize_meshes_fwd_static(_p(verts), verts.shape[0], _p(faces), faces.shape[0], _p(first_idx),
                                           _p(num_faces), int(N), int(H), int(W), float(blur_radius), int(K),
                                           int(bin_size), int(max_faces_per_bin or 0), int(sched), int(options),
                                           _p(pix_to_face), _p(zbuf), _p(bary), _p(dists), _p(status_out),
                                           _stream(dev))
    _check("rasterize_meshes_fwd_static", rc)


def rasterize_meshes_bwd(verts, faces, first_idx, num_faces, H, W, blur_radius, K, bin_size, max_faces_per_bin,
                         flags, pix_to_face, grad_zbuf, grad_bary, grad_dists, grad_verts, workspace):
    dev = verts.device
    _require(verts, "verts", torch.float32, dev)
    _require(faces, "faces", torch.int32, dev)
    _require(first_idx, "mesh_to_face_first_idx", torch.int64, dev)
    _require(num_faces, "num_faces_per_mesh", torch.int64, dev)
    _require(pix_to_face, "pix_to_face", torch.int32, dev)
    for t, n in ((grad_zbuf, "grad_zbuf"), (grad_bary, "grad_bary"), (grad_dists, "grad_dists"),
                 (grad_verts, "grad_verts")):
        _require(t, n, torch.float32, dev)
    _require(workspace, "workspace", torch.uint8, dev)
    N = _mesh_shapes(verts, faces, first_idx, num_faces)
    shp = (N, int(H), int(W), int(K))
    _same_shape("N,H,W,K", shp, (pix_to_face, "pix_to_face"), (grad_zbuf, "grad_zbuf"), (grad_dists, "grad_dists"))
    _same_shape("N,H,W,K", shp + (3,), (grad_bary, "grad_bary"))
    _same_shape("verts", verts.shape, (grad_verts, "grad_verts"))
    rc = lib().rasterize_meshes_bwd(_p(verts), verts.shape[0], _p(faces), faces.shape[0], _p(first_idx),
                                    _p(num_faces), int(N), int(H), int(W), float(blur_radius), int(K),
                                    int(bin_size), int(max_faces_per_bin or 0), int(flags), _p(pix_to_face),
                                    _p(grad_zbuf), _p(grad_bary), _p(grad_dists), _p(grad_verts), _p(workspace),
                                    workspace.numel(), _stream(dev))
    _check("rasterize_meshes_bwd", rc)


def rast_bin_count(verts, faces, first_idx, num_faces, H, W, blur_radius, bin_size, workspace):
    dev = verts.device
    _require(verts, "verts", torch.float32, dev)
    _require(faces, "faces", torch.int32, dev)
    _require(first_idx, "mesh_to_face_first_idx", torch.int64, dev)
    _require(num_faces, "num_faces_per_mesh", torch.int64, dev)
    _require(workspace, "workspace", torch.uint8, dev)
    _mesh_shapes(verts, faces, first_idx, num_faces)
    rc = lib().rast_bin_count(_p(verts), verts.shape[0], _p(faces), faces.shape[0], _p(first_idx), _p(num_faces),
                              int(first_idx.shape[0]), int(H), int(W), float(blur_radius), int(bin_size),
                              _p(workspace), workspace.numel(), _stream(dev))
    _check("rast_bin_count", rc)


def rast_query_status(workspace):
    """(status, max_bin_count) of the last call on this workspace; synchronises the stream."""
    st = ctypes.c_int(0)
    mx = ctypes.c_int(0)
    _check("rast_query_status", lib().rast_query_status(_p(workspace), ctypes.byref(st), ctypes.byref(mx),
                                                         _stream(workspace.device)))
    return int(st.value), int(mx.value)


def _same_shape(ref, shape, *named):
    """Raise unless every given tensor has exactly `shape` (checked before any launch)."""
    for t, n in named:
        if t is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{n} has shape {tuple(t.shape)}, expected {tuple(shape)} (from {ref})")


def silhouette_blend_fwd(pix_to_face, dists, sigma, alpha):
    dev = dists.device
    _require(pix_to_face, "pix_to_face", torch.int32, dev)
    _require(dists, "dists", torch.float32, dev)
    _require(alpha, "alpha", torch.float32, dev)
    _same_shape("dists", dists.shape, (pix_to_face, "pix_to_face"))
    _same_shape("dists", dists.shape[:-1], (alpha, "alpha"))
    K = dists.shape[-1]
    P = dists.numel() // K
    _check("silhouette_blend_fwd",
           lib().silhouette_blend_fwd(_p(pix_to_face), _p(dists), P, int(K), float(sigma), _p(alpha), _stream(dev)))


def silhouette_blend_bwd(pix_to_face, dists, grad_alpha, sigma, grad_dists):
    dev = dists.device
    _require(pix_to_face, "pix_to_face", torch.int32, dev)
    _require(dists, "dists", torch.float32, dev)
    _require(grad_alpha, "grad_alpha", torch.float32, dev)
    _require(grad_dists, "grad_dists", torch.float32, dev)
    _same_shape("dists", dists.shape, (pix_to_face, "pix_to_face"), (grad_dists, "grad_dists"))
    _same_shape("dists", dists.shape[:-1], (grad_alpha, "grad_alpha"))
    K = dists.shape[-1]
    P = dists.numel() // K
    _check("silhouette_blend_bwd",
           lib().silhouette_blend_bwd(_p(pix_to_face), _p(dists), _p(grad_alpha), P, int(K), float(sigma),
                                      _p(grad_dists), _stream(dev)))


def rast_set_kernel_events(kernel: int, begin, end):
    """begin/end: raw hipEvent_t handles (ints) or None to switch off."""
    b = None if begin is None else ctypes.c_void_p(begin)
    e = None if end is None else ctypes.c_void_p(end)
    _check("rast_set_kernel_events", lib().rast_set_kernel_events(int(kernel), b, e))


def softmax_blend_fwd(pix_to_face, zbuf, dists, colors, sigma, gamma, znear, zfar, image):
    dev = dists.device
    _require(pix_to_face, "pix_to_face", torch.int32, dev)
    for t, n in ((zbuf, "zbuf"), (dists, "dists"), (colors, "colors"), (image, "image")):
        _require(t, n, torch.float32, dev)
    C = colors.shape[-1]
    _same_shape("dists", dists.shape, (pix_to_face, "pix_to_face"), (zbuf, "zbuf"))
    _same_shape("dists", tuple(dists.shape) + (C,), (colors, "colors"))
    _same_shape("dists", tuple(dists.shape[:-1]) + (C,), (image, "image"))
    K = dists.shape[-1]
    P = dists.numel() // K
    _check("softmax_blend_fwd",
           lib().softmax_blend_fwd(_p(pix_to_face), _p(zbuf), _p(dists), _p(colors), P, K, C, float(sigma),
                                   float(gamma), float(znear), float(zfar), _p(image), _stream(dev)))


def softmax_blend_bwd(pix_to_face, zbuf, dists, colors, sigma, gamma, znear, zfar, grad_image, grad_zbuf, grad_dists,
                      grad_colors):
    dev = dists.device
    _require(pix_to_face, "pix_to_face", torch.int32, dev)
    for t, n in ((zbuf, "zbuf"), (dists, "dists"), (colors, "colors"), (grad_image, "grad_image"),
                 (grad_zbuf, "grad_zbuf"), (grad_dists, "grad_dists"), (grad_colors, "grad_colors")):
        _require(t, n, torch.float32, dev)
    C = colors.shape[-1]
    _same_shape("dists", dists.shape, (pix_to_face, "pix_to_face"), (zbuf, "zbuf"), (grad_zbuf, "grad_zbuf"),
                (grad_dists, "grad_dists"))
    _same_shape("dists", tuple(dists.shape) + (C,), (colors, "colors"), (grad_colors, "grad_colors"))
    _same_shape("dists", tuple(dists.shape[:-1]) + (C,), (grad_image, "grad_image"))
    K = dists.shape[-1]
    P = dists.numel() // K
    _check("softmax_blend_bwd",
           lib().softmax_blend_bwd(_p(pix_to_face), _p(zbuf), _p(dists), _p(colors), P, K, C, float(sigma),
                                   float(gamma), float(znear), float(zfar), _p(grad_image), _p(grad_zbuf),
                                   _p(grad_dists), _p(grad_colors), _stream(dev)))


# ---------------------------------------------------------------------------
# point clouds
# ---------------------------------------------------------------------------
def rast_points_workspace_size(N, H, W, P) -> int:
    out = ctypes.c_size_t(0)
    _check("rast_points_workspace_size",
           lib().rast_points_workspace_size(int(N), int(H), int(W), int(P), ctypes.byref(out)))
    return int(out.value)


def _cloud_shapes(points, first_idx, num_points):
    """Shapes of the packed point inputs; returns N."""
    if points.dim() != 2 or points.shape[1] != 3:
        raise ValueError(f"points must be (P,3), got {tuple(points.shape)}")
    if first_idx.dim() != 1 or tuple(num_points.shape) != tuple(first_idx.shape):
        raise ValueError("cloud_to_first_idx and num_points_per_cloud must be (N,) each")
    return first_idx.shape[0]


def rasterize_points_fwd(points, first_idx, num_points, H, W, radius, K, idx, zbuf, dists, workspace):
    dev = points.device
    _require(points, "points", torch.float32, dev)
    _require(first_idx, "cloud_to_first_idx", torch.int64, dev)
    _require(num_points, "num_points_per_cloud", torch.int64, dev)
    _require(idx, "idx", torch.int32, dev)
    _require(zbuf, "zbuf", torch.float32, dev)
    _require(dists, "dists", torch.float32, dev)
    _require(workspace, "workspace", torch.uint8, dev)
    N = _cloud_shapes(points, first_idx, num_points)
    _same_shape("N,H,W,K", (N, int(H), int(W), int(K)), (idx, "idx"), (zbuf, "zbuf"), (dists, "dists"))
    rc = lib().rasterize_points_fwd(_p(points), points.shape[0], _p(first_idx), _p(num_points), int(N), int(H),
                                    int(W), float(radius), int(K), _p(idx), _p(zbuf), _p(dists), _p(workspace),
                                    workspace.numel(), _stream(dev))
    _check("rasterize_points_fwd", rc)


def rasterize_points_bwd(points, first_idx, num_points, H, W, radius, K, flags, idx, grad_zbuf, grad_dists,
                         grad_points, workspace):
    dev = points.device
    _require(points, "points", torch.float32, dev)
    _require(first_idx, "cloud_to_first_idx", torch.int64, dev)
    _require(num_points, "num_points_per_cloud", torch.int64, dev)
    _require(idx, "idx", torch.int32, dev)
    for t, n in ((grad_zbuf, "grad_zbuf"), (grad_dists, "grad_dists"), (grad_points, "grad_points")):
        _require(t, n, torch.float32, dev)
    _require(workspace, "workspace", torch.uint8, dev)
    N = _cloud_shapes(points, first_idx, num_points)
    _same_shape("N,H,W,K", (N, int(H), int(W), int(K)), (idx, "idx"), (grad_zbuf, "grad_zbuf"),
                (grad_dists, "grad_dists"))
    _same_shape("points", points.shape, (grad_points, "grad_points"))
    rc = lib().rasterize_points_bwd(_p(points), points.shape[0], _p(first_idx), _p(num_points), int(N), int(H),
                                    int(W), float(radius), int(K), int(flags), _p(idx), _p(grad_zbuf),
                                    _p(grad_dists), _p(grad_points), _p(workspace), workspace.numel(), _stream(dev))
    _check("rasterize_points_bwd", rc)


def _composite_shapes(idx, weights, features, image, num_points):
    """(npix, K, P, D); features None = all ones (D from the image, P given)."""
    _same_shape("idx", idx.shape, (weights, "weights"))
    if features is not None:
        if features.dim() != 2:
            raise ValueError(f"features must be (P,D), got {tuple(features.shape)}")
        P, D = features.shape
    else:
        if num_points is None:
            raise ValueError("without a feature table the number of points must be given")
        P, D = int(num_points), int(image.shape[-1])
    _same_shape("idx", tuple(idx.shape[:-1]) + (D,), (image, "image"))
    K = idx.shape[-1]
    return idx.numel() // K if K else 0, K, P, D


def points_composite_fwd(idx, weights, features, mode, radius, image, num_points=None):
    """features None: every feature is 1 (silhouette compositing)."""
    dev = idx.device
    _require(idx, "idx", torch.int32, dev)
    for t, n in ((weights, "weights"), (features, "features"), (image, "image")):
        _require(t, n, torch.float32, dev)
    npix, K, P, D = _composite_shapes(idx, weights, features, image, num_points)
    _check("points_composite_fwd",
           lib().points_composite_fwd(_p(idx), _p(weights), _p(features), P, npix, K, D, int(mode), float(radius),
                                      _p(image), _stream(dev)))


def points_composite_bwd(idx, weights, features, mode, radius, grad_image, grad_weights, grad_features,
                         num_points=None):
    dev = idx.device
    _require(idx, "idx", torch.int32, dev)
    for t, n in ((weights, "weights"), (features, "features"), (grad_image, "grad_image"),
                 (grad_weights, "grad_weights"), (grad_features, "grad_features")):
        _require(t, n, torch.float32, dev)
    npix, K, P, D = _composite_shapes(idx, weights, features, grad_image, num_points)
    _same_shape("idx", idx.shape, (grad_weights, "grad_weights"))
    if features is not None:
        _same_shape("features", features.shape, (grad_features, "grad_features"))
    _check("points_composite_bwd",
           lib().points_composite_bwd(_p(idx), _p(weights), _p(features), P, npix, K, D, int(mode), float(radius),
                                      _p(grad_image), _p(grad_weights), _p(grad_features), _stream(dev)))
