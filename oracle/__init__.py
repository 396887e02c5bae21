"""FP64 CPU oracle for the batched mesh rasterizer, the point-cloud
rasterizer, and the blending and compositing steps.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and it never
imports the product path: the two share nothing but the seeded input
generator, which holds none of the method's arithmetic.

The rasterizer oracles are plain C (``oracle_rast.c`` for meshes,
``oracle_points.c`` for point clouds, built here with gcc and loaded with
ctypes); the blend oracle is NumPy in float64 (``blend.py``), as are the
point compositing oracle (``points.py``) and the silhouette-fitting loss and
its gradient (``silfit.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle_rast.c"), os.path.join(_HERE, "oracle_points.c")]
# ORACLE_LIB_PATH names another build of the same sources (the sanitized
# build of the CPU checks); by default the in-tree liboracle.so
_LIB = os.environ.get("ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")
_lib = None
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def _stale() -> bool:
    return not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS)


def build(force: bool = True, sanitize: bool = False, out: Optional[str] = None) -> str:
    """Compile the C oracles into liboracle.so (gcc, -O2, OpenMP, no
    fast-math), or with AddressSanitizer and UndefinedBehaviorSanitizer into
    `out`."""
    path = out or _LIB
    if force or sanitize or out or _stale():
        tmp = path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O1" if sanitize else "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-fno-fast-math", "-ffp-contract=off"] + (SANITIZE if sanitize else []) + _SRCS + ["-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _stale():
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.oracle_rasterize.argtypes = [P, i64, P, i64, P, P, ci, ci, ci, ctypes.c_double, ci, P, i64,
                                     P, P, P, P, P, P, ci, ci]
    lib.oracle_rasterize.restype = ci
    lib.oracle_candidates.argtypes = [P, P, P, P, ci, ci, ci, ctypes.c_double, P, i64, ci, P, P, P, P, P, P, ci, ci]
    lib.oracle_candidates.restype = ci
    lib.oracle_fragments_fixed.argtypes = [P, P, ci, ci, ci, ci, P, ctypes.c_int64, P, P, P, P, P, ci, ci]
    lib.oracle_fragments_fixed.restype = ci
    lib.oracle_backward.argtypes = [P, i64, P, ci, ci, ci, ci, P, i64, P, P, P, P, P, ci, ci]
    lib.oracle_backward.restype = ci
    lib.oracle_points_rasterize.argtypes = [P, i64, P, P, ci, ci, ci, ctypes.c_double, ci, P, i64, P, P, P, P, ci]
    lib.oracle_points_rasterize.restype = ci
    lib.oracle_points_backward.argtypes = [P, i64, ci, ci, ci, ci, P, i64, P, P, P, P, ci]
    lib.oracle_points_backward.restype = ci
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ci
    _lib = lib
    return lib


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


# Bits of the per-pixel ambiguity mask (see oracle_rast.c)
AMB_M1, AMB_M2, AMB_M3, AMB_M4, AMB_M5, AMB_M7, AMB_M8 = 1, 2, 4, 8, 16, 64, 128
AMB_BITS = dict(M1=AMB_M1, M2=AMB_M2, M3=AMB_M3, M4=AMB_M4, M5=AMB_M5, M7=AMB_M7, M8=AMB_M8)
# Per-face classes of candidates(): counts; counts but within a margin of not
# counting; does not count but within a margin of counting
CLS_COUNTS, CLS_BORDER_IN, CLS_BORDER_OUT = 0, 1, 2

# Rasterizer options (bits; see oracle_rast.c for their definitions)
PERSPECTIVE_CORRECT = 0x100
CLIP_BARYCENTRIC = 0x200
CULL_BACKFACES = 0x400


def rasterize(verts, faces, first_idx, num_faces, image_size, blur_radius, faces_per_pixel,
              pixels=None, nthreads: Optional[int] = None, options: int = 0):
    """Brute-force FP64 rasterization.

    verts (V,3) (float32 inputs are promoted exactly), faces (F,3) global ids,
    first_idx/num_faces (N,).  ``pixels``: optional 1-D array of linear pixel
    ids n*H*W + r*W + c; default every pixel.  Returns a dict with p2f (int64),
    zbuf, bary, dists (float64), amb (uint8 bit mask, AMB_*) and nhits (int64),
    shaped (N,H,W,K[,3]) for full images or (npix,K[,3]) for a pixel list.
    """
    lib = _load()
    H, W = image_size
    K = int(faces_per_pixel)
    N = int(np.asarray(first_idx).shape[0])
    v = _f64(verts)
    f = _i64(faces)
    fi = _i64(first_idx)
    nf = _i64(num_faces)
    pix = None if pixels is None else _i64(pixels)
    npix = N * H * W if pix is None else pix.shape[0]
    p2f = np.empty((npix, K), np.int64)
    zbuf = np.empty((npix, K), np.float64)
    bary = np.empty((npix, K, 3), np.float64)
    dists = np.empty((npix, K), np.float64)
    amb = np.empty((npix,), np.uint8)
    nh = np.empty((npix,), np.int64)
    rc = lib.oracle_rasterize(_ptr(v), v.shape[0], _ptr(f), f.shape[0], _ptr(fi), _ptr(nf), N, H, W,
                              float(blur_radius), K, _ptr(pix), npix, _ptr(p2f), _ptr(zbuf), _ptr(bary),
                              _ptr(dists), _ptr(amb), _ptr(nh), int(options), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_rasterize rejected its arguments")
    out = dict(p2f=p2f, zbuf=zbuf, bary=bary, dists=dists, amb=amb, nhits=nh)
    if pix is None:
        out = {k: a.reshape((N, H, W) + a.shape[1:]) for k, a in out.items()}
    return out


def candidates(verts, faces, first_idx, num_faces, image_size, blur_radius, pixels, cap: int = 64,
               nthreads: Optional[int] = None, options: int = 0):
    """Every face that counts for each listed pixel, or lies within a margin
    of counting, sorted by (z, face id): f (int64, -1 past the end), z, bary
    (3), dists, cls (CLS_*), each (npix, cap), and n (npix,), the number of
    such faces (only the first cap are listed when n > cap)."""
    lib = _load()
    H, W = image_size
    N = int(np.asarray(first_idx).shape[0])
    v = _f64(verts)
    f = _i64(faces)
    fi = _i64(first_idx)
    nf = _i64(num_faces)
    pix = _i64(pixels)
    npix = pix.shape[0]
    cap = int(cap)
    cf = np.empty((npix, cap), np.int64)
    cz = np.empty((npix, cap), np.float64)
    cw = np.empty((npix, cap, 3), np.float64)
    cd = np.empty((npix, cap), np.float64)
    cc = np.empty((npix, cap), np.uint8)
    n = np.empty((npix,), np.int64)
    rc = lib.oracle_candidates(_ptr(v), _ptr(f), _ptr(fi), _ptr(nf), N, H, W, float(blur_radius), _ptr(pix), npix,
                               cap, _ptr(cf), _ptr(cz), _ptr(cw), _ptr(cd), _ptr(cc), _ptr(n), int(options),
                               nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_candidates rejected its arguments")
    return dict(f=cf, z=cz, bary=cw, dists=cd, cls=cc, n=n)


def fragments_fixed(verts, faces, image_size, p2f, nthreads: Optional[int] = None, pixels=None, options: int = 0):
    """zbuf, bary, dists (float64) and the per-slot edge-tie mask for a given
    face choice p2f (N,H,W,K); the forward map with the selection frozen.
    With ``pixels`` (linear pixel ids), p2f is (npix,K) rows of those pixels."""
    lib = _load()
    H, W = image_size
    p = _i64(p2f)
    N, K = p.shape[0], p.shape[-1]
    pix = None if pixels is None else _i64(pixels)
    if pix is not None and pix.shape[0] != N:
        raise ValueError("one p2f row per listed pixel")
    v = _f64(verts)
    f = _i64(faces)
    zbuf = np.empty(p.shape, np.float64)
    bary = np.empty(p.shape + (3,), np.float64)
    dists = np.empty(p.shape, np.float64)
    tie = np.empty(p.shape, np.uint8)
    lib.oracle_fragments_fixed(_ptr(v), _ptr(f), N, H, W, K, _ptr(pix), 0 if pix is None else pix.shape[0],
                               _ptr(p), _ptr(zbuf), _ptr(bary), _ptr(dists), _ptr(tie), int(options),
                               nthreads or default_threads())
    return zbuf, bary, dists, tie


def backward(verts, faces, image_size, p2f, grad_zbuf=None, grad_bary=None, grad_dists=None,
             nthreads: Optional[int] = None, pixels=None, N: Optional[int] = None, options: int = 0):
    """Analytic FP64 dL/dverts (V,3) for L = <gz,zbuf> + <gb,bary> + <gd,dists>
    over the slots of p2f (N,H,W,K).  With ``pixels`` (linear pixel ids),
    p2f and the grads are (npix,K[,3]) rows of those pixels instead; N is
    then the number of images."""
    lib = _load()
    H, W = image_size
    p = _i64(p2f)
    K = p.shape[-1]
    pix = None if pixels is None else _i64(pixels)
    if pix is None:
        N = p.shape[0]
    elif N is None:
        N = int(pix.max()) // (H * W) + 1 if pix.size else 1
    v = _f64(verts)
    f = _i64(faces)
    gz = None if grad_zbuf is None else _f64(grad_zbuf)
    gb = None if grad_bary is None else _f64(grad_bary)
    gd = None if grad_dists is None else _f64(grad_dists)
    out = np.empty(v.shape, np.float64)
    rc = lib.oracle_backward(_ptr(v), v.shape[0], _ptr(f), N, H, W, K, _ptr(pix), 0 if pix is None else pix.shape[0],
                             _ptr(p), _ptr(gz), _ptr(gb), _ptr(gd), _ptr(out), int(options),
                             nthreads or default_threads())
    if rc != 0:
        raise MemoryError("oracle_backward failed")
    return out


def rasterize_points(points, first_idx, num_points, image_size, radius, points_per_pixel, pixels=None,
                     nthreads: Optional[int] = None):
    """FP64 brute-force point rasterizer (oracle_points.c).  points (P,3);
    first_idx/num_points (N,).  Returns dict idx (int64), zbuf, dists
    (float64) shaped (N,H,W,K) -- or (npix,K) rows with ``pixels`` -- and
    amb (uint8 per pixel, see the C source)."""
    lib = _load()
    H, W = image_size
    pts = _f64(points)
    fi = _i64(first_idx)
    npts = _i64(num_points)
    N = fi.shape[0]
    K = int(points_per_pixel)
    pix = None if pixels is None else _i64(pixels)
    rows = N * H * W if pix is None else pix.shape[0]
    idx = np.empty((rows, K), np.int64)
    zbuf = np.empty((rows, K), np.float64)
    dists = np.empty((rows, K), np.float64)
    amb = np.empty(rows, np.uint8)
    rc = lib.oracle_points_rasterize(_ptr(pts), pts.shape[0], _ptr(fi), _ptr(npts), N, H, W, float(radius), K,
                                     _ptr(pix), 0 if pix is None else pix.shape[0], _ptr(idx), _ptr(zbuf),
                                     _ptr(dists), _ptr(amb), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_points_rasterize rejected its arguments")
    out = dict(idx=idx, zbuf=zbuf, dists=dists, amb=amb)
    if pix is None:
        out = {k: a.reshape((N, H, W) + a.shape[1:]) for k, a in out.items()}
    return out


def points_backward(points, image_size, idx, grad_zbuf=None, grad_dists=None, pixels=None, N=None,
                    nthreads: Optional[int] = None):
    """Analytic FP64 dL/dpoints (P,3) for L = <gz, zbuf> + <gd, dists> over
    the slots of idx (N,H,W,K), or of (npix,K) rows with ``pixels``."""
    lib = _load()
    H, W = image_size
    pts = _f64(points)
    ix = _i64(idx)
    K = ix.shape[-1]
    pix = None if pixels is None else _i64(pixels)
    if pix is None:
        N = ix.shape[0]
    gz = None if grad_zbuf is None else _f64(grad_zbuf)
    gd = None if grad_dists is None else _f64(grad_dists)
    out = np.empty(pts.shape, np.float64)
    rc = lib.oracle_points_backward(_ptr(pts), pts.shape[0], int(N or 1), H, W, K, _ptr(pix),
                                    0 if pix is None else pix.shape[0], _ptr(ix), _ptr(gz), _ptr(gd), _ptr(out),
                                    nthreads or default_threads())
    if rc != 0:
        raise MemoryError("oracle_points_backward failed")
    return out


from .points import (alpha_composite, alpha_composite_backward, norm_composite,  # noqa: E402,F401
                     norm_composite_backward, splat_alpha)
from .blend import (iou_loss, silhouette_blend, silhouette_blend_backward, softmax_blend,  # noqa: E402,F401
                    softmax_blend_backward)
