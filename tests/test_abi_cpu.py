"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2007_08501_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rast.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:int|const char\*|void|size_t)\s+(\w+)\s*\(", text, flags=re.M)
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rast_workspace_size", "rasterize_meshes_fwd", "rasterize_meshes_bwd", "rast_bin_count",
              "rast_query_status", "rast_status_string", "silhouette_blend_fwd", "silhouette_blend_bwd"):
        assert n in names
    assert set(names) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_status_strings():
    for code in (_lib.RAST_OK, _lib.RAST_EINVAL, _lib.RAST_EWORKSPACE, _lib.RAST_EHIP, _lib.RAST_EOVERFLOW,
                 _lib.RAST_EMESH, _lib.RAST_EREUSE, _lib.RAST_ESCRATCH):
        s = _lib.status_string(code)
        assert s and s != "unknown status"
    assert _lib.status_string(12345) == "unknown status"


def ws_size(*args):
    out = ctypes.c_size_t(0)
    rc = _lib.lib().rast_workspace_size(*args, ctypes.byref(out))
    return rc, out.value


def test_workspace_size_validation_and_growth():
    rc, a = ws_size(1, 64, 64, 320, 0, 0)
    assert rc == 0 and a >= 256 + 320 * 64
    rc, b = ws_size(1, 64, 64, 320, 8, 100)
    assert rc == 0 and b >= a + 64 * 100 * 4
    rc, c = ws_size(1, 64, 64, 320, 8, 200)
    assert rc == 0 and c > b
    assert ws_size(0, 64, 64, 320, 0, 0)[0] == _lib.RAST_EINVAL        # N
    assert ws_size(1, 64, 64, -1, 0, 0)[0] == _lib.RAST_EINVAL         # F
    assert ws_size(1, 64, 64, 320, 12, 10)[0] == _lib.RAST_EINVAL      # not a multiple of 8
    assert ws_size(1, 64, 64, 320, 1024, 10)[0] == _lib.RAST_EINVAL    # > max bin
    assert ws_size(1, 64, 64, 320, 8, 0)[0] == _lib.RAST_EINVAL        # M
    assert _lib.lib().rast_workspace_size(1, 64, 64, 320, 0, 0, None) == _lib.RAST_EINVAL


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first


def fwd(**kw):
    a = dict(verts=FAKE, V=3, faces=FAKE, F=1, first=FAKE, nf=FAKE, N=1, H=8, W=8, blur=0.0, K=1, bs=0, M=0,
             sched=0, opts=0, p2f=FAKE, zbuf=FAKE, bary=FAKE, dists=FAKE, ws=None, wsb=0, stream=None)
    a.update(kw)
    return _lib.lib().rasterize_meshes_fwd(a["verts"], a["V"], a["faces"], a["F"], a["first"], a["nf"], a["N"],
                                           a["H"], a["W"], a["blur"], a["K"], a["bs"], a["M"], a["sched"],
                                           a["opts"], a["p2f"], a["zbuf"], a["bary"], a["dists"], a["ws"], a["wsb"],
                                           a["stream"])


@pytest.mark.parametrize("kw", [
    dict(N=0), dict(H=0), dict(W=-3), dict(K=0), dict(K=65), dict(blur=-1.0), dict(blur=float("nan")),
    dict(blur=float("inf")), dict(bs=4), dict(bs=8, M=0), dict(bs=520, M=4), dict(sched=2), dict(V=-1),
    dict(F=-1), dict(F=1 << 31), dict(H=1, W=1 << 22, K=64), dict(verts=None), dict(faces=None), dict(first=None), dict(nf=None),
    dict(p2f=None), dict(zbuf=None), dict(bary=None), dict(dists=None), dict(opts=1), dict(opts=0x800),
    dict(opts=-1),
])
def test_forward_rejects_bad_arguments(kw):
    assert fwd(**kw) == _lib.RAST_EINVAL


def test_forward_rejects_bad_workspace():
    assert fwd(ws=None, wsb=1 << 20) == _lib.RAST_EWORKSPACE
    # every option combination passes validation (and then needs a workspace)
    for o in (0x100, 0x200, 0x400, 0x700):
        assert fwd(opts=o) == _lib.RAST_EWORKSPACE
    assert fwd(ws=ctypes.c_void_p(0x1001), wsb=1 << 20) == _lib.RAST_EWORKSPACE  # misaligned
    assert fwd(ws=ctypes.c_void_p(0x1000), wsb=16) == _lib.RAST_EWORKSPACE      # too small


def test_backward_rejects_bad_arguments():
    L = _lib.lib()
    args = [FAKE, 3, FAKE, 1, FAKE, FAKE, 1, 8, 8, 0.0, 1, 0, 0, 0, FAKE, None, None, None, FAKE, None, 0, None]
    assert L.rasterize_meshes_bwd(*args) == _lib.RAST_EWORKSPACE
    reuse = list(args)
    reuse[13] = _lib.RAST_BWD_REUSE_FORWARD
    assert L.rasterize_meshes_bwd(*reuse) == _lib.RAST_EWORKSPACE
    reuse[13] = _lib.RAST_BWD_REUSE_FORWARD | 0x700  # the forward's options ride along
    assert L.rasterize_meshes_bwd(*reuse) == _lib.RAST_EWORKSPACE
    for i, v in ((14, None), (18, None), (10, 100), (9, -1.0), (4, None), (5, None), (6, 0), (11, 12), (11, -8),
                 (13, 2), (13, -1), (13, 0x800)):
        bad = list(args)
        bad[i] = v
        assert L.rasterize_meshes_bwd(*bad) == _lib.RAST_EINVAL, i
    bad = list(args)
    bad[11], bad[12] = 8, 0  # binned without a capacity
    assert L.rasterize_meshes_bwd(*bad) == _lib.RAST_EINVAL


def test_bin_count_and_blend_reject_bad_arguments():
    L = _lib.lib()
    assert L.rast_bin_count(FAKE, 3, FAKE, 1, FAKE, FAKE, 1, 8, 8, 0.0, 0, None, 0, None) == _lib.RAST_EINVAL
    assert L.rast_bin_count(FAKE, 3, FAKE, 1, FAKE, FAKE, 1, 8, 8, 0.0, 8, None, 0, None) == _lib.RAST_EWORKSPACE
    assert L.silhouette_blend_fwd(FAKE, FAKE, 10, 4, 0.0, FAKE, None) == _lib.RAST_EINVAL
    assert L.silhouette_blend_fwd(FAKE, FAKE, 10, 0, 1e-4, FAKE, None) == _lib.RAST_EINVAL
    assert L.silhouette_blend_fwd(None, FAKE, 10, 4, 1e-4, FAKE, None) == _lib.RAST_EINVAL
    assert L.silhouette_blend_bwd(FAKE, FAKE, FAKE, 10, 4, -1.0, FAKE, None) == _lib.RAST_EINVAL
    assert L.silhouette_blend_bwd(FAKE, FAKE, None, 10, 4, 1e-4, FAKE, None) == _lib.RAST_EINVAL
    assert L.rast_query_status(None, None, None, None) == _lib.RAST_EINVAL


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2007_08501_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "oracle_rast" not in text and "liboracle" not in text, fn


def test_softmax_blend_rejects_bad_arguments():
    L = _lib.lib()
    # p2f, zbuf, dists, colors, P, K, C, sigma, gamma, znear, zfar, image, stream
    good = [FAKE, FAKE, FAKE, FAKE, 0, 4, 3, 1e-4, 1e-4, 1.0, 100.0, FAKE, None]
    assert L.softmax_blend_fwd(*good) == _lib.RAST_OK  # P = 0: nothing to launch
    for i, v in ((5, 0), (5, 65), (6, 0), (6, 9), (7, 0.0), (7, float("nan")), (8, -1.0), (9, 100.0), (10, 1.0),
                 (10, float("inf")), (4, -1)):
        bad = list(good)
        bad[i] = v
        assert L.softmax_blend_fwd(*bad) == _lib.RAST_EINVAL, i
    bad = list(good)
    bad[4], bad[0] = 10, None
    assert L.softmax_blend_fwd(*bad) == _lib.RAST_EINVAL
    # bwd: ..., grad_image, grad_zbuf, grad_dists, grad_colors, stream; the gradients may be NULL
    gb = good[:11] + [FAKE, None, None, None, None]
    assert L.softmax_blend_bwd(*gb) == _lib.RAST_OK
    bad = list(gb)
    bad[4], bad[11] = 10, None
    assert L.softmax_blend_bwd(*bad) == _lib.RAST_EINVAL


def test_points_workspace_size():
    L = _lib.lib()
    out = ctypes.c_size_t(0)
    assert L.rast_points_workspace_size(8, 256, 256, 1600000, ctypes.byref(out)) == _lib.RAST_OK
    assert out.value >= 1600000 * 24 + 8 * 1024 * 4
    small = out.value
    assert L.rast_points_workspace_size(8, 256, 256, 100, ctypes.byref(out)) == _lib.RAST_OK
    assert out.value < small
    assert L.rast_points_workspace_size(0, 256, 256, 100, ctypes.byref(out)) == _lib.RAST_EINVAL
    assert L.rast_points_workspace_size(1, 256, 256, -1, ctypes.byref(out)) == _lib.RAST_EINVAL
    assert L.rast_points_workspace_size(1, 256, 256, (1 << 30) + 1, ctypes.byref(out)) == _lib.RAST_EINVAL
    assert L.rast_points_workspace_size(1, 256, 256, 10, None) == _lib.RAST_EINVAL


def pfwd(**kw):
    a = dict(pts=FAKE, P=10, first=FAKE, num=FAKE, N=1, H=8, W=8, r=0.1, K=4, idx=FAKE, zbuf=FAKE, dists=FAKE,
             ws=None, wsb=0, stream=None)
    a.update(kw)
    return _lib.lib().rasterize_points_fwd(a["pts"], a["P"], a["first"], a["num"], a["N"], a["H"], a["W"], a["r"],
                                           a["K"], a["idx"], a["zbuf"], a["dists"], a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("kw", [
    dict(N=0), dict(H=0), dict(W=-1), dict(K=0), dict(K=65), dict(r=-0.1), dict(r=float("nan")),
    dict(r=float("inf")), dict(r=2.5), dict(P=-1), dict(P=(1 << 30) + 1), dict(H=16385), dict(W=20000),
    dict(pts=None), dict(first=None), dict(num=None), dict(idx=None), dict(zbuf=None), dict(dists=None),
])
def test_points_forward_rejects_bad_arguments(kw):
    assert pfwd(**kw) == _lib.RAST_EINVAL


def test_points_forward_and_backward_reject_bad_workspace():
    assert pfwd() == _lib.RAST_EWORKSPACE
    assert pfwd(ws=ctypes.c_void_p(0x1001), wsb=1 << 20) == _lib.RAST_EWORKSPACE
    assert pfwd(ws=ctypes.c_void_p(0x1000), wsb=64) == _lib.RAST_EWORKSPACE
    L = _lib.lib()
    # points, P, first, num, N, H, W, r, K, flags, idx, gz, gd, grad, ws, wsb, stream
    args = [FAKE, 10, FAKE, FAKE, 1, 8, 8, 0.1, 4, 0, FAKE, None, None, FAKE, None, 0, None]
    assert L.rasterize_points_bwd(*args) == _lib.RAST_EWORKSPACE
    for i, v in ((9, 2), (9, -1), (10, None), (13, None), (0, None), (7, -1.0), (8, 0), (2, None)):
        bad = list(args)
        bad[i] = v
        assert L.rasterize_points_bwd(*bad) == _lib.RAST_EINVAL, i


def test_points_composite_rejects_bad_arguments():
    L = _lib.lib()
    # idx, weights, features, P, npix, K, D, mode, radius, image, stream
    good = [FAKE, FAKE, FAKE, 10, 0, 4, 3, 0, 0.0, FAKE, None]
    assert L.points_composite_fwd(*good) == _lib.RAST_OK  # no pixels: nothing to launch
    for i, v in ((5, 0), (5, 65), (6, 0), (6, 9), (7, 4), (7, -1), (3, -1), (4, -1)):
        bad = list(good)
        bad[i] = v
        assert L.points_composite_fwd(*bad) == _lib.RAST_EINVAL, i
    fd = list(good)
    fd[7] = _lib.RAST_COMPOSITE_FROM_DISTS  # needs a positive radius
    assert L.points_composite_fwd(*fd) == _lib.RAST_EINVAL
    fd[8] = 0.01
    assert L.points_composite_fwd(*fd) == _lib.RAST_OK
    bad = list(good)
    bad[4], bad[0] = 10, None
    assert L.points_composite_fwd(*bad) == _lib.RAST_EINVAL
    # bwd: ..., grad_image, grad_weights, grad_features (may be NULL), stream
    gb = good[:9] + [FAKE, FAKE, None, None]
    assert L.points_composite_bwd(*gb) == _lib.RAST_OK
    bad = list(gb)
    bad[4], bad[10] = 10, None
    assert L.points_composite_bwd(*bad) == _lib.RAST_EINVAL


def test_static_forward_refuses_oversize_before_any_launch():
    """rasterize_meshes_fwd_static: a problem whose workspace would exceed the
    static scratch is refused on the host (no device is touched: the
    pointers below are never dereferenced)."""
    L = _lib.lib()
    dummy = ctypes.c_void_p(256)
    H = W = 64
    nbins = (H // 8) * (W // 8)
    M = _lib.RAST_STATIC_SCRATCH_BYTES // (4 * nbins) + 1
    rc, need = ws_size(1, H, W, 320, 8, M)
    assert rc == 0 and need > _lib.RAST_STATIC_SCRATCH_BYTES
    args = [dummy, 162, dummy, 320, dummy, dummy, 1, H, W, 0.0, 1, 8, M, 0, 0, dummy, dummy, dummy, dummy, None, None]
    assert L.rasterize_meshes_fwd_static(*args) == _lib.RAST_ESCRATCH
    # argument checks come first, as for the workspace form
    bad = list(args)
    bad[10] = 0  # K
    assert L.rasterize_meshes_fwd_static(*bad) == _lib.RAST_EINVAL

