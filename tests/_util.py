"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare it with the oracle under the stated tolerances.

Tolerances (fixed by the workload contract and the FP32/FP64 arithmetic):
  pix_to_face  exact on pixels the oracle does not flag as ambiguous, and a
               correct answer (by the oracle's candidates) on flagged ones
  bary         abs(dw_i) <= 1e-5 * max(1, abs(w_i))
  zbuf         abs(dz)   <= 1e-5 (1e-5 * sum_i abs(w_i z_i) if some abs(w_i) > 1)
  dists        abs(dd)   <= 1e-5 and <= 1e-5 * abs(d) + 1e-12
  grad_verts   max abs error <= 1e-3 * max abs(reference) and
               L2 error <= 1e-3 * L2 norm of the reference
The relative branches exist because an FP32 barycentric of an outside pixel
near a sliver can be far above 1, where FP32 storage alone rounds it by more
than 1e-5.
"""
import sys

import numpy as np
import torch

import oracle
from oracle import validity as _validity
from paper_2007_08501_amd import _lib
from paper_2007_08501_amd.raster import empty_fragments

TOL_VAL = 1e-5
TOL_GRAD = 1e-3


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def threads():
    return min(16, oracle.default_threads())


def to_dev(b, dev="cuda"):
    return (torch.from_numpy(b.verts).to(dev), torch.from_numpy(b.faces).to(dev),
            torch.from_numpy(b.first_idx).to(dev), torch.from_numpy(b.num_faces).to(dev))


def run_fwd(b, bs, M=None, sched=0, K=None, dev_inputs=None, check=True, options=0):
    v, f, fi, nf = dev_inputs or to_dev(b)
    H, W = b.image_size
    K = K or b.faces_per_pixel
    N = fi.shape[0]
    if bs > 0 and M is None:
        M = bin_capacity(b, bs, (v, f, fi, nf))
    out = empty_fragments(N, H, W, K, v.device)
    ws = _lib.alloc_workspace(_lib.rast_workspace_size(N, H, W, f.shape[0], bs, M or 0), v.device)
    _lib.rasterize_meshes_fwd(v, f, fi, nf, H, W, b.blur_radius, K, bs, M or 0, sched, out.pix_to_face, out.zbuf,
                              out.bary, out.dists, ws, options)
    if check:
        st, _ = _lib.rast_query_status(ws)
        assert st == _lib.RAST_OK, _lib.status_string(st)
    return out, ws


def bin_capacity(b, bs, dev_inputs=None):
    """Exact largest bin count for bin size bs (counting pass)."""
    v, f, fi, nf = dev_inputs or to_dev(b)
    H, W = b.image_size
    wsc = _lib.alloc_workspace(_lib.rast_workspace_size(fi.shape[0], H, W, f.shape[0], bs, 1), v.device)
    _lib.rast_bin_count(v, f, fi, nf, H, W, b.blur_radius, bs, wsc)
    st, mx = _lib.rast_query_status(wsc)
    assert st == _lib.RAST_OK
    return max(1, mx)


def run_bwd(b, p2f, gz, gb, gd, dev_inputs=None, bs=0, M=None, check=True, flags=0, ws=None):
    """Backward through the C ABI; bs/M are the binning of the forward
    (bs 0 = per-face form).  flags/ws: reuse a forward's workspace."""
    v, f, fi, nf = dev_inputs or to_dev(b)
    H, W = b.image_size
    N, K = p2f.shape[0], p2f.shape[-1]
    if bs > 0 and M is None:
        M = bin_capacity(b, bs, (v, f, fi, nf))
    gv = torch.empty_like(v)
    if ws is None:
        ws = _lib.alloc_workspace(_lib.rast_workspace_size(N, H, W, f.shape[0], bs, M or 0), v.device)
    t = lambda a: None if a is None else (a if isinstance(a, torch.Tensor) else torch.from_numpy(a).to(v.device))
    _lib.rasterize_meshes_bwd(v, f, fi, nf, H, W, b.blur_radius, K, bs, M or 0, flags, p2f, t(gz), t(gb), t(gd), gv,
                              ws)
    if check:
        st, _ = _lib.rast_query_status(ws)
        assert st == _lib.RAST_OK, _lib.status_string(st)
    torch.cuda.synchronize()
    return gv


def frag_numpy(out, pix=None):
    """Fragments as numpy; with pix (linear pixel ids) only those pixels."""
    res = {}
    for name, t in zip(("p2f", "zbuf", "bary", "dists"), out):
        if pix is not None:
            N, H, W = t.shape[:3]
            flat = t.reshape((N * H * W,) + tuple(t.shape[3:]))
            t = flat[torch.from_numpy(np.asarray(pix)).to(t.device)]
        res[name] = t.detach().cpu().numpy()
    return res


def compare_fwd(g, o, b, where="", pixels=None, options=0, verts=None, faces=None):
    """GPU fragments g against the oracle's o for batch b (the checks of
    oracle.validity.compare_fragments, with this module's thread count)."""
    return _validity.compare_fragments(g, o, b.verts if verts is None else verts, b.faces if faces is None else faces,
                                       b.first_idx, b.num_faces, b.image_size, b.blur_radius, where=where,
                                       pixels=pixels, options=options, nthreads=threads())


def compare_grad(g, ref, where=""):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.abs(g - ref)
    mx = np.abs(ref).max()
    assert d.max() <= TOL_GRAD * mx, f"{where}: grad max err {d.max()} vs scale {mx}"
    assert np.linalg.norm(g - ref) <= TOL_GRAD * np.linalg.norm(ref), f"{where}: grad L2 err"
    return float(d.max() / mx) if mx > 0 else 0.0


def invariants_torch(out, fi, nf, blur):
    """Properties that hold at any size, checked on the device."""
    p2f, z, b, d = out
    valid = p2f >= 0
    assert not (valid[..., 1:] & ~valid[..., :-1]).any(), "valid slots are not a prefix"
    vv = valid[..., 1:] & valid[..., :-1]
    assert ((z[..., 1:] - z[..., :-1])[vv] >= 0).all(), "zbuf decreases along k"
    s = b.sum(-1)
    sc = torch.clamp(b.abs().sum(-1), min=1.0)
    assert ((s - 1).abs()[valid] <= 1e-5 * sc[valid]).all(), "bary does not sum to 1"
    inside = (b > 0).all(-1)
    assert (d[valid & inside] < 0).all()
    out_ = valid & ~inside
    assert ((d[out_] >= 0) & (d[out_] < blur)).all()
    N = p2f.shape[0]
    lo = fi.view(N, 1, 1, 1)
    hi = (fi + nf).view(N, 1, 1, 1)
    assert (((p2f >= lo) & (p2f < hi)) | ~valid).all(), "face of another mesh"
    assert (z[~valid] == -1).all() and (d[~valid] == -1).all()
    return int(valid.sum())


def tie_masked_grads(b, p2f_np, gz, gb, gd, pixels=None):
    """Zero grad_dists on slots whose nearest edge is (nearly) tied (M6).
    With pixels, p2f_np holds the rows of those pixels and only their rows
    of gd (full (N,H,W,K)) are examined."""
    if pixels is None:
        _, _, _, tie = oracle.fragments_fixed(b.verts, b.faces, b.image_size, p2f_np, nthreads=threads())
        return gz, gb, np.where(tie.astype(bool), np.float32(0), gd).astype(np.float32)
    _, _, _, tie = oracle.fragments_fixed(b.verts, b.faces, b.image_size, p2f_np, nthreads=threads(),
                                          pixels=pixels)
    gd = gd.copy()
    flat = gd.reshape(-1, gd.shape[-1])
    flat[pixels] = np.where(tie.astype(bool), np.float32(0), flat[pixels])
    return gz, gb, gd
