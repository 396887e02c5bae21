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
import _validity
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
        res[name] = t.cpu().numpy()
    return res


def compare_fwd(g, o, b, where="", pixels=None, options=0, verts=None, faces=None):
    """GPU fragments g against the oracle's o (dicts of arrays, rows of the
    same pixels: full images, or the listed `pixels`), for batch b (its
    verts/faces unless given).  Returns stats.

    Face ids: exactly the oracle's on unflagged pixels; up to permutations
    inside runs of tied depths where the only flag is such a tie (M8); and on
    every flagged pixel, a correct answer by the oracle's candidate list
    (tests/_validity.py).  Values of every filled slot against the oracle's
    FP64 values of the same face at the same pixel:
      bary   abs(dw_i) <= 1e-5 * max(1, abs(w_i))
      zbuf   abs(dz)   <= 1e-5, or 1e-5 * sum_i abs(w_i z_i) where some abs(w_i) > 1
      dists  abs(dd)   <= 1e-5 and <= 1e-5 * abs(d) + 1e-12
    """
    verts = b.verts if verts is None else verts
    faces = b.faces if faces is None else faces
    K = o["p2f"].shape[-1]
    amb = o["amb"].reshape(-1).astype(np.int64)
    pg = g["p2f"].astype(np.int64).reshape(-1, K)
    po = o["p2f"].reshape(-1, K)
    npix = pg.shape[0]
    # pixel ids of the rows, for the candidate lists of flagged rows
    if pixels is None:
        rows_pix = np.arange(npix, dtype=np.int64)
    else:
        rows_pix = np.asarray(pixels, np.int64).reshape(-1)
    M8 = oracle.AMB_M8
    strict = amb == 0
    bad = (pg != po).any(-1) & strict
    nbad = int(bad.sum())
    assert nbad == 0, f"{where}: pix_to_face differs at {nbad} unambiguous pixels, e.g. {np.argwhere(bad)[:5]}"
    flagged = np.nonzero(~strict)[0]
    # reference values per row: the oracle's top-K rows for unflagged pixels,
    # the candidate records of the GPU's own faces for flagged ones
    ref_f, ref_z, ref_w, ref_d, ref_ok = po.copy(), o["zbuf"].reshape(-1, K).copy(), \
        o["bary"].reshape(-1, K, 3).copy(), o["dists"].reshape(-1, K).copy(), po >= 0
    n_order_only = 0
    if flagged.size:
        cap = 2 * K + 32
        c = oracle.candidates(verts, faces, b.first_idx, b.num_faces, b.image_size, b.blur_radius,
                              rows_pix[flagged], cap=cap, nthreads=threads(), options=options)
        for j, i in enumerate(flagged):
            why = _validity.valid_choice(pg[i], c["f"][j], c["z"][j], c["cls"][j], c["n"][j], K)
            assert why is None, f"{where}: row {i} (pixel {rows_pix[i]}, flags {amb[i]:#x}) GPU ids {pg[i]}: {why}"
            if amb[i] == M8:
                n_order_only += 1
                nf = int((po[i] >= 0).sum())
                assert _validity.equal_up_to_ties(pg[i], po[i], o["zbuf"].reshape(-1, K)[i, :nf]), \
                    f"{where}: row {i} ids {pg[i]} differ from the oracle's {po[i]} beyond tied runs"
            pos = {int(f): q for q, f in enumerate(c["f"][j]) if f >= 0}
            for k in range(K):
                f = int(pg[i, k])
                q = pos.get(f)
                ok = q is not None and int(c["cls"][j][q]) != _validity.CLS_BORDER_OUT
                ref_f[i, k] = f
                ref_ok[i, k] = ok
                if ok:
                    ref_z[i, k], ref_w[i, k], ref_d[i, k] = c["z"][j][q], c["bary"][j][q], c["dists"][j][q]
    gz, gw, gd = g["zbuf"].reshape(-1, K), g["bary"].reshape(-1, K, 3), g["dists"].reshape(-1, K)
    # empty slots are exactly -1
    emp = pg < 0
    assert (gz[emp] == -1).all() and (gd[emp] == -1).all() and (gw[emp] == -1).all(), f"{where}: empty slot values"
    valid = ref_ok & (pg >= 0)
    wv = ref_w[valid]
    dw = np.abs(gw[valid] - wv)
    assert (dw <= TOL_VAL * np.maximum(1.0, np.abs(wv))).all(), f"{where}: bary max err {dw.max()}"
    fz = np.asarray(verts, np.float64)[np.asarray(faces)[pg[valid]]][..., 2]  # (n,3) vertex z
    big_w = (np.abs(wv) > 1).any(-1)
    zscale = np.where(big_w, np.abs(wv * fz).sum(-1), 1.0)
    dz = np.abs(gz[valid] - ref_z[valid])
    assert (dz <= TOL_VAL * zscale).all(), f"{where}: zbuf max err {(dz / zscale).max()}"
    dref = ref_d[valid]
    dd = np.abs(gd[valid] - dref)
    assert (dd <= TOL_VAL).all(), f"{where}: dists max err {dd.max()}"
    assert (dd <= TOL_VAL * np.abs(dref) + 1e-12).all(), \
        f"{where}: dists max relative err {(dd / np.maximum(np.abs(dref), 1e-30)).max()}"
    per_bit = {k: float(((amb & v) != 0).mean()) for k, v in oracle.AMB_BITS.items()}
    return dict(amb_frac=float((~strict).mean()), amb_bits=per_bit, checked_flagged=int(flagged.size),
                order_only=n_order_only, slots=int(valid.sum()), rel_branch=int(big_w.sum()),
                bary_err=float(dw.max()) if dw.size else 0.0, z_err=float(dz.max()) if dz.size else 0.0,
                d_err=float(dd.max()) if dd.size else 0.0)


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
