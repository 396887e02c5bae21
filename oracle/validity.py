"""Is a rasterizer's face choice for one pixel a correct answer?

Where the oracle flags a pixel (a decision within the margin tau of flipping,
or depths tied within tau), more than one list of K face ids is correct.
This module decides, from the oracle's candidate list of the pixel (every
face that counts or lies within a margin of counting, with its FP64 depth and
class; ``oracle.candidates``), whether a given list is one of them:

  1. its ids are distinct, each a candidate (a face that counts, or one on
     the margin of counting);
  2. by the oracle's depths it is sorted up to ties: each next depth is at
     least the previous one minus tau;
  3. nothing that must count is missing: every face of class CLS_COUNTS that
     is not listed lies at or beyond the list's last depth minus tau, and
     only when the list is full (K entries);
  4. the candidate list is long enough to decide 1-3.

The exact comparison on unflagged pixels stays in force beside this; here
pixels whose only flag is an order tie inside the first K (M8) must also
match the oracle exactly up to permutations inside each run of tied depths.
Pure NumPy, and test infrastructure like the rest of this package (the
tests and the benchmark's oracle leg use it): the checker itself is tested on
the CPU with mistakes planted into the oracle's own answers.
"""
import numpy as np

TAU = 1e-6
TOL_VAL = 1e-5  # value tolerance of the fragments (bary, zbuf, dists)
CLS_COUNTS, CLS_BORDER_IN, CLS_BORDER_OUT = 0, 1, 2


def valid_choice(ids, cand_f, cand_z, cand_cls, n_cand, K, tau=TAU):
    """None if the list `ids` (K ints, -1 = empty) is a correct answer for a
    pixel with the given candidates (the pixel's rows of
    oracle.candidates), else a string saying why not."""
    ids = [int(x) for x in ids]
    g = [x for x in ids if x >= 0]
    if ids[:len(g)] != g:
        return f"filled slots are not a prefix: {ids}"
    if len(set(g)) != len(g):
        return f"a face appears twice: {g}"
    cap = len(cand_f)
    listed = int(min(n_cand, cap))
    pos = {int(cand_f[j]): j for j in range(listed)}
    for x in g:
        if x not in pos:
            if n_cand > cap:
                return f"face {x} is not among the first {cap} of {n_cand} candidates (list too short to decide)"
            return f"face {x} neither counts nor is within a margin of counting"
    zg = [float(cand_z[pos[x]]) for x in g]
    for k in range(len(zg) - 1):
        if zg[k + 1] < zg[k] - tau:
            return f"slots {k}, {k + 1} out of depth order: {zg[k]!r} > {zg[k + 1]!r}"
    chosen = set(g)
    for j in range(listed):
        if int(cand_cls[j]) != CLS_COUNTS:
            continue
        f = int(cand_f[j])
        if f in chosen:
            continue
        if len(g) < K:
            return f"face {f} counts (z {cand_z[j]!r}) but is missing from a list with room ({len(g)} < {K})"
        if float(cand_z[j]) < zg[-1] - tau:
            return f"face {f} counts and is nearer (z {cand_z[j]!r}) than the list's last ({zg[-1]!r})"
    if n_cand > cap:
        # faces beyond the listed candidates lie at or beyond the last listed depth
        last = float(cand_z[cap - 1])
        if len(g) < K or last < zg[-1] - tau:
            return f"{n_cand} candidates exceed the {cap} listed: cannot show that none is missing"
    return None


def tied_runs(z, tau=TAU):
    """Half-open index ranges of maximal runs of sorted depths whose
    neighbours differ by less than tau."""
    runs, s = [], 0
    for k in range(1, len(z) + 1):
        if k == len(z) or abs(z[k] - z[k - 1]) >= tau:
            runs.append((s, k))
            s = k
    return runs


def equal_up_to_ties(ids, ref_ids, ref_z, tau=TAU):
    """True if `ids` equals the oracle's `ref_ids` except for permutations
    inside runs of tied depths (ref_z, the oracle's sorted depths of its
    filled slots)."""
    ids = [int(x) for x in ids]
    ref = [int(x) for x in ref_ids]
    if len(ids) != len(ref):
        return False
    nf = sum(1 for x in ref if x >= 0)
    if [x >= 0 for x in ids] != [x >= 0 for x in ref]:
        return False
    for s, e in tied_runs([float(v) for v in ref_z[:nf]], tau):
        if sorted(ids[s:e]) != sorted(ref[s:e]):
            return False
    return True


def compare_fragments(g, o, verts, faces, first_idx, num_faces, image_size, blur_radius, where="", pixels=None,
                      options=0, nthreads=None, tol=TOL_VAL):
    """GPU fragments g against the oracle's o (dicts of arrays, rows of the
    same pixels: full images, or the listed `pixels`) for the mesh batch
    (verts, faces, first_idx, num_faces) at the given image size and blur
    radius.  Raises AssertionError on the first violation; returns stats.

    Face ids: exactly the oracle's on unflagged pixels; up to permutations
    inside runs of tied depths where the only flag is such a tie (M8); and on
    every flagged pixel, a correct answer by the oracle's candidate list
    (valid_choice above).  Values of every filled slot against the oracle's
    FP64 values of the same face at the same pixel:
      bary   abs(dw_i) <= 1e-5 * max(1, abs(w_i))
      zbuf   abs(dz)   <= 1e-5, or 1e-5 * sum_i abs(w_i z_i) where some abs(w_i) > 1
      dists  abs(dd)   <= 1e-5 and <= 1e-5 * abs(d) + 1e-12
    """
    from . import AMB_BITS, AMB_M8, candidates
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
    M8 = AMB_M8
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
        c = candidates(verts, faces, first_idx, num_faces, image_size, blur_radius,
                              rows_pix[flagged], cap=cap, nthreads=nthreads, options=options)
        for j, i in enumerate(flagged):
            why = valid_choice(pg[i], c["f"][j], c["z"][j], c["cls"][j], c["n"][j], K)
            assert why is None, f"{where}: row {i} (pixel {rows_pix[i]}, flags {amb[i]:#x}) GPU ids {pg[i]}: {why}"
            if amb[i] == M8:
                n_order_only += 1
                nf = int((po[i] >= 0).sum())
                assert equal_up_to_ties(pg[i], po[i], o["zbuf"].reshape(-1, K)[i, :nf]), \
                    f"{where}: row {i} ids {pg[i]} differ from the oracle's {po[i]} beyond tied runs"
            pos = {int(f): q for q, f in enumerate(c["f"][j]) if f >= 0}
            for k in range(K):
                f = int(pg[i, k])
                q = pos.get(f)
                ok = q is not None and int(c["cls"][j][q]) != CLS_BORDER_OUT
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
    assert (dw <= tol * np.maximum(1.0, np.abs(wv))).all(), f"{where}: bary max err {dw.max()}"
    fz = np.asarray(verts, np.float64)[np.asarray(faces)[pg[valid]]][..., 2]  # (n,3) vertex z
    big_w = (np.abs(wv) > 1).any(-1)
    zscale = np.where(big_w, np.abs(wv * fz).sum(-1), 1.0)
    dz = np.abs(gz[valid] - ref_z[valid])
    assert (dz <= tol * zscale).all(), f"{where}: zbuf max err {(dz / zscale).max()}"
    dref = ref_d[valid]
    dd = np.abs(gd[valid] - dref)
    assert (dd <= tol).all(), f"{where}: dists max err {dd.max()}"
    assert (dd <= tol * np.abs(dref) + 1e-12).all(), \
        f"{where}: dists max relative err {(dd / np.maximum(np.abs(dref), 1e-30)).max()}"
    per_bit = {k: float(((amb & v) != 0).mean()) for k, v in AMB_BITS.items()}
    return dict(amb_frac=float((~strict).mean()), amb_bits=per_bit, checked_flagged=int(flagged.size),
                order_only=n_order_only, slots=int(valid.sum()), rel_branch=int(big_w.sum()),
                bary_err=float(dw.max()) if dw.size else 0.0, z_err=float(dz.max()) if dz.size else 0.0,
                d_err=float(dd.max()) if dd.size else 0.0)
