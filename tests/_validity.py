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
Pure NumPy: the checker itself is tested on the CPU with mistakes planted
into the oracle's own answers.
"""
import numpy as np

TAU = 1e-6
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
