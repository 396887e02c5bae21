"""Pins of the oracle's decision-margin bits and candidate lists.

Every bit of the ambiguity mask (tau = 1e-6 in linear NDC units) gets a hand
case where it must fire and near misses, 2e-6 on either side of the
decision, where it must stay clear.  Expected values follow from the closed
forms of triangle T (see test_oracle_pins): w(x,y) = (-(x+y)/2, (x+1)/2,
(y+1)/2), z = (x + 2y + 5)/2, nearest-edge squared distances (y+1)^2,
(x+y)^2/2, (x+1)^2 on edges (a,b), (b,c), (c,a).

The second half checks the validity checker of tests/_validity.py against
mistakes planted into the oracle's own answers on the CPU.
"""
import math

import numpy as np
import pytest

from oracle import validity as _validity
import oracle

T_VERTS = np.array([[-1.0, -1.0, 1.0], [1.0, -1.0, 2.0], [-1.0, 1.0, 3.0]])
T_FACES = np.array([[0, 1, 2]])
M1, M2, M3, M4, M5, M7, M8 = (oracle.AMB_BITS[k] for k in ("M1", "M2", "M3", "M4", "M5", "M7", "M8"))


def centers(n):
    return [1.0 - (2 * i + 1) / n for i in range(n)]


def raster(v, f, blur, K=1, size=4, options=0):
    return oracle.rasterize(v, f, [0], [len(f)], (size, size), blur, K, options=options)


def cands(v, f, blur, pix, options=0, size=4):
    return oracle.candidates(v, f, [0], [len(f)], (size, size), blur, np.asarray(pix), cap=8, options=options)


# ------------------------------------------------------------------ M1

@pytest.mark.parametrize("shift,fires", [(1e-6, True), (3e-6, False)])
def test_M1_edge_within_tau_at_zero_blur(shift, fires):
    # T moved by +shift in x: its edge (b, c) is the line x + y = shift, so the
    # four centres on x + y = 0 lie inside, shift/sqrt(2) from the edge
    v = T_VERTS + [shift, 0.0, 0.0]
    o = raster(v, T_FACES, 0.0)
    on = [(0, 3), (1, 2), (2, 1), (3, 0)]
    for r in range(4):
        for c in range(4):
            exp = M1 if (fires and (r, c) in on) else 0
            assert o["amb"][0, r, c] == exp, (r, c, o["amb"][0, r, c])
    for r, c in on:  # inside either way: T is the answer
        assert o["p2f"][0, r, c, 0] == 0
    ca = cands(v, T_FACES, 0.0, [0 * 16 + 0 * 4 + 3])
    assert ca["n"][0] == 1 and ca["cls"][0, 0] == (oracle.CLS_BORDER_IN if fires else oracle.CLS_COUNTS)


# ------------------------------------------------------------------ M2

@pytest.mark.parametrize("delta,fires,counts", [(0.0, True, False), (2e-6, False, True), (-2e-6, False, False)])
def test_M2_distance_within_tau_of_blur_radius(delta, fires, counts):
    # pixels (0,1) and (1,0) are outside T at squared distance 1/2 exactly
    # (nearest point (-1/4, 1/4) resp. (1/4, -1/4) on edge (b, c)); the blur
    # radius is put at linear distance sqrt(1/2) + delta (exactly 1/2 for delta 0)
    blur = 0.5 if delta == 0.0 else (math.sqrt(0.5) + delta) ** 2
    o = raster(T_VERTS, T_FACES, blur)
    for r in range(4):
        for c in range(4):
            exp = M2 if (fires and (r, c) in [(0, 1), (1, 0)]) else 0
            assert o["amb"][0, r, c] == exp, (r, c, o["amb"][0, r, c])
    for r, c in [(0, 1), (1, 0)]:
        assert (o["p2f"][0, r, c, 0] == 0) == counts
        assert o["dists"][0, r, c, 0] == (0.5 if counts else -1.0)
    ca = cands(T_VERTS, T_FACES, blur, [1])  # pixel (0,1)
    if fires:
        assert ca["n"][0] == 1 and ca["f"][0, 0] == 0 and ca["cls"][0, 0] == oracle.CLS_BORDER_OUT
        assert ca["dists"][0, 0] == 0.5 and ca["z"][0, 0] == (0.25 + 1.5 + 5) / 2
    else:
        assert ca["n"][0] == (1 if counts else 0)
        if counts:
            assert ca["cls"][0, 0] == oracle.CLS_COUNTS


# ------------------------------------------------------------------ M3 / M8

# T2 covers every pixel centre of a 4x4 image at a constant depth z2.
T2 = np.array([[-3.0, -1.5, 0.0], [3.0, -1.5, 0.0], [0.0, 3.0, 0.0]])


def with_T2(z2):
    v = np.concatenate([T_VERTS, T2 + [0.0, 0.0, z2]])
    return v, np.array([[0, 1, 2], [3, 4, 5]])


def tied_pixels(blur):
    # centres where T counts with z = 17/8 (x + 2y = -3/4): (2,2) inside, and
    # (3,0) on T's edge, which counts under blur
    out = []
    for r, y in enumerate(centers(4)):
        for c, x in enumerate(centers(4)):
            w = (-(x + y) / 2, (x + 1) / 2, (y + 1) / 2)
            d2 = min((y + 1) ** 2, (x + y) ** 2 / 2, (x + 1) ** 2)
            if (min(w) > 0 or d2 < blur) and (x + 2 * y + 5) / 2 == 17 / 8:
                out.append((r, c))
    return out


@pytest.mark.parametrize("dz,tie", [(5e-7, True), (-5e-7, True), (2e-6, False), (-2e-6, False)])
def test_M3_set_tie_and_M8_order_tie(dz, tie):
    blur = 0.2
    v, f = with_T2(17 / 8 + dz)
    tp = tied_pixels(blur)
    assert tp == [(2, 2), (3, 0)]
    k1 = raster(v, f, blur, K=1)
    k2 = raster(v, f, blur, K=2)
    k3 = raster(v, f, blur, K=3)
    for r in range(4):
        for c in range(4):
            t = tie and (r, c) in tp
            # K = 1: the tie decides which face is kept (M3); K = 2: both are
            # kept and only their order is tied (M8); K = 3: likewise
            assert k1["amb"][0, r, c] == (M3 if t else 0), (r, c)
            assert k2["amb"][0, r, c] == (M8 if t else 0), (r, c)
            assert k3["amb"][0, r, c] == (M8 if t else 0), (r, c)
    # the oracle's order is still (z, id)
    for r, c in tp:
        exp = [0, 1] if dz > 0 else [1, 0]
        assert list(k2["p2f"][0, r, c]) == exp


def test_M3_only_at_the_set_boundary():
    # three faces at one pixel: T (z 17/8) and two copies of T2 at 17/8 + 5e-7
    # and 17/8 + 3e-6.  K = 1: T and the first copy tie at the boundary (M3).
    # K = 2: the boundary pair (first copy, second copy) is 2.5e-6 apart; the
    # tie is inside the first two: M8 only.  K = 3: M8 only.
    v = np.concatenate([T_VERTS, T2 + [0, 0, 17 / 8 + 5e-7], T2 + [0, 0, 17 / 8 + 3e-6]])
    f = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
    amb = {K: raster(v, f, 0.2, K=K)["amb"][0, 2, 2] for K in (1, 2, 3)}
    assert amb == {1: M3, 2: M8, 3: M8}


# ------------------------------------------------------------------ M4

@pytest.mark.parametrize("z0,fires,counts", [(5e-7, True, True), (-5e-7, True, False), (2e-6, False, True),
                                             (-2e-6, False, False)])
def test_M4_depth_within_tau_of_zero(z0, fires, counts):
    # T lowered so that its depth at pixel (2,2) is z0 (T's depth there is 17/8)
    v = T_VERTS - [0.0, 0.0, 17 / 8 - z0]
    o = raster(v, T_FACES, 0.0)
    assert o["amb"][0, 2, 2] == (M4 if fires else 0)
    assert (o["p2f"][0, 2, 2, 0] == 0) == counts
    # (3,0) has the same depth (x + 2y = -3/4) but lies on T's edge, which at
    # zero blur is M1 as well -- unless its depth keeps it out either way;
    # every other pixel has |z| >= 1/8 - |z0|
    assert o["amb"][0, 3, 0] == (M1 | M4 if fires else (M1 if z0 > 0 else 0))
    others = np.ones((4, 4), bool)
    others[2, 2] = others[3, 0] = False
    assert ((o["amb"][0] & M4)[others] == 0).all()
    ca = cands(v, T_FACES, 0.0, [2 * 4 + 2])
    if fires:
        assert ca["n"][0] == 1
        assert ca["cls"][0, 0] == (oracle.CLS_BORDER_IN if counts else oracle.CLS_BORDER_OUT)
    else:
        assert ca["n"][0] == (1 if counts else 0)


# ------------------------------------------------------------------ M5

@pytest.mark.parametrize("rel,fires,counts", [(5e-4, True, True), (-5e-4, True, False), (1e-2, False, True),
                                              (-1e-2, False, False)])
def test_M5_area_near_the_degeneracy_threshold(rel, fires, counts):
    # a tiny right triangle at the centre of pixel (2,2), legs 1e-4 and
    # 1e-4 (1 + rel): doubled area 1e-8 (1 + rel); with blur 0.2 it counts
    # (unless degenerate) at that pixel only, the others being >= 1/2 away
    p = (-0.25, -0.25)
    v = np.array([[p[0], p[1], 1.0], [p[0] + 1e-4, p[1], 1.0], [p[0], p[1] + 1e-4 * (1 + rel), 1.0]])
    E = (v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1])
    assert abs(E / 1e-8 - (1 + rel)) < 1e-9
    o = raster(v, T_FACES, 0.2)
    for r in range(4):
        for c in range(4):
            assert o["amb"][0, r, c] == (M5 if (fires and (r, c) == (2, 2)) else 0), (r, c)
    assert (o["p2f"][0, 2, 2, 0] == 0) == counts
    ca = cands(v, T_FACES, 0.2, [10])
    if fires:
        assert ca["n"][0] == 1
        assert ca["cls"][0, 0] == (oracle.CLS_BORDER_IN if counts else oracle.CLS_BORDER_OUT)
    else:
        assert ca["n"][0] == (1 if counts else 0)


def test_M5_not_raised_by_a_face_far_from_the_pixel():
    # the same near-threshold triangle far from every centre but (2,2): only
    # that pixel is flagged, never the whole image
    p = (-0.25, -0.25)
    v = np.array([[p[0], p[1], 1.0], [p[0] + 1e-4, p[1], 1.0], [p[0], p[1] + 1e-4 * (1 - 5e-4), 1.0]])
    o = raster(v, T_FACES, 0.0, size=16)
    assert (o["amb"] == 0).all()  # blur 0: the degenerate face would count nowhere


# ------------------------------------------------------------------ M7

@pytest.mark.parametrize("z0,fires", [(5e-7, True), (2e-6, False)])
def test_M7_vertex_depth_near_zero_under_perspective(z0, fires):
    v = T_VERTS.copy()
    v[0, 2] = z0
    PC = oracle.PERSPECTIVE_CORRECT
    o = raster(v, T_FACES, 0.0, options=PC)
    plain = raster(v, T_FACES, 0.0)
    inside = [(1, 3), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)]
    for r, c in inside:
        assert bool(o["amb"][0, r, c] & M7) == fires, (r, c)
        assert plain["amb"][0, r, c] & M7 == 0
    # pixels T does not cover are never flagged M7
    for r, c in [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0)]:
        assert o["amb"][0, r, c] & M7 == 0


# ------------------------------------------------------------------ M6

@pytest.mark.parametrize("shift,tie", [(0.0, True), (5e-7, True), (2e-6, False)])
def test_M6_edge_tie_at_pixel_3_3(shift, tie):
    # at (3,3), p = (-3/4, -3/4): edges (a,b) (y = -1) and (c,a) (x = -1) are
    # both 1/4 away; moving a and c to x = -1 - shift puts edge (c,a) at
    # 1/4 + shift.  At (2,2) the nearest edge, (b,c) at sqrt(1/8), is alone.
    v = T_VERTS.copy()
    v[[0, 2], 0] -= shift
    p2f = np.full((1, 4, 4, 1), -1)
    p2f[0, 3, 3, 0] = 0
    p2f[0, 2, 2, 0] = 0
    _, _, _, t = oracle.fragments_fixed(v, T_FACES, (4, 4), p2f)
    assert t[0, 3, 3, 0] == (1 if tie else 0)
    assert t[0, 2, 2, 0] == 0


# ------------------------------------------------------------------ candidates

def test_candidates_equal_the_forward_on_counting_faces():
    rng = np.random.default_rng(3)
    from test_oracle_pins import random_soup
    v, f, fi, nf = random_soup(rng)
    H, W = 24, 20
    full = oracle.rasterize(v, f, fi, nf, (H, W), 2e-2, 64)
    pix = np.arange(fi.shape[0] * H * W)
    c = oracle.candidates(v, f, fi, nf, (H, W), 2e-2, pix, cap=64)
    cnt = c["cls"] != 255
    counting = cnt & (c["cls"] != oracle.CLS_BORDER_OUT)
    fp = full["p2f"].reshape(-1, 64)
    for i in range(pix.size):
        assert list(c["f"][i][counting[i]]) == list(fp[i][fp[i] >= 0])
    assert (full["nhits"].reshape(-1) <= c["n"]).all()


# ------------------------------------------------------------------ the validity checker, with planted mistakes

def oracle_view(K=4, blur=2e-2, seed=11):
    from test_oracle_pins import random_soup
    rng = np.random.default_rng(seed)
    v, f, fi, nf = random_soup(rng)
    H, W = 24, 20
    o = oracle.rasterize(v, f, fi, nf, (H, W), blur, K)
    pix = np.arange(fi.shape[0] * H * W)
    c = oracle.candidates(v, f, fi, nf, (H, W), blur, pix, cap=2 * K + 32)
    return o, c, K


def test_checker_accepts_the_oracle_and_rejects_planted_mistakes():
    o, c, K = oracle_view()
    p2f = o["p2f"].reshape(-1, K)
    nh = o["nhits"].reshape(-1)
    checked = {"swap": 0, "drop": 0, "foreign": 0, "dup": 0, "short": 0}
    rng = np.random.default_rng(0)
    for i in range(p2f.shape[0]):
        args = (c["f"][i], c["z"][i], c["cls"][i], c["n"][i], K)
        assert _validity.valid_choice(p2f[i], *args) is None, i
        zs = c["z"][i]
        filled = int((p2f[i] >= 0).sum())
        if filled >= 2:
            z0 = zs[list(c["f"][i]).index(p2f[i, 0])]
            z1 = zs[list(c["f"][i]).index(p2f[i, 1])]
            bad = p2f[i].copy()
            bad[[0, 1]] = bad[[1, 0]]
            if z1 - z0 >= 1e-6:
                assert _validity.valid_choice(bad, *args) is not None
                checked["swap"] += 1
            bad = p2f[i].copy()
            bad[1] = bad[0]
            assert _validity.valid_choice(bad, *args) is not None
            checked["dup"] += 1
        if filled >= 1:
            # a face of the same mesh that does not count here
            n = i // (24 * 20)
            others = np.setdiff1d(np.arange(o["p2f"].max() + 1), c["f"][i])
            if others.size:
                bad = p2f[i].copy()
                bad[filled - 1] = rng.choice(others)
                assert _validity.valid_choice(bad, *args) is not None
                checked["foreign"] += 1
            # dropping the last face leaves room for a face that counts
            bad = p2f[i].copy()
            bad[filled - 1] = -1
            assert _validity.valid_choice(bad, *args) is not None
            checked["short"] += 1
        if nh[i] > K:
            # replacing the K-th by the (K+1)-th is only right when they tie
            counting = [int(x) for x, cl in zip(c["f"][i], c["cls"][i]) if cl in (0, 1)]
            bad = p2f[i].copy()
            bad[K - 1] = counting[K]
            zK1, zK = zs[K - 1], zs[K]
            if zK - zK1 >= 1e-6:
                assert _validity.valid_choice(bad, *args) is not None
                checked["drop"] += 1
    assert min(checked.values()) > 20, checked


def test_checker_accepts_tie_swaps_and_border_faces():
    # T and a copy of T2 tied within tau at pixel (2,2); K = 1: either face
    v, f = with_T2(17 / 8 + 5e-7)
    c = cands(v, f, 0.2, [10])
    args = (c["f"][0], c["z"][0], c["cls"][0], c["n"][0], 1)
    assert _validity.valid_choice([0], *args) is None
    assert _validity.valid_choice([1], *args) is None
    # not tied: only the nearer one
    v, f = with_T2(17 / 8 + 2e-6)
    c = cands(v, f, 0.2, [10])
    args = (c["f"][0], c["z"][0], c["cls"][0], c["n"][0], 1)
    assert _validity.valid_choice([0], *args) is None
    assert _validity.valid_choice([1], *args) is not None
    # a face on the blur margin may be taken or left (M2 case at pixel (0,1))
    c = cands(T_VERTS, T_FACES, 0.5, [1])
    args = (c["f"][0], c["z"][0], c["cls"][0], c["n"][0], 1)
    assert _validity.valid_choice([0], *args) is None
    assert _validity.valid_choice([-1], *args) is None
    # equal_up_to_ties: permutations inside a tied run only
    assert _validity.equal_up_to_ties([1, 0, 2], [0, 1, 2], [1.0, 1.0 + 5e-7, 2.0])
    assert not _validity.equal_up_to_ties([0, 2, 1], [0, 1, 2], [1.0, 1.0 + 5e-7, 2.0])
