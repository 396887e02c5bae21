"""Seeded synthetic inputs: icospheres, packed heterogeneous batches, upstream grads.

This module builds *inputs only*.  It holds none of the rasterizer's arithmetic
(no pixel grid, no barycentrics, no distances) and imports nothing else from
this package, so both the HIP path and the FP64 oracle can be fed from it
without sharing any code of the method.

The paper benchmarks the renderer on homogeneous and heterogeneous batches of
ShapeNet meshes (Section 3, "Implementation Details"; Appendix A); ShapeNet is
not available here, so subdivided icospheres stand in for it.  Their template
sizes match the paper's sphere templates (642 verts / 1280 faces and
2562 verts / 5120 faces, Section 4.1), which are icosphere levels 3 and 4.

Coordinates produced here are already in the rasterizer's view space: x, y in
normalised device coordinates and z a depth that is positive in front of the
camera.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "icosphere",
    "Batch",
    "pack",
    "transform_mesh",
    "make_config",
    "upstream_grads",
    "random_rotation",
    "silhouette_fit_problem",
    "CONFIG_NAMES",
]

_PHI = (1.0 + math.sqrt(5.0)) / 2.0


def _icosahedron():
    """12 unit vertices (cyclic permutations of (0, +-1, +-phi)), sorted
    lexicographically, and the 20 faces: vertex triples that are pairwise at
    the minimum distance, oriented so that the normal points away from the
    centre, rotated so the smallest index comes first, then sorted."""
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * _PHI))
            pts.append((s1, s2 * _PHI, 0.0))
            pts.append((s2 * _PHI, 0.0, s1))
    v = np.array(pts, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    order = np.lexsort((v[:, 2], v[:, 1], v[:, 0]))
    v = v[order]
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    dmin = d[d > 1e-9].min()
    adj = np.abs(d - dmin) < 1e-9
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    a, b, c = v[i], v[j], v[k]
                    n = np.cross(b - a, c - a)
                    if np.dot(n, a + b + c) > 0:
                        faces.append((i, j, k))
                    else:
                        faces.append((i, k, j))
    faces = sorted(faces)
    assert len(faces) == 20
    return v, np.array(faces, dtype=np.int64)


def icosphere(level: int):
    """Unit icosphere subdivided ``level`` times.

    Each face (a, b, c) is split into (a, ab, ca), (b, bc, ab), (c, ca, bc),
    (ab, bc, ca); edge midpoints are created once per undirected edge, in the
    order they are first met, and pushed onto the unit sphere.  The result has
    V = 10*4**level + 2 vertices and F = 20*4**level faces, all with outward
    (counter-clockwise seen from outside) winding.  Returns float64 verts and
    int64 faces.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    verts, faces = _icosahedron()
    vlist = [verts]
    nv = verts.shape[0]
    for _ in range(level):
        f = faces
        # undirected edges in first-met order: per face (a,b), (b,c), (c,a)
        e = np.stack([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=1).reshape(-1, 2)
        key = np.minimum(e[:, 0], e[:, 1]) * (1 << 32) + np.maximum(e[:, 0], e[:, 1])
        uniq, first_pos, inv = np.unique(key, return_index=True, return_inverse=True)
        # rank unique edges by first appearance
        order = np.argsort(first_pos, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        mid_id = nv + rank[inv].reshape(-1, 3)  # per face: ab, bc, ca
        allv = np.concatenate(vlist, axis=0)
        ue = np.stack([uniq >> 32, uniq & ((1 << 32) - 1)], axis=1)[order]
        m = 0.5 * (allv[ue[:, 0]] + allv[ue[:, 1]])
        m /= np.linalg.norm(m, axis=1, keepdims=True)
        vlist = [allv, m]
        nv += m.shape[0]
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        ab, bc, ca = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
        nf = np.stack(
            [
                np.stack([a, ab, ca], 1),
                np.stack([b, bc, ab], 1),
                np.stack([c, ca, bc], 1),
                np.stack([ab, bc, ca], 1),
            ],
            axis=1,
        ).reshape(-1, 3)
        faces = nf
    verts = np.concatenate(vlist, axis=0)
    assert verts.shape[0] == 10 * 4**level + 2
    assert faces.shape[0] == 20 * 4**level
    return verts, faces


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised N(0, I4) quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array(
        [
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ]
    )


def transform_mesh(u, noise=None, rot=None, scale=(1.0, 1.0, 1.0), ndc_scale=1.0, offset=(0.0, 0.0), dz=0.0):
    """Per-mesh transform in a fixed order: noise, rotation, per-axis scale,
    xy NDC scale, xy offset, z shift.  Float64 in, float64 out."""
    u = np.array(u, dtype=np.float64, copy=True)
    if noise is not None:
        u = u + noise
    if rot is not None:
        u = u @ np.asarray(rot).T
    u = u * np.asarray(scale, dtype=np.float64)[None, :]
    u[:, :2] *= ndc_scale
    u[:, 0] += offset[0]
    u[:, 1] += offset[1]
    u[:, 2] += dz
    return u


@dataclass
class Batch:
    """A packed heterogeneous mesh batch plus rasterization settings.

    verts: (V,3) float32; faces: (F,3) int32 global vertex ids;
    first_idx / num_faces: (N,) int64 face range of each mesh.
    """

    name: str
    verts: np.ndarray
    faces: np.ndarray
    first_idx: np.ndarray
    num_faces: np.ndarray
    verts_first_idx: np.ndarray
    num_verts: np.ndarray
    image_size: tuple
    faces_per_pixel: int
    blur_radius: float
    bin_size: Optional[int]
    max_faces_per_bin: Optional[int]
    levels: List[int] = field(default_factory=list)
    seed: int = 0
    backward: bool = True

    @property
    def N(self):
        return int(self.first_idx.shape[0])

    @property
    def slots(self):
        H, W = self.image_size
        return self.N * H * W * self.faces_per_pixel


def pack(mesh_list):
    """Concatenate (verts, faces) pairs into the packed layout: faces are offset
    by the running vertex count; returns verts f32, faces i32, first_idx i64,
    num_faces i64, verts_first_idx i64, num_verts i64."""
    vs, fs, fi, nf, vi, nv = [], [], [], [], [], []
    voff = 0
    foff = 0
    for v, f in mesh_list:
        vs.append(np.asarray(v, dtype=np.float64))
        fs.append(np.asarray(f, dtype=np.int64) + voff)
        fi.append(foff)
        nf.append(len(f))
        vi.append(voff)
        nv.append(len(v))
        voff += len(v)
        foff += len(f)
    verts = np.concatenate(vs, 0).astype(np.float32) if vs else np.zeros((0, 3), np.float32)
    faces = np.concatenate(fs, 0).astype(np.int32) if fs else np.zeros((0, 3), np.int32)
    return (
        np.ascontiguousarray(verts),
        np.ascontiguousarray(faces),
        np.array(fi, dtype=np.int64),
        np.array(nf, dtype=np.int64),
        np.array(vi, dtype=np.int64),
        np.array(nv, dtype=np.int64),
    )


_SPHERE_CACHE = {}


def _sphere(level):
    if level not in _SPHERE_CACHE:
        _SPHERE_CACHE[level] = icosphere(level)
    return _SPHERE_CACHE[level]


CONFIG_NAMES = {
    1: "1 x icosphere L2, 64x64, K=1, blur 0, naive, forward only",
    2: "8 x icosphere L4 (rotated), 256x256, K=4, blur 1e-4, bin 32, M 10000",
    3: "32 x icosphere L{2,3,4,5} heterogeneous, 512x512, K=8, blur 1e-4, autotuned",
    4: "4 x icosphere L7, 1024x1024, K=16, blur 1e-5",
    5: "20 views x icosphere L4 silhouette fit, 128x128, K=50, sigma 1e-4",
}

# blur radius of the silhouette-fit config: the squared distance at which
# sigmoid(-d/sigma) falls to 1e-4 for sigma = 1e-4
SIL_SIGMA = 1e-4
SIL_BLUR = math.log(1.0 / 1e-4 - 1.0) * 1e-4


def make_config(i: int, batch: int = 0, level_override: Optional[int] = None,
                image_override: Optional[int] = None, n_override: Optional[int] = None) -> Batch:
    """Synthetic workload i (1..5) for seeded batch ``batch`` (0..4).

    Seed = 1000*i + batch; per-mesh draw order: level, noise (V,3),
    quaternion (4), scales (3), offsets (2), dz (1) -- only the draws that the
    config uses are made.  The *_override arguments shrink a config for quick
    tests (fewer meshes, lower level, smaller image) without changing its
    recipe otherwise.
    """
    seed = 1000 * i + batch
    rng = np.random.default_rng(seed)
    meshes = []
    levels = []
    if i == 1:
        n, lvl, img, K, blur, bs, M = 1, 2, 64, 1, 0.0, 0, None
        for _ in range(n_override or n):
            L = level_override if level_override is not None else lvl
            v, f = _sphere(L)
            noise = rng.standard_normal(v.shape) * 0.01
            meshes.append((transform_mesh(v, noise=noise, ndc_scale=0.8, dz=2.0), f))
            levels.append(L)
        backward = False
    elif i == 2:
        n, lvl, img, K, blur, bs, M = 8, 4, 256, 4, 1e-4, 32, 10000
        for _ in range(n_override or n):
            L = level_override if level_override is not None else lvl
            v, f = _sphere(L)
            noise = rng.standard_normal(v.shape) * 0.01
            R = random_rotation(rng)
            meshes.append((transform_mesh(v, noise=noise, rot=R, ndc_scale=0.8, dz=2.0), f))
            levels.append(L)
        backward = True
    elif i == 3:
        n, img, K, blur, bs, M = 32, 512, 8, 1e-4, None, None
        for _ in range(n_override or n):
            L = int(rng.choice([2, 3, 4, 5]))
            if level_override is not None:
                L = min(L, level_override)
            v, f = _sphere(L)
            noise = rng.standard_normal(v.shape) * 0.02
            R = random_rotation(rng)
            sc = rng.uniform(0.5, 1.0, size=3)
            off = rng.uniform(-0.3, 0.3, size=2)
            dz = rng.uniform(1.5, 3.0)
            meshes.append((transform_mesh(v, noise=noise, rot=R, scale=sc, offset=off, dz=dz), f))
            levels.append(L)
        backward = True
    elif i == 4:
        n, lvl, img, K, blur, bs, M = 4, 7, 1024, 16, 1e-5, None, None
        for _ in range(n_override or n):
            L = level_override if level_override is not None else lvl
            v, f = _sphere(L)
            noise = rng.standard_normal(v.shape) * 0.005
            meshes.append((transform_mesh(v, noise=noise, ndc_scale=0.9, dz=2.0), f))
            levels.append(L)
        backward = True
    elif i == 5:
        prob = silhouette_fit_problem(level=level_override if level_override is not None else 4,
                                      n_views=n_override or 20, seed=seed)
        verts = prob.view_verts(np.zeros_like(prob.base))
        meshes = [(verts[v], prob.faces) for v in range(prob.n_views)]
        levels = [prob.level] * prob.n_views
        img, K, blur, bs, M = 128, 50, SIL_BLUR, None, None
        backward = True
    else:
        raise ValueError(f"unknown config {i}")
    if image_override is not None:
        img = image_override
    verts, faces, fi, nf, vi, nv = pack(meshes)
    return Batch(
        name=f"cfg{i}", verts=verts, faces=faces, first_idx=fi, num_faces=nf,
        verts_first_idx=vi, num_verts=nv, image_size=(img, img), faces_per_pixel=K,
        blur_radius=float(np.float32(blur)), bin_size=bs, max_faces_per_bin=M,
        levels=levels, seed=seed, backward=backward,
    )


def upstream_grads(batch: Batch, seed: Optional[int] = None):
    """Seeded N(0,1) float32 upstream gradients for zbuf, bary, dists, drawn in
    that order from default_rng(seed + 500)."""
    s = (batch.seed if seed is None else seed) + 500
    rng = np.random.default_rng(s)
    H, W = batch.image_size
    shp = (batch.N, H, W, batch.faces_per_pixel)
    gz = rng.standard_normal(shp, dtype=np.float32)
    gb = rng.standard_normal(shp + (3,), dtype=np.float32)
    gd = rng.standard_normal(shp, dtype=np.float32)
    return gz, gb, gd


@dataclass
class SilhouetteFitProblem:
    """Inputs of the silhouette-fitting loop: a unit icosphere template, a
    target shape (the template with a seeded low-frequency radial
    displacement), and the per-view rigid transforms."""

    level: int
    base: np.ndarray          # (V,3) float64 template
    target: np.ndarray        # (V,3) float64 displaced sphere
    faces: np.ndarray         # (F,3) int64
    rotations: np.ndarray     # (n_views,3,3) float64
    n_views: int
    ndc_scale: float = 0.8
    dz: float = 2.0

    def view_verts(self, offsets, use_target=False):
        """(n_views, V, 3) float64 view-space verts of template+offsets (or target)."""
        u = self.target if use_target else self.base + offsets
        out = np.einsum("vij,nj->vni", self.rotations, u)
        out[..., :2] *= self.ndc_scale
        out[..., 2] += self.dz
        return out


def silhouette_fit_problem(level=4, n_views=20, seed=5000, amplitude=0.1):
    """Target radius r(u) = 1 + amplitude * g(u), g(u) = mean_j sin(f_j * (a_j . u) + phi_j)
    with a_j uniform unit vectors, f_j in {1,2,3}, phi_j in [0, 2pi), j = 1..3.
    View v rotates by R_x(30 deg) . R_y(2 pi v / n_views)."""
    rng = np.random.default_rng(seed)
    v, f = icosphere(level)
    a = rng.standard_normal((3, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    freq = rng.integers(1, 4, size=3).astype(np.float64)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=3)
    g = np.mean(np.sin(freq[None, :] * (v @ a.T) + phase[None, :]), axis=1)
    target = v * (1.0 + amplitude * g)[:, None]
    el = math.radians(30.0)
    Rx = np.array([[1, 0, 0], [0, math.cos(el), -math.sin(el)], [0, math.sin(el), math.cos(el)]])
    rots = []
    for k in range(n_views):
        az = 2.0 * math.pi * k / n_views
        Ry = np.array([[math.cos(az), 0, math.sin(az)], [0, 1, 0], [-math.sin(az), 0, math.cos(az)]])
        rots.append(Rx @ Ry)
    return SilhouetteFitProblem(level=level, base=v, target=target, faces=f,
                                rotations=np.stack(rots), n_views=n_views)


# ---------------------------------------------------------------- point clouds

POINT_CONFIG_NAMES = {
    1: "1 cloud x 2,000 points, 64x64, K=8, radius 0.05",
    2: "4 clouds x {1k, 3k, 5k, 8k} points, 96x96, K=16, radius 0.03",
    3: "8 clouds x 200,000 points, 256x256, K=50, radius 0.01",
}


@dataclass
class PointBatch:
    """A packed heterogeneous point-cloud batch plus rasterization settings.

    points: (P,3) float32, x and y in NDC, z the depth; first_idx /
    num_points: (N,) int64 point range of each cloud."""

    name: str
    points: np.ndarray
    first_idx: np.ndarray
    num_points: np.ndarray
    image_size: Tuple[int, int]
    points_per_pixel: int
    radius: float
    seed: int

    @property
    def N(self) -> int:
        return int(self.first_idx.shape[0])


def sample_surface(level: int, n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniformly distributed over the surface of the level-`level`
    icosphere (faces chosen with probability proportional to their area,
    then a uniform point in the face).  Float64 (n,3)."""
    v, f = icosphere(level)
    tri = v[f]
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    face = rng.choice(f.shape[0], size=n, p=area / area.sum())
    r1 = np.sqrt(rng.uniform(size=n))
    r2 = rng.uniform(size=n)
    a, b, c = tri[face, 0], tri[face, 1], tri[face, 2]
    return (1 - r1)[:, None] * a + (r1 * (1 - r2))[:, None] * b + (r1 * r2)[:, None] * c


def make_points_config(i: int, batch: int = 0, n_override: Optional[int] = None,
                       image_override: Optional[int] = None, points_override: Optional[int] = None) -> PointBatch:
    """Seeded synthetic point-cloud workloads: clouds sampled from sphere
    surfaces (a stand-in for points sampled from ShapeNet meshes), each with a
    random rotation, xy scaled into NDC and z shifted in front of the camera.
    Seed 7000 + 100 * i + batch; per cloud the draws are: size, surface
    samples, rotation, xy offset, z shift."""
    seed = 7000 + 100 * i + batch
    rng = np.random.default_rng(seed)
    if i == 1:
        sizes, img, K, radius, ndc = [2000], 64, 8, 0.05, 0.8
    elif i == 2:
        sizes, img, K, radius, ndc = [1000, 3000, 5000, 8000], 96, 16, 0.03, 0.7
    elif i == 3:
        sizes, img, K, radius, ndc = [200000] * 8, 256, 50, 0.01, 0.8
    else:
        raise ValueError(f"unknown point config {i}")
    if n_override is not None:
        sizes = (sizes * n_override)[:n_override]
    if points_override is not None:
        sizes = [points_override] * len(sizes)
    clouds = []
    for n in sizes:
        u = sample_surface(3, n, rng)
        R = random_rotation(rng)
        off = rng.uniform(-0.1, 0.1, size=2)
        dz = rng.uniform(1.8, 2.2)
        clouds.append(transform_mesh(u, rot=R, ndc_scale=ndc, offset=off, dz=dz))
    pts = np.concatenate(clouds).astype(np.float32)
    num = np.array(sizes, dtype=np.int64)
    first = np.concatenate([[0], np.cumsum(num)[:-1]]).astype(np.int64)
    if image_override is not None:
        img = image_override
    return PointBatch(name=f"pts{i}", points=pts, first_idx=first, num_points=num, image_size=(img, img),
                      points_per_pixel=K, radius=float(np.float32(radius)), seed=seed)


def point_grads(batch: PointBatch, channels: int = 3):
    """Seeded float32 inputs of the point backward and compositing tests:
    upstream gradients for zbuf and dists (N,H,W,K), per-point features
    (P, channels) in [0, 1), and an upstream gradient of the composited image
    (N,H,W,channels); drawn in that order from default_rng(seed + 500)."""
    rng = np.random.default_rng(batch.seed + 500)
    H, W = batch.image_size
    shp = (batch.N, H, W, batch.points_per_pixel)
    gz = rng.standard_normal(shp, dtype=np.float32)
    gd = rng.standard_normal(shp, dtype=np.float32)
    feat = rng.uniform(size=(batch.points.shape[0], channels)).astype(np.float32)
    gimg = rng.standard_normal((batch.N, H, W, channels), dtype=np.float32)
    return gz, gd, feat, gimg
