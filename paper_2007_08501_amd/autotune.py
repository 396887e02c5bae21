"""Autotuner for the forward's bin size, bin capacity and scheduler.

For each candidate bin size the counting pass gives the exact largest bin
count, which sizes max_faces_per_bin (rounded up to 32); each candidate
(bin size, scheduler) is then timed forward+backward with HIP events on the
current stream, all candidates in turn in each of several rounds (the median
per candidate), and the fastest is cached per device and problem signature
(image size, K, blur, face count, spread of faces per mesh).  The
single-pass form (bin_size 0) is a candidate when its work is small.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, dataclass
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import _lib
from .raster import count_max_faces_per_bin, empty_fragments, forward_into, round_up, workspace

DEFAULT_BIN_SIZES = (8, 16, 24, 32, 48, 64)


@dataclass
class Choice:
    bin_size: int
    max_faces_per_bin: int
    sched: int
    ms: float


_cache: Dict[str, Choice] = {}


def _cache_path() -> Optional[str]:
    return os.environ.get("RAST_AUTOTUNE_CACHE")


def _load_file():
    p = _cache_path()
    if p and os.path.exists(p):
        try:
            with open(p) as fh:
                for k, v in json.load(fh).items():
                    _cache.setdefault(k, Choice(**v))
        except (OSError, ValueError, TypeError):
            pass


def _save_file():
    p = _cache_path()
    if p:
        tmp = p + ".tmp"
        with open(tmp, "w") as fh:
            json.dump({k: asdict(v) for k, v in _cache.items()}, fh, indent=1)
        os.replace(tmp, p)


def signature(verts, faces, first_idx, num_faces, H, W, blur, K) -> str:
    dev = torch.cuda.get_device_name(verts.device)
    nf = num_faces.detach().to("cpu", torch.float64)
    mean = float(nf.mean()) if nf.numel() else 0.0
    spread = float(nf.std()) / mean if nf.numel() > 1 and mean > 0 else 0.0
    bucket = int(round(math.log2(max(mean, 1.0)) * 2)), int(round(spread * 4))
    return f"{dev}|N{first_idx.shape[0]}|{H}x{W}|K{K}|b{blur:.3e}|F{faces.shape[0]}|h{bucket[0]}.{bucket[1]}"


def _prepare_candidate(verts, faces, first_idx, num_faces, H, W, blur, K, bs, M, sched, grads, out, gv, ws):
    """One forward(+backward) step of a candidate into the given outputs and
    workspace, run once (None if the candidate reports an error, e.g. a bin
    overflow)."""
    def step():
        forward_into(verts, faces, first_idx, num_faces, H, W, blur, K, bs, M, sched, out, ws)
        if grads is not None:
            _lib.rasterize_meshes_bwd(verts, faces, first_idx, num_faces, H, W, blur, K, bs, M,
                                      _lib.RAST_BWD_REUSE_FORWARD, out.pix_to_face, grads[0], grads[1], grads[2], gv,
                                      ws)

    step()
    st, _ = _lib.rast_query_status(ws)
    return step if st == _lib.RAST_OK else None


def _time_step(step) -> float:
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    step()
    b.record()
    b.synchronize()
    return a.elapsed_time(b)


def _time_candidates(verts, faces, first_idx, num_faces, H, W, blur, K, cands, grads, reps):
    """Median time of each candidate (inf if it fails), the candidates timed in
    turn within each of reps rounds, after one untimed round: a drift of the
    clock over the tuning (the GPU ramping up) then affects every candidate
    alike instead of penalising the first ones.  The steps run one after the
    other on the current stream, so they share the output buffers (and the
    device's scratch workspace, while it is large enough)."""
    N = first_idx.shape[0]
    out = empty_fragments(N, H, W, K, verts.device)
    gv = torch.empty_like(verts)
    steps = []
    for bs, M, sc in cands:
        ws = workspace(verts.device, _lib.rast_workspace_size(N, H, W, faces.shape[0], bs, M))
        steps.append(_prepare_candidate(verts, faces, first_idx, num_faces, H, W, blur, K, bs, M, sc, grads, out, gv,
                                        ws))
    for step in steps:
        if step is not None:
            step()
    times = [[] for _ in cands]
    for _ in range(reps):
        for i, step in enumerate(steps):
            if step is not None:
                times[i].append(_time_step(step))
    return [sorted(t)[len(t) // 2] if t else float("inf") for t in times]


def autotune(verts, faces, first_idx, num_faces, H, W, blur, K, bin_sizes: Iterable[int] = DEFAULT_BIN_SIZES,
             scheds: Tuple[int, ...] = (_lib.RAST_SCHED_GRID, _lib.RAST_SCHED_PERSISTENT), backward: bool = True,
             reps: int = 5, include_single_pass: Optional[bool] = None, max_list_bytes: int = 1 << 31,
             force: bool = False) -> Choice:
    """Pick (bin_size, max_faces_per_bin, sched) for this problem; cached."""
    if not _cache:
        _load_file()
    key = signature(verts, faces, first_idx, num_faces, H, W, blur, K) + ("|bwd" if backward else "")
    if not force and key in _cache:
        return _cache[key]
    N = first_idx.shape[0]
    grads = None
    if backward:
        g = torch.Generator(device=verts.device)
        g.manual_seed(0)
        shp = (N, H, W, K)
        grads = (torch.randn(shp, device=verts.device, generator=g),
                 torch.randn(shp + (3,), device=verts.device, generator=g),
                 torch.randn(shp, device=verts.device, generator=g))
    if include_single_pass is None:
        # every pixel against every face of its mesh: affordable only when small
        work = float(H * W) * float(faces.shape[0])
        include_single_pass = work <= 2e9
    best = None
    cands = []
    if include_single_pass:
        cands.append((0, 0, _lib.RAST_SCHED_GRID))
    for bs in bin_sizes:
        if bs > max(H, W) * 2 or bs % _lib.RAST_TILE:
            continue
        mx = count_max_faces_per_bin(verts, faces, first_idx, num_faces, H, W, blur, bs)
        M = round_up(mx, 32)
        nbins = N * ((H + bs - 1) // bs) * ((W + bs - 1) // bs)
        if nbins * M * 4 > max_list_bytes:
            continue
        for sc in scheds:
            cands.append((bs, M, sc))
    for (bs, M, sc), ms in zip(cands, _time_candidates(verts, faces, first_idx, num_faces, H, W, blur, K, cands,
                                                        grads, reps)):
        if best is None or ms < best.ms:
            best = Choice(bs, M, sc, ms)
    if best is None:
        raise RuntimeError("autotune found no feasible configuration")
    _cache[key] = best
    _save_file()
    return best
