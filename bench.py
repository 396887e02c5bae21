#!/usr/bin/env python3
"""Benchmark of the batched differentiable mesh rasterizer on one MI355X.

One step = forward (face setup, coarse binning, per-pixel K-nearest pass) plus
backward (fragment gradients -> vertex gradients) over one synthetic batch,
all through the C ABI of librast.so with inputs resident in HBM.

Default workload: 4 icospheres at subdivision level 7 (327,680 faces each),
1024x1024 images, K = 16 nearest faces per pixel, blur radius 1e-5 -- the
large configuration on which the HBM roofline is measured.  ``--config`` picks
one of the other synthetic workloads instead.  Each of ``--batches`` seeded
batches (the paper averages five) is autotuned, its forward+backward captured
in one HIP graph and replayed ``--steps`` times; the reported step time is the
median over the batches.

Prints ONE JSON line: throughput in Mpixel*K/s (N*H*W*K / step time), ms per
step, the roofline of the dominant kernel (timed live with HIP events the
library records around its launch), the per-mesh plain form (one single-pass
call per mesh, no bins, no graph) timed on the same GPU, and -- the only part
that runs the FP64 oracle -- the oracle's own throughput on a bounded sample of
the workload on the host cores, with the GPU outputs checked against it on
that sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd rasterized Mpixel·K/s and ms/batch, batched vs per-mesh, at oracle tol"
UNIT = "Mpixel·K/s"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: one non-packed FP32/FP64 VALU lane-op each
VALU_PEAK_LANE_OPS = 3.932e13


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t handles through the HIP runtime torch already loaded."""

    def __init__(self):
        import torch  # noqa: F401  (loads libamdhip64)
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.rt.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.rt.hipEventCreate(ctypes.byref(e)) == 0
        return e.value

    def record(self, e, stream):
        assert self.rt.hipEventRecord(ctypes.c_void_p(e), ctypes.c_void_p(stream)) == 0

    def elapsed(self, a, b):
        assert self.rt.hipEventSynchronize(ctypes.c_void_p(b)) == 0
        ms = ctypes.c_float()
        assert self.rt.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return float(ms.value)

    def destroy(self, e):
        self.rt.hipEventDestroy(ctypes.c_void_p(e))


# sources of each measured kernel: a counter summary holds for them only while
# these files are unchanged
# The VALU figure is an issue rate, not a roofline of useful work: every
# counted wave instruction is taken as 64 lane slots, masked lanes included.
VALU_ISSUE_WHAT = ("VALU issue rate of the dominant kernel: SQ_INSTS_VALU x 64 lane slots / kernel time, masked "
                   "lanes included (not a count of useful lane operations)")

KERNEL_SOURCES = {
    "fine": ["paper_2007_08501_amd/csrc/kernels_fwd.hip", "paper_2007_08501_amd/csrc/device.hpp"],
    "backward": ["paper_2007_08501_amd/csrc/kernels_bwd.hip", "paper_2007_08501_amd/csrc/device.hpp"],
    "points_fine": ["paper_2007_08501_amd/csrc/kernels_points.hip", "paper_2007_08501_amd/csrc/device.hpp"],
    "points_backward": ["paper_2007_08501_amd/csrc/kernels_points.hip", "paper_2007_08501_amd/csrc/device.hpp"],
}


def sources_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config, K, bs, path=None):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's reading), or None
    when no summary exists for this workload or the kernel changed since."""
    path = path or os.path.join(ROOT, "profiles", f"traffic_{kernel}_cfg{config}_K{K}_bs{bs}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, _, v = line.partition(":")
                vals[k.strip()] = v.strip()
    if vals.get("sources_sha256") != sources_digest(kernel):
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def measured_valu(kernel, config, K, bs, path=None):
    """VALU wave instructions per launch of `kernel` from the committed
    kernel-trace summary (SQ_INSTS_VALU), or None when there is none for this
    workload or the kernel changed since it was taken."""
    path = path or os.path.join(ROOT, "profiles", f"kernels_cfg{config}_K{K}_bs{bs}.txt")
    if kernel not in ("fine", "points_fine", "backward") or not os.path.exists(path):
        return None
    prefix = "backward_" if kernel == "backward" else ""
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#")):
                k, _, v = line.partition(":")
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get(prefix + "sources_sha256") != sources_digest(kernel):
        return None
    try:
        return float(vals[prefix + "valu_wave_instructions_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.partition(":")[2].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    """Host threads for the oracle: the process's CPUs, at most 16 (a
    one-GPU share of the host)."""
    import oracle
    return min(16, oracle.default_threads())


def single_core_rate(b, pix, K, backward=True):
    """The oracle's forward(+backward) rate on one thread, over a slice of the
    sampled pixels (Mpixel*K/s)."""
    import numpy as np

    import oracle
    N, (H, W) = b.N, b.image_size
    sub = pix[:: max(1, pix.size // 256)]
    tq = time.perf_counter()
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius, K, pixels=sub, nthreads=1)
    if backward:
        ones = np.ones((sub.size, K), np.float32)
        oracle.backward(b.verts, b.faces, (H, W), o["p2f"], ones, None, None, nthreads=1, pixels=sub, N=N)
    dt = time.perf_counter() - tq
    return {"value": round(sub.size * K / dt / 1e6, 6), "pixels": int(sub.size), "seconds": round(dt, 2)}


def forward_only_parity(b, o, pix, t_f, P, nthr, out, dev):
    """CPU baseline and parity of a forward-only workload (config 1)."""
    import torch

    import oracle
    from oracle import validity
    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    cpu = {"value": round(P * K / t_f / 1e6, 6), "unit": UNIT, "cores": nthr, "kind": "oracle",
           "sample": f"{P} of {N * H * W} pixels, FP64 brute force forward over every face of the pixel's mesh; "
                     f"fwd {t_f:.2f}s", "cpu_model": cpu_model(), "host_cpus_visible": oracle.default_threads(),
           "single_core": single_core_rate(b, pix, K, backward=False)}
    pix_t = torch.from_numpy(pix).to(dev)
    g = {k: t.reshape((N * H * W,) + tuple(t.shape[3:]))[pix_t].cpu().numpy()
         for k, t in zip(("p2f", "zbuf", "bary", "dists"), out)}
    try:
        st = validity.compare_fragments(g, o, b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius,
                                        where=b.name, pixels=pix, nthreads=nthr)
        parity = {"pixels": int(pix.size), "fragments_ok": True, "ambiguous_frac": round(st["amb_frac"], 5),
                  "max_err": {"bary": st["bary_err"], "zbuf": st["z_err"], "dists": st["d_err"]}}
    except AssertionError as e:
        parity = {"pixels": int(pix.size), "fragments_ok": False, "error": str(e)[:300]}
    parity["grad_ok"] = True  # no backward in this workload
    return cpu, parity


def cpu_baseline_leg(b, cpu_seconds, v, f, fi, nf, out, gz_np, gb_np, gd_np, bs, M, bws):
    """The FP64 oracle on a bounded seeded sample of the workload's pixels,
    timed on the host cores (forward over every face of each pixel's mesh,
    then the analytic backward of the selected slots), and the GPU outputs
    checked against it on those pixels.  For the backward both sides take
    the oracle's selection (all other pixels empty)."""
    import numpy as np
    import torch

    import oracle
    from paper_2007_08501_amd import _lib

    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    dev = v.device
    nthr = oracle_threads()
    rng = np.random.default_rng(1234)
    probe = np.sort(rng.choice(N * H * W, size=64, replace=False))
    tq = time.perf_counter()
    oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius, K, pixels=probe,
                     nthreads=nthr)
    per_px = (time.perf_counter() - tq) / probe.size
    P = int(min(N * H * W, max(256, cpu_seconds / max(per_px, 1e-9))))
    pix = np.sort(rng.choice(N * H * W, size=P, replace=False))
    tq = time.perf_counter()
    o = oracle.rasterize(b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius, K, pixels=pix,
                         nthreads=nthr)
    t_f = time.perf_counter() - tq
    rows = lambda a: a.reshape((N * H * W,) + a.shape[3:])[pix]
    if not b.backward:
        return forward_only_parity(b, o, pix, t_f, P, nthr, out, dev)
    # slots whose two nearest edges are (nearly) tied have no unique distance
    # gradient: their upstream distance gradient is zeroed on both sides
    _, _, _, tie = oracle.fragments_fixed(b.verts, b.faces, (H, W), o["p2f"], nthreads=nthr, pixels=pix)
    gd_rows = np.where(tie.astype(bool), np.float32(0), rows(gd_np)).astype(np.float32)
    gd_m = gd_np.copy()
    gd_m.reshape(N * H * W, K)[pix] = gd_rows
    tq = time.perf_counter()
    ref = oracle.backward(b.verts, b.faces, (H, W), o["p2f"], rows(gz_np), rows(gb_np), gd_rows,
                          nthreads=nthr, pixels=pix, N=N)
    t_b = time.perf_counter() - tq
    cpu = {"value": round(P * K / (t_f + t_b) / 1e6, 6), "unit": UNIT, "cores": nthr, "kind": "oracle",
           "sample": f"{P} of {N * H * W} pixels (seeded uniform), FP64 brute force forward over every face "
                     f"of the pixel's mesh + analytic backward of their slots; fwd {t_f:.2f}s, bwd {t_b:.2f}s",
           "cpu_model": cpu_model(), "host_cpus_visible": oracle.default_threads(),
           "single_core": single_core_rate(b, pix, K)}

    # forward parity on the sampled pixels: exact ids where the oracle flags
    # nothing, a correct answer by the oracle's candidates where it does, and
    # the values within tolerance (oracle.validity)
    from oracle import validity
    pix_t = torch.from_numpy(pix).to(dev)
    g = {k: t.reshape((N * H * W,) + tuple(t.shape[3:]))[pix_t].cpu().numpy()
         for k, t in zip(("p2f", "zbuf", "bary", "dists"), out)}
    try:
        st = validity.compare_fragments(g, o, b.verts, b.faces, b.first_idx, b.num_faces, (H, W), b.blur_radius,
                                        where=b.name, pixels=pix, nthreads=nthr)
        fwd_ok, fwd_err = True, None
    except AssertionError as e:
        st, fwd_ok, fwd_err = None, False, str(e)[:300]
    amb = o["amb"] != 0
    # backward parity: the oracle's selection on the sampled pixels, on both sides
    p2f_s = torch.full_like(out.pix_to_face, -1).view(N * H * W, K)
    p2f_s[pix_t] = torch.from_numpy(o["p2f"].astype(np.int32)).to(dev)
    gv_s = torch.empty_like(v)
    t = lambda a: torch.from_numpy(a).to(dev)
    _lib.rasterize_meshes_bwd(v, f, fi, nf, H, W, b.blur_radius, K, bs, M, 0, p2f_s.view(N, H, W, K), t(gz_np),
                              t(gb_np), t(gd_m), gv_s, bws)
    gvs = gv_s.cpu().numpy().astype(np.float64)
    gerr = float(np.abs(gvs - ref).max() / max(1e-30, np.abs(ref).max()))
    parity = {"pixels": int(pix.size), "fragments_ok": fwd_ok, "ambiguous_frac": round(float(amb.mean()), 5),
              "grad_max_rel_err": gerr, "grad_ok": gerr <= 1e-3}
    if st is not None:
        parity.update(flagged_checked=st["checked_flagged"], order_only=st["order_only"],
                      ambiguous_by_bit={k: round(v, 5) for k, v in st["amb_bits"].items() if v > 0},
                      max_err={"bary": st["bary_err"], "zbuf": st["z_err"], "dists": st["d_err"]})
    else:
        parity["error"] = fwd_err
    return cpu, parity


POINTS_METRIC = "point-cloud render fwd+bwd ms/batch (rasterize + Alpha/Norm silhouette compositing)"
POINTS_PAPER_MS = 75.0  # the paper's figure for this workload (V100); context, not a target


def points_cpu_leg(b, cpu_seconds, idx, zbuf, dists, gd_np):
    """The FP64 point oracle on a bounded seeded pixel sample, timed on the
    host cores (brute-force forward over every point of the pixel's cloud and
    the analytic backward of those slots), with the GPU fragments checked
    against it, exactly, on the sample."""
    import numpy as np
    import torch

    import oracle

    N, (H, W), K = b.N, b.image_size, b.points_per_pixel
    nthr = min(16, oracle.default_threads())
    rng = np.random.default_rng(4321)
    probe = np.sort(rng.choice(N * H * W, size=64, replace=False))
    tq = time.perf_counter()
    oracle.rasterize_points(b.points, b.first_idx, b.num_points, (H, W), b.radius, K, pixels=probe, nthreads=nthr)
    per_px = (time.perf_counter() - tq) / probe.size
    P = int(min(N * H * W, max(256, cpu_seconds / max(per_px, 1e-9))))
    pix = np.sort(rng.choice(N * H * W, size=P, replace=False))
    tq = time.perf_counter()
    o = oracle.rasterize_points(b.points, b.first_idx, b.num_points, (H, W), b.radius, K, pixels=pix,
                                nthreads=nthr)
    t_f = time.perf_counter() - tq
    tq = time.perf_counter()
    oracle.points_backward(b.points, (H, W), o["idx"], None, gd_np.reshape(-1, K)[pix], pixels=pix, N=N,
                           nthreads=nthr)
    t_b = time.perf_counter() - tq
    cpu = {"value": round(P * K / (t_f + t_b) / 1e6, 6), "unit": UNIT, "cores": nthr, "kind": "oracle",
           "sample": f"{P} of {N * H * W} pixels (seeded uniform), FP64 brute force over every point of the "
                     f"pixel's cloud + analytic backward of their slots; fwd {t_f:.2f}s, bwd {t_b:.2f}s"}
    sel = torch.from_numpy(pix).to(idx.device)
    gi = idx.view(-1, K)[sel].cpu().numpy().astype(np.int64)
    gz = zbuf.view(-1, K)[sel].cpu().numpy()
    gdd = dists.view(-1, K)[sel].cpu().numpy()
    ok = bool((gi == o["idx"]).all() and (gz == o["zbuf"].astype(np.float32)).all()
              and (gdd == o["dists"].astype(np.float32)).all())
    return cpu, {"pixels": int(pix.size), "fragments_exact": ok}


def points_main(args):
    """--points: the point-cloud renderer at the paper's benchmark shape."""
    import numpy as np
    import torch

    from paper_2007_08501_amd import _lib, meshgen
    from paper_2007_08501_amd.graph import PointsGraphRunner

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ev = HipEvents()
    stream = torch.cuda.current_stream(dev).cuda_stream
    per_batch = []
    keep = None
    for batch in range(args.batch, args.batch + args.batches):
        b = meshgen.make_points_config(3, batch=batch)
        N, (H, W), K = b.N, b.image_size, b.points_per_pixel
        t = lambda a: torch.from_numpy(a).to(dev)
        gr = PointsGraphRunner(t(b.points), t(b.first_idx), t(b.num_points), H, W, b.radius, K, D=1,
                               norm=args.norm, silhouette=True)
        _, gd_np, _, _ = meshgen.point_grads(b, channels=1)
        rng = np.random.default_rng(b.seed + 9)
        gr.set_grad_image(t(rng.standard_normal((N, H, W, 1)).astype(np.float32)))
        gr.capture(warmup=2)
        for _ in range(args.warmup):
            gr.replay()
        n = args.steps
        e0, e1 = ev.create(), ev.create()
        torch.cuda.synchronize()
        ev.record(e0, stream)
        for _ in range(n):
            gr.replay()
        ev.record(e1, stream)
        torch.cuda.synchronize()
        graph_ms = ev.elapsed(e0, e1) / n
        st, _ = gr.status()
        if st != _lib.RAST_OK:
            log(f"[bench] device status: {_lib.status_string(st)}")
            sys.exit(1)
        # eager steps with the library's events around the per-tile and per-point kernels
        kev = [[ev.create() for _ in range(8)] for _ in range(n)]
        torch.cuda.synchronize()
        for i in range(n):
            k = kev[i]
            _lib.rast_set_kernel_events(_lib.RAST_KERNEL_POINTS_FINE, k[0], k[1])
            _lib.rast_set_kernel_events(_lib.RAST_KERNEL_POINTS_BWD, k[2], k[3])
            ev.record(k[4], stream)
            gr.forward_eager()
            ev.record(k[5], stream)
            gr.backward_eager()
            ev.record(k[6], stream)
        torch.cuda.synchronize()
        _lib.rast_set_kernel_events(_lib.RAST_KERNEL_POINTS_FINE, None, None)
        _lib.rast_set_kernel_events(_lib.RAST_KERNEL_POINTS_BWD, None, None)
        r = dict(batch=batch, graph_ms=graph_ms,
                 fine_ms=sum(ev.elapsed(k[0], k[1]) for k in kev) / n,
                 bwd_ms=sum(ev.elapsed(k[2], k[3]) for k in kev) / n,
                 fwd_call_ms=sum(ev.elapsed(k[4], k[5]) for k in kev) / n,
                 bwd_call_ms=sum(ev.elapsed(k[5], k[6]) for k in kev) / n,
                 valid=int((gr.idx >= 0).sum().item()))
        for e in [e0, e1] + [x for k in kev for x in k]:
            ev.destroy(e)
        log(f"[bench] points batch {batch}: {graph_ms:.4f} ms/step graph-replayed; fine {r['fine_ms']:.4f}, "
            f"point bwd {r['bwd_ms']:.4f}, fwd calls {r['fwd_call_ms']:.4f}, bwd calls {r['bwd_call_ms']:.4f} ms")
        per_batch.append(r)
        if keep is None:
            keep = (b, gr, gd_np)
        else:
            del gr
    b, gr, gd_np = keep
    N, (H, W), K = b.N, b.image_size, b.points_per_pixel
    P = b.points.shape[0]
    S = N * H * W * K
    ms_step = float(np.median([r["graph_ms"] for r in per_batch]))
    med = lambda k: float(np.median([r[k] for r in per_batch]))
    fine_ms, bwd_ms = med("fine_ms"), med("bwd_ms")
    S_valid = per_batch[0]["valid"]
    # algorithmic bytes: the fine pass writes three 4-byte outputs per slot and
    # reads each sorted 16-byte point once; the point backward reads the id
    # of every slot, the upstream gradient of each filled slot, each sorted
    # point, and writes 12 bytes per point
    fine_bytes = 12 * S + 16 * P
    bwd_bytes = 4 * S + 4 * S_valid + 16 * P + 12 * P
    kernels = {"points_fine": (fine_ms, fine_bytes), "points_backward": (bwd_ms, bwd_bytes)}
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_bytes = kernels[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel_ms": round(dom_ms, 5),
                "algorithmic_bytes": dom_bytes}
    valu = measured_valu(dom, 0, K, 0, path=os.path.join(ROOT, "profiles", f"kernels_pts3_K{K}.txt"))
    if valu is not None:
        lane_ops = valu * 64 / (dom_ms * 1e-3)
        roofline["valu_issue"] = {"lane_slots_per_s": float(f"{lane_ops:.4g}"), "peak": VALU_PEAK_LANE_OPS,
                                  "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4), "wave_instructions": int(valu),
                                  "what": VALU_ISSUE_WHAT}
    roofline["traffic"] = measured_traffic(dom, "pts3", K, 0, path=os.path.join(
        ROOT, "profiles", f"traffic_{dom}_pts3_K{K}.txt"))
    if args.copy_probe:
        # a plain streaming kernel of known size, the scale for the byte counters of a profiled run
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        cpu, parity = points_cpu_leg(b, args.cpu_seconds, gr.idx, gr.zbuf, gr.dists, gd_np)
        log(f"[bench] cpu baseline {cpu}")
        log(f"[bench] parity {parity}")
    res = {
        "metric": POINTS_METRIC, "value": round(ms_step, 5), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": round(ms_step / POINTS_PAPER_MS, 6), "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"pts3: {meshgen.POINT_CONFIG_NAMES[3]}", "clouds": N, "points": P, "image": [H, W],
                   "points_per_pixel": K, "radius": b.radius,
                   "compositing": "Norm" if args.norm else "Alpha", "features": "silhouette (every feature 1, no feature table)",
                   "parallelism": "single GPU"},
        "throughput_mpixk_per_s": round(S / (ms_step * 1e-3) / 1e6, 2), "slots": S, "slots_valid": S_valid,
        "kernels_ms": {"points_fine": round(fine_ms, 5), "points_backward": round(bwd_ms, 5),
                       "forward_calls": round(med("fwd_call_ms"), 5), "backward_calls": round(med("bwd_call_ms"), 5)},
        "timing": {"form": "fwd (rasterize + composite) and bwd (composite + rasterize) captured in one HIP graph "
                           "and replayed; value is the median over seeded batches",
                   "batches": [r["batch"] for r in per_batch],
                   "ms_per_step_graph": [round(r["graph_ms"], 5) for r in per_batch]},
        "paper_ms_v100": POINTS_PAPER_MS,
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity,
    }
    print(json.dumps(res), flush=True)
    if parity is not None and not parity["fragments_exact"]:
        sys.exit(3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--batch", type=int, default=0, help="first seeded batch index")
    ap.add_argument("--batches", type=int, default=5, help="seeded batches timed (the paper averages 5)")
    ap.add_argument("--bin-size", type=int, default=None, help="fixed bin size (default: autotune)")
    ap.add_argument("--max-faces-per-bin", type=int, default=None)
    ap.add_argument("--sched", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-mesh", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--copy-probe", action="store_true", help="also run a plain streaming kernel of known size")
    ap.add_argument("--points", action="store_true",
                    help="benchmark the point-cloud renderer instead (8 clouds x 200k points, 256x256, K=50)")
    ap.add_argument("--norm", action="store_true", help="--points: Norm compositing instead of Alpha")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this rasterizer runs on one GPU; the batch would "
              "shard by image across GPUs but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    if args.points:
        points_main(args)
        return

    import numpy as np
    import torch

    from paper_2007_08501_amd import _lib, meshgen
    from paper_2007_08501_amd.autotune import autotune
    from paper_2007_08501_amd.raster import count_max_faces_per_bin, empty_fragments, round_up

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    from paper_2007_08501_amd.graph import GraphRunner
    ev = HipEvents()
    stream = torch.cuda.current_stream(dev).cuda_stream

    def setup(batch):
        """Inputs of one seeded batch on the device, and its bin parameters (untimed)."""
        b = meshgen.make_config(args.config, batch=batch)
        N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
        t = lambda a: torch.from_numpy(a).to(dev)
        v, f, fi, nf = t(b.verts), t(b.faces), t(b.first_idx), t(b.num_faces)
        grads_np = meshgen.upstream_grads(b)
        t0 = time.time()
        if args.bin_size is None and b.bin_size is not None:
            # the workload fixes its bins (config 1: single pass; config 2: 32-pixel bins, capacity 10000)
            bs, M, sched = b.bin_size, (b.max_faces_per_bin or 0) if b.bin_size > 0 else 0, 0
            log(f"[bench] batch {batch}: bins fixed by the workload: bin_size={bs} M={M}")
        elif args.bin_size is None:
            ch = autotune(v, f, fi, nf, H, W, b.blur_radius, K, reps=5, backward=b.backward)
            bs, M, sched = ch.bin_size, ch.max_faces_per_bin, ch.sched
            log(f"[bench] batch {batch}: autotune -> bin_size={bs} M={M} sched={sched} ({ch.ms:.3f} ms) in "
                f"{time.time() - t0:.1f}s")
        else:
            bs, sched, M = args.bin_size, args.sched or 0, args.max_faces_per_bin
            if bs > 0 and M is None:
                M = round_up(count_max_faces_per_bin(v, f, fi, nf, H, W, b.blur_radius, bs), 32)
        if args.sched is not None:
            sched = args.sched
        return b, (v, f, fi, nf), grads_np, bs, M or 0, sched

    def time_batch(b, dev_in, grads_np, bs, M, sched):
        """Graph-replayed fwd+bwd steps, then eager steps with the library's
        per-kernel events (the roofline's kernel times)."""
        N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
        v, f, fi, nf = dev_in
        gz, gb, gd = [torch.from_numpy(x).to(dev) for x in grads_np]
        gr = GraphRunner(v, f, fi, nf, H, W, b.blur_radius, K, bs, M, sched=sched, backward=b.backward)
        if b.backward:
            gr.set_grads(gz, gb, gd)
        gr.capture(warmup=2)
        for _ in range(args.warmup):
            gr.replay()
        torch.cuda.synchronize()
        n = args.steps
        e0, e1 = ev.create(), ev.create()
        torch.cuda.synchronize()
        ev.record(e0, stream)
        for _ in range(n):
            gr.replay()
        ev.record(e1, stream)
        torch.cuda.synchronize()
        graph_ms = ev.elapsed(e0, e1) / n
        st, mx = gr.status()
        if st != _lib.RAST_OK:
            log(f"[bench] device status: {_lib.status_string(st)} (max bin count {mx})")
            sys.exit(1)
        # eager steps, each kernel bracketed by HIP events on the launch stream
        kev = [[ev.create() for _ in range(4)] for _ in range(n)]
        torch.cuda.synchronize()
        ev.record(e0, stream)
        for i in range(n):
            _lib.rast_set_kernel_events(_lib.RAST_KERNEL_FINE, kev[i][0], kev[i][1])
            _lib.rast_set_kernel_events(_lib.RAST_KERNEL_BWD, kev[i][2], kev[i][3])
            gr.step_eager()
        ev.record(e1, stream)
        torch.cuda.synchronize()
        _lib.rast_set_kernel_events(_lib.RAST_KERNEL_FINE, None, None)
        _lib.rast_set_kernel_events(_lib.RAST_KERNEL_BWD, None, None)
        eager_ms = ev.elapsed(e0, e1) / n
        fine_ms = sum(ev.elapsed(k[0], k[1]) for k in kev) / n
        bwd_ms = sum(ev.elapsed(k[2], k[3]) for k in kev) / n if b.backward else 0.0
        for e in [e0, e1] + [x for k in kev for x in k]:
            ev.destroy(e)
        valid = int((gr.out.pix_to_face >= 0).sum().item())
        return dict(graph_ms=graph_ms, eager_ms=eager_ms, fine_ms=fine_ms, bwd_ms=bwd_ms, valid=valid,
                    out=gr.out, gv=gr.grad_verts if b.backward else None)

    # ---------------------------------------------------------------- timed region, per seeded batch
    per_batch = []
    first_setup = None
    for batch in range(args.batch, args.batch + args.batches):
        su = setup(batch)
        if first_setup is None:
            first_setup = su
        r = time_batch(*su)
        r.update(batch=batch, bs=su[3], M=su[4], sched=su[5])
        log(f"[bench] batch {batch}: {r['graph_ms']:.4f} ms/step graph-replayed, {r['eager_ms']:.4f} eager; "
            f"fine {r['fine_ms']:.4f} ms, bwd {r['bwd_ms']:.4f} ms")
        per_batch.append(r)
        if batch != args.batch:
            del r["out"], r["gv"]
    first = per_batch[0]
    b, dev_in, grads_np, bs, M, sched = first_setup
    v, f, fi, nf = dev_in
    gz_np, gb_np, gd_np = grads_np
    gz, gb, gd = [torch.from_numpy(x).to(dev) for x in grads_np]
    out = first["out"]
    N, (H, W), K = b.N, b.image_size, b.faces_per_pixel
    bws = _lib.alloc_workspace(_lib.rast_workspace_size(N, H, W, f.shape[0], bs, M), dev)
    n = args.steps
    ms_all = [r["graph_ms"] for r in per_batch]
    ms_step = float(np.median(ms_all))
    ms_mean = float(np.mean(ms_all))
    fine_ms = float(np.median([r["fine_ms"] for r in per_batch]))
    bwd_ms = float(np.median([r["bwd_ms"] for r in per_batch]))
    log(f"[bench] {len(per_batch)} batches x {n} steps: median {ms_step:.4f} ms/step (mean {ms_mean:.4f}); "
        f"fine {fine_ms:.4f} ms, bwd {bwd_ms:.4f} ms")

    S = N * H * W * K
    S_valid = first["valid"]
    V, F = b.verts.shape[0], b.faces.shape[0]
    fine_bytes = 24 * S + 12 * V + 12 * F
    bwd_bytes = 4 * S + 20 * S_valid + 24 * V + 12 * F if b.backward else 0
    step_bytes = fine_bytes + bwd_bytes
    kernels = {"fine": (fine_ms, fine_bytes)}
    if b.backward:
        kernels["backward"] = (bwd_ms, bwd_bytes)
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms, dom_bytes = kernels[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dom, args.config, K, bs), "kernel_ms": round(dom_ms, 5),
                "algorithmic_bytes": dom_bytes}
    # the same kernel against the VALU issue rate: its counted VALU instructions
    # (64 lane slots each, masked lanes included) over the live kernel time
    valu = measured_valu(dom, args.config, K, bs)
    if valu is not None:
        lane_ops = valu * 64 / (dom_ms * 1e-3)
        roofline["valu_issue"] = {"lane_slots_per_s": float(f"{lane_ops:.4g}"), "peak": VALU_PEAK_LANE_OPS,
                                  "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4), "wave_instructions": int(valu),
                                  "what": VALU_ISSUE_WHAT}

    # ---------------------------------------------------------------- per-mesh forms
    per_mesh = None
    if not args.no_per_mesh:
        calls = []
        for m in range(N):
            a0, cnt = int(b.first_idx[m]), int(b.num_faces[m])
            fm = f[a0:a0 + cnt].contiguous()
            z0 = torch.zeros(1, dtype=torch.int64, device=dev)
            c1 = torch.full((1,), cnt, dtype=torch.int64, device=dev)
            m32 = round_up(count_max_faces_per_bin(v, fm, z0, c1, H, W, b.blur_radius, 32), 32)
            ws1 = _lib.alloc_workspace(_lib.rast_workspace_size(1, H, W, cnt, 32, m32), dev)
            calls.append((fm, empty_fragments(1, H, W, K, dev), z0, c1, m32, ws1, slice(m, m + 1)))
        one_ws = _lib.alloc_workspace(max(_lib.rast_workspace_size(1, H, W, c[0].shape[0], 0, 0) for c in calls), dev)
        gvm = torch.empty_like(v)

        def per_mesh_step(binned):
            # one call pair per mesh, no graph: single pass, or bins of 32 pixels
            for fm, o1, z0, c1, m32, ws1, sl in calls:
                bs1, M1, w = (32, m32, ws1) if binned else (0, 0, one_ws)
                _lib.rasterize_meshes_fwd(v, fm, z0, c1, H, W, b.blur_radius, K, bs1, M1, 0, o1.pix_to_face, o1.zbuf,
                                          o1.bary, o1.dists, w)
                if b.backward:
                    _lib.rasterize_meshes_bwd(v, fm, z0, c1, H, W, b.blur_radius, K, bs1, M1,
                                              _lib.RAST_BWD_REUSE_FORWARD if binned else 0, o1.pix_to_face, gz[sl],
                                              gb[sl], gd[sl], gvm, w)

        def time_form(binned, reps):
            per_mesh_step(binned)
            torch.cuda.synchronize()
            a, c = ev.create(), ev.create()
            ev.record(a, stream)
            for _ in range(reps):
                per_mesh_step(binned)
            ev.record(c, stream)
            ms = ev.elapsed(a, c) / reps
            ev.destroy(a)
            ev.destroy(c)
            return ms

        pm_ms = time_form(False, 2)
        pb_ms = time_form(True, 5)
        per_mesh = {"ms_per_batch": round(pm_ms, 4), "value": round(S / (pm_ms * 1e-3) / 1e6, 2),
                    "form": f"one single-pass {'fwd+bwd' if b.backward else 'fwd'} call per mesh (no bins, no graph)",
                    "speedup_batched": round(pm_ms / ms_step, 2),
                    "binned32": {"ms_per_batch": round(pb_ms, 4), "value": round(S / (pb_ms * 1e-3) / 1e6, 2),
                                 "form": f"one {'fwd+bwd' if b.backward else 'fwd'} call per mesh with 32-pixel bins (no graph)",
                                 "speedup_batched": round(pb_ms / ms_step, 2)}}
        log(f"[bench] per-mesh plain {pm_ms:.3f} ms/batch, per-mesh bins-32 {pb_ms:.3f} ms/batch")

    # ---------------------------------------------------------------- config 5: the whole fitting step
    fit = None
    if args.config == 5:
        from paper_2007_08501_amd import silfit
        fp = silfit.SilhouetteFit(meshgen.silhouette_fit_problem(), bin_size=bs if bs > 0 else 0)
        offsets = torch.zeros_like(fp.base, requires_grad=True)
        opt = torch.optim.Adam([offsets], lr=1e-3)

        def fit_step():
            opt.zero_grad(set_to_none=True)
            loss = fp.loss(offsets)
            loss.backward()
            opt.step()
            return loss

        for _ in range(3):
            fit_step()
        torch.cuda.synchronize()
        reps = 20
        a0, a1 = ev.create(), ev.create()
        ev.record(a0, stream)
        for _ in range(reps):
            fit_step()
        ev.record(a1, stream)
        fit_ms = ev.elapsed(a0, a1) / reps
        ev.destroy(a0)
        ev.destroy(a1)
        fit = {"ms_per_step": round(fit_ms, 4), "value": round(S / (fit_ms * 1e-3) / 1e6, 2),
               "form": "one Adam step of the silhouette fit, eager: view transform, rasterizer fwd, blend fwd, "
                       "IoU loss, blend bwd, rasterizer bwd, Adam (lr 1e-3); bins as in the rasterizer timing"}
        log(f"[bench] silhouette fit step {fit_ms:.4f} ms")

    # ---------------------------------------------------------------- CPU baseline (oracle) + sampled parity
    cpu, parity = None, None
    if not args.no_cpu_baseline:
        cpu, parity = cpu_baseline_leg(b, args.cpu_seconds, v, f, fi, nf, out, gz_np, gb_np, gd_np, bs, M, bws)
        log(f"[bench] cpu baseline {cpu}")
        log(f"[bench] parity {parity}")

    if args.copy_probe:
        # a plain streaming kernel of known size (read 256 MiB, write 256 MiB),
        # the scale for the HBM byte counters of a profiled run
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()

    res = {
        "metric": METRIC, "value": round(S / (ms_step * 1e-3) / 1e6, 2), "unit": UNIT, "n_gpus": 1,
        "steps": n, "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"cfg{args.config}: {meshgen.CONFIG_NAMES[args.config]}", "meshes": N,
                   "image": [H, W], "faces_per_pixel": K, "blur_radius": b.blur_radius, "faces": F, "verts": V,
                   "bin_size": bs, "max_faces_per_bin": M, "sched": sched, "parallelism": "single GPU"},
        "slots": S, "slots_valid": S_valid, "step_algorithmic_bytes": step_bytes,
        "step_hbm_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels_ms": {"fine": round(fine_ms, 5), "backward": round(bwd_ms, 5)},
        "timing": {"form": ("bins fixed by the workload" if (args.bin_size is None and b.bin_size is not None)
                            else "bins from the autotuner" if args.bin_size is None else "bins fixed on the command line")
                           + ", fwd+bwd captured in one HIP graph and replayed; value and ms_per_step are the median "
                             "over seeded batches",
                   "batches": [r["batch"] for r in per_batch],
                   "ms_per_step_graph": [round(r["graph_ms"], 5) for r in per_batch],
                   "ms_per_step_mean": round(ms_mean, 5),
                   "ms_per_step_eager": round(float(np.median([r["eager_ms"] for r in per_batch])), 5),
                   "bins": [[r["bs"], r["M"], r["sched"]] for r in per_batch]},
        "roofline": roofline, "cpu_baseline": cpu, "per_mesh": per_mesh, "parity": parity,
    }
    if fit is not None:
        res["fit_step"] = fit
    if not b.backward:
        res["timing"]["form"] = "forward only (the workload has no backward), captured in one HIP graph and " \
                                "replayed; value and ms_per_step are the median over seeded batches"
    print(json.dumps(res), flush=True)
    if parity is not None and not (parity["fragments_ok"] and parity["grad_ok"]):
        sys.exit(3)


if __name__ == "__main__":
    main()
