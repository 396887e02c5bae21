"""Build librast.so (the HIP rasterizer library) in-tree with hipcc for gfx950.

    python -m paper_2007_08501_amd.build

Every HIP translation unit is compiled with:
  -ffp-contract=off      the forward and backward kernels must evaluate each
                         (pixel, face) pair with identical instructions
  -munsafe-fp-atomics    hardware float atomics for the backward's scatter
  -Xclang -target-feature -Xclang -packed-fp32-ops
                         no packed FP32 instructions in the generated code
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librast.so")
SOURCES = ["api.hip", "kernels_fwd.hip", "kernels_bwd.hip", "kernels_blend.hip", "kernels_points.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-munsafe-fp-atomics",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result",
            "-I" + os.path.join(HERE, "..", "include")]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (the CPU checks of
# the argument validation and workspace layout); the device code is built as
# usual.  Each flag is scoped to the host pass.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
                 "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host",
                 "-shared-libsan"]


def build(verbose: bool = False, sanitize_host: bool = False, out: str = None) -> str:
    """Compile every source and link librast.so (or `out`); always rebuilds."""
    cc = hipcc()
    lib_path = out or LIB
    objdir = os.path.join(HERE, "_build" if not sanitize_host else "_build_san")
    os.makedirs(objdir, exist_ok=True)
    extra = SANITIZE_HOST if sanitize_host else []
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc] + flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(f"[{s}]\n{t}" for s, t in failed))
    tmp = lib_path + ".tmp%d" % os.getpid()
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + extra + objs + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
