"""Builds libcaps.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcaps.so")

SOURCES = ["caps_api.hip", "caps_build.hip", "caps_search.hip", "caps_mfma.hip", "caps_router.hip", "caps_server.hip", "caps_io.hip", "caps_util.hip", "caps_static.hip"]
# caps_scan_inst.hip once per (precision, kind): the matrix-core scan
# instantiations, compiled in parallel (CAPS_PREC_BF16 = 1, FP8 = 2, FP16 = 3;
# kinds: approximate keys, exact main pass, exact rescue pass, exact main pass
# with survivor counts, seed lists)
INSTANCES = [(f"caps_scan_{name}_{kind}", ["-DCAPS_INST_PREC=%d" % prec, "-DCAPS_INST_KIND=%d" % kd])
             for name, prec in (("bf16", 1), ("fp8", 2), ("fp16", 3))
             for kind, kd in (("approx", 0), ("exact", 1), ("rescue", 2), ("exactcnt", 3), ("seed", 4))]

# -ffp-contract=off: every fused multiply-add in the kernels is written out
# explicitly (fmaf); the compiler must not fuse anything else, so that the
# FP32 arithmetic is exactly the specified sequence.
# -packed-fp32-ops off: the packed FP32 VALU forms are not used.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def _stale(obj: str, src: str) -> bool:
    """An object is stale when it is older than its source or any header
    of the library (every source includes some of them)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.join(HERE, "..", "include", "caps.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return any(os.path.getmtime(f) > t for f in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source to an object in parallel, then links.  With
    incremental=True, objects newer than their sources and the headers are
    kept."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    jobs = [(src, src.replace(".hip", ".o"), []) for src in SOURCES]
    jobs += [("caps_scan_inst.hip", name + ".o", defs) for name, defs in INSTANCES]
    objs_all = []
    for src, oname, defs in jobs:
        obj = os.path.join(objdir, oname)
        objs_all.append(obj)
        if incremental and not _stale(obj, src):
            continue
        cmd = [hipcc()] + [f for f in FLAGS if f != "-shared"] + defs + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = []
    for src, obj, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out + err)
            failed.append(src)
    objs = objs_all
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    tmp = LIB + ".tmp"
    # hipBLASLt: the learned router's two inference products
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhipblaslt"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libcaps.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
