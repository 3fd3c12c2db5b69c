"""Build the HIP library liblbm2p.so in-tree for gfx950.

Three translation units: the C ABI, the FP64 step (no floating-point
contraction, so it rounds exactly as written and matches the CPU oracle bit for
bit) and the FP32 step (fused multiply-adds and fast single-precision division
allowed).  Packed FP32 instructions are disabled for all device code.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm2p.so")

COMMON = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]
UNITS = [
    ("lbm2p.hip", ["-ffp-contract=off"]),
    ("lbm2p_f64.hip", ["-ffp-contract=off"]),
    ("lbm2p_f32.hip", ["-ffp-contract=fast", "-fno-hip-fp32-correctly-rounded-divide-sqrt"]),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))


def build(verbose=True, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src, flags in UNITS:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        _run([hipcc] + COMMON + flags + list(extra) + ["-c", os.path.join(CSRC, src), "-o", obj],
             verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
