"""Build libdinr.so (the gfx950 HIP library behind include/dinr.h) in-tree.

Every source is compiled to its own object in parallel (hipcc -c), then the
objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["dinr_api.hip", "kernels.hip", "wgrad.hip", "server.hip", "probe.hip"]
# the fused MLP kernel is instantiated once per (precision, mode): FP32/BF16 x
# forward, backward, fused one-pass, query, grouped one-pass
MLP_UNITS = [(prec, mode) for prec in (0, 1) for mode in (0, 1, 2, 3, 4)]
LIB = os.path.join(HERE, "libdinr.so")
OBJ_DIR = os.path.join(HERE, "_build")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-fast-math", "-ffp-contract=on",
    "-I" + os.path.join(ROOT, "include"),
]


def _filter(out: str) -> str:
    return "\n".join(ln for ln in out.splitlines() if "packed-fp32-ops" not in ln)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)

    def compile_one(unit):
        src, defs = unit
        tag = "".join(f"_{v}" for v in defs.values())
        obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + tag + ".o")
        cmd = [hipcc] + FLAGS + [f"-D{k}={v}" for k, v in defs.items()] + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        proc = subprocess.run(cmd, capture_output=True, text=True)
        return obj, proc.returncode, _filter(proc.stdout + proc.stderr)

    units = [(s, {}) for s in SOURCES] + \
        [("mlp_inst.hip", {"DINR_INST_PREC": p, "DINR_INST_MODE": m}) for p, m in MLP_UNITS]
    jobs = max(1, min(len(units), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, units))
    failed = [(o, msg) for o, rc, msg in results if rc != 0]
    if failed:
        for _, msg in failed:
            sys.stderr.write(msg + "\n")
        raise RuntimeError("hipcc failed building libdinr.so")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _, _ in results] + \
        ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(_filter(proc.stdout + proc.stderr) + "\n")
        raise RuntimeError("linking libdinr.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
