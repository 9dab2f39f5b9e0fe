"""Build the HIP libraries in-tree for gfx950 (hipcc cross-compiles; no GPU needed).

librfi.so       -- the method (csrc/api.cpp, pipeline.cpp, ccm.hip, ccm_long.hip, eig_lane.hip,
                   eig_wave.hip, eig_tri.hip, flag.hip, bandpass.hip, serve.cpp, batch.cpp)
librfi_synth.so -- the GPU input generator (csrc/synth.hip) and the streaming-read
                   reference of the HBM roofline (csrc/stream_read.hip)

Every call recompiles (objects go to _build/, the libraries next to this file).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # no packed-FP32 instructions anywhere (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

LIBS = {
    "librfi.so": ["api.cpp", "pipeline.cpp", "ccm.hip", "ccm_long.hip", "eig_lane.hip", "eig_wave.hip",
                  "eig_tri.hip", "flag.hip", "bandpass.hip", "serve.cpp", "batch.cpp"],
    "librfi_synth.so": ["synth.hip", "stream_read.hip"],
}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> dict:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for v in LIBS.values() for s in v if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    out = {}
    for lib, parts in LIBS.items():
        o = [objs[s] for s in parts if s in objs]
        path = os.path.join(PKG, lib)
        tmp = path + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + o
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed for {lib}:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, path)
        out[lib] = path
        if verbose:
            print(f"built {path}")
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
