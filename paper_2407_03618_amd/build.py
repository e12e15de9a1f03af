"""Builds the gfx950 HIP library ``libbm25_mi355x.so`` in-tree with hipcc.

Usage: ``python -m paper_2407_03618_amd.build`` (or ``build()`` from Python). Every call
recompiles every translation unit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_NAME = "libbm25_mi355x.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]

# the gather's matrix-core instructions keep their accumulators in ordinary VGPRs, so the kernel's
# register count (and occupancy) stays that of its vector-unit form
MFMA_VGPR = ["-mllvm", "-amdgpu-mfma-vgpr-form"]

UNITS = [
    ("tokenize.hip", []),
    ("index_build.hip", []),
    ("search.hip", []),
    ("util.hip", []),
    ("serve.hip", []),
    ("search_inst.hip", ["-DBM25_ST=F32", "-DBM25_ST_SUFFIX=f32", *MFMA_VGPR]),
    ("search_inst.hip", ["-DBM25_ST=F16", "-DBM25_ST_SUFFIX=f16", *MFMA_VGPR]),
    ("search_inst.hip", ["-DBM25_ST=BF16", "-DBM25_ST_SUFFIX=bf16", *MFMA_VGPR]),
]


def _compile(unit, extra, verbose):
    src = os.path.join(CSRC, unit)
    tag = "_".join(x.split("=")[-1] for x in extra if x.startswith("-DBM25_ST_SUFFIX"))
    obj = os.path.join(BUILD_DIR, os.path.splitext(unit)[0] + (f"_{tag}" if tag else "") + ".o")
    cmd = [_hipcc(), *COMMON, "-I", BUILD_DIR, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {unit}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    # Unicode tables of the tokenizer, generated from this Python's character database
    gen = os.path.join(CSRC, "gen_unicode_tables.py")
    r = subprocess.run([sys.executable, gen, os.path.join(BUILD_DIR, "unicode_tables.inc")],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"unicode table generation failed:\n{r.stdout}\n{r.stderr}")
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u[0], u[1], verbose), UNITS))
    tmp = LIB_PATH + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
