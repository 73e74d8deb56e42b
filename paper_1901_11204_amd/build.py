"""Build libpairs.so for gfx950 with hipcc, in-tree.

    python -m paper_1901_11204_amd.build
"""
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpairs.so")
SOURCES = [os.path.join(CSRC, "pairs.hip")]
PROBE_LIB = os.path.join(PKG, "libvaluprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "valu_probe.hip")]
AB_LIB = os.path.join(PKG, "libpairs_ab.so")
AB_SOURCES = [os.path.join(CSRC, "ab_straightforward.hip")]
ARCH = "gfx950"


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def build_cmd(out: str, extra=(), sources=None):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # hardware float atomics; IEEE semantics without contraction
            "-munsafe-fp-atomics", "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
            # the SLP vectorizer packs per-pair predicate bits into vectors in
            # the unrolled sweeps, which costs VALU instructions on gfx950
            "-fno-slp-vectorize",
            # matrix-instruction results in VGPRs, where the comparisons read
            # them, rather than in AGPRs copied out one register at a time
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            "-I", INCLUDE, "-I", CSRC, *extra, "-o", out, *(sources or SOURCES)]


def _compile(lib, sources, verbose):
    tmp = lib + ".tmp"
    cmd = build_cmd(tmp, sources=sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compile libpairs.so, the VALU issue-rate probe library and the
    benchmark's assignment-comparison library."""
    _compile(LIB, SOURCES, verbose)
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    _compile(AB_LIB, AB_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
