"""Build libfcat.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfcat.so")
CEILINGS = os.path.join(HERE, "fcat_ceilings")      # device-ceiling microbenchmark (stand-alone program)
SOURCES = ["fcat_abi.hip", "fcat_kernels.hip", "fcat_split.hip", "fcat_mlp.hip", "fcat_noise.hip", "fcat_dose.hip", "fcat_fdk.hip", "fcat_optics.hip", "fcat_adjoint.hip"]
ARCH = os.environ.get("FCAT_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are switched off for all device code.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, obj: str, extra: list[str]) -> None:
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if noisy:
        sys.stderr.write("\n".join(noisy) + "\n")


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compile every HIP source and link libfcat.so.  Always rebuilds."""
    extra = list(extra or [])
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], extra), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra, os.path.join(CSRC, "fcat_ceilings.hip"), "-o", CEILINGS + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for fcat_ceilings.hip:\n{r.stdout}\n{r.stderr}")
    os.replace(CEILINGS + ".tmp", CEILINGS)
    if verbose:
        print(f"built {LIB} and {CEILINGS}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
