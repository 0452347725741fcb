"""Build libmri.so (HIP, gfx950) in-tree.

    python -m paper_2211_03293_amd.build        # or build() from __graft_entry__

Steps: embed the run-time compiled kernel sources (spec_kernels.inc and
spec_abi.h) as C strings, then compile every .hip/.cpp under csrc/ with hipcc
into paper_2211_03293_amd/libmri.so, linked against hipRTC.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmri.so")
ARCH = os.environ.get("MRI_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# developer knobs: extra -D definitions and another output path (tuning builds)
EXTRA = os.environ.get("MRI_EXTRA_DEFS", "").split()
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", CSRC, "-I", INCLUDE, "-Wall", "-Wno-unused-function"]


def _embed(name: str, symbol: str) -> str:
    with open(os.path.join(CSRC, name)) as f:
        text = f.read()
    delim = "MRI_EMBED"
    assert f"){delim}\"" not in text
    return f'extern const char {symbol}[];\nconst char {symbol}[] = R"{delim}({text}){delim}";\n'


def _write_embedded() -> str:
    os.makedirs(BUILD, exist_ok=True)
    path = os.path.join(BUILD, "embedded_sources.cpp")
    body = (_embed("spec_kernels.inc", "mri_spec_kernels_src") +
            _embed("spec_abi.h", "mri_spec_abi_src") + _embed("mri_math.h", "mri_math_src"))
    old = open(path).read() if os.path.exists(path) else None
    if old != body:
        with open(path, "w") as f:
            f.write(body)
    return path


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, *EXTRA, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True, out: str | None = None) -> str:
    global BUILD
    out = out or os.environ.get("MRI_LIB_OUT") or LIB
    if out != LIB:
        BUILD = os.path.join(HERE, "_build", os.path.basename(out).replace(".so", ""))
    emb = _write_embedded()
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))
    srcs.append(emb)
    jobs = int(os.environ.get("MAX_JOBS", "8"))
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = out + f".tmp{os.getpid()}"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", flush=True)
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
