"""Build libnsmi.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2509_13307_amd.build          # or build() from Python

Every translation unit is compiled with -O3 for gfx950 and with packed FP32
instructions disabled; the objects are linked into
paper_2509_13307_amd/lib/libnsmi.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libnsmi.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "emulator.hip", "mlp_fused.hip", "mlp_f64.hip", "likelihood.hip", "shear.hip", "shear_adjoint.hip", "sampler.hip", "adjoint.hip", "hmc.hip", "noalloc.hip", "tune_cache.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(os.path.dirname(HERE), "include")]


def _source_id():
    """Hash of every source and header of the library: keys the on-disk
    autotuning cache to this build's kernels."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(os.path.dirname(HERE), "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".cpp", ".h")):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = [HIPCC, *FLAGS, f"-DNSMI_SRC_ID=\"{_source_id()}\"", "-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj, out


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    if verbose:
        for _, out in results:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
