"""Build libhca.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2105_00448_amd.build

Every translation unit under csrc/ is compiled for gfx950 only; objects go to
_build/ at the repository root and the shared library next to this file.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhca.so")

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]
# per-file extra flags: the CA decides integers from floating point and must
# round every operation exactly as written
EXTRA = {
    "k_ca.hip": ["-ffp-contract=off"],
}
SOURCES = ["runtime.cpp", "runtime.cpp:32", "capi.cpp", "mlp_runtime.cpp", "k_setup.hip", "k_solver.hip",
           "k_ode.hip", "k_ca.hip", "k_mg.hip", "k_mlp.hip", "noalloc.hip"]
# runtime.cpp is compiled once per field storage precision ("runtime.cpp:32":
# FP32 storage, its own namespace)
VARIANTS = {"32": ["-DHCA_REAL=float", "-DHCA_RT_NS=rt32"]}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(unit):
    src, _, variant = unit.partition(":")
    obj = os.path.join(BUILD, src + (f".{variant}" if variant else "") + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = ([hipcc(), "-c"] + lang + [os.path.join(CSRC, src), "-o", obj] + COMMON + EXTRA.get(src, [])
           + VARIANTS.get(variant, []))
    r = subprocess.run(cmd, capture_output=True, text=True)
    return unit, obj, r


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s.partition(":")[0]))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = []
    for src, obj, r in results:
        msg = (r.stdout + r.stderr).strip()
        # the host pass does not know the GPU-only target feature: harmless
        lines = [l for l in msg.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
        if verbose and lines:
            print(f"[{src}]\n" + "\n".join(lines), file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
