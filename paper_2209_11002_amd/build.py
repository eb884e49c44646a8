"""Build the EDAA HIP library (libedaa.so) in-tree for gfx950 with hipcc."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libedaa.so")
# (source, extra defines, object name); edaa_inst.hip is compiled once per p
MAX_P = 16
UNITS = ([("edaa_inst.hip", [f"-DEDAA_INST_P={p}"], f"edaa_inst_p{p}.o") for p in range(MAX_P, 0, -1)]
         + [("edaa_persist.hip", [], "edaa_persist.o"), ("edaa_kernels.hip", [], "edaa_kernels.o"),
            ("edaa_grad.hip", [], "edaa_grad.o"),
            ("edaa_api.hip", [], "edaa_api.o")])
ARCH = os.environ.get("EDAA_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{INCLUDE}", f"-I{CSRC}"]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def _compile(unit):
    src, defines, name = unit
    obj = os.path.join(BUILD, name)
    cmd = [_hipcc(), *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    return obj, out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = int(os.environ.get("MAX_JOBS", 0)) or os.cpu_count() or 4
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, 16))) as ex:
        results = list(ex.map(_compile, UNITS))
    if verbose:
        for _, out in results:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *[o for o, _ in results]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
