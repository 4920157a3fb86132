"""Build liblbfast.so (the C-ABI library of include/lbfast.h) for gfx950.

Each HIP translation unit is compiled by hipcc in parallel, then linked into
one shared library placed next to this file.  Packed FP32 instructions are
disabled for all device code (-packed-fp32-ops).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbfast.so")
ARCH = os.environ.get("LBFAST_ARCH", "gfx950")

SOURCES = ["step_h_f64.hip", "step_h_f32.hip", "step_h_f16s.hip", "step_h_bf16s.hip",
           "step_h_f16su.hip",
           "step_f64.hip", "step_f32.hip", "step_f16s.hip", "step_bf16s.hip", "step_f16su.hip",
           "adjoint_f64.hip", "adjoint_f32.hip", "phase.hip", "aux.hip", "noalloc.hip", "lbfast.cpp"]

COMMON = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, verbose, flags, build_dir, csrc):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + flags + ["-I", csrc] + lang + ["-c", os.path.join(csrc, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if msgs.strip() and verbose:
        print(msgs, flush=True)
    return obj


def build(verbose: bool = False, jobs: int = None, out: str = None, defines=(),
          csrc: str = None) -> str:
    """Compile every translation unit and link `out` (default: liblbfast.so
    next to this file).  `defines` adds -D flags and `csrc` replaces the source
    directory (tuning experiments build elsewhere)."""
    lib = out or LIB
    csrc = csrc or CSRC
    flags = [f for f in COMMON if f != CSRC] + [f"-D{d}" for d in defines]
    build_dir = os.path.join(os.path.dirname(lib), "_build_" + os.path.basename(lib)) \
        if out else BUILD
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, flags, build_dir, csrc), SOURCES))
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    import time
    t0 = time.time()
    build(verbose="-v" in sys.argv)
    print(f"built {LIB} in {time.time() - t0:.1f} s")
