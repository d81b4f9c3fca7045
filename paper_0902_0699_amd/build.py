"""Build libpaperkern.so in-tree with hipcc for gfx950.

    python -m paper_0902_0699_amd.build        (or python paper_0902_0699_amd/build.py)
    python -m paper_0902_0699_amd.build --stale   (recompile only out-of-date objects)

Every HIP source is compiled with packed FP32 instructions disabled.
"""

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpaperkern.so")
# the pass and batched kernel instances come first: they take longest to compile
SOURCES = [
    # longest compiles first, so that the parallel build ends with short ones
    "pk_pass_f64r5.hip", "pk_batched_f64.hip", "pk_batched_f32.hip", "pk_pass_f64bwd.hip", "pk_pass_f32r5.hip",
    "pk_pass_f32bwd.hip", "pk_pass_f64r3.hip", "pk_pass_f64t.hip", "pk_plan.cpp", "pk_api.cpp", "pk_search.hip",
    "pk_density.hip", "pk_shor.hip", "pk_kernels.hip", "pk_pass_f32r3.hip", "pk_repeat_f64.hip", "pk_pass_f64.hip",
    "pk_pass_f32.hip", "pk_repeat_f32.hip"]
# rocSOLVER (and the rocBLAS handle it runs on) gives the density matrix's eigenvalues
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _stale(src, obj):
    """An object is stale when it is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in (CSRC, INCLUDE) for f in os.listdir(d) if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose=False, jobs=None, only_stale=False):
    """Compile every source to an object in parallel, then link the shared library.
    ``only_stale`` recompiles only objects older than their source or a header."""
    if jobs is None:
        jobs = max(1, min(8, os.cpu_count() or 1))
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function",
        # keep the four register-bit variants of each gate as separate code: merging
        # them selects registers through pointers and moves the tile to scratch
        "-mllvm", "-simplifycfg-sink-common=false",
    ]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        if only_stale and not _stale(os.path.join(CSRC, src), obj):
            continue
        cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common
        if verbose:
            print(" ".join(cmd), flush=True)
        # compiler output goes to a file: a pipe nobody reads would block the compiler
        log = open(obj + ".log", "w+b")
        procs.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
        while len([p for p in procs if p[1].poll() is None]) >= jobs:
            time.sleep(0.2)
    failed = []
    for src, p, log in procs:
        p.wait()
        log.seek(0)
        out = log.read().decode(errors="replace")
        log.close()
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out:
            sys.stderr.write(out)
    for src, out in failed:
        sys.stderr.write(out)
    if failed:
        raise RuntimeError("hipcc failed on %s" % ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + LIBS
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, only_stale="--stale" in sys.argv))
