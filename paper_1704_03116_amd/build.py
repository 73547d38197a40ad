"""Build libdope.so (the C-ABI library of include/dope.h) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdope.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code (no float arithmetic is on this path anyway).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


# Stencils whose kernels are compiled in a translation unit of their own (dope_kernels.hip with DOPE_CONN set),
# so that the build runs in parallel; the unit without DOPE_CONN holds the launchers and the stencil-free kernels.
STENCILS = [4, 8, 24, 48, 80, 6, 32, 122, 256]


# The instrumented variant: the block max-flow of the 3x3 stencils checks its cut (DOPE_DEBUG) and reports a
# violation as a solver error; every other unit is the normal build's object.
DEBUG_OUT = os.path.join(HERE, "libdope_debug.so")
DEBUG_STENCILS = [4, 8, 6]


def build(verbose: bool = False, debug: bool = True) -> str:
    """Builds libdope.so and, unless debug is False, libdope_debug.so.  Returns the path of libdope.so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    kern = os.path.join(CSRC, "dope_kernels.hip")
    units = [([kern], "dope_kernels_main.o", [])] + \
            [([kern], f"dope_kernels_{c}.o", [f"-DDOPE_CONN={c}"]) for c in STENCILS] + \
            [([os.path.join(CSRC, "dope_abi.cpp")], "dope_abi.o", []),
             ([os.path.join(CSRC, "dope_noalloc.hip")], "dope_noalloc.o", []),
             ([os.path.join(CSRC, "dope_probe.hip")], "dope_probe.o", []),
             ([os.path.join(CSRC, "dope_multilabel.hip")], "dope_multilabel.o", [])]
    debug_units = [([kern], f"dope_kernels_{c}_debug.o", [f"-DDOPE_CONN={c}", "-DDOPE_DEBUG"])
                   for c in DEBUG_STENCILS] if debug else []
    compile_flags = [f for f in FLAGS if f != "-shared"]

    def compile_one(unit):
        srcs, obj, extra = unit
        cmd = [HIPCC] + compile_flags + extra + ["-c", "-o", os.path.join(objdir, obj)] + srcs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return os.path.join(objdir, obj)

    def link(objs, out):
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)

    workers = max(1, min(len(units) + len(debug_units), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, units + debug_units))
    link(objs[:len(units)], OUT)
    if debug:
        swap = {f"dope_kernels_{c}.o": f"dope_kernels_{c}_debug.o" for c in DEBUG_STENCILS}
        link([os.path.join(objdir, swap.get(os.path.basename(o), os.path.basename(o))) for o in objs[:len(units)]],
             DEBUG_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
