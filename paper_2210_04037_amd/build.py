"""Build libfv.so (the C-ABI library) for gfx950 with hipcc, in-tree."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfv.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # multiply-adds fused per source expression: every inlined copy of a
    # function rounds alike, so a value (a tile cell's primitives, a face
    # flux computed by two neighbouring tiles) does not depend on which code
    # path formed it
    "-ffp-contract=on",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# per translation unit: the FP32-bulk kernels take fast reciprocals and
# approximate transcendental functions, the FP64 form keeps IEEE arithmetic
# The face and halo phases of the stage kernels are loops over items; hoisting
# their constants (EOS and log/exp coefficients) out of them keeps those in
# registers across the whole phase for no gain, so machine-level
# loop-invariant code motion is off for the two kernel units.
KERNEL_UNIT = ["-mllvm", "-disable-machine-licm"]
UNITS = [
    ("fv_api.hip", []),
    ("fv_fp64.hip", KERNEL_UNIT),
    ("fv_fp32.hip", KERNEL_UNIT + ["-fno-hip-fp32-correctly-rounded-divide-sqrt",
                                   "-freciprocal-math", "-fapprox-func",
                                   "-fno-math-errno"]),
]


def build(verbose=False, extra=()):
    """Compile the units in parallel, link libfv.so."""
    objs, procs = [], []
    for src, flags in UNITS:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = ([hipcc()] + FLAGS + flags + list(extra)
               + ["-c", "-o", obj, os.path.join(CSRC, src)])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed.append(src)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
