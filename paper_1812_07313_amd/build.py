"""Build libbhq.so in-tree with hipcc for gfx950.

    python -m paper_1812_07313_amd.build

Compiles the HIP kernels, the C-ABI layer and the host list builder into
``paper_1812_07313_amd/libbhq.so``.  Packed FP32 instructions are disabled
for all device code (``-packed-fp32-ops``); the compiler emits plain VALU
FP32 operations.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbhq.so")
ARCH = os.environ.get("BHQ_OFFLOAD_ARCH", "gfx950")

SOURCES = ["bhq_kernels.hip", "bhq_tree.hip", "bhq_integrate.hip", "bhq_pm.hip",
           "bhq_order.hip", "bhq_upload.hip", "bhq_api.cpp", "bhq_lists.cpp"]
# the tree builders take their floating-point decisions with the same
# operations on host and device, the leapfrog updates round like plain
# FP64 arithmetic, and the particle-mesh kernels must find a particle's
# mesh cell with the same bits in every kernel: no fused multiply-adds there
NO_CONTRACT = {"bhq_tree.hip", "bhq_lists.cpp", "bhq_integrate.hip", "bhq_order.hip",
               "bhq_pm.hip"}
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# the force kernels' occupancy instances are requests: where a kernel's LDS
# cannot host that many waves the compiler keeps its own register allocation
# and would report it for every such instance
QUIET = {"bhq_kernels.hip": ["-Wno-pass-failed"]}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


PROBES = ["valu_rates", "interaction_rates", "mfma_cell_term"]
PROBE_DIR = os.path.join(PKG, "probes")


def build_probes(cc, verbose=False):
    """The measurement programs behind the FP32 ceiling of the force
    kernels (probes/*.cpp, HIP for gfx950), as executables next to their
    sources."""
    cmds = []
    for name in PROBES:
        cmd = [cc, "-O3", "-std=c++17", "--offload-arch=" + ARCH, "-x", "hip"] + DEVICE_FLAGS + [
            "-I", CSRC, "-o", os.path.join(PROBE_DIR, name),
            os.path.join(PROBE_DIR, name + ".cpp")]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
    with concurrent.futures.ThreadPoolExecutor(len(cmds)) as pool:
        for f in [pool.submit(subprocess.run, c, check=True) for c in cmds]:
            f.result()


def build(verbose=False, extra=()):
    """Compile every source and link libbhq.so (always rebuilds)."""
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        cmd = [cc, "-c", "-O3", "-std=c++17", "-fPIC", "-Wall",
               "--offload-arch=" + ARCH, "-I", INCLUDE, "-I", CSRC]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + DEVICE_FLAGS + ["-munsafe-fp-atomics"]
        if src in NO_CONTRACT:
            cmd += ["-ffp-contract=off"]
        cmd += QUIET.get(src, [])
        cmd += list(extra) + ["-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the sources compile independently: one compiler process each
    workers = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(subprocess.run, c, check=True) for c in cmds]:
            f.result()
    build_probes(cc, verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
