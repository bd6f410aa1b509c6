"""Compiles the HIP/C++ sources into the in-tree shared library libdgmg.so
(gfx950 code objects, host setup with OpenMP)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgmg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# packed FP32 instructions are disabled for all device code
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", "-Wno-unused-function",
          "-Wno-unused-result"]
HOST_SOURCES = ["setup_fem.cpp", "setup_mg.cpp"]
HIP_SOURCES = ["solver.hip", "setup_dev.hip"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("compilation failed")
    return r


# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only
# (each flag behind -Xarch_host: no device code is instrumented)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all", "-g"]


def build(verbose=False, sanitize=False):
    """Compiles libdgmg.so; sanitize=True builds _build_san/libdgmg_san.so
    with the host code under ASan + UBSan instead (load it with
    DGMG_LIB=<path> and the clang ASan runtime preloaded)."""
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    extra = SANITIZE if sanitize else []
    jobs = []
    for src in HOST_SOURCES:
        o = os.path.join(objdir, src + ".o")
        # plain C++ (hipcc would otherwise compile .cpp files as HIP for a default target)
        jobs.append(([HIPCC, "-x", "c++"] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", o], o))
    for src in HIP_SOURCES:
        o = os.path.join(objdir, src + ".o")
        jobs.append(([HIPCC, "-x", "hip"] + DEVICE_FLAGS + COMMON + extra +
                     ["-c", os.path.join(CSRC, src), "-o", o], o))
    # the translation units are independent: compile them concurrently
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [o for _, o in jobs]
    out = os.path.join(objdir, "libdgmg_san.so") if sanitize else LIB
    tmp = out + ".tmp"
    link_extra = (["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-shared-libsan"] if sanitize else [])
    _run([HIPCC] + DEVICE_FLAGS + link_extra + ["-shared", "-fopenmp", "-o", tmp] + objs +
         ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, out)
    if sanitize:
        return out
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
