"""Build libslse.so for gfx950 in-tree with hipcc (one object per source, then link)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libslse.so")
SOURCES = [
    "k_resid_grad.hip",
    "k_update.hip",
    "k_srht.hip",
    "k_factor.hip",
    "k_adjoint.hip",
    "k_countsketch_gauss.hip",
    "k_batched.hip",
    "k_bandwidth.hip",
    "slse_host.hip",
]
ARCH = os.environ.get("SLSE_ARCH", "gfx950")
FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-c", *FLAGS, os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = max(1, min(8, len(srcs), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


ASAN_LIB = os.path.join(BUILD, "asan", "libslse_host_asan.so")


def asan_runtime():
    """The compiler's AddressSanitizer runtime (to preload into a host process)."""
    r = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def asan_build_is_current():
    if not os.path.exists(ASAN_LIB):
        return False
    t = os.path.getmtime(ASAN_LIB)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [
        os.path.join(HERE, "..", "include", "slse.h"), os.path.abspath(__file__)]
    return all(os.path.getmtime(f) <= t for f in deps if os.path.exists(f))


def build_host_asan(verbose=True):
    """The library with AddressSanitizer and UBSan on the host driver
    (slse_host.hip: the context, the solve and batch plans, the C-ABI entry
    points); the kernel objects are the regular ones.  For CPU runs of the
    host-only entry points (parameter helpers, the batch-plan check) in a
    process that preloads asan_runtime()."""
    out = os.path.join(BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    host_src = "slse_host.hip"
    kern = [s for s in SOURCES if s != host_src and os.path.exists(os.path.join(CSRC, s))]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined"]
    host_obj = os.path.join(out, "slse_host.o")

    def one(src):
        if src == host_src:
            r = subprocess.run(["hipcc", "-c", *flags, os.path.join(CSRC, src), "-o", host_obj],
                               capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc (host ASan) failed for {src}:\n{r.stderr}")
            return host_obj
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) >= max(
                os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC)):
            return obj
        return _compile(src)

    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max(1, min(8, len(kern) + 1))) as ex:
        objs = list(ex.map(one, [host_src] + kern))
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", *objs, "-o", ASAN_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (host ASan) failed:\n{r.stderr}")
    if verbose:
        print(f"built {ASAN_LIB}")
    return ASAN_LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
