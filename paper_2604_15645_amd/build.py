"""Build libpinn.so (HIP kernels + C ABI host code) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpinn.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIP_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
    # packed FP32 VALU instructions stay off: some of their forms have given wrong results
    # on this hardware without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
SOURCES = ["k_forward_fp32.hip", "k_forward_bf16x3.hip", "k_forward_fp16x3.hip", "k_backward_fp32.hip",
           "k_backward_bf16x3.hip", "k_backward_fp16x3.hip", "k_batched.hip", "k_misc.hip", "k_fp64.hip", "pinn_noalloc.hip",
           "pinn_api.cpp"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    """Compile every source and link libpinn.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(min(len(SOURCES), max(2, os.cpu_count() or 2))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def asan_runtime():
    """The AddressSanitizer runtime of the ROCm clang (preloaded to run sanitized builds
    from an uninstrumented Python), or None."""
    import glob
    root = os.environ.get("ROCM_PATH", "/opt/rocm")
    c = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                      "libclang_rt.asan-x86_64.so")))
    return c[-1] if c else None


def build_host_asan():
    """libpinn with its host code (argument checks, planning, workspace layout, launch
    set-up) built with AddressSanitizer and UndefinedBehaviorSanitizer; the kernels are the
    objects of the last build().  Written to _build/libpinn_asan.so, which is returned."""
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, "pinn_api_asan.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [hipcc()] + HIP_FLAGS + ["-g"] + san + ["-c", os.path.join(CSRC, "pinn_api.cpp"), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    objs = [os.path.join(BUILD, s + ".o") for s in SOURCES if s != "pinn_api.cpp"]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError("build() first: missing %s" % missing)
    out = os.path.join(BUILD, "libpinn_asan.so")
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + san[:4] + ["-o", out] + objs + [obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
