"""Build libpkm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1602_06693_amd.build [--jobs N] [--host-sanitize | --host-tsan]

Every translation unit under csrc/ is compiled to an object under _build/
and linked into paper_1602_06693_amd/libpkm.so.  Always recompiles.

--host-sanitize builds _build/hostsan/libpkm_hostsan.so instead: the host
code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
(device code unchanged), for tests of the host-side logic on a machine
without a GPU.  Load it with the compiler's ASan runtime preloaded
(hostsan_runtime() names it).  --host-tsan builds
_build/hosttsan/libpkm_hosttsan.so with ThreadSanitizer in the host code,
for a program built with -fsanitize=thread that links it.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libpkm.so")
ARCH = os.environ.get("PKM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs: the products feed exp2 and the
    # next MFMA directly, without accumulator-register copies
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result",
]


# host-only instrumentation: every sanitizer flag is scoped to the host
# compilation, never to the gfx950 code objects
HOSTSAN_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g",
]
HOSTSAN_DIR = os.path.join(OBJ, "hostsan")
HOSTSAN_LIB = os.path.join(HOSTSAN_DIR, "libpkm_hostsan.so")
# ThreadSanitizer, also host code only (the eigensolver's worker threads);
# the program that loads this library must itself be built with it
HOSTTSAN_FLAGS = [
    "-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g",
]
HOSTTSAN_DIR = os.path.join(OBJ, "hosttsan")
HOSTTSAN_LIB = os.path.join(HOSTTSAN_DIR, "libpkm_hosttsan.so")


def hostsan_runtime():
    """Path of the clang ASan runtime that a host-sanitized libpkm needs
    preloaded, or None."""
    import glob
    llvm = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "llvm")
    hits = sorted(glob.glob(os.path.join(llvm, "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    hits += sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[0] if hits else None


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, outdir=OBJ, extra=()):
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{p.stdout}\n{p.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False, host_sanitize: bool = False,
          host_tsan: bool = False) -> str:
    assert not (host_sanitize and host_tsan), "one sanitizer build at a time"
    outdir = HOSTSAN_DIR if host_sanitize else HOSTTSAN_DIR if host_tsan else OBJ
    lib = HOSTSAN_LIB if host_sanitize else HOSTTSAN_LIB if host_tsan else LIB
    extra = HOSTSAN_FLAGS if host_sanitize else HOSTTSAN_FLAGS if host_tsan else ()
    os.makedirs(outdir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2) - 1), 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, outdir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stdout}\n{p.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} from {len(objs)} objects")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--host-sanitize", action="store_true")
    ap.add_argument("--host-tsan", action="store_true")
    a = ap.parse_args()
    build(a.jobs, verbose=True, host_sanitize=a.host_sanitize, host_tsan=a.host_tsan)
    sys.exit(0)
