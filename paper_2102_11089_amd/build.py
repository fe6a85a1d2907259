"""Build the HIP library ``libldpcci.so`` in-tree for gfx950 (hipcc cross-compiles without a GPU).

Usage: ``python -m paper_2102_11089_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libldpcci.so")
SOURCES = ["host.cpp", "dynamic.hip", "baseline.hip", "multiedge.hip", "batch.hip", "unrolled.hip", "sweep.hip",
           "noalloc.hip", "probe.hip"]
HEADERS = ["common.hpp", "kernels.hpp", "dyn_frame.hpp"]
ARCH = os.environ.get("LDPCCI_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources_digest() -> str:
    """sha256 over the library's HIP/C++ sources (name + content, sorted by name): ties a stored
    measurement to the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _compile_link(out: str, extra: list, verbose: bool, jobs: int) -> str:
    """Compile every HIP source with FLAGS + extra (one compiler process per source, in parallel)
    and link them into the shared library `out`."""
    import concurrent.futures
    import shutil
    import tempfile
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 8))
    work = tempfile.mkdtemp(prefix="ldpcci_build_")
    try:
        objs = [os.path.join(work, os.path.basename(src) + ".o") for src in srcs]

        def compile_one(src, obj):
            cmd = ["hipcc", *FLAGS, *extra, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(compile_one, s, o) for s, o in zip(srcs, objs)]:
                f.result()
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(work, ignore_errors=True)
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source (always recompiles) and link them into one shared library."""
    return _compile_link(LIB, [], verbose, jobs)


# Self-checking build for development and tests: after every single-edge update the kernels
# recompute the touched neighbourhood's derived state from its definition and count mismatches
# into the buffer whose device address the environment variable LDPCCI_SELFCHECK holds.
SELFCHECK_LIB = os.path.join(HERE, "libldpcci_selfcheck.so")


def build_selfcheck(verbose: bool = False, jobs: int = 0) -> str:
    """Compile the self-checking variant of the library (always recompiles)."""
    return _compile_link(SELFCHECK_LIB, ["-DLDPC_SELFCHECK"], verbose, jobs)


# Phase-timing build for development: the single-edge and multi-edge kernels sum clock64() deltas
# per phase into the buffer whose device address LDPCCI_PROF holds (profcase's `phase` case).
PROFILE_LIB = os.path.join(HERE, "libldpcci_profile.so")


def build_profile(verbose: bool = False, jobs: int = 0) -> str:
    """Compile the phase-timing variant of the library (always recompiles)."""
    return _compile_link(PROFILE_LIB, ["-DLDPC_PROFILE"], verbose, jobs)


# Host-side sanitizers: the host code (argument validation, table building, layout sizing) is
# instrumented with AddressSanitizer and UndefinedBehaviorSanitizer; device code never is.
SAN_DIR = os.path.join(HERE, "_build")
SAN_LIB = os.path.join(SAN_DIR, "libldpcci_asan.so")
SAN_HOST_SOURCES = ("host.cpp", "noalloc.hip")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-shared-libsan"]


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to be preloaded into the process that loads
    the sanitized library)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/llvm/lib/clang")
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    """Build SAN_LIB (host code sanitized) unless one built from the current sources exists."""
    import concurrent.futures
    import shutil
    import tempfile
    stamp = os.path.join(SAN_DIR, "sources.sha256")
    digest = sources_digest()
    if os.path.exists(SAN_LIB) and os.path.exists(stamp) and open(stamp).read().strip() == digest:
        return SAN_LIB
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    work = tempfile.mkdtemp(prefix="ldpcci_asan_")
    try:
        objs = [os.path.join(work, os.path.basename(src) + ".o") for src in srcs]

        def compile_one(src, obj):
            extra = SAN_FLAGS if os.path.basename(src) in SAN_HOST_SOURCES else []
            cmd = ["hipcc", *[f for f in FLAGS if f != "-O3"], "-O1", "-g", *extra, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1, 8)) as ex:
            for f in [ex.submit(compile_one, s, o) for s, o in zip(srcs, objs)]:
                f.result()
        cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-shared-libsan", "-o", SAN_LIB,
               *objs]
        subprocess.check_call(cmd)
        with open(stamp, "w") as fh:
            fh.write(digest + "\n")
    finally:
        shutil.rmtree(work, ignore_errors=True)
    return SAN_LIB


if __name__ == "__main__":
    # python -m paper_2102_11089_amd.build [selfcheck|profile]: the library, or one of its variants
    which = sys.argv[1] if len(sys.argv) > 1 else ""
    out = {"selfcheck": build_selfcheck, "profile": build_profile}.get(which, build)(verbose=True)
    print(out)
    sys.exit(0)
