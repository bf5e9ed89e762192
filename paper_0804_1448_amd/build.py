"""Build the HIP library ``libknn.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libknn.so")
# measurement only (the benchmark's peak-rate micro-kernels), not the k-NN ABI
PEAKS_SRC = "knn_peaks.hip"
PEAKS_LIB = os.path.join(PKG, "libknn_peaks.so")
SOURCES = ["knn_kernels.hip", "knn_api.cpp", "knn_server.cpp", "knn_noalloc.hip", "knn_wide.hip", "knn_wide_bf16.hip", "knn_wide_f16.hip", "knn_wide_f32.hip", "knn_lane.hip", "knn_lane_l2.hip"] + [
    f"knn_fused_{unit}_{v}.hip" for unit in ("f32lo", "f32hi", "bf16", "f16", "l1", "linf") for v in ("s", "l")]

# Packed float32 instructions are disabled on purpose: the compiler emits
# them by itself from ordinary float code, and this library does not use them.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build (host code
# only: the device code of this build is the ordinary one), for the CPU tests
# of the host logic; loaded with the toolchain's ASan runtime preloaded.
ASAN_LIB = os.path.join(ROOT, "_build", "libknn_asan.so")
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src: str, obj: str, extra=()):
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), cmd


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link ``libknn.so`` and
    ``libknn_peaks.so``; always recompiles."""
    import tempfile

    with tempfile.TemporaryDirectory(prefix="knn_build_") as tmpd:
        jobs = []
        for s in SOURCES:
            obj = os.path.join(tmpd, s + ".o")
            jobs.append((obj, *_compile(os.path.join(CSRC, s), obj)))
        pobj = os.path.join(tmpd, PEAKS_SRC + ".o")
        pproc, pcmd = _compile(os.path.join(CSRC, PEAKS_SRC), pobj)
        errs = []
        for obj, proc, cmd in jobs:
            out, err = proc.communicate()
            lines = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln]
            if proc.returncode != 0:
                errs.append(" ".join(cmd) + "\n" + "\n".join(lines))
            elif verbose and lines:
                print("\n".join(lines), file=sys.stderr)
        _, perr = pproc.communicate()
        if pproc.returncode != 0:
            errs.append(" ".join(pcmd) + "\n" + perr)
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n\n".join(errs))
        tmp = LIB + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *[o for o, _, _ in jobs], "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stderr)
        os.replace(tmp, LIB)
        ptmp = PEAKS_LIB + ".tmp"
        res = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", pobj, "-o", ptmp],
                             capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stderr)
        os.replace(ptmp, PEAKS_LIB)
    return LIB


def asan_runtime() -> str:
    """The toolchain's shared ASan runtime (to preload into the host process)."""
    import glob

    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return found[-1]


def build_host_sanitized(verbose: bool = False) -> str:
    """Compile every source with host AddressSanitizer and UBSan into
    _build/libknn_asan.so; always recompiles."""
    import tempfile

    os.makedirs(os.path.dirname(ASAN_LIB), exist_ok=True)
    with tempfile.TemporaryDirectory(prefix="knn_asan_") as tmpd:
        jobs = []
        for s in SOURCES:
            obj = os.path.join(tmpd, s + ".o")
            jobs.append((obj, *_compile(os.path.join(CSRC, s), obj, SANITIZE_FLAGS)))
        errs = []
        for obj, proc, cmd in jobs:
            _, err = proc.communicate()
            if proc.returncode != 0:
                errs.append(" ".join(cmd) + "\n" + err)
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n\n".join(errs))
        tmp = ASAN_LIB + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", *[o for o, _, _ in jobs], "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stderr)
        os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
