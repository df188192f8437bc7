"""Build libskls.so (HIP for gfx950) in-tree with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libskls.so")
SOURCES = ["api.cpp", "profile.cpp", "noalloc.hip", "sketch.hip", "dense.hip", "lsqr.hip", "leverage.hip", "learned.hip", "lowrank.hip", "regress.hip", "lp.hip", "stage2.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libskls)")


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-fvisibility=hidden",
        "-Wall",
        "-Wno-unused-function",
        # no packed fp32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-I", CSRC,
    ]


def build(verbose: bool = True, jobs: int = 6) -> str:
    """Compile every source to an object and link libskls.so (always rebuilds)."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [cc, *flags(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            time.sleep(0.05)
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and any("warning" in ln for ln in lines):
            print("\n".join(lines), file=sys.stderr)
    if failed:
        msg = "\n\n".join(f"== {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    subprocess.run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", file=sys.stderr)
    return LIB


# Host-code sanitizers: every flag applies to the host compilation only
# (-Xarch_host); the device code is built as usual and not instrumented.  The
# result serves host-side checks of the C ABI (argument validation,
# workspace arithmetic).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(outdir: str, driver: str, jobs: int = 6) -> str:
    """Compile the library's host code with AddressSanitizer and
    UndefinedBehaviorSanitizer into ``outdir`` and link it with the C program
    ``driver``; returns the path of the executable."""
    cc = hipcc()
    os.makedirs(outdir, exist_ok=True)
    base = [f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SAN_FLAGS]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [cc, *base, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            time.sleep(0.05)
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            failed.append(f"== {src}\n{out}")
    if failed:
        raise RuntimeError("sanitized host build failed:\n" + "\n".join(failed))
    lib = os.path.join(outdir, "libskls_host_san.so")
    subprocess.run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib, *objs, *SAN_FLAGS], check=True)
    exe = os.path.join(outdir, "abi_check")
    drv_obj = os.path.join(outdir, "driver.o")
    subprocess.run([cc, "-x", "c", "-O1", "-g", "-I", os.path.join(ROOT, "include"), *SAN_FLAGS, "-c", driver,
                    "-o", drv_obj], check=True)
    subprocess.run([cc, "-o", exe, drv_obj, lib, *SAN_FLAGS, f"-Wl,-rpath,{outdir}"], check=True)
    return exe


if __name__ == "__main__":
    build()
