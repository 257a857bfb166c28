"""Compile the HIP library libpbdsbi.so for gfx950, in-tree."""
from __future__ import annotations

import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("pb_kernels.hip", "pb_batch.hip", "pb_tree.hip", "pb_noalloc.hip", "pb_capi.hip")]
# plain C++ host logic (no device code), also built by the host sanitizer test
HOST_SOURCES = [os.path.join(HERE, "csrc", "pb_host.cpp")]
LIB = os.path.join(HERE, "libpbdsbi.so")
# the same library with its host code under sanitizers (device code
# unchanged), loaded only by the sanitizer tests: SAN_LIB with AddressSanitizer
# and UndefinedBehaviorSanitizer (ROCm's ASan runtime preloaded; its
# interceptor of HSA memory-pool allocations needs device ASan, so this one
# runs without a GPU), UBSAN_LIB with UndefinedBehaviorSanitizer alone
# (minimal runtime), which runs on the GPU
SAN_LIB = os.path.join(HERE, "libpbdsbi_hostsan.so")
UBSAN_LIB = os.path.join(HERE, "libpbdsbi_hostubsan.so")
LLVM = "/opt/rocm/lib/llvm"
ARCH = "gfx950"

# Packed FP32 instructions are kept out of the build (they are not trusted on
# this hardware).  The flag reaches the host pass too, which ignores it with a
# warning: no driver form sends a -Xclang pair to the device pass alone.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def device_targets(path: str = LIB) -> set:
    """The offload targets of the device code objects bundled in a library."""
    with open(path, "rb") as f:
        data = f.read()
    return {m.decode() for m in re.findall(rb"amdgcn-amd-amdhsa-[a-z0-9:+-]*gfx[0-9a-z]+", data)}


def _run(cmd: list) -> subprocess.CompletedProcess:
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    return res


def _link(out: str, hip_flags: list, host_objs: list, link_flags: list, tag: str,
          verbose: bool) -> str:
    """Compile every HIP source to its own object in parallel (one fat binary
    per object), link them with the host objects into `out` (atomically),
    and check that the device code is gfx950's only."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = out + ".tmp"
    objs = [os.path.join(HERE, os.path.splitext(os.path.basename(src))[0] + f"_{tag}.o")
            for src in SOURCES]
    compile_flags = [f for f in hip_flags if f != "-shared"]
    cmds = [[hipcc(), *compile_flags, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    try:
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            results = list(ex.map(_run, cmds))
        # host objects after "-x none": given as C++ sources, hipcc would drop
        # --offload-arch and build device code for its default target
        res = _run([hipcc(), *hip_flags, *link_flags, "-o", tmp, *objs, "-x", "none", *host_objs])
    finally:
        for obj in objs + list(host_objs):
            if os.path.exists(obj):
                os.remove(obj)
    if verbose:
        for r in results + [res]:
            if r.stdout or r.stderr:
                print(r.stdout + r.stderr)
    targets = device_targets(tmp)
    if targets != {f"amdgcn-amd-amdhsa--{ARCH}"}:
        os.remove(tmp)
        raise RuntimeError(f"built device code targets {sorted(targets)}, expected only {ARCH}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Always recompiles; writes libpbdsbi.so atomically next to this file.
    The plain C++ host sources are compiled to objects by the host compiler."""
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(HERE, os.path.splitext(os.path.basename(src))[0] + ".o")
        _run([os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall",
              "-c", src, "-o", obj])
        objs.append(obj)
    return _link(LIB, HIPCC_FLAGS, objs, [], "prod", verbose)


def sanitizer_runtime(name: str) -> str | None:
    """A shared sanitizer runtime of ROCm's clang (libclang_rt.<name>-x86_64.so),
    or None."""
    base = os.path.join(LLVM, "lib", "clang")
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        path = os.path.join(base, ver, "lib", "linux", f"libclang_rt.{name}-x86_64.so")
        if os.path.exists(path):
            return path
    return None


def build_hostsan(kind: str = "asan", verbose: bool = False) -> str:
    """Always recompiles SAN_LIB (kind "asan": -fsanitize=address,undefined)
    or UBSAN_LIB (kind "ubsan": -fsanitize=undefined, minimal runtime): every
    -fsanitize after -Xarch_host, so the device code is built as in LIB; the
    plain C++ host sources by ROCm's clang++ (the same runtime as the HIP host
    code)."""
    out = SAN_LIB if kind == "asan" else UBSAN_LIB
    if kind == "asan":
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer"]
        host_san = ["-Xarch_host", "-fsanitize=address,undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all",
                    "-Xarch_host", "-fno-omit-frame-pointer"]
    else:
        san = ["-fsanitize=undefined", "-fsanitize-minimal-runtime", "-fno-sanitize-recover=all"]
        host_san = ["-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fsanitize-minimal-runtime",
                    "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(HERE, os.path.splitext(os.path.basename(src))[0] + f"_{kind}.o")
        _run([os.path.join(LLVM, "bin", "clang++"), "-O1", "-g", "-std=c++17", "-fPIC",
              "-pthread", *san, "-c", src, "-o", obj])
        objs.append(obj)
    flags = [f for f in HIPCC_FLAGS if f != "-O3"]
    return _link(out, ["-O2", "-Xarch_host", "-g", *flags, *host_san], objs, ["-shared-libsan"],
                 kind, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
