"""Build ``libtvstencil.so`` (HIP kernels + C ABI) in-tree for gfx950.

Every translation unit is compiled with ``-ffp-contract=off`` and without
fast-math: the library's bit-exactness rests on each product and sum being
rounded separately, in canonical order.  Packed FP32 instructions are
disabled for the device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtvstencil.so")

ARCH = os.environ.get("TVS_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, f))
    return out


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    hs.append(os.path.join(ROOT, "include", "tvstencil.h"))
    return max(os.path.getmtime(h) for h in hs)


# Host sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) for the
# host side of the library: plan validation, tuning strings and cache, the
# server's policy.  Device code is built as usual (no GPU sanitizer).
SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-omit-frame-pointer -shared-libsan").split()
SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_BUILD, "libtvstencil.so")


def _compile(src: str, verbose: bool, newer_than: float = None, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src) + ".o")
    if newer_than is not None and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > newer_than and t > os.path.getmtime(src):
            return obj
    cmd = [HIPCC, *COMMON, *(SANITIZE if sanitize else []), "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature; that warning is expected
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn and verbose:
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False,
          sanitize: bool = False) -> str:
    """Compile every source (incremental: only those older than their object
    or than any header) and link the library.  sanitize: a host-sanitized
    copy in _build/sanitize/ instead (load it with the sanitizer runtime
    preloaded; see sanitizer_env)."""
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(8, len(srcs))
    newer = _headers_mtime() if incremental else None
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, newer, sanitize), srcs))
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *(SANITIZE if sanitize else []),
           *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def sanitizer_env() -> dict:
    """Environment for running the CPU tests against the sanitized builds:
    the sanitizer runtime preloaded, leak checks off (the interpreter's own
    allocations are not this library's), both libraries redirected."""
    rt = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                "TVS_LIBRARY": SAN_LIB,
                "TVS_ORACLE_LIBRARY": os.path.join(SAN_BUILD, "liboracle.so")})
    return env


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        # host-sanitized library and oracle, then the CPU test suite against them
        print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv, sanitize=True))
        sys.path.insert(0, ROOT)
        from oracle import build as obuild
        print(obuild.build(sanitize=True))
        sys.exit(subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                                 os.path.join(ROOT, "tests")], env=sanitizer_env()).returncode)
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
