"""Compile the C oracle into ``oracle/liboracle.so`` (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off and no fast-math: every product and sum is rounded on its
# own; -O2 without -march keeps the generic x86-64 instruction set (no FMA).
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer copy in
    _build/sanitize/ (built with clang so that it shares the runtime the
    sanitized library uses)."""
    if sanitize:
        out = os.path.join(os.path.dirname(HERE), "_build", "sanitize", "liboracle.so")
        os.makedirs(os.path.dirname(out), exist_ok=True)
        cc = ["/opt/rocm/llvm/bin/clang", "-fsanitize=address,undefined", "-shared-libsan",
              "-fno-omit-frame-pointer"]
    else:
        out, cc = LIB, ["gcc"]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [*cc, *CFLAGS, os.path.join(HERE, "oracle.c"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
