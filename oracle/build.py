"""Build the FP64 CPU oracle (plain C, gcc, OpenMP) into ``oracle/liboracle.so``.

Test infrastructure only: the oracle checks the GPU library and is never a
fallback for it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "abc_oracle.c")
SEG_SRC = os.path.join(HERE, "seg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the oracle into ``out`` (default ``oracle/liboracle.so``).

    ``sanitize`` adds AddressSanitizer and UndefinedBehaviorSanitizer (host code
    only, gcc; every finding aborts).  Such a library must be loaded into a
    process that preloads the ASan runtime (``asan_runtime()``)."""
    lib = out or LIB
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all"] if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c99", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-fast-math", "-o", lib + ".tmp", SRC, SEG_SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def asan_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime (to preload into a sanitized run)."""
    return subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()


if __name__ == "__main__":
    print(build(verbose=True))
