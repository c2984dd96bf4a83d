"""Compile the C oracle (plain gcc, no fast-math) into oracle/liborc.so."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path(sanitized: bool = False) -> str:
    return os.path.join(_HERE, "liborc_san.so" if sanitized else "liborc.so")


def build_oracle(verbose: bool = False, sanitized: bool = False) -> str:
    """liborc.so, or with sanitized=True liborc_san.so built with the address
    and undefined-behaviour sanitizers (loaded only when ORACLE_LIB names it)."""
    src = os.path.join(_HERE, "orc.c")
    out = library_path(sanitized)
    tmp = out + ".tmp"
    flags = ["-O2"] if not sanitized else ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                           "-fno-sanitize-recover=undefined"]
    cmd = ["gcc", *flags, "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose=True))
