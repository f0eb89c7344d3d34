"""Build step of the FP64 oracle library (test infrastructure).

Compiles ``phisft_oracle.cpp`` with the host C++ compiler into
``libphisft_oracle.so`` next to it. Generic x86-64 code (no -march=native) so
the library built here also runs on another host.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "phisft_oracle.cpp")


def library_path(sanitize: bool = False) -> str:
    return os.path.join(HERE, "libphisft_oracle_san.so" if sanitize else "libphisft_oracle.so")


def build_oracle(sanitize: bool = False, verbose: bool = False) -> str:
    out = library_path(sanitize)
    cmd = ["g++", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Wextra", "-o", out + ".tmp", SOURCE]
    if sanitize:
        cmd[1:1] = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    else:
        cmd[1:1] = ["-O3"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose=True))
