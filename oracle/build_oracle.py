"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libmmc_oracle.so.

Plain gcc, no GPU toolchain: the oracle shares nothing with the HIP library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libmmc_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "mmc_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
           "-o", SO + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
