"""Compile the FP64 CPU oracle (test infrastructure) into oracle/libmmc_oracle.so.

Plain gcc, no GPU toolchain: the oracle shares nothing with the HIP library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libmmc_oracle.so")


def build(verbose: bool = False, out: str = SO, sanitize: bool = False) -> str:
    """Compile the oracle into `out`; sanitize: with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; errors abort), for the
    sanitizer test."""
    src = os.path.join(HERE, "mmc_oracle.c")
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
                           "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
