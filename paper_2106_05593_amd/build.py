"""Build libmmc.so (the HIP library behind include/mmc.h) for gfx950, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libmmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# (source, extra defines, object name); the y pass is compiled once per layer count
UNITS = [("csrc/api.cpp", [], "api.o"), ("csrc/setup.cpp", [], "setup.o"), ("csrc/kernels.hip", [], "kernels.o"), ("csrc/sweep.hip", [], "sweep.o"),
         ("csrc/demag.hip", [], "demag.o"), ("csrc/persist.hip", [], "persist.o"),
         ("csrc/fused.hip", [], "fused.o"), ("csrc/ystage.hip", [], "ystage.o")] + \
        [("csrc/ypass.hip", ["-DMMC_NZ=%d" % k], "ypass_nz%d.o" % k) for k in range(1, 9)]


def build(verbose: bool = False, out: str = SO, defines=()) -> str:
    """Compile every unit and link `out` (default: the in-tree libmmc.so);
    defines: extra -D flags for every unit."""
    build_dir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(build_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              # packed FP32 instructions stay off
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
              "-I", os.path.join(ROOT, "include")]

    def compile_unit(u):
        src, defs, obj = u
        obj_path = os.path.join(build_dir, obj)
        cmd = [HIPCC] + common + list(defines) + defs + ["-x", "hip", "-c", os.path.join(HERE, src), "-o", obj_path]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr))
        return obj_path

    workers = max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(compile_unit, UNITS))
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", out + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
