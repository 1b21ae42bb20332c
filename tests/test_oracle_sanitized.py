"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): a sanitized build of the oracle, in a temporary folder,
drives every family of entry points (Philox, mean field, Newell tensor, FFT
and direct demag, local energy changes, energies, colour passes, runs with
grains, cubic anisotropy and a temperature profile, serial MMC) in a child
process; any memory error or undefined behaviour aborts it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
O._SO = sys.argv[2]
import workloads
O.philox((1, 2, 3, 4), (5, 6))
for mf in (0, 1):
    for T in (300.0, 700.0, 800.0):
        O.meanfield(mf, T, 700.0)
O.newell(1e-9, 2e-9, 0.0, 1e-9, 1e-9, 1e-9)
O.newell(40e-9, 3e-9, 2e-9, 2e-9, 2e-9, 1e-9)
grid, cell = (7, 5, 3), (3e-9, 2e-9, 2e-9)
N = 7 * 5 * 3
m = workloads.random_state(N, seed=3).astype(np.float64)
O.DemagPlan(grid, cell)(m)
O.demag_direct(grid, cell, m)
mat = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0)
S = O.System(grid, cell, T=400.0, D0=1e-3, K2=1e5, B=(0.01, 0.0, 0.1), demag=True, seed=2, **mat)
S.energy(m)
S.subsweep(m, 3, 1, 30.0)
S.run(S.init_state("random"), 4, cone_deg=30, adapt_every=2)
gid, ng = workloads.voronoi_grains(grid, cell, 4e-9, seed=1)
ea, K1, K2, Tc = workloads.grain_properties(ng, seed=2)
G = O.System(grid, cell, T=650.0, demag=True, seed=3, Ms0=1e6, A0=1e-11, K1=0.0, Tc=700.0, cls=gid, ea=ea,
             K1s=K1, K2s=K2, Tcs=Tc, bscale=0.1, Tcl=np.linspace(500.0, 800.0, ng),
             cubic_axes=np.tile(np.eye(3), (ng, 1, 1)), kscale=True)
G.run(G.init_state("uniform"), 3, cone_deg=30, adapt_every=0)
R = O.System((6, 4, 1), (5e-9,) * 3, T=300.0, demag=True, seed=4, **mat)
R.serial_run(R.init_state("uniform"), 3, cone_deg=30)
R.serial_run(R.init_state("uniform"), 2, cone_deg=30, self_term=True)
print("sanitized oracle: ok", flush=True)
'''


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    from oracle import build_oracle
    so = build_oracle.build(out=str(tmp_path / "libmmc_oracle_san.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", DRIVER, ROOT, so], env=env, capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "sanitized oracle: ok" in r.stdout
