"""Switching-time experiment on the oracle: the parallel MMC algorithm (frozen
demag field, refreshed once per sweep as in the paper, or before each colour
pass) against the serial one whose demag field is updated after every
accepted move (paper Sec. III, the comparison of switching statistics).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  One event is a
chain started uniform against the field; its switching time is the first
sweep after which <m_x> along the field is positive (max_sweeps when it does
not switch).  Events run in worker processes (spawned, one OpenMP thread
each); every event is seeded, so results do not depend on the worker count.
"""
import os
import multiprocessing as mp

import numpy as np

from . import oracle as O


def _system(p, seed, refresh_per_sweep):
    return O.System(p["grid"], p["cell"], Ms0=p["Ms0"], A0=p["A0"], K1=p["K1"], Tc=p["Tc"], T=p["T"], B=p["B"],
                    demag=True, refresh_per_sweep=refresh_per_sweep, seed=seed, chain_id=0)


def switch_time(args):
    """args = (workload dict, seed, mode) with mode "parallel1" / "parallel2"
    (demag refreshes per sweep), "serial" (Eq. 14 with the current field) or
    "serial_exact" (exact energy change, self term included)."""
    p, seed, mode = args
    S = _system(p, seed, 2 if mode == "parallel2" else 1)
    m = S.init_state("uniform", direction=p["init_dir"])
    d = np.asarray(p["B"], dtype=np.float64)
    d /= np.linalg.norm(d)
    cone, win, h, chunk = p["cone_deg"], 0, None, 100
    for sw0 in range(0, p["max_sweeps"], chunk):
        if mode.startswith("serial"):
            ser, cone, win, h, _ = S.serial_run(m, chunk, sweep0=sw0, cone_deg=cone, adapt_every=p["adapt_every"],
                                                window=win, h=h, self_term=mode == "serial_exact")
        else:
            ser, cone, win = S.run(m, chunk, sweep0=sw0, cone_deg=cone, adapt_every=p["adapt_every"], window=win)
        k = np.nonzero(ser[:, :3] @ d > 0)[0]
        if len(k):
            return sw0 + int(k[0])
    return p["max_sweeps"]


def switch_times(p, seeds, mode, workers=8):
    """Switching times of the events with the given seeds."""
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return np.array(pool.map(switch_time, [(p, int(s), mode) for s in seeds]))
    finally:
        if old is None:
            del os.environ["OMP_NUM_THREADS"]
        else:
            os.environ["OMP_NUM_THREADS"] = old
