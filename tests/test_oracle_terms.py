"""Relative size of the free-energy terms of trial moves (paper Sec. III and
App. B, Fig. 11): for a Ni80Fe20 element at room temperature the exchange
change of a trial move dominates, and the demag change is one to two orders
smaller, which is what makes a demag field frozen over a colour pass (or a
sweep) acceptable.  Mean |dF| per term over proposals drawn like the sweep's
(uniform on a 30 degree cap, length factor in [1 - sigma, 1 + sigma])."""
import numpy as np


def test_exchange_dominates_demag(oracle_mod):
    grid, cell = (40, 20, 4), (5e-9,) * 3
    S = oracle_mod.System(grid, cell, Ms0=8.6e5, A0=1.3e-11, K1=0.0, Tc=870.0, T=300.0, demag=True, seed=2)
    c = S.coeffs()
    N = S.N
    rng = np.random.default_rng(3)
    import workloads
    m = workloads.perturbed_uniform_state(N, seed=8, L=c["me"], spread=0.15, axis=(1.0, 0.0, 0.0)).astype(np.float64)
    h = S.demag(m)
    omc = 1.0 - np.cos(np.radians(30.0))
    dF = []
    for p in rng.integers(0, N, 400):
        a = m[:, p]
        n = a / np.linalg.norm(a)
        t = rng.uniform() * omc
        ct, st, ph = 1.0 - t, np.sqrt(t * (2.0 - t)), 2.0 * np.pi * rng.uniform()
        e1 = np.cross(n, [0.0, 0.0, 1.0] if abs(n[2]) < 0.9 else [1.0, 0.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(n, e1)
        nb = ct * n + st * (np.cos(ph) * e1 + np.sin(ph) * e2)
        f = 1.0 + c["sigma"] * (2.0 * rng.uniform() - 1.0)
        dF.append(S.delta_F(m, int(p), f * np.linalg.norm(a) * nb, h))
    mean = np.abs(np.array(dF)).mean(axis=0)       # ex, dmi, anis, zeeman, long, demag (kT units)
    print("mean |dF|/kT: exchange %.3g, longitudinal %.3g, demag %.3g" % (mean[0], mean[4], mean[5]))
    assert mean[0] > 10.0 * mean[5]
    assert mean[5] > 0.0
