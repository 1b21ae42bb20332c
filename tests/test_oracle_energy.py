"""Pins of the oracle's free-energy terms and per-move changes.

* Per-move dF (what the sweep uses) must equal the change of the total energy
  for every local term (exchange, DMI, anisotropy, Zeeman, longitudinal).
  For the frozen demag term the paper uses dF_d = -V mu0 dM.H_d (Eq. 14), whose
  difference from the exact total-energy change is (mu0 V Ms0^2/2) dm.N(0).dm.
* The totals match closed forms on uniform states, spin spirals and cycloids.
"""
import numpy as np
import pytest

KB = 1.380649e-23
MU0 = 4e-7 * np.pi


def _system(oracle_mod, T=420.0, demag=True, grains=False, B=(0.02, -0.05, 0.3)):
    grid, cell = (6, 5, 3), (4e-9, 3e-9, 2e-9)
    kw = dict(Ms0=8e5, A0=1.3e-11, D0=1.5e-3, K1=4e5, K2=1.2e5, Tc=700.0, T=T, B=B,
              easy_axis=(0.3, 0.2, 0.93), demag=demag)
    if grains:
        N = int(np.prod(grid))
        rng = np.random.default_rng(5)
        cls = rng.integers(0, 3, N)
        ea = rng.normal(size=(3, 3))
        ea /= np.linalg.norm(ea, axis=1)[:, None]
        kw.update(cls=cls, ea=ea, K1s=[4e5, 2e5, 6e5], K2s=[1e5, 0, 3e4], Tcs=[700.0, 650.0, 430.0], bscale=0.1)
    return oracle_mod.System(grid, cell, **kw)


@pytest.mark.parametrize("T,grains", [(420.0, False), (650.0, True), (760.0, False)])
def test_delta_F_equals_energy_change(oracle_mod, T, grains):
    S = _system(oracle_mod, T=T, grains=grains)
    rng = np.random.default_rng(6)
    m = rng.normal(size=(3, S.N)) * 0.4
    kT = KB * T
    h = S.demag(m)
    E0 = S.energy(m, h)
    V = np.prod(S.cell)
    for _ in range(40):
        p = int(rng.integers(0, S.N))
        mB = m[:, p] + rng.normal(size=3) * 0.2
        dF = S.delta_F(m, p, mB, h)
        m1 = m.copy()
        m1[:, p] = mB
        E1 = S.energy(m1)          # fresh demag field of the new state
        dE = E1 - E0
        scale = np.abs(E0).max() + np.abs(E1).max()
        for k in range(5):
            assert abs(dF[k] * kT - dE[k]) < 1e-11 * scale, k
        D = mB - m[:, p]
        N0 = oracle_mod.newell(0, 0, 0, *S.cell)
        N0 = np.array([[N0[0], N0[3], N0[4]], [N0[3], N0[1], N0[5]], [N0[4], N0[5], N0[2]]])
        self_term = 0.5 * MU0 * V * S.s.Ms0**2 * D @ N0 @ D
        assert abs(dE[5] - dF[5] * kT - self_term) < 1e-11 * scale


def test_uniform_state_closed_forms(oracle_mod):
    S = _system(oracle_mod, demag=False)
    V, N, kT = np.prod(S.cell), S.N, KB * S.s.T
    c = S.coeffs()
    th = 0.7
    for L in [0.3, c["me"], 0.95]:
        u = np.array([np.sin(th), 0.0, np.cos(th)])
        m = np.tile((L * u)[:, None], (1, N))
        E = S.energy(m)
        e = np.array([0.3, 0.2, 0.93]); e /= np.linalg.norm(e)
        d2 = (L * u @ e) ** 2
        assert abs(E[0]) < 1e-30 and abs(E[1]) < 1e-30
        assert np.isclose(E[2], N * V * (4e5 * (1 - d2) + 1.2e5 * (1 - d2) ** 2), rtol=1e-13)
        assert np.isclose(E[3], -N * V * 8e5 * (L * u) @ np.array([0.02, -0.05, 0.3]), rtol=1e-13)
        Fl = c["la"] * (L * L - c["me"] ** 2) ** 2
        assert np.isclose(E[4], N * kT * Fl, rtol=1e-12, atol=1e-30)


def test_spiral_and_cycloid_closed_forms(oracle_mod):
    grid, cell = (16, 4, 2), (4e-9, 3e-9, 2e-9)
    S = oracle_mod.System(grid, cell, Ms0=8e5, A0=1.3e-11, D0=1.5e-3, K1=0.0, Tc=700.0, T=300.0)
    nx, ny, nz = grid
    V = np.prod(cell)
    k = 0.37 / cell[0]
    x = np.tile(np.arange(nx), ny * nz)
    # cycloid in the xz plane: m = (sin kx, 0, cos kx)
    m = np.stack([np.sin(k * cell[0] * x), 0 * x, np.cos(k * cell[0] * x)])
    E = S.energy(m)
    nb = (nx - 1) * ny * nz
    assert np.isclose(E[0], nb * V * 1.3e-11 * (2 - 2 * np.cos(k * cell[0])) / cell[0] ** 2, rtol=1e-12)
    # Eq. 15 energy density -D (m_z d_x m_x - m_x d_x m_z) -> -D k; per x-bond sin(k h)/h
    assert np.isclose(E[1], -nb * V * 1.5e-3 * np.sin(k * cell[0]) / cell[0], rtol=1e-12)
    # a helix (rotation in the plane normal to x) carries no interfacial DMI energy
    m = np.stack([0 * x, np.sin(k * cell[0] * x), np.cos(k * cell[0] * x)])
    assert abs(S.energy(m)[1]) < 1e-12 * abs(E[1])


def test_exchange_dmi_isotropic_about_z(oracle_mod):
    S = _system(oracle_mod, demag=False)
    rng = np.random.default_rng(8)
    m = rng.normal(size=(3, S.N))
    E = S.energy(m)
    a = 1.1
    R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    E2 = S.energy(R @ m)
    assert np.isclose(E[0], E2[0], rtol=1e-12) and np.isclose(E[1], E2[1], rtol=1e-12)
