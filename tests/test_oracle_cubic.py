"""Pins of the oracle's cubic anisotropy (paper Sec. II, Eq. 12) and of the
me^{l(l+1)/2} temperature law of the anisotropy constants (Sec. III, Fe film).

* Uniform states along the crystal's <100>, <110> and <111> directions have
  the textbook cubic energies 0, K1/4 and K1/3 + K2/27 per unit volume, for
  any orientation of the crystal axes and any magnetization length (the
  energy depends on direction cosines only).
* The energy is invariant under the cubic group: permutations and sign
  changes of the crystal axes.
* The per-move dF equals the change of the total energy (cubic, per-class
  axes, per-class temperatures, scaled constants).
* With the temperature law a constant of order l scales as me^l(l+1)/2:
  uniaxial K1, K2 (orders 2, 4) by me^3, me^10; cubic K1, K2 (orders 4, 6) by
  me^10, me^21; the anisotropy vanishes at and above Tc.
* Macrospins sample exp(-F_cubic/kT) over directions (Eq. 1 with a length
  independent term, Eq. 6): <a^4 + b^4 + g^4> and <a^2 b^2 g^2> against 2-D
  quadrature over the sphere, for an easy-<100> and an easy-<111> crystal.
"""
import numpy as np
import pytest

KB = 1.380649e-23


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 2] *= -1
    return q.T            # rows: the crystal axes


def _cubic_system(oracle_mod, axes, K1=4.8e4, K2=-1.0e4, T=300.0, kscale=False, **kw):
    return oracle_mod.System((5, 4, 3), (2e-9, 2e-9, 2e-9), Ms0=1.71e6, A0=2.1e-11, K1=K1, K2=K2, Tc=1044.0,
                             T=T, cubic_axes=axes, kscale=kscale, **kw)


def test_principal_directions(oracle_mod):
    for seed in range(3):
        R = _rot(seed)
        S = _cubic_system(oracle_mod, R)
        V, N = np.prod(S.cell), S.N
        dirs = {(1, 0, 0): 0.0, (0, 1, 0): 0.0, (0, 0, -1): 0.0,
                (1, 1, 0): 4.8e4 / 4, (0, -1, 1): 4.8e4 / 4,
                (1, 1, 1): 4.8e4 / 3 - 1.0e4 / 27, (-1, 1, -1): 4.8e4 / 3 - 1.0e4 / 27}
        for d, w in dirs.items():
            n = np.array(d, float) @ R
            n /= np.linalg.norm(n)
            for L in (0.2, 0.77, 1.3):
                m = np.tile((L * n)[:, None], (1, N))
                E = S.energy(m)
                assert abs(E[2] - N * V * w) < 1e-12 * N * V * 4.8e4, (seed, d, L, E[2], N * V * w)


def test_cubic_group_invariance(oracle_mod):
    R = _rot(7)
    rng = np.random.default_rng(8)
    m = rng.normal(size=(3, 60)) * 0.5
    ref = _cubic_system(oracle_mod, R).energy(m)[2]
    for perm in ([1, 0, 2], [2, 0, 1], [0, 2, 1]):
        for sg in ([1, 1, 1], [-1, 1, 1], [1, -1, -1]):
            Rp = R[perm] * np.array(sg)[:, None]
            assert np.isclose(_cubic_system(oracle_mod, Rp).energy(m)[2], ref, rtol=1e-13, atol=0)
    # a generic rotation of the axes changes it
    assert not np.isclose(_cubic_system(oracle_mod, _rot(9)).energy(m)[2], ref, rtol=1e-3, atol=0)


@pytest.mark.parametrize("kscale,grains", [(False, False), (True, False), (True, True)])
def test_delta_F_equals_energy_change(oracle_mod, kscale, grains):
    grid = (5, 4, 3)
    N = int(np.prod(grid))
    kw = {}
    axes = _rot(3)
    if grains:
        rng = np.random.default_rng(4)
        cls = rng.integers(0, 3, N)
        axes = np.stack([_rot(s) for s in (10, 11, 12)])
        kw = dict(cls=cls, ea=np.tile([0.0, 0.0, 1.0], (3, 1)), K1s=[4.8e4, 3e4, -2e4], K2s=[-1e4, 2e4, 5e3],
                  Tcs=[1044.0, 900.0, 1000.0], bscale=0.1, Tcl=[300.0, 700.0, 950.0])
    S = _cubic_system(oracle_mod, axes, kscale=kscale, **kw)
    rng = np.random.default_rng(6)
    m = rng.normal(size=(3, N)) * 0.4
    E0 = S.energy(m)
    Tcl = np.asarray(kw.get("Tcl", [300.0] * 3))
    cls = kw.get("cls", np.zeros(N, dtype=int))
    for _ in range(40):
        p = int(rng.integers(0, N))
        mB = m[:, p] + rng.normal(size=3) * 0.2
        dF = S.delta_F(m, p, mB)
        m1 = m.copy()
        m1[:, p] = mB
        dE = S.energy(m1) - E0
        kT = KB * Tcl[cls[p]]
        assert abs(dF[2] * kT - dE[2]) < 1e-11 * (abs(E0[2]) + 1e-30), (p, dF[2] * kT, dE[2])


def test_temperature_law(oracle_mod):
    """Each order's exponent, from the ratio of scaled to unscaled energies."""
    R = _rot(2)
    rng = np.random.default_rng(3)
    m = rng.normal(size=(3, 60)) * 0.6
    for T in (300.0, 800.0, 1040.0):
        me = oracle_mod.meanfield(1, T, 1044.0, 9.2740100783e-24)[0]
        for K1, K2, p in ((4.8e4, 0.0, 10), (0.0, -1e4, 21)):
            on = _cubic_system(oracle_mod, R, K1, K2, T=T, kscale=True).energy(m)[2]
            off = _cubic_system(oracle_mod, R, K1, K2, T=T).energy(m)[2]
            assert np.isclose(on, off * me ** p, rtol=1e-12, atol=0), (T, p)
        for K1, K2, p in ((4e5, 0.0, 3), (0.0, 1e5, 10)):
            kw = dict(Ms0=1e6, A0=0.0, K1=K1, K2=K2, Tc=1044.0, T=T, easy_axis=(0.3, 0.1, 0.9))
            on = oracle_mod.System((4, 5, 3), (2e-9,) * 3, kscale=True, **kw).energy(m)[2]
            off = oracle_mod.System((4, 5, 3), (2e-9,) * 3, **kw).energy(m)[2]
            assert np.isclose(on, off * me ** p, rtol=1e-12, atol=0), (T, p)
    # at and above Tc the scaled anisotropy vanishes
    for T in (1044.0, 1100.0):
        assert _cubic_system(oracle_mod, R, T=T, kscale=True).energy(m)[2] == 0.0


def _sphere_quadrature(ka1, ka2):
    th = np.linspace(0.0, np.pi, 1201)
    ph = np.linspace(0.0, 2 * np.pi, 2401)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    a, b, g = np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)
    a2, b2, g2 = a * a, b * b, g * g
    F = ka1 * (a2 * b2 + a2 * g2 + b2 * g2) + ka2 * a2 * b2 * g2
    w = np.exp(-(F - F.min())) * np.sin(TH)
    I = lambda f: np.trapezoid(np.trapezoid(w * f, ph, axis=1), th)
    Z = I(1.0)
    return I(a2 * a2 + b2 * b2 + g2 * g2) / Z, I(a2 * b2 * g2) / Z


@pytest.mark.parametrize("ka1,ka2", [(4.0, -0.8), (-4.0, 0.0), (0.0, 60.0)])
def test_macrospin_cubic(oracle_mod, ka1, ka2):
    T, Tc = 300.0, 1044.0
    h = 5e-9
    V, kT = h ** 3, KB * T
    R = _rot(5)
    S = oracle_mod.System((64, 64, 1), (h,) * 3, Ms0=1.71e6, A0=0.0, K1=ka1 * kT / V, K2=ka2 * kT / V, Tc=Tc, T=T,
                          lenmode=1, seed=31, cubic_axes=R)
    m = S.init_state("random")
    ser, cone, win = S.run(m, 600, cone_deg=30, adapt_every=100)
    s4, s6 = [], []
    sw = 600
    for _ in range(60):
        ser, cone, win = S.run(m, 10, sweep0=sw, cone_deg=cone, adapt_every=100, window=win)
        sw += 10
        n = R @ (m / np.linalg.norm(m, axis=0))
        s4.append((n ** 4).sum(axis=0).mean())
        s6.append((n[0] ** 2 * n[1] ** 2 * n[2] ** 2).mean())
    q4, q6 = _sphere_quadrature(ka1, ka2)

    def bse(x, nb=10):
        x = np.asarray(x)
        b = x[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
        return b.mean(), b.std(ddof=1) / np.sqrt(nb)

    v4, e4 = bse(s4)
    v6, e6 = bse(s6)
    assert abs(v4 - q4) < 4 * e4 + 1e-3, (v4, q4, e4)
    assert abs(v6 - q6) < 4 * e6 + 2e-4, (v6, q6, e6)
