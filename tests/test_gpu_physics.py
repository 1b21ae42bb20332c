"""The GPU path against closed forms and independent numerics (not against the
oracle): pins of the library's own host set-up and demag path that would catch
a misreading shared by the library and the oracle.

  * Demag (Sec. III, Eq. 14): for a uniformly magnetised rectangular block the
    block average of h = H_d / Ms0 is minus the block's demagnetizing factors,
    which Aharoni's closed form gives (A. Aharoni, J. Appl. Phys. 83, 3432
    (1998)); the cross components average to zero.  This checks the library's
    Newell tensor, its spectrum and the FFT kernels together, on the
    one-kernel and the staged y pass.
  * Mean field (Eqs. 8, 9): below Tc a chain starts at |m| = me(T), the root
    of the mean-field equation, here solved from scratch with brentq.
  * Above Tc (Eq. 7): the start length is sqrt(<m^2>) under the density
    m^2 exp(-F(m)/kT) of the length, F/kT = a2 m^2 + a4 m^4 with
    a2 = V Ms0 / (2 chi kT) and a4 = a2 c Tc / (T - Tc), chi the zero-field
    mean-field susceptibility (mu / (k (T - Tc)) for J = 1/2 and
    mu / (3 k (T - Tc)) for the Langevin form; c = 1/6 and 3/10), by
    adaptive quadrature.
  * Length-move width (Eq. 13): sigma = min(2 me sqrt(kT chi / (V Ms0)), 0.03)
    with chi = dm/dB from central differences of the brentq solution.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

from test_oracle_demag import aharoni

pytestmark = pytest.mark.gpu

KB = 1.380649e-23
MUB = 9.2740100783e-24
MAT = dict(Ms0=1e6, A0=1e-11, K1=0.0, Tc=700.0)


@pytest.fixture(scope="module")
def pkg():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_05593_amd as p
    return p


def _solve_m(model, T, Tc, B, mu=MUB, lo=1e-12):
    """Mean-field m at field B (tesla) by brentq on [lo, 1] (lo selects the
    positive branch when B < 0)."""
    if model == 1:
        g = lambda m: np.tanh((Tc * m + mu * B / KB) / T) - m
    else:
        def L(x):
            return 1.0 / np.tanh(x) - 1.0 / x if abs(x) > 1e-3 else x / 3.0 - x**3 / 45.0
        g = lambda m: L((3 * Tc * m + mu * B / KB) / T) - m
    return brentq(g, lo, 1.0, xtol=1e-16, rtol=1e-15, maxiter=500)


@pytest.mark.parametrize("grid,cell", [((10, 6, 3), (5e-9,) * 3), ((24, 24, 1), (4e-9, 4e-9, 2e-9)),
                                       ((64, 48, 4), (5e-9, 4e-9, 3e-9)), ((300, 20, 2), (3e-9,) * 3),
                                       ((20, 16, 10), (2e-9,) * 3)])
def test_uniform_block_demag_matches_aharoni(pkg, grid, cell):
    N = int(np.prod(grid))
    D = aharoni(*(np.array(grid, dtype=np.float64) * np.array(cell)))
    ch = pkg.Chain(grid, cell, T=300.0, demag=True, **MAT)
    for ax in range(3):
        m = np.zeros((3, N), dtype=np.float32)
        m[ax] = 1.0
        ch.set_m(m)
        h = ch.demag_field().astype(np.float64)
        print(grid, ax, -h[ax].mean(), D[ax])
        assert abs(-h[ax].mean() - D[ax]) < 2e-6
        other = [k for k in range(3) if k != ax]
        assert np.abs(h[other].mean(axis=1)).max() < 2e-6
    ch.close()


@pytest.mark.parametrize("mf", [0, 1])
@pytest.mark.parametrize("t", [0.3, 0.7, 0.95])
def test_start_length_below_tc_is_me(pkg, mf, t):
    T = t * MAT["Tc"]
    ch = pkg.Chain((8, 4, 1), (5e-9,) * 3, T=T, mf=mf, init=0, **MAT)
    L = np.linalg.norm(ch.get_m().astype(np.float64), axis=0)
    me = _solve_m(mf, T, MAT["Tc"], 0.0)
    assert np.abs(L / me - 1.0).max() < 1e-6, (L[0], me)
    ch.close()


@pytest.mark.parametrize("mf", [0, 1])
@pytest.mark.parametrize("t", [1.02, 1.1, 1.5])
def test_start_length_above_tc_is_rms_length(pkg, mf, t):
    Tc, T = MAT["Tc"], t * MAT["Tc"]
    cell = (5e-9, 4e-9, 2e-9)
    V = float(np.prod(cell))
    chi = MUB / ((1.0 if mf == 1 else 3.0) * KB * (T - Tc))
    a2 = V * MAT["Ms0"] / (2.0 * chi * KB * T)
    a4 = a2 * (1.0 / 6.0 if mf == 1 else 0.3) * Tc / (T - Tc)
    w = np.exp(-0.25 * np.log(a4)) if a2 < 1 else 1.0 / np.sqrt(a2)
    f = lambda m, k: m**k * np.exp(-(a2 * m * m + a4 * m**4))
    up = 20.0 * w
    m4 = quad(f, 0.0, up, args=(4,), epsabs=0, epsrel=1e-12, limit=200)[0]
    m2 = quad(f, 0.0, up, args=(2,), epsabs=0, epsrel=1e-12, limit=200)[0]
    expect = np.sqrt(m4 / m2)
    ch = pkg.Chain((8, 4, 1), cell, T=T, mf=mf, init=0, **MAT)
    L = np.linalg.norm(ch.get_m().astype(np.float64), axis=0)
    print(mf, T, L[0], expect)
    assert np.abs(L / expect - 1.0).max() < 2e-6
    ch.close()


@pytest.mark.parametrize("mf", [0, 1])
@pytest.mark.parametrize("t", [0.6, 0.9, 0.99])
def test_length_move_width(pkg, mf, t):
    Tc, T = MAT["Tc"], t * MAT["Tc"]
    cell = (3e-9, 3e-9, 3e-9)
    V = float(np.prod(cell))
    me = _solve_m(mf, T, Tc, 0.0)
    dB, lo = 1e-3, 0.5 * me
    chi = (_solve_m(mf, T, Tc, dB, lo=lo) - _solve_m(mf, T, Tc, -dB, lo=lo)) / (2 * dB)
    chi2 = (_solve_m(mf, T, Tc, dB / 2, lo=lo) - _solve_m(mf, T, Tc, -dB / 2, lo=lo)) / dB
    chi = chi2 + (chi2 - chi) / 3.0                     # Richardson step
    sigma = min(2.0 * me * np.sqrt(KB * T * chi / (V * MAT["Ms0"])), 0.03)
    ch = pkg.Chain((8, 4, 1), cell, T=T, mf=mf, init=0, **MAT)
    got = ch.stats()["sigma"]
    print(mf, T, got, sigma)
    assert abs(got / sigma - 1.0) < 1e-5
    ch.close()


@pytest.mark.parametrize("lenmove", [0, 1])
def test_macrospin_length_law(pkg, lenmove):
    """Isotropic macrospins (3 nm cells, no exchange, anisotropy, field or
    demag, 0.9 Tc, J = 1/2): the per-sweep FP64 means of |m|^2 over 20,000
    sweeps of 256x256 cells against the stationary law of the length move's
    own kernel, solved on a log-length grid from coefficients computed here
    (me by brentq, chi by Richardson differences, la = V Ms0 / (8 chi me^2 kT),
    sigma by Eq. 13 with its cap).  The paper's rule (lenmove 0) lands on its
    law, which differs from the Eq. 1 value; the exact rule (lenmove 1) on the
    Eq. 1 value."""
    from paper_2106_05593_amd.hysteresis import blocked_se
    from test_oracle_sampler import length_chain_m2
    Tc, T, cell, Ms0 = 700.0, 630.0, 3e-9, 1e6
    V = cell ** 3
    me = _solve_m(1, T, Tc, 0.0)
    dB, lo = 1e-3, 0.5 * me
    chi = (_solve_m(1, T, Tc, dB, lo=lo) - _solve_m(1, T, Tc, -dB, lo=lo)) / (2 * dB)
    chi2 = (_solve_m(1, T, Tc, dB / 2, lo=lo) - _solve_m(1, T, Tc, -dB / 2, lo=lo)) / dB
    chi = chi2 + (chi2 - chi) / 3.0
    c = {"me": me, "below": 1, "la": V * Ms0 / (8 * chi * me * me * KB * T), "lb": 0.0, "lbc": 0.0,
         "sigma": min(2.0 * me * np.sqrt(KB * T * chi / (V * Ms0)), 0.03)}
    law, eq1 = length_chain_m2(c, lenmove, c["sigma"] / 64)
    ch = pkg.Chain((256, 256, 1), (cell,) * 3, Ms0=Ms0, A0=0.0, K1=0.0, Tc=Tc, T=T, lenmove=lenmove, seed=31,
                   init=0)
    assert abs(ch.stats()["sigma"] / c["sigma"] - 1) < 1e-5
    ch.sweep(500)
    x = np.concatenate([np.asarray(ch.sweep_record(5000))[:, 3] for _ in range(4)])
    got, se = float(x.mean()), blocked_se(x)
    print("lenmove", lenmove, "sampled %.7f +- %.1e, kernel law %.7f, Eq. 1 %.7f" % (got, se, law, eq1), flush=True)
    ch.close()
    assert abs(got - law) < 4 * se + 2e-6 * law
    if lenmove == 0:
        assert abs(law - eq1) > 20 * se
    else:
        assert abs(law / eq1 - 1) < 1e-5
