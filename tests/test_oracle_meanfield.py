"""Pins of the oracle's mean-field and longitudinal coefficients (paper Sec. II,
Eqs. 7-9 and 13).

The paper gives the Langevin (classical) forms; the J=1/2 Brillouin form
(m = tanh(m Tc/T)) is the same construction with B_1/2 = tanh.  The pins use
closed-form limits and an independent numerical derivative of the mean-field
solution, not the oracle's own formulas.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

KB = 1.380649e-23
MUB = 9.2740100783e-24


def _solve_m(model, T, Tc, B, mu=MUB, lo=1e-12, hi=1.0):
    """Mean-field m at applied field B (tesla) solved from scratch with brentq
    on the bracket [lo, hi] (which selects the branch)."""
    if model == 1:
        g = lambda m: np.tanh((Tc * m + mu * B / KB) / T) - m
    else:
        def L(x):   # Langevin function; two-term series where coth(x) - 1/x cancels
            return 1.0 / np.tanh(x) - 1.0 / x if abs(x) > 1e-3 else x / 3.0 - x**3 / 45.0
        g = lambda m: L((3 * Tc * m + mu * B / KB) / T) - m
    if g(hi) == 0.0:      # deep below Tc the root rounds to 1
        return hi
    return brentq(g, lo, hi, xtol=1e-16, rtol=1e-15, maxiter=500)


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("t", [0.05, 0.3, 0.6, 0.9, 0.97])
def test_me_fixed_point(oracle_mod, model, t):
    Tc = 700.0
    me, _ = oracle_mod.meanfield(model, t * Tc, Tc)
    assert abs(me - _solve_m(model, t * Tc, Tc, 0.0)) < 1e-12


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("t", [0.3, 0.6, 0.9, 1.05, 1.3])
def test_chi_is_field_derivative(oracle_mod, model, t):
    """chi_par = dm/dB at B = 0 (the meaning of Eq. 8), by central difference."""
    Tc = 700.0
    T = t * Tc
    _, inv_chi = oracle_mod.meanfield(model, T, Tc)
    dB = 1e-4
    if t < 1:
        me = _solve_m(model, T, Tc, 0.0)
        lo, hi = 0.5 * me, 1.0           # the +me branch
    else:
        lo, hi = -0.5, 0.5                       # m(B) odd, m(0) = 0
    # Richardson-extrapolated central difference
    d1 = (_solve_m(model, T, Tc, dB, lo=lo, hi=hi) - _solve_m(model, T, Tc, -dB, lo=lo, hi=hi)) / (2 * dB)
    d2 = (_solve_m(model, T, Tc, 2 * dB, lo=lo, hi=hi) - _solve_m(model, T, Tc, -2 * dB, lo=lo, hi=hi)) / (4 * dB)
    d = (4 * d1 - d2) / 3
    assert abs(d * inv_chi - 1.0) < 1e-6


def test_limits(oracle_mod):
    Tc = 700.0
    # me -> 1 as T -> 0
    assert oracle_mod.meanfield(1, 1.0, Tc)[0] > 1 - 1e-12
    # near Tc: me^2 -> 3(1 - T/Tc) (J=1/2), 5/3 (1 - T/Tc) (Langevin)
    eps = 1e-5
    for model, c in [(1, 3.0), (0, 5.0 / 3.0)]:
        me, _ = oracle_mod.meanfield(model, (1 - eps) * Tc, Tc)
        assert abs(me * me / (c * eps) - 1) < 1e-3
    # above Tc: chi = mu / (k (T-Tc)) (J=1/2), mu / (3k (T-Tc)) (Langevin)
    for model, c in [(1, 1.0), (0, 3.0)]:
        me, inv_chi = oracle_mod.meanfield(model, 800.0, Tc)
        assert me == 0.0
        assert abs(inv_chi / (c * KB * 100.0 / MUB) - 1) < 1e-14


def _sys(oracle_mod, T, mf=1, h=5e-9, **kw):
    return oracle_mod.System((4, 4, 1), (h,) * 3, Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0, T=T, mf=mf, **kw)


@pytest.mark.parametrize("mf", [0, 1])
def test_quartic_coefficient_continuous_at_tc(oracle_mod, mf):
    """Eq. 7: the m^4 coefficient of F_l/kT is continuous across Tc (below:
    la*m^4; above: lbc*m^4) when the above-Tc constant matches the model
    (3/10 Langevin as printed, 1/6 for J=1/2)."""
    below = _sys(oracle_mod, 700.0 * (1 - 1e-7), mf=mf).coeffs()
    above = _sys(oracle_mod, 700.0 * (1 + 1e-7), mf=mf).coeffs()
    assert below["below"] == 1 and above["below"] == 0
    assert abs(below["la"] / above["lbc"] - 1) < 1e-5
    assert above["lb"] < 1e-6 * above["lbc"]


def test_sigma_is_width_of_m2_gaussian(oracle_mod):
    """Eq. 13: f_l/m^2 is a Gaussian in m^2 of mean me^2 and std sigma (uncapped)."""
    c = _sys(oracle_mod, 300.0).coeffs()
    assert c["sigma"] < 0.03
    assert abs(c["sigma"] - 1.0 / np.sqrt(2 * c["la"])) < 1e-12 * c["sigma"]
    hot = _sys(oracle_mod, 699.0, h=2e-9).coeffs()   # small cell: width above the cap
    assert 1.0 / np.sqrt(2 * hot["la"]) > 0.03
    assert hot["sigma"] == 0.03
    assert _sys(oracle_mod, 800.0).coeffs()["sigma"] == 0.03
    assert _sys(oracle_mod, 300.0, sigma_fixed=0.05).coeffs()["sigma"] == 0.05


def test_initial_length_above_tc(oracle_mod):
    """Above Tc the initial length is sqrt(<m^2>) of f_l (me = 0 is absorbing)."""
    c = _sys(oracle_mod, 770.0).coeffs()
    m = np.linspace(0, 1, 400001)
    w = m**2 * np.exp(-(c["lb"] * m**2 + c["lbc"] * m**4))
    m2 = np.trapezoid(w * m**2, m) / np.trapezoid(w, m)
    assert abs(c["m0"] ** 2 / m2 - 1) < 1e-8
