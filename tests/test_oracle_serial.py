"""Pins of the oracle's serial MMC with the exact demag interaction (paper
Sec. III, the comparison of the parallel algorithm with a serial one in which
the demag field is updated after every accepted move; App. B).

* With demag off the serial sweep (colour 0 cells in index order, then colour
  1 cells, same Philox numbers) equals the parallel sweep bit for bit.
* The field it keeps current equals a fresh demag field of the final state
  (direct sum and FFT convolution).
* With the self term the accepted dF add up to the change of the total free
  energy (the demag part of each dF is then the exact energy change); Eq. 14
  with the current field alone misses that term.
"""
import numpy as np


def _system(oracle_mod, demag, **kw):
    grid, cell = (9, 7, 2), (4e-9, 4e-9, 3e-9)
    base = dict(Ms0=8e5, A0=1.3e-11, D0=1.2e-3, K1=2e5, K2=3e4, Tc=700.0, T=450.0, B=(0.02, -0.03, 0.1),
                easy_axis=(0.2, 0.1, 0.97), demag=demag, seed=3, chain_id=1)
    base.update(kw)
    return oracle_mod.System(grid, cell, **base)


def test_serial_equals_parallel_without_demag(oracle_mod):
    a = _system(oracle_mod, False)
    b = _system(oracle_mod, False)
    ma = a.init_state("random")
    mb = ma.copy()
    sa, ca, wa = a.run(ma, 30, cone_deg=40, adapt_every=7)
    sb, cb, wb, _, _ = b.serial_run(mb, 30, cone_deg=40, adapt_every=7)
    assert np.array_equal(ma, mb)
    assert np.array_equal(sa[:, 4], sb[:, 4]) and (ca, wa) == (cb, wb)
    assert np.allclose(sa[:, :4], sb[:, :4], rtol=1e-13, atol=1e-15)


def test_kept_field_is_the_fresh_field(oracle_mod):
    S = _system(oracle_mod, True)
    m = S.init_state("random")
    _, _, _, h, _ = S.serial_run(m, 6, cone_deg=60)
    scale = np.abs(h).max()
    assert np.abs(h - S.serial_field(m)).max() < 1e-12 * scale
    assert np.abs(h - oracle_mod.demag_direct(S.grid, S.cell, m)).max() < 1e-11 * scale
    assert np.abs(h - S.demag(m)).max() < 1e-9 * scale


def test_accepted_dF_add_up_to_the_energy_change(oracle_mod):
    for kw in (dict(), dict(T=760.0, lenmode=1)):
        S = _system(oracle_mod, True, **kw)
        m = S.init_state("random")
        E0 = S.energy(m).sum()
        m2 = m.copy()
        _, _, _, _, dE = S.serial_run(m, 5, cone_deg=50, self_term=True)
        E1 = S.energy(m).sum()
        assert abs((E1 - E0) - dE) < 1e-9 * abs(E1 - E0), (E1 - E0, dE)
        # without the self term (Eq. 14 with the current field) the sum misses it
        _, _, _, _, dE2 = S.serial_run(m2, 5, cone_deg=50)
        E2 = S.energy(m2).sum()
        assert abs((E2 - E0) - dE2) > 1e-6 * abs(E2 - E0)


def test_switching_statistics_parallel_vs_serial():
    """The paper's check of the frozen-field approximation by switching
    statistics: a platelet near its coercive field switches after the same
    distribution of sweep counts with the parallel algorithm (demag refreshed
    once per sweep) and with the serial one (field updated after every
    accepted move); 96 events each, two-sample Kolmogorov-Smirnov test."""
    from scipy.stats import ks_2samp
    import workloads
    from oracle import switching
    p = workloads.SWITCHING
    seeds = np.arange(96) + 1000
    par = switching.switch_times(p, seeds, "parallel1")
    ser = switching.switch_times(p, seeds + 5000, "serial")
    print("parallel mean %.0f median %.0f; serial mean %.0f median %.0f"
          % (par.mean(), np.median(par), ser.mean(), np.median(ser)))
    assert np.median(par) < 0.8 * p["max_sweeps"] and np.median(ser) < 0.8 * p["max_sweeps"]
    assert ks_2samp(par, ser).pvalue > 1e-3
