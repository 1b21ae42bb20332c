"""Equilibrium statistics: the FP32 GPU chain and the FP64 oracle chain
(independent seeds) agree on <m_z>, <|m|^2> within 3 combined standard errors
(batch means after 20 % burn-in)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAT = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0)


def batch_mean_se(x, nb=20):
    x = x[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
    return x.mean(), x.std(ddof=1) / np.sqrt(nb)


def _compare(gpu_series, ora_series, burn):
    for col, name in ((2, "<mz>"), (3, "<|m|^2>")):
        g, sg = batch_mean_se(gpu_series[burn:, col])
        o, so = batch_mean_se(ora_series[burn:, col])
        z = (g - o) / np.hypot(sg, so)
        print("%s gpu %.6f +- %.2e  oracle %.6f +- %.2e  z = %.2f" % (name, g, sg, o, so, z))
        assert abs(z) < 3.0


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_05593_amd as p
    p.lib()
    return p


def test_plain_small_workload(pkg):
    """32x32x1 cells of 5 nm, 300 K, 0.1 T, fixed 30 deg cone, sigma 0.05, 2000 sweeps."""
    from oracle import oracle as O
    kw = dict(T=300.0, B=(0, 0, 0.1), sigma_fixed=0.05, **MAT)
    n = 2000
    g = pkg.Chain((32, 32, 1), (5e-9,) * 3, seed=101, adapt_every=0, cone_deg=30, **kw)
    gs = g.sweep_record(n)
    o = O.System((32, 32, 1), (5e-9,) * 3, seed=202, **kw)
    m = o.init_state("uniform")
    os_, _, _ = o.run(m, n, cone_deg=30, adapt_every=0)
    _compare(gs, os_, n // 5)


@pytest.mark.parametrize("lenmove", [0, 1])
def test_dmi_film_with_demag(pkg, lenmove):
    """64x64x1 cells of 4x4x2 nm with DMI and demag, 0.5 Tc, 0.5 T along z."""
    from oracle import oracle as O
    kw = dict(T=350.0, B=(0, 0, 0.5), D0=1.5e-3, demag=True, **MAT)
    n = 1500
    g = pkg.Chain((64, 64, 1), (4e-9, 4e-9, 2e-9), seed=303, adapt_every=100, lenmove=lenmove, **kw)
    gs = g.sweep_record(n)
    o = O.System((64, 64, 1), (4e-9, 4e-9, 2e-9), seed=404, lenmode=lenmove, **kw)
    m = o.init_state("uniform")
    os_, _, _ = o.run(m, n, cone_deg=30, adapt_every=100)
    _compare(gs, os_, n // 5)


def test_dmi_film_full_size(pkg):
    """The DMI film at its full size: 256x256x1 cells of 4x4x2 nm, D0 = 1.5
    mJ/m^2, demag, 0.5 Tc, zero field, random directions at |m| = me.  From a
    random start at zero field the textures keep coarsening, so <m_z> drifts
    and has no stationary error; the local quantity <|m|^2> equilibrates
    within the burn-in and is compared within 3 combined standard errors over
    sweeps 150-600 (independent seeds), and both chains keep <m_z> near zero."""
    from oracle import oracle as O
    kw = dict(T=350.0, B=(0, 0, 0), D0=1.5e-3, demag=True, **MAT)
    grid, cell = (256, 256, 1), (4e-9, 4e-9, 2e-9)
    n, burn = 600, 150
    g = pkg.Chain(grid, cell, seed=707, adapt_every=100, init=1, **kw)
    gs = g.sweep_record(n)
    o = O.System(grid, cell, seed=808, **kw)
    m = o.init_state("random")
    os_, _, _ = o.run(m, n, cone_deg=30, adapt_every=100)
    a, sa = batch_mean_se(gs[burn:, 3], nb=15)
    b, sb = batch_mean_se(os_[burn:, 3], nb=15)
    z = (a - b) / np.hypot(sa, sb)
    print("<|m|^2> gpu %.6f +- %.2e  oracle %.6f +- %.2e  z = %.2f" % (a, sa, b, sb, z))
    assert abs(z) < 3.0
    assert abs(gs[burn:, 2].mean()) < 0.05 and abs(os_[burn:, 2].mean()) < 0.05


def test_above_tc_granular(pkg):
    """Grains with scattered Tc around T, weak exchange across boundaries."""
    import workloads
    from oracle import oracle as O
    grid, cell = (24, 24, 4), (3e-9,) * 3
    cls, ng = workloads.voronoi_grains(grid, cell, 10e-9, seed=5)
    ea, K1, K2, Tc = workloads.grain_properties(ng, seed=6)
    n = 1500
    g = pkg.Chain(grid, cell, T=690.0, B=(0, 0, 0.3), demag=True, seed=505, adapt_every=100, **MAT)
    g.set_grains(cls, ea, K1, K2, Tc, 0.1)
    gs = g.sweep_record(n)
    o = O.System(grid, cell, T=690.0, B=(0, 0, 0.3), demag=True, seed=606, Ms0=MAT["Ms0"], A0=MAT["A0"],
                 K1=0.0, Tc=700.0, cls=cls, ea=ea, K1s=K1, K2s=K2, Tcs=Tc, bscale=0.1)
    m = o.init_state("uniform")
    os_, _, _ = o.run(m, n, cone_deg=30, adapt_every=100)
    _compare(gs, os_, n // 5)


def test_switching_statistics_gpu_vs_serial_oracle(pkg):
    """The paper's parallel-vs-serial switching check with the GPU chain as the
    parallel algorithm (demag refreshed once per sweep): its switching-time
    distribution on the platelet near its coercive field matches that of the
    oracle's serial MMC (demag field updated after every accepted move);
    96 events each, two-sample Kolmogorov-Smirnov test."""
    from scipy.stats import ks_2samp
    import workloads
    from oracle import switching
    p = workloads.SWITCHING
    d = np.asarray(p["B"]) / np.linalg.norm(p["B"])
    times = []
    for i in range(96):
        c = pkg.Chain(p["grid"], p["cell"], Ms0=p["Ms0"], A0=p["A0"], K1=p["K1"], Tc=p["Tc"], T=p["T"], B=p["B"],
                      demag=True, refresh_per_sweep=1, seed=3000 + i, cone_deg=p["cone_deg"],
                      adapt_every=p["adapt_every"], init=0, init_dir=p["init_dir"])
        t = p["max_sweeps"]
        for sw0 in range(0, p["max_sweeps"], 100):
            k = np.nonzero(c.sweep_record(100)[:, :3] @ d > 0)[0]
            if len(k):
                t = sw0 + int(k[0])
                break
        times.append(t)
    gpu = np.array(times)
    ser = switching.switch_times(p, np.arange(96) + 6000, "serial")
    print("gpu parallel mean %.0f median %.0f; oracle serial mean %.0f median %.0f"
          % (gpu.mean(), np.median(gpu), ser.mean(), np.median(ser)))
    assert np.median(gpu) < 0.8 * p["max_sweeps"]
    assert ks_2samp(gpu, ser).pvalue > 1e-3


@pytest.mark.parametrize("ka1,ka2", [(4.0, -0.8), (0.0, 60.0)])
def test_macrospin_cubic_gpu(pkg, ka1, ka2):
    """Independent cells (no exchange, no demag) with cubic anisotropy in the
    exact length mode sample exp(-F_cubic/kT) over directions: the GPU chain's
    <a^4 + b^4 + g^4> and <a^2 b^2 g^2> along the crystal axes against 2-D
    quadrature over the sphere (the oracle's pin, now on the GPU path)."""
    from test_oracle_cubic import _rot, _sphere_quadrature
    T, h = 300.0, 5e-9
    V, kT = h ** 3, 1.380649e-23 * T
    R = _rot(5)
    c = pkg.Chain((64, 64, 1), (h,) * 3, Ms0=1.71e6, A0=0.0, K1=0.0, Tc=1044.0, T=T, lenmove=1, seed=41, init=1,
                  adapt_every=100, cone_deg=30)
    c.set_anisotropy("cubic", R[:2], ka1 * kT / V, ka2 * kT / V)
    c.sweep(600)
    s4, s6 = [], []
    for _ in range(80):
        c.sweep(10)
        m = c.get_m().astype(np.float64)
        n = R @ (m / np.linalg.norm(m, axis=0))
        s4.append((n ** 4).sum(axis=0).mean())
        s6.append((n[0] ** 2 * n[1] ** 2 * n[2] ** 2).mean())
    q4, q6 = _sphere_quadrature(ka1, ka2)
    v4, e4 = batch_mean_se(np.array(s4), nb=10)
    v6, e6 = batch_mean_se(np.array(s6), nb=10)
    print("gpu <sum a^4> %.5f +- %.1e (quadrature %.5f); <a2b2g2> %.6f +- %.1e (%.6f)" % (v4, e4, q4, v6, e6, q6))
    assert abs(v4 - q4) < 4 * e4 + 1e-3
    assert abs(v6 - q6) < 4 * e6 + 2e-4


def test_macrospins_at_their_own_temperatures_gpu(pkg):
    """Temperature profile on the GPU path: independent cells of two classes
    held at 0.6 Tc and 1.05 Tc (exact length mode) each sample Eq. 1 at their
    own temperature: <m_z> and <|m|^2> per class against the single-temperature
    quadrature that pins the oracle."""
    from oracle import oracle as O
    from test_oracle_sampler import quadrature
    Tc, Bz, K1 = 700.0, 0.1, 5e4
    temps = np.array([0.6 * Tc, 1.05 * Tc])
    N = 64 * 64
    cls = (np.arange(N) % 2).astype(np.uint32)
    c = pkg.Chain((64, 64, 1), (5e-9,) * 3, Ms0=1e6, A0=0.0, K1=K1, Tc=Tc, T=temps[0], B=(0, 0, Bz), lenmove=1,
                  sigma_fixed=0.25, seed=23, init=0)
    c.set_grains(cls, np.tile([0.0, 0.0, 1.0], (2, 1)), np.full(2, K1), np.zeros(2), np.full(2, Tc), 1.0)
    c.set_grain_temperatures(temps)
    # sigma = 0.25 keeps the cone small below Tc, so directions relax slowly: long burn-in, spaced snapshots
    c.sweep(5000)
    snaps = []
    for _ in range(80):
        c.sweep(50)
        snaps.append(c.get_m().astype(np.float64))
    snaps = np.array(snaps)
    for k, T in enumerate(temps):
        ref = O.System((4, 4, 1), (5e-9,) * 3, Ms0=1e6, A0=0.0, K1=K1, Tc=Tc, T=T, B=(0, 0, Bz))
        mz_q, m2_q = quadrature(ref, K1, Bz)
        sel = snaps[:, :, cls == k]
        mz, se_mz = batch_mean_se(sel[:, 2, :].mean(axis=1), nb=10)
        m2, se_m2 = batch_mean_se((sel ** 2).sum(axis=1).mean(axis=1), nb=10)
        print("T %.0f: <mz> %.5f +- %.1e (quadrature %.5f); <m2> %.5f +- %.1e (%.5f)" % (T, mz, se_mz, mz_q, m2, se_m2, m2_q))
        assert abs(mz - mz_q) < 4 * se_mz + 2e-3
        assert abs(m2 - m2_q) < 4 * se_m2 + 2e-3
