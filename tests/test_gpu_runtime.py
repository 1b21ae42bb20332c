"""Runtime behaviour of the GPU library through the C-ABI: batches equal
chains run alone (bitwise), checkpoint/resume is bit-exact, runs are
deterministic, statistics bookkeeping and cone adaptation follow the rule,
and invalid input is rejected with the documented status."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MAT = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0)


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_05593_amd as p
    p.lib()
    return p


def _chains(pkg, specs):
    return [pkg.Chain(s["grid"], (5e-9,) * 3, T=s["T"], B=s["B"], demag=s.get("demag", True), seed=7,
                      chain_id=s["chain_id"], init=1, **MAT) for s in specs]


def test_batch_equals_sequential(pkg):
    specs = workloads.batch_chain_params(6, seed=0)
    for s in specs:                      # keep the test small: shrink the large grids
        s["grid"] = tuple(min(v, 96) for v in s["grid"][:2]) + (s["grid"][2],)
    specs[0]["demag"] = False
    a = _chains(pkg, specs)
    b = _chains(pkg, specs)
    batch = pkg.Batch(a)
    batch.sweep(7)
    batch.sweep(7)                        # replay of the captured graph
    batch.sync()
    for c in b:
        c.sweep(14)
    for ca, cb in zip(a, b):
        assert np.array_equal(ca.get_m(), cb.get_m())
        sa, sb = ca.stats(), cb.stats()
        assert sa["sweeps"] == sb["sweeps"] == 14
        assert sa["accepts_last"] == sb["accepts_last"] and sa["cone_deg"] == sb["cone_deg"]
    # changing a chain's field rebuilds the graph; results still match
    a[1].set_field((0, 0, 0.3))
    b[1].set_field((0, 0, 0.3))
    batch.sweep(3)
    batch.sync()
    b[1].sweep(3)
    assert np.array_equal(a[1].get_m(), b[1].get_m())
    batch.close()


def test_batch_shape_groups_equal_sequential(pkg):
    """Chains of one shape share launches (grains, grain temperatures, cubic
    anisotropy, DMI, adaptive cone, demag once per sweep); a temperature or anisotropy change
    in one of them regroups; results equal the chains run alone, bit for bit."""
    grid, cell = (40, 24, 2), (4e-9, 4e-9, 3e-9)
    N = int(np.prod(grid))
    gid, ng = workloads.voronoi_grains(grid, cell, seed=3, spacing=12e-9)
    ea, K1, K2, Tc = workloads.grain_properties(ng, seed=4)

    cub_axes = np.array([[1.0, 1.0, 0.0], [-1.0, 1.0, 0.3]])

    def make(i, grains, cub):
        c = pkg.Chain(grid, cell, T=300.0 + 40.0 * i, B=(0.0, 0.01 * i, 0.1 - 0.05 * i), D0=1e-3, demag=True,
                      refresh_per_sweep=1, seed=11 + i, chain_id=i, adapt_every=3, init=1, **MAT)
        if grains:
            c.set_grains(gid, ea, K1, K2, Tc, 0.1)
            if i == 2:                   # a temperature gradient across the grains of one chain
                c.set_grain_temperatures(np.linspace(250.0, 750.0, ng))
        if cub:
            c.set_anisotropy("cubic", cub_axes, 3e5, -5e4, me_scaling=True)
        return c
    # (grains, cubic anisotropy): cubic chains form groups of their own
    kinds = [(False, False), (False, True), (True, False), (False, False), (True, True), (False, True)]
    a = [make(i, *k) for i, k in enumerate(kinds)]
    b = [make(i, *k) for i, k in enumerate(kinds)]
    batch = pkg.Batch(a)
    batch.sweep(5)
    batch.sync()
    a[3].set_temperature(610.0)
    a[0].set_anisotropy("cubic", cub_axes, 2e5, 0.0)
    batch.sweep(4)
    batch.sync()
    for c in b:
        c.sweep(5)
    b[3].set_temperature(610.0)
    b[0].set_anisotropy("cubic", cub_axes, 2e5, 0.0)
    for c in b:
        c.sweep(4)
    for ca, cb in zip(a, b):
        assert np.array_equal(ca.get_m(), cb.get_m())
        assert ca.get_state() == cb.get_state()
        assert ca.stats()["m2_mean"] == cb.stats()["m2_mean"]
    batch.close()


def test_checkpoint_resume_bit_exact(pkg):
    grid = (40, 36, 2)
    kw = dict(T=500.0, B=(0.0, 0.05, 0.2), demag=True, D0=1e-3, seed=11, adapt_every=10, init=1, **MAT)
    a = pkg.Chain(grid, (4e-9, 4e-9, 2e-9), **kw)
    a.sweep(35)
    m_mid = a.get_m()
    state = a.get_state()
    a.sweep(35)
    b = pkg.Chain(grid, (4e-9, 4e-9, 2e-9), **kw)
    b.set_m(m_mid)
    b.set_state(*state)
    b.sweep(35)
    assert np.array_equal(a.get_m(), b.get_m())
    assert a.get_state() == b.get_state()


def test_deterministic_and_record(pkg):
    grid = (33, 17, 3)
    outs = []
    for _ in range(2):
        c = pkg.Chain(grid, (5e-9,) * 3, T=600.0, B=(0, 0, 0.1), demag=True, seed=3, init=1, adapt_every=5, **MAT)
        s = c.sweep_record(12)
        outs.append((c.get_m(), s, c.stats()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    m, s, st = outs[0]
    N = m.shape[1]
    m64 = m.astype(np.float64)
    assert np.allclose(s[-1, :3], m64.mean(axis=1), rtol=0, atol=1e-12)
    assert np.isclose(s[-1, 3], (m64**2).sum(axis=0).mean(), rtol=1e-12)
    assert st["sweeps"] == 12 and st["accepts_last"] == int(s[-1, 4])
    assert 0 < s[:, 4].max() <= N


def test_sweep_timed_sampling(pkg):
    """Instrumented sweeps run the same kernels (bitwise same state) and count
    the launches of the sampled sweeps only."""
    grid = (48, 40, 2)
    kw = dict(T=550.0, B=(0, 0, 0.2), demag=True, seed=5, init=1, adapt_every=4, **MAT)
    a = pkg.Chain(grid, (5e-9,) * 3, **kw)
    b = pkg.Chain(grid, (5e-9,) * 3, **kw)
    a.sweep(7)
    ms, cnt = b.sweep_timed(7, every=3)           # sweeps 0, 3, 6 instrumented
    assert np.array_equal(a.get_m(), b.get_m()) and a.get_state() == b.get_state()
    assert list(cnt) == [6, 6, 6, 6, 3]
    assert np.all(ms > 0)
    ms1, cnt1 = b.sweep_timed(2)
    assert list(cnt1) == [4, 4, 4, 4, 2]
    with pytest.raises(pkg.MMCError) as e:
        b.sweep_timed(2, every=0)
    assert e.value.status == -1


def test_cone_adaptation_on_device(pkg):
    from oracle import oracle as O
    # no coupling, tiny length moves, high T: acceptance ~ 1 -> +1 degree per window
    c = pkg.Chain((16, 16, 1), (5e-9,) * 3, Ms0=1e6, A0=0.0, K1=0.0, Tc=700.0, T=1400.0, sigma_fixed=1e-4,
                  adapt_every=20, cone_deg=30, demag=False)
    c.sweep(100)
    assert c.stats()["cone_deg"] == 35
    c = pkg.Chain((16, 16, 1), (5e-9,) * 3, T=50.0, sigma_fixed=1e-3, adapt_every=20, cone_deg=120, demag=False, **MAT)
    c.sweep(60)
    assert c.stats()["cone_deg"] == 117


def test_invalid_inputs(pkg):
    c = pkg.Chain((8, 8, 1), (5e-9,) * 3, T=300.0, **MAT)
    m = np.ones((3, 64), dtype=np.float32)
    m[:, 5] = 0.0
    with pytest.raises(pkg.MMCError) as e:
        c.set_m(m)
    assert e.value.status == -2
    m[:, 5] = np.nan
    with pytest.raises(pkg.MMCError):
        c.set_m(m)
    with pytest.raises(pkg.MMCError) as e:
        c.sweep(-1)
    assert e.value.status == -1
    with pytest.raises(pkg.MMCError) as e:
        c.set_temperature(0.0)
    assert e.value.status == -2
    with pytest.raises(pkg.MMCError) as e:
        c.demag_field()                 # demag off for this chain
    assert e.value.status == -5
    with pytest.raises(pkg.MMCError) as e:
        pkg.Chain((8, 8, 9), (5e-9,) * 3, T=300.0, demag=True, **MAT)
    assert e.value.status == -6
    with pytest.raises(pkg.MMCError) as e:
        pkg.Chain((8, 8, 1), (5e-9,) * 3, T=300.0, cone_deg=181, **MAT)
    assert e.value.status == -1


def test_single_cell_and_tiny_grids(pkg):
    from oracle import oracle as O
    for grid in [(1, 1, 1), (2, 1, 1), (1, 3, 1), (3, 3, 3)]:
        c = pkg.Chain(grid, (5e-9,) * 3, T=650.0, B=(0, 0, 0.2), demag=True, seed=1, init=1, **MAT)
        s = c.sweep_record(20)
        assert np.all(np.isfinite(s))
        N = int(np.prod(grid))
        m = c.get_m()
        h = c.demag_field().astype(np.float64)
        ref = O.DemagPlan(grid, (5e-9,) * 3)(m.astype(np.float64))
        assert np.abs(h - ref).max() < 1e-6 * max(1e-30, np.abs(ref).max())
