"""GPU parity against the FP64 oracle, through the C-ABI.

Bars (FP32 GPU vs FP64 oracle):
  * Philox streams and checkerboard indexing: exact (identical uniforms and
    identical sets of updated cells).
  * One colour pass from an identical state: identical accept/reject decisions
    except for moves within 1e-5 of the acceptance cut-off, i.e. where the
    oracle's log-acceptance margin k ln f - dF/kT - ln u3 is within
    DECISION_TOL = 1e-5 of 0 (FP32 rounding of the proposal and of dF), and
    accepted states within 2e-6 of |m|.
  * Demag field: relative L2 error <= 1e-5.
  * Energy: each term within 2e-6 of the total magnitude.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DECISION_TOL = 1e-5


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="module")
def mmc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2106_05593_amd as pkg
    pkg.lib()
    return pkg


def _pair(O, mmc, grid, cell, **kw):
    okw = dict(kw)
    for k in ("cone_deg", "adapt_every", "init", "init_dir", "refresh_per_sweep_gpu"):
        okw.pop(k, None)
    ch = mmc.Chain(grid, cell, **kw)
    ref = O.System(grid, cell, **{k: v for k, v in okw.items() if k not in ("lenmove",)},
                   lenmode=kw.get("lenmove", 0))
    return ch, ref


MAT = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0)


def _decision_check(O, ch, ref, m0, sweep, colour, cone, h=None):
    N = m0.shape[1]
    ch.set_m(m0)
    ch.set_state(sweep, cone, 0)
    ht = torch.from_numpy(h.astype(np.float32)).cuda() if h is not None else None
    acc = ch.subsweep(colour, ht).cpu().numpy().astype(np.int16)
    m_gpu = ch.get_m()
    h64 = h.astype(np.float32).astype(np.float64) if h is not None else None
    m_or, acc_o, margin, mB, _ = ref.subsweep(m0.astype(np.float64), sweep, colour, float(cone), h=h64)
    mine = acc_o >= 0
    assert np.array_equal(acc == 255, ~mine), "colour sets differ"
    mism = mine & (acc != acc_o)
    worst = np.abs(margin[mism]).max() if mism.any() else 0.0
    print("colour %d: %d cells, %d accepted, %d mismatches, worst |margin| %.2e"
          % (colour, mine.sum(), (acc_o == 1).sum(), mism.sum(), worst))
    assert worst < DECISION_TOL
    both_acc = mine & (acc == 1) & (acc_o == 1)
    both_rej = (acc == 0) & (acc_o == 0)
    scale = np.linalg.norm(m0, axis=0)
    err = np.abs(m_gpu - mB)[:, both_acc].max(axis=0) / scale[both_acc] if both_acc.any() else np.zeros(1)
    assert err.max() < 2e-6, err.max()
    assert np.array_equal(m_gpu[:, both_rej], m0[:, both_rej])
    assert np.array_equal(m_gpu[:, ~mine], m0[:, ~mine])
    return mism.sum(), mine.sum()


@pytest.mark.parametrize("lenmove", [0, 1])
def test_init_state_matches_oracle(O, mmc, lenmove):
    grid, cell = (13, 7, 3), (5e-9,) * 3
    for T in (300.0, 770.0):
        ch, ref = _pair(O, mmc, grid, cell, T=T, seed=77, chain_id=5, init=1, lenmove=lenmove, **MAT)
        m = ch.get_m().astype(np.float64)
        r = ref.init_state("random")
        assert np.abs(m - r).max() < 3e-6 * np.abs(r).max()


@pytest.mark.parametrize("case", ["plain", "dmi_tilted", "ragged_3d", "exact", "hot"])
def test_subsweep_decisions_no_demag(O, mmc, case):
    kw = dict(T=300.0, B=(0.0, 0.0, 0.1), seed=5, chain_id=3, sigma_fixed=0.05, **MAT)
    grid, cell = (32, 32, 1), (5e-9,) * 3
    if case == "dmi_tilted":
        grid, cell = (40, 24, 1), (4e-9, 4e-9, 2e-9)
        kw.update(D0=1.5e-3, K2=1e5, easy_axis=(0.2, -0.3, 0.9), B=(0.05, -0.02, 0.2), sigma_fixed=0.0, T=350.0)
    if case == "ragged_3d":
        grid = (17, 9, 5)
        kw.update(D0=-2e-3, T=520.0, sigma_fixed=0.0)
    if case == "exact":
        kw.update(lenmove=1, T=650.0, sigma_fixed=0.0)
    if case == "hot":
        kw.update(T=760.0, sigma_fixed=0.0)
    ch, ref = _pair(O, mmc, grid, cell, **kw)
    N = int(np.prod(grid))
    tot_mis = tot = 0
    for trial in range(4):
        c = ref.coeffs()
        L = c["m0"]
        m0 = workloads.perturbed_uniform_state(N, seed=10 + trial, L=L, spread=0.4)
        for colour in (0, 1):
            a, b = _decision_check(O, ch, ref, m0, sweep=1000 * trial + 7, colour=colour, cone=[30, 5, 90, 180][trial])
            tot_mis += a
            tot += b
    assert tot_mis <= max(2, 1e-3 * tot)


def test_subsweep_decisions_with_demag_field(O, mmc):
    grid, cell = (24, 20, 3), (4e-9, 4e-9, 2e-9)
    kw = dict(T=450.0, B=(0.0, 0.0, 0.0), seed=9, chain_id=1, demag=True, D0=1e-3, **MAT)
    ch, ref = _pair(O, mmc, grid, cell, **kw)
    N = int(np.prod(grid))
    m0 = workloads.perturbed_uniform_state(N, seed=3, L=ref.coeffs()["m0"], spread=0.5, axis=(1, 0, 0.3))
    h = ref.demag(m0.astype(np.float64))
    for colour in (0, 1):
        _decision_check(O, ch, ref, m0, sweep=42, colour=colour, cone=40, h=h)


@pytest.mark.parametrize("grid,cell", [((1, 1, 1), (5e-9,) * 3), ((7, 1, 1), (5e-9,) * 3), ((8, 8, 2), (5e-9,) * 3),
                                       ((13, 6, 3), (4e-9, 4e-9, 2e-9)), ((33, 17, 4), (3e-9, 5e-9, 2e-9)),
                                       ((64, 64, 8), (3e-9,) * 3), ((256, 256, 1), (4e-9, 4e-9, 2e-9)),
                                       ((48, 300, 2), (5e-9, 4e-9, 3e-9)), ((64, 520, 4), (5e-9,) * 3),
                                       ((40, 150, 8), (3e-9,) * 3), ((24, 200, 6), (4e-9, 3e-9, 2e-9)),
                                       ((16, 300, 8), (2e-9,) * 3), ((20, 270, 6), (3e-9, 3e-9, 2e-9)),
                                       # x transforms of length 512 (257 <= nx <= 512) and 1024 (nx > 512)
                                       ((400, 40, 2), (5e-9,) * 3), ((300, 24, 8), (3e-9,) * 3),
                                       ((512, 16, 4), (5e-9, 4e-9, 3e-9)), ((1024, 8, 4), (5e-9,) * 3),
                                       ((600, 12, 1), (4e-9, 4e-9, 2e-9)),
                                       # the batched workload's two-layer grids (y pass of 512 and 1024 points)
                                       ((256, 256, 2), (5e-9,) * 3), ((512, 512, 2), (5e-9,) * 3),
                                       # the staged y pass: more than 8 layers (the 10-layer film of the
                                       # paper's Fe example, up to the 32-layer maximum), and a padded y of
                                       # 4096 points whose 3 nz signals exceed the one-kernel pass's registers
                                       ((24, 40, 10), (2e-9,) * 3), ((300, 20, 9), (3e-9, 3e-9, 2e-9)),
                                       ((40, 30, 16), (3e-9, 3e-9, 2e-9)), ((16, 520, 12), (4e-9, 3e-9, 2e-9)),
                                       ((12, 20, 32), (2e-9,) * 3), ((8, 1100, 5), (5e-9,) * 3),
                                       ((5, 3, 11), (4e-9, 4e-9, 2e-9)),
                                       # the largest transforms: x length 2048 (nx > 1024) and a 4096-point
                                       # padded y (ny > 1024) on the one-kernel y pass
                                       ((1100, 6, 2), (5e-9,) * 3), ((2048, 3, 1), (4e-9, 4e-9, 2e-9)),
                                       ((16, 1100, 2), (5e-9,) * 3), ((6, 2048, 1), (3e-9,) * 3)])
def test_demag_field_matches_oracle(O, mmc, grid, cell):
    N = int(np.prod(grid))
    ch = mmc.Chain(grid, cell, T=300.0, demag=True, **MAT)
    m = workloads.random_state(N, seed=N)
    ch.set_m(m)
    h = ch.demag_field().astype(np.float64)
    ref = O.DemagPlan(grid, cell)(m.astype(np.float64))
    rel = np.linalg.norm(h - ref) / np.linalg.norm(ref)
    print(grid, "rel L2 %.2e" % rel)
    assert rel < 1e-5


@pytest.mark.parametrize("demag", [False, True])
def test_energy_matches_oracle(O, mmc, demag):
    grid, cell = (20, 18, 3), (4e-9, 4e-9, 2e-9)
    kw = dict(T=420.0, B=(0.01, 0.02, -0.1), D0=1.5e-3, K2=2e5, easy_axis=(0.1, 0.2, 1.0), demag=demag, **MAT)
    ch, ref = _pair(O, mmc, grid, cell, **kw)
    N = int(np.prod(grid))
    m = workloads.random_state(N, seed=2, lmin=0.3, lmax=0.9)
    ch.set_m(m)
    E, terms = ch.energy()
    Eo = ref.energy(m.astype(np.float64))
    scale = np.abs(Eo).sum()
    assert np.abs(terms - Eo).max() < 2e-6 * scale, (terms, Eo)
    assert abs(E - Eo.sum()) < 2e-6 * scale


@pytest.mark.parametrize("with_demag,nx", [(False, 30), (True, 30), (True, 40)])
def test_subsweep_decisions_temperature_profile(O, mmc, with_demag, nx):
    """Non-uniform temperature profile: grains at their own temperatures
    (below and above Tc), DMI, grain-boundary exchange scale, optional demag;
    rows of odd and of even slot counts."""
    grid, cell = (nx, 22, 2), (4e-9, 4e-9, 3e-9)
    N = int(np.prod(grid))
    gid, ng = workloads.voronoi_grains(grid, cell, 9e-9, 5)
    ea, K1, K2, Tc = workloads.grain_properties(ng, seed=6)
    Tg = np.linspace(350.0, 760.0, ng)             # a temperature gradient across the grains
    kw = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0, T=500.0, B=(0.0, 0.05, 0.2), D0=1.2e-3, seed=13, chain_id=2)
    ch = mmc.Chain(grid, cell, demag=with_demag, **kw)
    ch.set_grains(gid, ea, K1, K2, Tc, 0.3)
    ch.set_grain_temperatures(Tg)
    ref = O.System(grid, cell, demag=with_demag, cls=gid, ea=ea, K1s=K1, K2s=K2, Tcs=Tc, bscale=0.3, Tcl=Tg, **kw)
    c = ref.coeffs()
    for trial in range(3):
        m0 = workloads.random_state(N, seed=40 + trial, lmin=0.3, lmax=1.0)
        h = ref.demag(m0.astype(np.float32).astype(np.float64)) if with_demag else None
        for colour in (0, 1):
            _decision_check(O, ch, ref, m0, sweep=77 + trial, colour=colour, cone=[25, 90, 180][trial], h=h)
    # energy with the profile: the longitudinal and anisotropy terms at each grain's own kT
    m = workloads.random_state(N, seed=9, lmin=0.3, lmax=0.9)
    ch.set_m(m)
    E, terms = ch.energy()
    Eo = ref.energy(m.astype(np.float64))
    scale = np.abs(Eo).sum()
    assert np.abs(terms - Eo).max() < 2e-6 * scale, (terms, Eo)
    # NULL profile: back to the chain temperature
    ch.set_grain_temperatures(None)
    with pytest.raises(mmc.MMCError):
        ch.set_grain_temperatures(np.ones(ng + 1) * 300.0)


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 2] *= -1
    return q.T            # rows: orthonormal crystal axes


@pytest.mark.parametrize("case,nx", [("uniform", 34), ("grains_profile_demag", 34), ("uniform", 32),
                                     ("grains_profile_demag", 40), ("uniform_exact", 32)])
def test_subsweep_decisions_cubic(O, mmc, case, nx):
    """Cubic anisotropy (Eq. 12) with the me^{l(l+1)/2} law: one crystal for
    every cell (with DMI), or one per grain at per-grain temperatures with
    demag.  Constants are large (V K1/kT ~ 3, V K2/kT ~ 10), the exchange is
    weak and every length sits at its grain's m0, so the cubic term decides
    many moves (on the oracle, dropping it changes 20-90 of ~900 decisions
    per pass for the single crystal and 2-20 with grains and demag); rows of
    odd and of even slot counts."""
    grid, cell = (nx, 26, 2), (3e-9, 3e-9, 3e-9)
    N = int(np.prod(grid))
    kw = dict(Ms0=1.71e6, A0=2e-12, K1=0.0, Tc=1044.0, T=300.0, B=(0.05, 0.0, 0.02), seed=17, chain_id=3)
    demag = case.endswith("demag")
    if case.startswith("uniform"):
        kw["D0"] = 1.0e-3
        R = _rot(1)
        lm = 1 if case.endswith("exact") else 0        # length move: paper's or exact (log-uniform)
        ch = mmc.Chain(grid, cell, demag=False, lenmove=lm, **kw)
        ch.set_anisotropy("cubic", R[:2], 5e5, -2e6, me_scaling=True)
        ref = O.System(grid, cell, demag=False, cubic_axes=R, kscale=True, lenmode=lm, **dict(kw, K1=5e5, K2=-2e6))
        L = np.full(N, ref.coeffs()["m0"])
    else:
        gid, ng = workloads.voronoi_grains(grid, cell, 9e-9, 8)
        Rs = np.stack([_rot(100 + k) for k in range(ng)])
        rng = np.random.default_rng(9)
        Kc1 = rng.uniform(-4e5, 6e5, ng)
        Kc2 = rng.uniform(-2e6, 2e6, ng)
        Tc = rng.normal(1044.0, 30.0, ng)
        Tg = np.where(np.arange(ng) % 5 == 4, 1080.0, np.linspace(250.0, 650.0, ng))   # every 5th above Tc
        ea = np.tile([0.0, 0.0, 1.0], (ng, 1))
        ch = mmc.Chain(grid, cell, demag=True, **kw)
        ch.set_grains(gid, ea, np.zeros(ng), np.zeros(ng), Tc, 0.2)
        ch.set_grain_temperatures(Tg)
        ch.set_anisotropy("cubic", Rs[:, :2, :], Kc1, Kc2, me_scaling=True)
        ref = O.System(grid, cell, demag=True, cls=gid, ea=ea, K1s=Kc1, K2s=Kc2, Tcs=Tc, bscale=0.2, Tcl=Tg,
                       cubic_axes=Rs, kscale=True, **kw)
        L = np.array([ref.coeffs(k)["m0"] for k in range(ng)])[gid]
    for trial in range(3):
        m0 = (workloads.random_state(N, seed=60 + trial, lmin=1.0, lmax=1.0) * L[None, :]).astype(np.float32)
        h = ref.demag(m0.astype(np.float32).astype(np.float64)) if demag else None
        for colour in (0, 1):
            _decision_check(O, ch, ref, m0, sweep=91 + trial, colour=colour, cone=[20, 70, 180][trial], h=h)
    m = workloads.random_state(N, seed=19, lmin=0.3, lmax=0.9)
    ch.set_m(m)
    E, terms = ch.energy()
    Eo = ref.energy(m.astype(np.float64))
    scale = np.abs(Eo).sum()
    assert np.abs(terms - Eo).max() < 2e-6 * scale, (terms, Eo)
    assert abs(terms[2] - Eo[2]) < 1e-5 * abs(Eo[2]), (terms[2], Eo[2])   # the cubic term on its own
    # back to the uniaxial form (zero constants here): the anisotropy energy vanishes
    ch.set_anisotropy("uniaxial")
    assert abs(ch.energy()[1][2]) < 1e-30 + 1e-9 * scale


def test_set_anisotropy_errors(mmc):
    ch = mmc.Chain((8, 8, 1), (3e-9,) * 3, Ms0=1.71e6, A0=2.1e-11, K1=0.0, Tc=1044.0, T=300.0)
    ax = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    for bad in (dict(axes=np.array([[1.0, 0, 0], [2.0, 0, 0]]), K1=1e4, K2=0.0),      # parallel axes
                dict(axes=np.array([[0.0, 0, 0], [0.0, 1, 0]]), K1=1e4, K2=0.0),      # zero axis
                dict(axes=np.tile(ax, (2, 1, 1)), K1=1e4, K2=0.0)):                   # 2 sets, no grains
        with pytest.raises(mmc.MMCError):
            ch.set_anisotropy("cubic", **bad)
    with pytest.raises(mmc.MMCError):
        ch.set_anisotropy("cubic", ax, np.nan, 0.0)
    ch.set_anisotropy("cubic", ax, 1e4, 0.0)
    ch.set_anisotropy("uniaxial", me_scaling=True)


def test_uniaxial_temperature_law(O, mmc):
    """The me^{l(l+1)/2} law on the uniaxial form (K1 order 2: me^3, K2 order
    4: me^10): decisions and energy terms against the oracle."""
    grid, cell = (24, 20, 2), (4e-9, 4e-9, 3e-9)
    N = int(np.prod(grid))
    kw = dict(Ms0=1e6, A0=2e-12, K1=2e6, K2=8e5, Tc=700.0, T=560.0, B=(0.0, 0.02, 0.05), seed=29,
              easy_axis=(0.2, -0.3, 0.9))
    ch = mmc.Chain(grid, cell, **kw)
    ch.set_anisotropy("uniaxial", me_scaling=True)
    ref = O.System(grid, cell, kscale=True, **kw)
    m0 = (workloads.random_state(N, seed=70, lmin=1.0, lmax=1.0) * ref.coeffs()["m0"]).astype(np.float32)
    for colour in (0, 1):
        _decision_check(O, ch, ref, m0, sweep=5, colour=colour, cone=60)
    ch.set_m(m0)
    terms = ch.energy()[1]
    Eo = ref.energy(m0.astype(np.float64))
    assert abs(terms[2] - Eo[2]) < 1e-5 * abs(Eo[2]), (terms[2], Eo[2])
    unscaled = O.System(grid, cell, **kw).energy(m0.astype(np.float64))[2]
    assert abs(Eo[2]) < 0.5 * abs(unscaled)         # me < 1: the law lowers the anisotropy


# Split-precision y-direction DFT stages (matrix cores, hi + lo products in FP32):
# every shape class the split path supports (padded y lengths 256 .. 2048, two
# and one radix-16 stages each way, even layer counts 2 .. 8)
SPLIT_GRIDS = [((64, 200, 2), (5e-9,) * 3), ((48, 300, 2), (5e-9, 4e-9, 3e-9)), ((64, 520, 4), (5e-9,) * 3),
               ((40, 100, 8), (3e-9,) * 3), ((16, 300, 8), (2e-9,) * 3), ((24, 400, 6), (4e-9, 3e-9, 2e-9)),
               ((256, 256, 2), (5e-9,) * 3), ((300, 270, 4), (3e-9,) * 3)]
# relative L2 error bars against the FP64 oracle: 1e-3 for split BF16 (16
# significant bits per operand); split FP16 keeps 22 bits per operand and
# is held to the FP32 bar
SPLIT_TOL = {"split_bf16": 1e-3, "split_fp16": 1e-5}


@pytest.mark.parametrize("mode", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("grid,cell", SPLIT_GRIDS)
def test_demag_field_split_matches_oracle(O, mmc, grid, cell, mode):
    N = int(np.prod(grid))
    ch = mmc.Chain(grid, cell, T=300.0, demag=mode, **MAT)
    m = workloads.random_state(N, seed=N + 1)
    ch.set_m(m)
    h = ch.demag_field().astype(np.float64)
    ref = O.DemagPlan(grid, cell)(m.astype(np.float64))
    rel = np.linalg.norm(h - ref) / np.linalg.norm(ref)
    # also a nearly uniform state: large low-frequency bins, small others
    mu = workloads.perturbed_uniform_state(N, seed=4, L=0.9, spread=0.05)
    ch.set_m(mu)
    hu = ch.demag_field().astype(np.float64)
    refu = O.DemagPlan(grid, cell)(mu.astype(np.float64))
    relu = np.linalg.norm(hu - refu) / np.linalg.norm(refu)
    print(grid, mode, "rel L2 %.2e (random), %.2e (near uniform)" % (rel, relu))
    assert rel < SPLIT_TOL[mode] and relu < SPLIT_TOL[mode]
    ch.close()


def test_demag_split_rejects_unsupported_shapes(mmc):
    # odd layer count, padded y too short, and nz 8 with a 512-point y transform
    for grid in [(64, 300, 3), (64, 100, 2), (40, 200, 8)]:
        with pytest.raises(mmc.MMCError) as ei:
            mmc.Chain(grid, (5e-9,) * 3, T=300.0, demag="split_bf16", **MAT)
        assert ei.value.status == mmc.MMC_ERR_UNSUPPORTED
