"""Parity at the full benchmark size (1024 x 1024 x 4 cells of 5 nm, demag on),
through the C-ABI, in the launch configuration the benchmark times, and at
the full size of its granular Fe film leg.

* demag field: sampled cells against the oracle's direct sum over all 4.2 M
  source cells (relative error per sampled vector <= 1e-5 of the field scale);
* one colour pass, whole grid: identical decisions except for moves within
  1e-5 of the acceptance cut-off (the oracle's log-acceptance margin).
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GRID, CELL = (1024, 1024, 4), (5e-9, 5e-9, 5e-9)
MAT = dict(Ms0=1e6, A0=1e-11, K1=5e5, Tc=700.0)
DECISION_TOL = 1e-5     # |k ln f - dF/kT - ln u3| of a move whose decisions may differ


@pytest.fixture(scope="module")
def chain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_05593_amd import Chain
    ch = Chain(GRID, CELL, T=630.0, B=(0, 0, 1.0), demag=True, seed=21, **MAT)
    yield ch
    ch.close()


def test_demag_sampled_cells(chain):
    from oracle import oracle as O
    N = int(np.prod(GRID))
    m = workloads.perturbed_uniform_state(N, seed=5, L=0.4, spread=0.5)
    chain.set_m(m)
    h = chain.demag_field()
    rng = np.random.default_rng(3)
    nx, ny, nz = GRID
    corners = [0, nx - 1, (ny - 1) * nx, N - 1]
    cells = np.concatenate([corners, rng.integers(0, N, 4)])
    print("sampled cells", cells.tolist(), flush=True)
    ref = O.demag_direct_at(GRID, CELL, m.astype(np.float64), cells)
    scale = np.abs(ref).max()
    err = np.abs(h[:, cells].T.astype(np.float64) - ref).max()
    print("max abs error %.3e of field scale %.3e" % (err, scale))
    assert err < 1e-5 * scale


def test_colour_pass_whole_grid(chain):
    from oracle import oracle as O
    N = int(np.prod(GRID))
    ref = O.System(GRID, CELL, T=630.0, B=(0, 0, 1.0), demag=True, seed=21, **MAT)
    c = ref.coeffs()
    m = workloads.perturbed_uniform_state(N, seed=9, L=c["me"], spread=0.3)
    # a smooth synthetic frozen field (input, not computed by either side)
    x = np.arange(N) % GRID[0]
    hz = (-0.3 + 0.1 * np.sin(2 * np.pi * x / GRID[0])).astype(np.float32)
    h = np.stack([0.05 * np.cos(2 * np.pi * x / 97.0), 0.02 * np.ones(N), hz]).astype(np.float32)
    for colour, sweep in ((0, 123456), (1, 7)):
        chain.set_m(m)
        chain.set_state(sweep, 17, 0)
        acc = chain.subsweep(colour, torch.from_numpy(h).cuda()).cpu().numpy().astype(np.int16)
        _, acc_o, margin, _, _ = ref.subsweep(m.astype(np.float64), sweep, colour, 17.0, h=h.astype(np.float64))
        mine = acc_o >= 0
        assert np.array_equal(acc == 255, ~mine)
        mism = mine & (acc != acc_o)
        worst = np.abs(margin[mism]).max() if mism.any() else 0.0
        print("colour %d: %d cells, %d accepted, %d mismatches, worst |margin| %.2e"
              % (colour, mine.sum(), (acc_o == 1).sum(), mism.sum(), worst))
        assert worst < DECISION_TOL


def test_fe_film_colour_pass_whole_grid():
    """The granular Fe film of the benchmark's second leg at its full size
    (400 x 400 x 8 cells of 2 nm, 10k Voronoi grains coupled by demag only,
    cubic anisotropy with the me^{l(l+1)/2} law), the colour-pass kernel it
    times: whole-grid decisions against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2106_05593_amd import Chain
    p = workloads.FE_FILM
    grid, cell = p["grid"], p["cell"]
    N = int(np.prod(grid))
    gid, ng = workloads.voronoi_grains(grid, cell, p["grain_spacing"], seed=7)
    kw = dict(Ms0=p["Ms0"], A0=p["A0"], Tc=p["Tc"], T=p["T"], B=p["B"], demag=True, seed=5)
    ch = Chain(grid, cell, K1=0.0, **kw)
    ea = np.tile([0.0, 0.0, 1.0], (ng, 1))
    ch.set_grains(gid, ea, np.zeros(ng), np.zeros(ng), np.full(ng, p["Tc"]), p["bscale"])
    ax = np.array(p["cubic_axes"])
    ch.set_anisotropy("cubic", ax, p["K1c"], p["K2c"], me_scaling=True)
    R = np.stack([ax[0], ax[1], np.cross(ax[0], ax[1])])
    ref = O.System(grid, cell, K1=0.0, cls=gid, ea=ea, K1s=np.full(ng, p["K1c"]), K2s=np.full(ng, p["K2c"]),
                   Tcs=np.full(ng, p["Tc"]), bscale=p["bscale"], cubic_axes=R, kscale=True, **kw)
    c = ref.coeffs()
    m = workloads.perturbed_uniform_state(N, seed=4, L=c["me"], spread=0.4, axis=(1.0, 0.0, 0.0))
    x = np.arange(N) % grid[0]
    h = np.stack([-0.2 + 0.05 * np.sin(2 * np.pi * x / grid[0]), 0.03 * np.cos(2 * np.pi * x / 53.0),
                  -0.1 * np.ones(N)]).astype(np.float32)
    for colour, sweep in ((0, 31), (1, 90001)):
        ch.set_m(m)
        ch.set_state(sweep, 25, 0)
        acc = ch.subsweep(colour, torch.from_numpy(h).cuda()).cpu().numpy().astype(np.int16)
        _, acc_o, margin, _, _ = ref.subsweep(m.astype(np.float64), sweep, colour, 25.0, h=h.astype(np.float64))
        mine = acc_o >= 0
        assert np.array_equal(acc == 255, ~mine)
        mism = mine & (acc != acc_o)
        worst = np.abs(margin[mism]).max() if mism.any() else 0.0
        print("colour %d: %d cells, %d accepted, %d mismatches, worst |margin| %.2e"
              % (colour, mine.sum(), (acc_o == 1).sum(), mism.sum(), worst))
        assert worst < DECISION_TOL
    ch.close()


@pytest.mark.parametrize("mode,tol", [("fp32", 1e-5), ("split_bf16", 1e-3), ("split_fp16", 1e-5)])
def test_demag_sampled_cells_granular_grid(mode, tol):
    """The granular workload's grid (512x512x8 cells of 3 nm) in each demag
    precision: sampled cells (corners and random) against the oracle's direct
    sum over all 2.1 M source cells, error per sampled vector within tol of the
    field scale (1e-5 FP32 and split FP16, 1e-3 split BF16)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_2106_05593_amd import Chain
    grid, cell = (512, 512, 8), (3e-9, 3e-9, 3e-9)
    N = int(np.prod(grid))
    ch = Chain(grid, cell, T=600.0, demag=mode, seed=2, **MAT)
    m = workloads.perturbed_uniform_state(N, seed=8, L=0.6, spread=0.6)
    ch.set_m(m)
    h = ch.demag_field()
    ch.close()
    rng = np.random.default_rng(4)
    nx, ny, nz = grid
    corners = [0, nx - 1, (ny - 1) * nx, N - 1]
    cells = np.concatenate([corners, rng.integers(0, N, 4)])
    print(mode, "sampled cells", cells.tolist(), flush=True)
    ref = O.demag_direct_at(grid, cell, m.astype(np.float64), cells)
    scale = np.abs(ref).max()
    err = np.abs(h[:, cells].T.astype(np.float64) - ref).max()
    print("%s: max abs error %.3e of field scale %.3e" % (mode, err, scale))
    assert err < tol * scale
