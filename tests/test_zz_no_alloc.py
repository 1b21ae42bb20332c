"""The allocation-free energy entry point (mmc_energy_noalloc) against
mmc_energy through the C-ABI: two calls in a row, the second on a smaller
grid, each equal to mmc_energy's terms and total for the same state."""
import numpy as np
import pytest

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


def _check_against_energy(ch, out):
    out.fill_(np.nan)
    ch.energy_noalloc(out)
    ch.sync()
    got = out.cpu().numpy()
    tot, terms = ch.energy()
    print("terms", terms, "total", tot, flush=True)
    assert np.all(np.isfinite(got))
    # same kernel, same partial sums, same FP64 summation order: equal doubles
    assert np.array_equal(got[:6], terms), (got[:6], terms)
    assert got[6] == tot, (got[6], tot)


def test_energy_noalloc_matches_energy(pkg):
    torch.cuda.set_device(0)
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    # first call: 512x512x4 cells with demag, more cells than 2048 blocks of
    # 256 threads cover (the energy kernel strides), after two sweeps
    print("call 1: 512x512x4, demag on", flush=True)
    big = pkg.Chain((512, 512, 4), (5e-9,) * 3, T=630.0, B=(0, 0, 0.2), demag=True, seed=5, init=1, **MAT)
    big.sweep(2)
    _check_against_energy(big, out)
    big.close()
    # second call, smaller input: 40x36x2 with DMI and demag; the scratch still
    # holds the first call's partials past this call's block count
    print("call 2: 40x36x2, DMI and demag on", flush=True)
    small = pkg.Chain((40, 36, 2), (4e-9, 4e-9, 2e-9), T=350.0, D0=1.5e-3, demag=True, seed=9, init=1, **MAT)
    small.sweep(3)
    _check_against_energy(small, out)
    # and without demag, on the same output buffer
    print("call 3: 40x36x2 without demag", flush=True)
    nod = pkg.Chain((40, 36, 2), (4e-9, 4e-9, 2e-9), T=350.0, D0=1.5e-3, demag=False, seed=9, init=1, **MAT)
    _check_against_energy(nod, out)
    small.close()
    nod.close()


def test_energy_noalloc_rejects_bad_arguments(pkg):
    from paper_2106_05593_amd import mmc
    ch = pkg.Chain((8, 8, 1), (5e-9,) * 3, T=300.0, seed=1, **MAT)
    assert mmc.lib().mmc_energy_noalloc(ch._h, None) == mmc.MMC_ERR_ARG
    assert mmc.lib().mmc_energy_noalloc(None, None) == mmc.MMC_ERR_ARG
    ch.close()
