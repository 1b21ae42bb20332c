"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds only input generation (grids, material constants, random states, grain
maps, temperature profiles, chain parameter draws); none of the Monte Carlo
arithmetic.  Material and workload sizes follow the thin-film and
granular-media settings of the paper's examples (nm cells, Tc of a few hundred
K, Ms0 ~ 1 MA/m).
"""
import numpy as np

MUB = 9.2740100783e-24

# Material of the small plain case: Ms0 = 1 MA/m, A = 10 pJ/m, Ku = 0.5 MJ/m^3
# along z, Tc = 700 K, J = 1/2 mean field with mu = mu_B.
BASE_MATERIAL = dict(Ms0=1.0e6, A0=1.0e-11, K1=5.0e5, K2=0.0, easy_axis=(0.0, 0.0, 1.0), Tc=700.0, mu=MUB, mf=1)

WORKLOADS = {
    # plain, no demag: 32x32x1 cells of 5 nm, 300 K, 0.1 T along z, fixed cone 30 deg, sigma 0.05
    "plain_32x32x1": dict(grid=(32, 32, 1), cell=(5e-9, 5e-9, 5e-9), T=300.0, B=(0.0, 0.0, 0.1), demag=False,
                          D0=0.0, cone_deg=30, adapt_every=0, sigma_fixed=0.05, sweeps=2000, init=0),
    # DMI thin film with demag: 256x256x1 cells of 4x4x2 nm, T = 0.5 Tc, zero field, random start
    "film_256x256x1": dict(grid=(256, 256, 1), cell=(4e-9, 4e-9, 2e-9), T=350.0, B=(0.0, 0.0, 0.0), demag=True,
                           D0=1.5e-3, cone_deg=30, adapt_every=100, sigma_fixed=0.0, sweeps=10000, init=1),
    # hysteresis workload: 1024x1024x4 cells of 5 nm, demag on, T = 0.9 Tc / 1.1 Tc, field along z
    "loop_1024x1024x4": dict(grid=(1024, 1024, 4), cell=(5e-9, 5e-9, 5e-9), T=630.0, B=(0.0, 0.0, 1.0), demag=True,
                             D0=0.0, cone_deg=30, adapt_every=100, sigma_fixed=0.0, sweeps=200, init=0),
    # granular: 512x512x8 cells of 3 nm, Voronoi grains of 10 nm mean spacing, T = 600 K
    "granular_512x512x8": dict(grid=(512, 512, 8), cell=(3e-9, 3e-9, 3e-9), T=600.0, B=(0.0, 0.0, 0.0), demag=True,
                               D0=0.0, cone_deg=30, adapt_every=100, sigma_fixed=0.0, sweeps=5000, init=1),
}

BATCH_SIZES = [(64, 64, 1), (128, 128, 1), (256, 256, 2), (512, 512, 2)]

# Granular Fe film with cubic anisotropy (the paper's Fig. 5 problem, Sec. III):
# Ms0 1.71 MA/m, A0 21 pJ/m, cubic K1 48 kJ/m^3 and K2 -10 kJ/m^3 with the
# me^{l(l+1)/2} law, Tc 1044 K, 300 K, 2 nm cells, 3-D Voronoi grains of 10 nm
# mean seed spacing that interact through the demag field only (exchange
# across grain boundaries 0), crystal axes along x, y, z in every grain, field
# along the in-plane cubic easy axis x.  800x800 nm in the plane as in the
# paper; 16 nm thick (8 cells) where the paper has 20 nm (10 cells), since
# the demag path here handles at most 8 layers; open boundaries.
FE_FILM = dict(grid=(400, 400, 8), cell=(2e-9, 2e-9, 2e-9), Ms0=1.71e6, A0=2.1e-11, K1c=4.8e4, K2c=-1.0e4,
               Tc=1044.0, T=300.0, B=(0.05, 0.0, 0.0), grain_spacing=10e-9, bscale=0.0,
               cubic_axes=((1.0, 0.0, 0.0), (0.0, 1.0, 0.0)), init_dir=(1.0, 0.0, 0.0))

# Switching events of a small Ni80Fe20 platelet (a scaled-down stand-in for the
# 400x200x5 nm ellipse of the parallel-vs-serial comparison): 80x40x5 nm in
# 5 nm cells, no crystal anisotropy (the demag interaction sets the easy axis
# along x), 300 K, started uniform along -x with a field of 0.14 T along +x,
# near its coercive field (median switching after ~1000 sweeps).
SWITCHING = dict(grid=(16, 8, 1), cell=(5e-9, 5e-9, 5e-9), Ms0=8.6e5, A0=1.3e-11, K1=0.0, Tc=870.0, T=300.0,
                 B=(0.14, 0.0, 0.0), init_dir=(-1.0, 0.0, 0.0), cone_deg=30, adapt_every=100, max_sweeps=2000)


def random_state(N, seed, lmin=0.5, lmax=1.0):
    """(3, N) float32: isotropic directions, lengths uniform in [lmin, lmax]."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(3, N))
    v /= np.linalg.norm(v, axis=0)
    L = rng.uniform(lmin, lmax, N)
    return (v * L).astype(np.float32)


def perturbed_uniform_state(N, seed, L=0.9, spread=0.3, axis=(0, 0, 1)):
    """(3, N) float32 near a uniform state (typical of an ordered magnet)."""
    rng = np.random.default_rng(seed)
    v = np.array(axis, dtype=np.float64)[:, None] + spread * rng.normal(size=(3, N))
    v /= np.linalg.norm(v, axis=0)
    return (v * L * rng.uniform(0.97, 1.03, N)).astype(np.float32)


def voronoi_grains(grid, cell, spacing, seed):
    """3-D Voronoi grains: Poisson seeds at density spacing^-3 in the box, each
    cell centre assigned to the nearest seed (ties to the lower index).
    Returns (grain id per cell, natural order; number of grains)."""
    nx, ny, nz = grid
    box = np.array(grid) * np.array(cell)
    rng = np.random.default_rng(seed)
    n = max(1, int(rng.poisson(np.prod(box) / spacing**3)))
    seeds = rng.uniform(0, 1, (n, 3)) * box
    xs = (np.arange(nx) + 0.5) * cell[0]
    ys = (np.arange(ny) + 0.5) * cell[1]
    zs = (np.arange(nz) + 0.5) * cell[2]
    from scipy.spatial import cKDTree
    tree = cKDTree(seeds)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    _, idx = tree.query(pts)
    return idx.astype(np.uint32), n


def grain_properties(n, seed, Ku=7e5, Tc_mean=700.0, Tc_sigma_frac=0.05, cone_deg=10.0):
    """Per-grain easy axis uniform on a cap of `cone_deg` about z, K1, Tc ~ N(mean, sigma)."""
    rng = np.random.default_rng(seed)
    ct = 1 - rng.uniform(0, 1, n) * (1 - np.cos(np.radians(cone_deg)))
    st = np.sqrt(1 - ct * ct)
    ph = 2 * np.pi * rng.uniform(0, 1, n)
    ea = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    Tc = rng.normal(Tc_mean, Tc_sigma_frac * Tc_mean, n)
    return ea, np.full(n, Ku), np.zeros(n), Tc


def batch_chain_params(n_chains, seed, Tc=700.0):
    """Chain draws of the batched workload: size from BATCH_SIZES, T ~ U[0.2,1.2] Tc, Hz ~ U[-0.5,0.5] T."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_chains):
        out.append(dict(grid=BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))], T=float(rng.uniform(0.2, 1.2) * Tc),
                        B=(0.0, 0.0, float(rng.uniform(-0.5, 0.5))), chain_id=i))
    return out


def gaussian_temperature_classes(grid, cell, width, T_centre, T_edge, levels=16):
    """Gaussian temperature profile across the film plane (centre T_centre,
    T_edge far out, full width `width` in metres between the 1/e points of the
    rise), binned into `levels` classes of equal temperature.  Returns (class
    id per cell in natural order, class temperatures); pass them as grains of
    the material's constants and as grain temperatures."""
    nx, ny, nz = grid
    xs = (np.arange(nx) + 0.5 - nx / 2) * cell[0]
    ys = (np.arange(ny) + 0.5 - ny / 2) * cell[1]
    r2 = xs[None, :] ** 2 + ys[:, None] ** 2
    T = T_edge + (T_centre - T_edge) * np.exp(-r2 / (width / 2) ** 2)
    lo, hi = min(T_edge, T_centre), max(T_edge, T_centre)
    k = np.clip(((T - lo) / max(hi - lo, 1e-300) * levels).astype(np.int64), 0, levels - 1)
    T_of = lo + (np.arange(levels) + 0.5) * (hi - lo) / levels
    cls = np.broadcast_to(k[None, :, :], (nz, ny, nx)).reshape(-1).astype(np.uint32)
    return cls, T_of
