"""Pins of the oracle's demag tensor and convolution (paper Sec. III, Eq. 14).

The tensor is the cell-averaged (Newell) tensor; the oracle evaluates the
closed form near and a multipole expansion of the cell average far.  Pins:
  * exact values: cube self term 1/3, trace of the self term = 1;
  * Aharoni's independent closed form for the demag factors of a rectangular
    prism (J. Appl. Phys. 83, 3432 (1998)): the self term of one cell, and the
    box-averaged field of a uniformly magnetized block of cells (the cell-
    averaged tensor sums exactly to the block's factor);
  * the point-dipole limit far away;
  * agreement of the two independent forms (closed form / expansion) where both
    are accurate;
  * derivatives of 1/r against mpmath numerical differentiation;
  * FFT convolution == brute-force direct sum.
"""
import itertools

import numpy as np
import pytest


def aharoni_dz(a, b, c):
    """Aharoni's D_z of a prism with sides 2a x 2b x 2c (along x, y, z)."""
    r = np.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((rab + a) / (rab - a))
         + a / (2 * c) * np.log((rab + b) / (rab - b))
         + c / (2 * a) * np.log((rbc - b) / (rbc + b))
         + c / (2 * b) * np.log((rac - a) / (rac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a**3 + b**3 - 2 * c**3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) * r / (3 * a * b * c)
         + c / (a * b) * (rac + rbc)
         - (rab**3 + rbc**3 + rac**3) / (3 * a * b * c))
    return t / np.pi


def aharoni(Lx, Ly, Lz):
    a, b, c = Lx / 2, Ly / 2, Lz / 2
    return np.array([aharoni_dz(b, c, a), aharoni_dz(c, a, b), aharoni_dz(a, b, c)])


def test_aharoni_formula_self_consistent():
    assert abs(aharoni(1, 1, 1)[2] - 1 / 3) < 1e-14
    rng = np.random.default_rng(1)
    for _ in range(20):
        L = rng.uniform(0.1, 3.0, 3)
        assert abs(aharoni(*L).sum() - 1) < 1e-12


def test_self_term(oracle_mod):
    N = oracle_mod.newell(0, 0, 0, 5e-9, 5e-9, 5e-9)
    assert np.allclose(N[:3], 1 / 3, atol=1e-14) and np.allclose(N[3:], 0, atol=1e-14)
    for cell in [(4e-9, 4e-9, 2e-9), (3e-9, 5e-9, 1e-9), (2e-9, 7e-9, 3e-9)]:
        N = oracle_mod.newell(0, 0, 0, *cell)
        assert abs(N[:3].sum() - 1) < 1e-13
        assert np.allclose(N[:3], aharoni(*cell), rtol=0, atol=1e-12)


def test_symmetry_and_parity(oracle_mod):
    h = (4e-9, 4e-9, 2e-9)
    rng = np.random.default_rng(2)
    for _ in range(20):
        i, j, k = rng.integers(-15, 16, 3)
        X, Y, Z = i * h[0], j * h[1], k * h[2]
        N = oracle_mod.newell(X, Y, Z, *h)
        for sx, sy, sz in itertools.product([1, -1], repeat=3):
            M = oracle_mod.newell(sx * X, sy * Y, sz * Z, *h)
            assert np.allclose(M[:3], N[:3], rtol=0, atol=1e-8 * np.abs(N).max())
            assert np.allclose(M[3], sx * sy * N[3], rtol=0, atol=1e-8 * np.abs(N).max())
            assert np.allclose(M[4], sx * sz * N[4], rtol=0, atol=1e-8 * np.abs(N).max())
            assert np.allclose(M[5], sy * sz * N[5], rtol=0, atol=1e-8 * np.abs(N).max())
        # swapping the roles of x and y (with the cell sizes) swaps xx <-> yy and xz <-> yz
        S = oracle_mod.newell(Y, X, Z, h[1], h[0], h[2])
        assert np.allclose([S[1], S[0], S[2], S[3], S[5], S[4]], N, rtol=0, atol=1e-8 * np.abs(N).max())


def test_near_far_agree(oracle_mod):
    """The closed form and the cell-average expansion are independent; where
    both are accurate (8-12 cells) they must agree."""
    rng = np.random.default_rng(3)
    for h in [(5e-9,) * 3, (4e-9, 4e-9, 2e-9), (3e-9, 3e-9, 3e-9)]:
        hm = max(h)
        for _ in range(10):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            r = rng.uniform(8.5, 12.0) * hm
            X, Y, Z = d * r
            a = oracle_mod.newell(X, Y, Z, *h, kind="exact")
            b = oracle_mod.newell(X, Y, Z, *h, kind="far", order=6)
            assert np.abs(a - b).max() < 2e-7 * np.abs(a).max()


def test_point_dipole_limit(oracle_mod):
    h = (4e-9, 4e-9, 2e-9)
    V = np.prod(h)
    for R in [np.array([300, 17, 3]) * 4e-9, np.array([-200, 150, 40]) * 4e-9]:
        N = oracle_mod.newell(*R, *h)
        r = np.linalg.norm(R)
        D = V / (4 * np.pi * r**3) * (np.eye(3) - 3 * np.outer(R, R) / r**2)
        ref = np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])
        assert np.abs(N - ref).max() < 1e-4 * np.abs(ref).max()


def test_dinvr_against_numerical_derivatives(oracle_mod):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    x0, y0, z0 = 1.3, -0.7, 2.1
    f = lambda x, y, z: 1 / mp.sqrt(x * x + y * y + z * z)
    for a, b, c in [(2, 0, 0), (1, 1, 0), (0, 1, 1), (4, 0, 0), (2, 2, 0), (1, 1, 2), (3, 1, 2), (6, 0, 2), (2, 2, 2)]:
        ref = mp.diff(f, (x0, y0, z0), (a, b, c))
        got = oracle_mod.dinvr(a, b, c, x0, y0, z0)
        assert abs(got - float(ref)) < 1e-12 * max(1.0, abs(float(ref)))


@pytest.mark.parametrize("grid,cell", [((8, 8, 2), (5e-9,) * 3), ((5, 3, 3), (4e-9, 4e-9, 2e-9)),
                                       ((16, 16, 1), (4e-9, 4e-9, 2e-9)), ((6, 10, 3), (3e-9, 5e-9, 2e-9)),
                                       ((1, 1, 1), (5e-9,) * 3), ((7, 1, 1), (5e-9,) * 3)])
def test_fft_equals_direct_sum(oracle_mod, grid, cell):
    rng = np.random.default_rng(4)
    N = int(np.prod(grid))
    m = rng.normal(size=(3, N))
    h1 = oracle_mod.demag_direct(grid, cell, m)
    h2 = oracle_mod.DemagPlan(grid, cell)(m)
    assert np.abs(h1 - h2).max() < 1e-12 * np.abs(h1).max()
    cells = rng.integers(0, N, 5)
    h3 = oracle_mod.demag_direct_at(grid, cell, m, cells)
    assert np.abs(h3 - h1[:, cells].T).max() < 1e-12 * np.abs(h1).max()


@pytest.mark.parametrize("grid,cell", [((10, 6, 3), (5e-9,) * 3), ((24, 24, 1), (4e-9, 4e-9, 2e-9)),
                                       ((40, 9, 2), (3e-9, 3e-9, 3e-9))])
def test_uniform_block_matches_aharoni(oracle_mod, grid, cell):
    """Block-average of h for uniform m = -(Aharoni factor of the block)."""
    N = int(np.prod(grid))
    D = aharoni(*(np.array(grid) * np.array(cell)))
    plan = oracle_mod.DemagPlan(grid, cell)
    for ax in range(3):
        m = np.zeros((3, N))
        m[ax] = 1.0
        h = plan(m)
        assert abs(-h[ax].mean() - D[ax]) < 2e-9
        other = [k for k in range(3) if k != ax]
        assert np.abs(h[other].mean(axis=1)).max() < 1e-12
