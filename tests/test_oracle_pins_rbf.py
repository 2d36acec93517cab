"""Pins of the oracle's Gaussian blob sum and of its reinitialisation solvers
(no GPU): the blob kernel against the cutoff of Eq. (2), the partition of
unity of a fine lattice of blobs, conjugate gradients against a dense LAPACK
solve, and the Fourier-diagonal lattice solution against the real-space
periodic sum."""
import numpy as np
import pytest

import oracle
import workloads as wl


def test_blob_kernel_is_the_derivative_of_the_cutoff_mass():
    """zeta_sigma(rho) = g'(rho) / (4 pi rho^2) with g = 4 pi rho^3 q(rho) the
    enclosed mass of Eq. (2) (q from the pinned pair factors)."""
    sigma = 0.37
    for ros in (0.1, 0.5, 1.0, 1.7, 3.0, 4.5):
        rho = ros * sigma
        hh = 1e-5 * sigma
        g = lambda r: 4.0 * np.pi * r ** 3 * oracle.pair_factors(r, sigma)[0][0]
        gp = (g(rho + hh) - g(rho - hh)) / (2 * hh)
        src = dict(x=[0.0], y=[0.0], z=[0.0], sigma=[sigma])
        d = np.array([0.48, -0.6, 0.64]) * rho
        w = oracle.gaussian_sum(src, [[1.0, -2.0, 0.5]], points=d[None, :])
        zeta = gp / (4.0 * np.pi * rho * rho)
        assert np.allclose(w[0], zeta * np.array([1.0, -2.0, 0.5]), rtol=1e-8, atol=0)


def test_fine_lattice_of_blobs_is_a_partition_of_unity():
    """sum_j h^3 zeta_sigma(x - x_j) = 1 up to exp(-2 pi^2 sigma^2 / h^2)
    (Poisson summation) on an unbounded lattice; here a periodic one."""
    n, L = 12, 3.0
    x, y, z, h = wl.lattice_positions(n, L)
    sigma = 1.5 * h
    case = dict(x=x, y=y, z=z, sigma=np.full(x.size, sigma))
    gam = np.full((x.size, 3), h ** 3)
    pts = np.random.default_rng(1).uniform(0, L, (50, 3))
    w = oracle.gaussian_sum(case, gam, points=pts, shifts=oracle.image_shifts(2, L))
    assert np.abs(w - 1.0).max() <= 1e-13


def _cloud(n=300, seed=2):
    c = wl.random_cloud(n, seed=seed, L=1.0, core=0.0)
    c["sigma"] = np.full(n, 0.09)
    return c


def test_conjugate_gradients_match_a_dense_solve():
    case = _cloud()
    n = case["n"]
    rng = np.random.default_rng(3)
    omega = rng.standard_normal((n, 3))
    # dense matrix column by column from unit strengths
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros((n, 3))
        e[j, 0] = 1.0
        A[:, j] = oracle.gaussian_sum(case, e)[:, 0]
    assert np.allclose(A, A.T, rtol=1e-13, atol=0)
    ref = np.linalg.solve(A, omega)
    g, it, res = oracle.rbf_cg(case, omega, tol=1e-13, maxiter=5000)
    assert np.all(res <= 1e-13)
    assert np.linalg.norm(g - ref) <= 1e-8 * np.linalg.norm(ref)


def _smooth_lattice(n, seed, kmax=2, sigma_h=1.5, L=2 * np.pi):
    x, y, z, h = wl.lattice_positions(n, L)
    rng = np.random.default_rng(seed)
    om = np.zeros((x.size, 3))
    for _ in range(6):
        k = rng.integers(-kmax, kmax + 1, 3) * (2 * np.pi / L)
        ph = rng.uniform(0, 2 * np.pi)
        om += np.outer(np.cos(k[0] * x + k[1] * y + k[2] * z + ph), rng.standard_normal(3))
    case = dict(x=x, y=y, z=z, sigma=np.full(x.size, sigma_h * h), lattice_n=n, L=L)
    return case, om


def test_lattice_solution_matches_periodic_conjugate_gradients():
    """Cores as wide as the spacing keep the lattice system well conditioned
    in float64, so the two solvers agree to rounding."""
    n, L = 8, 2 * np.pi
    case, om = _smooth_lattice(n, seed=4, sigma_h=1.0)
    gl = oracle.rbf_lattice(case, om)
    gc, it, res = oracle.rbf_cg(case, om, tol=1e-13, maxiter=2000, shifts=oracle.image_shifts(2, L))
    assert np.all(res <= 1e-13)
    assert np.linalg.norm(gl - gc) <= 1e-10 * np.linalg.norm(gl)


@pytest.mark.parametrize("n,sigma_h", [(8, 1.5), (12, 1.5), (10, 1.0)])
def test_lattice_blob_sum_matches_real_space_images(n, sigma_h):
    """The DFT route of the periodic blob sum against the real-space sum over
    image shifts, at the lattice points and at shifted points."""
    L = 2 * np.pi
    case, _ = _smooth_lattice(n, seed=7, sigma_h=sigma_h)
    g = np.random.default_rng(8).standard_normal((n ** 3, 3))
    sh = oracle.image_shifts(2, L)
    h = L / n
    for dl in (None, (-0.5 * h, -0.5 * h, -0.5 * h), (0.2 * h, 0.7 * h, -0.4 * h)):
        f = oracle.gaussian_lattice(case, g, offset=dl)
        pts = np.stack([case["x"], case["y"], case["z"]], 1) + (0.0 if dl is None else np.asarray(dl))
        r = oracle.gaussian_sum(case, g, points=pts, shifts=sh)
        assert np.abs(f - r).max() <= 1e-11 * np.abs(r).max()


@pytest.mark.parametrize("n,seed", [(8, 5), (12, 6)])
def test_lattice_solution_reproduces_the_vorticity_in_real_space(n, seed):
    """The periodic real-space blob sum of the Fourier-diagonal solution gives
    back the vorticity at every lattice point."""
    L = 2 * np.pi
    case, om = _smooth_lattice(n, seed=seed, kmax=3, sigma_h=1.0)
    g = oracle.rbf_lattice(case, om)
    back = oracle.gaussian_sum(case, g, shifts=oracle.image_shifts(2, L))
    assert np.abs(back - om).max() <= 1e-10 * np.abs(om).max()


def test_conjugate_gradients_with_the_lattice_product_match_the_lattice_solution():
    """CG with the DFT product over every periodic image (the route the GPU
    reinitialisation is checked with at lattice sizes the real-space sum cannot
    reach) converges to the Fourier-diagonal solution."""
    n = 10
    case, om = _smooth_lattice(n, seed=9, kmax=2, sigma_h=1.0)
    gl = oracle.rbf_lattice(case, om)
    gc, it, res = oracle.rbf_cg(case, om, tol=1e-13, maxiter=2000, matvec=lambda v: oracle.gaussian_lattice(case, v))
    assert np.all(res <= 1e-13) and np.all(it >= 2)
    assert np.linalg.norm(gl - gc) <= 1e-10 * np.linalg.norm(gl)
