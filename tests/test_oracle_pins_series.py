"""Pins of the oracle's Fourier-series, shifted-lattice, energy-spectrum and
Heun-step routes against facts fixed by mathematics (no GPU): another route
to the same sum, closed forms, exact invariants.  Each would fail for a
plausible mistake (a wrong sign of a phase, a transposed index, a dropped
alias, a wrong stage weight)."""
import numpy as np
import pytest

import oracle
import workloads as wl

L2PI = 2.0 * np.pi


def _tiny_periodic(n=4, seed=1, sigma=0.45):
    xs, ys, zs, h = wl.lattice_positions(n)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((3, n ** 3))
    a -= a.mean(1, keepdims=True)
    return dict(x=xs, y=ys, z=zs, ax=a[0], ay=a[1], az=a[2], sigma=np.full(n ** 3, sigma), lattice_n=n, L=L2PI)


# ----------------------------------------------------------------------------
# Fourier series with phases factored per axis
# ----------------------------------------------------------------------------
def test_separable_series_equals_dense_phase_series():
    """Same terms, another way of forming the phases: off the lattice, at the
    particles and at other points."""
    case = wl.random_cloud(300, seed=5, L=L2PI, core=0.55, zero_mean=True, periodic=True)
    pts = np.random.default_rng(6).uniform(0, L2PI, (77, 3))
    for kw in ({}, dict(points=pts)):
        u1, J1 = oracle.fourier_points(case, L2PI, 9, **kw)
        u2, J2 = oracle.fourier_series_points(case, L2PI, 9, chunk=64, **kw)
        assert np.abs(u1 - u2).max() <= 1e-12 * np.abs(u1).max()
        assert np.abs(J1 - J2).max() <= 1e-12 * np.abs(J1).max()


def test_separable_series_matches_lattice_alias_folding():
    """On a cell-centred lattice whose positions are exact in float32 (h = 1),
    the pointwise series equals the FFT route with folded aliases."""
    case = wl.turbulence_case(16, seed=9, L=16.0)
    us, Js = oracle.spectral_lattice(case)
    uf, Jf = oracle.fourier_series_points(case, 16.0, 12)
    assert np.linalg.norm(uf - us) <= 1e-11 * np.linalg.norm(us)
    assert np.linalg.norm(Jf - Js) <= 1e-11 * np.linalg.norm(Js)


def test_separable_series_taylor_green_off_lattice():
    """alpha = omega_TG h^3 on a lattice: the periodic blob field is
    exp(-3 sigma^2/2) u_TG at ANY point (closed form), with its gradient."""
    d = wl.taylor_green_case(16, periodic=True)
    sig = float(d["sigma"][0])
    pts = np.random.default_rng(3).uniform(0, L2PI, (500, 3))
    u, J = oracle.fourier_series_points(d, L2PI, 4, points=pts)
    f = np.exp(-1.5 * sig * sig)
    sx, sy, sz = np.sin(pts[:, 0]), np.sin(pts[:, 1]), np.sin(pts[:, 2])
    cx, cy, cz = np.cos(pts[:, 0]), np.cos(pts[:, 1]), np.cos(pts[:, 2])
    uTG = np.stack([sx * cy * cz, -cx * sy * cz, 0 * sx], 1) * f
    assert np.abs(u - uTG).max() <= 2e-6 * np.abs(uTG).max()  # alpha is float32-rounded
    assert abs(J[:, 0, 0] - f * cx * cy * cz).max() <= 2e-6 * f
    assert abs(J[:, 2, 1] - f * cx * sy * sz).max() <= 2e-6 * f
    assert np.abs(np.trace(J, axis1=1, axis2=2)).max() <= 1e-6 * f  # div u = 0


# ----------------------------------------------------------------------------
# lattice route at shifted points (probe lattice)
# ----------------------------------------------------------------------------
def test_shifted_lattice_by_one_cell_is_a_roll():
    """Shifting every evaluation point by exactly one cell along x reads the
    unshifted field one lattice index further on."""
    case = _tiny_periodic(n=6, seed=2, sigma=0.6)
    h = L2PI / 6
    u0, J0 = oracle.spectral_lattice(case)
    u1, J1 = oracle.spectral_lattice(case, offset=(h, 0.0, 0.0))
    r = lambda a: np.roll(a.reshape((6, 6, 6) + a.shape[1:]), -1, axis=0).reshape(a.shape)
    assert np.abs(u1 - r(u0)).max() <= 1e-12 * np.abs(u0).max()
    assert np.abs(J1 - r(J0)).max() <= 1e-12 * np.abs(J0).max()


@pytest.mark.parametrize("delta", [(-0.5, -0.5, -0.5), (0.3, -0.1, 0.45)])
def test_shifted_lattice_matches_pointwise_series(delta):
    case = _tiny_periodic(n=6, seed=4, sigma=0.5)
    h = L2PI / 6
    dl = np.asarray(delta) * h
    us, Js = oracle.spectral_lattice(case, offset=dl)
    pts = np.stack([case["x"], case["y"], case["z"]], 1) + dl
    uf, Jf = oracle.fourier_points(case, L2PI, 14, points=pts)
    assert np.abs(us - uf).max() <= 1e-9 * np.abs(us).max()
    assert np.abs(Js - Jf).max() <= 1e-9 * np.abs(Js).max()


# ----------------------------------------------------------------------------
# energy spectrum
# ----------------------------------------------------------------------------
def test_energy_spectrum_single_mode_and_parseval():
    n = 16
    x, y, z, h = wl.lattice_positions(n)
    u = np.stack([0 * x, np.cos(3 * x), 0 * x], 1)          # one mode, |k| = 3
    E = oracle.energy_spectrum(u, n, L2PI)
    assert abs(E[3] - 0.25) <= 1e-14 and abs(E.sum() - 0.25) <= 1e-14
    v = np.stack([np.sin(2 * y) * np.cos(z), np.cos(4 * x), 0.5 + 0 * x], 1)
    Ev = oracle.energy_spectrum(v, n, L2PI)
    # (sin 2y cos z): |k| = sqrt 5 -> shell 2, energy 1/8; cos 4x: shell 4, 1/4; mean 0.5: shell 0, 1/8
    assert abs(Ev[2] - 0.125) <= 1e-14 and abs(Ev[4] - 0.25) <= 1e-14 and abs(Ev[0] - 0.125) <= 1e-14
    rng = np.random.default_rng(1)
    w = rng.standard_normal((n ** 3, 3))
    Ew = oracle.energy_spectrum(w, n, L2PI)
    assert abs(Ew.sum() - 0.5 * np.mean(np.sum(w * w, 1))) <= 1e-12 * Ew.sum()


# ----------------------------------------------------------------------------
# Heun step
# ----------------------------------------------------------------------------
def _state(n=20, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, (3, n))
    a = rng.standard_normal((3, n))
    return dict(x=p[0], y=p[1], z=p[2], ax=a[0], ay=a[1], az=a[2], sigma=np.full(n, 0.1))


def test_heun_step_on_a_linear_system_is_the_second_order_taylor_map():
    """For dalpha/dt = M alpha and dx/dt = B x, Heun's rule gives
    (I + dt M + dt^2 M^2 / 2) exactly; sigma^2 grows by 2 nu dt."""
    rng = np.random.default_rng(2)
    M = rng.standard_normal((3, 3))
    B = rng.standard_normal((3, 3))
    case = _state()
    dt, nu = 0.07, 0.3
    out = oracle.heun_step(case, dt, nu, lambda x, a, s: (x @ B.T, a @ M.T))
    x0 = np.stack([case["x"], case["y"], case["z"]], 1)
    a0 = np.stack([case["ax"], case["ay"], case["az"]], 1)
    I = np.eye(3)
    assert np.allclose(out["alpha"], a0 @ (I + dt * M + 0.5 * dt * dt * M @ M).T, rtol=0, atol=1e-14)
    assert np.allclose(out["x"], x0 @ (I + dt * B + 0.5 * dt * dt * B @ B).T, rtol=0, atol=1e-14)
    assert np.allclose(out["sigma"] ** 2, 0.01 + 2 * nu * dt, rtol=1e-14, atol=0)


def test_heun_step_stage_two_sees_the_predicted_core_and_wraps():
    """The second stage is evaluated at sigma*^2 = sigma^2 + 2 nu dt and at
    the wrapped predictor; positions end inside [lo, lo + L)."""
    case = _state(n=8, seed=3)
    seen = []

    def rates(x, a, s):
        seen.append((x.copy(), s.copy()))
        return np.full_like(x, 3.0), np.zeros_like(a)

    out = oracle.heun_step(case, 0.5, 0.2, rates, L=1.0, lo=(0.0, 0.0, 0.0))
    assert np.allclose(seen[1][1] ** 2, 0.01 + 0.2, rtol=1e-14)
    assert np.all((seen[1][0] >= 0) & (seen[1][0] < 1.0))
    x0 = np.stack([case["x"], case["y"], case["z"]], 1)
    assert np.allclose(out["x"], np.mod(x0 + 1.5, 1.0), atol=1e-14)


def test_heun_step_with_the_direct_sum_conserves_total_strength():
    """The transpose reading of Eq. (3) sums to zero over the particles at
    every stage, so a Heun step keeps sum alpha."""
    case = wl.random_cloud(200, seed=8, L=1.0, core=0.08)

    def rates(x, a, s):
        c = dict(x=x[:, 0], y=x[:, 1], z=x[:, 2], ax=a[:, 0], ay=a[:, 1], az=a[:, 2], sigma=s)
        r = oracle.direct(c)
        return r["u"], r["da_t"]

    out = oracle.heun_step(case, 0.05, 0.0, rates)
    a0 = np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)
    assert np.abs(out["alpha"].sum(0) - a0.sum(0)).max() <= 1e-13 * np.abs(a0).sum()
    assert not np.allclose(out["alpha"], a0)
