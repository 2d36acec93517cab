"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(no GPU).  Each test would fail for a plausible mistake in the oracle: a
dropped term, a wrong sign or index, a transposed operand, a wrong branch."""
import json
import os

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gauss3(r, sigma):
    """Normalised 3-D Gaussian core zeta_sigma(r)."""
    return (2.0 * np.pi * sigma * sigma) ** -1.5 * np.exp(-0.5 * r * r / (sigma * sigma))


# ----------------------------------------------------------------------------
# Eq. (2): g is the Gaussian mass enclosed in a ball of radius rho
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("ros", [1e-3, 0.05, 0.3, 0.49, 0.51, 1.0, 2.0, 4.0, 7.0])
def test_cutoff_is_enclosed_gaussian_mass(ros):
    sigma = 0.37
    rho = ros * sigma
    q, _ = oracle.pair_factors(rho, sigma)
    g = q[0] * 4.0 * np.pi * rho ** 3
    mass, _ = integrate.quad(lambda r: 4.0 * np.pi * r * r * gauss3(r, sigma), 0.0, rho,
                             epsabs=0.0, epsrel=1e-13, limit=200)
    assert abs(g - mass) <= 2e-12 * mass + 1e-300


@pytest.mark.parametrize("ros", [1e-3, 0.2, 0.49, 0.51, 1.5, 5.0])
def test_qprime_from_gaussian_density(ros):
    """d/drho [g/(4 pi rho^3)] with g' = 4 pi rho^2 zeta_sigma (the derivative of
    the enclosed mass), compared with the oracle's q'/rho."""
    sigma = 0.8
    rho = ros * sigma
    q, qpr = oracle.pair_factors(rho, sigma)
    g = q[0] * 4.0 * np.pi * rho ** 3
    gp = 4.0 * np.pi * rho * rho * gauss3(rho, sigma)
    t1, t2 = gp / (4.0 * np.pi * rho ** 3), 3.0 * g / (4.0 * np.pi * rho ** 4)
    dq = t1 - t2
    # the reference itself cancels for rho << sigma: bound by the terms' size
    assert abs(qpr[0] * rho - dq) <= 1e-10 * (abs(t1) + abs(t2))


def test_single_blob_limits():
    """Near the centre a blob rotates rigidly with Omega = omega(0)/3 =
    alpha zeta(0)/3; far away it is a point vortex alpha x r / (4 pi rho^3)."""
    sigma = 0.5
    alpha = np.array([0.3, -0.2, 0.9])
    src = dict(x=[0.0], y=[0.0], z=[0.0], ax=[alpha[0]], ay=[alpha[1]], az=[alpha[2]], sigma=[sigma])
    # near target
    eps = 1e-4 * sigma
    d = np.array([0.6, -0.3, 0.74]) * eps
    case = {k: np.asarray(v, dtype=np.float64) for k, v in src.items()}
    case2 = {k: np.concatenate([case[k], [v]]) for k, v in
             dict(x=d[0], y=d[1], z=d[2], ax=0.0, ay=0.0, az=0.0, sigma=sigma).items()}
    out = oracle.direct(case2, targets=[1])
    omega0 = alpha * gauss3(0.0, sigma)
    u_rigid = np.cross(omega0 / 3.0, d)
    assert np.allclose(out["u"][0], u_rigid, rtol=1e-7, atol=0)
    # far target
    D = np.array([4.0, 3.0, -12.0]) * sigma
    case3 = {k: np.concatenate([case[k], [v]]) for k, v in
             dict(x=D[0], y=D[1], z=D[2], ax=0.0, ay=0.0, az=0.0, sigma=sigma).items()}
    out = oracle.direct(case3, targets=[1])
    u_pt = np.cross(alpha, D) / (4.0 * np.pi * np.linalg.norm(D) ** 3)
    assert np.allclose(out["u"][0], u_pt, rtol=1e-13, atol=0)


def test_blob_of_blobs_velocity():
    """A fine lattice of small blobs (core s) sampling a big Gaussian vorticity
    alpha0 zeta_S induces the field of one blob of core sqrt(S^2 + s^2)."""
    S, s, n = 0.5, 0.12, 40
    h = 10.0 * S / n
    c = (np.arange(n) + 0.5) * h - 5.0 * S
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    a0 = np.array([0.2, 0.5, -0.4])
    w = gauss3(np.sqrt(X * X + Y * Y + Z * Z), S) * h ** 3
    tg = np.array([[0.31, -0.22, 0.17], [0.9, 0.4, -0.6], [1.6, -1.1, 0.8]])
    case = dict(x=np.concatenate([X, tg[:, 0]]), y=np.concatenate([Y, tg[:, 1]]),
                z=np.concatenate([Z, tg[:, 2]]),
                ax=np.concatenate([a0[0] * w, np.zeros(3)]), ay=np.concatenate([a0[1] * w, np.zeros(3)]),
                az=np.concatenate([a0[2] * w, np.zeros(3)]), sigma=np.full(X.size + 3, s))
    out = oracle.direct(case, targets=np.arange(X.size, X.size + 3))
    big = dict(x=[0.0] + list(tg[:, 0]), y=[0.0] + list(tg[:, 1]), z=[0.0] + list(tg[:, 2]),
               ax=[a0[0], 0, 0, 0], ay=[a0[1], 0, 0, 0], az=[a0[2], 0, 0, 0],
               sigma=[np.sqrt(S * S + s * s)] * 4)
    ref = oracle.direct(big, targets=[1, 2, 3])
    assert np.abs(out["u"] - ref["u"]).max() <= 1e-6 * np.abs(ref["u"]).max()
    assert np.abs(out["J"] - ref["J"]).max() <= 1e-6 * np.abs(ref["J"]).max()


def _cloud(n=60, seed=3, sigma=0.21):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, size=(3, n))
    a = rng.standard_normal((3, n))
    return dict(x=p[0], y=p[1], z=p[2], ax=a[0], ay=a[1], az=a[2], sigma=np.full(n, sigma))


def test_gradient_matches_finite_differences():
    case = _cloud()
    out = oracle.direct(case)
    # probe: a massless target moved along each axis (4th-order central FD)
    i = 7
    hh = 1e-3
    J_fd = np.zeros((3, 3))
    for k in range(3):
        vals = []
        for st in (-2, -1, 1, 2):
            pos = np.array([case["x"][i], case["y"][i], case["z"][i]])
            pos[k] += st * hh
            c2 = {kk: np.concatenate([v, [0.0]]) for kk, v in case.items()}
            c2["x"][-1], c2["y"][-1], c2["z"][-1] = pos
            c2["sigma"][-1] = case["sigma"][0]
            # drop source i so the probe sees the same field as target i minus its own blob,
            # then add the self blob analytically via the oracle with i kept: keep all sources
            vals.append(oracle.direct(c2, targets=[c2["x"].size - 1])["u"][0])
        J_fd[k] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * hh)
    assert np.abs(J_fd - out["J"][i]).max() <= 1e-8 * np.abs(out["J"][i]).max()


def test_divergence_free_and_vorticity_identity():
    case = _cloud(80, seed=5)
    out = oracle.direct(case)
    J = out["J"]
    tr = J[:, 0, 0] + J[:, 1, 1] + J[:, 2, 2]
    assert np.abs(tr).max() <= 1e-12 * np.abs(J).max()
    # classical - transpose = (curl u) x alpha_i, curl u_a = eps_abc J_bc
    w = np.stack([J[:, 1, 2] - J[:, 2, 1], J[:, 2, 0] - J[:, 0, 2], J[:, 0, 1] - J[:, 1, 0]], axis=1)
    a = np.stack([case["ax"], case["ay"], case["az"]], axis=1)
    assert np.allclose(out["da_c"] - out["da_t"], np.cross(w, a), rtol=0, atol=1e-12 * np.abs(out["da_t"]).max())


def test_transpose_scheme_conserves_total_strength():
    """Eq. (3) as printed is pairwise antisymmetric: sum_i dalpha_i = 0."""
    case = _cloud(70, seed=11)
    out = oracle.direct(case)
    scale = np.abs(out["da_t"]).sum(axis=0).max()
    assert np.abs(out["da_t"].sum(axis=0)).max() <= 1e-13 * scale
    # the "omega . grad u" reading is not conservative for generic strengths
    assert np.abs(out["da_c"].sum(axis=0)).max() > 1e-4 * scale


def test_uniform_strength_zero_net_velocity():
    case = _cloud(50, seed=2)
    for k in ("ax", "ay", "az"):
        case[k] = np.full(50, {"ax": 0.3, "ay": -0.7, "az": 0.5}[k])
    out = oracle.direct(case)
    assert np.abs(out["u"].sum(axis=0)).max() <= 1e-13 * np.abs(out["u"]).sum()


def test_point_inversion_and_rotation():
    case = _cloud(40, seed=8)
    out = oracle.direct(case)
    inv = dict(case, x=-case["x"], y=-case["y"], z=-case["z"])
    oi = oracle.direct(inv)
    assert np.allclose(oi["u"], -out["u"], rtol=0, atol=1e-13 * np.abs(out["u"]).max())
    assert np.allclose(oi["da_t"], out["da_t"], rtol=0, atol=1e-13 * np.abs(out["da_t"]).max())
    # proper rotation
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    ph = -0.4
    Rx = np.array([[1, 0, 0], [0, np.cos(ph), -np.sin(ph)], [0, np.sin(ph), np.cos(ph)]])
    R = Rx @ Rz
    P = R @ np.stack([case["x"], case["y"], case["z"]])
    A = R @ np.stack([case["ax"], case["ay"], case["az"]])
    rot = dict(case, x=P[0], y=P[1], z=P[2], ax=A[0], ay=A[1], az=A[2])
    orot = oracle.direct(rot)
    assert np.allclose(orot["u"], out["u"] @ R.T, rtol=0, atol=1e-12 * np.abs(out["u"]).max())
    assert np.allclose(orot["da_t"], out["da_t"] @ R.T, rtol=0, atol=1e-12 * np.abs(out["da_t"]).max())
    assert np.allclose(orot["J"], np.einsum("ab,ibc,dc->iad", R, out["J"], R), rtol=0,
                       atol=1e-12 * np.abs(out["J"]).max())


@pytest.mark.parametrize("zt", [0.0, 0.7, -1.3])
def test_ring_axis_velocity_sign(zt):
    """A ring with alpha along +phi (right-handed about +z) drives the fluid on
    its axis along +z with the circular-loop value Gamma R^2 / (2 (R^2+z^2)^1.5)."""
    rng = np.random.default_rng(0)
    ring = wl.ring_case(257, rng, radius=1.0, core=0.1, jitter=0.0, circulation=1.0)
    case = {k: np.concatenate([np.asarray(ring[k], np.float64), [v]]) for k, v in
            dict(x=0.0, y=0.0, z=zt, ax=0.0, ay=0.0, az=0.0, sigma=0.1).items()}
    out = oracle.direct(case, targets=[case["x"].size - 1])
    # float32-rounded ring: compare the discrete sum of its exact geometry
    x = np.asarray(ring["x"], np.float64)
    y = np.asarray(ring["y"], np.float64)
    rr = np.sqrt(x * x + y * y)
    gam_eff = np.sum(np.hypot(ring["ax"].astype(np.float64), ring["ay"].astype(np.float64))) / (2 * np.pi * rr.mean())
    uz = gam_eff * rr.mean() ** 2 / (2.0 * (rr.mean() ** 2 + zt * zt) ** 1.5)
    assert out["u"][0, 2] > 0
    assert abs(out["u"][0, 2] - uz) <= 1e-6 * uz
    assert np.abs(out["u"][0, :2]).max() <= 1e-6 * uz


# ----------------------------------------------------------------------------
# periodic convention
# ----------------------------------------------------------------------------
def test_taylor_green_periodic_closed_form():
    """alpha = omega_TG h^3 on the lattice: the periodic blob field is exactly
    exp(-3 sigma^2 / 2) u_TG (only |k|^2 = 3 modes are present)."""
    d = wl.taylor_green_case(16, periodic=True)
    u, J = oracle.spectral_lattice(d)
    x = np.stack([d["x"], d["y"], d["z"]], 1).astype(np.float64)
    sig = float(d["sigma"][0])
    f = np.exp(-1.5 * sig * sig)
    sx, sy, sz = np.sin(x[:, 0]), np.sin(x[:, 1]), np.sin(x[:, 2])
    cx, cy, cz = np.cos(x[:, 0]), np.cos(x[:, 1]), np.cos(x[:, 2])
    uTG = np.stack([sx * cy * cz, -cx * sy * cz, 0 * sx], 1) * f
    JTG = np.zeros_like(J)
    JTG[:, 0, 0] = cx * cy * cz
    JTG[:, 1, 0] = -sx * sy * cz
    JTG[:, 2, 0] = -sx * cy * sz
    JTG[:, 0, 1] = sx * sy * cz
    JTG[:, 1, 1] = -cx * cy * cz
    JTG[:, 2, 1] = cx * sy * sz
    JTG *= f
    # alpha is float32-rounded: ~1e-7 relative
    assert np.abs(u - uTG).max() <= 1e-6 * np.abs(uTG).max()
    assert np.abs(J - JTG).max() <= 1e-6 * np.abs(JTG).max()


def _tiny_periodic(n=4, seed=1, sigma=0.45):
    L = 2 * np.pi
    xs, ys, zs, h = wl.lattice_positions(n)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((3, n ** 3))
    a -= a.mean(1, keepdims=True)
    return dict(x=xs, y=ys, z=zs, ax=a[0], ay=a[1], az=a[2], sigma=np.full(n ** 3, sigma),
                lattice_n=n, L=L)


def test_spectral_lattice_matches_pointwise_fourier_series():
    case = _tiny_periodic()
    us, Js = oracle.spectral_lattice(case)
    uf, Jf = oracle.fourier_points(case, case["L"], 12)
    assert np.abs(us - uf).max() <= 1e-7 * np.abs(us).max()
    assert np.abs(Js - Jf).max() <= 1e-7 * np.abs(Js).max()


def test_cube_ordered_image_sum_converges_to_spectral_plus_surface_term():
    case = _tiny_periodic()
    L = case["L"]
    us, Js = oracle.spectral_lattice(case)
    du = oracle.surface_term(case, L)
    tg = [0, 5, 17, 42]
    errs = []
    for M in (4, 13):
        b = oracle.brute_images(case, M, L, targets=tg)
        errs.append(np.abs(b["u"] - (us[tg] + du)).max() / np.abs(us).max())
        # without the surface term the cube-ordered sum does not converge to the spectral one
        assert np.abs(b["u"] - us[tg]).max() / np.abs(us).max() > 0.05
        assert np.abs(b["J"] - Js[tg]).max() / np.abs(Js).max() < 0.02
    # error falls roughly as 1/M^2: (13/4)^2 ~ 10.6
    assert errs[1] < errs[0] / 5.0
    assert errs[1] < 1e-3


def test_paper_table1_flop_convention():
    """Table 1 and the sustained-performance arithmetic (Sec. 4.5)."""
    with open(os.path.join(GOLDEN, "paper_table1_flops.json")) as f:
        t = json.load(f)
    bs, st = t["biot_savart"], t["stretching"]
    assert sum(bs.values()) == t["total_biot_savart"] == 70
    assert sum(st.values()) == t["total_stretching"] == 104
    pf = 4096 * 256 ** 3 * 19 * 512 * (70 + 104) / 108.0
    assert abs(pf / 1e15 - t["sustained_pflops"]) < 0.01


# ----------------------------------------------------------------------------
# Eq. (1) at points that are not particles (separate target sets)
# ----------------------------------------------------------------------------
def test_points_far_field_is_singular_biot_savart_of_total_strength():
    """Far from a compact cloud every cutoff is 1 and u -> (sum alpha) x x / (4 pi |x|^3),
    with a relative correction of order (cloud size / distance)."""
    case = _cloud(60, seed=8)
    A = np.array([np.sum(case["ax"]), np.sum(case["ay"]), np.sum(case["az"])], dtype=np.float64)
    c0 = np.array([np.mean(case["x"]), np.mean(case["y"]), np.mean(case["z"])], dtype=np.float64)
    d = np.array([[1.0, 0.3, -0.2], [-0.4, 1.0, 0.7], [0.2, -0.6, -1.0]])
    for R in (1e3, 1e4):
        pts = c0 + R * d
        u = oracle.direct_points(case, pts)["u"]
        r = pts - c0
        ref = np.cross(A, r) / (4 * np.pi * np.linalg.norm(r, axis=1)[:, None] ** 3)
        err = np.abs(u - ref).max() / np.abs(ref).max()
        assert err <= 10.0 / R, (R, err)


def test_points_match_particle_sums_and_are_divergence_free():
    """At the particles' own positions the point sum equals the particle sum
    (the self pair contributes nothing), and off the particles tr J = 0."""
    case = _cloud(70, seed=9)
    pts = np.stack([case["x"], case["y"], case["z"]], axis=1).astype(np.float64)
    a = oracle.direct_points(case, pts)
    b = oracle.direct(case)
    assert np.allclose(a["u"], b["u"], rtol=0, atol=1e-14 * np.abs(b["u"]).max())
    off = np.random.default_rng(3).uniform(-0.2, 1.2, size=(50, 3))
    J = oracle.direct_points(case, off)["J"]
    assert np.abs(J[:, 0, 0] + J[:, 1, 1] + J[:, 2, 2]).max() <= 1e-12 * np.abs(J).max()


# ----------------------------------------------------------------------------
# Eq. (2) with unequal cores: each pair uses its source's core
# ----------------------------------------------------------------------------
def test_each_pair_uses_the_source_core():
    """Two blobs with different cores: the velocity each induces on the other,
    and its gradient, follow from the Gaussian vorticity of the *source* blob
    alone (enclosed mass by quadrature, gradient by central differences of
    that field), not from the target's core or a mix of the two."""
    sig = np.array([0.2, 0.5])
    x = np.array([[0.0, 0.0, 0.0], [0.3, 0.1, -0.05]])
    a = np.array([[0.2, -0.4, 1.0], [0.7, 0.3, -0.6]])
    case = dict(x=x[:, 0], y=x[:, 1], z=x[:, 2], ax=a[:, 0], ay=a[:, 1], az=a[:, 2], sigma=sig, n=2)
    ref = oracle.direct(case)

    def field(p, j):  # velocity at p of blob j alone: (enclosed mass / 4 pi rho^3) alpha_j x (p - x_j)
        r = p - x[j]
        rho = np.linalg.norm(r)
        mass, _ = integrate.quad(lambda s: 4.0 * np.pi * s * s * gauss3(s, sig[j]), 0.0, rho,
                                 epsabs=0.0, epsrel=1e-13, limit=200)
        return mass / (4.0 * np.pi * rho ** 3) * np.cross(a[j], r)

    h = 1e-5
    for i, j in ((0, 1), (1, 0)):
        u = field(x[i], j)
        assert np.allclose(ref["u"][i], u, rtol=1e-10, atol=1e-14)
        # the gradient also holds the particle's own blob: zero velocity at its centre but the
        # rigid rotation omega(0)/3 there, which drops out of the stretching term
        J = np.empty((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[k] = (field(x[i] + e, j) + field(x[i] + e, i) - field(x[i] - e, j) - field(x[i] - e, i)) / (2.0 * h)
        assert np.allclose(ref["J"][i], J, rtol=1e-6, atol=1e-9 * np.abs(J).max())
        # the target's own core would give a clearly different velocity here
        other = dict(case, sigma=np.array([sig[i], sig[i]]))
        assert not np.allclose(oracle.direct(other)["u"][i], u, rtol=1e-3)
