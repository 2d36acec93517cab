"""Pins of the FP64 expansion oracle (oracle/expansions.py; Sec. 3.1) against
facts that do not come from it: closed forms of the low-order solid
harmonics (their normalisation and the Condon-Shortley phase), Laplace's
equation, the addition theorem for 1/|x - y|, convergence of a multipole
expansion to the direct potential, and the velocity and gradient of a local
expansion against the FP64 direct Biot-Savart sum of the C oracle."""
import numpy as np
import pytest

import oracle
from oracle import expansions as ex


def test_closed_forms_of_low_orders():
    rng = np.random.default_rng(1)
    v = rng.uniform(-1, 1, (20, 3))
    x, y, z = v.T
    r = np.sqrt(np.sum(v * v, 1))
    R = ex.regular(2, v)
    I = ex.irregular(1, v)
    assert np.allclose(R[:, ex.idx(0, 0)], 1.0, atol=1e-15)
    assert np.allclose(R[:, ex.idx(1, 0)], z, atol=1e-15)
    assert np.allclose(R[:, ex.idx(1, 1)], -(x + 1j * y) / 2, atol=1e-15)
    assert np.allclose(R[:, ex.idx(1, -1)], (x - 1j * y) / 2, atol=1e-15)
    assert np.allclose(R[:, ex.idx(2, 0)], (2 * z * z - x * x - y * y) / 4, atol=1e-15)
    assert np.allclose(R[:, ex.idx(2, 2)], (x + 1j * y) ** 2 / 8, atol=1e-15)
    assert np.allclose(I[:, ex.idx(0, 0)], 1 / r, rtol=1e-14)
    assert np.allclose(I[:, ex.idx(1, 0)], z / r ** 3, rtol=1e-14)
    assert np.allclose(I[:, ex.idx(1, 1)], -(x + 1j * y) / r ** 3, rtol=1e-14)


def test_addition_theorem():
    rng = np.random.default_rng(2)
    for _ in range(5):
        a = rng.standard_normal(3)
        b = rng.standard_normal(3)
        xv = 1.5 * a / np.linalg.norm(a)
        yv = 0.3 * b / np.linalg.norm(b)
        p = 30
        s = np.sum(np.conj(ex.regular(p, yv)) * ex.irregular(p, xv))
        assert abs(s.imag) < 1e-14
        assert abs(s.real - 1.0 / np.linalg.norm(xv - yv)) < 1e-13


@pytest.mark.parametrize("kind", ["regular", "irregular"])
def test_harmonics_satisfy_laplace(kind):
    rng = np.random.default_rng(3)
    v = rng.uniform(0.4, 0.9, (8, 3)) * rng.choice([-1, 1], (8, 3))
    f = getattr(ex, kind)
    p, h = 6, 1e-3
    lap = -6.0 * f(p, v)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap = lap + f(p, v + e) + f(p, v - e)
    lap /= h * h
    scale = np.abs(f(p, v)).max() + 1.0
    assert np.abs(lap).max() <= 1e-5 * scale * 1e2


def test_multipole_converges_to_the_direct_potential():
    rng = np.random.default_rng(4)
    c = np.array([0.1, -0.2, 0.3])
    s = 0.5
    pts = c + 0.5 * s * rng.uniform(-1, 1, (40, 3))
    q = rng.standard_normal((40, 3))
    xt = c + 2.0 * rng.standard_normal((30, 3))
    xt = c + (xt - c) * (1.0 / np.linalg.norm(xt - c, axis=1))[:, None] * 1.2
    ref = np.stack([np.sum(q[:, k][None, :] / np.linalg.norm(xt[:, None, :] - pts[None, :, :], axis=2), axis=1)
                    for k in range(3)], 1)
    errs = []
    for p in (2, 4, 8, 16, 24):
        M = ex.multipole(pts, q, c, s, p)
        errs.append(np.abs(ex.potential_multipole(M, c, s, xt, p) - ref).max() / np.abs(ref).max())
    # sources within 0.433 of c, targets at 1.2: each two orders gain about (0.36)^2
    for a, b in zip(errs, errs[1:]):
        assert b < a
    assert errs[-1] < 1e-9
    # the compact storage round trip
    Mc = ex.compact_from_full(ex.multipole(pts, q, c, s, 8), 8)
    assert np.allclose(ex.full_from_compact(Mc, 8), ex.multipole(pts, q, c, s, 8), atol=1e-14)


def test_local_expansion_velocity_and_gradient_match_direct_biot_savart():
    """Far point vortices (tiny cores, so the cutoff of Eq. (2) is 1) seen from
    points near c: u and du_l/dx_k from the local expansion of the three
    potentials equal the FP64 direct sum of the C oracle."""
    rng = np.random.default_rng(5)
    c = np.array([0.2, 0.1, -0.1])
    s = 1.0  # targets within 0.52 s of c, as in a cell (|x - c| / s <= sqrt(3)/2)
    ns, nt = 25, 12
    d = rng.standard_normal((ns, 3))
    src = c + 3.0 * d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(1.0, 1.5, (ns, 1))
    tgt = c + 0.3 * rng.uniform(-1, 1, (nt, 3))
    alpha = rng.standard_normal((ns, 3))
    p = 22
    L = ex.local_of_points(src, ex.strengths(alpha), c, s, p)
    u, J = ex.velocity_local(L, c, s, tgt, p)
    pos = np.concatenate([src, tgt])
    al = np.concatenate([alpha, np.zeros((nt, 3))])
    case = dict(x=pos[:, 0], y=pos[:, 1], z=pos[:, 2], ax=al[:, 0], ay=al[:, 1], az=al[:, 2],
                sigma=np.full(ns + nt, 1e-4))
    ref = oracle.direct(case, targets=np.arange(ns, ns + nt))
    assert np.abs(u - ref["u"]).max() <= 1e-10 * np.abs(ref["u"]).max()
    assert np.abs(J - ref["J"]).max() <= 1e-8 * np.abs(ref["J"]).max()


def test_vectorised_forms_agree_with_the_single_cell_forms():
    rng = np.random.default_rng(6)
    p = 6
    pts = rng.uniform(0, 1, (50, 3))
    q = rng.standard_normal((50, 3))
    group = rng.integers(0, 4, 50)
    cen = rng.uniform(0, 1, (4, 3))
    side = rng.uniform(0.5, 1.5, 4)
    M = ex.multipoles(pts, q, cen[group], side[group], group, 4, p)
    for g in range(4):
        sel = group == g
        assert np.allclose(M[g], ex.multipole(pts[sel], q[sel], cen[g], side[g], p), atol=1e-13)
    L = ex.local_of_points(pts[:5] + 5.0, q[:5], cen[0], side[0], p)
    x = cen[0] + 0.2 * rng.uniform(-1, 1, (7, 3))
    one = ex.potential_local(L, cen[0], side[0], x, p)
    many = ex.potential_local(np.broadcast_to(L, (7,) + L.shape), np.broadcast_to(cen[0], (7, 3)),
                              np.full(7, side[0]), x, p)
    assert np.allclose(one, many, rtol=1e-14, atol=0)
    u1, J1 = ex.velocity_local(L, cen[0], side[0], x, p)
    u2, J2 = ex.velocity_local(np.broadcast_to(L, (7,) + L.shape), np.broadcast_to(cen[0], (7, 3)),
                               np.full(7, side[0]), x, p)
    assert np.allclose(u1, u2, rtol=1e-9, atol=0) and np.allclose(J1, J2, rtol=1e-7, atol=0)
