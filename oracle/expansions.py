"""FP64 definitions of the spherical-harmonic expansions that carry the far
field between cells (Sec. 3.1: the multipole expansion of a cell's particles,
the local expansion of the field from far cells, and the velocity and its
gradient obtained from them), for checking the library's operators one at a
time.

TEST INFRASTRUCTURE ONLY: used by ``tests/``; the product library never
imports, links or calls anything here, and nothing here comes from the
product package.

The field is that of three Laplace potentials
    psi_k(x) = sum_j q_jk / |x - x_j|,   q_j = alpha_j / (4 pi),   k = x, y, z,
whose curl is the Biot-Savart velocity of point vortices (the far-field limit
of Eqs. (1)-(2), where the cutoff is 1).  Scaled solid harmonics
    R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n+m)!
    I_n^m(r) = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1}
(P_n^m with the Condon-Shortley phase, ``scipy.special.lpmv``), for which
    1/|x - y| = sum_{n >= 0} sum_{|m| <= n} conj(R_n^m(y)) I_n^m(x),  |y| < |x|
(the addition theorem; pinned in the tests, not assumed).  A cell of centre c
and side s carries
    multipole Mt_n^m = sum_j q_j conj(R_n^m((x_j - c)/s)),
              psi(x) = (1/s) sum Mt_n^m I_n^m((x - c)/s) away from the cell,
    local     psi(x) = (1/s) sum Lt_n^m R_n^m((x - c)/s) inside it,
with coefficients of a real field satisfying c_n^{-m} = (-1)^m conj(c_n^m).

Arrays of coefficients use the full order range: index n*n + n + m for
-n <= m <= n <= p, shape (..., (p+1)^2).
"""
import math

import numpy as np
from scipy.special import lpmv


def nfull(p):
    return (p + 1) * (p + 1)


def idx(n, m):
    return n * n + n + m


def _sph(v):
    v = np.atleast_2d(np.asarray(v, dtype=np.float64))
    r = np.sqrt(np.sum(v * v, axis=1))
    safe = np.where(r > 0, r, 1.0)
    ct = np.where(r > 0, v[:, 2] / safe, 1.0)
    phi = np.arctan2(v[:, 1], v[:, 0])
    return r, np.clip(ct, -1.0, 1.0), phi


def regular(p, v):
    """R_n^m(v) for every row of v (shape (npts, 3)): complex (npts, (p+1)^2)."""
    r, ct, phi = _sph(v)
    out = np.zeros((r.size, nfull(p)), dtype=np.complex128)
    for n in range(p + 1):
        rn = r ** n
        for m in range(0, n + 1):
            val = rn * lpmv(m, n, ct) * np.exp(1j * m * phi) / math.factorial(n + m)
            out[:, idx(n, m)] = val
            if m > 0:
                out[:, idx(n, -m)] = (-1) ** m * np.conj(val)
    return out


def irregular(p, v):
    """I_n^m(v) for every row of v (nonzero vectors): complex (npts, (p+1)^2)."""
    r, ct, phi = _sph(v)
    out = np.zeros((r.size, nfull(p)), dtype=np.complex128)
    for n in range(p + 1):
        rn = r ** (n + 1)
        for m in range(0, n + 1):
            val = math.factorial(n - m) * lpmv(m, n, ct) * np.exp(1j * m * phi) / rn
            out[:, idx(n, m)] = val
            if m > 0:
                out[:, idx(n, -m)] = (-1) ** m * np.conj(val)
    return out


def full_from_compact(c, p):
    """Coefficients stored for 0 <= m <= n only (index n(n+1)/2 + m, last axis)
    -> the full order range, by c_n^{-m} = (-1)^m conj(c_n^m)."""
    c = np.asarray(c)
    out = np.zeros(c.shape[:-1] + (nfull(p),), dtype=np.complex128)
    for n in range(p + 1):
        for m in range(n + 1):
            v = c[..., n * (n + 1) // 2 + m]
            out[..., idx(n, m)] = v
            if m > 0:
                out[..., idx(n, -m)] = (-1) ** m * np.conj(v)
    return out


def compact_from_full(c, p):
    c = np.asarray(c)
    return np.stack([c[..., idx(n, m)] for n in range(p + 1) for m in range(n + 1)], axis=-1)


def strengths(alpha):
    """q_j = alpha_j / (4 pi), shape (n, 3)."""
    return np.asarray(alpha, dtype=np.float64) / (4.0 * np.pi)


def multipole(pts, q, centre, s, p):
    """Mt[k, :] = sum_j q_jk conj(R((x_j - c)/s)): complex (3, (p+1)^2)."""
    R = regular(p, (np.asarray(pts, dtype=np.float64) - np.asarray(centre, dtype=np.float64)) / s)
    return np.asarray(q, dtype=np.float64).T @ np.conj(R)


def multipoles(pts, q, centres, sides, group, ngroups, p):
    """The multipole of every group of points about its own centre at once:
    point i belongs to group[i], whose centre and side are given per point
    (centres (n, 3), sides (n,)).  Returns complex (ngroups, 3, (p+1)^2)."""
    pts = np.asarray(pts, dtype=np.float64)
    v = (pts - np.asarray(centres, dtype=np.float64)) / np.asarray(sides, dtype=np.float64)[:, None]
    cR = np.conj(regular(p, v))
    q = np.asarray(q, dtype=np.float64)
    out = np.zeros((ngroups, 3, nfull(p)), dtype=np.complex128)
    for k in range(3):
        np.add.at(out[:, k, :], np.asarray(group), q[:, k, None] * cR)
    return out


def local_of_points(pts, q, centre, s, p):
    """Local coefficients of the field of point sources outside the sphere
    through the points x: psi(x) = sum_j q_j / |x - x_j| =
    (1/s) sum_{n <= p} Lt_n^m R_n^m((x - c)/s) + O(rest) with
    Lt_n^m = sum_j q_j conj(I_n^m((x_j - c)/s)) (the addition theorem with the
    roles of the two points exchanged)."""
    I = irregular(p, (np.asarray(pts, dtype=np.float64) - np.asarray(centre, dtype=np.float64)) / s)
    return np.asarray(q, dtype=np.float64).T @ np.conj(I)


def potential_multipole(M, centre, s, x, p):
    """psi_k(x) = (1/s) sum Mt I((x - c)/s): real (npts, 3)."""
    I = irregular(p, (np.atleast_2d(x) - np.asarray(centre, dtype=np.float64)) / s)
    return np.real(I @ np.asarray(M).T) / s


def potential_local(L, centre, s, x, p):
    """psi_k(x) = (1/s) sum Lt R((x - c)/s): real (npts, 3).  L is (3, (p+1)^2)
    for one expansion, or (npts, 3, (p+1)^2) with centre (npts, 3) and s (npts,)
    for one expansion per point."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    s = np.asarray(s, dtype=np.float64)
    sc = s[:, None] if s.ndim == 1 else s
    R = regular(p, (x - np.asarray(centre, dtype=np.float64)) / sc)
    L = np.asarray(L)
    if L.ndim == 2:
        return np.real(R @ L.T) / sc
    return np.real(np.einsum("in,ikn->ik", R, L)) / sc


_D1 = ((-2, 1.0 / 12.0), (-1, -8.0 / 12.0), (1, 8.0 / 12.0), (2, -1.0 / 12.0))


def velocity_local(L, centre, s, x, p, h=3e-3):
    """u = curl psi and J_kl = du_l/dx_k of a local expansion at the points x,
    by fourth-order central differences (step h s) of the float64 potential:
    J_kl = eps_{l n m} d_k d_n psi_m.  One expansion, or one per point as in
    potential_local.  Returns u (npts, 3), J (npts, 3, 3)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    s = np.asarray(s, dtype=np.float64)
    hh = h * s[:, None] if s.ndim == 1 else h * s
    hd = hh[:, 0] if np.ndim(hh) == 2 else hh
    e = np.eye(3)
    # H[i, k, n, m] = d_k d_n psi_m
    H = np.zeros((x.shape[0], 3, 3, 3))
    G = np.zeros((x.shape[0], 3, 3))  # G[i, n, m] = d_n psi_m
    for n in range(3):
        for a, wa in _D1:
            hs = hd[:, None] if np.ndim(hd) == 1 else hd
            G[:, n, :] += wa * potential_local(L, centre, s, x + a * hh * e[n], p) / hs
            for k in range(3):
                for b, wb in _D1:
                    H[:, k, n, :] += wa * wb * potential_local(L, centre, s, x + a * hh * e[n] + b * hh * e[k],
                                                               p) / (hs * hs)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    u = np.einsum("lnm,inm->il", eps, G)
    J = np.einsum("lnm,iknm->ikl", eps, H)
    return u, J
