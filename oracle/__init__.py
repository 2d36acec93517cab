"""FP64 CPU oracle for one evaluation of the regularised Biot-Savart velocity
and the vortex-stretching term (Yokota et al., Sec. 2.1, Eqs. (1)-(3)).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product library never
imports, links or calls anything here, and this package imports nothing from
the product package.

Routes
------
* ``direct``            free-space (or explicit image list) O(N^2) sum, plain
                        C/OpenMP in float64 (``direct.c``), returns u and the
                        gradient J_kl = du_l/dx_k; the stretching term of
                        Eq. (3) is a contraction of J with alpha_i.
* ``spectral_lattice``  exact periodic sum (zero-mean convention) for sources
                        and targets on the cell-centred lattice, via its
                        Fourier series: u_hat = i k x omega_hat / k^2 with the
                        Gaussian blob factor exp(-sigma^2 k^2 / 2); the sum over
                        all wavevectors is folded onto the lattice by summing
                        aliases.
* ``fourier_points``    the same Fourier series evaluated pointwise for a few
                        off-lattice particles (tiny N only).
* ``surface_term``      (1/3V) sum_j x_j x alpha_j: the difference between the
                        cube-ordered image sum and the zero-mean Fourier sum.
* ``brute_images``      cube-ordered image sum over |n|_inf <= M (tiny N).

Readings of the paper taken here (its text is silent or ambiguous):
* sign of Eq. (1): physical Biot-Savart, u = curl psi, -lap psi = omega;
* the core in Eq. (2) is the source core sigma_j;
* Eq. (3) literal form ("transpose"): dalpha_i = J_i . alpha_i, i.e.
  (dalpha_i)_k = J_kl alpha_l; the text's "omega . grad u" ("classical") is
  (dalpha_i)_l = alpha_k J_kl and is returned too;
* periodic result: the cube-ordered lattice sum equals the zero-mean Fourier
  sum plus the surface term; the library reports the zero-mean form.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int64, dp, dp, dp,
                                      dp, dp, dp, dp, ctypes.c_int64, dp, dp, dp]
        lib.oracle_direct.restype = None
        lib.oracle_pair_factors.argtypes = [ctypes.c_int64, dp, dp, dp, dp]
        lib.oracle_pair_factors.restype = None
        _LIB = lib
    return _LIB


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pair_factors(rho, sigma):
    """q(rho) and q'(rho)/rho of Eqs. (1)-(2) (float64, elementwise)."""
    rho = _d(np.atleast_1d(rho))
    sigma = _d(np.broadcast_to(sigma, rho.shape))
    q = np.empty_like(rho)
    qp = np.empty_like(rho)
    _lib().oracle_pair_factors(rho.size, _p(rho), _p(sigma), _p(q), _p(qp))
    return q, qp


def stretching(J, alpha):
    """Both readings of Eq. (3) from the gradient J[i,k,l] = du_l/dx_k.

    transpose: (dalpha)_k = sum_l J_kl alpha_l   (Eq. (3) as printed)
    classical: (dalpha)_l = sum_k alpha_k J_kl   ("omega . grad u")"""
    da_t = np.einsum("ikl,il->ik", J, alpha)
    da_c = np.einsum("ik,ikl->il", alpha, J)
    return da_t, da_c


def direct(case, targets=None, shifts=None):
    """FP64 direct sum over every source (and every shift in ``shifts``).

    ``case``: dict with float arrays x, y, z, ax, ay, az, sigma (sources; also
    the targets unless ``targets`` (an index array) selects a subset).
    Returns dict(u=(nt,3), J=(nt,3,3), da_t=(nt,3), da_c=(nt,3))."""
    sx, sy, sz = _d(case["x"]), _d(case["y"]), _d(case["z"])
    sax, say, saz = _d(case["ax"]), _d(case["ay"]), _d(case["az"])
    ssig = _d(case["sigma"])
    if targets is None:
        tx, ty, tz = sx, sy, sz
        ta = np.stack([sax, say, saz], axis=1)
    else:
        idx = np.asarray(targets, dtype=np.int64)
        tx, ty, tz = _d(sx[idx]), _d(sy[idx]), _d(sz[idx])
        ta = np.stack([sax[idx], say[idx], saz[idx]], axis=1)
    nt = tx.size
    if shifts is None:
        nsh = 0
        sh = np.zeros(3)
    else:
        sh = _d(np.asarray(shifts).reshape(-1, 3))
        nsh = sh.shape[0]
    u = np.empty((nt, 3))
    J = np.empty((nt, 3, 3))
    _lib().oracle_direct(nt, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz),
                         _p(sax), _p(say), _p(saz), _p(ssig), nsh, _p(sh), _p(u), _p(J))
    da_t, da_c = stretching(J, ta)
    return dict(u=u, J=J, da_t=da_t, da_c=da_c)


def direct_points(case, points, shifts=None):
    """FP64 direct sum of Eq. (1) at arbitrary points (velocity and gradient;
    the points carry no strength and are not sources).  ``points``: (m, 3).
    Returns dict(u=(m,3), J=(m,3,3))."""
    pts = _d(np.asarray(points, dtype=np.float64).reshape(-1, 3))
    sx, sy, sz = _d(case["x"]), _d(case["y"]), _d(case["z"])
    sax, say, saz = _d(case["ax"]), _d(case["ay"]), _d(case["az"])
    ssig = _d(case["sigma"])
    tx, ty, tz = _d(pts[:, 0]), _d(pts[:, 1]), _d(pts[:, 2])
    if shifts is None:
        nsh, sh = 0, np.zeros(3)
    else:
        sh = _d(np.asarray(shifts).reshape(-1, 3))
        nsh = sh.shape[0]
    nt = tx.size
    u = np.empty((nt, 3))
    J = np.empty((nt, 3, 3))
    _lib().oracle_direct(nt, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz),
                         _p(sax), _p(say), _p(saz), _p(ssig), nsh, _p(sh), _p(u), _p(J))
    return dict(u=u, J=J)


def image_shifts(M, L):
    """All lattice shifts n*L with |n|_inf <= M, ordered by shell."""
    r = np.arange(-M, M + 1)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    n = n[np.argsort(np.abs(n).max(axis=1), kind="stable")]
    return n.astype(np.float64) * L


def brute_images(case, M, L, targets=None):
    """Cube-ordered periodic image sum over |n|_inf <= M (tiny inputs only)."""
    return direct(case, targets=targets, shifts=image_shifts(M, L))


def surface_term(case, L):
    """(1/3V) sum_j x_j x alpha_j : cube-ordered image sum minus the zero-mean
    Fourier sum for a net-zero total strength (the dipole-layer term of a
    conditionally convergent lattice sum taken over growing cubes)."""
    x = np.stack([_d(case["x"]), _d(case["y"]), _d(case["z"])], axis=1)
    a = np.stack([_d(case["ax"]), _d(case["ay"]), _d(case["az"])], axis=1)
    return np.cross(x, a).sum(axis=0) / (3.0 * L ** 3)


def fourier_points(case, L, kmax, targets=None, points=None):
    """Zero-mean periodic velocity and gradient by the Fourier series summed
    over wavevectors k = 2 pi m / L, 0 < |m|_inf <= kmax (tiny N; uniform sigma).

    u(x) = (1/V) sum_k i k x S(k) exp(-sigma^2 k^2/2) / k^2 exp(i k.x),
    S(k) = sum_j alpha_j exp(-i k.x_j)."""
    sig = float(np.asarray(case["sigma"])[0])
    x = np.stack([_d(case["x"]), _d(case["y"]), _d(case["z"])], axis=1)
    a = np.stack([_d(case["ax"]), _d(case["ay"]), _d(case["az"])], axis=1)
    xt = x if targets is None else x[np.asarray(targets)]
    if points is not None:  # arbitrary evaluation points (m, 3)
        xt = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    r = np.arange(-kmax, kmax + 1)
    m = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    m = m[np.any(m != 0, axis=1)]
    k = (2.0 * np.pi / L) * m
    k2 = np.sum(k * k, axis=1)
    w = np.exp(-0.5 * sig * sig * k2) / k2
    S = np.exp(-1j * (k @ x.T)) @ a                       # (nk, 3)
    V = L ** 3
    kxS = np.cross(k, S)                                 # (nk, 3)
    ph = np.exp(1j * (xt @ k.T))                         # (nt, nk)
    u = np.real((ph * w) @ (1j * kxS)) / V
    # J_kl = d u_l / d x_k : multiply by i k_k
    J = np.empty((xt.shape[0], 3, 3))
    for kk in range(3):
        J[:, kk, :] = np.real((ph * (w * 1j * k[:, kk])) @ (1j * kxS)) / V
    return u, J


def spectral_lattice(case, aliases=None, workers=None):
    """Exact zero-mean periodic u and J at the n^3 cell-centred lattice.

    Sources and targets sit at x = (i+1/2) h, h = L/n, flattened [i, j, k]
    (x slowest), uniform sigma.  With A(kappa) the DFT of alpha over lattice
    indices, the value at lattice point t of the Fourier series summed over
    every wavevector k' = 2 pi (kappa + n m) / L folds into
        u(t) = IDFT[ (i/V) P(kappa) x A(kappa) ],
        P(kappa) = sum_m k' exp(-sigma^2 |k'|^2 / 2) / |k'|^2,
    and J_kl(t) = IDFT[ -(1/V) sum_ab eps_{lab} Q_ka(kappa) A_b(kappa) ],
        Q_ka(kappa) = sum_m k'_k k'_a exp(-sigma^2 |k'|^2 / 2) / |k'|^2,
    (IDFT normalised as a plain sum over kappa) with kappa centred in [-n/2, n/2) and m over {-aliases..aliases}^3 (default: enough
    folds that the first omitted Gaussian factor is below 1e-18); k'=0 is
    dropped (zero mean).  Returns (u (N,3), J (N,3,3)) in the input order."""
    import scipy.fft as sfft
    n = int(case["lattice_n"])
    L = float(case["L"])
    sig = float(np.asarray(case["sigma"])[0])
    N = n ** 3
    if aliases is None:
        # smallest fold count whose first omitted wavevector has a Gaussian
        # factor below 1e-18: sigma |k'| >= 9.1 for |kappa + n m| >= n (a + 1/2)
        aliases = max(1, int(np.ceil(9.1 / (sig * 2.0 * np.pi * n / L) - 0.5)))
    a = np.stack([_d(case["ax"]), _d(case["ay"]), _d(case["az"])], axis=0).reshape(3, n, n, n)
    A = sfft.fftn(a, axes=(1, 2, 3), workers=workers)
    del a
    kap = np.fft.fftfreq(n, d=1.0 / n)
    kap = np.where(kap >= n // 2, kap - n, kap)  # centred: [-n/2, n/2)
    tw = 2.0 * np.pi / L
    P = np.zeros((3, n, n, n))
    Q = np.zeros((6, n, n, n))  # xx yy zz xy xz yz
    KX, KY, KZ = np.meshgrid(kap, kap, kap, indexing="ij", sparse=True)
    rng = range(-aliases, aliases + 1)
    for mx in rng:
        for my in rng:
            for mz in rng:
                kx = tw * (KX + n * mx)
                ky = tw * (KY + n * my)
                kz = tw * (KZ + n * mz)
                k2 = kx * kx + ky * ky + kz * kz
                with np.errstate(divide="ignore", invalid="ignore"):
                    w = np.where(k2 > 0, np.exp(-0.5 * sig * sig * k2) / k2, 0.0)
                P[0] += kx * w
                P[1] += ky * w
                P[2] += kz * w
                Q[0] += kx * kx * w
                Q[1] += ky * ky * w
                Q[2] += kz * kz * w
                Q[3] += kx * ky * w
                Q[4] += kx * kz * w
                Q[5] += ky * kz * w
    V = L ** 3
    # u_l = (i/V) (P x A)_l
    PxA = np.stack([P[1] * A[2] - P[2] * A[1], P[2] * A[0] - P[0] * A[2], P[0] * A[1] - P[1] * A[0]])
    del P
    u = np.real(sfft.ifftn(1j * PxA * (N / V), axes=(1, 2, 3), workers=workers)).reshape(3, N).T.copy()
    del PxA
    Qm = [[Q[0], Q[3], Q[4]], [Q[3], Q[1], Q[5]], [Q[4], Q[5], Q[2]]]
    J = np.empty((N, 3, 3))
    for k in range(3):
        # (Q_k. x A)_l = eps_{lab} Q_ka A_b
        qa = [Qm[k][0], Qm[k][1], Qm[k][2]]
        QxA = [qa[1] * A[2] - qa[2] * A[1], qa[2] * A[0] - qa[0] * A[2], qa[0] * A[1] - qa[1] * A[0]]
        for l in range(3):
            J[:, k, l] = np.real(sfft.ifftn(-QxA[l] * (N / V), workers=workers)).reshape(N)
    return u, J
