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
* ``fourier_series_points``  the series of ``fourier_points`` with each phase
                        factored over the axes (matrix products over the
                        particles): every particle of a 32^3 off-lattice set.
* ``spectral_lattice(offset=delta)``  the lattice route evaluated at the
                        lattice points shifted by delta (e.g. a probe lattice
                        at the cell corners).
* ``energy_spectrum``   shell-binned kinetic energy spectrum E(k) of a
                        velocity sampled on a uniform lattice (Sec. 4.3).
* ``heun_step``         one two-stage Runge-Kutta (Heun) step of x, alpha and
                        sigma^2 (Sec. 2.1, Eqs. (1), (3), (4)) from any rate
                        function (``direct`` or the Fourier series).
* ``gaussian_sum``, ``gaussian_lattice``, ``rbf_cg``, ``rbf_lattice`` (``rbf.py``, ``gauss.c``):
                        the Gaussian blob sum and the strengths that reproduce
                        a vorticity field at the particles (reinitialisation).

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
        if not hasattr(lib, "oracle_gauss_sum"):  # a copy built before gauss.c existed
            from . import build as _b
            _b.build()
            lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int64, dp, dp, dp,
                                      dp, dp, dp, dp, ctypes.c_int64, dp, dp, dp]
        lib.oracle_direct.restype = None
        lib.oracle_pair_factors.argtypes = [ctypes.c_int64, dp, dp, dp, dp]
        lib.oracle_pair_factors.restype = None
        lib.oracle_gauss_sum.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int64, dp, dp, dp,
                                         dp, dp, dp, dp, ctypes.c_int64, dp, dp]
        lib.oracle_gauss_sum.restype = None
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


def spectral_lattice(case, aliases=None, workers=None, offset=None):
    """Exact zero-mean periodic u and J at the n^3 cell-centred lattice
    (or, with ``offset`` = delta, at the lattice points shifted by delta).

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
    dropped (zero mean).  Returns (u (N,3), J (N,3,3)) in the input order.

    Shifted points x_t + delta: every wavevector k' picks up the phase
    exp(i k'.delta), which differs between aliases, so P and Q are summed with
    it (complex) before the inverse DFT; delta = 0 is the unshifted sum."""
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
    shifted = offset is not None and np.any(np.asarray(offset, dtype=np.float64) != 0.0)
    dl = np.asarray(offset if shifted else (0.0, 0.0, 0.0), dtype=np.float64)
    P = np.zeros((3, n, n, n), dtype=np.complex128 if shifted else np.float64)
    Q = np.zeros((6, n, n, n), dtype=P.dtype)  # xx yy zz xy xz yz
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
                if shifted:
                    w = w * np.exp(1j * (kx * dl[0] + ky * dl[1] + kz * dl[2]))
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


def fourier_series_points(case, L, kmax, points=None, chunk=2048):
    """The Fourier series of ``fourier_points`` (zero-mean periodic u and J,
    wavevectors k = 2 pi m / L with 0 < |m|_inf <= kmax, uniform sigma), summed
    with each phase written as a product over the axes,
    exp(i k.x) = exp(i k_x x) exp(i k_y y) exp(i k_z z), so that
    S(k) = sum_j alpha_j exp(-i k.x_j) and the sums at the evaluation points
    become matrix products over the particle (or point) index: the same terms,
    cheap enough for every particle of a 32^3 set.  ``points`` (m, 3) default
    to the particles.  Returns (u (m,3), J (m,3,3)), J_kl = du_l/dx_k."""
    sig = float(np.asarray(case["sigma"])[0])
    x = np.stack([_d(case["x"]), _d(case["y"]), _d(case["z"])], axis=1)
    a = np.stack([_d(case["ax"]), _d(case["ay"]), _d(case["az"])], axis=1)
    xt = x if points is None else np.asarray(points, dtype=np.float64).reshape(-1, 3)
    m = np.arange(-kmax, kmax + 1)
    K = (2.0 * np.pi / L) * m                  # wavenumbers along one axis
    M = K.size
    # S[c, a, b, d] = sum_j alpha_c,j e^{-i K_a x_j} e^{-i K_b y_j} e^{-i K_d z_j}
    S = np.zeros((3 * M, M * M), dtype=np.complex128)
    for j0 in range(0, x.shape[0], chunk):
        xs = x[j0:j0 + chunk]
        ex = np.exp(-1j * np.outer(xs[:, 0], K))
        ey = np.exp(-1j * np.outer(xs[:, 1], K))
        ez = np.exp(-1j * np.outer(xs[:, 2], K))
        T = (ey[:, :, None] * ez[:, None, :]).reshape(xs.shape[0], M * M)
        Aw = (a[j0:j0 + chunk, :, None] * ex[:, None, :]).reshape(xs.shape[0], 3 * M)
        S += Aw.T @ T
    S = S.reshape(3, M, M, M)
    KX, KY, KZ = np.meshgrid(K, K, K, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(k2 > 0, np.exp(-0.5 * sig * sig * k2) / k2, 0.0)
    V = L ** 3
    kxS = np.stack([KY * S[2] - KZ * S[1], KZ * S[0] - KX * S[2], KX * S[1] - KY * S[0]])
    Cu = 1j * kxS * w / V                      # u_l(x) = Re sum_k Cu_l(k) e^{i k.x}
    Kc = (KX, KY, KZ)
    C = [Cu[l] for l in range(3)] + [1j * Kc[k] * Cu[l] for k in range(3) for l in range(3)]
    C = np.stack(C).reshape(12, M, M * M)     # [q, a, (b, d)]
    Cm = C.transpose(0, 1, 2).reshape(12 * M, M * M)
    out = np.empty((xt.shape[0], 12))
    for t0 in range(0, xt.shape[0], chunk):
        pt = xt[t0:t0 + chunk]
        ex = np.exp(1j * np.outer(pt[:, 0], K))
        ey = np.exp(1j * np.outer(pt[:, 1], K))
        ez = np.exp(1j * np.outer(pt[:, 2], K))
        T = (ey[:, :, None] * ez[:, None, :]).reshape(pt.shape[0], M * M)
        R = (T @ Cm.T).reshape(pt.shape[0], 12, M)
        out[t0:t0 + chunk] = np.real(np.einsum("tqa,ta->tq", R, ex))
    u = out[:, :3].copy()
    J = out[:, 3:].reshape(-1, 3, 3).copy()
    return u, J


def energy_spectrum(u, n, L):
    """Shell-binned kinetic energy spectrum of a velocity field sampled on an
    n^3 uniform lattice (flattened [i, j, k], x index slowest; ``u`` (n^3, 3)):
    with u_hat(kappa) = (1/n^3) sum_t u(x_t) exp(-2 pi i kappa.t / n) (the
    Fourier coefficients of the sampled field), E(k) = 1/2 sum of |u_hat|^2
    over the integer wavevectors kappa with round(|kappa|) = k, for
    k = 0 .. round(sqrt(3) n / 2) (the lattice corner |kappa| = sqrt(3) n / 2
    rounds up).  Wavenumbers are in units of 2 pi / L (L
    does not change the values); sum_k E(k) = 1/2 mean |u|^2 (Parseval)."""
    u = np.asarray(u, dtype=np.float64).reshape(n, n, n, 3)
    uh = np.fft.fftn(u, axes=(0, 1, 2)) / float(n ** 3)
    e = 0.5 * np.sum(np.abs(uh) ** 2, axis=3)
    kap = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY, KZ = np.meshgrid(kap, kap, kap, indexing="ij")
    shell = np.rint(np.sqrt(KX * KX + KY * KY + KZ * KZ)).astype(np.int64)
    return np.bincount(shell.ravel(), weights=e.ravel(), minlength=int(np.floor(np.sqrt(3.0) * n / 2)) + 1)


def heun_step(case, dt, nu, rates, L=None, lo=(0.0, 0.0, 0.0)):
    """One step of Heun's method (the two-stage explicit trapezoidal
    Runge-Kutta rule) for the particle system of Sec. 2.1: dx/dt = u (Eq. 1),
    dalpha/dt = the stretching term (Eq. 3), d sigma^2/dt = 2 nu (Eq. 4).

    ``rates(x (N,3), alpha (N,3), sigma (N,))`` returns (u, dalpha), each
    (N,3) float64.  Stage 1 at the current state; the predictor
    x* = x + dt u, alpha* = alpha + dt dalpha, sigma*^2 = sigma^2 + 2 nu dt;
    stage 2 at the predictor; then x += dt/2 (u + u*), alpha += dt/2
    (dalpha + dalpha*), sigma^2 += 2 nu dt.  With a period L, positions are
    wrapped into [lo, lo + L) after each stage.  Returns dict(x, alpha, sigma)
    in float64."""
    x0 = np.stack([_d(case["x"]), _d(case["y"]), _d(case["z"])], axis=1)
    a0 = np.stack([_d(case["ax"]), _d(case["ay"]), _d(case["az"])], axis=1)
    s0 = _d(case["sigma"])
    lo = np.asarray(lo, dtype=np.float64)

    def wrap(x):
        return x if L is None else lo + np.mod(x - lo, L)

    u1, d1 = rates(x0, a0, s0)
    s1 = np.sqrt(s0 * s0 + 2.0 * nu * dt)
    u2, d2 = rates(wrap(x0 + dt * u1), a0 + dt * d1, s1)
    return dict(x=wrap(x0 + 0.5 * dt * (u1 + u2)), alpha=a0 + 0.5 * dt * (d1 + d2), sigma=s1)


from .rbf import gaussian_sum, gaussian_lattice, rbf_cg, rbf_lattice  # noqa: E402,F401
