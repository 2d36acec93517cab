"""FP64 oracle for the radial-basis-function reinitialisation of the particle
strengths (Sec. 2.1, last paragraph; Sec. 2.2; Sec. 3.4).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
library imports or calls this module.

The vorticity carried by particles of strengths gamma_j and cores sigma_j is
omega(x) = sum_j gamma_j zeta_{sigma_j}(x - x_j), with zeta the normalised
Gaussian whose enclosed mass is the cutoff g of Eq. (2).  Reinitialising
means: given the vorticity omega_i at the particle positions x_i, find the
strengths that reproduce it there,

    sum_j zeta_sigma(x_i - x_j) gamma_j = omega_i      for every i,

one linear system per vorticity component, with the same symmetric positive
definite matrix when every core is the same sigma.  Reading taken here (the
method's own reference is not available): the system is solved by plain
conjugate gradients from gamma = 0, each component separately, stopping when
||omega - A gamma|| <= tol ||omega||.

Routes
------
* ``gaussian_sum``  the matrix-vector product, a direct FP64 sum in C
                    (``gauss.c``), free space or over an explicit image list.
* ``rbf_cg``        plain conjugate gradients with that product.
* ``gaussian_lattice`` the same sum over every periodic image for strengths
                    on the cell-centred lattice with one core, by the DFT: the
                    periodic matrix is a lattice convolution, diagonal in the
                    discrete Fourier basis with eigenvalues
                    (N/V) sum_m exp(-sigma^2 |k'|^2 / 2) over the aliases
                    k' = 2 pi (kappa + n m) / L (also at shifted points).
* ``rbf_lattice``   the exact solution on that lattice: divide by them.
"""
import numpy as np

from . import _d, _lib, _p


def gaussian_sum(case, gamma, points=None, shifts=None):
    """w_i = sum_n sum_j gamma_j zeta_{sigma_j}(t_i - x_j - shift_n) in float64.

    ``case``: the particles (x, y, z, sigma); ``gamma`` (N, 3) their
    strengths; ``points`` (m, 3) the evaluation points (default: the
    particles); ``shifts`` (s, 3) image shifts (default: free space).
    Returns (m, 3)."""
    sx, sy, sz, sg = _d(case["x"]), _d(case["y"]), _d(case["z"]), _d(case["sigma"])
    g = np.asarray(gamma, dtype=np.float64).reshape(-1, 3)
    gx, gy, gz = _d(g[:, 0]), _d(g[:, 1]), _d(g[:, 2])
    if points is None:
        tx, ty, tz = sx, sy, sz
    else:
        pt = np.asarray(points, dtype=np.float64).reshape(-1, 3)
        tx, ty, tz = _d(pt[:, 0]), _d(pt[:, 1]), _d(pt[:, 2])
    if shifts is None:
        nsh, sh = 0, np.zeros(3)
    else:
        sh = _d(np.asarray(shifts, dtype=np.float64).reshape(-1, 3))
        nsh = sh.shape[0]
    out = np.empty((tx.size, 3))
    _lib().oracle_gauss_sum(tx.size, _p(tx), _p(ty), _p(tz), sx.size, _p(sx), _p(sy), _p(sz),
                            _p(gx), _p(gy), _p(gz), _p(sg), nsh, _p(sh), _p(out))
    return out


def rbf_cg(case, omega, tol=1e-10, maxiter=1000, shifts=None, matvec=None):
    """Strengths gamma with sum_j zeta(x_i - x_j) gamma_j = omega_i by plain
    conjugate gradients from gamma = 0, for each of the three components on
    its own, until ||r|| <= tol ||omega|| (r = omega - A gamma, updated
    recursively) or maxiter iterations.  The product A v is the direct sum
    (``gaussian_sum``, free space or over ``shifts``) unless ``matvec`` (a
    function of an (N, 3) array) is given, e.g. ``gaussian_lattice`` for every
    periodic image of a lattice.  Returns (gamma (N,3), iterations (3,),
    relative residual (3,))."""
    om = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    zero = np.zeros_like(om)

    if matvec is None:
        def matvec(v):
            return gaussian_sum(case, v, shifts=shifts)

    gamma = zero.copy()
    iters = np.zeros(3, dtype=np.int64)
    res = np.zeros(3)
    for c in range(3):
        b = om[:, c]
        bn = np.linalg.norm(b)
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        k = 0
        while k < maxiter and np.sqrt(rr) > tol * bn:
            v = zero.copy()
            v[:, c] = p
            Ap = matvec(v)[:, c]
            alpha = rr / (p @ Ap)
            x += alpha * p
            r -= alpha * Ap
            rr_new = r @ r
            p = r + (rr_new / rr) * p
            rr = rr_new
            k += 1
        gamma[:, c] = x
        iters[c] = k
        res[c] = np.sqrt(rr) / bn if bn > 0 else 0.0
    return gamma, iters, res


def _lattice_symbol(case, aliases, offset):
    """(N/V) sum_m exp(-sigma^2 |k'|^2 / 2) exp(i k'.delta) on the DFT grid of
    the n^3 lattice, k' = 2 pi (kappa + n m) / L, kappa centred."""
    n = int(case["lattice_n"])
    L = float(case["L"])
    sig = float(np.asarray(case["sigma"])[0])
    if aliases is None:
        aliases = max(1, int(np.ceil(9.1 / (sig * 2.0 * np.pi * n / L) - 0.5)))
    kap = np.fft.fftfreq(n, d=1.0 / n)
    kap = np.where(kap >= n // 2, kap - n, kap)
    KX, KY, KZ = np.meshgrid(kap, kap, kap, indexing="ij", sparse=True)
    tw = 2.0 * np.pi / L
    dl = np.zeros(3) if offset is None else np.asarray(offset, dtype=np.float64)
    shifted = bool(np.any(dl != 0.0))
    lam = np.zeros((n, n, n), dtype=np.complex128 if shifted else np.float64)
    rng = range(-aliases, aliases + 1)
    for mx in rng:
        for my in rng:
            for mz in rng:
                kx, ky, kz = tw * (KX + n * mx), tw * (KY + n * my), tw * (KZ + n * mz)
                f = np.exp(-0.5 * sig * sig * (kx * kx + ky * ky + kz * kz))
                if shifted:
                    f = f * np.exp(1j * (kx * dl[0] + ky * dl[1] + kz * dl[2]))
                lam = lam + f
    return lam * (n ** 3 / L ** 3)


def gaussian_lattice(case, gamma, offset=None, aliases=None):
    """The periodic blob sum of strengths on the cell-centred n^3 lattice (one
    core sigma, period L), evaluated at the lattice points shifted by
    ``offset`` (default: at the lattice points): the sum over every image is a
    lattice convolution, IDFT[Lambda_delta DFT(gamma)] with
    Lambda_delta(kappa) = (N/V) sum_m exp(-sigma^2 |k'|^2 / 2) exp(i k'.delta).
    Returns (N, 3)."""
    n = int(case["lattice_n"])
    lam = _lattice_symbol(case, aliases, offset)
    g = np.asarray(gamma, dtype=np.float64).reshape(n, n, n, 3)
    w = np.fft.ifftn(np.fft.fftn(g, axes=(0, 1, 2)) * lam[:, :, :, None], axes=(0, 1, 2))
    return np.real(w).reshape(n ** 3, 3)


def rbf_lattice(case, omega, aliases=None):
    """Exact strengths on the periodic cell-centred n^3 lattice (one core
    sigma, period L, points (i + 1/2) h flattened [i, j, k]): the periodic
    blob sum is diagonal in the DFT basis (``gaussian_lattice``), so
    gamma = IDFT[DFT(omega) / Lambda_0].  The matrix is badly conditioned for
    cores wider than the spacing (Lambda_0 falls like exp(-3 pi^2 sigma^2 /
    (2 h^2)) at the highest lattice wavevector), so rounding in omega reaches
    gamma amplified in those modes; the vorticity the strengths represent is
    unaffected.  Returns gamma (N, 3)."""
    n = int(case["lattice_n"])
    lam = _lattice_symbol(case, aliases, None)
    om = np.asarray(omega, dtype=np.float64).reshape(n, n, n, 3)
    gh = np.fft.fftn(om, axes=(0, 1, 2)) / lam[:, :, :, None]
    return np.real(np.fft.ifftn(gh, axes=(0, 1, 2))).reshape(n ** 3, 3)
