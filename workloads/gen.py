"""Input generators for the vortex-particle workloads.

Every function is seeded (numpy PCG64 ``default_rng``) and returns a dict with
float32 SoA arrays ``x, y, z, ax, ay, az, sigma`` plus metadata.  Values are
drawn in float64 and rounded once to float32; consumers that need float64 (the
oracle) widen those float32 values exactly.

Workload shapes follow the paper's test conditions (Sec. 4.2): a periodic cube
of side 2*pi, particles on a uniform lattice, Gaussian cores sigma tied to the
lattice spacing.  The paper's own turbulence initial condition came from an
external spectral code that is not available; ``turbulence_case`` stands in
for it with a random-phase solenoidal field of prescribed spectrum, which is
how the paper describes constructing its validation initial conditions
(Sec. 2.2).
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def _pack(x, y, z, ax, ay, az, sigma, **meta):
    d = dict(
        x=np.ascontiguousarray(x, dtype=np.float32),
        y=np.ascontiguousarray(y, dtype=np.float32),
        z=np.ascontiguousarray(z, dtype=np.float32),
        ax=np.ascontiguousarray(ax, dtype=np.float32),
        ay=np.ascontiguousarray(ay, dtype=np.float32),
        az=np.ascontiguousarray(az, dtype=np.float32),
        sigma=np.ascontiguousarray(sigma, dtype=np.float32),
    )
    d.update(meta)
    d["n"] = int(d["x"].shape[0])
    return d


def lattice_positions(n, L=TWO_PI):
    """Cell-centred lattice (i+1/2)h, h=L/n, flattened with index order [i, j, k]
    (x index slowest).  Returns float64 arrays (x, y, z) and h."""
    h = L / n
    c = (np.arange(n, dtype=np.float64) + 0.5) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel(), h


def taylor_green_case(n=32, L=TWO_PI, core=1.5, periodic=False):
    """Plain tiny configuration: Taylor-Green vorticity sampled on an n^3 lattice.

    omega = (-cos x sin y sin z, -sin x cos y sin z, 2 sin x sin y cos z) is the
    curl of u = (sin x cos y cos z, -cos x sin y cos z, 0); strengths are
    alpha = omega(x_j) h^3 and every core is sigma = core*h."""
    x, y, z, h = lattice_positions(n, L)
    wx = -np.cos(x) * np.sin(y) * np.sin(z)
    wy = -np.sin(x) * np.cos(y) * np.sin(z)
    wz = 2.0 * np.sin(x) * np.sin(y) * np.cos(z)
    v = h ** 3
    sig = np.full(x.shape, core * h)
    return _pack(x, y, z, wx * v, wy * v, wz * v, sig, h=h, L=L, lattice_n=n,
                 periodic=periodic, box_lo=(0.0, 0.0, 0.0), kind="taylor_green")


def turbulence_case(n=128, seed=2, k0=4.0, L=TWO_PI, core=1.5):
    """Isotropic-turbulence-shaped lattice field.

    A random-phase solenoidal velocity is drawn in Fourier space with energy
    spectrum E(k) ~ k^4 exp(-2 (k/k0)^2): complex Gaussian modes projected
    onto the plane normal to k, Nyquist modes dropped, scaled so the sampled
    field has u_rms = 1.  Vorticity omega = curl u is evaluated spectrally at
    the cell centres (i+1/2)h, strengths are alpha_j = omega(x_j) h^3 with the
    float64 mean removed (a periodic vorticity field has zero mean), then
    rounded to float32.  Box [0, L)^3, cores sigma = core*h."""
    rng = np.random.default_rng(seed)
    h = L / n
    kf = np.fft.fftfreq(n, d=1.0 / n)  # integer wavenumbers, centred order
    KX, KY, KZ = np.meshgrid(kf, kf, kf, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kmag = np.sqrt(k2)
    nyq = (np.abs(KX) == n // 2) | (np.abs(KY) == n // 2) | (np.abs(KZ) == n // 2)
    xi = (rng.standard_normal((3,) + k2.shape) + 1j * rng.standard_normal((3,) + k2.shape))
    kk = np.where(k2 == 0, 1.0, k2)
    kdotxi = (KX * xi[0] + KY * xi[1] + KZ * xi[2]) / kk
    xi[0] -= KX * kdotxi
    xi[1] -= KY * kdotxi
    xi[2] -= KZ * kdotxi
    spec = kmag ** 4 * np.exp(-2.0 * (kmag / k0) ** 2)
    amp = np.sqrt(spec / (8.0 * np.pi * np.where(k2 == 0, 1.0, k2)))
    amp[(k2 == 0) | nyq] = 0.0
    uh = xi * amp
    del xi, kdotxi
    # evaluate at cell centres: phase shift by h/2 in each direction
    kw = TWO_PI / L
    shift = np.exp(1j * kw * (KX + KY + KZ) * (0.5 * h))
    u = np.real(np.fft.ifftn(uh * shift, axes=(1, 2, 3)))
    urms = np.sqrt(np.mean(np.sum(u ** 2, axis=0)) / 3.0)
    uh /= urms
    # omega_hat = i k x u_hat  (k in physical units)
    wxh = 1j * kw * (KY * uh[2] - KZ * uh[1])
    wyh = 1j * kw * (KZ * uh[0] - KX * uh[2])
    wzh = 1j * kw * (KX * uh[1] - KY * uh[0])
    del uh
    w = [np.real(np.fft.ifftn(c * shift)) for c in (wxh, wyh, wzh)]
    del wxh, wyh, wzh, shift
    v = h ** 3
    a = [(wi.ravel() * v) for wi in w]
    a = [ai - ai.mean() for ai in a]
    x, y, z, _ = lattice_positions(n, L)
    sig = np.full(x.shape, core * h)
    return _pack(x, y, z, a[0], a[1], a[2], sig, h=h, L=L, lattice_n=n,
                 periodic=True, box_lo=(0.0, 0.0, 0.0), kind="turbulence", seed=seed)


def ring_case(nb, rng, radius=1.0, core=0.1, jitter=0.02, circulation=1.0):
    """One Gaussian vortex-ring cloud in the z=0 plane, circulation Gamma.

    phi_j = 2 pi j / N, x_j = R (cos phi_j, sin phi_j, 0) + U(-jitter, jitter)^3,
    alpha_j = Gamma (2 pi R / N) (-sin phi_j, cos phi_j, 0), sigma_j = core."""
    phi = TWO_PI * np.arange(nb, dtype=np.float64) / nb
    j = rng.uniform(-jitter, jitter, size=(3, nb))
    x = radius * np.cos(phi) + j[0]
    y = radius * np.sin(phi) + j[1]
    z = j[2]
    s = circulation * TWO_PI * radius / nb
    ax = -s * np.sin(phi)
    ay = s * np.cos(phi)
    az = np.zeros(nb)
    sig = np.full(nb, core)
    return _pack(x, y, z, ax, ay, az, sig, periodic=False, kind="ring")


def ring_batch(nprob=512, seed=4, nmin=1024, nmax=65536):
    """Batch of independent free-space ring problems with log-uniform sizes.

    Returns (list_of_problem_dicts, offsets) where offsets[b] is the first
    particle of problem b in the concatenated arrays."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=nprob))).astype(np.int64)
    probs = [ring_case(int(nb), rng) for nb in sizes]
    offsets = np.zeros(nprob + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return probs, offsets


def random_cloud(n, seed=0, L=1.0, core=0.05, lo=(0.0, 0.0, 0.0), zero_mean=False, periodic=False):
    """Uniform random particles in [lo, lo+L)^3 with Gaussian-random strengths."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, L, size=(3, n)) + np.asarray(lo, dtype=np.float64)[:, None]
    a = rng.standard_normal((3, n)) * (L ** 3 / max(n, 1))
    if zero_mean:
        a -= a.mean(axis=1, keepdims=True)
    sig = np.full(n, core)
    return _pack(p[0], p[1], p[2], a[0], a[1], a[2], sig, L=L, periodic=periodic,
                 box_lo=tuple(lo), kind="random")


def clustered_cloud(n, seed=0, centres=((0.3, 0.3, 0.3), (0.7, 0.65, 0.7)), width=0.06, core=0.004):
    """Gaussian clusters of equal size (a deep, adaptive octree with sparse
    outskirts) inside the unit cube, Gaussian-random strengths."""
    rng = np.random.default_rng(seed)
    c = np.asarray(centres, dtype=np.float64)
    k = rng.integers(0, len(c), size=n)
    p = c[k] + width * rng.standard_normal((n, 3))
    p = np.clip(p, 0.02, 0.98).T
    a = rng.standard_normal((3, n)) / max(n, 1)
    sig = np.full(n, core)
    return _pack(p[0], p[1], p[2], a[0], a[1], a[2], sig, L=1.0, periodic=False, box_lo=(0.0, 0.0, 0.0),
                 kind="clusters")


def varcore_case(n=128, seed=2, core_seed=7, lo=0.75, hi=1.25):
    """``turbulence_case`` with per-particle cores: each sigma_j is the lattice
    core times an independent U(lo, hi) draw (seeded by ``core_seed``)."""
    case = turbulence_case(n, seed=seed)
    rng = np.random.default_rng(core_seed)
    out = dict(case)
    out["sigma"] = (np.asarray(case["sigma"], np.float64) * rng.uniform(lo, hi, case["n"])).astype(np.float32)
    out["kind"] = "turbulence_varcore"
    out["core_seed"] = core_seed
    return out


def graded_cores(case, amp=0.5):
    """``case`` with cores that vary smoothly across the domain, as after core
    spreading in a region of strong diffusion: sigma_j = sigma_j (1 + amp
    sin(2 pi x_j / L)), so the cores in one part of the box are up to (1+amp)
    /(1-amp) times those in another while neighbouring particles have nearly
    equal cores."""
    L = float(case["L"])
    out = dict(case)
    f = 1.0 + amp * np.sin(TWO_PI * np.asarray(case["x"], np.float64) / L)
    out["sigma"] = (np.asarray(case["sigma"], np.float64) * f).astype(np.float32)
    out["kind"] = str(case.get("kind", "")) + "_graded_cores"
    return out


def corner_lattice(n, L=TWO_PI):
    """Probe points at the cell corners i h, h = L/n (offset h/2 from the
    cell-centred particle lattice), flattened [i, j, k]; float32 (x, y, z)."""
    g = np.arange(n) * (L / n)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return tuple(np.ascontiguousarray(a.ravel(), dtype=np.float32) for a in (X, Y, Z))


def jittered(case, frac=0.4, seed=0):
    """The particles of a lattice case moved off the lattice: each coordinate
    gets an independent U(-frac h, frac h) displacement (seeded), wrapped into
    the periodic cube [0, L).  Strengths and cores are unchanged.  A value that
    rounds up to L in float32 is moved down by one float32 ulp, so every
    coordinate stays inside the cube."""
    L = float(case["L"])
    h = float(case["h"])
    rng = np.random.default_rng(seed)
    out = dict(case)
    for k in ("x", "y", "z"):
        v = np.mod(np.asarray(case[k], np.float64) + rng.uniform(-frac * h, frac * h, case["n"]), L)
        f = v.astype(np.float32)
        f = np.where(f.astype(np.float64) >= L, np.nextafter(f, np.float32(0)), f)
        out[k] = np.ascontiguousarray(f, dtype=np.float32)
    out["kind"] = str(case.get("kind", "")) + "_jittered"
    out.pop("lattice_n", None)
    out["jitter"] = (frac, seed)
    return out


def checksum(arrays):
    """Fingerprint of the given arrays, to confirm that regenerated inputs are
    the ones stored expected values were computed on: per array, the float64
    sum of |a_i| and the weighted sum of (1 + i mod 97) a_i (order-sensitive)."""
    out = []
    for a in arrays:
        a = np.asarray(a, np.float64).ravel()
        w = 1.0 + (np.arange(a.size) % 97)
        out += [float(np.sum(np.abs(a))), float(np.dot(w, a))]
    return out


def checksum_matches(a, b):
    """Whether two fingerprints from ``checksum`` agree to float64 summation rounding."""
    if len(a) != len(b):
        return False
    for k in range(0, len(a), 2):
        tol = 1e-11 * 98.0 * max(abs(a[k]), abs(b[k]), 1e-300)
        if abs(a[k] - b[k]) > tol or abs(a[k + 1] - b[k + 1]) > tol:
            return False
    return True


def case_arrays(case):
    """The seven input arrays of a case in a fixed order."""
    return [case[k] for k in ("x", "y", "z", "ax", "ay", "az", "sigma")]
