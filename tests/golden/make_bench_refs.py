"""Write the expected values that bench.py's accuracy checks compare against.

Each file holds, for a seeded sample of targets of one benchmark workload, the
FP64 oracle's velocity (and stretching term, Eq. (3) in its transpose reading)
at those targets, with a fingerprint of the inputs the values were computed on.
Only the oracle computes them; bench.py reads the files and never runs the
oracle itself.

    python tests/golden/make_bench_refs.py [c2 c3 c4 c5 var targets ptargets]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def _alpha(case):
    return np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)


def _write(name, title, reference, fingerprint, idx, cols, vals):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write("# %s\n" % title)
        f.write("# reference: %s\n" % reference)
        f.write("# written by tests/golden/make_bench_refs.py (FP64 oracle only)\n")
        f.write("# fingerprint %s\n" % " ".join("%.17g" % v for v in fingerprint))
        f.write("# columns: index %s\n" % " ".join(cols))
        for i, row in zip(idx, vals):
            f.write("%d %s\n" % (i, " ".join("%.12e" % v for v in row)))
    print("wrote", path, len(idx), "rows", flush=True)


def lattice_refs(n, seed, name, count=2048, sample_seed=33):
    """Periodic lattice: exact zero-mean periodic sum by the Fourier series."""
    case = wl.turbulence_case(n, seed=seed)
    idx = np.sort(np.random.default_rng(sample_seed).choice(case["n"], size=count, replace=False))
    us, Js = oracle.spectral_lattice(case)
    das, _ = oracle.stretching(Js, _alpha(case))
    _write(name, "periodic %d^3 turbulence-shaped lattice (seed %d), %d targets drawn with seed %d"
           % (n, seed, count, sample_seed),
           "exact FP64 periodic sum (Fourier series on the lattice), zero-mean convention",
           wl.checksum(wl.case_arrays(case)), idx, ("ux", "uy", "uz", "dax", "day", "daz"),
           np.concatenate([us[idx], das[idx]], 1))


def varcore_refs(n=128, count=1024, sample_seed=71):
    """Free space, per-particle cores: FP64 direct sum at sampled particles."""
    case = wl.varcore_case(n)
    idx = np.sort(np.random.default_rng(sample_seed).choice(case["n"], size=count, replace=False))
    ref = oracle.direct(case, targets=idx)
    _write("bench_var_%d.txt" % n, "free-space %d^3 turbulence-shaped lattice (seed 2) with sigma_j = 1.5 h "
           "U(0.75, 1.25) (seed 7), %d targets drawn with seed %d" % (n, count, sample_seed),
           "FP64 direct sum over all sources, each with its own core",
           wl.checksum(wl.case_arrays(case)), idx, ("ux", "uy", "uz", "dax", "day", "daz"),
           np.concatenate([ref["u"], ref["da_t"]], 1))


def targets_refs(n=128, count=1024, sample_seed=72):
    """Free space, probe lattice at the cell corners: FP64 direct sum at sampled probes."""
    case = wl.turbulence_case(n, seed=2)
    pts = wl.corner_lattice(n)
    idx = np.sort(np.random.default_rng(sample_seed).choice(pts[0].size, size=count, replace=False))
    P = np.stack([p[idx] for p in pts], 1).astype(np.float64)
    ref = oracle.direct_points(case, P)
    _write("bench_targets_%d.txt" % n, "free-space %d^3 turbulence-shaped lattice (seed 2) and the %d^3 probe "
           "lattice at the cell corners, %d probes drawn with seed %d" % (n, n, count, sample_seed),
           "FP64 direct sum of Eq. (1) at the probe points",
           wl.checksum(wl.case_arrays(case) + list(pts)), idx, ("ux", "uy", "uz"), ref["u"])


def periodic_targets_refs(n=128, count=1024, sample_seed=73):
    """Periodic, probe lattice at the cell corners: the exact zero-mean
    periodic sum at the lattice shifted by -h/2 (Fourier series) at sampled
    probes, and the energy spectrum E(k) of that exact field at every probe."""
    case = wl.turbulence_case(n, seed=2)
    pts = wl.corner_lattice(n)
    h = case["h"]
    us, _ = oracle.spectral_lattice(case, offset=(-0.5 * h, -0.5 * h, -0.5 * h))
    idx = np.sort(np.random.default_rng(sample_seed).choice(pts[0].size, size=count, replace=False))
    fp = wl.checksum(wl.case_arrays(case) + list(pts))
    _write("bench_targets_periodic_%d.txt" % n, "periodic %d^3 turbulence-shaped lattice (seed 2) and the %d^3 probe "
           "lattice at the cell corners, %d probes drawn with seed %d" % (n, n, count, sample_seed),
           "exact FP64 zero-mean periodic sum (Fourier series at the lattice shifted by -h/2)",
           fp, idx, ("ux", "uy", "uz"), us[idx])
    E = oracle.energy_spectrum(us, n, case["L"])
    _write("bench_spectrum_periodic_%d.txt" % n, "energy spectrum of the exact velocity at every probe of the "
           "periodic %d^3 probe lattice (same inputs)" % n,
           "oracle.energy_spectrum of the exact FP64 zero-mean periodic velocity at the %d^3 probes" % n,
           fp, np.arange(E.size), ("E",), E[:, None])


def rings_refs(nprob=512, seed=4, per=4, sample_seed=74):
    """512 free-space rings: FP64 direct sum of each problem alone at a few
    sampled particles of that problem (indices into the concatenated arrays)."""
    probs, off = wl.ring_batch(nprob, seed=seed)
    rng = np.random.default_rng(sample_seed)
    idx, vals = [], []
    for b, pr in enumerate(probs):
        loc = np.sort(rng.choice(pr["n"], size=per, replace=False))
        ref = oracle.direct(pr, targets=loc)
        idx += list(off[b] + loc)
        vals.append(np.concatenate([ref["u"], ref["da_t"]], 1))
    arrays = [np.concatenate([pr[k] for pr in probs]) for k in ("x", "y", "z", "ax", "ay", "az", "sigma")]
    _write("bench_c4_rings.txt", "%d free-space Gaussian vortex rings (seed %d), %d particles of each drawn with seed %d"
           % (nprob, seed, per, sample_seed), "FP64 direct sum over the particles of the same ring",
           wl.checksum(arrays), np.asarray(idx), ("ux", "uy", "uz", "dax", "day", "daz"), np.concatenate(vals))


def main(which):
    if "c2" in which:
        lattice_refs(128, 2, "bench_c2_128.txt")
    if "c3" in which:
        lattice_refs(256, 3, "bench_c3_256.txt")
    if "c5" in which:
        lattice_refs(256, 5, "bench_c5_256.txt")
    if "c4" in which:
        rings_refs()
    if "var" in which:
        varcore_refs()
    if "targets" in which:
        targets_refs()
    if "ptargets" in which:
        periodic_targets_refs()


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3", "c4", "c5", "var", "targets", "ptargets"])
