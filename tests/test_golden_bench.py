"""The stored expected values that bench.py's accuracy checks read
(tests/golden/bench_*.txt) are the FP64 oracle's, on the inputs the bench
regenerates: their input fingerprints match the seeded workloads and sampled
rows agree with the oracle recomputed here."""
import os

import numpy as np
import pytest

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read(name):
    fp, cols = None, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if not line.startswith("#"):
                break
            if line.startswith("# fingerprint"):
                fp = [float(v) for v in line.split()[2:]]
            elif line.startswith("# columns:"):
                cols = line.split()[2:]
    tab = np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)
    return fp, cols, tab[:, 0].astype(np.int64), tab[:, 1:]


def _close(a, b):
    # values are stored with 13 significant digits
    return np.allclose(a, b, rtol=1e-11, atol=1e-11 * np.abs(b).max())


@pytest.fixture(scope="module")
def c2_case():
    return wl.turbulence_case(128, seed=2)


def test_c2_reference_is_the_spectral_oracle(c2_case):
    fp, cols, idx, val = _read("bench_c2_128.txt")
    assert cols == ["index", "ux", "uy", "uz", "dax", "day", "daz"]
    assert wl.checksum_matches(fp, wl.checksum(wl.case_arrays(c2_case)))
    assert idx.size == 2048 and np.all(np.diff(idx) > 0) and idx[-1] < c2_case["n"]
    us, Js = oracle.spectral_lattice(c2_case)
    alpha = np.stack([c2_case["ax"], c2_case["ay"], c2_case["az"]], 1).astype(np.float64)
    das, _ = oracle.stretching(Js, alpha)
    assert _close(val[:, :3], us[idx]) and _close(val[:, 3:], das[idx])


def test_var_reference_is_the_direct_oracle():
    var = wl.varcore_case(128)
    fp, cols, idx, val = _read("bench_var_128.txt")
    assert cols == ["index", "ux", "uy", "uz", "dax", "day", "daz"]
    assert wl.checksum_matches(fp, wl.checksum(wl.case_arrays(var)))
    s = np.arange(0, idx.size, idx.size // 8)
    ref = oracle.direct(var, targets=idx[s])
    assert _close(val[s, :3], ref["u"]) and _close(val[s, 3:], ref["da_t"])


def test_targets_reference_is_the_direct_oracle(c2_case):
    pts = wl.corner_lattice(128)
    fp, cols, idx, val = _read("bench_targets_128.txt")
    assert cols == ["index", "ux", "uy", "uz"]
    assert wl.checksum_matches(fp, wl.checksum(wl.case_arrays(c2_case) + list(pts)))
    s = np.arange(0, idx.size, idx.size // 8)
    P = np.stack([p[idx[s]] for p in pts], 1).astype(np.float64)
    assert _close(val[s], oracle.direct_points(c2_case, P)["u"])


def test_periodic_targets_and_spectrum_references_are_the_spectral_oracle(c2_case):
    pts = wl.corner_lattice(128)
    fp, cols, idx, val = _read("bench_targets_periodic_128.txt")
    fp2, cols2, ks, E = _read("bench_spectrum_periodic_128.txt")
    assert cols == ["index", "ux", "uy", "uz"] and cols2 == ["index", "E"]
    arrays = wl.case_arrays(c2_case) + list(pts)
    assert wl.checksum_matches(fp, wl.checksum(arrays)) and wl.checksum_matches(fp2, wl.checksum(arrays))
    h = c2_case["h"]
    us, _ = oracle.spectral_lattice(c2_case, offset=(-0.5 * h, -0.5 * h, -0.5 * h))
    assert _close(val, us[idx])
    Eref = oracle.energy_spectrum(us, 128, c2_case["L"])
    assert np.array_equal(ks, np.arange(Eref.size)) and _close(E[:, 0], Eref)


def test_fingerprint_detects_other_inputs(c2_case):
    fp = wl.checksum(wl.case_arrays(c2_case))
    moved = dict(c2_case)
    moved["ax"] = np.roll(c2_case["ax"], 1)  # same values, another order
    assert not wl.checksum_matches(fp, wl.checksum(wl.case_arrays(moved)))
    assert wl.checksum_matches(fp, wl.checksum(wl.case_arrays(dict(c2_case))))


@pytest.mark.slow
@pytest.mark.parametrize("name,seed", [("bench_c3_256.txt", 3), ("bench_c5_256.txt", 5)])
def test_256_reference_is_the_spectral_oracle(name, seed):
    """Every stored row of the 256^3 workloads recomputed with the exact
    periodic sum (about a minute and 5 GB per workload)."""
    case = wl.turbulence_case(256, seed=seed)
    fp, cols, idx, val = _read(name)
    assert cols == ["index", "ux", "uy", "uz", "dax", "day", "daz"]
    assert wl.checksum_matches(fp, wl.checksum(wl.case_arrays(case)))
    assert idx.size == 2048 and np.all(np.diff(idx) > 0) and idx[-1] < case["n"]
    us, Js = oracle.spectral_lattice(case)
    us = us[idx]
    alpha = np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64)[idx]
    das, _ = oracle.stretching(Js[idx], alpha)
    del Js
    assert _close(val[:, :3], us) and _close(val[:, 3:], das)


def test_c4_reference_is_the_direct_oracle():
    probs, off = wl.ring_batch(512, seed=4)
    arrays = [np.concatenate([pr[k] for pr in probs]) for k in ("x", "y", "z", "ax", "ay", "az", "sigma")]
    fp, cols, idx, val = _read("bench_c4_rings.txt")
    assert cols == ["index", "ux", "uy", "uz", "dax", "day", "daz"]
    assert wl.checksum_matches(fp, wl.checksum(arrays))
    assert idx.size == 4 * 512 and idx[-1] < off[-1]
    for b in (0, 97, 300, 511):  # each stored row is the direct sum over its own ring only
        rows = np.nonzero((idx >= off[b]) & (idx < off[b + 1]))[0]
        assert rows.size == 4
        ref = oracle.direct(probs[b], targets=idx[rows] - off[b])
        assert _close(val[rows, :3], ref["u"]) and _close(val[rows, 3:], ref["da_t"])


def test_bench_reader_refuses_other_inputs_without_aborting(c2_case):
    """bench.py's reader gives the stored rows for the inputs they were
    computed on, and no rows (errors reported as null) for other inputs or a
    missing file."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "bench_for_test", os.path.join(os.path.dirname(GOLDEN), os.pardir, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    idx, val, what = bench.golden("bench_c2_128.txt", wl.case_arrays(c2_case))
    assert idx.size == 2048 and val.shape == (2048, 6) and "Fourier" in what
    other = dict(c2_case)
    other["sigma"] = c2_case["sigma"] * np.float32(1.01)
    idx, val, what = bench.golden("bench_c2_128.txt", wl.case_arrays(other))
    assert idx.size == 0 and what.startswith("unavailable") and bench.rel_l2(val[:, :3], val[:, :3]) is None
    idx, val, what = bench.golden("no_such_file.txt", wl.case_arrays(c2_case))
    assert idx.size == 0 and what.startswith("unavailable")
