"""Benchmark: one FMM step (fmm_build + fmm_evaluate: velocity and stretching)
of the 128^3-particle periodic turbulence-shaped lattice at p = 10,
theta = 0.5, on one MI355X.

Prints ONE JSON line.  ``value`` is the whole-step P2P pair-interaction
throughput (P2P pairs per step / wall time per step, inputs resident in HBM);
``ms_per_step`` is the FMM step time.  The P2P kernel's own rate, the phase
split, the accuracy against the exact FP64 periodic sum, the roofline of the
dominant kernel (P2P, ALU-bound) and the FP64 oracle timed on the host cores
ride along in the same line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM step time & P2P Gpair-interactions/s at 128^3 particles, p=10, ≤1e-4 err"
PEAK_FP32_MFMA_TFLOPS = 157.3        # published dense FP32 matrix-core peak of MI355X (the M2L products)
PEAK_BF16_MFMA_TFLOPS = 2500.0       # published dense bf16 matrix-core peak of MI355X (split-product M2L)
PEAK_FP32_VALU_TFLOPS = 157.3        # published FP32 vector peak of MI355X (256 CU, 2.4 GHz); non-packed FMA with
                                      # vector-register operands reaches 84-94% of it, a run of FMAs that each read a
                                      # scalar register or share a register bank half that
FLOPS_PER_PAIR = 59                   # gfx950 ISA of the P2P pair body (s >= 1 form): 24 FMA + 6 MUL + 3 SUB + 2 TRANS, FMA = 2
PAPER_FLOPS_PER_PAIR = 174            # Table 1 convention (70 + 104)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="lattice points per axis")
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--ncrit", type=int, default=64)
    ap.add_argument("--ncrit-c4", type=int, default=384,
                    help="leaf size of the ring batch: a ring's leaves hold a short arc, so larger leaves are "
                         "needed to fill the 64-lane P2P waves (a sweep over 128..1024 measured 384 fastest)")
    ap.add_argument("--images", type=int, default=6)
    ap.add_argument("--kahan", type=int, default=0)
    ap.add_argument("--m2l-form", type=int, default=None, help="batched-M2L products (library default if not given)")
    ap.add_argument("--overlap", type=int, default=None, help="evaluation order (library default if not given)")
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy check against stored FP64 oracle values")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-overlap-pass", action="store_true",
                    help="skip the extra timings of the two-stream (overlap = 1) step and of the tuned settings "
                         "(profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "var", "targets", "rbf"],
                    help="c2: 128^3 periodic step (default, the headline line); c3: 256^3 float32 vs "
                         "mixed vs float64 forms; c4: 512 batched ring problems vs sequential; c5: 256^3 "
                         "autotuned RK2 step; var: 128^3 free space with per-particle cores vs uniform; targets: "
                         "128^3 particles and a 128^3 probe lattice; rbf: 128^3 reinitialisation of the strengths")
    ap.add_argument("--microbench", action="store_true",
                    help="only measure VALU FP32 FMA / exp2 / rsq issue rates and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for HBM bytes) and exit")
    return ap.parse_args()


def kernel_hash(names=("p2p.hip", "cutoff_fits.h", "common.h")):
    """Hash of the sources a kernel is compiled from (default: the P2P kernel's)."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1106_5273_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def golden(name, arrays):
    """Stored FP64 oracle values at a seeded sample of targets of a workload
    (``tests/golden/<name>``, written by ``tests/golden/make_bench_refs.py``):
    returns (indices, values, reference).  A missing file, or one computed on
    other inputs than the regenerated ones, gives no rows and says why (the
    errors are then reported as null)."""
    import numpy as np
    import workloads as wl
    path = os.path.join(ROOT, "tests", "golden", name)
    none = (np.zeros(0, np.int64), np.zeros((0, 6)))
    ref, fp = "", None
    try:
        with open(path) as f:
            for line in f:
                if not line.startswith("#"):
                    break
                if line.startswith("# reference:"):
                    ref = line.split(":", 1)[1].strip()
                elif line.startswith("# fingerprint"):
                    fp = [float(v) for v in line.split()[2:]]
        tab = np.loadtxt(path, comments="#", ndmin=2)
    except (OSError, ValueError) as e:
        return none + ("unavailable: %s" % e,)
    if fp is None or not wl.checksum_matches(fp, wl.checksum(arrays)):
        return none + ("unavailable: %s was computed on other inputs than this workload's" % path,)
    return tab[:, 0].astype(np.int64), tab[:, 1:], ref


def rel_l2(a, b):
    import numpy as np
    if b.size == 0:
        return None
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def m2l_object(st, ms, p):
    """Roofline figures of the batched M2L kernel.  Algorithmic work: 6 (p+1)^4
    flops per translation (three potentials, complex products of (p+1)^2 / 2
    coefficients).  Float32 and split-product (six bf16 products per float32
    product) forms are priced in float32-equivalent flops against the float32
    matrix peak; the three-product form is not float32-accurate, so its
    issued bf16 products are priced against the bf16 matrix peak."""
    alg = st["m2l_entries"] * 6 * (p + 1) ** 4 / (ms * 1e-3) / 1e12
    split = st["m2l_split"]
    o = {"kernel": "k_m2lb_x6" if split else "k_m2lb", "translations": st["m2l_entries"], "ms": ms,
         "flops_per_translation": 6 * (p + 1) ** 4}
    if split == 2:
        o.update(products="reduced-precision split bfloat16 (three bf16 products per float32 product)",
                 issued_bf16_tflops=3 * alg, achieved=3 * alg, peak=PEAK_BF16_MFMA_TFLOPS, unit="TFLOP/s",
                 frac=3 * alg / PEAK_BF16_MFMA_TFLOPS)
    else:
        o.update(products="split bfloat16 (six bf16 products per float32 product)" if split else "float32",
                 issued_bf16_tflops=6 * alg if split else None, bf16_peak=PEAK_BF16_MFMA_TFLOPS,
                 achieved=alg, peak=PEAK_FP32_MFMA_TFLOPS, unit="TFLOP/s", frac=alg / PEAK_FP32_MFMA_TFLOPS)
    return o


def traffic_from_profile(pairs_per_launch):
    """HBM bytes per P2P launch from committed rocprofv3 counter summaries,
    valid only for the kernel source they were taken with."""
    path = os.path.join(ROOT, "profiles", "p2p_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("p2p_source_sha256_16") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _omp_threads(k):
    """Sets the OpenMP thread count of the host process (the oracle's C code is
    OpenMP) through libgomp; returns False where libgomp cannot be loaded."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return False
    gomp.omp_set_num_threads(int(k))
    return True


def cpu_baseline(case, seconds):
    """FP64 direct oracle on a bounded sample: random targets against all
    sources of the central box, on every host core, in growing chunks until
    about `seconds` of CPU work have been timed; then a smaller sample on one
    core.  Also the full N^2 time these rates imply at 128^3 and 256^3."""
    import numpy as np

    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = case["n"]
    order = np.random.default_rng(123).permutation(n)
    oracle.direct(case, targets=order[:4])  # load the library, fault in the inputs

    def timed_sample(start, budget):
        done, chunk, dt = 0, 16, 0.0
        while dt < budget and start + done < n:
            idx = order[start + done:start + done + chunk]
            t0 = time.perf_counter()
            oracle.direct(case, targets=idx)
            el = time.perf_counter() - t0
            dt += el
            done += len(idx)
            if el < 0.25 * budget:
                chunk *= 2
        return done, dt

    done, dt = timed_sample(0, seconds)
    rate = done * n / dt
    res = {"value": rate / 1e9, "unit": "Gpair/s", "cores": cores, "kind": "oracle",
           "sample": "%d random targets x %d sources of the central box (free-space FP64 direct sum), %.1f s"
                     % (done, n, dt),
           "full_n2_seconds_128cubed": float(128 ** 3) ** 2 / rate,
           "full_n2_seconds_256cubed": float(256 ** 3) ** 2 / rate}
    if _omp_threads(1):
        d1, t1 = timed_sample(done, max(2.0, seconds / 4))
        _omp_threads(cores)
        r1 = d1 * n / t1
        res["single_core"] = {"value": r1 / 1e9, "unit": "Gpair/s", "cores": 1,
                              "sample": "%d further targets x %d sources, %.1f s" % (d1, n, t1),
                              "full_n2_seconds_128cubed": float(128 ** 3) ** 2 / r1,
                              "full_n2_seconds_256cubed": float(256 ** 3) ** 2 / r1}
    return res


def _line(metric, value, unit, ms, args, workload, extra, higher=True):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
         "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
         "data": "synthetic", "config": {"workload": workload}}
    d.update(extra)
    return d


def bench_batched(args, vf, wl):
    """512 independent free-space ring problems: one forest build + one
    evaluation (replayed as a hipGraph) against 512 separate build+evaluate
    calls on the same GPU."""
    import numpy as np
    import torch
    probs, off = wl.ring_batch(512, seed=4)
    cat = {k: np.concatenate([p[k] for p in probs]) for k in ("x", "y", "z", "ax", "ay", "az", "sigma")}
    t = tuple(torch.from_numpy(cat[k]).cuda() for k in ("x", "y", "z", "ax", "ay", "az", "sigma"))
    n = int(off[-1])
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    res = {}
    with torch.cuda.stream(st):
        out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(6))
        ctx = vf.Context(p=8, ncrit=args.ncrit_c4, use_graph=1, stream=st)
        ctx.build_batched(off, t[0], t[1], t[2], t[6])
        for _ in range(args.warmup):
            ctx.evaluate(*t, out=out)
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.evaluate(*t, out=out)
        st.synchronize()
        res["batched_evaluate_graph_ms"] = (time.perf_counter() - t0) * 1e3 / args.steps
        batched_out = [o.cpu().numpy().astype(np.float64) for o in out]
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.build_batched(off, t[0], t[1], t[2], t[6])
        st.synchronize()
        res["batched_build_ms"] = (time.perf_counter() - t0) * 1e3 / args.steps
        stats = ctx.stats()
        ctx.close()
        # sequential: one context, 512 build+evaluate calls on slices
        ctx = vf.Context(p=8, ncrit=args.ncrit_c4, stream=st)
        views = [tuple(x[off[b]:off[b + 1]] for x in t) for b in range(len(probs))]
        outs = [tuple(o[off[b]:off[b + 1]] for o in out) for b in range(len(probs))]
        for v, o in zip(views[:8], outs[:8]):
            ctx.build(v[0], v[1], v[2], v[6])
            ctx.evaluate(*v, out=o)
        st.synchronize()
        t0 = time.perf_counter()
        for v, o in zip(views, outs):
            ctx.build(v[0], v[1], v[2], v[6])
            ctx.evaluate(*v, out=o)
        st.synchronize()
        res["sequential_build_evaluate_ms"] = (time.perf_counter() - t0) * 1e3
        ctx.close()
    if not args.no_check:
        idx, ref, what = golden("bench_c4_rings.txt", [cat[k] for k in ("x", "y", "z", "ax", "ay", "az", "sigma")])
        seq_out = [o.cpu().numpy().astype(np.float64) for o in out]
        for name, o in (("batched", batched_out), ("sequential", seq_out)):
            u = np.stack(o[:3], 1)[idx]
            da = np.stack(o[3:], 1)[idx]
            res["rel_l2_%s_vs_oracle_%d" % (name, idx.size)] = {"u": rel_l2(u, ref[:, :3]),
                                                               "dalpha": rel_l2(da, ref[:, 3:])}
        res["oracle_reference"] = what
    total = res["batched_build_ms"] + res["batched_evaluate_graph_ms"]
    line = _line("512 ring problems, build+evaluate throughput", n / (total * 1e-3) / 1e6, "Mparticles/s", total, args,
                 "512 free-space Gaussian vortex rings, N log-uniform in [1024, 65536], p=8, ncrit=%d, "
                 "batched forest" % args.ncrit_c4,
                 {"p2p_pairs": stats["p2p_pairs"], "n": n, "m2l_entries": stats["m2l_entries"],
                  "m2l_groups": stats["m2l_groups"], "p2p_blocks": stats["p2p_blocks"], "speedup_vs_sequential":
                  res["sequential_build_evaluate_ms"] / total, **res})
    print(json.dumps(line), flush=True)


def bench_rk(args, vf, wl):
    """256^3 periodic lattice: autotune (p, theta, ncrit) under rel-L2 <= 1e-4,
    then time Heun RK2 steps (two builds + evaluations each)."""
    import numpy as np
    import torch
    n1 = args.n if args.n != 128 else 256
    case = wl.turbulence_case(n1, seed=5)
    t = [x.clone() for x in vf.case_to_device(case)]
    ctx = vf.Context(p=10, periodic=1, box_len=2 * np.pi, images=args.images)
    tune = ctx.autotune(*t, max_rel_l2=1e-4)
    h = 2 * np.pi / n1
    ctx.build(t[0], t[1], t[2], t[6])
    u = ctx.evaluate(*t)
    umax = float(torch.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2).max())
    acc = None
    if not args.no_check:  # the first stage's evaluation with the tuned settings
        idx, ref, what = golden("bench_c5_%d.txt" % n1, wl.case_arrays(case))
        uu = np.stack([o.cpu().numpy() for o in u[:3]], 1).astype(np.float64)[idx]
        dd = np.stack([o.cpu().numpy() for o in u[3:]], 1).astype(np.float64)[idx]
        acc = {"rel_l2_u": rel_l2(uu, ref[:, :3]), "rel_l2_dalpha": rel_l2(dd, ref[:, 3:]), "targets": int(idx.size),
               "reference": what}
    dt = 0.25 * h / umax
    for _ in range(args.warmup):
        ctx.rk_step(dt, 0.0, *t)
    torch.cuda.synchronize()
    ph = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.rk_step(dt, 0.0, *t)
        ph.append(ctx.timings())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    phases = {k: float(np.mean([p[k] for p in ph])) for k in ph[0]}
    # the tree statistics describe the last build (the step's second stage);
    # both stages are off the lattice after the warm-up steps, so twice its
    # pair count estimates the pairs of one step
    pairs2 = ctx.stats()["p2p_pairs"]
    gps = 2 * pairs2 / (phases["p2p_ms"] * 1e-3)
    line = _line("RK2 step time at 256^3 (autotuned)", ms / 1e3, "s/step", ms, args,
                 "periodic 256^3 turbulence-shaped lattice, Heun RK2 (2 x build+evaluate), autotuned",
                 {"tune": tune, "dt": dt, "stage1_accuracy": acc,
                  "step_phases_ms": phases, "phases_note": "summed over the two stages of a step",
                  "p2p_pairs_last_stage": pairs2, "p2p_gpair_s_estimate": gps / 1e9,
                  "p2p_frac_estimate": gps * FLOPS_PER_PAIR / 1e12 / PEAK_FP32_VALU_TFLOPS},
                 higher=False)
    print(json.dumps(line), flush=True)


def bench_precision(args, vf, wl):
    """256^3 periodic lattice, p = 10: the float32, mixed and float64 forms of
    the same tree.  Reports each form's step time, its difference from the
    float64 form (rounding error) and its error against the exact periodic sum
    on 2,048 random targets (stored oracle values)."""
    import numpy as np
    import torch
    n1 = args.n if args.n != 128 else 256
    case = wl.turbulence_case(n1, seed=3)
    t = vf.case_to_device(case)
    outs, res = {}, {}
    for prec, name in ((2, "fp64"), (0, "fp32"), (1, "mixed")):
        ctx = vf.Context(p=args.p, theta=args.theta, ncrit=args.ncrit, periodic=1, box_len=2 * np.pi,
                         images=args.images, precision=prec)
        out = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))
        steps = 1 if prec == 2 else args.steps
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t, out=out)
        torch.cuda.synchronize()
        ph = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.build(t[0], t[1], t[2], t[6])
            ctx.evaluate(*t, out=out)
            ph.append(ctx.timings())
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st = ctx.stats()
        ctx.close()
        outs[name] = (np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64),
                      np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64))
        res[name] = {"ms_per_step": ms, "steps": steps,
                     "phases_ms": {k: float(np.mean([p[k] for p in ph])) for k in ph[0]}}
        print("precision %s: %.1f ms/step" % (name, ms), file=sys.stderr, flush=True)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    u64, d64 = outs["fp64"]
    for name in ("fp32", "mixed"):
        res[name]["rel_l2_vs_fp64_form"] = {"u": rel(outs[name][0], u64), "dalpha": rel(outs[name][1], d64)}
    if not args.no_check:
        idx, ref, what = golden("bench_c3_%d.txt" % n1, wl.case_arrays(case))
        for name in ("fp64", "fp32", "mixed"):
            res[name]["rel_l2_vs_oracle_%d" % idx.size] = {"u": rel_l2(outs[name][0][idx], ref[:, :3]),
                                                           "dalpha": rel_l2(outs[name][1][idx], ref[:, 3:])}
        res["oracle_reference"] = what
    ms = res["fp32"]["ms_per_step"]
    line = _line("precision forms at %d^3: step time and rounding error" % n1, st["p2p_pairs"] / (ms * 1e-3) / 1e9,
                 "Gpair/s", ms, args,
                 "periodic %d^3 turbulence-shaped lattice (seed 3), p=%d, theta=%g, images=%d; float32 / mixed / "
                 "float64 forms of one tree" % (n1, args.p, args.theta, args.images),
                 {"p2p_pairs": st["p2p_pairs"], "forms": res})
    print(json.dumps(line), flush=True)


def bench_varcore(args, vf, wl):
    """Per-particle cores (Eq. 2 with each source's own sigma_j): the 128^3
    turbulence-shaped lattice in free space with sigma_j = 1.5 h U(0.75, 1.25),
    against the same particles with the uniform core, and with cores graded
    across the box (1.5 h (1 + 0.5 sin x)), where each source cell's own
    largest core sets its core gap.  Reports the step times and the error of
    the per-particle run on 1,024 random targets against the float64 direct
    sum."""
    import numpy as np
    import torch
    case = wl.turbulence_case(args.n, seed=2)
    var = wl.varcore_case(args.n)
    graded = wl.graded_cores(case, 0.5)
    res, outs = {}, {}
    for name, c in (("uniform", case), ("per_particle", var), ("graded", graded)):
        t = vf.case_to_device(c)
        ctx = vf.Context(p=args.p, theta=args.theta, ncrit=args.ncrit, periodic=0, box_len=2 * np.pi)
        out = tuple(torch.empty(c["n"], dtype=torch.float32, device="cuda") for _ in range(6))
        for _ in range(max(args.warmup, 1)):
            ctx.build(t[0], t[1], t[2], t[6])
            ctx.evaluate(*t, out=out)
        torch.cuda.synchronize()
        ph = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.build(t[0], t[1], t[2], t[6])
            ctx.evaluate(*t, out=out)
            ph.append(ctx.timings())
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        st = ctx.stats()
        ctx.close()
        outs[name] = (np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64),
                      np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64))
        res[name] = {"ms_per_step": ms, "p2p_pairs": st["p2p_pairs"], "sigma_min": st["sigma_min"],
                     "sigma_max": st["sigma_max"],
                     "phases_ms": {k: float(np.mean([p[k] for p in ph])) for k in ph[0]}}
        print("%s cores: %.1f ms/step" % (name, ms), file=sys.stderr, flush=True)
    if not args.no_check:
        idx, ref, what = golden("bench_var_%d.txt" % args.n, wl.case_arrays(var))
        res["per_particle"]["rel_l2_vs_oracle_%d" % idx.size] = {
            "u": rel_l2(outs["per_particle"][0][idx], ref[:, :3]),
            "dalpha": rel_l2(outs["per_particle"][1][idx], ref[:, 3:]), "reference": what}
    r = res["per_particle"]
    line = _line("per-particle cores at %d^3: step time" % args.n, r["p2p_pairs"] / (r["ms_per_step"] * 1e-3) / 1e9,
                 "Gpair/s", r["ms_per_step"], args,
                 "free-space %d^3 turbulence-shaped lattice (root cube [0, 2 pi)^3), sigma_j = 1.5 h U(0.75, 1.25) "
                 "(seed 7), p=%d, theta=%g; the same particles with the uniform core beside it" % (args.n, args.p, args.theta),
                 {"forms": res, "slowdown_vs_uniform": r["ms_per_step"] / res["uniform"]["ms_per_step"]})
    print(json.dumps(line), flush=True)


def bench_targets(args, vf, wl):
    """Velocity on a probe lattice that is not the particle lattice: the
    128^3 turbulence-shaped particles in free space and 128^3 probe points at
    the cell corners (offset h/2), one tree over both; against the particles
    alone.  Error on 1,024 random probes against the float64 direct sum."""
    import numpy as np
    import torch
    case = wl.turbulence_case(args.n, seed=2)
    pts = list(wl.corner_lattice(args.n))
    t = vf.case_to_device(case)
    T = [torch.tensor(p, device="cuda") for p in pts]
    res = {}

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    # root cube = bounding cube: a cube aligned with the particle lattice would put every probe on a
    # cell face, where float32 rounding of the keys moves some probes into the neighbouring cell
    ctx = vf.Context(p=args.p, theta=args.theta, ncrit=args.ncrit, periodic=0)
    out = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))
    res["particles_only_ms_per_step"] = timed(lambda: (ctx.build(t[0], t[1], t[2], t[6]), ctx.evaluate(*t, out=out)))
    ctx.close()
    # the tree holds two points (a particle and a probe) per lattice cell: leaves of 2 ncrit points
    ctx = vf.Context(p=args.p, theta=args.theta, ncrit=2 * args.ncrit, periodic=0)
    outt = tuple(torch.empty(case["n"] if k < 6 else pts[0].size, dtype=torch.float32, device="cuda")
                 for k in range(9))

    def step():
        ctx.build_targets(t[0], t[1], t[2], t[6], *T)
        ctx.evaluate_targets(t[3], t[4], t[5], out=outt)

    ms = timed(step)
    st = ctx.stats()
    res["with_targets_ms_per_step"] = ms
    res["p2p_pairs"] = st["p2p_pairs"]
    res["phases_ms"] = ctx.timings()
    ctx.close()
    if not args.no_check:
        idx, ref, what = golden("bench_targets_%d.txt" % args.n, wl.case_arrays(case) + pts)
        tu = np.stack([o.cpu().numpy() for o in outt[6:9]], 1).astype(np.float64)[idx]
        res["rel_l2_u_targets_vs_oracle_%d" % idx.size] = rel_l2(tu, ref)
        res["oracle_reference"] = what
    # periodic: the same particles and probes in the periodic cube, and the
    # energy spectrum of the probe velocities
    # the periodic cube starts a quarter spacing below 0, so that neither the particles ((i + 1/2) h) nor the
    # probes (i h) sit on an octree face: every leaf then holds both points of each of its lattice cells
    q = -0.25 * case["h"]
    ctx = vf.Context(p=args.p, theta=args.theta, ncrit=2 * args.ncrit, periodic=1, box_len=2 * np.pi,
                     box_lo=(q, q, q), images=args.images)
    ms_p = timed(step)
    st = ctx.stats()
    E = None

    def spectrum():
        nonlocal E
        E = ctx.energy_spectrum(args.n, *outt[6:9])

    ms_e = timed(spectrum)
    per = {"ms_per_step": ms_p, "p2p_pairs": st["p2p_pairs"], "phases_ms": ctx.timings(),
           "energy_spectrum_ms": ms_e, "energy_spectrum_shells_1_to_12": [float(v) for v in E[1:13]]}
    ctx.close()
    if not args.no_check:
        idx, ref, what = golden("bench_targets_periodic_%d.txt" % args.n, wl.case_arrays(case) + pts)
        tu = np.stack([o.cpu().numpy() for o in outt[6:9]], 1).astype(np.float64)[idx]
        per["rel_l2_u_targets_vs_oracle_%d" % idx.size] = rel_l2(tu, ref)
        per["oracle_reference"] = what
        ks, Eref, what = golden("bench_spectrum_periodic_%d.txt" % args.n, wl.case_arrays(case) + pts)
        if Eref.size:
            Eref = Eref[:, 0]
            per["energy_spectrum_max_shell_error_vs_oracle"] = float(np.max(np.abs(E - Eref) / (Eref + 1e-30 * Eref.sum())
                                                                     * (Eref > 1e-8 * Eref.sum())))
            per["energy_spectrum_total_vs_oracle"] = float(E.sum() / Eref.sum() - 1.0)
    res["periodic"] = per
    m = pts[0].size
    line = _line("velocity at %d^3 probe points beside %d^3 particles: step time" % (args.n, args.n),
                 m / (ms * 1e-3) / 1e6, "Mtargets/s", ms, args,
                 "free-space %d^3 turbulence-shaped lattice with a %d^3 probe lattice at the cell corners, p=%d, "
                 "theta=%g, ncrit=%d (particles and probes); one tree over both, against the particles alone; "
                 "the periodic cube with the energy spectrum of the probe velocities beside it"
                 % (args.n, args.n, args.p, args.theta, 2 * args.ncrit), res)
    print(json.dumps(line), flush=True)


GAUSS_FLOPS_PER_PAIR = 15  # gfx950 ISA of the Gaussian-sum pair body: 3 SUB + 1 MUL + 5 FMA (x2) + 1 EXP2


def bench_rbf(args, vf, wl):
    """Radial-basis-function reinitialisation of the strengths on the 128^3
    periodic turbulence-shaped lattice (sigma = 1.5h): the tree built once with
    core-overlap gap 6, then conjugate gradients to a relative residual of
    1e-4 from omega = alpha / h^3, each product a Gaussian-sum pass over the
    near-field lists.  The residual is the solver's own (the parity tests check
    the true residual with the FP64 periodic operator)."""
    import numpy as np
    import torch
    L = 2 * np.pi
    case = wl.turbulence_case(args.n, seed=2)
    t = vf.case_to_device(case)
    h = case["h"]
    om = [torch.from_numpy((np.asarray(case[k], np.float64) / h ** 3).astype(np.float32)).cuda()
          for k in ("ax", "ay", "az")]
    ctx = vf.Context(p=args.p, theta=args.theta, ncrit=args.ncrit, sigma_gap=6.0, periodic=1, box_len=L,
                     images=args.images)
    ctx.build(t[0], t[1], t[2], t[6])
    g = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(3))
    for _ in range(max(1, args.warmup)):
        ctx.rbf_reinit(*om, tol=1e-4, maxiter=200, out=g)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(ctx.rbf_reinit(*om, tol=1e-4, maxiter=200, out=g)[1])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    info = infos[-1]
    mv = float(np.mean([i["matvec_ms"] / max(1, i["matvecs"]) for i in infos]))
    pairs = info["pairs"]
    ach = pairs * GAUSS_FLOPS_PER_PAIR / (mv * 1e-3) / 1e12
    ctx.close()
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "gaussian_sum_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tj = json.load(f)
        if tj.get("source_sha256_16") == kernel_hash(("rbf.hip", "common.h")):
            traffic = tj.get("hbm_bytes_per_launch")
    res = {"iterations": list(info["iterations"]), "residual": list(info["residual"]), "gaussian_sums": info["matvecs"],
           "pairs_per_sum": pairs, "gaussian_sum_kernel_ms": mv, "gaussian_sum_gpair_s": pairs / (mv * 1e-3) / 1e9,
           "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_FP32_VALU_TFLOPS, "traffic": traffic, "kernel": "k_gauss",
                        "flops_per_pair": GAUSS_FLOPS_PER_PAIR}}
    line = _line("RBF reinitialisation of %d^3 strengths to 1e-4 residual: time per solve" % args.n,
                 case["n"] / (ms * 1e-3) / 1e6, "Mparticles/s", ms, args,
                 "periodic %d^3 turbulence-shaped lattice, sigma=1.5h, Gaussian sums over the near-field lists "
                 "(p=%d, theta=%g, ncrit=%d, sigma_gap=6), conjugate gradients from zero to 1e-4"
                 % (args.n, args.p, args.theta, args.ncrit), res)
    print(json.dumps(line), flush=True)


def _time_overlap(ctx1, t, case, args, pairs):
    """Time the same steps with the near field on its own stream beside the far field."""
    import torch
    out1 = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))
    for _ in range(max(1, args.warmup)):
        ctx1.build(t[0], t[1], t[2], t[6])
        ctx1.evaluate(*t, out=out1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx1.build(t[0], t[1], t[2], t[6])
        ctx1.evaluate(*t, out=out1)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t1) * 1e3 / args.steps
    ph = ctx1.timings()
    ctx1.close()
    return {"ms_per_step": ms1, "gpair_s": pairs / (ms1 * 1e-3) / 1e9, "p2p_interval_ms": ph["p2p_ms"],
            "evaluate_ms": ph["evaluate_ms"]}


def _time_tuned(vf, wl, t, case, args, params):
    """The same workload and accuracy check with the settings vfmm_autotune
    chooses for a 1e-4 bound (p, theta, ncrit, core-overlap gap, precision
    form, M2L product form, evaluation order), timed like the main line."""
    import numpy as np
    import torch
    ctx = vf.Context(**params)
    t0 = time.perf_counter()
    r = ctx.autotune(*t, max_rel_l2=1e-4)
    tune_s = time.perf_counter() - t0
    out = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))
    for _ in range(max(1, args.warmup)):
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t, out=out)
    torch.cuda.synchronize()
    ph = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t, out=out)
        ph.append(ctx.timings())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    st = ctx.stats()
    ctx.close()
    res = {"chosen_by": "vfmm_autotune, max_rel_l2 = 1e-4 against its p = 12, theta = 0.35 reference",
           "p": r["p"], "theta": r["theta"], "ncrit": r["ncrit"], "sigma_gap": r["sigma_gap"],
           "precision": r["precision"], "m2l_form": r["m2l_form"], "overlap": r["overlap"],
           "tuner_err_u": r["err_u"], "tuner_err_dalpha": r["err_dalpha"], "tuner_worst_u": r["worst_u"],
           "tuner_worst_dalpha": r["worst_dalpha"], "configurations_tried": r["tried"],
           "tuner_seconds": tune_s, "ms_per_step": ms, "p2p_pairs_per_step": st["p2p_pairs"],
           "m2l_translations": st["m2l_entries"],
           "phases_ms": {k: float(np.mean([p[k] for p in ph])) for k in ph[0]}}
    if not args.no_check:
        idx, ref, _ = golden("bench_c2_%d.txt" % args.n, wl.case_arrays(case))
        u = np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64)[idx]
        da = np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64)[idx]
        res["accuracy"] = {"rel_l2_u": rel_l2(u, ref[:, :3]), "rel_l2_dalpha": rel_l2(da, ref[:, 3:]),
                           "targets": int(idx.size)}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; sharding over several GPUs is not implemented "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.microbench:
        import ctypes
        mb = ctypes.CDLL(os.path.join(ROOT, "paper_1106_5273_amd", "libvfmm_mb.so"))
        mb.vfmm_mb_rate.restype = ctypes.c_float
        mb.vfmm_mb_rate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        blocks, iters = 256 * 64, 400
        ops = blocks * 256.0 * iters * 16 * 8
        res = {}
        for kind, name in ((0, "fma_vector_operand"), (1, "fma_scalar_operand"), (2, "exp2"), (3, "rsq"),
                           (4, "fma_dpp_row_broadcast_operand"), (5, "fma_vop3"), (6, "fma_vop3_scalar_src1"),
                           (7, "fma_vop3_scalar_addend"), (8, "mov_from_scalar"),
                           (9, "fma_accumulator_bank_shared_with_source"), (10, "fma_fixed_registers_no_shared_bank"),
                           (11, "fma7_exp1_mix")):
            ms = mb.vfmm_mb_rate(kind, blocks, iters if kind not in (2, 3) else iters // 4)
            n_ops = ops if kind not in (2, 3) else ops / 4
            res[name + "_lane_ops_per_s"] = n_ops / (ms * 1e-3)
        res["fma_tflops"] = 2 * res["fma_vector_operand_lane_ops_per_s"] / 1e12
        print(json.dumps(res), flush=True)
        return
    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)
        return

    import paper_1106_5273_amd as vf
    import workloads as wl

    torch.cuda.set_device(0)
    if args.workload == "c4":
        return bench_batched(args, vf, wl)
    if args.workload == "c5":
        return bench_rk(args, vf, wl)
    if args.workload == "targets":
        return bench_targets(args, vf, wl)
    if args.workload == "var":
        return bench_varcore(args, vf, wl)
    if args.workload == "c3":
        return bench_precision(args, vf, wl)
    if args.workload == "rbf":
        return bench_rbf(args, vf, wl)
    L = 2 * np.pi
    case = wl.turbulence_case(args.n, seed=2)
    t = vf.case_to_device(case)
    params = dict(p=args.p, theta=args.theta, ncrit=args.ncrit, sigma_gap=5.0, periodic=1, box_len=L,
                  images=args.images, kahan=args.kahan)
    if args.m2l_form is not None:
        params["m2l_form"] = args.m2l_form
    if args.overlap is not None:
        params["overlap"] = args.overlap
    ctx = vf.Context(**params)
    out = tuple(torch.empty(case["n"], dtype=torch.float32, device="cuda") for _ in range(6))

    def step():
        ctx.build(t[0], t[1], t[2], t[6])
        ctx.evaluate(*t, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        phases.append(ctx.timings())  # synchronises the stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = wall * 1e3 / args.steps
    st = ctx.stats()
    pairs = st["p2p_pairs"]
    p2p_ms = float(np.mean([p["p2p_ms"] for p in phases]))
    mean_ph = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}

    acc = {}
    if not args.no_check:
        idx, ref, what = golden("bench_c2_%d.txt" % args.n, wl.case_arrays(case))
        u = np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64)[idx]
        da = np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64)[idx]
        acc = {"rel_l2_u": rel_l2(u, ref[:, :3]), "rel_l2_dalpha": rel_l2(da, ref[:, 3:]),
               "targets": int(idx.size), "reference": what}

    achieved = pairs * FLOPS_PER_PAIR / (p2p_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(pairs)
    # the same steps with the near field on a second stream beside the far field
    # (overlap = 1, informational: the P2P kernel then shares the GPU)
    ov = None
    ctx1 = None if args.no_overlap_pass else vf.Context(**dict(params, overlap=1))
    if ctx1 is not None:
        ov = _time_overlap(ctx1, t, case, args, pairs)
    tuned = None if args.no_overlap_pass else _time_tuned(vf, wl, t, case, args, params)
    line = {
        "metric": METRIC,
        "value": pairs / (ms * 1e-3) / 1e9,
        "unit": "Gpair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "periodic 128^3 turbulence-shaped lattice, one velocity+stretching FMM step "
                               "(build+evaluate)" if args.n == 128 else "periodic %d^3 lattice" % args.n,
                   "n": case["n"], "p": args.p, "theta": args.theta, "ncrit": args.ncrit, "sigma_gap": 5.0,
                   "images": args.images, "kahan": args.kahan, "seed": 2,
                   "m2l_form": ctx.params.m2l_form, "overlap": ctx.params.overlap},
        "p2p_pairs_per_step": pairs,
        "p2p_kernel_ms": p2p_ms,
        "p2p_kernel_gpair_s": pairs / (p2p_ms * 1e-3) / 1e9,
        "paper_convention_gflops": pairs * PAPER_FLOPS_PER_PAIR / (p2p_ms * 1e-3) / 1e9,
        "phases_ms": mean_ph,
        "tree": {"ncells": st["ncells"], "nleaves": st["nleaves"], "depth": st["depth"],
                 "m2l": st["m2l_entries"], "p2p_entries": st["p2p_entries"], "m2l_keys": st["m2l_keys"],
                 "m2l_groups": st["m2l_groups"], "m2l_items": st["m2l_items"]},
        "accuracy": acc,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
                     "kernel": "k_p2p", "flops_per_pair": FLOPS_PER_PAIR},
        "m2l": m2l_object(st, mean_ph["m2l_ms"], args.p),
        "overlap_streams": ov,
        "tuned": tuned,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
