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
PEAK_FP32_VALU_TFLOPS = 157.3        # 256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
FLOPS_PER_PAIR = 79                   # gfx950 ISA of the P2P pair body (s >= 1 form): 29 FMA + 16 MUL + 3 SUB + 2 TRANS, FMA = 2
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
    ap.add_argument("--images", type=int, default=6)
    ap.add_argument("--kahan", type=int, default=0)
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy check against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for HBM bytes) and exit")
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1106_5273_amd", "csrc", "p2p.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


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


def cpu_baseline(case, seconds):
    """FP64 direct oracle on a bounded sample: a subset of targets against all
    sources of the central box, on every host core."""
    import numpy as np

    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = case["n"]
    rng = np.random.default_rng(123)
    nt = 8
    t0 = time.perf_counter()
    oracle.direct(case, targets=rng.choice(n, nt, replace=False))
    dt = time.perf_counter() - t0
    nt = int(max(8, min(n, nt * seconds / max(dt, 1e-3))))
    idx = rng.choice(n, nt, replace=False)
    t0 = time.perf_counter()
    oracle.direct(case, targets=idx)
    dt = time.perf_counter() - t0
    pairs = nt * n
    return {"value": pairs / dt / 1e9, "unit": "Gpair/s", "cores": cores, "kind": "oracle",
            "sample": "%d random targets x %d sources of the central box (free-space FP64 direct sum), %.1f s"
                      % (nt, n, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is described in DESIGN.md, "
              "not implemented (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

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
    L = 2 * np.pi
    case = wl.turbulence_case(args.n, seed=2)
    t = vf.case_to_device(case)
    params = dict(p=args.p, theta=args.theta, ncrit=args.ncrit, sigma_gap=5.0, periodic=1, box_len=L,
                  images=args.images, kahan=args.kahan)
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
        import oracle
        u = np.stack([o.cpu().numpy() for o in out[:3]], 1).astype(np.float64)
        da = np.stack([o.cpu().numpy() for o in out[3:]], 1).astype(np.float64)
        us, Js = oracle.spectral_lattice(case)
        das, _ = oracle.stretching(Js, np.stack([case["ax"], case["ay"], case["az"]], 1).astype(np.float64))
        acc = {"rel_l2_u": float(np.linalg.norm(u - us) / np.linalg.norm(us)),
               "rel_l2_dalpha": float(np.linalg.norm(da - das) / np.linalg.norm(das)),
               "reference": "exact FP64 periodic sum (Fourier series on the lattice), zero-mean convention"}

    achieved = pairs * FLOPS_PER_PAIR / (p2p_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(pairs)
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
                   "images": args.images, "kahan": args.kahan, "seed": 2},
        "p2p_pairs_per_step": pairs,
        "p2p_kernel_ms": p2p_ms,
        "p2p_kernel_gpair_s": pairs / (p2p_ms * 1e-3) / 1e9,
        "paper_convention_gflops": pairs * PAPER_FLOPS_PER_PAIR / (p2p_ms * 1e-3) / 1e9,
        "phases_ms": mean_ph,
        "tree": {"ncells": st["ncells"], "nleaves": st["nleaves"], "depth": st["depth"],
                 "m2l": st["m2l_entries"], "p2p_entries": st["p2p_entries"]},
        "accuracy": acc,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
                     "kernel": "k_p2p", "flops_per_pair": FLOPS_PER_PAIR},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
