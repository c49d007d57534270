"""Benchmark of the CTMRG hot path on one MI355X.

Workload: the two-sublattice purification at D = 6 (double-layer leg
d = 36), chi = 72, A and B drawn i.i.d. N(0,1) from seed 1234 and scaled to
unit max-abs, fused across the z bond (d * chi = 2592).  The environment is
first converged for 20 sweeps (untimed set-up).  One step is one CTMRG sweep:
the left, right, up and down absorption moves, each with its enlarged
corners, half-system and cut products, truncated projector SVD and
renormalisation.  Throughput is reported as GFLOP/s of algorithmic work,
2 W per move with W = 5 chi^2 d^4 + 3 chi^3 d^3 + 8 chi^3 d^2 + 6 chi^3 d
multiply-adds (the projector SVD is timed but not counted).

Prints one JSON line on stdout; everything else goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_F64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def move_macs(chi, d):
    return (5.0 * chi ** 2 * d ** 4 + 3.0 * chi ** 3 * d ** 3 + 8.0 * chi ** 3 * d ** 2
            + 6.0 * chi ** 3 * d)


def executed_move_macs(chi, d):
    """MACs the implementation executes per move in steady state: two of the
    four enlarged corners are recomputed (the other two are cached), the
    three n^3 products, the two projector products, the renormalisation;
    the subspace SVD products are listed separately."""
    n = chi * d
    corners = 2 * (chi ** 3 * d + chi ** 3 * d ** 2 + chi ** 2 * d ** 4)
    halves = 3.0 * n ** 3
    proj = 2.0 * n * n * chi
    renorm = chi ** 2 * d ** 4 + 2 * chi ** 3 * d ** 2 + 2 * chi ** 3 * d + chi ** 3 * d
    return corners + halves + proj + renorm


def cpu_baseline(D, chi, seed, moves=2):
    """The FP64 oracle on the host cores: `moves` absorption moves from the
    boundary start at the benchmark shape (each with a full LAPACK SVD of the
    n x n cut matrix)."""
    from oracle import ctmrg as O
    from paper_1906_02220_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    A, B = synth.random_purification(D, seed)
    K = O.composite(A, B, 2)
    a = O.double_layer(K)
    arot = [O.rotate(a, k) for k in range(4)]
    env = O.init_env(D * D, chi, O.boundary_vector_double_layer(D))
    t0 = time.perf_counter()
    for k in (0, 2, 1, 3)[:moves]:
        O.left_move(env, arot, k, chi)
    dt = time.perf_counter() - t0
    gflops = moves * 2.0 * move_macs(chi, D * D) / dt / 1e9
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d absorption moves from the boundary start at D=%d chi=%d (full LAPACK SVD "
                      "of the %dx%d cut matrix per move), %.1f s" % (moves, D, chi, chi * D * D,
                                                                    chi * D * D, dt)}


COPY_BYTES = 512 << 20


def calibrate_copy(torch):
    """Three plain device-to-device copies of COPY_BYTES each: the kernel the
    HBM byte counters are scaled against."""
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}), flush=True)


def kernel_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_1906_02220_amd", "csrc", "gemm_f64.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(path):
    """HBM bytes per launch of the n^3 GEMM from the counter summary (lines
    'key: value'); None when the summary is missing or was taken on another
    version of the GEMM source."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("gemm_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--converge", type=int, default=20, help="untimed sweeps before warmup")
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=72)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_dgemm_rr_cut_D6_chi72.txt"),
                    help="HBM-counter summary of the n^3 GEMM (bytes per launch)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_1906_02220_amd import ctm, synth

    D, chi, seed = args.D, args.chi, args.seed
    d = D * D
    n = chi * d
    A, B = synth.random_purification(D, seed)
    ctx = ctm.Context(0)
    env = ctm.Environment.from_purification(ctx, A, B, 2, chi)
    log("bench: converging %d sweeps at D=%d chi=%d (n=%d)" % (args.converge, D, chi, n))
    t0 = time.perf_counter()
    env.sweep(args.converge, 0.0)
    log("bench: converged in %.2f s, kappa %.15g" % (time.perf_counter() - t0, env.norm()))
    for _ in range(args.warmup):
        env.sweep(1, 0.0)

    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        env.sweep(1, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c0, ms0, fl0 = ctx.timing_get(0)   # the n x n x n FP64 GEMMs
    c1, ms1, fl1 = ctx.timing_get(1)   # every dense contraction kernel
    c2, ms2, fl2 = ctx.timing_get(2)   # whole moves
    ctx.timing(False)

    ms_step = 1e3 * dt / args.steps
    moves = 4 * args.steps
    alg_flops = 2.0 * move_macs(chi, d) * moves
    value = alg_flops / dt / 1e9
    exe_flops = 2.0 * executed_move_macs(chi, d) * moves
    # roofline of the dominant kernel: the n^3 FP64 GEMM (2 n^3 flops per launch)
    per_launch = 2.0 * float(n) ** 3
    avg_ms = ms0 / max(c0, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    traffic = read_traffic(args.traffic)

    # a9: bond metric, norm and one expectation value on the converged environment
    H = synth.bond_operator_real(synth.random_coefficients(6))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kappa = env.norm()
    e_h = env.expect(H)
    E = env.bond_metric()
    torch.cuda.synchronize()
    fu_ms = 1e3 * (time.perf_counter() - t1)

    out = {
        "metric": "CTMRG move GFLOP/s (%MFMA peak), D=6 chi=72: mixed vs FP64 at <=1e-8 err",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rhombic-lattice CTMRG sweep of a random D=6 purification, chi=72 "
                               "(d=36, cut n=2592), seed 1234, after %d converging sweeps" % args.converge,
                   "D": D, "chi": chi, "d": d, "n": n, "gamma": "z", "precision": "FP64",
                   "step": "one sweep = 4 absorption moves (L, R, U, D)"},
        "ms_per_move": round(ms_step / 4.0, 3),
        "pct_fp64_mfma_peak_algorithmic": round(100.0 * value / (PEAK_F64_TFLOPS * 1e3), 2),
        "executed_gflops": round(exe_flops / dt / 1e9, 2),
        "pct_fp64_mfma_peak_executed": round(100.0 * exe_flops / dt / 1e9 / (PEAK_F64_TFLOPS * 1e3), 2),
        "gemm_share_of_move_time": round(ms1 / max(ms2, 1e-9), 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_TFLOPS, 4),
                     "traffic": traffic,
                     "kernel": "dgemm_rr<96,96,16,2,2,0> (n x n x n, n=%d)" % n,
                     "launches": c0, "avg_launch_ms": round(avg_ms, 4)},
        "fu_metric_ms": round(fu_ms, 3),
        "kappa": kappa,
        "energy_bond": e_h,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(D, chi, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
