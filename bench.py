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

# Concurrent environments of the batch measurement each run on their own
# stream; HIP maps streams onto this many hardware queues (its default is 4).
# Set before HIP starts; at least 16, never above 32.
try:
    _q = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _q = 4
os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(_q, 16)))

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


def cpu_baseline(D, chi, seed, moves=16):
    """The FP64 oracle on the host cores: `moves` absorption moves from the
    boundary start at the benchmark shape, cycling L, R, U, D (each with a
    full LAPACK SVD of the n x n cut matrix).  The rate divides the
    algorithmic work of exactly the moves that ran by their time."""
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
    order = cpu_baseline_order(moves)
    t0 = time.perf_counter()
    for k in order:
        O.left_move(env, arot, k, chi)
    dt = time.perf_counter() - t0
    gflops = len(order) * 2.0 * move_macs(chi, D * D) / dt / 1e9
    return {"value": float("%.6g" % gflops), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d absorption moves (%d sweeps L, R, U, D) from the boundary start at D=%d "
                      "chi=%d, each with a full LAPACK SVD of the %dx%d cut matrix, %.1f s" % (
                          len(order), len(order) // 4, D, chi, chi * D * D, chi * D * D, dt),
            "moves": len(order), "seconds": dt}


def cpu_baseline_order(moves):
    """Directions of the CPU sample's moves: the sweep order L, R, U, D
    repeated until `moves` moves."""
    return [(0, 2, 1, 3)[i % 4] for i in range(moves)]


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


def kernel_source_hash(source):
    import hashlib
    path = os.path.join(ROOT, "paper_1906_02220_amd", "csrc", source)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


TRAFFIC = {  # counter summary and kernel source per precision mode
    0: ("traffic_dgemm_rr_cut_D6_chi72.txt", "gemm_f64.hip"),
    3: ("traffic_gemm_bf16s3_cut_D6_chi72.txt", "gemm_mixed.hip"),
}


def read_traffic(mode):
    """HBM bytes per launch of the mode's n^3 product from its counter
    summary (lines 'key: value'); None when there is none or it was taken on
    another version of the kernel source."""
    if mode not in TRAFFIC:
        return None
    name, source = TRAFFIC[mode]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("gemm_source_sha256_16") != kernel_source_hash(source):
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


MODE_NAMES = {0: "f64", 1: "f32", 3: "bf16x3", 4: "bf16x4"}
PRECISION_TEXT = {
    0: "FP64 MFMA throughout",
    1: "a4/a5/a7 sweep contractions: FP32 MFMA, FP32 accumulation; projector SVD, small products "
       "and the a9 ring FP64",
    3: "a4/a5/a7 sweep contractions: 3 BF16 slices (6 slice products), FP32 accumulation over K "
       "chunks of 128, FP64 chunk sums; projector SVD, small products and the a9 ring FP64",
    4: "a4/a5/a7 sweep contractions: 4 BF16 slices (10 slice products), FP32 accumulation over K "
       "chunks of 128, FP64 chunk sums; projector SVD, small products and the a9 ring FP64",
}
PEAK_TFLOPS = {0: 78.6, 1: 157.3, 3: 2500.0, 4: 2500.0}
SLICE_PRODUCTS = {0: 1, 1: 1, 3: 6, 4: 10}
KERNEL_NAMES = {0: "dgemm_rr<96,96,16,2,2,0,true,true>", 1: "gemm_f32x1_kernel<0>",
                3: "gemm_bf16s_kernel<3,0,8>", 4: "gemm_bf16s_kernel<4,0,8>"}


def run_mode(ctx, ctm, torch, A, B, H, D, chi, mode, args, converge=None):
    """Converge, warm up and time `args.steps` sweeps in one precision mode
    with per-launch timing off (the value); then as many sweeps again with
    HIP events around every launch (the kernel averages of the roofline);
    then the bond metric, norm and <H_bond> of the environment."""
    d = D * D
    n = chi * d
    converge = args.converge if converge is None else converge
    env = ctm.Environment.from_purification(ctx, A, B, 2, chi, precision=mode)
    log("bench: mode %s: converging %d sweeps at D=%d chi=%d (n=%d)" % (
        MODE_NAMES[mode], converge, D, chi, n))
    t0 = time.perf_counter()
    _, _, delta = env.sweep(converge, 0.0)
    log("bench: converged in %.2f s, kappa %.15g, delta %.3e" % (time.perf_counter() - t0,
                                                                 env.norm(), delta))
    for _ in range(args.warmup):
        env.sweep(1, 0.0)
    ctx.timing(False)
    torch.cuda.synchronize()
    # one call of args.steps sweeps (it returns once the stream has drained;
    # the corner spectra of its delta are taken after its last two sweeps)
    t0 = time.perf_counter()
    env.sweep(args.steps, 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kappa_prev, e_prev = env.norm(), env.expect(H)
    # second pass: the same number of sweeps with per-launch HIP events
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    _, _, delta = env.sweep(args.steps, 0.0)
    torch.cuda.synchronize()
    c0, ms0, _ = ctx.timing_get(0)   # the n x n x n cut-matrix products
    c1, ms1, _ = ctx.timing_get(1)   # every dense contraction kernel
    c2, ms2, _ = ctx.timing_get(2)   # whole moves
    ctx.timing(False)
    moves = 4 * args.steps
    gflops = 2.0 * move_macs(chi, d) * moves / dt / 1e9
    # roofline of the dominant kernel: one n x n x n product per launch, the
    # method's 2 n^3 flops per launch against the peak of the dtype the
    # kernel computes in; the executed MFMA flops (slice products x 2 n^3)
    # are reported beside it
    per_launch = 2.0 * float(n) ** 3
    avg_ms = ms0 / max(c0, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    executed = SLICE_PRODUCTS[mode] * achieved
    traffic = read_traffic(mode)
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[mode],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[mode], 4),
            "traffic": traffic,
            "traffic_GBps": None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1),
            "kernel": "%s (n x n x n, n=%d)" % (KERNEL_NAMES[mode], n),
            "flops_per_launch": per_launch, "launches": c0, "avg_launch_ms": round(avg_ms, 4),
            "slice_products_per_launch": SLICE_PRODUCTS[mode],
            "executed_achieved": round(executed, 3),
            "executed_frac": round(executed / PEAK_TFLOPS[mode], 4)}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kappa = env.norm()
    e_h = env.expect(H)
    env.bond_metric()
    torch.cuda.synchronize()
    fu_ms = 1e3 * (time.perf_counter() - t1)
    env.close()
    return {"gflops": gflops, "ms_per_move": 1e3 * dt / moves,
            "executed_gflops": 2.0 * executed_move_macs(chi, d) * moves / dt / 1e9,
            "pct_mfma_peak_of_dtype": 100.0 * gflops / (PEAK_TFLOPS[mode] * 1e3),
            "contraction_share_of_move_time": ms1 / max(ms2, 1e-9),
            "contraction_only_gflops": 2.0 * move_macs(chi, d) * moves / max(ms1 * 1e-3, 1e-12) / 1e9,
            "roofline": roof, "fu_ms": fu_ms, "kappa": kappa, "energy_bond": e_h,
            "delta_last_sweep": delta,
            # how far the environment itself still moves over the last
            # args.steps sweeps: the floor under any comparison of modes
            "self_change_kappa": abs(kappa / kappa_prev - 1.0),
            "self_change_energy": abs(e_h - e_prev)}


def run_structured(ctx, ctm, torch, synth, H, D, chi, modes, args):
    """The structured stand-in for near-critical spectra beside the random
    case: the honeycomb Ising state at K = 0.6 (critical K_c = 0.658, D = 2)
    zero-padded to D and gauged with seeded random invertible matrices on
    every bond (seed 1234), so that most of the cut matrix's singular values
    sit at rounding level.  Timed like the random case, in every mode the
    random case ran, after args.structured_converge converging sweeps;
    `within_1e-8` names the modes whose kappa and <H_bond> both stay within
    1e-8 of FP64 here, `kappa_within_1e-8` those whose kappa does."""
    A0, B0 = synth.honeycomb_ising_tensors(0.6, 0.6, 0.6)
    A, B = synth.pad_and_gauge(A0, B0, D, 1234)
    conv = args.structured_converge
    res = {"workload": "honeycomb Ising state, K=0.6 on every bond, padded from D=2 to D=%d and "
                       "gauged (seed 1234), chi=%d, %d sweeps after %d converging" % (
                           D, chi, args.steps, conv)}
    runs = {m: run_mode(ctx, ctm, torch, A, B, H, D, chi, m, args, converge=conv) for m in modes}
    ref = runs[0]
    for m, r in runs.items():
        res[MODE_NAMES[m]] = {"gflops": round(r["gflops"], 2), "ms_per_move": round(r["ms_per_move"], 3),
                              "kappa": r["kappa"], "energy_bond": r["energy_bond"],
                              "err_kappa_vs_fp64": abs(r["kappa"] / ref["kappa"] - 1.0),
                              "err_energy_vs_fp64": abs(r["energy_bond"] - ref["energy_bond"]),
                              "delta_last_sweep": r["delta_last_sweep"],
                              "self_change_kappa": r["self_change_kappa"],
                              "self_change_energy": r["self_change_energy"]}
    res["within_1e-8"] = [MODE_NAMES[m] for m in runs if m != 0 and
                          max(res[MODE_NAMES[m]]["err_kappa_vs_fp64"],
                              res[MODE_NAMES[m]]["err_energy_vs_fp64"]) <= 1e-8]
    res["kappa_within_1e-8"] = [MODE_NAMES[m] for m in runs if m != 0 and
                                res[MODE_NAMES[m]]["err_kappa_vs_fp64"] <= 1e-8]
    res["_errs"] = {m: (res[MODE_NAMES[m]]["err_kappa_vs_fp64"],
                        res[MODE_NAMES[m]]["err_energy_vs_fp64"]) for m in runs}
    return res


def run_batch(ctm, torch, synth, count, warm, steps, uniform=None):
    """Batched sweeps: `count` independent purifications with (D, chi) drawn
    uniformly from {4,5,6,7} x {32,48,72,96} (seed 777), A and B i.i.d.
    N(0,1) in FP32 (seed 778 + i), scaled to unit max-abs, contractions in
    the FP32 mode.  Timed: `steps` sweeps of the whole batch after `warm`,
    with the environments in turn on one context, concurrently on one
    context each, concurrently with autotuned tilings and graph replay, and in
    lock-step with the n x n x n products of all environments grouped into
    persistent launches (one context each).  With `uniform` = (D, chi) every
    environment has that shape instead."""
    if uniform is None:
        rng = np.random.default_rng(777)
        Ds = rng.choice([4, 5, 6, 7], size=count).tolist()
        chis = rng.choice([32, 48, 72, 96], size=count).tolist()
        cfg = list(zip(Ds, chis))
        what = "(D, chi) uniform on {4,5,6,7} x {32,48,72,96} (seed 777)"
        variants = (("in_turn", True, False, False, False),
                    ("concurrent", False, False, False, False),
                    ("concurrent_autotuned_graphs", False, True, True, False),
                    ("lockstep_grouped", False, False, False, True))
    else:
        cfg = [tuple(uniform)] * count
        what = "all D=%d, chi=%d" % tuple(uniform)
        variants = (("in_turn", True, False, False, False),
                    ("concurrent_autotuned_graphs", False, True, True, False),
                    ("lockstep_grouped", False, False, False, True))
    work = sum(2.0 * move_macs(chi, D * D) * 4 for D, chi in cfg)
    out = {"workload": "%d purifications, %s, FP32 entries, FP32 contraction mode" % (count, what),
           "envs": [[int(D), int(chi)] for D, chi in cfg], "sweeps_timed": steps,
           "unit": "GFLOP/s (sum over the batch, algorithmic)"}
    for name, one_ctx, tune, graphs, grouped in variants:
        ctxs = [ctm.Context(0)] if one_ctx else [ctm.Context(0) for _ in cfg]
        for c in ctxs:
            c.autotune(tune)
            c.graphs(graphs)
        envs = []
        for i, (D, chi) in enumerate(cfg):
            A, B = synth.random_purification(D, 778 + i, dtype=np.float32)
            envs.append(ctm.Environment.from_purification(ctxs[0 if one_ctx else i], A, B, 2, chi,
                                                          precision=ctm.CTM_PREC_F32))
        ctm.sweep_batch(envs, warm, grouped=grouped)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctm.sweep_batch(envs, steps, grouped=grouped)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"value": round(work * steps / dt / 1e9, 2),
                     "ms_per_batch_sweep": round(1e3 * dt / steps, 3)}
        log("bench: batch %s %s: %.1f ms per batch sweep" % (what, name, 1e3 * dt / steps))
        if name == "in_turn":
            kappas = [e.norm() for e in envs]
        for e in envs:
            e.close()
        for c in ctxs:
            c.close()
    # every member's environment norm against the same member run in FP64
    # for the same number of sweeps (all variants give identical results)
    ctxs = [ctm.Context(0) for _ in cfg]
    envs = []
    for i, (D, chi) in enumerate(cfg):
        A, B = synth.random_purification(D, 778 + i, dtype=np.float32)
        envs.append(ctm.Environment.from_purification(ctxs[i], A, B, 2, chi,
                                                      precision=ctm.CTM_PREC_F64))
    ctm.sweep_batch(envs, warm + steps)
    errs = [abs(k / e.norm() - 1.0) for k, e in zip(kappas, envs)]
    for e in envs:
        e.close()
    for c in ctxs:
        c.close()
    out["err_kappa_vs_fp64_per_env"] = [float("%.3g" % x) for x in errs]
    out["err_kappa_vs_fp64_max"] = max(errs)
    best = max(("concurrent_autotuned_graphs", "lockstep_grouped"), key=lambda k: out[k]["value"])
    out["best"] = best
    out["speedup_vs_in_turn"] = round(out[best]["value"] / out["in_turn"]["value"], 3)
    return out


def run_grad(ctm, synth, reps):
    """Reverse-mode gradient on the differentiation workload: D = 5, chi = 50
    (n = 1250), seeds 5 (A, B) and 6 (bond operator), 30 fixed sweeps,
    checkpoints every 5 sweeps, projector cutoff 5e-8, gradient of
    ln kappa + <H_bond> with respect to A and B.  One untimed call, then
    `reps` timed calls; also the plain forward (30 sweeps and both
    observables) for the ratio."""
    A, B = synth.random_purification(5, 5)
    H = synth.bond_operator_real(synth.random_coefficients(6))
    ctx = ctm.Context(0)
    kw = dict(op=H, w_log_kappa=1.0, w_expect=1.0, checkpoint_every=5, eps_cut=5e-8)
    ctm.grad_purification(ctx, A, B, 2, 50, 30, **kw)
    t0 = time.perf_counter()
    for _ in range(reps):
        lk, ex, gA, gB, info = ctm.grad_purification(ctx, A, B, 2, 50, 30, **kw)
    dt = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    env = ctm.Environment.from_purification(ctx, A, B, 2, 50, eps_cut=5e-8)
    env.sweep(30)
    env.norm()
    env.expect(H)
    df = time.perf_counter() - t0
    env.close()
    ctx.close()
    log("bench: gradient %.1f ms (forward alone %.1f ms)" % (1e3 * dt, 1e3 * df))
    return {"workload": "d(ln kappa + <H_bond>)/d(A, B), D=5 chi=50 (n=1250), 30 sweeps, "
                        "checkpoints every 5, eps_cut 5e-8, seeds 5/6, FP64",
            "ms_per_gradient": round(1e3 * dt, 2), "ms_forward_only": round(1e3 * df, 2),
            "gradient_over_forward": round(dt / df, 2),
            "ms_first_forward": round(info["ms_forward"], 2),
            "ms_recompute": round(info["ms_recompute"], 2),
            "ms_reverse": round(info["ms_backward"], 2),
            "cg_iters_per_move": round(info["cg_iters_total"] / max(info["moves"], 1), 2),
            "cg_iters_max": info["cg_iters_max"],
            "tape_MB": round(info["tape_bytes"] / 2 ** 20, 1),
            "checkpoint_MB": round(info["checkpoint_bytes"] / 2 ** 20, 1),
            "log_kappa": lk, "energy_bond": ex}


def run_fu(ctm, synth, reps):
    """Full-update bond update at the benchmark's shape: random D = 6
    purification (seed 1234), gamma = z, Kitaev-Heisenberg bond term at
    phi = -63 degrees, tau = 0.02; environment of the gated composite (4D = 24
    inside, d = 36 outside) from 20 sweeps at chi = 72 in FP64; 10 ALS rounds.
    Timed: `reps` calls after one untimed call, and the same with 0 rounds
    for the ALS share."""
    A, B = synth.random_purification(6, 1234)
    H = synth.kitaev_heisenberg_bond(np.deg2rad(-63.0), 2)
    ctx = ctm.Context(0)
    ctm.fu_bond_update(ctx, A, B, 2, H, 0.02, 72, 20, 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        A2, B2, errs = ctm.fu_bond_update(ctx, A, B, 2, H, 0.02, 72, 20, 10)
    dt = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        ctm.fu_bond_update(ctx, A, B, 2, H, 0.02, 72, 20, 0)
    d0 = (time.perf_counter() - t0) / reps
    ctx.close()
    log("bench: full-update bond update %.1f ms (%.1f ms without ALS)" % (1e3 * dt, 1e3 * d0))
    return {"workload": "one eeFU bond update: D=6 (seed 1234), gamma=z, KH phi=-63 deg, tau=0.02, "
                        "environment of the gated composite from 20 sweeps at chi=72 (FP64), "
                        "10 ALS rounds (216 x 216 normal matrices)",
            "ms_per_bond_update": round(1e3 * dt, 2),
            "ms_environment_and_setup": round(1e3 * d0, 2),
            "ms_per_als_round": round(1e3 * (dt - d0) / 10, 3),
            "error_start": errs[0], "error_after_10_rounds": errs[-1]}


def run_xi(ctm, synth, reps):
    """Correlation length of the benchmark environment: D = 6, chi = 72, seed
    1234, 20 sweeps; the column transfer matrix with the site row (dimension
    chi^2 d = 186624), 40 Arnoldi steps, 4 leading eigenvalues.  Once on the
    FP64 environment and once on the BF16x3 one (whose 2 chi^2 d^4 transfer
    product also runs in BF16x3)."""
    A, B = synth.random_purification(6, 1234)
    out = {"workload": "column transfer matrix (T1, a, T3) of the D=6 chi=72 environment after "
                       "20 sweeps (dimension 186624), 40 Arnoldi steps"}
    for name, prec in (("f64", ctm.CTM_PREC_F64), ("bf16x3", ctm.CTM_PREC_BF16X3)):
        ctx = ctm.Context(0)
        env = ctm.Environment.from_purification(ctx, A, B, 2, 72, precision=prec)
        env.sweep(20)
        env.transfer_spectrum(0, True, 4, 40)
        t0 = time.perf_counter()
        for _ in range(reps):
            ev, xi = env.transfer_spectrum(0, True, 4, 40)
        dt = (time.perf_counter() - t0) / reps
        env.close()
        ctx.close()
        log("bench: transfer spectrum (%s environment) %.1f ms, xi %.6f" % (name, 1e3 * dt, xi))
        eps = [float(-np.log(abs(e) / abs(ev[0]))) for e in ev[1:]]
        out[name] = {"ms": round(1e3 * dt, 2), "xi": xi, "eps_2_3_4": eps}
    # the FP64 figures also at the top level, as before
    out.update({"ms": out["f64"]["ms"], "xi": out["f64"]["xi"], "eps_2_3_4": out["f64"]["eps_2_3_4"]})
    return out


# per-mode figures: rates and times to 6 decimals; errors, changes and the
# observables to 4 significant digits (rounding them to decimals would turn
# a change of 1e-13 into 0)
_SIGNIFICANT = ("err_kappa_vs_fp64", "err_energy_vs_fp64", "self_change_kappa", "self_change_energy",
                "delta_last_sweep")


def _fmt(k, v):
    if not isinstance(v, float):
        return v
    if k in ("kappa", "energy_bond"):
        return v
    if k in _SIGNIFICANT:
        return float("%.4g" % v)
    return round(v, 6)


def select_headline(runs, structured):
    """The headline mode: the fastest reduced-precision mode whose error
    against FP64 stays within a bound on both workloads, the tightest bound
    of (1e-8, 1e-7) that some mode meets; FP64 itself if none does.  The
    error is the environment norm kappa on both the random and the
    structured workload, and <H_bond> on the random one (the metric's
    workload).  On the structured workload <H_bond> is reported but not
    gated: there FP64's own <H_bond> still moves between sweeps by more
    than the bound (self_change_energy), and the comparison cannot resolve
    it."""
    rule = ("kappa within the bound of FP64 on the random and the structured workload, "
            "<H_bond> within the bound on the random workload")
    for tol in (1e-8, 1e-7):
        ok = []
        for m, r in runs.items():
            if m == 0:
                continue
            errs = [r["err_kappa_vs_fp64"], r["err_energy_vs_fp64"]]
            if structured is not None:
                errs.append(structured["_errs"][m][0])
            if max(errs) <= tol:
                ok.append(m)
        if ok:
            return min(ok, key=lambda m: runs[m]["ms_per_move"]), tol, rule
    return 0, 0.0, rule


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
    ap.add_argument("--batch", type=int, default=32,
                    help="environments of the batched-sweep measurement (0: skip it)")
    ap.add_argument("--grad", type=int, default=3,
                    help="timed calls of the gradient measurement (0: skip it)")
    ap.add_argument("--fu", type=int, default=2,
                    help="timed calls of the full-update measurement (0: skip it)")
    ap.add_argument("--structured", type=int, default=1,
                    help="also time the structured (padded honeycomb Ising) case (0: skip it)")
    ap.add_argument("--structured-converge", type=int, default=40,
                    help="untimed sweeps of the structured case before warmup")
    ap.add_argument("--modes", default="0,1,3,4",
                    help="precision modes to time (0 FP64, 1 FP32, 3/4 BF16 slices); FP64 always runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this library has no multi-GPU path "
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
    H = synth.bond_operator_real(synth.random_coefficients(6))
    ctx = ctm.Context(0)
    modes = [int(m) for m in args.modes.split(",")]
    if ctm.CTM_PREC_F64 not in modes:
        modes = [ctm.CTM_PREC_F64] + modes
    runs = {}
    for mode in modes:
        runs[mode] = run_mode(ctx, ctm, torch, A, B, H, D, chi, mode, args)
    ref = runs[ctm.CTM_PREC_F64]
    for mode, r in runs.items():
        r["err_kappa_vs_fp64"] = abs(r["kappa"] / ref["kappa"] - 1.0)
        r["err_energy_vs_fp64"] = abs(r["energy_bond"] - ref["energy_bond"])
        r["speedup_vs_fp64"] = ref["ms_per_move"] / r["ms_per_move"]
    structured = None
    if args.structured:
        structured = run_structured(ctx, ctm, torch, synth, H, D, chi, modes, args)
    head, bound, rule = select_headline(runs, structured)
    h = runs[head]
    dtype = MODE_NAMES[head]

    out = {
        "metric": "CTMRG move GFLOP/s (%MFMA peak), D=6 chi=72: mixed vs FP64 at <=1e-8 err",
        "value": round(h["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(4.0 * h["ms_per_move"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "rhombic-lattice CTMRG sweep of a random D=6 purification, chi=72 "
                               "(d=36, cut n=2592), seed 1234, after %d converging sweeps" % args.converge,
                   "D": D, "chi": chi, "d": d, "n": n, "gamma": "z",
                   "precision": PRECISION_TEXT[head],
                   "step": "one sweep = 4 absorption moves (L, R, U, D)"},
        "ms_per_move": round(h["ms_per_move"], 3),
        "error_bound_vs_fp64": bound,
        "headline_rule": rule,
        "err_kappa_vs_fp64": h["err_kappa_vs_fp64"],
        "err_energy_vs_fp64": h["err_energy_vs_fp64"],
        "structured_err_kappa_vs_fp64": (None if structured is None else
                                         structured[dtype]["err_kappa_vs_fp64"]),
        "structured_err_energy_vs_fp64": (None if structured is None else
                                          structured[dtype]["err_energy_vs_fp64"]),
        "executed_gflops": round(h["executed_gflops"], 2),
        "mixed_vs_fp64_speedup": round(h["speedup_vs_fp64"], 3),
        "fp64": {"value": round(ref["gflops"], 2), "ms_per_move": round(ref["ms_per_move"], 3),
                 "pct_fp64_mfma_peak_algorithmic": round(100.0 * ref["gflops"] / (PEAK_F64_TFLOPS * 1e3), 2),
                 "roofline": ref["roofline"]},
        "modes": {MODE_NAMES[m]: {k: _fmt(k, v) for k, v in r.items() if k != "roofline"}
                  for m, r in runs.items()},
        "roofline": h["roofline"],
        "fu_metric_ms": round(h["fu_ms"], 3),
        "kappa": h["kappa"],
        "energy_bond": h["energy_bond"],
    }
    if structured is not None:
        structured.pop("_errs")
        out["structured"] = structured
    if args.batch > 0:
        out["batch"] = run_batch(ctm, torch, synth, args.batch, 3, 2)
        out["batch_uniform"] = run_batch(ctm, torch, synth, args.batch, 3, 4, uniform=(4, 32))
    if args.grad > 0:
        out["grad"] = run_grad(ctm, synth, args.grad)
    if args.grad > 0:
        out["xi"] = run_xi(ctm, synth, 2)
    if args.fu > 0:
        out["fu"] = run_fu(ctm, synth, args.fu)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(D, chi, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
