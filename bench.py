#!/usr/bin/env python
"""Benchmark: contracted SHGO nuclear-attraction integrals/s on one MI355X (gfx950).

Workload (default): the high-l sweep -- 49 classes (l_a, l_b) in {0..6}^2 x 2041 uncontracted
shell pairs (100,009 pairs), exponents log-uniform [0.05, 100], centers uniform in a 10-bohr
cube, 64 point nuclei with Z in {1..10} (seed 2, ``synth.high_l_sweep``).

A step is one ``shgo_execute`` of a plan whose inputs already sit in HBM: primitive
normalisation, pair classification/screening/class sort, and every class kernel (Gaussian
product, shift, product rule, Boys, nucleus sum, contraction, scatter) -- all on the device.

Output: one JSON line on stdout. ``value`` = integrals/s over the K timed steps (HIP events on
the stream the library launches on, bracketed by device synchronisation). ``roofline`` refers
to the dominant class kernel, timed live with per-kernel HIP events recorded by the library
during the same timed steps; its algorithmic FLOPs come from the per-(primitive pair, nucleus)
and per-primitive-pair operation counts of the vector-coupling route (``model_flops``).
``cpu_baseline`` times the CPU oracle (all host threads) on a bounded, class-stratified sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contracted SHGO nuclear-attraction integrals/s at 1 GPU; % FP64 vector peak"
# MI355X: 256 CUs x 2.4 GHz x 64 lanes x 2 flops (FP64 FMA) per lane-cycle
FP64_VECTOR_PEAK = 256 * 2.4e9 * 64 * 2
NNZ_SHIFT = [1, 6, 21, 56, 117, 214, 353]  # nonzero real shift coefficients for l = 0..6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------------------------
# algorithmic operation counts (FP64 flops, FMA = 2, exp = 20)
# ----------------------------------------------------------------------------------------------
def _gaunt_nnz():
    sys.path.insert(0, os.path.join(ROOT, "paper_2404_16245_amd", "csrc"))
    import gen_classes
    g = gen_classes.real_gaunt_table()
    out = {}
    for la in range(7):
        for lb in range(7):
            out[(la, lb)] = int(np.count_nonzero(g[:(la + 1) ** 2, :(lb + 1) ** 2, :]))
    return out


def model_flops(la, lb, gaunt_nnz):
    """(flops per (primitive pair, nucleus), flops per primitive pair)."""
    kmin = min(la, lb)
    Lm = la + lb
    n_w = sum((Lm - 2 * k + 1) ** 2 for k in range(kmin + 1))              # W(L, M, k) entries
    n_lk = sum(1 + min(kmin, (Lm - L) // 2) for L in range(Lm + 1))          # (L, k) pairs
    nucleus = (9 + (20 + 14 + 3 * Lm) + kmin + 3 * n_lk + 4 * (Lm + 1) ** 2 + 2 * n_w)
    pair = (40 + n_w + 2 * gaunt_nnz[(la, lb)] + 4 * (la + 1) ** 2 + 4 * (lb + 1) ** 2
            + 2 * (NNZ_SHIFT[la] + NNZ_SHIFT[lb]) + 2 * NNZ_SHIFT[la] * (lb + 1) ** 2
            + 2 * (2 * la + 1) * NNZ_SHIFT[lb] + 2 * (2 * la + 1) * (2 * lb + 1))
    return nucleus, pair


def class_id(la, lb):
    a, b = max(la, lb), min(la, lb)
    return a * (a + 1) // 2 + b


def surviving_prim_pairs(basis, pa, pb, screen):
    """Primitive pairs per shell pair that pass exp(-ab/(a+b) |A-B|^2) > screen (all if screen = 0)."""
    ka = basis.nprim[pa].astype(np.int64)
    kb = basis.nprim[pb].astype(np.int64)
    if not screen > 0:
        return ka * kb
    n = ka * kb
    rep = np.repeat(np.arange(len(pa)), n)
    start = np.concatenate([[0], np.cumsum(n)[:-1]])
    local = np.arange(int(n.sum())) - np.repeat(start, n)
    i = local // np.repeat(kb, n)
    j = local % np.repeat(kb, n)
    ea = basis.expo[basis.prim_off[pa][rep] + i]
    eb = basis.expo[basis.prim_off[pb][rep] + j]
    R2 = np.sum((basis.center[pa] - basis.center[pb]) ** 2, axis=1)[rep]
    keep = np.exp(-ea * eb / (ea + eb) * R2) > screen
    return np.bincount(rep, weights=keep, minlength=len(pa)).astype(np.int64)


def workload_flops(basis, nuclei, pa, pb, screen=0.0):
    """Model flops per class id (primitive pairs after screening) and in total."""
    gn = _gaunt_nnz()
    la, lb = basis.l[pa].astype(np.int64), basis.l[pb].astype(np.int64)
    hi, lo = np.maximum(la, lb), np.minimum(la, lb)
    cid = hi * (hi + 1) // 2 + lo
    npp = surviving_prim_pairs(basis, np.asarray(pa), np.asarray(pb), screen)
    per_class = np.zeros(28)
    for c in np.unique(cid):
        a = int((np.sqrt(8 * c + 1) - 1) // 2)
        b = int(c - a * (a + 1) // 2)
        nucl, pair = model_flops(a, b, gn)
        per_class[c] = float(npp[cid == c].sum()) * (nuclei.n * nucl + pair)
    return per_class, float(per_class.sum())


# ----------------------------------------------------------------------------------------------
# HBM traffic from the committed rocprofv3 counter summary (null when the kernel has changed)
# ----------------------------------------------------------------------------------------------
def kernel_source_hash():
    h = hashlib.sha256()
    for rel in ("paper_2404_16245_amd/csrc/shgo.hip", "paper_2404_16245_amd/csrc/gen_classes.py"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_tag):
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ----------------------------------------------------------------------------------------------
# CPU baseline: the oracle on a class-stratified sample
# ----------------------------------------------------------------------------------------------
def cpu_baseline(basis, nuclei, pa, pb, target_s):
    import oracle
    la, lb = basis.l[pa], basis.l[pb]
    order = {}
    for c in sorted(set(zip(la.tolist(), lb.tolist()))):
        order[c] = np.nonzero((la == c[0]) & (lb == c[1]))[0]
    threads = os.cpu_count() or 1

    def sample(k):
        return np.concatenate([v[:k] for v in order.values()])

    pilot_k = 4
    s = sample(pilot_k)
    t0 = time.perf_counter()
    oracle.nuc_blocks(basis, nuclei, pa[s], pb[s], nthreads=threads)
    pilot = time.perf_counter() - t0
    per_pair_class = max(pilot / pilot_k, 1e-6)
    kmax = max(len(v) for v in order.values())
    k = int(min(kmax, max(pilot_k, target_s / per_pair_class)))
    s = sample(k)
    t0 = time.perf_counter()
    oracle.nuc_blocks(basis, nuclei, pa[s], pb[s], nthreads=threads)
    dt = time.perf_counter() - t0
    n_int = int(oracle.block_sizes(basis, pa[s], pb[s]).sum())
    return {"value": n_int / dt, "unit": "integrals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {k} pairs of each of the {len(order)} classes ({len(s)} pairs, {n_int} integrals, "
                      f"{dt:.1f} s wall, OpenMP over pairs)"}


# ----------------------------------------------------------------------------------------------
# the batched and gradient forms, measured beside the plain line
# ----------------------------------------------------------------------------------------------
def _time_ms(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure_batched(shgo, synth, torch, steps):
    """200-atom molecule (l <= 4, K 1..8, screened 1e-12), full V: autotuned schedule, one
    hipGraph-captured evaluation per step."""
    basis, nuclei = synth.batched_molecule(seed=3)
    screen = 1e-12
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    ms_eager = _time_ms(torch, lambda: shgo.shgo_execute(plan, out), steps, 2)
    tune_ms, chosen = shgo.shgo_plan_autotune(plan, out, rounds=5)
    ms = _time_ms(torch, lambda: shgo.shgo_execute_graph(plan, out), steps, 2)
    pa, pb = synth.all_pairs(basis.n_shells)
    _, flops = workload_flops(basis, nuclei, pa, pb, screen)
    return {"workload": "200 atoms, 20-bohr box, l=0..4, K uniform 1..8, screened exp(-mu R^2) > 1e-12, full V, "
                        "seed 3; autotuned schedule, hipGraph replay",
            "nbf": basis.nbf(), "integrals_per_step": plan.integrals, "ms_per_step": ms,
            "integrals_per_s": plan.integrals / (ms * 1e-3), "ms_per_step_eager_untuned": ms_eager,
            "tune_candidates_ms": [float(x) for x in tune_ms], "tune_chosen": chosen,
            "model_flops_per_step": flops, "fp64_model_tflops": flops / (ms * 1e-3) / 1e12,
            "fp64_vector_peak_frac": flops / (ms * 1e-3) / FP64_VECTOR_PEAK}


def measure_overlap(shgo, synth, torch, steps):
    """Overlap matrix S of the batched molecule's basis (nbf 5000, K 1..8), full matrix: the plan's
    pair build and the overlap kernel per step. Bound by writing S (8 nbf^2 bytes)."""
    basis, nuclei = synth.batched_molecule(seed=3)
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, 0.0)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    ms = _time_ms(torch, lambda: shgo.shgo_execute_overlap(plan, out), steps, 2)
    nbytes = 8.0 * plan.output_size
    return {"workload": "overlap S of the 200-atom batched molecule's basis (l=0..4, K 1..8), full matrix, seed 3",
            "nbf": basis.nbf(), "integrals_per_step": plan.integrals, "ms_per_step": ms,
            "integrals_per_s": plan.integrals / (ms * 1e-3), "output_bytes": nbytes,
            "output_GB_per_s": nbytes / (ms * 1e-3) / 1e9, "hbm_peak_frac": nbytes / (ms * 1e-3) / 8e12}


def measure_gradient(shgo, synth, torch, steps):
    """500-atom molecule (l <= 3, K 1..6, screened 1e-12): dE/dR_nuclei and dE/dR_centers of
    E = sum D V with a random symmetric D, by the adjoint kernel; the forward V beside it."""
    basis, nuclei = synth.gradient_molecule(seed=5)
    screen = 1e-12
    D = torch.as_tensor(synth.density(basis.nbf(), seed=5), device="cuda")
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
    dn = torch.empty((nuclei.n, 3), dtype=torch.float64, device="cuda")
    dc = torch.empty((basis.n_shells, 3), dtype=torch.float64, device="cuda")
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    ms_grad = _time_ms(torch, lambda: shgo.shgo_execute_grad(plan, D, dn, dc, e), steps, 1)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    ms_fwd = _time_ms(torch, lambda: shgo.shgo_execute(plan, out), steps, 1)
    total = (dn.sum(0) + dc.sum(0)).abs().max().item()
    scale = max(dn.abs().max().item(), dc.abs().max().item())
    return {"workload": "500 atoms, 30-bohr box, l=0..3, K uniform 1..6, screened 1e-12, D iid N(0, 0.1^2) "
                        "symmetric, seed 5", "nbf": basis.nbf(), "nuclei": nuclei.n,
            "ms_per_gradient": ms_grad, "ms_per_forward": ms_fwd, "energy": e.item(),
            "translation_sum_rule_rel": total / scale}


# ----------------------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="high_l_sweep", choices=["high_l_sweep", "small_molecule", "batched"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and gradient forms")
    ap.add_argument("--no-tune", action="store_true", help="time the model schedule, without autotuning")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run a plain device copy of this many bytes (calibrates HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1"}))
        log("bench.py: the path runs on one GPU per process; multi-GPU runs are not implemented (--gpus 1)")
        sys.exit(2)

    import torch
    import paper_2404_16245_amd as shgo
    from paper_2404_16245_amd import synth

    if not torch.cuda.is_available():
        log("bench.py: no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")
    ctx = shgo.context(0)

    screen = 0.0
    if args.workload == "high_l_sweep":
        basis, nuclei, pa, pb = synth.high_l_sweep(seed=2)
        plan = shgo.shgo_plan_pairs(ctx, basis, nuclei, pa, pb, screen)
        desc = ("high-l sweep: 49 (l_a,l_b) classes x 2041 uncontracted shell pairs, l<=6, exponents "
                "log-uniform [0.05,100], 10-bohr cube, 64 nuclei Z in 1..10, seed 2")
        cfg = {"workload": desc, "shell_pairs": int(len(pa)), "nuclei": nuclei.n, "classes": 49, "seed": 2}
    elif args.workload == "small_molecule":
        basis, nuclei = synth.small_molecule(seed=1)
        pa, pb = synth.all_pairs(basis.n_shells)
        plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
        desc = "4 atoms in a 6-bohr cube, s/p/d shells with 3 primitives, full V matrix, seed 1"
        cfg = {"workload": desc, "nbf": basis.nbf(), "nuclei": nuclei.n, "seed": 1}
    else:
        basis, nuclei = synth.batched_molecule(seed=3)
        pa, pb = synth.all_pairs(basis.n_shells)
        screen = 1e-12
        plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
        desc = ("200 atoms in a 20-bohr box, shells l=0..4, K uniform 1..8, screened exp(-mu R^2) > 1e-12, "
                "full V matrix, seed 3")
        cfg = {"workload": desc, "nbf": basis.nbf(), "nuclei": nuclei.n, "seed": 3}

    out = torch.empty(plan.output_size, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    tune = None
    if not args.no_tune:
        # one-time schedule tuning of the plan (not part of the timed steps)
        ms_c, chosen = shgo.shgo_plan_autotune(plan, out, rounds=5)
        weights, slices = shgo.shgo_plan_get_schedule(plan)
        tune = {"candidates_ms": [float(x) for x in ms_c], "chosen": chosen,
                "tiles_per_item": {int(c): int(v) for c, v in enumerate(slices)}}
    if args.copy_bytes > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the kernel's
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"bench: {args.workload}, {plan.integrals} integrals per step, warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()

    shgo.shgo_plan_set_timing(plan, args.steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        shgo.shgo_execute(plan, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    phase_ms, nrec = shgo.shgo_plan_phase_ms(plan)
    shgo.shgo_plan_set_timing(plan, 0)
    ms_per_step = total_ms / args.steps
    value = plan.integrals * args.steps / (total_ms * 1e-3)
    log(f"bench: {ms_per_step:.4f} ms/step, {value:.4e} integrals/s")

    per_class_flops, total_flops = workload_flops(basis, nuclei, pa, pb, screen)
    avg_phase_ms = phase_ms / max(nrec, 1)
    kern_s = avg_phase_ms[1] * 1e-3
    achieved = total_flops / kern_s / 1e12
    tag = f"k_integrals_{args.workload}"
    traffic = traffic_from_profile(tag)
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / (FP64_VECTOR_PEAK / 1e12), "traffic": traffic,
                "kernel": "k_integrals (persistent, every class)", "kernel_ms": avg_phase_ms[1],
                "model_flops_per_launch": total_flops}
    step_tflops = total_flops / (ms_per_step * 1e-3) / 1e12
    res = {"metric": METRIC, "value": value, "unit": "integrals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
           "integrals_per_step": plan.integrals,
           "fp64_model_tflops": step_tflops, "fp64_vector_peak_frac": step_tflops / (FP64_VECTOR_PEAK / 1e12),
           "pair_build_ms": avg_phase_ms[0], "roofline": roofline, "schedule_tuning": tune}
    if not args.no_forms and args.workload == "high_l_sweep":
        log("bench: batched form")
        res["batched"] = measure_batched(shgo, synth, torch, max(3, args.steps // 2))
        log("bench: gradient form")
        res["gradient"] = measure_gradient(shgo, synth, torch, 3)
        log("bench: overlap form")
        res["overlap"] = measure_overlap(shgo, synth, torch, 5)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(basis, nuclei, pa, pb, args.cpu_seconds)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
