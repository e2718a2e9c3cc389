#!/usr/bin/env python
"""Benchmark: contracted SHGO nuclear-attraction integrals/s on one MI355X (gfx950).

Workload (default): the batched molecule -- 200 atoms in a 20-bohr box, one shell per l = 0..4 per
atom, K uniform 1..8 primitives, exponents log-uniform [0.1, 50], Z in 1..8, primitive pairs
screened by exp(-mu R^2) > 1e-12, the full V matrix (nbf 5000), seed 3 (``synth.batched_molecule``).

A step is one ``shgo_execute`` of a plan whose inputs already sit in HBM: primitive
normalisation, pair classification/screening/class sort, and the persistent integral kernel
(Gaussian product, shift, product rule, Boys, nucleus sum, contraction, scatter over every class)
-- all on the device. The plan is autotuned once before the timed steps.

Output: one JSON line on stdout. ``value`` = integrals/s over the K timed steps (HIP events on the
stream the library launches on, bracketed by device synchronisation); integrals count the shell
pairs that keep a primitive pair, (2la+1)(2lb+1) each. ``roofline`` refers to the integral kernel,
timed live with HIP events the library records around its launch on the same stream during the
same timed steps; its algorithmic FLOPs come from the per-(primitive pair, nucleus) and
per-primitive-pair operation counts of the vector-coupling route (``model_flops``) over the
surviving primitive pairs. ``cpu_baseline`` times the CPU oracle on a class-stratified random
sample of the same workload's kept shell pairs, with every host thread (and, beside it, one
thread). Extra blocks: the high-l sweep (49 (l_a, l_b) classes x 2041 uncontracted pairs, each
class also timed alone), the gradient, and the overlap matrix.
"""
import argparse
import re
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


def _count_ops(code):
    """FP64 flops of generated straight-line code: fma = 2, any other binary + - * = 1 (index
    arithmetic and the adjoint-table pointers excluded)."""
    n = 0
    for line in code.splitlines():
        line = re.sub(r"//.*$", "", line)
        line = re.sub(r"const double\* w = adj \+ \d+;", "", line)
        line = re.sub(r"\[[^\]]*\]", "", line)
        n += 2 * line.count("fma(")
        prev = None
        for t in re.findall(r"[A-Za-z_][A-Za-z_0-9.]*|\d+\.\d*(?:e-?\d+)?|\d+|[-+*/=(),;{}<>]", line):
            if t == "*" or (t in "+-" and prev is not None and (re.match(r"[A-Za-z_0-9.]", prev) or prev == ")")):
                n += 1
            prev = t
    return n


def grad_model_flops(la, lb):
    """(flops per (primitive pair, nucleus), flops per primitive pair) of the adjoint gradient:
    the generated adjoint nucleus step (solid harmonics and their gradients, G and dG/dT per entry,
    five products per W entry, eight accumulators) counted from its code, plus the nucleus's frame
    geometry, Boys F_0..F_{la+lb+1} as in the forward model, the gradient assembly and the three
    nuclear-gradient adds; per primitive pair the adjoint quadruples (2 products and 1 or 3 FMAs
    per coupling term of classes (la, lb), (la-1, lb), (la, lb-1), 25 per entry) and 60 for P, K
    and the shift powers."""
    sys.path.insert(0, os.path.join(ROOT, "paper_2404_16245_amd", "csrc"))
    import gen_classes
    t = gen_classes.emit_grad(la, lb)
    i = t.index("void step(")
    body = t[t.index("{", t.index("acc)[8]", i)):t.index("\n  }\n", i)]
    lm, kmin = la + lb, min(la, lb)
    nucleus = _count_ops(body) + 3 + 13 + 5 + 1 + (20 + 14 + 3 * (lm + 2)) + 2 * kmin + 14 + 6 + 2 + 18
    terms = gen_classes.grad_tables(la, lb)
    pair = 60 + 25 * len(gen_classes.grad_entries(la, lb)) + sum(4 if t[0] == 0 else 8 for t in terms)
    return nucleus, pair


def gradient_flops(basis, nuclei, pa, pb, screen):
    """Model flops of one gradient evaluation over the kept primitive pairs of every class."""
    la, lb = basis.l[pa].astype(np.int64), basis.l[pb].astype(np.int64)
    hi, lo = np.maximum(la, lb), np.minimum(la, lb)
    npp = surviving_prim_pairs(basis, np.asarray(pa), np.asarray(pb), screen)
    total = 0.0
    for a in range(int(hi.max()) + 1):
        for b in range(a + 1):
            m = (hi == a) & (lo == b)
            if m.any():
                nucl, pair = grad_model_flops(a, b)
                total += float(npp[m].sum()) * (nuclei.n * nucl + pair)
    return total


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
KERNEL_SOURCES = ("paper_2404_16245_amd/csrc/shgo_integrals.hip", "paper_2404_16245_amd/csrc/shgo_integrals_kernel.h",
                  "paper_2404_16245_amd/csrc/shgo_internal.h", "paper_2404_16245_amd/csrc/schedule.h",
                  "paper_2404_16245_amd/csrc/gen_classes.py")


def kernel_source_hash():
    """Hash of the sources the integral kernel is compiled from."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
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
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(basis, nuclei, pa, pb, screen, target_s, threads):
    """The oracle on a class-stratified random sample of the kept shell pairs: the same fraction of
    every (la, lb) class, sized by a pilot run to about target_s seconds. Returns (integrals/s,
    sample description, seconds)."""
    import oracle
    keep = surviving_prim_pairs(basis, pa, pb, screen) > 0
    la, lb = basis.l[pa], basis.l[pb]
    cls = np.maximum(la, lb) * 16 + np.minimum(la, lb)
    rng = np.random.default_rng(2024)
    groups = [rng.permutation(np.nonzero(keep & (cls == c))[0]) for c in np.unique(cls[keep])]

    def sample(frac):
        return np.concatenate([g[:max(1, int(round(frac * len(g))))] for g in groups])

    def run(sel):
        t0 = time.perf_counter()
        oracle.nuc_blocks(basis, nuclei, pa[sel], pb[sel], screen=screen, nthreads=threads)
        return time.perf_counter() - t0

    pilot = 0.002
    dt = run(sample(pilot))
    frac = float(min(1.0, max(pilot, pilot * target_s / max(dt, 1e-3))))
    sel = sample(frac)
    dt = run(sel)
    n_int = int(oracle.block_sizes(basis, pa[sel], pb[sel]).sum())
    desc = (f"{100 * frac:.2f}% of the kept shell pairs of each of the {len(groups)} (la,lb) classes, drawn at "
            f"random ({len(sel)} pairs, {n_int} integrals, {dt:.1f} s wall, {threads} OpenMP thread(s) over pairs)")
    return n_int / dt, desc, dt


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


def timed_steps(shgo, torch, plan, out, steps, warmup):
    """K timed executions of a plan (after W warm ones) with the library's phase timers on: (ms per
    step from events around the loop, mean ms of phase 0 (pair build) and phase 1 (integral
    kernel) from the events the library records around its launches on the same stream)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    shgo.shgo_plan_set_timing(plan, steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        shgo.shgo_execute(plan, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    phase_ms, nrec = shgo.shgo_plan_phase_ms(plan)
    shgo.shgo_plan_set_timing(plan, 0)
    return total_ms / steps, phase_ms / max(nrec, 1)


SWEEP_CLASS_COPIES = 32


def measure_sweep(shgo, synth, torch, steps):
    """The high-l sweep (49 (la, lb) classes x 2041 uncontracted pairs, 64 nuclei, seed 2): all
    classes in one autotuned plan, then each (la, lb) class alone, in a plan of its own pairs listed
    SWEEP_CLASS_COPIES times (2041 pairs are 32 tiles, too few to occupy 256 compute units)."""
    basis, nuclei, pa, pb = synth.high_l_sweep(seed=2)
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_pairs(ctx, basis, nuclei, pa, pb, 0.0)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    shgo.shgo_plan_autotune(plan, out, rounds=5)
    ms, ph = timed_steps(shgo, torch, plan, out, steps, 3)
    per_class_flops, flops = workload_flops(basis, nuclei, pa, pb, 0.0)
    res = {"workload": "high-l sweep: 49 (l_a,l_b) classes x 2041 uncontracted shell pairs, l<=6, exponents "
                       "log-uniform [0.05,100], 10-bohr cube, 64 nuclei Z in 1..10, seed 2; autotuned",
           "integrals_per_step": plan.integrals, "ms_per_step": ms, "integrals_per_s": plan.integrals / (ms * 1e-3),
           "kernel_ms": ph[1], "pair_build_ms": ph[0], "model_flops_per_launch": flops,
           "kernel_fp64_peak_frac": flops / (ph[1] * 1e-3) / FP64_VECTOR_PEAK, "per_class": []}
    gn = _gaunt_nnz()
    for la in range(7):
        for lb in range(7):
            sel = np.tile(np.nonzero((basis.l[pa] == la) & (basis.l[pb] == lb))[0], SWEEP_CLASS_COPIES)
            p1 = shgo.shgo_plan_pairs(ctx, basis, nuclei, pa[sel], pb[sel], 0.0)
            o1 = torch.empty(p1.output_size, dtype=torch.float64, device="cuda")
            ms1, ph1 = timed_steps(shgo, torch, p1, o1, 20, 3)
            nucl, pair = model_flops(max(la, lb), min(la, lb), gn)
            f1 = len(sel) * (nuclei.n * nucl + pair)
            res["per_class"].append({"la": la, "lb": lb, "pairs": int(len(sel)), "copies": SWEEP_CLASS_COPIES,
                                     "integrals": p1.integrals,
                                     "ms_per_step": ms1, "kernel_ms": ph1[1],
                                     "integrals_per_s": p1.integrals / (ms1 * 1e-3),
                                     "kernel_fp64_peak_frac": f1 / (ph1[1] * 1e-3) / FP64_VECTOR_PEAK})
            del p1, o1
    return res


def measure_mixed(shgo, synth, torch, steps):
    """The batched molecule in mixed precision (the coupling in binary32 double-float arithmetic),
    autotuned like the FP64 line: time per V, and the per-element difference from the FP64 path's
    V (itself within 1e-11 relative of the oracle; the tests compare the mixed V with the oracle)."""
    basis, nuclei = synth.batched_molecule(seed=3)
    ctx = shgo.context(0)
    plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, 1e-12)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    ref = out.clone()
    shgo.shgo_plan_set_precision(plan, "mixed")
    shgo.shgo_plan_autotune(plan, out, rounds=5)
    ms, ph = timed_steps(shgo, torch, plan, out, steps, 3)
    err = (out - ref).abs()
    big = ref.abs() > 1e-10
    rel = err[big] / ref.abs()[big]
    large = ref.abs() > 1e-6 * ref.abs().max()
    rel_large = (err[large] / ref.abs()[large]).max().item()
    return {"workload": "batched molecule (as the headline), coupling in binary32 double-float arithmetic; "
                        "Boys, exp(-mu R^2), prefactors, nucleus sums and the contraction in binary64",
            "integrals_per_step": plan.integrals, "ms_per_step": ms, "integrals_per_s": plan.integrals / (ms * 1e-3),
            "kernel_ms": ph[1], "pair_build_ms": ph[0],
            "vs_fp64_path": {"max_abs": err.max().item(), "rms_abs": err.pow(2).mean().sqrt().item(),
                             "max_rel": rel.max().item(), "rms_rel": rel.pow(2).mean().sqrt().item(),
                             "rel_floor": 1e-10, "max_rel_above_1e-6_of_max": rel_large}}


def measure_cartesian(shgo, synth, torch, steps):
    """The same V by the Cartesian (McMurchie-Davidson) route on the same GPU: the batched molecule
    (l <= 4) and the gradient form's 500-atom molecule (l <= 3), each beside the solid-harmonic
    route on the same plan (eager launches, the default schedule, and the autotuned one)."""
    out = {}
    for name, (basis, nuclei) in (("batched_molecule", synth.batched_molecule(seed=3)),
                                  ("gradient_molecule", synth.gradient_molecule(seed=5))):
        ctx = shgo.context(0)
        plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, 1e-12)
        v = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
        ms_cart = _time_ms(torch, lambda: shgo.shgo_execute_cartesian(plan, v), max(2, steps // 4), 1)
        vc = v.clone()
        ms_shgo = _time_ms(torch, lambda: shgo.shgo_execute(plan, v), steps, 2)
        shgo.shgo_plan_autotune(plan, v, rounds=3)
        ms_tuned = _time_ms(torch, lambda: shgo.shgo_execute(plan, v), steps, 2)
        d = (vc - v).abs().max().item() / v.abs().max().item()
        out[name] = {"nbf": basis.nbf(), "integrals_per_step": plan.integrals, "ms_cartesian": ms_cart,
                     "ms_solid_harmonic": ms_shgo, "ms_solid_harmonic_tuned": ms_tuned,
                     "speedup": ms_cart / ms_shgo, "speedup_tuned": ms_cart / ms_tuned,
                     "max_diff_rel_to_max": d}
    return out


def unique_quartets(n_shells):
    """Shell quartets (a, b, c, d) with a >= b, c >= d and pair (a, b) >= pair (c, d): one of each
    set of quartets that the eightfold permutational symmetry of (ab|cd) relates."""
    a, b = np.tril_indices(n_shells)
    i, j = np.tril_indices(len(a))
    return np.stack([a[i], b[i], a[j], b[j]], axis=1).astype(np.int32)


def eri_workload(synth):
    return synth.molecule(seed=7, n_atoms=10, box=8.0, ls=(0, 1, 2), kmax=3)


def eri_cpu_baseline(synth, n_sample=200):
    """The two-electron oracle on one thread over a sample of the same unique quartets."""
    from oracle import eri as eri_oracle
    basis, _ = eri_workload(synth)
    q = unique_quartets(len(basis.l))
    sel = q[np.random.default_rng(7).choice(len(q), n_sample, replace=False)]
    t0 = time.perf_counter()
    for quartet in sel:
        eri_oracle.eri_block(basis, *quartet)
    dt = time.perf_counter() - t0
    n = int(np.prod(2 * np.asarray(basis.l)[sel] + 1, axis=1).sum())
    return {"value": n / dt, "unit": "integrals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} of the unique quartets of the two-electron workload"}


def eri_model_flops(basis, quartets):
    """Model FP64 flops of k_eri over a quartet list of pair classes (la, lb), (lc, ld) (each pair
    with its higher l first). Per primitive quartet: Y += K_cd I B'_ket^T (2 NW1 NW2 NCD + 2 NW1 NCD),
    the two-center matrix (3 per Gaunt term of every entry), the h table (per entry L + n + 19),
    Boys values (16 + 3 LT + 30) and solid harmonics (5 (LT+1)^2), and 30 for the pair geometry.
    Per bra primitive pair: the block += K_ab B'_bra Y (2 NAB NW1 NCD + 2 NAB NCD). The pair
    records' build is not counted."""
    sys.path.insert(0, os.path.join(ROOT, "paper_2404_16245_amd", "csrc"))
    import gen_classes
    G = gen_classes.real_gaunt_table()
    ents = {}
    for la in range(3):
        for lb in range(la + 1):
            ents[(la, lb)] = gen_classes.eri_class_tables(la, lb)[0]
    gn = (np.abs(G) > gen_classes.KEEP).sum(axis=2)
    per = {}

    def flops(c1, c2):
        if (c1, c2) not in per:
            e1, e2 = ents[c1], ents[c2]
            nab, ncd = (2 * c1[0] + 1) * (2 * c1[1] + 1), (2 * c2[0] + 1) * (2 * c2[1] + 1)
            i1 = [L * L + M + L for (L, M, k) in e1]
            i2 = [L * L + M + L for (L, M, k) in e2]
            terms = int(gn[np.ix_(i1, i2)].sum())
            lt = sum(c1) + sum(c2)
            h = sum(L + n + 19 for L in range(lt + 1) for n in range((lt - L) // 2 + 1))
            nw1, nw2 = len(e1), len(e2)
            per[(c1, c2)] = (2 * nw1 * nw2 * ncd + 2 * nw1 * ncd + 3 * terms + h + 16 + 3 * lt + 30
                             + 5 * (lt + 1) ** 2 + 30, 2 * nab * nw1 * ncd + 2 * nab * ncd)
        return per[(c1, c2)]
    ls, npr = np.asarray(basis.l), np.asarray(basis.nprim)
    total = 0.0
    for q in np.asarray(quartets):
        la, lb, lc, ld = (int(ls[x]) for x in q)
        c1, c2 = (max(la, lb), min(la, lb)), (max(lc, ld), min(lc, ld))
        f_pq, f_bra = flops(c1, c2)
        nb = float(npr[q[0]] * npr[q[1]])
        total += nb * float(npr[q[2]] * npr[q[3]]) * f_pq + nb * f_bra
    return total


def measure_eri(shgo, synth, torch, steps):
    """Two-electron blocks (ab|cd) of every unique shell quartet of a 10-atom molecule (shells
    s, p, d on each atom, K 1..3), one call per step: the upload of the quartet list, the pair
    weights and the kernel, waited for."""
    basis, _ = eri_workload(synth)
    q = unique_quartets(len(basis.l))
    ls = np.asarray(basis.l)
    n_int = int(np.prod(2 * ls[q] + 1, axis=1).sum())
    prim = np.asarray(basis.nprim)
    n_prim_q = int(np.prod(prim[q], axis=1).sum())
    flops = eri_model_flops(basis, q)
    shgo.eri_blocks(basis, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        shgo.eri_blocks(basis, q)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"workload": "every unique quartet of a 10-atom molecule (s, p, d shells, K 1..3), seed 7",
            "n_shells": int(len(ls)), "quartets": int(len(q)), "primitive_quartets": n_prim_q,
            "integrals_per_step": n_int, "ms_per_step": ms, "integrals_per_s": n_int / (ms * 1e-3),
            "primitive_quartets_per_s": n_prim_q / (ms * 1e-3), "model_flops_per_step": flops,
            "fp64_model_tflops": flops / (ms * 1e-3) / 1e12,
            "fp64_vector_peak_frac": flops / (ms * 1e-3) / FP64_VECTOR_PEAK}


def measure_overlap(shgo, synth, torch, steps):
    """Overlap matrix S of the batched molecule's basis (nbf 5000, K 1..8), full matrix: the overlap
    kernels per step (a matrix plan's overlap enumerates its pairs without the pair build; the
    contraction weights are computed when the plan is made). Bound by writing S (8 nbf^2 bytes)."""
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
    pa, pb = synth.all_pairs(basis.n_shells)
    flops = gradient_flops(basis, nuclei, pa, pb, screen)
    return {"workload": "500 atoms, 30-bohr box, l=0..3, K uniform 1..6, screened 1e-12, D iid N(0, 0.1^2) "
                        "symmetric, seed 5", "nbf": basis.nbf(), "nuclei": nuclei.n,
            "ms_per_gradient": ms_grad, "ms_per_forward": ms_fwd, "gradient_over_forward": ms_grad / ms_fwd,
            "model_flops_per_gradient": flops, "fp64_vector_peak_frac": flops / (ms_grad * 1e-3) / FP64_VECTOR_PEAK,
            "energy": e.item(), "translation_sum_rule_rel": total / scale}


# ----------------------------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_molecule",
                    choices=["batched_molecule", "high_l_sweep", "small_molecule"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the sweep, gradient and overlap blocks")
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
    if args.workload == "batched_molecule":
        basis, nuclei = synth.batched_molecule(seed=3)
        pa, pb = synth.all_pairs(basis.n_shells)
        screen = 1e-12
        plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
        info = shgo.shgo_plan_get_info(plan)
        desc = ("batched molecule: 200 atoms in a 20-bohr box, shells l=0..4 per atom, K uniform 1..8, exponents "
                "log-uniform [0.1,50], Z in 1..8, screened exp(-mu R^2) > 1e-12, full V matrix, seed 3")
        cfg = {"workload": desc, "nbf": basis.nbf(), "atoms": nuclei.n, "shell_pairs": info["candidate_pairs"],
               "shell_pairs_kept": info["kept_pairs"], "prim_pairs_kept": info["kept_prim_pairs"], "screen": screen,
               "seed": 3}
    elif args.workload == "high_l_sweep":
        basis, nuclei, pa, pb = synth.high_l_sweep(seed=2)
        plan = shgo.shgo_plan_pairs(ctx, basis, nuclei, pa, pb, screen)
        desc = ("high-l sweep: 49 (l_a,l_b) classes x 2041 uncontracted shell pairs, l<=6, exponents "
                "log-uniform [0.05,100], 10-bohr cube, 64 nuclei Z in 1..10, seed 2")
        cfg = {"workload": desc, "shell_pairs": int(len(pa)), "nuclei": nuclei.n, "classes": 49, "seed": 2}
    else:
        basis, nuclei = synth.small_molecule(seed=1)
        pa, pb = synth.all_pairs(basis.n_shells)
        plan = shgo.shgo_plan_matrix(ctx, basis, nuclei, screen)
        desc = "4 atoms in a 6-bohr cube, s/p/d shells with 3 primitives, full V matrix, seed 1"
        cfg = {"workload": desc, "nbf": basis.nbf(), "nuclei": nuclei.n, "seed": 1}

    out = torch.empty(plan.output_size, dtype=torch.float64, device=dev)
    tune = None
    if not args.no_tune:
        # one-time schedule tuning of the plan (not part of the timed steps)
        ms_c, chosen = shgo.shgo_plan_autotune(plan, out, rounds=5)
        _, tiles = shgo.shgo_plan_get_schedule(plan)
        tune = {"candidates_ms": [float(x) for x in ms_c], "chosen": chosen,
                "tiles_per_item": {int(c): int(v) for c, v in enumerate(tiles)}}
    if args.copy_bytes > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters calibrate the kernel's
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"bench: {args.workload}, {plan.integrals} integrals per step, warmup {args.warmup}, steps {args.steps}")
    ms_per_step, phase = timed_steps(shgo, torch, plan, out, args.steps, args.warmup)
    value = plan.integrals / (ms_per_step * 1e-3)
    log(f"bench: {ms_per_step:.4f} ms/step, {value:.4e} integrals/s")

    _, total_flops = workload_flops(basis, nuclei, pa, pb, screen)
    kern_s = phase[1] * 1e-3
    achieved = total_flops / kern_s / 1e12
    tag = f"k_integrals_{args.workload}"
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved / (FP64_VECTOR_PEAK / 1e12), "traffic": traffic_from_profile(tag),
                "kernel": "k_integrals (persistent, every class)", "kernel_ms": phase[1],
                "model_flops_per_launch": total_flops}
    step_tflops = total_flops / (ms_per_step * 1e-3) / 1e12
    res = {"metric": METRIC, "value": value, "unit": "integrals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
           "integrals_per_step": plan.integrals, "fp64_model_tflops": step_tflops,
           "fp64_vector_peak_frac": step_tflops / (FP64_VECTOR_PEAK / 1e12), "pair_build_ms": phase[0],
           "roofline": roofline, "schedule_tuning": tune}
    if not args.no_forms:
        del out
        log("bench: high-l sweep, all classes and each class alone")
        res["high_l_sweep"] = measure_sweep(shgo, synth, torch, args.steps)
        log("bench: mixed-precision form")
        res["mixed_precision"] = measure_mixed(shgo, synth, torch, args.steps)
        log("bench: Cartesian route")
        res["cartesian_route"] = measure_cartesian(shgo, synth, torch, args.steps)
        log("bench: gradient form")
        res["gradient"] = measure_gradient(shgo, synth, torch, 3)
        log("bench: overlap form")
        res["overlap"] = measure_overlap(shgo, synth, torch, 5)
        log("bench: two-electron blocks")
        res["two_electron"] = measure_eri(shgo, synth, torch, 3)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        # the host's share of cores (OMP_NUM_THREADS where the launcher sets it, else at most 16)
        threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or min(16, os.cpu_count() or 1)
        v, desc_s, _ = cpu_baseline(basis, nuclei, pa, pb, screen, args.cpu_seconds, threads)
        v1, desc_1, _ = cpu_baseline(basis, nuclei, pa, pb, screen, args.cpu_seconds / 2, 1)
        res["cpu_baseline"] = {"value": v, "unit": "integrals/s", "cores": threads, "kind": "oracle",
                               "sample": desc_s, "cpu_model": cpu_model(), "value_1_thread": v1,
                               "sample_1_thread": desc_1}
        if "two_electron" in res:
            res["cpu_baseline"]["two_electron"] = eri_cpu_baseline(synth)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
