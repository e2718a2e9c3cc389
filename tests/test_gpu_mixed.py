"""Mixed precision (SHGO_PREC_MIXED): the product-rule and shift coupling of every primitive pair in
binary32 double-float arithmetic (error-free transformations), the rest in binary64, against the
FP64 oracle.

Bar, derived from the arithmetic: the coupling's inputs are split into float pairs (about 2^-48
relative) and every double-float product and sum keeps about 2^-47 relative, so the block entries
carry a few hundred units of 2^-47 relative to the sum of their terms' magnitudes; the shift powers
t^(l-l1) cancel by up to 1e3 for l <= 4, which leaves about 1e-11 relative. The tests hold every
element to |V - V_oracle| <= 1e-13 + 1e-9 |V_oracle|, a hundredfold margin that is still ten times
tighter than the 1e-8 relative the mixed form is meant to keep. Classes with la > 4 keep the
binary64 coupling in the mixed kernel and are held to the FP64 bar.
"""
import numpy as np
import pytest

import helpers
import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL_MIXED, ATOL = 1e-9, 1e-13
RTOL_FP64 = 1e-11


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as s
    s.context(0)
    return s


def error_stats(got, ref, floor=1e-10):
    """Max and RMS absolute error, and max and RMS relative error over elements with |ref| > floor."""
    err = np.abs(got - ref)
    big = np.abs(ref) > floor
    rel = err[big] / np.abs(ref[big])
    return {"max_abs": float(err.max()), "rms_abs": float(np.sqrt(np.mean(err ** 2))),
            "max_rel": float(rel.max()) if rel.size else 0.0,
            "rms_rel": float(np.sqrt(np.mean(rel ** 2))) if rel.size else 0.0}


def assert_bar(got, ref, rtol, what):
    err = np.abs(got - ref)
    bad = err > ATOL + rtol * np.abs(ref)
    if bad.any():
        i = int(np.argmax(np.where(bad, err, -1)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} elements out of tolerance; worst at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r}")


def run_pairs(shgo, b, n, pa, pb, precision, screen=0.0):
    import torch
    plan = shgo.shgo_plan_pairs(shgo.context(0), b, n, pa, pb, screen)
    shgo.shgo_plan_set_precision(plan, precision)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_every_class_mixed(shgo):
    # 20 uncontracted pairs of every (la, lb) class, both orientations; the double-float coupling
    # for la, lb <= 4, the binary64 coupling above
    hb, hn, pa, pb = synth.high_l_sweep(seed=41, pairs_per_class=20)
    got = run_pairs(shgo, hb, hn, pa, pb, "mixed")
    blocks = oracle.split_blocks(oracle.nuc_blocks(hb, hn, pa, pb), hb, pa, pb)
    gblocks = oracle.split_blocks(got, hb, pa, pb)
    worst = {}
    for k in range(len(pa)):
        la, lb = int(hb.l[pa[k]]), int(hb.l[pb[k]])
        rtol = RTOL_MIXED if max(la, lb) <= 4 else RTOL_FP64
        assert_bar(gblocks[k], blocks[k], rtol, f"pair {k}, class ({la},{lb})")
        if max(la, lb) <= 4:
            r = np.abs(gblocks[k] - blocks[k]) / (np.abs(blocks[k]) + 1e-300)
            worst[(la, lb)] = max(worst.get((la, lb), 0.0), float(r[np.abs(blocks[k]) > 1e-10].max(initial=0.0)))
    print("max relative error per class (la, lb <= 4):", {k: f"{v:.1e}" for k, v in sorted(worst.items())})
    # the mixed form really runs different arithmetic from the FP64 form
    fp64 = run_pairs(shgo, hb, hn, pa, pb, "fp64")
    assert not np.array_equal(got, fp64)


def test_precision_switch_and_graph(shgo):
    import torch
    b, n = synth.molecule(seed=43, n_atoms=10, box=9.0, ls=(0, 1, 2, 3, 4), kmax=6)
    ref = oracle.nuc_matrix(b, n, screen=1e-12).reshape(-1)
    plan = shgo.shgo_plan_matrix(shgo.context(0), b, n, 1e-12)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    fp64 = out.cpu().numpy()
    assert_bar(fp64, ref, RTOL_FP64, "fp64 before the switch")
    shgo.shgo_plan_set_precision(plan, "mixed")
    for r in range(3):
        out.fill_(float("nan"))
        shgo.shgo_execute_graph(plan, out)
        torch.cuda.synchronize()
        mixed = out.cpu().numpy()
        assert_bar(mixed, ref, RTOL_MIXED, f"mixed graph replay {r}")
        assert np.array_equal(mixed.reshape(b.nbf(), -1), mixed.reshape(b.nbf(), -1).T)
    shgo.shgo_plan_set_precision(plan, "fp64")
    out.fill_(float("nan"))
    shgo.shgo_execute_graph(plan, out)
    torch.cuda.synchronize()
    back = out.cpu().numpy()
    # the FP64 form again (a fresh graph of the FP64 kernel), equal up to the rounding order of
    # the accumulator's atomic adds
    assert np.all(np.abs(back - fp64) <= 1e-13 + 1e-12 * np.abs(fp64))
    with pytest.raises(shgo.ShgoError) as e:
        shgo.shgo_plan_set_precision(plan, 7)
    assert e.value.status == shgo.SHGO_ERR_INVALID_ARG


def test_single_call_mixed(shgo):
    b, n = synth.small_molecule(seed=1)
    V = shgo.nuclear_attraction(b, n, precision="mixed").cpu().numpy()
    assert_bar(V, oracle.nuc_matrix(b, n), RTOL_MIXED, "4-atom s/p/d matrix, mixed")


def test_batched_workload_mixed_stratified(shgo):
    """The mixed-precision batched form at full size (the 200-atom molecule, l <= 4, K 1..8,
    screened 1e-12) in the bench's launch configuration (autotuned schedule): every pair that keeps
    48 or more primitive pairs, 40 kept pairs of each class and 40 fully screened ones against the
    oracle; the per-element error statistics are printed."""
    import torch
    b, n = synth.batched_molecule(seed=3)
    screen = 1e-12
    plan = shgo.shgo_plan_matrix(shgo.context(0), b, n, screen)
    shgo.shgo_plan_set_precision(plan, "mixed")
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    shgo.shgo_plan_autotune(plan, out, rounds=1)
    out.fill_(float("nan"))
    shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    nbf = b.nbf()
    V = out.cpu().numpy().reshape(nbf, nbf)
    assert not np.isnan(V).any()
    assert np.array_equal(V, V.T)
    pa, pb = synth.all_pairs(b.n_shells)
    ns = helpers.surviving_prim_pairs(b, pa, pb, screen)
    rng = np.random.default_rng(5)
    hi, lo = np.maximum(b.l[pa], b.l[pb]), np.minimum(b.l[pa], b.l[pb])
    sel = [np.nonzero(ns >= 48)[0]]
    for la in range(5):
        for lb in range(la + 1):
            cls = np.nonzero((hi == la) & (lo == lb) & (ns > 0))[0]
            sel.append(rng.choice(cls, min(40, len(cls)), replace=False))
    zero = rng.choice(np.nonzero(ns == 0)[0], 40, replace=False)
    sel = np.unique(np.concatenate(sel))
    ref = oracle.split_blocks(oracle.nuc_blocks(b, n, pa[sel], pb[sel], screen=screen), b, pa[sel], pb[sel])
    off = b.shell_offsets()
    blk = lambda a, c: V[off[a]:off[a] + 2 * b.l[a] + 1, off[c]:off[c] + 2 * b.l[c] + 1]  # noqa: E731
    got = np.concatenate([blk(pa[k], pb[k]).ravel() for k in sel])
    refv = np.concatenate([r.ravel() for r in ref])
    print(f"mixed batched, {len(sel)} pairs, {got.size} elements:", error_stats(got, refv))
    assert_bar(got, refv, RTOL_MIXED, f"{len(sel)} stratified pairs, mixed")
    for k in zero:
        assert np.all(blk(pa[k], pb[k]) == 0.0)
