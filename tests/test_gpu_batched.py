"""Batched launch: graph capture, tiles per work item, schedules and the autotuner, on screened
contracted molecules, against the oracle."""
import numpy as np
import pytest

import helpers
import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-11, 1e-13
NC = 36  # (la, lb) classes, la >= lb, l <= 7


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as m
    m.load_library()
    return m


def assert_parity(got, ref, what):
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), f"{what}: {int(bad.sum())} elements off, max abs err {err.max():.3e}"


def _plan(shgo, b, n, screen):
    import torch
    plan = shgo.shgo_plan_matrix(shgo.context(0), b, n, screen)
    out = torch.empty(plan.output_size, dtype=torch.float64, device="cuda")
    return plan, out


@pytest.fixture(scope="module")
def molecule():
    b, n = synth.molecule(seed=61, n_atoms=12, box=9.0, ls=(0, 1, 2, 3, 4), kmax=6)
    return b, n, oracle.nuc_matrix(b, n, screen=1e-12).reshape(-1)


def test_graph_replays_match_eager(shgo, molecule):
    import torch
    b, n, ref = molecule
    plan, out_e = _plan(shgo, b, n, 1e-12)
    shgo.shgo_execute(plan, out_e)
    torch.cuda.synchronize()
    eager = out_e.cpu().numpy()
    assert_parity(eager, ref, "eager")
    out_g = torch.full_like(out_e, float("nan"))
    other = torch.empty_like(out_e)
    for r in range(3):
        shgo.shgo_execute_graph(plan, out_g)
        torch.cuda.synchronize()
        got = out_g.cpu().numpy()
        assert not np.isnan(got).any(), f"replay {r}: {int(np.isnan(got).sum())} elements not written"
        # the integral kernel adds group contributions atomically: equal up to rounding order
        d = np.abs(got - eager)
        assert np.all(d <= 1e-13 + 1e-12 * np.abs(eager)), f"replay {r}: max diff {d.max():.3e}"
        assert_parity(got, ref, f"replay {r}")
        out_g.fill_(float("nan"))
        shgo.shgo_execute(plan, other)  # eager work between replays
        torch.cuda.synchronize()
        assert_parity(other.cpu().numpy(), ref, f"eager after replay {r}")


@pytest.mark.parametrize("tiles", ["one", "max", "mixed"])
def test_tiles_per_item_and_weights(shgo, molecule, tiles):
    import torch
    b, n, ref = molecule
    plan, out = _plan(shgo, b, n, 1e-12)
    tmax = np.array([shgo.shgo_max_tiles(c) for c in range(NC)], np.int32)
    t = {"one": np.ones(NC, np.int32), "max": tmax,
         "mixed": np.minimum(tmax, np.arange(NC, dtype=np.int32) % 3 + 1)}[tiles]
    # any positive weights give the same integrals; they only order the work items
    weight = np.random.default_rng(len(tiles)).uniform(1.0, 1e6, NC).astype(np.float32)
    shgo.shgo_plan_set_schedule(plan, weight, t)
    w2, t2 = shgo.shgo_plan_get_schedule(plan)
    assert np.array_equal(w2, weight) and np.array_equal(t2, t)
    shgo.shgo_execute(plan, out)
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), ref, f"tiles {tiles}")


def test_schedule_validation(shgo, molecule):
    b, n, _ = molecule
    plan, _ = _plan(shgo, b, n, 1e-12)
    ones = np.ones(NC, np.float32)
    for w in (np.zeros(NC, np.float32), np.full(NC, np.nan, np.float32), np.full(NC, 2e6, np.float32)):
        with pytest.raises(shgo.ShgoError) as e:
            shgo.shgo_plan_set_schedule(plan, w, np.ones(NC, np.int32))
        assert e.value.status == shgo.SHGO_ERR_INVALID_ARG
    with pytest.raises(shgo.ShgoError) as e:
        shgo.shgo_plan_set_schedule(plan, ones, np.full(NC, 8, np.int32))
    assert e.value.status == shgo.SHGO_ERR_INVALID_ARG  # (6,6) blocks allow one tile per item
    with pytest.raises(shgo.ShgoError) as e:
        shgo.shgo_plan_set_schedule(plan, ones, np.zeros(NC, np.int32))
    assert e.value.status == shgo.SHGO_ERR_INVALID_ARG


def test_autotune_keeps_results(shgo, molecule):
    import torch
    b, n, ref = molecule
    plan, out = _plan(shgo, b, n, 1e-12)
    ms, chosen = shgo.shgo_plan_autotune(plan, out, rounds=2)
    assert 0 <= chosen < shgo.SHGO_TUNE_CANDIDATES and np.all(ms > 0)
    assert ms[chosen] == ms.min()
    # the installed schedule (the kept candidate after the per-class refinement) is a valid one
    w, t = shgo.shgo_plan_get_schedule(plan)
    tmax = np.array([shgo.shgo_max_tiles(c) for c in range(NC)])
    assert np.all((t >= 1) & (t <= tmax)) and np.all((w >= 1.0) & (w <= 1e6))
    out.fill_(float("nan"))
    shgo.shgo_execute_graph(plan, out)
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), ref, "after tuning, graph")


def test_batched_workload_stratified(shgo):
    """The batched workload at full size (200 atoms, l <= 4, K <= 8, screened 1e-12) in the bench's
    launch configuration (autotuned schedule, graph replay): every pair that keeps 48 or more
    primitive pairs (the longest work items), 40 kept pairs of each (la, lb) class and 40 fully
    screened ones against the oracle, element by element; exact symmetry; zero blocks where
    nothing survives."""
    import torch
    b, n = synth.batched_molecule(seed=3)
    screen = 1e-12
    plan, out = _plan(shgo, b, n, screen)
    shgo.shgo_plan_autotune(plan, out, rounds=1)
    out.fill_(float("nan"))
    shgo.shgo_execute_graph(plan, out)
    torch.cuda.synchronize()
    nbf = b.nbf()
    V = out.cpu().numpy().reshape(nbf, nbf)
    assert not np.isnan(V).any()
    assert np.array_equal(V, V.T)
    pa, pb = synth.all_pairs(b.n_shells)
    ns = helpers.surviving_prim_pairs(b, pa, pb, screen)
    rng = np.random.default_rng(3)
    hi, lo = np.maximum(b.l[pa], b.l[pb]), np.minimum(b.l[pa], b.l[pb])
    sel = [np.nonzero(ns >= 48)[0]]
    for la in range(5):
        for lb in range(la + 1):
            cls = np.nonzero((hi == la) & (lo == lb) & (ns > 0))[0]
            sel.append(rng.choice(cls, min(40, len(cls)), replace=False))
    zero = rng.choice(np.nonzero(ns == 0)[0], 40, replace=False)
    sel = np.unique(np.concatenate(sel))
    assert len(sel) > 1400
    ref = oracle.split_blocks(oracle.nuc_blocks(b, n, pa[sel], pb[sel], screen=screen), b, pa[sel], pb[sel])
    off = b.shell_offsets()
    blk = lambda a, c: V[off[a]:off[a] + 2 * b.l[a] + 1, off[c]:off[c] + 2 * b.l[c] + 1]  # noqa: E731
    got = np.concatenate([blk(pa[k], pb[k]).ravel() for k in sel])
    assert_parity(got, np.concatenate([r.ravel() for r in ref]), f"{len(sel)} stratified pairs")
    for k in zero:
        assert np.all(blk(pa[k], pb[k]) == 0.0)
