"""bench.py's host logic on the CPU: the one-GPU guard, the algorithmic flop model that the
roofline divides by, and the traffic figure's tie to the kernel sources."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2404_16245_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_model_flops_per_nucleus_step():
    nnz = bench._gaunt_nnz()
    # the per-(primitive pair, nucleus) model: 52 flops for (0,0), 1818 for (6,6)
    assert bench.model_flops(0, 0, nnz)[0] == 52
    assert bench.model_flops(6, 6, nnz)[0] == 1818
    # more work for every larger class
    steps = [bench.model_flops(la, lb, nnz)[0] for la in range(7) for lb in range(la + 1)]
    assert all(x > 0 for x in steps)
    assert bench.model_flops(6, 5, nnz)[0] < bench.model_flops(6, 6, nnz)[0]


def test_sweep_model_flops_per_launch():
    # the roofline's algorithmic flops for the high-l sweep (49 classes x 2041 pairs, 64 nuclei)
    basis, nuclei, pa, pb = synth.high_l_sweep(seed=2)
    _, total = bench.workload_flops(basis, nuclei, pa, pb, 0.0)
    assert total == 4600891594


def test_surviving_prim_pairs_screening():
    b, _ = synth.long_contractions(seed=71)
    pa, pb = synth.all_pairs(b.n_shells)
    full = bench.surviving_prim_pairs(b, pa, pb, 0.0)
    assert np.array_equal(full, b.nprim[pa].astype(np.int64) * b.nprim[pb])
    kept = bench.surviving_prim_pairs(b, pa, pb, 1e-6)
    assert np.all(kept <= full) and kept.sum() < full.sum()
    # a shell with itself (R = 0) keeps every primitive pair
    same = pa == pb
    assert np.array_equal(kept[same], full[same])


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    tag = "k_integrals_high_l_sweep"
    v = bench.traffic_from_profile(tag)
    assert v is None or v > 0
    current = bench.kernel_source_hash()
    # a summary is read only while its source hash is the current one
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: current)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (prof / f"traffic_{tag}.txt").write_text("source_hash: 0000000000000000\nhbm_bytes_per_launch: 123\n")
    assert bench.traffic_from_profile(tag) is None
    (prof / f"traffic_{tag}.txt").write_text(f"# a comment: 1\nsource_hash: {current}\nhbm_bytes_per_launch: 123\n")
    assert bench.traffic_from_profile(tag) == 123.0


def test_batched_flop_model_counts_the_kept_primitive_pairs():
    # the headline's algorithmic flops use the primitive pairs that survive screening; their number
    # is the library's own host count
    import paper_2404_16245_amd as shgo
    b, n = synth.batched_molecule(seed=3)
    pa, pb = synth.all_pairs(b.n_shells)
    kept = bench.surviving_prim_pairs(b, pa, pb, 1e-12)
    st, _, info = shgo.shgo_check_call(b, n, shgo.options(screen=1e-12))
    assert st == 0 and int(kept.sum()) == info["kept_prim_pairs"] and int((kept > 0).sum()) == info["kept_pairs"]
    per_class, total = bench.workload_flops(b, n, pa, pb, 1e-12)
    assert total == per_class.sum() > 0 and np.count_nonzero(per_class) == 15


def test_cpu_baseline_sample_is_stratified():
    # a small molecule: the sample takes the same fraction of every class's kept pairs
    b, n = synth.molecule(seed=11, n_atoms=8, box=12.0, ls=(0, 1, 2), kmax=3)
    pa, pb = synth.all_pairs(b.n_shells)
    v, desc, dt = bench.cpu_baseline(b, n, pa, pb, 1e-12, 0.05, 1)
    assert v > 0 and dt > 0 and "6 (la,lb) classes" in desc and "1 OpenMP thread" in desc
    assert bench.cpu_model()


def test_gradient_model_counts_the_generated_step():
    # fma = 2 flops, other binary + - * = 1; indices, unary minus and comments are not counted
    assert bench._count_ops("a = fma(b, c, a); d = -e[3] * f[2 + 1]; g = h + i - j;  // x - y") == 2 + 1 + 2
    n00, p00 = bench.grad_model_flops(0, 0)
    # (0,0): one W entry, five FMAs on it, eight accumulator FMAs and the product -t^0 F_1 = 27,
    # plus the per-nucleus geometry, Boys (orders 0..1), assembly and nuclear-gradient terms
    assert n00 == 27 + 3 + 13 + 5 + 1 + (20 + 14 + 3 * 2) + 0 + 14 + 6 + 2 + 18
    assert p00 == 60 + 25 * 1 + 4 * 1
    per_nucleus = [bench.grad_model_flops(la, lb)[0] for la, lb in [(1, 0), (1, 1), (2, 1), (2, 2), (3, 3)]]
    assert per_nucleus == sorted(per_nucleus)
    # the adjoint step does several times the forward step's arithmetic
    gn = bench._gaunt_nnz()
    assert bench.grad_model_flops(3, 3)[0] > 4 * bench.model_flops(3, 3, gn)[0]


def test_unique_quartets_cover_each_symmetry_class_once():
    # eight index permutations relate (ab|cd); the list holds one canonical member of each orbit
    n = 6
    q = bench.unique_quartets(n)
    npair = n * (n + 1) // 2
    assert len(q) == npair * (npair + 1) // 2
    canon = set()
    for a in range(n):
        for b in range(n):
            for c in range(n):
                for d in range(n):
                    orbit = {(a, b, c, d), (b, a, c, d), (a, b, d, c), (b, a, d, c),
                             (c, d, a, b), (d, c, a, b), (c, d, b, a), (d, c, b, a)}
                    canon.add(max(orbit))
    assert {tuple(map(int, x)) for x in q} == canon
