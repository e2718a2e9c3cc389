"""CPU replay of the integral kernel's schedule and layout arithmetic under AddressSanitizer and
UBSan (tests/native/sched_replay.cpp): the pair build, the work-item list, every item's tasks,
LDS offsets and output indices of the test and bench workloads, for the default schedule and for
one-tile, largest and random tiles per item. It checks every index against its buffer and that
every item, task, shell-pair slot and output element is covered exactly once."""
import os
import subprocess

import numpy as np
import pytest

from paper_2404_16245_amd import SHGO_LMAX, SHGO_NUM_CLASSES, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_replay.cpp")
CSRC = os.path.join(ROOT, "paper_2404_16245_amd", "csrc")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    d = tmp_path_factory.mktemp("replay")
    exe = str(d / "sched_replay")
    gen = os.path.join(CSRC, "generated", "shgo_meta.inc")
    if not os.path.exists(gen):
        subprocess.run(["python", os.path.join(CSRC, "gen_classes.py"), os.path.join(CSRC, "generated",
                                                                                     "shgo_classes.inc")], check=True)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC, SRC, "-o", exe]
    subprocess.run(cmd, check=True)
    return exe, d


def _class_max_tiles():
    out = []
    for la in range(SHGO_LMAX + 1):
        for lb in range(la + 1):
            nab = (2 * la + 1) * (2 * lb + 1)
            out.append(min(8, 20448 // (nab * 65 + 256)))
    return out


def write_input(path, basis, nuclei, screen, full, pa=None, pb=None, schedules=()):
    f = lambda x: repr(float(x))  # noqa: E731  (shortest round-trip decimal)
    lines = [f"{1 if full else 0} {basis.n_shells} {nuclei.n} {f(screen)} {0 if full else len(pa)}"]
    for s in range(basis.n_shells):
        c = basis.center[s]
        lines.append(f"{int(basis.l[s])} {int(basis.nprim[s])} {int(basis.prim_off[s])} {f(c[0])} {f(c[1])} {f(c[2])}")
    lines.append(str(len(basis.expo)))
    lines += [f"{f(e)} {f(d)}" for e, d in zip(basis.expo, basis.coef)]
    lines += [f"{f(p[0])} {f(p[1])} {f(p[2])} {f(z)}" for p, z in zip(nuclei.pos, nuclei.Z)]
    if not full:
        lines += [f"{a} {b}" for a, b in zip(pa, pb)]
    lines.append(str(len(schedules)))
    lines += [" ".join(str(int(t)) for t in s) for s in schedules]
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def schedules(seed):
    mx = _class_max_tiles()
    rng = np.random.default_rng(seed)
    return [[1] * SHGO_NUM_CLASSES, mx, [int(rng.integers(1, m + 1)) for m in mx]]


def run(replay, name, *args, **kw):
    exe, d = replay
    path = str(d / f"{name}.txt")
    write_input(path, *args, **kw)
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 1 + len(kw.get("schedules", ())) and all(l.startswith("ok ") for l in lines), r.stdout
    return lines


def test_replay_small_molecule(replay):
    b, n = synth.small_molecule(seed=1)
    run(replay, "small", b, n, 0.0, True, schedules=schedules(1))


@pytest.mark.parametrize("screen", [0.0, 1e-12, 1e-6])
def test_replay_long_contractions(replay, screen):
    # up to 400 primitive pairs per shell pair: saturated keys, long tiles cut into slices
    b, n = synth.long_contractions(seed=71)
    run(replay, f"long_{screen}", b, n, screen, True, schedules=schedules(2))


def test_replay_pair_list_ragged_swapped_repeated(replay):
    hb, hn, pa, pb = synth.high_l_sweep(seed=8, pairs_per_class=70, classes=[(6, 6), (2, 5), (1, 0), (4, 4)])
    rng = np.random.default_rng(3)
    rep = rng.choice(len(pa), 40, replace=False)
    pa, pb = np.concatenate([pa, pb[rep]]), np.concatenate([pb, pa[rep]])
    run(replay, "ragged", hb, hn, 0.0, False, pa, pb, schedules=schedules(3))


def test_replay_high_l_sweep(replay):
    hb, hn, pa, pb = synth.high_l_sweep(seed=2)
    run(replay, "sweep", hb, hn, 0.0, False, pa, pb, schedules=schedules(4)[:1])


def test_replay_contracted_molecule(replay):
    b, n = synth.molecule(seed=11, n_atoms=8, box=12.0, ls=(0, 1, 2, 3, 4), kmax=6)
    for screen in (0.0, 1e-12, 1e-4):
        run(replay, f"contracted_{screen}", b, n, screen, True, schedules=schedules(5))


@pytest.mark.slow
def test_replay_batched_molecule(replay):
    # the 200-atom molecule of the batched form (500,500 candidate pairs, nbf 5000)
    b, n = synth.batched_molecule(seed=3)
    run(replay, "batched", b, n, 1e-12, True, schedules=[])


def test_replay_l7_classes(replay):
    # l = 7 shells: one tile per (7,7) item (225 accumulator rows per pair), ragged tails, swapped
    # pairs, and a contracted molecule with l up to 7
    hb, hn, pa, pb = synth.high_l_sweep(seed=78, pairs_per_class=70, classes=[(7, b) for b in range(8)] + [(2, 7)])
    run(replay, "l7_pairs", hb, hn, 0.0, False, pa, pb, schedules=schedules(6))
    b, n = synth.molecule(seed=79, n_atoms=4, box=6.0, ls=(0, 2, 5, 7), kmax=4)
    run(replay, "l7_matrix", b, n, 1e-8, True, schedules=schedules(7))
