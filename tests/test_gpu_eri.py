"""Two-electron blocks (ab|cd) through the C ABI (shgo_eri_blocks) against the Hermite oracle
(oracle/eri.py), element by element: every ordered combination of s, p and d shells (both orders
inside each pair, so the kernel's swaps are covered), contracted shells of a synthetic molecule
with shells on one center, more quartets than the grid has wavefronts, a basis of more than 2048
shells (the host's hashed pair index), the error paths, the bench's own call (every unique
quartet of its 10-atom molecule) on a sample, and long contractions (several staging rounds).
Bar as for the nuclear attraction: 1e-13 + 1e-11 |ref|."""
import itertools

import numpy as np
import pytest

from oracle import eri
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-11, 1e-13


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as m
    m.context(0)
    return m


def assert_parity(got, ref, what):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    if bad.any():
        i = int(np.argmax(np.where(bad, err, -1)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} elements out of tolerance; worst at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r}")


def _basis(specs):
    centers, ls, expo, coef, nprim, off = [], [], [], [], [], []
    o = 0
    for l, c, e, d in specs:
        centers.append(c)
        ls.append(l)
        expo += list(e)
        coef += list(d)
        nprim.append(len(e))
        off.append(o)
        o += len(e)
    return synth.Basis(np.array(centers, float), np.array(ls, np.int32), np.array(nprim, np.int32),
                       np.array(off, np.int64), np.array(expo, float), np.array(coef, float))


def test_every_ordered_l_combination(shgo):
    # one primitive shell of each l on each of four centers; shell 3 c + l sits on center c
    rng = np.random.default_rng(11)
    cen = rng.normal(0, 1.0, (4, 3))
    specs = [(l, cen[c], [float(np.exp(rng.uniform(np.log(0.4), np.log(3.0))))], [1.0])
             for c in range(4) for l in range(3)]
    b = _basis(specs)
    quartets = np.array([[3 * k + ls[k] for k in range(4)] for ls in itertools.product(range(3), repeat=4)],
                        np.int32)
    got = shgo.eri_blocks(b, quartets).cpu().numpy()
    assert_parity(got, eri.eri_blocks(b, quartets), "81 ordered l-quartets")


def test_contracted_molecule_with_shared_centers(shgo):
    b, _ = synth.molecule(seed=12, n_atoms=3, box=4.0, ls=(0, 1, 2), kmax=3)
    rng = np.random.default_rng(13)
    n = len(b.l)
    quartets = rng.integers(0, n, (40, 4)).astype(np.int32)
    # quartets that repeat one shell, and all four on one shell
    quartets = np.vstack([quartets, [[0, 0, 0, 0], [1, 1, 2, 2], [3, 4, 3, 4], [n - 1, 0, n - 1, 0]]]).astype(np.int32)
    got = shgo.eri_blocks(b, quartets).cpu().numpy()
    assert_parity(got, eri.eri_blocks(b, quartets), "contracted quartets")


def test_many_quartets_grid_stride(shgo):
    # more quartets than the launch has wavefronts: the kernel strides over them
    b, _ = synth.molecule(seed=14, n_atoms=4, box=5.0, ls=(0, 1, 2), kmax=1)
    rng = np.random.default_rng(15)
    quartets = rng.integers(0, len(b.l), (9000, 4)).astype(np.int32)
    got = shgo.eri_blocks(b, quartets).cpu().numpy()
    sizes = np.prod(2 * np.asarray(b.l)[quartets] + 1, axis=1)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    assert got.shape == (offs[-1],)
    for k in rng.choice(len(quartets), 60, replace=False):
        assert_parity(got[offs[k]:offs[k + 1]], eri.eri_block(b, *quartets[k]).ravel(), f"quartet {k}")


def test_empty_and_errors(shgo):
    b, _ = synth.molecule(seed=16, n_atoms=2, box=3.0, ls=(0, 1, 2, 3), kmax=1)
    assert shgo.eri_blocks(b, np.zeros((0, 4), np.int32)).numel() == 0
    f = int(np.flatnonzero(np.asarray(b.l) == 3)[0])
    with pytest.raises(shgo.ShgoError) as e:
        shgo.eri_blocks(b, np.array([[0, 0, f, 0]], np.int32))
    assert e.value.status == shgo.SHGO_ERR_UNSUPPORTED_L
    with pytest.raises(shgo.ShgoError) as e:
        shgo.eri_blocks(b, np.array([[0, 0, len(b.l), 0]], np.int32))
    assert e.value.status == shgo.SHGO_ERR_INVALID_ARG


def test_many_shells_hashed_pair_index(shgo):
    # more than 2048 shells: the host indexes the distinct pairs with a hash map instead of the
    # dense n_shells^2 table; a few hundred quartets, some sharing pairs in both orders
    b, _ = synth.molecule(seed=17, n_atoms=700, box=30.0, ls=(0, 1, 2), kmax=1)
    assert len(b.l) > 2048
    rng = np.random.default_rng(18)
    q = rng.integers(0, len(b.l), (300, 4)).astype(np.int32)
    q[::7] = q[::7][:, [1, 0, 3, 2]]
    q = np.vstack([q, q[:20][:, [2, 3, 0, 1]]]).astype(np.int32)
    got = shgo.eri_blocks(b, q).cpu().numpy()
    sizes = np.prod(2 * np.asarray(b.l)[q] + 1, axis=1)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for k in rng.choice(len(q), 40, replace=False):
        assert_parity(got[offs[k]:offs[k + 1]], eri.eri_block(b, *q[k]).ravel(), f"quartet {k}")


def test_bench_workload_sampled(shgo):
    # the call bench.py times: every unique quartet of the 10-atom s/p/d molecule (108,345 quartets,
    # both kernel instances, the cost ordering at scale), checked on a sample: the costliest
    # quartets, quartets with a (d,d) pair and without, and random ones
    import bench
    b, _ = bench.eri_workload(synth)
    q = bench.unique_quartets(len(b.l))
    got = shgo.eri_blocks(b, q).cpu().numpy()
    ls, npr = np.asarray(b.l), np.asarray(b.nprim)
    dim = 2 * ls + 1
    sizes = dim[q[:, 0]] * dim[q[:, 1]] * dim[q[:, 2]] * dim[q[:, 3]]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    assert got.shape == (offs[-1],)
    rng = np.random.default_rng(21)
    dd = ((ls[q[:, 0]] == 2) & (ls[q[:, 1]] == 2)) | ((ls[q[:, 2]] == 2) & (ls[q[:, 3]] == 2))
    cost = np.prod(npr[q], axis=1) * sizes
    pick = np.concatenate([np.argsort(-cost)[:15], rng.choice(np.flatnonzero(dd), 20, replace=False),
                           rng.choice(np.flatnonzero(~dd), 20, replace=False), rng.choice(len(q), 20, replace=False)])
    for k in pick:
        assert_parity(got[offs[k]:offs[k + 1]], eri.eri_block(b, *q[k]).ravel(), f"quartet {k} {q[k]}")


def test_long_contractions_span_several_staging_rounds(shgo):
    # contractions of 4 and 5 primitives: 16 to 25 ket primitive pairs, so the kernel stages the
    # Boys values and harmonics in several rounds (5 slots in the small instance, 9 in the large);
    # (pp|pp) and (dp|ps) in the small instance, (dd|dd), (dd|ss) and (dd|pd) (ket swapped) in the
    # large one
    rng = np.random.default_rng(23)
    cen = rng.normal(0, 1.2, (3, 3))

    def shell(l, c, K):
        e = np.sort(np.exp(rng.uniform(np.log(0.15), np.log(12.0), K)))[::-1]
        return (l, cen[c], list(e), list(rng.uniform(0.2, 1.0, K)))

    b = _basis([shell(0, 0, 5), shell(1, 1, 4), shell(2, 2, 4), shell(2, 0, 4), shell(1, 2, 5)])
    q = np.array([[1, 4, 1, 4], [2, 1, 4, 0], [2, 3, 2, 3], [3, 2, 0, 0], [2, 3, 4, 2]], np.int32)
    assert_parity(shgo.eri_blocks(b, q).cpu().numpy(), eri.eri_blocks(b, q), "long contractions")
