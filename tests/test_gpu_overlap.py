"""The overlap matrix S through the C ABI (shgo_execute_overlap) against the oracle's overlap
blocks, element by element, and the invariants a normalized basis fixes (unit diagonal blocks of a
shell with itself, exact symmetry)."""
import numpy as np
import pytest

import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-11, 1e-13


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as m
    m.load_library()
    return m


def assert_parity(got, ref, what):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    assert not bad.any(), f"{what}: {int(bad.sum())} of {bad.size} off, max abs err {err.max():.3e}"


def matrix_from_blocks(b, pa, pb, flat):
    nbf = b.nbf()
    off = b.shell_offsets()
    S = np.full((nbf, nbf), np.nan)
    blocks = oracle.split_blocks(flat, b, pa, pb)
    for k, (a, c) in enumerate(zip(pa, pb)):
        na, nc = 2 * b.l[a] + 1, 2 * b.l[c] + 1
        S[off[a]:off[a] + na, off[c]:off[c] + nc] = blocks[k]
        S[off[c]:off[c] + nc, off[a]:off[a] + na] = blocks[k].T
    return S


def test_every_class_and_orientation(shgo):
    # 49 (la, lb) classes x 3 uncontracted pairs; (la < lb) pairs come back in the listed orientation
    b, _, pa, pb = synth.high_l_sweep(seed=7, pairs_per_class=3)
    got = shgo.overlap_pairs(b, pa, pb).cpu().numpy()
    assert_parity(got, oracle.overlap_blocks(b, pa, pb), "49 classes x 3 pairs")


def test_contracted_molecule_matrix(shgo):
    b, _ = synth.molecule(seed=11, n_atoms=8, box=6.0, ls=(0, 1, 2, 3, 4), kmax=6)
    S = shgo.overlap(b).cpu().numpy()
    pa, pb = synth.all_pairs(b.n_shells)
    assert_parity(S, matrix_from_blocks(b, pa, pb, oracle.overlap_blocks(b, pa, pb)), "contracted S")
    assert np.array_equal(S, S.T)
    # normalized contracted shells: a shell's block with itself is the identity
    off = b.shell_offsets()
    for s in range(b.n_shells):
        n = 2 * b.l[s] + 1
        assert np.allclose(S[off[s]:off[s] + n, off[s]:off[s] + n], np.eye(n), rtol=0, atol=1e-12)


def test_long_contractions_and_shared_centers(shgo):
    # up to 400 primitive pairs per shell pair; shells of one atom share a center (R = 0)
    b, _ = synth.long_contractions(seed=71)
    pa, pb = synth.all_pairs(b.n_shells)
    assert_parity(shgo.overlap(b).cpu().numpy(), matrix_from_blocks(b, pa, pb, oracle.overlap_blocks(b, pa, pb)),
                  "long contractions")


def test_pair_list_in_any_order(shgo):
    b, _ = synth.molecule(seed=19, n_atoms=4, box=5.0, ls=(0, 1, 2, 3, 5, 6), kmax=3)
    pa, pb = synth.all_pairs(b.n_shells)
    rng = np.random.default_rng(19)
    order = rng.permutation(len(pa))
    pa, pb = pa[order].copy(), pb[order].copy()
    flip = rng.random(len(pa)) < 0.5
    pa[flip], pb[flip] = pb[flip].copy(), pa[flip].copy()
    assert_parity(shgo.overlap_pairs(b, pa, pb).cpu().numpy(), oracle.overlap_blocks(b, pa, pb), "pair list")


# Wavefronts whose 64 lanes (or, in the last one, all active lanes) hold pairs of a single class
# store through LDS; the tests below make most wavefronts single-class.
@pytest.mark.parametrize("ls,n_atoms", [((1,), 15), ((2,), 20), ((0, 3), 16)])
def test_single_class_wavefronts_matrix(shgo, ls, n_atoms):
    # (1,): 120 pairs of class (1,1): one full wavefront and one with 56 active lanes;
    # (2,): 210 pairs of (2,2); (0, 3): classes of 136, 256 and 136 pairs, some wavefronts
    # straddling a class boundary (lane-by-lane stores) beside single-class ones
    b, _ = synth.molecule(seed=29 + n_atoms, n_atoms=n_atoms, box=6.0, ls=ls, kmax=3)
    S = shgo.overlap(b).cpu().numpy()
    pa, pb = synth.all_pairs(b.n_shells)
    assert_parity(S, matrix_from_blocks(b, pa, pb, oracle.overlap_blocks(b, pa, pb)), f"ls {ls}")
    assert np.array_equal(S, S.T)


def test_single_class_wavefronts_pair_list(shgo):
    # 140 pairs of class (3,2), about half listed as (d, f): two full single-class wavefronts and a
    # last one with 12 active lanes, each storing both orientations of the listed blocks
    b, _ = synth.molecule(seed=37, n_atoms=12, box=6.0, ls=(3, 2), kmax=2)
    f = np.nonzero(b.l == 3)[0]
    d = np.nonzero(b.l == 2)[0]
    rng = np.random.default_rng(37)
    pa = rng.choice(f, 140)
    pb = rng.choice(d, 140)
    flip = rng.random(140) < 0.5
    pa[flip], pb[flip] = pb[flip].copy(), pa[flip].copy()
    assert 50 < flip.sum() < 90
    got = shgo.overlap_pairs(b, pa, pb).cpu().numpy()
    assert_parity(got, oracle.overlap_blocks(b, pa, pb), "140 (3,2) pairs, half swapped")


def test_bench_basis_sampled(shgo):
    # the S that bench.py times: the 200-atom batched basis (nbf 5000, l = 0..4, K 1..8), whose
    # matrix plan enumerates each class's pairs from the shells ordered by l and primitive count;
    # checked on 40 sampled shell pairs of every (la, lb) class (both orientations in the matrix),
    # the unit diagonal of every shell's block with itself, and exact symmetry
    b, _ = synth.batched_molecule(seed=3)
    S = shgo.overlap(b).cpu().numpy()
    assert np.isfinite(S).all()
    assert np.array_equal(S, S.T)
    ls = np.asarray(b.l)
    off = np.asarray(b.shell_offsets())
    rng = np.random.default_rng(41)
    pa, pb = [], []
    for la in range(5):
        for lb in range(la + 1):
            sa, sb = np.flatnonzero(ls == la), np.flatnonzero(ls == lb)
            pa += list(rng.choice(sa, 40))
            pb += list(rng.choice(sb, 40))
    pa, pb = np.array(pa, np.int32), np.array(pb, np.int32)
    blocks = oracle.split_blocks(oracle.overlap_blocks(b, pa, pb), b, pa, pb)
    for k, (a, c) in enumerate(zip(pa, pb)):
        na, nc = 2 * ls[a] + 1, 2 * ls[c] + 1
        assert_parity(S[off[a]:off[a] + na, off[c]:off[c] + nc], blocks[k], f"pair ({a}, {c})")
    diag = np.concatenate([np.diag(S[o:o + 2 * l + 1, o:o + 2 * l + 1]) for o, l in zip(off, ls)])
    assert np.abs(diag - 1.0).max() < 1e-12
