"""The Cartesian (McMurchie-Davidson) route through the C ABI (shgo_execute_cartesian) against the
oracle, element by element, and against the solid-harmonic route on the same plan. Its nucleus
step is pinned on the CPU against the Hermite recursion of tests/xcheck.py
(tests/test_codegen.py). Bar as for the solid-harmonic route: 1e-13 + 1e-11 |ref|."""
import numpy as np
import pytest

import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-11, 1e-13
CART = [(a, b) for a in range(5) for b in range(5)]


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
    assert got.shape == ref.shape
    err = np.abs(got - ref)
    bad = err > ATOL + RTOL * np.abs(ref)
    if bad.any():
        i = int(np.argmax(np.where(bad, err, -1)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} elements out of tolerance; worst at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r}")


def test_cartesian_every_class_and_orientation(shgo):
    hb, hn, pa, pb = synth.high_l_sweep(seed=91, pairs_per_class=5, classes=CART)
    got = shgo.nuclear_attraction_cartesian_pairs(hb, hn, pa, pb).cpu().numpy()
    assert_parity(got, oracle.nuc_blocks(hb, hn, pa, pb), "Cartesian route, 25 classes x 5 pairs")


def test_cartesian_contracted_screened_matrix(shgo):
    b, n = synth.molecule(seed=92, n_atoms=10, box=10.0, ls=(0, 1, 2, 3, 4), kmax=6)
    for screen in (0.0, 1e-10):
        V = shgo.nuclear_attraction_cartesian(b, n, screen=screen).cpu().numpy()
        ref = oracle.nuc_matrix(b, n, screen=screen)
        assert_parity(V, ref, f"Cartesian route, contracted, screen {screen}")
        assert np.array_equal(V, V.T)
        # the two routes on one plan agree to the same bar
        Vs = shgo.nuclear_attraction(b, n, screen=screen).cpu().numpy()
        assert_parity(V, Vs, f"Cartesian against solid-harmonic route, screen {screen}")


def test_cartesian_many_pairs_per_class_and_long_contractions(shgo):
    # more pairs than the grid has wavefronts (the kernel strides), and shells of 16-20 primitives
    hb, hn, pa, pb = synth.high_l_sweep(seed=93, pairs_per_class=1500, classes=[(1, 0), (2, 2)])
    got = shgo.nuclear_attraction_cartesian_pairs(hb, hn, pa, pb).cpu().numpy()
    sel = np.random.default_rng(1).choice(len(pa), 200, replace=False)
    blocks = oracle.split_blocks(got, hb, pa, pb)
    ref = oracle.split_blocks(oracle.nuc_blocks(hb, hn, pa[sel], pb[sel]), hb, pa[sel], pb[sel])
    for k, r in zip(sel, ref):
        assert_parity(blocks[k], r, f"pair {k}")
    b, n = synth.long_contractions(seed=71)
    keep = b.l <= 4
    assert keep.all()
    V = shgo.nuclear_attraction_cartesian(b, n, screen=1e-12).cpu().numpy()
    assert_parity(V, oracle.nuc_matrix(b, n, screen=1e-12), "long contractions")


def test_cartesian_refuses_high_l(shgo):
    hb, hn, pa, pb = synth.high_l_sweep(seed=94, pairs_per_class=2, classes=[(5, 0)])
    with pytest.raises(shgo.ShgoError) as e:
        shgo.nuclear_attraction_cartesian_pairs(hb, hn, pa, pb)
    assert e.value.status == shgo.SHGO_ERR_UNSUPPORTED_L
