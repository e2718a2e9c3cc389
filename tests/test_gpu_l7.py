"""Shells of l = 7 (the product rule then reaches L = 14 and the Boys function order 14, 15 for the
gradient): every path through the C ABI against the oracle, whose own l = 7 blocks are pinned by
the McMurchie-Davidson cross-check and its __float128 instantiation (tests/test_oracle_integrals.py).
Bars as for l <= 6: V and S element by element to 1e-13 + 1e-11 |ref|, the gradient to 1e-10."""
import numpy as np
import pytest

import oracle
from paper_2404_16245_amd import synth

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-11, 1e-13
L7 = [(7, b) for b in range(8)] + [(0, 7), (3, 7), (6, 7)]


@pytest.fixture(scope="module")
def shgo():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_16245_amd as m
    m.context(0)
    return m


def assert_parity(got, ref, what, rtol=RTOL):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    err = np.abs(got - ref)
    bad = err > ATOL + rtol * np.abs(ref)
    if bad.any():
        i = int(np.argmax(np.where(bad, err, -1)))
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} elements out of tolerance; worst at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r}")


def test_l7_classes(shgo):
    hb, hn, pa, pb = synth.high_l_sweep(seed=77, pairs_per_class=6, classes=L7)
    got = shgo.nuclear_attraction_pairs(hb, hn, pa, pb).cpu().numpy()
    assert_parity(got, oracle.nuc_blocks(hb, hn, pa, pb), "l = 7 classes x 6 pairs")


def test_l7_ragged_tiles_and_swapped(shgo):
    # (7,7): one full 64-pair tile and a ragged tail (each item one tile: 225 entries of LDS per
    # pair); (2,7) listed swapped
    hb, hn, pa, pb = synth.high_l_sweep(seed=78, pairs_per_class=70, classes=[(7, 7), (2, 7)])
    got = shgo.nuclear_attraction_pairs(hb, hn, pa, pb).cpu().numpy()
    assert_parity(got, oracle.nuc_blocks(hb, hn, pa, pb), "ragged l = 7 tiles")


def test_l7_contracted_screened_matrix_and_mixed(shgo):
    b, n = synth.molecule(seed=79, n_atoms=4, box=6.0, ls=(0, 2, 5, 7), kmax=4)
    for screen in (0.0, 1e-8):
        ref = oracle.nuc_matrix(b, n, screen=screen)
        V = shgo.nuclear_attraction(b, n, screen=screen).cpu().numpy()
        assert_parity(V, ref, f"contracted l <= 7, screen {screen}")
        assert np.array_equal(V, V.T)
        # the mixed kernel keeps the binary64 coupling above l = 4
        Vm = shgo.nuclear_attraction(b, n, screen=screen, precision="mixed").cpu().numpy()
        assert_parity(Vm, ref, f"mixed, contracted l <= 7, screen {screen}", rtol=1e-9)


def test_l7_boys_orders(shgo):
    import torch
    T = np.concatenate([[0.0, 1e-10, 1e-3], np.linspace(0.02, 71.9, 150), np.linspace(71.9, 72.1, 21),
                        [72.5, 100.0, 500.0, 6.4e4]])
    ref = np.array([oracle.boys(15, t, precision=2) for t in T])
    F = shgo.shgo_boys(shgo.context(0), torch.tensor(T, device="cuda"), 15).cpu().numpy()
    err = np.abs(F - ref)
    assert np.all(err <= 2e-14 * np.abs(ref)), f"max rel err {np.max(err / np.abs(ref)):.3e}"


def test_l7_gradient(shgo):
    b, n = synth.molecule(seed=80, n_atoms=2, box=3.0, ls=(0, 3, 7), kmax=2)
    D = synth.density(b.nbf(), seed=8)
    dn, dc, e = shgo.nuclear_attraction_grad(b, n, D)
    rn, rc, rE = oracle.grad(b, n, D)
    scale = max(np.abs(rn).max(), np.abs(rc).max())
    for name, x, y in (("nuclei", dn.cpu().numpy(), rn), ("centers", dc.cpu().numpy(), rc)):
        err = np.abs(x - y)
        assert np.all(err <= 1e-10 * np.abs(y) + 1e-12 * scale), f"{name}: max err {err.max():.3e}"
    assert float(e.cpu().numpy()[0]) == pytest.approx(rE, rel=1e-11, abs=1e-12)


def test_l7_overlap(shgo):
    b, _, pa, pb = synth.high_l_sweep(seed=81, pairs_per_class=5, classes=L7 + [(2, 2), (4, 3)])
    got = shgo.overlap_pairs(b, pa, pb).cpu().numpy()
    assert_parity(got, oracle.overlap_blocks(b, pa, pb), "overlap, l = 7 classes")
