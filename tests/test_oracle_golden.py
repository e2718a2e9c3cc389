"""The oracle reproduces its stored results (tests/golden, written by make_golden.py)."""
import os

import numpy as np

import oracle
from paper_2404_16245_amd import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_small_molecule_matches_golden():
    bs, nuc = synth.small_molecule(seed=1)
    ref = np.loadtxt(os.path.join(GOLD, "small_molecule_seed1_V.txt"))
    V = oracle.nuc_matrix(bs, nuc)
    assert np.all(np.abs(V - ref) <= 1e-14 + 1e-12 * np.abs(ref))


def test_high_l_blocks_match_golden():
    hb, hn, pa, pb = synth.high_l_sweep(seed=2, pairs_per_class=1, classes=[(6, 6), (6, 0), (3, 5)])
    ref = np.loadtxt(os.path.join(GOLD, "high_l_seed2_blocks.txt"))
    B = oracle.nuc_blocks(hb, hn, pa, pb)
    assert np.all(np.abs(B - ref) <= 1e-14 + 1e-12 * np.abs(ref))
