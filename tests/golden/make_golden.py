"""Writes the stored expected values under tests/golden/ by calling only the oracle.

The paper prints no worked numerical example, so the stored values here are the oracle's own
results on seeded synthetic inputs; they guard the oracle against unintended changes (any
change to them must name, in its commit message, the passage of the paper that justifies it).

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2404_16245_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    bs, nuc = synth.small_molecule(seed=1)
    V = oracle.nuc_matrix(bs, nuc, precision=2)
    np.savetxt(os.path.join(HERE, "small_molecule_seed1_V.txt"), V, fmt="%.17e",
               header="nuclear-attraction matrix, 4-atom s/p/d molecule (synth.small_molecule seed 1), "
                      "oracle __float128 build, real solid-harmonic order m=-l..l, 36x36")
    hb, hn, pa, pb = synth.high_l_sweep(seed=2, pairs_per_class=1, classes=[(6, 6), (6, 0), (3, 5)])
    B = oracle.nuc_blocks(hb, hn, pa, pb, precision=2)
    np.savetxt(os.path.join(HERE, "high_l_seed2_blocks.txt"), B, fmt="%.17e",
               header="blocks of synth.high_l_sweep(seed=2, pairs_per_class=1, classes=[(6,6),(6,0),(3,5)]), "
                      "concatenated in pair order, oracle __float128 build")


if __name__ == "__main__":
    main()
