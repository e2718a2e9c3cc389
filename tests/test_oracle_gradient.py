"""Pins of the oracle's analytic gradient (dual numbers) of E = sum_ij D_ij V_ij.

The gradient is checked against five-point central differences of two forward routes -- the oracle's own
(itself pinned by the tests of test_oracle_integrals.py) and the independent Cartesian
McMurchie-Davidson route of xcheck -- and against two invariants: translation (the forces on
all centers and nuclei sum to zero) and rotation (the gradient turns with the molecule when the
density turns with it).
"""
import numpy as np
import pytest

import oracle
import xcheck
from paper_2404_16245_amd import synth


def _fd(f, x0, h):
    """Five-point central difference of f at x0 (error of order h^4)."""
    return (8.0 * (f(x0 + h) - f(x0 - h)) - (f(x0 + 2 * h) - f(x0 - 2 * h))) / (12.0 * h)


def _with_centers(b, cen):
    return synth.Basis(np.ascontiguousarray(cen), b.l, b.nprim, b.prim_off, b.expo, b.coef)


def _energy_oracle(b, n, D):
    return float(np.sum(D * oracle.nuc_matrix(b, n)))


def test_gradient_against_central_differences_of_the_oracle():
    b, n = synth.small_molecule(seed=1)
    D = synth.density(b.nbf(), seed=5)
    dn, dc, E = oracle.grad(b, n, D)
    assert E == pytest.approx(_energy_oracle(b, n, D), rel=1e-13)
    h = 2e-4
    for c in range(n.n):
        for x in range(3):
            def f(v):
                pos = n.pos.copy()
                pos[c, x] = v
                return _energy_oracle(b, synth.Nuclei(pos, n.Z), D)
            assert _fd(f, n.pos[c, x], h) == pytest.approx(dn[c, x], rel=1e-8, abs=1e-10)
    for s in range(b.n_shells):
        for x in range(3):
            def f(v):
                cen = b.center.copy()
                cen[s, x] = v
                return _energy_oracle(_with_centers(b, cen), n, D)
            assert _fd(f, b.center[s, x], h) == pytest.approx(dc[s, x], rel=1e-8, abs=1e-10)


def _energy_md(b, n, D):
    """E from the Cartesian McMurchie-Davidson route (no oracle code)."""
    off = b.shell_offsets()
    E = 0.0
    for a in range(b.n_shells):
        for c in range(a, b.n_shells):
            blk = xcheck.contracted_block(xcheck.md_nuclear_prim, b, n, a, c)
            da, dc = 2 * b.l[a] + 1, 2 * b.l[c] + 1
            Dt = D[off[a]:off[a] + da, off[c]:off[c] + dc]
            if a != c:
                Dt = Dt + D[off[c]:off[c] + dc, off[a]:off[a] + da].T
            E += float(np.sum(Dt * blk))
    return E


def test_gradient_against_central_differences_of_mcmurchie_davidson():
    rng = np.random.default_rng(11)
    cen = np.array([[0.0, 0.1, 0.0], [0.0, 0.1, 0.0], [1.1, -0.4, 0.7]])  # two shells share a center
    b = synth.Basis(cen, np.array([2, 1, 1], np.int32), np.array([1, 2, 1], np.int32), np.array([0, 1, 3], np.int64),
                    np.array([0.9, 1.7, 0.4, 1.2]), np.array([1.0, 0.6, 0.5, 1.0]))
    n = synth.Nuclei(np.array([[0.3, 0.2, -0.5], [1.0, -0.2, 0.9]]), np.array([3.0, 1.0]))
    nbf = b.nbf()
    D = rng.normal(0, 0.3, (nbf, nbf))
    D = D + D.T
    dn, dc, E = oracle.grad(b, n, D)
    assert E == pytest.approx(_energy_md(b, n, D), rel=1e-11)
    h = 2e-4
    for c, x in [(0, 0), (0, 2), (1, 1)]:
        def f(v):
            pos = n.pos.copy()
            pos[c, x] = v
            return _energy_md(b, synth.Nuclei(pos, n.Z), D)
        assert _fd(f, n.pos[c, x], h) == pytest.approx(dn[c, x], rel=1e-8, abs=1e-10)
    for s, x in [(0, 0), (1, 0), (1, 2), (2, 1)]:
        def f(v):
            c2 = cen.copy()
            c2[s, x] = v
            return _energy_md(_with_centers(b, c2), n, D)
        assert _fd(f, cen[s, x], h) == pytest.approx(dc[s, x], rel=1e-8, abs=1e-10)


def test_translation_sum_rule_and_zero_density():
    b, n = synth.molecule(seed=41, n_atoms=5, box=5.0, ls=(0, 1, 2, 3), kmax=3)
    D = synth.density(b.nbf(), seed=9)
    dn, dc, _ = oracle.grad(b, n, D)
    total = dn.sum(axis=0) + dc.sum(axis=0)
    assert np.abs(total).max() <= 1e-11 * np.abs(np.concatenate([dn, dc])).max()
    dn0, dc0, E0 = oracle.grad(b, n, np.zeros_like(D))
    assert E0 == 0.0 and not dn0.any() and not dc0.any()


def test_gradient_turns_with_the_molecule():
    b, n = synth.molecule(seed=43, n_atoms=3, box=4.0, ls=(0, 1, 2, 3), kmax=2)
    D = synth.density(b.nbf(), seed=10)
    Q = synth.random_rotation(12)
    # rotating the molecule turns each block of V by the real Wigner matrices; the density
    # turned the same way keeps E fixed, and the gradients turn as vectors
    W = [xcheck.real_wigner_d(l, Q) for l in range(4)]
    off = b.shell_offsets()
    U = np.zeros((b.nbf(), b.nbf()))
    for s in range(b.n_shells):
        d = 2 * b.l[s] + 1
        U[off[s]:off[s] + d, off[s]:off[s] + d] = W[b.l[s]]
    Dr = U @ D @ U.T
    dn, dc, E = oracle.grad(b, n, D)
    dnr, dcr, Er = oracle.grad(_with_centers(b, b.center @ Q.T), synth.Nuclei(n.pos @ Q.T, n.Z), Dr)
    assert Er == pytest.approx(E, rel=1e-10)
    scale = np.abs(np.concatenate([dn, dc])).max()
    assert np.allclose(dnr, dn @ Q.T, atol=1e-9 * scale)
    assert np.allclose(dcr, dc @ Q.T, atol=1e-9 * scale)
