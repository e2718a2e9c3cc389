"""Seeded synthetic inputs: molecules, basis sets, shell-pair lists and density matrices.

This module only draws random numbers and lays them out as plain arrays; it holds none of the
integral arithmetic (no normalisation, no Gaussian products). Both the GPU path and the CPU
oracle consume what it produces.

A *basis* is a set of shells, each a center, an angular momentum ``l`` and ``K`` primitives
(exponents and contraction coefficients that multiply *normalised* primitives), as in Eq. 1
of the paper. Nuclei are point charges (position, Z). Units are atomic (bohr).

Workloads (``numpy.random.default_rng(seed)``; "log-uniform [a, b]" means exp(U(ln a, ln b))):

* ``small_molecule``: 4 atoms uniform in a 6-bohr cube, Z in {1..8}; each atom carries s, p, d
  shells with 3 primitives, exponents log-uniform [0.1, 50], coefficients uniform [0.1, 1].
* ``high_l_sweep``: independent uncontracted shell pairs, ``pairs_per_class`` for each of the
  49 classes (l_a, l_b) in {0..6}^2, exponents log-uniform [0.05, 100], centers uniform in a
  10-bohr cube, 64 nuclei uniform in the same cube with Z in {1..10}. Pairs are shuffled so the
  class sort has work to do.
* ``molecule``: ``n_atoms`` atoms uniform in a cube of side ``box``, one shell per l in
  ``ls`` on every atom, K uniform in 1..``kmax``, exponents log-uniform [0.1, 50], coefficients
  uniform [0.1, 1], Z in {1..8} (200 atoms / 20 bohr / l <= 4 / K <= 8 for the batched
  workload; 500 atoms / 30 bohr / l <= 3 / K <= 6 for the gradient workload).
* ``density``: a symmetric matrix whose upper triangle (diagonal included) is N(0, 0.1^2).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Basis:
    center: np.ndarray    # float64 [n_shells, 3]
    l: np.ndarray         # int32   [n_shells]
    nprim: np.ndarray     # int32   [n_shells]
    prim_off: np.ndarray  # int64   [n_shells]
    expo: np.ndarray      # float64 [total primitives]
    coef: np.ndarray      # float64 [total primitives]

    @property
    def n_shells(self):
        return int(self.l.shape[0])

    def nbf(self):
        return int(np.sum(2 * self.l.astype(np.int64) + 1))

    def shell_offsets(self):
        d = 2 * self.l.astype(np.int64) + 1
        return np.concatenate([[0], np.cumsum(d)[:-1]]).astype(np.int64)

    def subset(self, shells):
        """A new basis holding only the given shells (in the given order)."""
        shells = np.asarray(shells, dtype=np.int64)
        nprim = self.nprim[shells]
        off = np.concatenate([[0], np.cumsum(nprim)[:-1]]).astype(np.int64)
        idx = np.concatenate([np.arange(self.prim_off[s], self.prim_off[s] + self.nprim[s]) for s in shells])
        return Basis(self.center[shells].copy(), self.l[shells].copy(), nprim.astype(np.int32), off,
                     self.expo[idx].copy(), self.coef[idx].copy())


@dataclass
class Nuclei:
    pos: np.ndarray  # float64 [n, 3]
    Z: np.ndarray    # float64 [n]

    @property
    def n(self):
        return int(self.Z.shape[0])


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _basis_from_lists(centers, ls, ks, rng, elo, ehi, clo, chi, unit_coef=False):
    ls = np.asarray(ls, dtype=np.int32)
    ks = np.asarray(ks, dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(ks)[:-1]]).astype(np.int64)
    n = int(ks.sum())
    expo = _log_uniform(rng, elo, ehi, n)
    coef = np.ones(n) if unit_coef else rng.uniform(clo, chi, n)
    return Basis(np.ascontiguousarray(centers, dtype=np.float64), ls, ks, off, expo, coef)


def small_molecule(seed=1, n_atoms=4, box=6.0, ls=(0, 1, 2), k=3):
    """4 atoms, s/p/d shells with 3 primitives each; returns (basis, nuclei)."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, box, (n_atoms, 3))
    Z = rng.integers(1, 9, n_atoms).astype(np.float64)
    centers = np.repeat(atoms, len(ls), axis=0)
    shell_l = np.tile(np.asarray(ls), n_atoms)
    basis = _basis_from_lists(centers, shell_l, np.full(len(shell_l), k), rng, 0.1, 50.0, 0.1, 1.0)
    return basis, Nuclei(atoms.copy(), Z)


def high_l_sweep(seed=2, pairs_per_class=2041, lmax=6, n_nuclei=64, box=10.0, classes=None):
    """Uncontracted shell pairs of every class (l_a, l_b); returns (basis, nuclei, pair_a, pair_b).

    Shell 2i and 2i+1 form pair i. ``classes`` restricts the sweep to a list of (l_a, l_b)."""
    rng = np.random.default_rng(seed)
    if classes is None:
        classes = [(a, b) for a in range(lmax + 1) for b in range(lmax + 1)]
    la = np.repeat([c[0] for c in classes], pairs_per_class)
    lb = np.repeat([c[1] for c in classes], pairs_per_class)
    perm = rng.permutation(la.shape[0])
    la, lb = la[perm], lb[perm]
    npair = la.shape[0]
    shell_l = np.empty(2 * npair, dtype=np.int32)
    shell_l[0::2] = la
    shell_l[1::2] = lb
    centers = rng.uniform(0.0, box, (2 * npair, 3))
    basis = _basis_from_lists(centers, shell_l, np.ones(2 * npair), rng, 0.05, 100.0, 1.0, 1.0, unit_coef=True)
    nuc = Nuclei(rng.uniform(0.0, box, (n_nuclei, 3)), rng.integers(1, 11, n_nuclei).astype(np.float64))
    pa = np.arange(0, 2 * npair, 2, dtype=np.int32)
    pb = np.arange(1, 2 * npair, 2, dtype=np.int32)
    return basis, nuc, pa, pb


def molecule(seed=3, n_atoms=200, box=20.0, ls=(0, 1, 2, 3, 4), kmax=8, zmax=8):
    """A synthetic molecule with one contracted shell per l per atom; returns (basis, nuclei)."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, box, (n_atoms, 3))
    Z = rng.integers(1, zmax + 1, n_atoms).astype(np.float64)
    centers = np.repeat(atoms, len(ls), axis=0)
    shell_l = np.tile(np.asarray(ls), n_atoms)
    ks = rng.integers(1, kmax + 1, len(shell_l))
    basis = _basis_from_lists(centers, shell_l, ks, rng, 0.1, 50.0, 0.1, 1.0)
    return basis, Nuclei(atoms.copy(), Z)


def batched_molecule(seed=3):
    """200 atoms in a 20-bohr box, shells l = 0..4, K uniform 1..8."""
    return molecule(seed=seed, n_atoms=200, box=20.0, ls=(0, 1, 2, 3, 4), kmax=8)


def gradient_molecule(seed=5):
    """500 atoms in a 30-bohr box, shells l = 0..3, K uniform 1..6."""
    return molecule(seed=seed, n_atoms=500, box=30.0, ls=(0, 1, 2, 3), kmax=6)


def long_contractions(seed=71):
    """Three atoms with s..g shells of 1 to 20 primitives: shell pairs of up to 400 primitive
    pairs, more than an 8-bit count holds, next to short ones; returns (basis, nuclei)."""
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, 3.0, (3, 3))
    ls = np.array([0, 3, 1, 2, 4, 2], np.int32)
    ks = np.array([16, 20, 4, 20, 16, 1], np.int32)
    basis = _basis_from_lists(atoms[[0, 0, 1, 1, 2, 2]], ls, ks, rng, 0.05, 500.0, 0.1, 1.0)
    return basis, Nuclei(atoms.copy(), np.array([3.0, 6.0, 8.0]))


def density(nbf, seed=5, sigma=0.1):
    """Symmetric matrix with iid N(0, sigma^2) upper triangle (diagonal included)."""
    rng = np.random.default_rng(seed + 1000)
    D = np.triu(rng.normal(0.0, sigma, (nbf, nbf)))
    return D + np.triu(D, 1).T


def random_rotation(seed):
    """A uniformly random proper rotation matrix (QR of a Gaussian matrix)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def all_pairs(n_shells):
    """Every unordered shell pair a <= b, as two int32 arrays."""
    a, b = np.triu_indices(n_shells)
    return a.astype(np.int32), b.astype(np.int32)
