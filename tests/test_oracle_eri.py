"""Pins of the two-electron oracle (oracle/eri.py) against what fixes it independently: the s-s-s-s
closed form with F_0 from erf, the Gaussian-transform quadrature of tests/xcheck.py (its own
Cartesian harmonics), the nuclear-attraction oracle in the limit of a point-like ket charge,
the permutational symmetry and rotational invariance of the integral."""
import math

import numpy as np
import pytest

import oracle
import xcheck
from oracle import eri
from paper_2404_16245_amd import synth

# the u-quadrature of the cross-check meets its 1e-13 request only to about 1e-12 where terms cancel
pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def test_ssss_closed_form():
    rng = np.random.default_rng(0)
    for _ in range(5):
        A, B, C, D = rng.normal(0, 1.2, (4, 3))
        a, b, c, d = np.exp(rng.uniform(np.log(0.2), np.log(8.0), 4))
        p, q = a + b, c + d
        P, Q = (a * A + b * B) / p, (c * C + d * D) / q
        alpha = p * q / (p + q)
        T = alpha * float((P - Q) @ (P - Q))
        F0 = 1.0 if T < 1e-15 else 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        ref = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * F0 * math.exp(
            -a * b / p * float((A - B) @ (A - B)) - c * d / q * float((C - D) @ (C - D)))
        got = eri.eri_prim_real(0, A, a, 0, B, b, 0, C, c, 0, D, d)[0, 0, 0, 0]
        assert got == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("ls", [(1, 0, 0, 0), (1, 0, 1, 0), (1, 1, 1, 0), (2, 0, 1, 1), (2, 1, 0, 2), (2, 2, 1, 0)])
def test_primitive_blocks_against_gaussian_transform_quadrature(ls):
    rng = np.random.default_rng(sum(ls) * 7 + ls[0])
    cen = rng.normal(0, 0.9, (4, 3))
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), 4))
    args = [x for k in range(4) for x in (ls[k], cen[k], ex[k])]
    got = eri.eri_prim_real(*args)
    ref = xcheck.quad_eri_prim(*args)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()


def _shells(specs):
    """Basis of single-primitive (or contracted) shells from (l, center, exponents, coefs)."""
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


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 1)])
def test_point_charge_limit_is_the_nuclear_attraction(la, lb):
    # a ket of two normalised s shells of exponent g at C is a unit charge of width ~1/sqrt(g); as
    # g grows, (ab|cc) -> int chi_a chi_b / |r - C|, which is -V_ab of a unit nucleus at C (the
    # nuclear-attraction oracle); the error is O(1/g), removed by Richardson extrapolation
    rng = np.random.default_rng(10 * la + lb)
    A, B, C = rng.normal(0, 1.0, (3, 3))
    ea, eb = rng.uniform(0.4, 2.0, 2), rng.uniform(0.4, 2.0, 1)
    da = rng.uniform(0.3, 1.0, 2)
    vals = []
    for g in (2e5, 4e5):
        bs = _shells([(la, A, ea, da), (lb, B, eb, [1.0]), (0, C, [g], [1.0]), (0, C, [g], [1.0])])
        vals.append(eri.eri_block(bs, 0, 1, 2, 3)[:, :, 0, 0])
    extrap = 2 * vals[1] - vals[0]
    bs = _shells([(la, A, ea, da), (lb, B, eb, [1.0])])
    V = oracle.nuc_blocks(bs, synth.Nuclei(C[None, :], np.array([1.0])), np.array([0], np.int32),
                          np.array([1], np.int32)).reshape(2 * la + 1, 2 * lb + 1)
    assert np.abs(extrap + V).max() <= 1e-8 * np.abs(V).max(), np.abs(extrap + V).max() / np.abs(V).max()


def test_permutational_symmetry():
    b, _ = synth.molecule(seed=5, n_atoms=2, box=3.0, ls=(0, 1, 2), kmax=2)
    q = (1, 5, 2, 4)  # l = 1, 2, 2, 1
    X = eri.eri_block(b, *q)
    assert np.allclose(eri.eri_block(b, q[1], q[0], q[2], q[3]), X.transpose(1, 0, 2, 3), rtol=1e-13, atol=1e-15)
    assert np.allclose(eri.eri_block(b, q[0], q[1], q[3], q[2]), X.transpose(0, 1, 3, 2), rtol=1e-13, atol=1e-15)
    assert np.allclose(eri.eri_block(b, q[2], q[3], q[0], q[1]), X.transpose(2, 3, 0, 1), rtol=1e-13, atol=1e-15)


def test_rotation_invariance():
    # rotating every center rotates each index of the block by the real Wigner matrix of its l
    rng = np.random.default_rng(3)
    Qr, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Qr) < 0:
        Qr[:, 0] *= -1
    cen = rng.normal(0, 1.0, (4, 3))
    ls = (2, 1, 1, 2)
    ex = [0.8, 1.3, 0.6, 1.1]
    X = eri.eri_prim_real(*[x for k in range(4) for x in (ls[k], cen[k], ex[k])])
    Y = eri.eri_prim_real(*[x for k in range(4) for x in (ls[k], Qr @ cen[k], ex[k])])
    Ds = [xcheck.real_wigner_d(l, Qr) for l in ls]
    Xr = np.einsum("ai,bj,ck,dl,ijkl->abcd", Ds[0], Ds[1], Ds[2], Ds[3], X)
    assert np.allclose(Xr, Y, rtol=1e-10, atol=1e-12 * np.abs(X).max())
