"""CPU checks of the GPU path's generated tables and algorithm (no GPU needed).

The class code emitted by ``csrc/gen_classes.py`` rests on: real solid harmonics by recurrence,
the real Gaunt table (product rule), the shift coefficients along the A->B axis (Eq. 8 with
mu = m), the constant rotation J and the z rotations. Each is checked here against facts
outside the generator, and ``emulate_block`` (a numpy run of exactly the emitted term lists)
is compared with the oracle for every class.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import xcheck
from paper_2404_16245_amd import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                "paper_2404_16245_amd", "csrc"))
import gen_classes as gc  # noqa: E402


def test_recurrence_harmonics_against_scipy_fit():
    pts = np.random.default_rng(0).normal(size=(6, 3))
    S = gc.solid_real(12, pts)
    for l in range(13):
        ref = np.array([xcheck.eval_real_solid(l, *p) for p in pts])
        assert np.allclose(S[:, l * l:(l + 1) ** 2], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_gaunt_table_reproduces_products():
    g = gc.real_gaunt_table()
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = rng.normal(size=3)
        r2 = float(v @ v)
        S = gc.solid_real(2 * gc.LMAX_SHELL, v[None])[0]
        for l1 in range(gc.LMAX_SHELL + 1):
            for l2 in range(gc.LMAX_SHELL + 1):
                for m1 in range(-l1, l1 + 1):
                    for m2 in range(-l2, l2 + 1):
                        i1, i2 = l1 * l1 + m1 + l1, l2 * l2 + m2 + l2
                        s = 0.0
                        for L in range(abs(l1 - l2), l1 + l2 + 1, 2):
                            k = (l1 + l2 - L) // 2
                            s += r2 ** k * float(g[i1, i2, L * L:(L + 1) ** 2] @ S[L * L:(L + 1) ** 2])
                        ref = S[i1] * S[i2]
                        assert abs(s - ref) <= 1e-12 * max(1.0, abs(ref))


def test_gaunt_table_against_clebsch_gordan():
    # real Gaunt = U_l1 (x) U_l2 (x) conj(U_L) applied to <l1 0 l2 0|L0><l1 m1 l2 m2|LM> (oracle's CG)
    def U(l):
        d = 2 * l + 1
        M = np.zeros((d, d), complex)
        h = 1 / math.sqrt(2)
        M[l, l] = 1
        for m in range(1, l + 1):
            M[m + l, m + l] = (-1) ** m * h
            M[m + l, -m + l] = h
            M[-m + l, -m + l] = 1j * h
            M[-m + l, m + l] = -1j * (-1) ** m * h
        return M
    g = gc.real_gaunt_table()
    for (l1, l2) in [(2, 3), (6, 6), (4, 1), (5, 5), (7, 7), (7, 2)]:
        for L in range(abs(l1 - l2), l1 + l2 + 1, 2):
            Gc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * L + 1))
            c0 = oracle.cg(l1, 0, l2, 0, L, 0)
            for u1 in range(-l1, l1 + 1):
                for u2 in range(-l2, l2 + 1):
                    if abs(u1 + u2) <= L:
                        Gc[u1 + l1, u2 + l2, u1 + u2 + L] = c0 * oracle.cg(l1, u1, l2, u2, L, u1 + u2)
            R = np.einsum("ai,bj,ck,ijk->abc", U(l1), U(l2), U(L).conj(), Gc)
            ours = g[l1 * l1:(l1 + 1) ** 2, l2 * l2:(l2 + 1) ** 2, L * L:(L + 1) ** 2]
            assert np.abs(ours - R.real).max() < 2e-15


@pytest.mark.parametrize("l", range(7))
def test_rotation_tables(l):
    J = gc.rot_x90(l)
    assert np.allclose(J @ J.T, np.eye(2 * l + 1), atol=1e-15)
    R = np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]])
    rng = np.random.default_rng(2 + l)
    th = 0.7
    cz = [math.cos(m * th) for m in range(l + 1)]
    sz = [math.sin(m * th) for m in range(l + 1)]
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    for _ in range(3):
        v = rng.normal(size=3)
        S = gc.solid_real(l, v[None])[0, l * l:]
        assert np.allclose(gc.solid_real(l, (R @ v)[None])[0, l * l:], J @ S, atol=1e-12)
        assert np.allclose(gc.solid_real(l, (Rz @ v)[None])[0, l * l:], gc.zrot(l, cz, sz) @ S, atol=1e-12)


def test_shift_along_z_keeps_m():
    rng = np.random.default_rng(3)
    v, t = rng.normal(size=3), 0.83
    S = gc.solid_real(gc.LMAX_SHELL, v[None])[0]
    St = gc.solid_real(gc.LMAX_SHELL, (v + [0, 0, t])[None])[0]
    for l in range(gc.LMAX_SHELL + 1):
        for m in range(-l, l + 1):
            s = sum(gc.trans_coef(l, l1, m) * t ** (l - l1) * S[l1 * l1 + m + l1] for l1 in range(abs(m), l + 1))
            assert s == pytest.approx(St[l * l + m + l], rel=1e-12, abs=1e-12)


def test_groups_partition_families():
    for LA in range(gc.LMAX_SHELL + 1):
        for LB in range(LA + 1):
            groups = gc.class_groups(LA, LB)
            units = sorted(u for g in groups for u in g)
            assert units == sorted(gc.class_units(LA, LB))
            cap = max(gc.class_cap(LA, LB), max(len(gc.unit_entries(LA, LB, u)) for u in units))
            assert all(sum(len(gc.unit_entries(LA, LB, u)) for u in g) <= cap for g in groups)
            # the half-families together hold every W entry of every |M| family exactly once
            ent = sorted(e for g in groups for u in g for e in gc.unit_entries(LA, LB, u))
            ref = sorted(e for mu in range(LA + LB + 1) for e in gc.family_entries(LA, LB, mu))
            assert ent == ref


CLASSES = [(la, lb) for la in range(7) for lb in range(la + 1)]


@pytest.mark.parametrize("la,lb", CLASSES)
def test_emulated_algorithm_against_oracle(la, lb):
    rng = np.random.default_rng(500 + 10 * la + lb)
    A, B = rng.uniform(0, 3, 3), rng.uniform(0, 3, 3)
    ea, eb = rng.uniform(0.3, 4, 2), rng.uniform(0.3, 4, 1)
    da, db = rng.uniform(0.1, 1, 2), np.ones(1)
    bs = synth.Basis(np.array([A, B]), np.array([la, lb], np.int32), np.array([2, 1], np.int32),
                     np.array([0, 2], np.int64), np.concatenate([ea, eb]), np.concatenate([da, db]))
    nuc = synth.Nuclei(rng.uniform(0, 3, (2, 3)), np.array([2.0, 5.0]))
    ref = oracle.nuc_blocks(bs, nuc, [0], [1], precision=2).reshape(2 * la + 1, 2 * lb + 1)
    wa, wb = xcheck.contracted_weights(la, ea, da), xcheck.contracted_weights(lb, eb, db)
    V = gc.emulate_block(la, lb, A, B, ea, wa, eb, wb, nuc.pos, nuc.Z)
    assert np.all(np.abs(V - ref) <= 1e-13 + 1e-11 * np.abs(ref))


def test_emulated_algorithm_on_z_axis_and_same_center():
    # R along z (identity frame) and R = 0 (A = B)
    nuc = synth.Nuclei(np.array([[0.2, -0.4, 1.1]]), np.array([3.0]))
    for B in ([0.0, 0.0, 1.3], [0.0, 0.0, -0.7], [0.0, 0.0, 0.0]):
        A = np.zeros(3)
        bs = synth.Basis(np.array([A, B]), np.array([4, 3], np.int32), np.array([1, 1], np.int32),
                         np.array([0, 1], np.int64), np.array([0.8, 1.9]), np.ones(2))
        ref = oracle.nuc_blocks(bs, nuc, [0], [1], precision=2).reshape(9, 7)
        wa, wb = xcheck.contracted_weights(4, [0.8], [1.0]), xcheck.contracted_weights(3, [1.9], [1.0])
        V = gc.emulate_block(4, 3, A, B, [0.8], wa, [1.9], wb, nuc.pos, nuc.Z)
        assert np.all(np.abs(V - ref) <= 1e-13 + 1e-11 * np.abs(ref))


# ---------------------------------------------------------------------------------------------
# gradient kernel tables and algorithm
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("l", range(1, 7))
def test_harmonic_gradients_and_gradient_matrices(l):
    rng = np.random.default_rng(60 + l)
    X = rng.normal(size=(4, 3))
    S, dS = gc.solid_real_grad(l, X)
    g = gc.grad_matrix(l)
    h = 1e-5
    for xi in range(3):
        e = np.zeros(3)
        e[xi] = h
        fd = (gc.solid_real(l, X + e) - gc.solid_real(l, X - e)) / (2 * h)
        assert np.allclose(dS[xi], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())
        # the gradient of S^l is a combination of S^{l-1}
        lower = gc.solid_real(l - 1, X)[:, (l - 1) ** 2:]
        assert np.allclose(dS[xi][:, l * l:], lower @ g[xi].T, rtol=1e-12, atol=1e-12 * np.abs(dS[xi]).max())


def test_grad_tables_cover_the_coupling():
    # the kind-0 table of each class is the forward coupling, term for term
    for la, lb in [(2, 1), (3, 3), (6, 4)]:
        fwd = gc.class_terms(la, lb)
        t0 = [t for t in gc.grad_tables(la, lb) if t[0] == 0]
        assert len(t0) == len(fwd)
        assert sorted(t[5] for t in t0) == sorted(t[7] for t in fwd)


GRAD_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 2), (3, 1), (3, 3), (4, 2), (5, 1), (6, 3)]


@pytest.mark.parametrize("la,lb", GRAD_CLASSES)
def test_emulated_gradient_against_oracle(la, lb):
    rng = np.random.default_rng(700 + 10 * la + lb)
    A, B = rng.uniform(0, 2, 3), rng.uniform(0, 2, 3)
    ea, eb = rng.uniform(0.3, 3, 2), rng.uniform(0.3, 3, 1)
    da, db = rng.uniform(0.2, 1, 2), np.ones(1)
    bs = synth.Basis(np.array([A, B]), np.array([la, lb], np.int32), np.array([2, 1], np.int32),
                     np.array([0, 2], np.int64), np.concatenate([ea, eb]), np.concatenate([da, db]))
    nuc = synth.Nuclei(rng.uniform(0, 2, (2, 3)), np.array([2.0, 5.0]))
    D = np.zeros((bs.nbf(), bs.nbf()))
    Dt = rng.normal(size=(2 * la + 1, 2 * lb + 1))
    D[:2 * la + 1, 2 * la + 1:] = Dt
    dn, dc, E = oracle.grad(bs, nuc, D)
    wa, wb = xcheck.contracted_weights(la, ea, da), xcheck.contracted_weights(lb, eb, db)
    Ee, dAe, dBe, dCe = gc.emulate_grad(la, lb, A, B, ea, wa, eb, wb, nuc.pos, nuc.Z, Dt)
    scale = max(1.0, np.abs(np.concatenate([dn, dc])).max())
    assert Ee == pytest.approx(E, rel=1e-12, abs=1e-13)
    assert np.allclose(dAe, dc[0], atol=1e-12 * scale)
    assert np.allclose(dBe, dc[1], atol=1e-12 * scale)
    assert np.allclose(dCe, dn, atol=1e-12 * scale)


def test_emulated_gradient_same_center_and_z_axis():
    # A = B (R = 0: the frame is the identity and the R-derivative comes from the l = 1 shifts)
    # and R along -z
    nuc = synth.Nuclei(np.array([[0.2, -0.4, 1.1], [0.5, 0.3, -0.2]]), np.array([3.0, 1.0]))
    rng = np.random.default_rng(9)
    for B in ([0.0, 0.0, 0.0], [0.0, 0.0, -0.9]):
        A = np.zeros(3)
        bs = synth.Basis(np.array([A, B]), np.array([3, 2], np.int32), np.array([1, 1], np.int32),
                         np.array([0, 1], np.int64), np.array([0.8, 1.9]), np.ones(2))
        D = np.zeros((12, 12))
        Dt = rng.normal(size=(7, 5))
        D[:7, 7:] = Dt
        dn, dc, E = oracle.grad(bs, nuc, D)
        wa, wb = xcheck.contracted_weights(3, [0.8], [1.0]), xcheck.contracted_weights(2, [1.9], [1.0])
        Ee, dAe, dBe, dCe = gc.emulate_grad(3, 2, A, B, [0.8], wa, [1.9], wb, nuc.pos, nuc.Z, Dt)
        scale = max(1.0, np.abs(np.concatenate([dn, dc])).max())
        assert Ee == pytest.approx(E, rel=1e-12, abs=1e-13)
        assert np.allclose(np.concatenate([dAe, dBe, dCe.reshape(-1)]),
                           np.concatenate([dc[0], dc[1], dn.reshape(-1)]), atol=1e-12 * scale)


@pytest.mark.parametrize("L", range(2 * gc.CART_LMAX + 1))
def test_cartesian_route_hermite_closed_form(L):
    # the closed form the Cartesian kernel's nucleus step is generated from, term by term, against
    # the McMurchie-Davidson recursion for R_tuv written independently in tests/xcheck.py
    rng = np.random.default_rng(10 + L)
    for _ in range(3):
        p = float(np.exp(rng.uniform(np.log(0.2), np.log(20.0))))
        PC = rng.normal(0, 0.8, 3)
        ref = xcheck._hermite_R(L, p, PC)
        T = p * float(PC @ PC)
        g = [(-2 * p) ** n * float(xcheck.boys_mp(n, T)) for n in range(L + 1)]
        tl = gc.tuv_list(L)
        assert len(tl) == (L + 1) * (L + 2) * (L + 3) // 6
        for n, terms in gc.cart_r_terms(L):
            got = sum(c * PC[0] ** a * PC[1] ** b * PC[2] ** cc * g[gn] for c, a, b, cc, gn in terms)
            want = ref(*tl[n])
            assert got == pytest.approx(want, rel=1e-11, abs=1e-13 * max(1.0, abs(want)))


def test_cartesian_route_real_harmonic_coefficients():
    # S^l_m as polynomials in the Cartesian monomials, against the recurrences at random points
    # and against the monomial expansion written independently in tests/xcheck.py
    pts = np.random.default_rng(4).normal(size=(7, 3))
    for l in range(gc.CART_LMAX + 1):
        C = gc.solid_real_poly(l)
        mono = gc.cart_monomials(l)
        assert len(mono) == (l + 1) * (l + 2) // 2
        M = np.array([[x ** i * y ** j * z ** k for (i, j, k) in mono] for (x, y, z) in pts])
        S = gc.solid_real(l, pts)[:, l * l:(l + 1) ** 2]
        assert np.allclose(M @ C.T, S, rtol=1e-13, atol=1e-13 * np.abs(S).max())
        ref = np.array([xcheck.eval_real_solid(l, *pt) for pt in pts])
        assert np.allclose(M @ C.T, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


ERI_LS = [(la, lb, lc, ld) for la in range(3) for lb in range(3) for lc in range(3) for ld in range(3)]


@pytest.mark.parametrize("ls", ERI_LS[::3] + [(2, 2, 2, 2), (0, 2, 1, 2)])
def test_emulated_two_electron_route_against_oracle(ls):
    # the solid-harmonic two-electron route (pair distributions in the pair frames, rotated to the
    # lab, the j-transform of |u|^{2k}, Gaunt coupling of the two sides) against the Hermite oracle
    from oracle import eri
    rng = np.random.default_rng(sum(l * 3 ** i for i, l in enumerate(ls)))
    cen = rng.normal(0, 1.0, (4, 3))
    ex = np.exp(rng.uniform(np.log(0.3), np.log(4.0), 4))
    args = [x for k in range(4) for x in (ls[k], cen[k], ex[k])]
    got = gc.emulate_eri_prim(*args)
    ref = eri.eri_prim_real(*args)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()


def test_emulated_two_electron_route_degenerate_geometries():
    # bra pair on one center, ket pair along z, and the two pair centers coinciding (T = 0)
    from oracle import eri
    A = np.array([0.3, -0.2, 0.5])
    C = np.array([0.0, 0.0, -0.4])
    D = np.array([0.0, 0.0, 0.9])
    # blocks of odd total l on one center vanish exactly: the scale is the (ss|ss) integral
    for ls in [(2, 1, 2, 0), (1, 1, 1, 1), (2, 2, 0, 2)]:
        for cen in ([A, A, C, D], [A, A, A, A]):
            args = [x for k in range(4) for x in (ls[k], cen[k], (0.9, 1.4, 0.7, 1.1)[k])]
            got, ref = gc.emulate_eri_prim(*args), eri.eri_prim_real(*args)
            scale = abs(eri.eri_prim_real(*[0 if i % 3 == 0 else x for i, x in enumerate(args)])[0, 0, 0, 0])
            assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), scale)
