"""Two-electron Coulomb integrals (ab|cd) over contracted real solid-harmonic Gaussians: the plain
textbook route (McMurchie-Davidson over Cartesian Gaussians, then the transform to the real solid
harmonics). Test infrastructure, like the rest of this package.

The paper's two-electron expressions (Eqs. 13-15 and the Supplement) are derived through a
Green's-function split whose intermediate formulas do not agree with each other, so the oracle
takes the integral's plain definition,
    (ab|cd) = int int chi_a(r1) chi_b(r1) chi_c(r2) chi_d(r2) / |r1 - r2| dr1 dr2,
with the basis of Eq. 1 (normalised primitives, renormalised contraction), and evaluates it by
the standard Hermite expansion: for primitive pairs (p, P) and (q, Q), alpha = pq/(p+q),
    (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd
              sum_tuv E^{ab}_tuv sum_t'u'v' (-1)^{t'+u'+v'} E^{cd}_t'u'v' R_{t+t', u+u', v+v'}(alpha, P - Q),
E the Hermite expansion coefficients of each Cartesian product about its center, R the Hermite
Coulomb integrals from the Boys function. Plain numpy in float64, written for clarity.
"""
import math

import numpy as np

from . import boys, solid_real


def cart_monomials(l):
    return [(l - s, s - k, k) for s in range(l + 1) for k in range(s + 1)]


_CART_REAL = {}


def cart_to_real(l):
    """C[m + l, q] with S^l_m(x, y, z) = sum_q C x^i y^j z^k over cart_monomials(l), fitted to the
    oracle's real solid harmonics at fixed points (exact up to rounding: a square-enough linear
    system of polynomials)."""
    if l not in _CART_REAL:
        mono = cart_monomials(l)
        pts = np.random.default_rng(1234 + l).normal(size=(4 * len(mono) + 8, 3))
        A = np.array([[x ** i * y ** j * z ** k for (i, j, k) in mono] for (x, y, z) in pts])
        S = np.array([solid_real(l, *p)[l * l:(l + 1) ** 2] for p in pts])
        C, *_ = np.linalg.lstsq(A, S, rcond=None)
        C = C.T
        C[np.abs(C) < 1e-13 * np.abs(C).max()] = 0.0
        _CART_REAL[l] = C
    return _CART_REAL[l]


def prim_norm(l, a):
    """N(l, alpha) of Eq. 1 for the real solid harmonics (Racah normalisation)."""
    dfact = 1.0
    for i in range(2 * l - 1, 0, -2):
        dfact *= i
    return math.sqrt(2.0 ** l * (2 * a) ** (l + 1.5) / (dfact * math.pi ** 1.5))


def shell_weights(basis, s):
    """Normalised contraction weights N_k d_k / sqrt(<chi|chi>) of shell s."""
    l = int(basis.l[s])
    o, K = int(basis.prim_off[s]), int(basis.nprim[s])
    a = np.asarray(basis.expo[o:o + K], dtype=float)
    d = np.asarray(basis.coef[o:o + K], dtype=float)
    N = np.array([prim_norm(l, x) for x in a])
    dfact = 1.0
    for i in range(2 * l - 1, 0, -2):
        dfact *= i
    ovl = (N[:, None] * N[None, :] * dfact * math.pi ** 1.5 / (2.0 ** l * (a[:, None] + a[None, :]) ** (l + 1.5)))
    norm = float(d @ ovl @ d)
    return a, N * d / math.sqrt(norm)


def hermite_E(i, j, xpa, xpb, p):
    """E^{ij}_t, t = 0..i+j: x_A^i x_B^j = sum_t E_t Lambda_t (Hermite Gaussians about P), K excluded."""
    E = np.zeros((i + 1, j + 1, i + j + 2))
    E[0, 0, 0] = 1.0
    for a in range(i + 1):
        for b in range(j + 1):
            if a == 0 and b == 0:
                continue
            for t in range(a + b + 1):
                if a > 0:
                    prev, x = E[a - 1, b], xpa
                else:
                    prev, x = E[a, b - 1], xpb
                v = x * prev[t] + (t + 1) * prev[t + 1]
                if t > 0:
                    v += prev[t - 1] / (2 * p)
                E[a, b, t] = v
    return E[i, j, :i + j + 1]


def hermite_R(L, alpha, R):
    """R_tuv(alpha, R) for t + u + v <= L by the McMurchie-Davidson recursion."""
    X, Y, Z = R
    F = boys(L, alpha * float(R @ R))
    Rn = np.zeros((L + 1, L + 1, L + 1, L + 1))
    for n in range(L + 1):
        Rn[n, 0, 0, 0] = (-2 * alpha) ** n * F[n]
    for tot in range(1, L + 1):
        for n in range(L - tot, -1, -1):
            for t in range(tot + 1):
                for u in range(tot - t + 1):
                    v = tot - t - u
                    if t > 0:
                        val = X * Rn[n + 1, t - 1, u, v] + ((t - 1) * Rn[n + 1, t - 2, u, v] if t > 1 else 0.0)
                    elif u > 0:
                        val = Y * Rn[n + 1, t, u - 1, v] + ((u - 1) * Rn[n + 1, t, u - 2, v] if u > 1 else 0.0)
                    else:
                        val = Z * Rn[n + 1, t, u, v - 1] + ((v - 1) * Rn[n + 1, t, u, v - 2] if v > 1 else 0.0)
                    Rn[n, t, u, v] = val
    return Rn[0]


def _pair_E(la, A, a, lb, B, b):
    """Hermite coefficients of every Cartesian product of the pair: [ncart_a * ncart_b, (L+1)^3]."""
    p = a + b
    P = (a * A + b * B) / p
    L = la + lb
    ma, mb = cart_monomials(la), cart_monomials(lb)
    out = np.zeros((len(ma) * len(mb), L + 1, L + 1, L + 1))
    for u, (i1, j1, k1) in enumerate(ma):
        for v, (i2, j2, k2) in enumerate(mb):
            ex = hermite_E(i1, i2, P[0] - A[0], P[0] - B[0], p)
            ey = hermite_E(j1, j2, P[1] - A[1], P[1] - B[1], p)
            ez = hermite_E(k1, k2, P[2] - A[2], P[2] - B[2], p)
            out[u * len(mb) + v, :len(ex), :len(ey), :len(ez)] = ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
    return p, P, out


def eri_prim_real(la, A, a, lb, B, b, lc, C, c, ld, D, d):
    """Unnormalised primitive (ab|cd) block over the real solid harmonics S^l_m (no N, no
    contraction): shape (2la+1, 2lb+1, 2lc+1, 2ld+1)."""
    A, B, C, D = (np.asarray(x, float) for x in (A, B, C, D))
    p, P, Eab = _pair_E(la, A, a, lb, B, b)
    q, Q, Ecd = _pair_E(lc, C, c, ld, D, d)
    L1, L2 = la + lb, lc + ld
    alpha = p * q / (p + q)
    R = hermite_R(L1 + L2, alpha, P - Q)
    Kab = math.exp(-a * b / p * float((A - B) @ (A - B)))
    Kcd = math.exp(-c * d / q * float((C - D) @ (C - D)))
    # contract: sum over (t,u,v) of the bra and (t',u',v') of the ket with R_{t+t',u+u',v+v'}
    sign = np.array([[[(-1.0) ** (t + u + v) for v in range(L2 + 1)] for u in range(L2 + 1)] for t in range(L2 + 1)])
    Ecd_s = Ecd * sign[None]
    Rm = np.zeros(((L1 + 1) ** 3, (L2 + 1) ** 3))
    for t in range(L1 + 1):
        for u in range(L1 + 1):
            for v in range(L1 + 1):
                if t + u + v > L1:
                    continue
                row = (t * (L1 + 1) + u) * (L1 + 1) + v
                Rm[row] = R[t:t + L2 + 1, u:u + L2 + 1, v:v + L2 + 1].reshape(-1)
    cart = Eab.reshape(Eab.shape[0], -1) @ Rm @ Ecd_s.reshape(Ecd_s.shape[0], -1).T
    cart *= 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * Kab * Kcd
    nca, ncb = len(cart_monomials(la)), len(cart_monomials(lb))
    ncc, ncd = len(cart_monomials(lc)), len(cart_monomials(ld))
    cart = cart.reshape(nca, ncb, ncc, ncd)
    return np.einsum("ai,bj,ck,dl,ijkl->abcd", cart_to_real(la), cart_to_real(lb), cart_to_real(lc),
                     cart_to_real(ld), cart)


def eri_block(basis, sa, sb, sc, sd):
    """Contracted (ab|cd) block of shells sa, sb, sc, sd: shape (2la+1, 2lb+1, 2lc+1, 2ld+1)."""
    ls = [int(basis.l[s]) for s in (sa, sb, sc, sd)]
    cen = [np.asarray(basis.center[s], float) for s in (sa, sb, sc, sd)]
    ws = [shell_weights(basis, s) for s in (sa, sb, sc, sd)]
    out = np.zeros(tuple(2 * l + 1 for l in ls))
    for ea, wa in zip(*ws[0]):
        for eb, wb in zip(*ws[1]):
            for ec, wc in zip(*ws[2]):
                for ed, wd in zip(*ws[3]):
                    out += wa * wb * wc * wd * eri_prim_real(ls[0], cen[0], ea, ls[1], cen[1], eb, ls[2], cen[2], ec,
                                                             ls[3], cen[3], ed)
    return out


def eri_blocks(basis, quartets):
    """Concatenated (ab|cd) blocks (row-major, a slowest) for quartets [n, 4] of shell indices."""
    return np.concatenate([eri_block(basis, *map(int, q)).ravel() for q in np.asarray(quartets)]) \
        if len(quartets) else np.zeros(0)
