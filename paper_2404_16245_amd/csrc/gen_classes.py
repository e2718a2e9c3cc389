"""Generator of the class-specific device code of the nuclear-attraction kernel.

For every class (LA, LB) with LA >= LB it emits straight-line HIP code for

* the nucleus step: real solid harmonics S^L_M(C) of the nucleus position relative to the
  Gaussian-product center P, in the frame whose z axis is the A->B axis (Eq. 2 normalisation,
  built with the standard sectoral and vertical recurrences), times
  G_{L,k}(T) = sum_{j<=k} T^j/j! Z F_{L+j}(T), accumulated into W(L, M, k) (the one-center
  Coulomb integral of Eq. 11's last line, completed with the product rule; Eq. 12 is the k = 0
  case);
* the coupling: the product rule of real solid harmonics (the supplement's Eq. 4 in the real
  basis) and the shift of both harmonics to P (Eq. 7, Eq. 8's coefficients). Along the A->B axis
  the shift keeps m, so the block is
    V'(ma, mb) = sum_{l1, l2} c(LA, l1, |ma|) t_a^{LA-l1} c(LB, l2, |mb|) t_b^{LB-l2}
                 sum_{L, M} g(l1 ma, l2 mb; L M) W_s(L, M, (l1 + l2 - L)/2)
  with t_a = beta R/p, t_b = -alpha R/p and c(l, l1, m) = sqrt(C(l+m, l1+m) C(l-m, l1-m));
* the rotation back to the laboratory frame, D^l(Q)^T = Z(phi) J^T Z(theta) J with the constant
  matrix J = D^l(rotation by +pi/2 about x) and z rotations Z.

The W entries of one class are split into half-families (the entries with M = +mu, or with
M = -mu) and packed into groups that each fit a register budget; one wavefront of the kernel
runs one group for 64 shell pairs.

The tables (real Gaunt coefficients g, the J matrices) are computed here by exact quadrature on
the unit sphere of polynomials evaluated with the same recurrences the kernel uses. The module
also offers ``emulate_block``, a numpy execution of exactly the emitted term lists, used by the
CPU tests to check the tables and the layout before any GPU run.

Usage: python gen_classes.py OUTPUT_HEADER [--cap N]
"""
import math
import os
import sys

import numpy as np

LMAX_SHELL = 7
DEFAULT_CAP = 64          # register budget of one group, in doubles of W
# Classes up to this la have a binary32 (double-float) coupling for the mixed-precision kernel;
# above it the mixed kernel keeps the binary64 coupling (the expanded double-float code of the
# l = 5, 6 classes, up to 12,000 terms per class, took most of ten minutes to compile).
MIXED_LMAX = 4
# Classes whose budget differs. Every group recomputes the nucleus geometry and the Boys row, so
# fewer groups save work while the nucleus loop stays nearly free of spills: (4, 4) runs in three
# groups of at most 56 (on the 200-atom batched molecule 5.6% faster than four of 44, and 15% and
# 50% faster than five of 36 and six of 32). (5, 5) and (6, 4) take four groups of at most 72 and
# (5, 3) and (6, 2) four of 44, so that with the tiles per work item that LDS allows there are
# eight tasks for the eight wavefronts of a workgroup.
CLASS_CAP = {(5, 5): 72, (6, 4): 72, (4, 4): 56, (5, 3): 44, (6, 2): 44}


def class_cap(LA, LB):
    return CLASS_CAP.get((LA, LB), DEFAULT_CAP)
KEEP = 1e-14              # drop real Gaunt coefficients below this magnitude


# ----------------------------------------------------------------------------------------------
# Real solid harmonics by recurrence (Racah normalisation, order m = -l..l, index l*l + m + l)
# ----------------------------------------------------------------------------------------------
def sect_coef(l):
    """S^{l+1}_{+-(l+1)} = f_l (x S^l_l -+ y S^l_{-l}) ... with f_0 = 1."""
    return 1.0 if l == 0 else math.sqrt((2 * l + 1) / (2 * l + 2))


def vert_coefs(l, m):
    """S^{l+1}_m = a z S^l_m - b r^2 S^{l-1}_m (|m| <= l)."""
    m = abs(m)
    den = math.sqrt((l + m + 1) * (l - m + 1))
    return (2 * l + 1) / den, math.sqrt((l + m) * (l - m)) / den


def solid_real(lmax, pts):
    """Real solid harmonics at points pts (N, 3) -> (N, (lmax+1)^2), in the dtype of pts
    (recurrence coefficients are evaluated in that dtype, so long double inputs give long
    double accuracy)."""
    pts = np.atleast_2d(pts)
    dt = pts.dtype
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    r2 = x * x + y * y + z * z
    S = np.zeros((pts.shape[0], (lmax + 1) ** 2), dtype=dt)
    idx = lambda l, m: l * l + m + l
    S[:, 0] = 1.0
    sc, ss = np.ones_like(x), np.zeros_like(x)
    for l in range(lmax):
        f = dt.type(1) if l == 0 else np.sqrt(dt.type(2 * l + 1) / dt.type(2 * l + 2))
        sc, ss = f * (x * sc - y * ss), f * (y * sc + x * ss)
        S[:, idx(l + 1, l + 1)] = sc
        S[:, idx(l + 1, -(l + 1))] = ss
    for m in range(0, lmax + 1):
        for sgn in ([1] if m == 0 else [1, -1]):
            mm = sgn * m
            prev = np.zeros_like(x)
            cur = S[:, idx(m, mm)].copy()
            for l in range(m, lmax):
                den = np.sqrt(dt.type((l + m + 1) * (l - m + 1)))
                a = dt.type(2 * l + 1) / den
                b = np.sqrt(dt.type((l + m) * (l - m))) / den
                nxt = a * z * cur - b * r2 * prev
                S[:, idx(l + 1, mm)] = nxt
                prev, cur = cur, nxt
    return S


def solid_real_grad(lmax, pts):
    """Real solid harmonics and their Cartesian gradients by forward-mode differentiation of the
    same recurrences: returns S (N, n) and dS (3, N, n), n = (lmax+1)^2, in the dtype of pts."""
    pts = np.atleast_2d(pts)
    dt = pts.dtype
    N = pts.shape[0]
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    r2 = x * x + y * y + z * z
    one, zero = np.ones(N, dtype=dt), np.zeros(N, dtype=dt)
    dx = [one, zero, zero]
    dy = [zero, one, zero]
    dz = [zero, zero, one]
    dr2 = [2 * x, 2 * y, 2 * z]
    S = np.zeros((N, (lmax + 1) ** 2), dtype=dt)
    dS = np.zeros((3, N, (lmax + 1) ** 2), dtype=dt)
    idx = lambda l, m: l * l + m + l
    S[:, 0] = 1.0
    sc, ss = one.copy(), zero.copy()
    dsc, dss = [zero.copy() for _ in range(3)], [zero.copy() for _ in range(3)]
    for l in range(lmax):
        f = dt.type(1) if l == 0 else np.sqrt(dt.type(2 * l + 1) / dt.type(2 * l + 2))
        nsc = f * (x * sc - y * ss)
        nss = f * (y * sc + x * ss)
        ndsc = [f * (dx[i] * sc + x * dsc[i] - dy[i] * ss - y * dss[i]) for i in range(3)]
        ndss = [f * (dy[i] * sc + y * dsc[i] + dx[i] * ss + x * dss[i]) for i in range(3)]
        sc, ss, dsc, dss = nsc, nss, ndsc, ndss
        S[:, idx(l + 1, l + 1)] = sc
        S[:, idx(l + 1, -(l + 1))] = ss
        for i in range(3):
            dS[i, :, idx(l + 1, l + 1)] = dsc[i]
            dS[i, :, idx(l + 1, -(l + 1))] = dss[i]
    for m in range(0, lmax + 1):
        for sgn in ([1] if m == 0 else [1, -1]):
            mm = sgn * m
            prev, dprev = zero.copy(), [zero.copy() for _ in range(3)]
            cur, dcur = S[:, idx(m, mm)].copy(), [dS[i, :, idx(m, mm)].copy() for i in range(3)]
            for l in range(m, lmax):
                den = np.sqrt(dt.type((l + m + 1) * (l - m + 1)))
                a = dt.type(2 * l + 1) / den
                b = np.sqrt(dt.type((l + m) * (l - m))) / den
                nxt = a * z * cur - b * r2 * prev
                dnxt = [a * (dz[i] * cur + z * dcur[i]) - b * (dr2[i] * prev + r2 * dprev[i]) for i in range(3)]
                S[:, idx(l + 1, mm)] = nxt
                for i in range(3):
                    dS[i, :, idx(l + 1, mm)] = dnxt[i]
                prev, cur, dprev, dcur = cur, nxt, dcur, dnxt
    return S, dS


def _gauss_legendre_ld(n):
    """Gauss-Legendre nodes and weights in long double (Newton refinement of numpy's)."""
    x0, _ = np.polynomial.legendre.leggauss(n)
    x = x0.astype(np.longdouble)
    for _ in range(4):
        p0, p1 = np.ones_like(x), x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / (x * x - 1)
        x = x - p1 / dp
    p0, p1 = np.ones_like(x), x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    w = 2 / ((1 - x * x) * dp * dp)
    return x, w


def sphere_grid(order):
    """Quadrature exact for polynomials of degree <= order on the unit sphere (long double)."""
    ngl = order // 2 + 2
    nphi = order + 2
    zg, wg = _gauss_legendre_ld(ngl)
    phi = np.longdouble(2) * np.arccos(np.longdouble(-1)) * np.arange(nphi, dtype=np.longdouble) / nphi
    Z, PHI = np.meshgrid(zg, phi, indexing="ij")
    W = np.outer(wg, np.full(nphi, np.longdouble(2) * np.arccos(np.longdouble(-1)) / nphi))
    s = np.sqrt(1 - Z * Z)
    pts = np.stack([s * np.cos(PHI), s * np.sin(PHI), Z], axis=-1).reshape(-1, 3)
    return pts, W.reshape(-1)


_GAUNT = None


def real_gaunt_table():
    """g[i1, i2, I] with S^{l1}_{m1} S^{l2}_{m2} = sum_{L,M} g r^{l1+l2-L} S^L_M, l1, l2 <= LMAX_SHELL."""
    global _GAUNT
    if _GAUNT is None:
        lm, Lm = LMAX_SHELL, 2 * LMAX_SHELL
        pts, w = sphere_grid(lm + lm + Lm + 2)
        S = solid_real(Lm, pts)
        n = (lm + 1) ** 2
        four_pi = 4 * np.arccos(np.longdouble(-1))
        norm = np.array([np.longdouble(2 * L + 1) / four_pi for L in range(Lm + 1) for _ in range(2 * L + 1)])
        wa = w[:, None] * S[:, :n]
        g = np.einsum("pa,pb,pc->abc", wa, S[:, :n], S) * norm[None, None, :]
        g = g.astype(np.float64)
        g[np.abs(g) < KEEP] = 0.0
        _GAUNT = g
    return _GAUNT


def rot_x90(l):
    """J = D^l(R) for R = rotation by +pi/2 about x: S^l(R v) = J S^l(v)."""
    pts, w = sphere_grid(2 * l + 2)
    R = np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]], dtype=np.longdouble)
    a = solid_real(l, pts @ R.T)[:, l * l:]
    b = solid_real(l, pts)[:, l * l:]
    J = np.longdouble(2 * l + 1) / (4 * np.arccos(np.longdouble(-1))) * np.einsum("p,pi,pj->ij", w, a, b)
    J = J.astype(np.float64)
    J[np.abs(J) < 1e-14] = 0.0
    return J


_GRADM = {}


def grad_matrix(l):
    """g[xi] ((2l+1) x (2l-1)): d/d(x, y, z)_xi S^l_m = sum_m' g[xi][m+l, m'+l-1] S^{l-1}_m', by exact
    sphere quadrature of the differentiated recurrences (l >= 1)."""
    if l not in _GRADM:
        pts, w = sphere_grid(2 * l)
        S, dS = solid_real_grad(l, pts)
        lo = S[:, (l - 1) ** 2:l * l]
        norm = np.longdouble(2 * l - 1) / (4 * np.arccos(np.longdouble(-1)))
        g = np.stack([norm * np.einsum("p,pi,pj->ij", w, dS[i][:, l * l:], lo) for i in range(3)]).astype(np.float64)
        g[np.abs(g) < 1e-14] = 0.0
        _GRADM[l] = g
    return _GRADM[l]


def monic_c(L, mu):
    """S^L_{+-mu} = monic_c(L, mu) * Q_L for the monic recurrences of the nucleus step."""
    c = 1.0
    for l in range(mu):
        c *= sect_coef(l)
    for l in range(mu, L):
        c *= vert_coefs(l, mu)[0]
    return c


def monic_e(l, mu):
    """e_l of the monic vertical recurrence Q_{l+1} = z Q_l - e_l r^2 Q_{l-1}."""
    a, b = vert_coefs(l, mu)
    a_prev = vert_coefs(l - 1, mu)[0]
    return b / (a * a_prev)


def trans_coef(l, l1, m):
    """c(l, l1, m) = eps_{l l1 m m} (Eq. 8): shift of S^l_m along z keeps m."""
    m = abs(m)
    return math.sqrt(math.comb(l + m, l1 + m) * math.comb(l - m, l1 - m))


# ----------------------------------------------------------------------------------------------
# Class layout: families, groups, W index map
# ----------------------------------------------------------------------------------------------
def kmax_of(LA, LB, L):
    return min(LB, (LA + LB - L) // 2)


def family_entries(LA, LB, mu):
    """Ordered W entries (L, M, k) of family |M| = mu: L ascending, k ascending, cos then sin."""
    out = []
    for L in range(mu, LA + LB + 1):
        for k in range(kmax_of(LA, LB, L) + 1):
            out.append((L, mu, k))
            if mu > 0:
                out.append((L, -mu, k))
    return out


def class_units(LA, LB):
    """Half-families (mu, sign): the entries with M = +mu (cosine type) or M = -mu (sine type).
    The two halves of a family run independent vertical recurrences, so they can sit in
    different groups."""
    return [(0, 1)] + [(mu, sg) for mu in range(1, LA + LB + 1) for sg in (1, -1)]


def unit_entries(LA, LB, unit):
    """Ordered W entries (L, M, k) of a half-family: L ascending, k ascending."""
    mu, sg = unit
    return [(L, sg * mu, k) for L in range(mu, LA + LB + 1) for k in range(kmax_of(LA, LB, L) + 1)]


def unit_of(M):
    return (abs(M), 1 if M >= 0 else -1)


def class_groups(LA, LB, cap=None):
    """Partition the half-families into groups of at most max(cap, largest half-family) entries
    (largest first, each into the least loaded group it fits)."""
    if cap is None:
        cap = class_cap(LA, LB)
    units = class_units(LA, LB)
    size = {u: len(unit_entries(LA, LB, u)) for u in units}
    c = max(cap, max(size.values()))
    groups = []
    for u in sorted(units, key=lambda v: (-size[v], v[0], -v[1])):
        best = None
        for gi, g in enumerate(groups):
            load = sum(size[v] for v in g)
            if load + size[u] <= c and (best is None or load < sum(size[v] for v in groups[best])):
                best = gi
        if best is None:
            groups.append([u])
        else:
            groups[best].append(u)
    groups = [sorted(g, key=lambda v: (v[0], -v[1])) for g in groups]
    groups.sort(key=lambda g: -sum(size[v] for v in g))
    return groups


def group_index(LA, LB, group):
    """{(L, M, k): position in the group's W array}."""
    idx = {}
    for u in group:
        for e in unit_entries(LA, LB, u):
            idx[e] = len(idx)
    return idx


def class_terms(LA, LB):
    """Coupling terms (ma, mb, l1, l2, L, M, k, coef) with coef = c_a c_b g."""
    g = real_gaunt_table()
    terms = []
    for ma in range(-LA, LA + 1):
        for mb in range(-LB, LB + 1):
            for l1 in range(abs(ma), LA + 1):
                ca = trans_coef(LA, l1, ma)
                for l2 in range(abs(mb), LB + 1):
                    cb = trans_coef(LB, l2, mb)
                    i1, i2 = l1 * l1 + ma + l1, l2 * l2 + mb + l2
                    for L in range(abs(l1 - l2), l1 + l2 + 1, 2):
                        for M in range(-L, L + 1):
                            v = g[i1, i2, L * L + M + L]
                            if v != 0.0:
                                terms.append((ma, mb, l1, l2, L, M, (l1 + l2 - L) // 2, ca * cb * v))
    return terms


# ----------------------------------------------------------------------------------------------
# numpy execution of the emitted algorithm (used by the CPU tests)
# ----------------------------------------------------------------------------------------------
def boys_np(mmax, T):
    """Boys function by mpmath (test helper for the emulation only)."""
    import mpmath
    mpmath.mp.dps = 30
    out = np.zeros(mmax + 1)
    for m in range(mmax + 1):
        if T == 0:
            out[m] = 1.0 / (2 * m + 1)
        else:
            a = mpmath.mpf(m) + 0.5
            out[m] = float(mpmath.gammainc(a, 0, T) / (2 * mpmath.mpf(T) ** a))
    return out


def frame(R):
    """(cos theta, sin theta, cos phi, sin phi) of the A->B axis, identity frame for R = 0."""
    Rl = float(np.linalg.norm(R))
    rho = float(math.hypot(R[0], R[1]))
    if Rl == 0.0:
        return 1.0, 0.0, 1.0, 0.0, 0.0
    ct, st = R[2] / Rl, rho / Rl
    cp, sp = (R[0] / rho, R[1] / rho) if rho > 0 else (1.0, 0.0)
    return ct, st, cp, sp, Rl


def rotate_into_frame(v, ct, st, cp, sp):
    u = cp * v[0] + sp * v[1]
    return np.array([ct * u - st * v[2], -sp * v[0] + cp * v[1], st * u + ct * v[2]])


def zrot(l, c, s):
    """Z(angle) for S^l given cos/sin of m*angle arrays c[m], s[m]."""
    Zm = np.zeros((2 * l + 1, 2 * l + 1))
    Zm[l, l] = 1.0
    for m in range(1, l + 1):
        Zm[l + m, l + m] = c[m]
        Zm[l + m, l - m] = -s[m]
        Zm[l - m, l + m] = s[m]
        Zm[l - m, l - m] = c[m]
    return Zm


def emulate_block(LA, LB, A, B, ea, wa, eb, wb, nuc_pos, nuc_Z, cap=None, boys=boys_np):
    """The V block (2LA+1) x (2LB+1) of shells (LA at A) x (LB at B), computed by the emitted
    algorithm in numpy. ``wa``/``wb`` are the final primitive weights (contraction x norm)."""
    A, B = np.asarray(A, float), np.asarray(B, float)
    ct, st, cp, sp, Rl = frame(B - A)
    th, ph = math.atan2(st, ct), math.atan2(sp, cp)
    groups = class_groups(LA, LB, cap)
    terms = class_terms(LA, LB)
    NA, NB = 2 * LA + 1, 2 * LB + 1
    Vp = np.zeros((NA, NB))
    LM = LA + LB
    for a_, wa_ in zip(ea, wa):
        for b_, wb_ in zip(eb, wb):
            p = a_ + b_
            P = (a_ * A + b_ * B) / p
            K = math.exp(-a_ * b_ / p * Rl * Rl)
            ta, tb = b_ * Rl / p, -a_ * Rl / p
            W = {}
            for c, Z in zip(nuc_pos, nuc_Z):
                C = rotate_into_frame(np.asarray(c) - P, ct, st, cp, sp)
                T = p * float(C @ C)
                F = boys(LM, T) * Z
                S = solid_real(LM, C[None])[0]
                for L in range(LM + 1):
                    for k in range(kmax_of(LA, LB, L) + 1):
                        G = sum(T ** j / math.factorial(j) * F[L + j] for j in range(k + 1))
                        for M in range(-L, L + 1):
                            W[(L, M, k)] = W.get((L, M, k), 0.0) + G * S[L * L + M + L]
            pre = -wa_ * wb_ * K
            for (ma, mb, l1, l2, L, M, k, coef) in terms:
                fk = pre * 2 * math.pi * math.factorial(k) / p ** (k + 1)
                Vp[ma + LA, mb + LB] += coef * ta ** (LA - l1) * tb ** (LB - l2) * fk * W.get((L, M, k), 0.0)
    # the group partition must cover every coupled W entry exactly once
    seen = {}
    for g in groups:
        for e in group_index(LA, LB, g):
            assert e not in seen
            seen[e] = 1
    for t in terms:
        assert (t[4], t[5], t[6]) in seen
    # rotate back: V = Da^T V' Db, D^T = Z(phi) J^T Z(theta) J
    def dT(l):
        cth = [math.cos(m * th) for m in range(l + 1)]
        sth = [math.sin(m * th) for m in range(l + 1)]
        cph = [math.cos(m * ph) for m in range(l + 1)]
        sph = [math.sin(m * ph) for m in range(l + 1)]
        J = rot_x90(l)
        return zrot(l, cph, sph) @ J.T @ zrot(l, cth, sth) @ J
    Dat, Dbt = dT(LA), dT(LB)
    return Dat @ Vp @ Dbt.T


def emulate_grad(LA, LB, A, B, ea, wa, eb, wb, nuc_pos, nuc_Z, Dt, boys=boys_np):
    """numpy run of the adjoint kernel for one shell pair (LA at A) x (LB at B), LA >= LB:
    E = sum Dt V_block and its gradients (dE/dA, dE/dB, dE/dc [n_nuc, 3]) from the emitted term
    tables, gradient matrices and forward-mode recurrences."""
    A, B = np.asarray(A, float), np.asarray(B, float)
    ct, st, cp, sp, Rl = frame(B - A)
    th, ph = math.atan2(st, ct), math.atan2(sp, cp)
    Qm = np.array([[ct * cp, ct * sp, -st], [-sp, cp, 0.0], [st * cp, st * sp, ct]])  # lab -> frame
    def dmat(l):   # D^l with D^T = Z(phi) J^T Z(theta) J
        cth = [math.cos(m * th) for m in range(l + 1)]
        sth = [math.sin(m * th) for m in range(l + 1)]
        cph = [math.cos(m * ph) for m in range(l + 1)]
        sph = [math.sin(m * ph) for m in range(l + 1)]
        J = rot_x90(l)
        return (zrot(l, cph, sph) @ J.T @ zrot(l, cth, sth) @ J).T
    Dp = dmat(LA) @ np.asarray(Dt, float) @ dmat(LB).T
    blocks = {0: Dp.reshape(-1)}
    if LA >= 1:
        g = grad_matrix(LA)
        blocks[1] = [(g[i].T @ Dp).reshape(-1) for i in range(3)]
    if LB >= 1:
        g = grad_matrix(LB)
        blocks[2] = [(Dp @ g[i]).reshape(-1) for i in range(3)]
    ents = grad_entries(LA, LB)
    tabs = grad_tables(LA, LB)
    LM = LA + LB
    E = 0.0
    dA, dB = np.zeros(3), np.zeros(3)
    dC = np.zeros((len(nuc_Z), 3))
    for a_, wa_ in zip(ea, wa):
        for b_, wb_ in zip(eb, wb):
            p = a_ + b_
            P = (a_ * A + b_ * B) / p
            mu = a_ * b_ / p
            K = math.exp(-mu * Rl * Rl)
            ta, tb = b_ * Rl / p, -a_ * Rl / p
            pre = -wa_ * wb_ * K
            fk = [pre * 2 * math.pi * math.factorial(k) / p ** (k + 1) for k in range(LB + 1)]
            s0 = np.zeros(len(ents))
            sa = np.zeros((3, len(ents)))
            sb = np.zeros((3, len(ents)))
            for kind, e, src, pa, pb, coef in tabs:
                f = coef * ta ** pa * tb ** pb
                if kind == 0:
                    s0[e] += f * blocks[0][src]
                elif kind == 1:
                    for i in range(3):
                        sa[i, e] += f * blocks[1][i][src]
                else:
                    for i in range(3):
                        sb[i, e] += f * blocks[2][i][src]
            scale = np.array([fk[e[2]] * monic_c(e[0], abs(e[1])) for e in ents])
            wbar = scale * s0
            wr = scale * (b_ / p * sa - a_ / p * sb)
            wr[2] += -2.0 * mu * Rl * wbar
            gP = np.zeros(3)
            eR = np.zeros(3)
            for ci, (c, Z) in enumerate(zip(nuc_pos, nuc_Z)):
                C = rotate_into_frame(np.asarray(c) - P, ct, st, cp, sp)
                T = p * float(C @ C)
                F = boys(LM + 1, T)
                S, dS = solid_real_grad(LM, C[None].astype(np.longdouble))
                S, dS = S.astype(float)[0], dS.astype(float)[:, 0]
                gr = np.zeros(3)
                for e, (L, M, k) in enumerate(ents):
                    cl = monic_c(L, abs(M))
                    q, dq = S[L * L + M + L] / cl, dS[:, L * L + M + L] / cl
                    G = sum(T ** j / math.factorial(j) * F[L + j] for j in range(k + 1))
                    Gp = -T ** k / math.factorial(k) * F[L + k + 1]
                    gr += Z * wbar[e] * (G * dq + Gp * q * 2 * p * C)
                    eR += Z * wr[:, e] * G * q
                    E += Z * wbar[e] * G * q
                dC[ci] += Qm.T @ gr
                gP -= gr
            dA += Qm.T @ (a_ / p * gP - eR)
            dB += Qm.T @ (b_ / p * gP + eR)
    return E, dA, dB, dC


# ----------------------------------------------------------------------------------------------
# Emission
# ----------------------------------------------------------------------------------------------
def lit(v):
    return repr(float(v))


def flit(v):
    """A float literal that reads back as exactly the binary32 value v."""
    v = np.float32(v)
    t = "%.9g" % float(v)
    assert np.float32(float(t)) == v
    if "e" not in t and "." not in t:
        t += ".0"
    return t + "f"


def emit_group(LA, LB, gi, group):
    LM = LA + LB
    idx = group_index(LA, LB, group)
    NW = len(idx)
    name = f"G{LA}{LB}_{gi}"
    o = []
    o.append(f"struct {name} {{")
    o.append(f"  static constexpr int NW = {NW};")
    # ---- nucleus step ----
    # Monic recurrences: with Q^mu_mu + i Q^-mu_mu = Z (x + iy)^mu and
    # Q_{L+1} = z Q_L - e_L r^2 Q_{L-1}, the real solid harmonics are S^L_{+-mu} = c_L Q^{+-mu}_L / Z
    # (c_L = prod of the sectoral and vertical recurrence coefficients); c_L is applied in scale().
    o.append("  static __device__ __forceinline__ void step(double (&W)[NW], double x, double y, double z, double r2,")
    o.append(f"                                               double Z, const double (&F)[{LM + 1}], const double (&tj)[{LB + 1}]) {{")
    # sectoral seeds Z (x + iy)^mu of the group's families: powers of two by squaring, the rest as
    # products of those (depth log2 mu instead of a chain of mu complex multiplications)
    needed = sorted(set(mu for (mu, sg) in group if mu > 0))
    if needed:
        o.append("    const double zr1 = x, zi1 = y;")
        k = 2
        while k <= max(needed):
            h = k // 2
            o.append(f"    const double zr{k} = fma(zr{h}, zr{h}, -zi{h} * zi{h}), zi{k} = 2.0 * zr{h} * zi{h};")
            k *= 2
        for mu in needed:
            bits = [1 << b for b in range(mu.bit_length()) if mu >> b & 1]
            ar, ai = f"zr{bits[0]}", f"zi{bits[0]}"
            for j, b in enumerate(bits[1:]):
                o.append(f"    const double pr{mu}_{j} = fma({ar}, zr{b}, -{ai} * zi{b}), "
                         f"pi{mu}_{j} = fma({ar}, zi{b}, {ai} * zr{b});")
                ar, ai = f"pr{mu}_{j}", f"pi{mu}_{j}"
            o.append(f"    const double sc{mu} = Z * {ar}, ss{mu} = Z * {ai};")
    for (mu, sg) in group:
        q = "Z" if mu == 0 else (f"sc{mu}" if sg > 0 else f"ss{mu}")
        o.append(f"    {{ // half-family M = {sg * mu}")
        o.append(f"      double cq = {q}, pq = 0.0;")
        for L in range(mu, LM + 1):
            if L > mu:
                if L - 1 == mu:
                    o.append("      pq = cq; cq = z * cq;")
                else:
                    e = monic_e(L - 1, mu)
                    o.append(f"      {{ const double nq = fma(z, cq, ({lit(-e)} * r2) * pq); pq = cq; cq = nq; }}")
            km = kmax_of(LA, LB, L)
            o.append(f"      {{ double g = F[{L}];")
            for k in range(km + 1):
                if k > 0:
                    o.append(f"        g = fma(tj[{k}], F[{L + k}], g);")
                o.append(f"        W[{idx[(L, sg * mu, k)]}] = fma(g, cq, W[{idx[(L, sg * mu, k)]}]);")
            o.append("      }")
        o.append("    }")
    o.append("  }")
    # ---- scaling by pre * 2 pi k!/p^{k+1} and the harmonic normalisation c_L ----
    # The constants of scale() and couple() are read from the group's table in memory rather than
    # written as literals: thousands of 64-bit literals would be materialised in scalar registers,
    # overflow them and be spilled to vector-register lanes.
    table = []
    slot = {}

    def tab(v):
        v = float(v)
        if v not in slot:
            slot[v] = len(table)
            table.append(v)
        return slot[v]

    o.append(f"  static __device__ __forceinline__ void scale(double (&W)[NW], const double (&fk)[{LB + 1}]) {{")
    o.append(f"    const CTab C = launder_table(kTab{LA}{LB}_{gi});")
    for (L, M, k), i in idx.items():
        o.append(f"    W[{i}] *= fk[{k}] * C[{tab(monic_c(L, abs(M)))}];")
    o.append("  }")
    # ---- coupling ----
    # Outputs are visited in blocks of equal (|ma|, |mb|): inside a block the sign variants
    # (ma, mb) = (+-|ma|, +-|mb|) share their coefficients up to sign, so their terms are
    # interleaved by coefficient magnitude and each materialised constant serves several FMAs.
    terms = [t for t in class_terms(LA, LB) if unit_of(t[5]) in group]
    NB = 2 * LB + 1
    blocks = {}
    for t in terms:
        blocks.setdefault((abs(t[0]), abs(t[1])), []).append(t)
    o.append(f"  static __device__ __forceinline__ void couple(const double (&W)[NW], const double (&ta)[{LA + 1}],")
    o.append(f"                                                 const double (&tb)[{LB + 1}], double* __restrict__ Vp) {{")
    o.append("    // Vp: this lane's entry (0, 0) of the tile accumulator; entries are SHGO_ACC_STRIDE apart")
    o.append(f"    const CTab C = launder_table(kTab{LA}{LB}_{gi});")
    for (aa, ab), ts in sorted(blocks.items()):
        outs = sorted(set((t[0], t[1]) for t in ts))
        name = {mm: f"v{i}" for i, mm in enumerate(outs)}
        o.append(f"    {{ // |ma| = {aa}, |mb| = {ab}")
        o.append("      double " + ", ".join(f"{name[mm]} = 0.0" for mm in outs) + ";")
        for l1 in sorted(set(t[2] for t in ts)):
            t1 = [t for t in ts if t[2] == l1]
            o1 = sorted(set((t[0], t[1]) for t in t1))
            o.append("      { double " + ", ".join(f"u{name[mm][1:]} = 0.0" for mm in o1) + ";")
            for l2 in sorted(set(t[3] for t in t1)):
                t2 = [t for t in t1 if t[3] == l2]
                o2 = sorted(set((t[0], t[1]) for t in t2))
                first = {mm: True for mm in o2}
                lines = []
                for t in sorted(t2, key=lambda t: (abs(t[7]), t[7] < 0, t[0], t[1], t[4], t[5])):
                    mm = (t[0], t[1])
                    e = f"e{name[mm][1:]}"
                    wi = idx[(t[4], t[5], t[6])]
                    c = t[7]
                    cref = f"C[{tab(abs(c))}]" if c > 0 else f"-C[{tab(abs(c))}]"
                    if first[mm]:
                        lines.append(f"double {e} = {cref} * W[{wi}];")
                        first[mm] = False
                    else:
                        lines.append(f"{e} = fma({cref}, W[{wi}], {e});")
                o.append("        { " + " ".join(lines))
                for mm in o2:
                    k = name[mm][1:]
                    if LB - l2 == 0:
                        o.append(f"          u{k} += e{k};")
                    else:
                        o.append(f"          u{k} = fma(tb[{LB - l2}], e{k}, u{k});")
                o.append("        }")
            for mm in o1:
                k = name[mm][1:]
                if LA - l1 == 0:
                    o.append(f"        {name[mm]} += u{k};")
                else:
                    o.append(f"        {name[mm]} = fma(ta[{LA - l1}], u{k}, {name[mm]});")
            o.append("      }")
        for mm in outs:
            o.append(f"      atomicAdd(Vp + {(mm[0] + LA) * NB + (mm[1] + LB)} * SHGO_ACC_STRIDE, {name[mm]});")
        o.append("    }")
    o.append("  }")
    # ---- coupling in binary32 with error-free transformations (mixed precision) ----
    # The same sums as couple(), with W, the shift powers and the coefficients as unevaluated
    # pairs hi + lo of floats (double-float values) and every product and sum done by the
    # error-free transformations of shgo_internal.h (TwoProd by fma, TwoSum); the block entry
    # hi + lo is added to the binary64 accumulator.
    if LA > MIXED_LMAX:
        o.append("};")
        head = [f"// constants of the scale and coupling of group {gi} of class ({LA}, {LB})",
                f"__device__ const double kTab{LA}{LB}_{gi}[{len(table)}] = {{{', '.join(lit(v) for v in table)}}};"]
        return "\n".join(head + o)
    ftable = []
    fslot = {}

    def ftab(v):
        v = float(v)
        if v not in fslot:
            fslot[v] = len(ftable)
            ftable.append(v)
        return fslot[v]

    o.append(f"  static __device__ __forceinline__ void couple_mixed(const double (&W)[NW], const double (&ta)[{LA + 1}],")
    o.append(f"                                                       const double (&tb)[{LB + 1}], double* __restrict__ Vp) {{")
    o.append(f"    const CTabF C = launder_table_f(kTabF{LA}{LB}_{gi});")
    o.append("    df w[NW];")
    o.append("#pragma unroll")
    o.append("    for (int i = 0; i < NW; ++i) w[i] = df_split(W[i]);")
    o.append(f"    df a[{LA + 1}], b[{LB + 1}];")
    o.append("#pragma unroll")
    o.append(f"    for (int i = 0; i <= {LA}; ++i) a[i] = df_split(ta[i]);")
    o.append("#pragma unroll")
    o.append(f"    for (int i = 0; i <= {LB}; ++i) b[i] = df_split(tb[i]);")
    for (aa, ab), ts in sorted(blocks.items()):
        outs = sorted(set((t[0], t[1]) for t in ts))
        name = {mm: f"v{i}" for i, mm in enumerate(outs)}
        o.append(f"    {{ // |ma| = {aa}, |mb| = {ab}")
        o.append("      df " + ", ".join(f"{name[mm]} = df_zero()" for mm in outs) + ";")
        for l1 in sorted(set(t[2] for t in ts)):
            t1 = [t for t in ts if t[2] == l1]
            o1 = sorted(set((t[0], t[1]) for t in t1))
            o.append("      { df " + ", ".join(f"u{name[mm][1:]} = df_zero()" for mm in o1) + ";")
            for l2 in sorted(set(t[3] for t in t1)):
                t2 = [t for t in t1 if t[3] == l2]
                o2 = sorted(set((t[0], t[1]) for t in t2))
                first = {mm: True for mm in o2}
                lines = []
                for t in sorted(t2, key=lambda t: (abs(t[7]), t[7] < 0, t[0], t[1], t[4], t[5])):
                    mm = (t[0], t[1])
                    e = f"e{name[mm][1:]}"
                    wi = idx[(t[4], t[5], t[6])]
                    c = t[7]
                    cref = f"df_coef(C, {ftab(abs(c))}, {'false' if c > 0 else 'true'})"
                    if first[mm]:
                        lines.append(f"df {e} = df_mul({cref}, w[{wi}]);")
                        first[mm] = False
                    else:
                        lines.append(f"{e} = df_fma({cref}, w[{wi}], {e});")
                o.append("        { " + " ".join(lines))
                for mm in o2:
                    k = name[mm][1:]
                    if LB - l2 == 0:
                        o.append(f"          u{k} = df_add(u{k}, e{k});")
                    else:
                        o.append(f"          u{k} = df_fma(b[{LB - l2}], e{k}, u{k});")
                o.append("        }")
            for mm in o1:
                k = name[mm][1:]
                if LA - l1 == 0:
                    o.append(f"        {name[mm]} = df_add({name[mm]}, u{k});")
                else:
                    o.append(f"        {name[mm]} = df_fma(a[{LA - l1}], u{k}, {name[mm]});")
            o.append("      }")
        for mm in outs:
            o.append(f"      atomicAdd(Vp + {(mm[0] + LA) * NB + (mm[1] + LB)} * SHGO_ACC_STRIDE, df_value({name[mm]}));")
        o.append("    }")
    o.append("  }")
    o.append("};")
    fpairs = []
    for v in ftable:
        hi = np.float32(v)
        lo = np.float32(v - float(hi))
        fpairs += [flit(hi), flit(lo)]
    head = [f"// constants of the scale and coupling of group {gi} of class ({LA}, {LB})",
            f"__device__ const double kTab{LA}{LB}_{gi}[{len(table)}] = {{{', '.join(lit(v) for v in table)}}};",
            f"// the coupling coefficients of the same group as float pairs hi, lo (hi + lo = c to 2^-48)",
            f"__device__ const float kTabF{LA}{LB}_{gi}[{len(fpairs)}] = {{{', '.join(fpairs)}}};"]
    return "\n".join(head + o)


def emit_rotation(l):
    """v <- Z(phi) J^T Z(theta) J v for a vector of length 2l+1."""
    J = rot_x90(l)
    n = 2 * l + 1
    o = [f"template <> struct Rot<{l}> {{",
         f"  static __device__ __forceinline__ void apply(double (&v)[{n}], const double* __restrict__ cth, "
         "const double* __restrict__ sth,",
         "                                              const double* __restrict__ cph, const double* __restrict__ sph) {"]
    def matvec(M, src, dst):
        for i in range(n):
            terms = [(M[i, j], j) for j in range(n) if M[i, j] != 0.0]
            if not terms:
                o.append(f"    const double {dst}{i} = 0.0;")
                continue
            e = f"{lit(terms[0][0])} * {src}[{terms[0][1]}]"
            for c, j in terms[1:]:
                e = f"fma({lit(c)}, {src}[{j}], {e})"
            o.append(f"    const double {dst}{i} = {e};")
    o.append(f"    double w[{n}];")
    matvec(J, "v", "a")
    for i in range(n):
        o.append(f"    w[{i}] = a{i};")
    # Z(theta)
    for m in range(1, l + 1):
        o.append(f"    {{ const double c = w[{l + m}], s = w[{l - m}];")
        o.append(f"      w[{l + m}] = cth[{m}] * c - sth[{m}] * s; w[{l - m}] = sth[{m}] * c + cth[{m}] * s; }}")
    matvec(J.T, "w", "b")
    for i in range(n):
        o.append(f"    v[{i}] = b{i};")
    for m in range(1, l + 1):
        o.append(f"    {{ const double c = v[{l + m}], s = v[{l - m}];")
        o.append(f"      v[{l + m}] = cph[{m}] * c - sph[{m}] * s; v[{l - m}] = sph[{m}] * c + cph[{m}] * s; }}")
    o.append("  }")
    o.append("};")
    return "\n".join(o)


def emit_rotation_inv(l):
    """v <- D v = J^T Z(-theta) J Z(-phi) v, the inverse of Rot<l> (laboratory -> pair frame)."""
    J = rot_x90(l)
    n = 2 * l + 1
    o = [f"template <> struct RotInv<{l}> {{",
         f"  static __device__ __forceinline__ void apply(double (&v)[{n}], const double* __restrict__ cth, "
         "const double* __restrict__ sth,",
         "                                              const double* __restrict__ cph, const double* __restrict__ sph) {"]

    def zrot_neg(vec, c, sn):
        for m in range(1, l + 1):
            o.append(f"    {{ const double c = {vec}[{l + m}], s = {vec}[{l - m}];")
            o.append(f"      {vec}[{l + m}] = {c}[{m}] * c + {sn}[{m}] * s; {vec}[{l - m}] = -{sn}[{m}] * c + {c}[{m}] * s; }}")

    def matvec(M, src, dst):
        for i in range(n):
            terms = [(M[i, j], j) for j in range(n) if M[i, j] != 0.0]
            if not terms:
                o.append(f"    const double {dst}{i} = 0.0;")
                continue
            e = f"{lit(terms[0][0])} * {src}[{terms[0][1]}]"
            for c, j in terms[1:]:
                e = f"fma({lit(c)}, {src}[{j}], {e})"
            o.append(f"    const double {dst}{i} = {e};")
    o.append(f"    double w[{n}];")
    zrot_neg("v", "cph", "sph")
    matvec(J, "v", "a")
    for i in range(n):
        o.append(f"    w[{i}] = a{i};")
    zrot_neg("w", "cth", "sth")
    matvec(J.T, "w", "b")
    for i in range(n):
        o.append(f"    v[{i}] = b{i};")
    o.append("  }")
    o.append("};")
    return "\n".join(o)


def grad_entries(LA, LB):
    """Canonical order of all W entries (L, M, k) of a class for the gradient kernel."""
    return list(group_index(LA, LB, class_units(LA, LB)).keys())


def grad_tables(LA, LB):
    """Term tables of the adjoint vectors of class (LA, LB), by entry of grad_entries:
    (kind, entry, src, pa, pb, coef) with kind 0: class (LA, LB) on the rotated density block,
    1: class (LA-1, LB) on the a-side gradient blocks, 2: class (LA, LB-1) on the b-side ones.
    src indexes the row-major block of that kind; pa, pb are the powers of t_a and t_b."""
    ent = {e: i for i, e in enumerate(grad_entries(LA, LB))}
    out = []
    specs = [(0, LA, LB)]
    if LA >= 1:
        specs.append((1, LA - 1, LB))
    if LB >= 1:
        specs.append((2, LA, LB - 1))
    for kind, la, lb in specs:
        nb = 2 * lb + 1
        for (ma, mb, l1, l2, L, M, k, coef) in class_terms(la, lb):
            out.append((kind, ent[(L, M, k)], (ma + la) * nb + (mb + lb), la - l1, lb - l2, coef))
    return out


def emit_grad(LA, LB):
    """Tables and the forward-mode nucleus step of the adjoint (gradient) kernel of class (LA, LB)."""
    LM = LA + LB
    ents = grad_entries(LA, LB)
    NW = len(ents)
    idx = {e: i for i, e in enumerate(ents)}
    o = [f"// ---- gradient, class ({LA}, {LB}) ----"]
    terms = sorted(grad_tables(LA, LB), key=lambda t: (t[1], t[0], t[2]))
    offs = [0] * (NW + 1)
    for t in terms:
        offs[t[1] + 1] += 1
    for i in range(NW):
        offs[i + 1] += offs[i]
    o.append(f"__device__ const int kGradOff{LA}{LB}[{NW + 1}] = {{{', '.join(map(str, offs))}}};")
    o.append(f"__device__ const GradTerm kGradTerm{LA}{LB}[{len(terms)}] = {{")
    for kind, e, src, pa, pb, coef in terms:
        o.append(f"  {{{lit(coef)}, {src}, {kind}, {pa}, {pb}}},")
    o.append("};")
    o.append(f"__device__ const int kGradK{LA}{LB}[{NW}] = {{{', '.join(str(e[2]) for e in ents)}}};")
    o.append(f"__device__ const double kGradC{LA}{LB}[{NW}] = {{{', '.join(lit(monic_c(e[0], abs(e[1]))) for e in ents)}}};")
    o.append(f"template <> struct GradClass<{LA}, {LB}> {{")
    o.append(f"  static constexpr int NW = {NW};")
    o.append(f"  static __device__ const int* off() {{ return kGradOff{LA}{LB}; }}")
    o.append(f"  static __device__ const GradTerm* terms() {{ return kGradTerm{LA}{LB}; }}")
    o.append(f"  static __device__ const int* kk() {{ return kGradK{LA}{LB}; }}")
    o.append(f"  static __device__ const double* cl() {{ return kGradC{LA}{LB}; }}")
    # nucleus step: Q and grad Q by forward-mode recurrences, contracted with the adjoint quadruples
    o.append("  // adj: LDS quadruples (Wbar, WRx, WRy, WRz) per entry; acc: 0-2 sum a grad Q, 3 sum b Q,")
    o.append("  // 4-6 sum (WR . G) Q, 7 sum a Q, with a = Wbar . G and b = Wbar . dG/dT")
    o.append("  static __device__ __forceinline__ void step(const double* __restrict__ adj, double x, double y, double z,")
    o.append(f"                                              double r2, const double (&F)[{LM + 2}], const double (&tj)[{LB + 1}],")
    o.append("                                              double (&acc)[8]) {")
    o.append("    double sc = 1.0, ss = 0.0, scp = 0.0, ssp = 0.0;")
    cur = 0
    for (mu, sg) in class_units(LA, LB):
        while cur < mu:
            o.append("    { const double nc = fma(x, sc, -y * ss), ns = fma(y, sc, x * ss); scp = sc; ssp = ss; sc = nc; ss = ns; }")
            cur += 1
        o.append(f"    {{ // half-family M = {sg * mu}")
        if mu == 0:
            o.append("      double q = 1.0, qx = 0.0, qy = 0.0, qz = 0.0;")
        elif sg > 0:
            o.append(f"      double q = sc, qx = {float(mu)} * scp, qy = {float(-mu)} * ssp, qz = 0.0;")
        else:
            o.append(f"      double q = ss, qx = {float(mu)} * ssp, qy = {float(mu)} * scp, qz = 0.0;")
        o.append("      double pq = 0.0, px = 0.0, py = 0.0, pz = 0.0;")
        for L in range(mu, LM + 1):
            if L > mu:
                if L - 1 == mu:
                    o.append("      { pq = q; px = qx; py = qy; pz = qz; q = z * pq; qx = z * px; qy = z * py; qz = fma(z, pz, pq); }")
                else:
                    e = -monic_e(L - 1, mu)
                    o.append(f"      {{ const double E = {lit(e)};")
                    o.append("        const double nq = fma(z, q, E * r2 * pq);")
                    o.append("        const double nx = fma(z, qx, E * fma(2.0 * x, pq, r2 * px));")
                    o.append("        const double ny = fma(z, qy, E * fma(2.0 * y, pq, r2 * py));")
                    o.append("        const double nz = fma(z, qz, q + E * fma(2.0 * z, pq, r2 * pz));")
                    o.append("        pq = q; px = qx; py = qy; pz = qz; q = nq; qx = nx; qy = ny; qz = nz; }")
            km = kmax_of(LA, LB, L)
            o.append("      { double g = 0.0, a = 0.0, b = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;")
            for k in range(km + 1):
                e = idx[(L, sg * mu, k)]
                if k == 0:
                    o.append(f"        g = F[{L}];")
                else:
                    o.append(f"        g = fma(tj[{k}], F[{L + k}], g);")
                o.append(f"        {{ const double* w = adj + {4 * e}; const double gp = -tj[{k}] * F[{L + k + 1}];")
                o.append("          a = fma(w[0], g, a); b = fma(w[0], gp, b); ex = fma(w[1], g, ex); ey = fma(w[2], g, ey); ez = fma(w[3], g, ez); }")
            o.append("        acc[0] = fma(a, qx, acc[0]); acc[1] = fma(a, qy, acc[1]); acc[2] = fma(a, qz, acc[2]);")
            o.append("        acc[3] = fma(b, q, acc[3]); acc[4] = fma(ex, q, acc[4]); acc[5] = fma(ey, q, acc[5]);")
            o.append("        acc[6] = fma(ez, q, acc[6]); acc[7] = fma(a, q, acc[7]); }")
        o.append("    }")
    o.append("  }")
    o.append("};")
    return "\n".join(o)


# ----------------------------------------------------------------------------------------------
# Cartesian route (McMurchie-Davidson), the comparison path on the same GPU
# ----------------------------------------------------------------------------------------------
CART_LMAX = 4  # shells of the Cartesian route: the product rule reaches L = 8 (165 Hermite integrals)


def cart_monomials(l):
    """Cartesian monomials x^i y^j z^k of degree l, index s(s+1)/2 + k with s = j + k."""
    return [(l - sj, sj - k, k) for sj in range(l + 1) for k in range(sj + 1)]


def tuv_list(L):
    """Hermite indices (t, u, v), t + u + v <= L, index N(N+1)(N+2)/6 + s(s+1)/2 + v with
    N = t + u + v and s = u + v."""
    return [(N - sj, sj - v, v) for N in range(L + 1) for sj in range(N + 1) for v in range(sj + 1)]


def hermite_a(t, i):
    """Coefficient of X^(t-2i) g_(n+t-i) in d^t/dX^t g_n, where d/dX g_n = X g_(n+1):
    t! / (2^i i! (t-2i)!), the number of ways to pair 2i of t derivatives."""
    return math.factorial(t) // (2 ** i * math.factorial(i) * math.factorial(t - 2 * i))


def solid_real_poly(l):
    """Coefficients C[m + l][q] of S^l_m(x, y, z) = sum_q C x^i y^j z^k over cart_monomials(l),
    built with the recurrences of solid_real in exact polynomial arithmetic (float coefficients)."""
    def mul(a, b):
        out = {}
        for ka, va in a.items():
            for kb, vb in b.items():
                k = (ka[0] + kb[0], ka[1] + kb[1], ka[2] + kb[2])
                out[k] = out.get(k, 0.0) + va * vb
        return out

    def add(a, b, fa=1.0, fb=1.0):
        out = {k: fa * v for k, v in a.items()}
        for k, v in b.items():
            out[k] = out.get(k, 0.0) + fb * v
        return out

    X, Y, Zp = {(1, 0, 0): 1.0}, {(0, 1, 0): 1.0}, {(0, 0, 1): 1.0}
    R2 = {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0}
    S = {(0, 0): {(0, 0, 0): 1.0}}
    sc, ss = {(0, 0, 0): 1.0}, {}
    for k in range(l):
        f = 1.0 if k == 0 else math.sqrt((2 * k + 1) / (2 * k + 2))
        sc, ss = add(mul(X, sc), mul(Y, ss), f, -f), add(mul(Y, sc), mul(X, ss), f, f)
        S[(k + 1, k + 1)], S[(k + 1, -(k + 1))] = sc, ss
    for m in range(l + 1):
        for sgn in ([1] if m == 0 else [1, -1]):
            mm = sgn * m
            prev, cur = {}, S[(m, mm)]
            for k in range(m, l):
                den = math.sqrt((k + m + 1) * (k - m + 1))
                a, b = (2 * k + 1) / den, math.sqrt((k + m) * (k - m)) / den
                nxt = add(mul(Zp, cur), mul(R2, prev), a, -b)
                S[(k + 1, mm)] = nxt
                prev, cur = cur, nxt
    mono = cart_monomials(l)
    C = np.zeros((2 * l + 1, len(mono)))
    for m in range(-l, l + 1):
        for q, ijk in enumerate(mono):
            C[m + l, q] = S[(l, m)].get(ijk, 0.0)
    return C


def cart_r_terms(L):
    """[(index, [(coef, a, b, c, n), ...])] of R_tuv = sum coef X^a Y^b Z^c g_n, in tuv_list order."""
    out = []
    for n, (t, u, v) in enumerate(tuv_list(L)):
        N = t + u + v
        terms = [(hermite_a(t, i) * hermite_a(u, j) * hermite_a(v, k), t - 2 * i, u - 2 * j, v - 2 * k, N - i - j - k)
                 for i in range(t // 2 + 1) for j in range(u // 2 + 1) for k in range(v // 2 + 1)]
        out.append((n, terms))
    return out


def emit_cart_r(L):
    """W[idx(t,u,v)] += Z R_tuv for t + u + v <= L, with R_tuv = d^t/dX^t d^u/dY^u d^v/dZ^v g_0,
    g_n = (-2p)^n F_n(p |C|^2) and d/dX g_n = X g_(n+1): the closed form
    R_tuv = sum_(i,j,k) a_ti a_uj a_vk X^(t-2i) Y^(u-2j) Z^(v-2k) g_(t+u+v-i-j-k)."""
    tl = tuv_list(L)
    o = [f"template <> struct CartR<{L}> {{",
         f"  static constexpr int NT = {len(tl)};",
         f"  static __device__ __forceinline__ void step(double (&W)[NT], double X, double Y, double Z, double Zc,",
         f"                                              const double (&g)[{L + 1}]) {{",
         f"    double px[{L + 1}], py[{L + 1}], pz[{L + 1}];",
         "    px[0] = 1.0; py[0] = 1.0; pz[0] = 1.0;",
         "#pragma unroll",
         f"    for (int k = 1; k <= {L}; ++k) {{ px[k] = px[k - 1] * X; py[k] = py[k - 1] * Y; pz[k] = pz[k - 1] * Z; }}"]
    for n, tl_terms in cart_r_terms(L):
        t, u, v = tl[n]
        terms = []
        for c, a, b, cc, gn in tl_terms:
            mono = [f"p{ax}[{e}]" for ax, e in (("x", a), ("y", b), ("z", cc)) if e]
            if c != 1:
                mono.append(f"{float(c)!r}")
            terms.append((" * ".join(mono) if mono else None, gn))
        expr = None
        for m, gn in terms:
            if expr is None:
                expr = f"g[{gn}]" if m is None else f"{m} * g[{gn}]"
            else:
                expr = f"fma({m}, g[{gn}], {expr})" if m is not None else f"g[{gn}] + {expr}"
        o.append(f"    W[{n}] = fma(Zc, {expr}, W[{n}]);  // R_{t}{u}{v}")
    o.append("  }")
    o.append("};")
    return "\n".join(o)


def emit_cart_header(lmax=CART_LMAX):
    out = ["// Generated by gen_classes.py -- do not edit. The Cartesian (McMurchie-Davidson) route:",
           "// Hermite Coulomb integrals R_tuv summed over nuclei, and the Cartesian-to-real-harmonic",
           "// coefficients of each l.",
           "#pragma once",
           f"constexpr int kCartLmax = {lmax};",
           "template <int L> struct CartR;"]
    for L in range(2 * lmax + 1):
        out.append(emit_cart_r(L))
    for l in range(lmax + 1):
        C = solid_real_poly(l)
        out.append(f"// S^{l}_m = sum_q kCartSph{l}[m + {l}][q] x^i y^j z^k over the degree-{l} monomials")
        rows = ["{" + ", ".join(lit(v) for v in row) + "}" for row in C]
        out.append(f"__device__ const double kCartSph{l}[{2 * l + 1}][{C.shape[1]}] = {{{', '.join(rows)}}};")
    return "\n".join(out) + "\n"


# ----------------------------------------------------------------------------------------------
# Two-electron integrals (ab|cd) by the solid-harmonic route
# ----------------------------------------------------------------------------------------------
# Each pair (a, b) is worked as in the nuclear-attraction kernel: the Gaussian product, the shifts
# to P in the pair frame (Eq. 7) and the product rule (Supplement Eq. 4) give its charge
# distribution as sum_{L,M,k} B(L,M,k) |u|^{2k} S^L_M(u) e^{-p u^2}, u = r - P, rotated to the
# laboratory frame. With S^L(u) e^{-p u^2} = (2p)^{-L} S^L(grad_P) e^{-p u^2} (Hobson's theorem) and
# |u|^{2k} S^L(u) e^{-p u^2} = (2p)^{-L} sum_j c_{L,k,j}(p) (grad_P^2)^j S^L(grad_P) e^{-p u^2}, the
# two-center integral of two such terms is a derivative of the s-s-s-s integral
# c F_0(alpha R^2), c = 2 pi^{5/2} / (p q sqrt(p+q)), alpha = pq/(p+q), R = P - Q:
#   (-1)^{L2} (grad_R^2)^{j1+j2} S^{L1}(grad_R) S^{L2}(grad_R) c F_0 =
#   (-1)^{L2} sum_{L,M} g(L1 M1, L2 M2; L M) S^L_M(R) h_{L, j1+j2+kappa}(R^2),  kappa = (L1+L2-L)/2,
# with the product rule applied to the gradients, h_{L,0} = c (-2 alpha)^L F_L(alpha R^2) (Hobson's
# theorem again) and h_{L,n+1} = 4 rho h'' + (4L+6) h' (the Laplacian of S^L(R) h(R^2), rho = R^2),
# which for n >= 1 is c (-2 alpha)^L alpha^n P_{L,n}(T) e^{-T}, T = alpha rho.
ERI_LMAX = 2  # shells of the two-electron path (pair distributions up to L = 4, L1 + L2 <= 8)


def _poly_Q(L, jmax, p):
    """Q_{L,j}(rho) (ascending coefficients, Fractions) with (grad^2)^j [S^L(u) e^{-p u^2}] =
    S^L(u) Q_{L,j}(u^2) e^{-p u^2}: Q_0 = 1, Q_{j+1} = 4 rho (Q'' - 2p Q' + p^2 Q) + (4L+6)(Q' - p Q)."""
    from fractions import Fraction as Fr

    def der(q):
        return [i * q[i] for i in range(1, len(q))] or [Fr(0)]

    def add(*qs):
        n = max(len(q) for q in qs)
        return [sum((q[i] if i < len(q) else Fr(0)) for q in qs) for i in range(n)]

    def scale(q, c):
        return [c * v for v in q]

    Qs = [[Fr(1)]]
    for _ in range(jmax):
        Q = Qs[-1]
        d1, d2 = der(Q), der(der(Q))
        inner = add(d2, scale(d1, -2 * p), scale(Q, p * p))
        Qs.append(add([Fr(0)] + scale(inner, 4), scale(add(d1, scale(Q, -p)), 4 * L + 6)))
    return Qs


def eri_gamma(L, kmax):
    """gamma[k][j] with c_{L,k,j}(p) = gamma p^{-(k+j)}: rho^k = sum_j c_{L,k,j} Q_{L,j}(rho)."""
    from fractions import Fraction as Fr
    n = kmax + 1
    out = np.zeros((n, n))
    for pv in (Fr(1), Fr(3, 2)):
        Qs = _poly_Q(L, kmax, pv)
        # solve the triangular system exactly: Q_j has degree j and leading coefficient (4p^2)^j
        c = [[Fr(0)] * n for _ in range(n)]
        for k in range(n):
            rem = [Fr(0)] * (k + 1)
            rem[k] = Fr(1)
            for j in range(k, -1, -1):
                coef = rem[j] / Qs[j][j]
                c[k][j] = coef
                for i in range(j + 1):
                    rem[i] -= coef * Qs[j][i]
        if pv == 1:
            out = np.array([[float(c[k][j]) for j in range(n)] for k in range(n)])
        else:  # the p^{-(k+j)} scaling the kernel relies on
            for k in range(n):
                for j in range(k + 1):
                    assert c[k][j] == Fr(out[k][j]).limit_denominator(10 ** 12) * pv ** (-(k + j)) or \
                        abs(float(c[k][j]) - out[k][j] * float(pv) ** (-(k + j))) <= 1e-15 * abs(out[k][j]) + 1e-300
    return out


def eri_P(L, n):
    """Integer coefficients of P_{L,n}(T), n >= 1: P_1 = -2, P_{n+1} = 4T(P'' - 2P' + P) + (4L+6)(P' - P)."""
    P = [-2]
    for _ in range(n - 1):
        d1 = [i * P[i] for i in range(1, len(P))] or [0]
        d2 = [i * d1[i] for i in range(1, len(d1))] or [0]
        m = max(len(P), len(d1), len(d2))
        at = lambda q, i: q[i] if i < len(q) else 0  # noqa: E731
        inner = [at(d2, i) - 2 * at(d1, i) + at(P, i) for i in range(m)]
        nxt = [0] * (m + 1)
        for i in range(m):
            nxt[i + 1] += 4 * inner[i]
            nxt[i] += (4 * L + 6) * (at(d1, i) - at(P, i))
        while len(nxt) > 1 and nxt[-1] == 0:
            nxt.pop()
        P = nxt
    return P


def eri_class_tables(LA, LB):
    """(entries [(L, M, k)], terms by entry [[(coef, e, pa, pb)]], rotation blocks [(L, k, [w by M])],
    (L, M) groups [(L, [w by k])]) of pair class (LA, LB), LA >= LB."""
    ents = grad_entries(LA, LB)
    idx = {e: i for i, e in enumerate(ents)}
    NB = 2 * LB + 1
    terms = [[] for _ in ents]
    for (ma, mb, l1, l2, L, M, k, coef) in class_terms(LA, LB):
        terms[idx[(L, M, k)]].append((coef, (ma + LA) * NB + (mb + LB), LA - l1, LB - l2))
    blocks = sorted(set((L, k) for (L, M, k) in ents))
    blk = [(L, k, [idx[(L, M, k)] for M in range(-L, L + 1)]) for (L, k) in blocks]
    lm = sorted(set((L, M) for (L, M, k) in ents))
    grp = [(L, [idx[(L, M, k)] for k in range(kmax_of(LA, LB, L) + 1)]) for (L, M) in lm]
    return ents, terms, blk, grp


def emit_eri_header(lmax=ERI_LMAX):
    classes = [(LA, LB) for LA in range(lmax + 1) for LB in range(LA + 1)]
    out = ["// Generated by gen_classes.py -- do not edit. Tables of the two-electron kernel: the pair",
           "// classes' coupling terms, rotation blocks and (L, M) groups, the real Gaunt coefficients of",
           "// the two-center products, and the coefficients of the Laplacian expansions.",
           "#pragma once",
           f"constexpr int kEriLmax = {lmax};",
           f"constexpr int kEriPairClasses = {len(classes)};",
           "struct EriTerm { double coef; int e, pa, pb; };",
           "struct EriGaunt { double g; int I, h; };  // coefficient, (L, M) index, h-table offset"]
    ent_base, term_off, terms_all, ents_all = [], [0], [], []
    blk_base, blk_all, grp_base, grp_all = [], [], [], []
    nw = []
    for (LA, LB) in classes:
        ents, terms, blk, grp = eri_class_tables(LA, LB)
        ent_base.append(len(ents_all))
        nw.append(len(ents))
        for e, ts in zip(ents, terms):
            ents_all.append(e)
            terms_all += ts
            term_off.append(len(terms_all))
        blk_base.append(len(blk_all))
        blk_all += blk
        grp_base.append(len(grp_all))
        grp_all += grp
    blk_base.append(len(blk_all))
    grp_base.append(len(grp_all))
    out.append(f"__device__ const int kEriNW[{len(nw)}] = {{{', '.join(map(str, nw))}}};")
    out.append(f"constexpr int kEriNWHost[{len(nw)}] = {{{', '.join(map(str, nw))}}};  // the same, for the host")
    out.append(f"constexpr int kEriNwMax = {max(nw)};")
    out.append(f"__device__ const int kEriEntBase[{len(ent_base)}] = {{{', '.join(map(str, ent_base))}}};")
    out.append(f"__device__ const int kEriEnt[{len(ents_all)}][3] = {{"
               + ", ".join(f"{{{L}, {M}, {k}}}" for (L, M, k) in ents_all) + "};")
    out.append(f"__device__ const int kEriTermOff[{len(term_off)}] = {{{', '.join(map(str, term_off))}}};")
    out.append(f"__device__ const EriTerm kEriTerm[{len(terms_all)}] = {{"
               + ", ".join(f"{{{lit(c)}, {e}, {pa}, {pb}}}" for (c, e, pa, pb) in terms_all) + "};")
    # rotation blocks: (L, k, first index into kEriBlkW); W indices by M = -L..L
    bw, bhead = [], []
    for (L, k, ws) in blk_all:
        bhead.append((L, k, len(bw)))
        bw += ws
    out.append(f"__device__ const int kEriBlkBase[{len(blk_base)}] = {{{', '.join(map(str, blk_base))}}};")
    out.append(f"__device__ const int kEriBlk[{len(bhead)}][3] = {{" + ", ".join(f"{{{a}, {b}, {c}}}" for a, b, c in bhead) + "};")
    out.append(f"__device__ const int kEriBlkW[{len(bw)}] = {{{', '.join(map(str, bw))}}};")
    gw, ghead = [], []
    for (L, ws) in grp_all:
        ghead.append((L, len(ws), len(gw)))
        gw += ws
    out.append(f"__device__ const int kEriGrpBase[{len(grp_base)}] = {{{', '.join(map(str, grp_base))}}};")
    out.append(f"__device__ const int kEriGrp[{len(ghead)}][3] = {{" + ", ".join(f"{{{a}, {b}, {c}}}" for a, b, c in ghead) + "};")
    out.append(f"__device__ const int kEriGrpW[{len(gw)}] = {{{', '.join(map(str, gw))}}};")
    # real Gaunt lists of the two-center products, L1, L2 <= 2 lmax
    G = real_gaunt_table()
    L12 = 2 * lmax
    n12 = (L12 + 1) ** 2
    goff, gl = [0], []
    hstride = 2 * lmax + L12 + 1  # orders n = 0..kEriNmax of the h table
    for i1 in range(n12):
        for i2 in range(n12):
            L1, L2 = math.isqrt(i1), math.isqrt(i2)
            for I in range(G.shape[2]):
                v = G[i1, i2, I]
                if abs(v) > KEEP:
                    L = math.isqrt(I)
                    gl.append((v, I, L * hstride + (L1 + L2 - L) // 2))
            goff.append(len(gl))
    out.append(f"constexpr int kEriL12 = {L12};")
    out.append(f"__device__ const int kEriGOff[{len(goff)}] = {{{', '.join(map(str, goff))}}};")
    gmax = max(b - a for a, b in zip(goff, goff[1:]))
    out.append(f"constexpr int kEriGmax = {gmax};  // longest list; kEriG ends with that many zero terms")
    out.append(f"constexpr int kEriGTerms = {len(gl)};")
    gl_pad = gl + [(0.0, 0, 0)] * gmax
    out.append(f"__device__ const EriGaunt kEriG[{len(gl_pad)}] = {{"
               + ", ".join(f"{{{lit(v)}, {I}, {h}}}" for v, I, h in gl_pad) + "};")
    kmax = lmax
    gam = np.zeros((L12 + 1, kmax + 1, kmax + 1))
    for L in range(L12 + 1):
        gam[L] = eri_gamma(L, kmax)
    out.append(f"__device__ const double kEriGamma[{L12 + 1}][{kmax + 1}][{kmax + 1}] = {{"
               + ", ".join("{" + ", ".join("{" + ", ".join(lit(v) for v in row) + "}" for row in gm) + "}" for gm in gam)
               + "};")
    LT = 2 * L12
    nmax = 2 * kmax + L12
    Pt = np.zeros((LT + 1, nmax + 1, nmax + 1))
    for L in range(LT + 1):
        for n in range(1, nmax + 1):
            for i, v in enumerate(eri_P(L, n)):
                Pt[L, n, i] = float(v)
    out.append(f"constexpr int kEriLT = {LT};")
    out.append(f"constexpr int kEriNmax = {nmax};")
    out.append(f"__device__ const double kEriP[{LT + 1}][{nmax + 1}][{nmax + 1}] = {{"
               + ", ".join("{" + ", ".join("{" + ", ".join(lit(v) for v in row) + "}" for row in pl) + "}" for pl in Pt)
               + "};")
    return "\n".join(out) + "\n"


def emulate_eri_prim(la, A, a, lb, B, b, lc, C, c, ld, D, d, boys=boys_np):
    """Unnormalised primitive (ab|cd) block (2la+1, 2lb+1, 2lc+1, 2ld+1) by the tables and steps the
    two-electron kernel runs, in numpy."""
    def side(l1, X1, e1, l2, X2, e2):
        swap = l1 < l2
        if swap:
            l1, X1, e1, l2, X2, e2 = l2, X2, e2, l1, X1, e1
        X1, X2 = np.asarray(X1, float), np.asarray(X2, float)
        ents, terms, blk, grp = eri_class_tables(l1, l2)
        ct, st, cp, sp, Rl = frame(X2 - X1)
        th, ph = math.atan2(st, ct), math.atan2(sp, cp)
        p = e1 + e2
        P = (e1 * X1 + e2 * X2) / p
        K = math.exp(-e1 * e2 / p * Rl * Rl)
        ta, tb = e2 * Rl / p, -e1 * Rl / p
        NA, NB = 2 * l1 + 1, 2 * l2 + 1
        Bx = np.zeros((NA * NB, len(ents)))
        for w, ts in enumerate(terms):
            for (coef, e, pa, pb) in ts:
                Bx[e, w] += coef * ta ** pa * tb ** pb

        def dT(l):
            c1 = [math.cos(m * th) for m in range(l + 1)]
            s1 = [math.sin(m * th) for m in range(l + 1)]
            c2 = [math.cos(m * ph) for m in range(l + 1)]
            s2 = [math.sin(m * ph) for m in range(l + 1)]
            J = rot_x90(l)
            return zrot(l, c2, s2) @ J.T @ zrot(l, c1, s1) @ J
        for (L, k, ws) in blk:
            Bx[:, ws] = Bx[:, ws] @ dT(L).T
        Bx = np.einsum("im,jn,mnw->ijw", dT(l1), dT(l2), Bx.reshape(NA, NB, -1)).reshape(NA * NB, -1)
        kmax = max(k for (L, M, k) in ents)
        for (L, ws) in grp:
            gm = eri_gamma(L, kmax)
            v = Bx[:, ws].copy()
            for j in range(len(ws)):
                Bx[:, ws[j]] = (2 * p) ** (-L) * sum(gm[k][j] * p ** (-(k + j)) * v[:, k] for k in range(j, len(ws)))
        if swap:
            Bx = Bx.reshape(NA, NB, -1).transpose(1, 0, 2).reshape(NA * NB, -1)
        return Bx, ents, p, P, K
    Bb, eb, p, P, Kab = side(la, A, a, lb, B, b)
    Bk, ek, q, Q, Kcd = side(lc, C, c, ld, D, d)
    alpha = p * q / (p + q)
    R = P - Q
    T = alpha * float(R @ R)
    cpre = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q))
    LT = la + lb + lc + ld
    F = boys(LT, T)
    S = solid_real(LT, R[None])[0]
    G = real_gaunt_table()
    def h(L, n):
        base = cpre * (-2 * alpha) ** L
        if n == 0:
            return base * F[L]
        return base * alpha ** n * float(np.polyval(np.array(eri_P(L, n), float)[::-1], T)) * math.exp(-T)
    I = np.zeros((len(eb), len(ek)))
    for i1, (L1, M1, j1) in enumerate(eb):
        for i2, (L2, M2, j2) in enumerate(ek):
            s = 0.0
            for L in range(abs(L1 - L2), L1 + L2 + 1, 2):
                kap = (L1 + L2 - L) // 2
                for M in range(-L, L + 1):
                    gv = G[L1 * L1 + M1 + L1, L2 * L2 + M2 + L2, L * L + M + L]
                    if gv != 0.0:
                        s += gv * S[L * L + M + L] * h(L, j1 + j2 + kap)
            I[i1, i2] = (-1) ** L2 * s
    out = Bb @ I @ Bk.T * Kab * Kcd
    return out.reshape(2 * la + 1, 2 * lb + 1, 2 * lc + 1, 2 * ld + 1)


def emit_grad_header(lmax=LMAX_SHELL):
    out = ["// gradient kernel: inverse rotations, gradient matrices of the real solid harmonics, and per class",
           "// the adjoint term tables and the forward-mode nucleus step",
           "struct GradTerm {",
           "  double coef;",
           "  int16_t src;",
           "  int8_t kind, pa, pb;",
           "};",
           "template <int LA, int LB> struct GradClass;"]
    for l in range(1, lmax + 1):
        g = grad_matrix(l)
        vals = ", ".join(lit(v) for v in g.reshape(-1))
        out.append(f"// d/d(x,y,z) S^{l}_m = sum_m' g[xi][m+{l}][m'+{l - 1}] S^{l - 1}_m'")
        out.append(f"__device__ const double kGradMat{l}[{g.size}] = {{{vals}}};")
    out.append("__device__ __forceinline__ const double* grad_matrix(int l) {")
    out.append("  switch (l) {")
    for l in range(1, lmax + 1):
        out.append(f"    case {l}: return kGradMat{l};")
    out.append("  }")
    out.append("  return nullptr;")
    out.append("}")
    for LA in range(lmax + 1):
        for LB in range(LA + 1):
            out.append(emit_grad(LA, LB))
    return "\n".join(out) + "\n"


def emit_rotations(lmax=LMAX_SHELL):
    out = ["// Generated by gen_classes.py -- do not edit. Rotation of a real solid-harmonic vector from the",
           "// pair frame (z along A->B) back to the laboratory frame, D^l(Q)^T = Z(phi) J^T Z(theta) J, and",
           "// its inverse D^l(Q) (laboratory -> pair frame).",
           "#pragma once",
           "",
           "template <int L> struct Rot;",
           "template <int L> struct RotInv;"]
    for l in range(lmax + 1):
        out.append(emit_rotation(l))
    for l in range(lmax + 1):
        out.append(emit_rotation_inv(l))
    return "\n".join(out) + "\n"


def emit_meta(cap=None, lmax=LMAX_SHELL):
    """Host- and device-visible class constants: the wavefront groups of every class."""
    qs = [len(class_groups(LA, LB, cap)) for LA in range(lmax + 1) for LB in range(LA + 1)]
    out = ["// Generated by gen_classes.py -- do not edit. Wavefront groups of each (la, lb) class of the",
           "// integral kernel, indexed by la(la+1)/2 + lb.",
           "#pragma once",
           f"constexpr int kClassGroups[{len(qs)}] = {{{', '.join(map(str, qs))}}};",
           "// classes with la up to this have the mixed-precision (double-float) coupling",
           f"constexpr int kMixedLmax = {MIXED_LMAX};"]
    return "\n".join(out) + "\n"


def emit_header(cap=None, lmax=LMAX_SHELL):
    out = ["// Generated by gen_classes.py -- do not edit. Class-specific code of the nuclear-attraction",
           "// kernel: nucleus step and coupling (product rule + shift along the A->B axis) per group.",
           f"// Group register budget: {cap if cap is not None else 'per class (class_cap)'} doubles.",
           "#pragma once",
           "",
           "// A group's constant table, read through the scalar data cache. The address passes through an",
           "// empty asm statement at every use, so that the loads stay at the use instead of being hoisted",
           "// out of the primitive-pair loop into scalar registers.",
           "typedef const __attribute__((address_space(4))) double* CTab;",
           "typedef const __attribute__((address_space(4))) float* CTabF;",
           "static __device__ __forceinline__ uint64_t launder_address(const void* p) {",
           "  const uint64_t v = (uint64_t)p;",
           "  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));",
           "  asm volatile(\"\" : \"+s\"(lo), \"+s\"(hi));",
           "  return ((uint64_t)hi << 32) | lo;",
           "}",
           "static __device__ __forceinline__ CTab launder_table(const double* p) { return (CTab)launder_address(p); }",
           "static __device__ __forceinline__ CTabF launder_table_f(const float* p) { return (CTabF)launder_address(p); }",
           "// coefficient k of a float-pair table, negated when neg",
           "static __device__ __forceinline__ df df_coef(CTabF C, int k, bool neg) {",
           "  const float h = C[2 * k], l = C[2 * k + 1];",
           "  return neg ? df{-h, -l} : df{h, l};",
           "}",
           "template <int LA, int LB> struct ClassInfo;",
           "template <int LA, int LB, int G> struct GroupOf;"]
    for LA in range(lmax + 1):
        for LB in range(LA + 1):
            groups = class_groups(LA, LB, cap)
            for gi, g in enumerate(groups):
                out.append(emit_group(LA, LB, gi, g))
            nwmax = max(len(group_index(LA, LB, g)) for g in groups)
            out.append(f"template <> struct ClassInfo<{LA}, {LB}> {{ static constexpr int Q = {len(groups)}; "
                       f"static constexpr int NWMAX = {nwmax}; }};")
            for gi, g in enumerate(groups):
                out.append(f"template <> struct GroupOf<{LA}, {LB}, {gi}> : G{LA}{LB}_{gi} {{}};")
    return "\n".join(out) + "\n"


def _write(path, text):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(text)
    os.replace(tmp, path)


def main(argv):
    """Writes shgo_classes.inc (the path given, default generated/shgo_classes.inc) and, beside it,
    shgo_rot.inc, shgo_meta.inc, shgo_grad.inc, shgo_cart.inc and shgo_eri.inc."""
    out = argv[1] if len(argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "generated",
                                                     "shgo_classes.inc")
    cap = None
    if "--cap" in argv:
        cap = int(argv[argv.index("--cap") + 1])
    d = os.path.dirname(out)
    os.makedirs(d, exist_ok=True)
    _write(out, emit_header(cap))
    _write(os.path.join(d, "shgo_rot.inc"), emit_rotations())
    _write(os.path.join(d, "shgo_meta.inc"), emit_meta(cap))
    _write(os.path.join(d, "shgo_grad.inc"), emit_grad_header())
    _write(os.path.join(d, "shgo_cart.inc"), emit_cart_header())
    _write(os.path.join(d, "shgo_eri.inc"), emit_eri_header())
    return out


if __name__ == "__main__":
    print(main(sys.argv))
