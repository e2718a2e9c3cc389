"""Independent cross-check routes that pin the oracle (test infrastructure).

None of this code uses the vector-coupling route, the Clebsch-Gordan or eps coefficients, the
oracle's Boys function or its solid-harmonic polynomial. It provides:

* ``real_solid_poly(l)``: real solid harmonics (order m = -l..l) as homogeneous Cartesian
  polynomials, obtained by least-squares fitting of scipy's Condon-Shortley spherical harmonics
  (Eq. 2 of the paper: Y^l_m = sqrt(4 pi/(2l+1)) r^l Y_lm, then the usual real combination).
* ``boys_mp(n, T)``: Boys function from mpmath's incomplete gamma function.
* ``md_nuclear(...)``: Cartesian McMurchie-Davidson (1978) nuclear-attraction integrals
  (Hermite expansion coefficients E, Hermite Coulomb integrals R) for a primitive pair, then
  the Cartesian -> real solid harmonic transform.
* ``quad_nuclear(...)``: the same integrals by a Gaussian transform of 1/|r - c|,
  1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt, analytic Gaussian moments for fixed t and
  adaptive 1-D quadrature over t.
* ``cart_overlap(...)``: overlap of two polynomial Gaussians from Gaussian moments.
"""
import functools
import math

import mpmath
import numpy as np
from scipy import integrate, special


# ----------------------------------------------------------------------------------------------
# Real solid harmonics as Cartesian polynomials
# ----------------------------------------------------------------------------------------------
def monomials(l):
    """Exponent triples (i, j, k) with i + j + k = l."""
    return [(i, j, l - i - j) for i in range(l, -1, -1) for j in range(l - i, -1, -1)]


def _sph_y(l, m, theta, phi):
    # complex spherical harmonic with Condon-Shortley phase; theta polar, phi azimuth
    if hasattr(special, "sph_harm_y"):
        return special.sph_harm_y(l, m, theta, phi)
    return special.sph_harm(m, l, phi, theta)


@functools.lru_cache(maxsize=None)
def real_solid_poly(l):
    """Coefficient matrix C[(m+l), monomial] with S^l_m(x,y,z) = sum_k C[m+l, k] x^i y^j z^k."""
    mons = monomials(l)
    rng = np.random.default_rng(12345 + l)
    npts = 6 * len(mons) + 20
    v = rng.normal(size=(npts, 3))
    r = np.linalg.norm(v, axis=1)
    theta = np.arccos(v[:, 2] / r)
    phi = np.arctan2(v[:, 1], v[:, 0])
    A = np.stack([v[:, 0] ** i * v[:, 1] ** j * v[:, 2] ** k for (i, j, k) in mons], axis=1)
    C = np.zeros((2 * l + 1, len(mons)))
    pref = math.sqrt(4 * math.pi / (2 * l + 1)) * r ** l
    for m in range(-l, l + 1):
        am = abs(m)
        yp = pref * _sph_y(l, am, theta, phi)       # Y^l_{|m|}
        yn = pref * _sph_y(l, -am, theta, phi)      # Y^l_{-|m|}
        if m == 0:
            s = yp.real
        elif m > 0:
            s = (((-1) ** am) * yp + yn).real / math.sqrt(2)
        else:
            s = (1j * (yn - ((-1) ** am) * yp)).real / math.sqrt(2)
        coef, *_ = np.linalg.lstsq(A, s, rcond=None)
        coef[np.abs(coef) < 1e-12] = 0.0
        C[m + l] = coef
    return C


def eval_real_solid(l, x, y, z):
    C = real_solid_poly(l)
    vals = np.array([x ** i * y ** j * z ** k for (i, j, k) in monomials(l)])
    return C @ vals


# ----------------------------------------------------------------------------------------------
# Boys function from mpmath's incomplete gamma function
# ----------------------------------------------------------------------------------------------
@functools.lru_cache(maxsize=200000)
def _boys_mp_cached(n, T):
    mpmath.mp.dps = 40
    if T == 0:
        return mpmath.mpf(1) / (2 * n + 1)
    Tm = mpmath.mpf(T)
    a = mpmath.mpf(n) + mpmath.mpf(1) / 2
    return mpmath.gammainc(a, 0, Tm) / (2 * Tm ** a)


def boys_mp(n, T):
    return float(_boys_mp_cached(int(n), float(T)))


# ----------------------------------------------------------------------------------------------
# Normalisation of a primitive (closed form; pinned separately by cart_overlap)
# ----------------------------------------------------------------------------------------------
def prim_norm(l, a):
    df = 1.0
    for i in range(2 * l - 1, 1, -2):
        df *= i
    return math.sqrt(2 ** l * (2 * a) ** (l + 1.5) / (df * math.pi ** 1.5))


def contracted_weights(l, expo, coef):
    """Weights w_k with chi = sum_k w_k S^l_m(r - A) exp(-a_k |r-A|^2) at unit self-overlap,
    computed from the polynomial overlap (no closed form for the contracted norm)."""
    expo = np.asarray(expo, float)
    coef = np.asarray(coef, float)
    N = np.array([prim_norm(l, a) for a in expo])
    w = coef * N
    C = real_solid_poly(l)
    ss = 0.0
    for i in range(len(expo)):
        for j in range(len(expo)):
            # <S^l_0 e^{-a_i r^2} | S^l_0 e^{-a_j r^2}>
            ss += w[i] * w[j] * cart_overlap_poly(C[l], l, np.zeros(3), expo[i], C[l], l, np.zeros(3), expo[j])
    return w / math.sqrt(ss)


# ----------------------------------------------------------------------------------------------
# Gaussian moments and polynomial overlaps
# ----------------------------------------------------------------------------------------------
def _moment(n, q):
    """int_{-inf}^{inf} y^n exp(-q y^2) dy."""
    if n % 2:
        return 0.0
    return math.gamma((n + 1) / 2) / q ** ((n + 1) / 2)


def _poly1d_shift(i, s):
    """Coefficients of (y + s)^i in powers of y."""
    return np.array([math.comb(i, a) * s ** (i - a) for a in range(i + 1)])


def _pair_1d(i, j, sa, sb, q):
    """int (y + sa)^i (y + sb)^j exp(-q y^2) dy."""
    pa = _poly1d_shift(i, sa)
    pb = _poly1d_shift(j, sb)
    prod = np.convolve(pa, pb)
    return sum(prod[n] * _moment(n, q) for n in range(len(prod)))


def cart_overlap_poly(ca, la, A, a, cb, lb, B, b, extra=None):
    """int P_a(r - A) P_b(r - B) exp(-a|r-A|^2 - b|r-B|^2 [- t2 |r - c|^2]) d^3r.

    ``ca``/``cb`` are coefficient vectors over monomials(la)/monomials(lb); ``extra`` = (t2, c)."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    if extra is None:
        q = a + b
        Q = (a * A + b * B) / q
        pref = math.exp(-a * b / q * float(np.dot(A - B, A - B)))
    else:
        t2, c = extra
        c = np.asarray(c, float)
        q = a + b + t2
        Q = (a * A + b * B + t2 * c) / q
        pref = math.exp(-(a * b * np.dot(A - B, A - B) + a * t2 * np.dot(A - c, A - c)
                          + b * t2 * np.dot(B - c, B - c)) / q)
    ma, mb = monomials(la), monomials(lb)
    sa = Q - A
    sb = Q - B
    tot = 0.0
    for u, (i1, j1, k1) in enumerate(ma):
        if ca[u] == 0.0:
            continue
        for v, (i2, j2, k2) in enumerate(mb):
            if cb[v] == 0.0:
                continue
            tot += ca[u] * cb[v] * (_pair_1d(i1, i2, sa[0], sb[0], q) * _pair_1d(j1, j2, sa[1], sb[1], q)
                                    * _pair_1d(k1, k2, sa[2], sb[2], q))
    return pref * tot


# ----------------------------------------------------------------------------------------------
# Quadrature route
# ----------------------------------------------------------------------------------------------
def quad_nuclear_prim(la, A, a, lb, B, b, c):
    """Real (2la+1) x (2lb+1) block of int S_a(r-A) e^{-a..} S_b(r-B) e^{-b..} / |r - c|
    (unnormalised primitives) by quadrature over the Gaussian-transform variable t."""
    Ca, Cb = real_solid_poly(la), real_solid_poly(lb)
    out = np.zeros((2 * la + 1, 2 * lb + 1))
    for i in range(2 * la + 1):
        for j in range(2 * lb + 1):
            f = lambda t: cart_overlap_poly(Ca[i], la, A, a, Cb[j], lb, B, b, extra=(t * t, c))
            # split [0, inf) for robustness; the integrand decays like t^-3
            v1, _ = integrate.quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13, limit=200)
            v2, _ = integrate.quad(f, 1.0, np.inf, epsabs=1e-15, epsrel=1e-13, limit=200)
            out[i, j] = 2.0 / math.sqrt(math.pi) * (v1 + v2)
    return out


# ----------------------------------------------------------------------------------------------
# McMurchie-Davidson route
# ----------------------------------------------------------------------------------------------
def _hermite_E(i, j, Xpa, Xpb, p):
    """E^{ij}_t for t = 0..i+j (1-D Hermite expansion of x_A^i x_B^j about P, without K)."""
    E = {(0, 0, 0): 1.0}

    def get(a, b, t):
        if t < 0 or t > a + b:
            return 0.0
        return E[(a, b, t)]

    for a in range(i + 1):
        for b in range(j + 1):
            if a == 0 and b == 0:
                continue
            for t in range(a + b + 1):
                if a > 0:
                    v = get(a - 1, b, t - 1) / (2 * p) + Xpa * get(a - 1, b, t) + (t + 1) * get(a - 1, b, t + 1)
                else:
                    v = get(a, b - 1, t - 1) / (2 * p) + Xpb * get(a, b - 1, t) + (t + 1) * get(a, b - 1, t + 1)
                E[(a, b, t)] = v
    return [get(i, j, t) for t in range(i + j + 1)]


def _hermite_R(L, p, PC):
    """R^0_{tuv} for t+u+v <= L (Hermite Coulomb integrals)."""
    X, Y, Z = PC
    T = p * float(np.dot(PC, PC))
    F = [boys_mp(n, T) for n in range(L + 1)]
    R = {}
    for n in range(L + 1):
        R[(0, 0, 0, n)] = (-2 * p) ** n * F[n]

    def get(t, u, v, n):
        if t < 0 or u < 0 or v < 0:
            return 0.0
        return R[(t, u, v, n)]

    for tot in range(1, L + 1):
        for n in range(L - tot, -1, -1):
            for t in range(tot + 1):
                for u in range(tot - t + 1):
                    v = tot - t - u
                    if t > 0:
                        val = (t - 1) * get(t - 2, u, v, n + 1) + X * get(t - 1, u, v, n + 1)
                    elif u > 0:
                        val = (u - 1) * get(t, u - 2, v, n + 1) + Y * get(t, u - 1, v, n + 1)
                    else:
                        val = (v - 1) * get(t, u, v - 2, n + 1) + Z * get(t, u, v - 1, n + 1)
                    R[(t, u, v, n)] = val
    return lambda t, u, v: R[(t, u, v, 0)]


def md_nuclear_prim(la, A, a, lb, B, b, c):
    """Real (2la+1) x (2lb+1) block of int S_a e^{-a..} S_b e^{-b..} / |r - c| (unnormalised)."""
    A = np.asarray(A, float)
    B = np.asarray(B, float)
    c = np.asarray(c, float)
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * float(np.dot(A - B, A - B)))
    Rf = _hermite_R(la + lb, p, P - c)
    ma, mb = monomials(la), monomials(lb)
    Vc = np.zeros((len(ma), len(mb)))
    for u, (i1, j1, k1) in enumerate(ma):
        for v, (i2, j2, k2) in enumerate(mb):
            Ex = _hermite_E(i1, i2, P[0] - A[0], P[0] - B[0], p)
            Ey = _hermite_E(j1, j2, P[1] - A[1], P[1] - B[1], p)
            Ez = _hermite_E(k1, k2, P[2] - A[2], P[2] - B[2], p)
            s = 0.0
            for t, ex in enumerate(Ex):
                for uu, ey in enumerate(Ey):
                    for vv, ez in enumerate(Ez):
                        s += ex * ey * ez * Rf(t, uu, vv)
            Vc[u, v] = 2 * math.pi / p * K * s
    return real_solid_poly(la) @ Vc @ real_solid_poly(lb).T


def contracted_block(route, basis, nuclei, sa, sb, keep=None):
    """Real V block for shells sa, sb using route ``md_nuclear_prim`` or ``quad_nuclear_prim``;
    ``keep`` (K_a x K_b booleans, or None for all) selects the primitive pairs that enter."""
    la, lb = int(basis.l[sa]), int(basis.l[sb])
    A, B = basis.center[sa], basis.center[sb]
    ea = basis.expo[basis.prim_off[sa]:basis.prim_off[sa] + basis.nprim[sa]]
    da = basis.coef[basis.prim_off[sa]:basis.prim_off[sa] + basis.nprim[sa]]
    eb = basis.expo[basis.prim_off[sb]:basis.prim_off[sb] + basis.nprim[sb]]
    db = basis.coef[basis.prim_off[sb]:basis.prim_off[sb] + basis.nprim[sb]]
    wa = contracted_weights(la, ea, da)
    wb = contracted_weights(lb, eb, db)
    out = np.zeros((2 * la + 1, 2 * lb + 1))
    for i, a in enumerate(ea):
        for j, b in enumerate(eb):
            if keep is not None and not keep[i, j]:
                continue
            for c, Z in zip(nuclei.pos, nuclei.Z):
                out -= Z * wa[i] * wb[j] * route(la, A, a, lb, B, b, c)
    return out


def real_wigner_d(l, Q):
    """D^l with S^l(Q x) = D^l S^l(x), by least squares over random points."""
    rng = np.random.default_rng(77 + l)
    X = rng.normal(size=(4 * (2 * l + 1) + 5, 3))
    Sx = np.array([eval_real_solid(l, *x) for x in X])
    SQx = np.array([eval_real_solid(l, *(Q @ x)) for x in X])
    Dt, *_ = np.linalg.lstsq(Sx, SQx, rcond=None)
    return Dt.T


# ----------------------------------------------------------------------------------------------
# Two-electron integrals by the Gaussian transform 1/r12 = (2/sqrt(pi)) int_0^inf exp(-u^2 r12^2) du
# ----------------------------------------------------------------------------------------------
def _eri_dim(i1, j1, i2, j2, A, B, C, D, a, b, c, d, u, nq):
    """int int (x1-A)^i1 (x1-B)^j1 (x2-C)^i2 (x2-D)^j2 e^{-a(x1-A)^2-b(x1-B)^2-c(x2-C)^2-d(x2-D)^2-u^2(x1-x2)^2}
    by Gauss-Hermite quadrature in the eigen-coordinates of the 2-D quadratic form (exact: the
    integrand is a polynomial of degree < 2 nq times the Gaussian)."""
    # quadratic form x^T M x - 2 g^T x + h
    M = np.array([[a + b + u * u, -u * u], [-u * u, c + d + u * u]])
    g = np.array([a * A + b * B, c * C + d * D])
    h = a * A * A + b * B * B + c * C * C + d * D * D
    xs = np.linalg.solve(M, g)
    c0 = h - g @ xs
    Lc = np.linalg.cholesky(M)                    # M = L L^T
    T = np.linalg.inv(Lc.T)                       # x = xs + T y, |y|^2 = (x - xs)^T M (x - xs)
    y, w = np.polynomial.hermite.hermgauss(nq)
    Y1, Y2 = np.meshgrid(y, y, indexing="ij")
    W = np.outer(w, w)
    X1 = xs[0] + T[0, 0] * Y1 + T[0, 1] * Y2
    X2 = xs[1] + T[1, 0] * Y1 + T[1, 1] * Y2
    f = (X1 - A) ** i1 * (X1 - B) ** j1 * (X2 - C) ** i2 * (X2 - D) ** j2
    return float(np.sum(W * f)) * abs(np.linalg.det(T)) * math.exp(-c0)


def quad_eri_prim(la, A, a, lb, B, b, lc, C, c, ld, D, d):
    """Real (2la+1)(2lb+1)(2lc+1)(2ld+1) primitive (ab|cd) block (unnormalised) by the Gaussian
    transform of 1/r12, Gauss-Hermite quadrature in each dimension and adaptive quadrature in u."""
    A, B, C, D = (np.asarray(x, float) for x in (A, B, C, D))
    ma, mb, mc, md = monomials(la), monomials(lb), monomials(lc), monomials(ld)
    nq = (la + lb + lc + ld) // 2 + 3
    cart = np.zeros((len(ma), len(mb), len(mc), len(md)))
    for ia, ea in enumerate(ma):
        for ib, eb in enumerate(mb):
            for ic, ec in enumerate(mc):
                for id_, ed in enumerate(md):
                    def f(u):
                        v = 1.0
                        for x in range(3):
                            v *= _eri_dim(ea[x], eb[x], ec[x], ed[x], A[x], B[x], C[x], D[x], a, b, c, d, u, nq)
                        return v
                    v1, _ = integrate.quad(f, 0.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)
                    v2, _ = integrate.quad(f, 1.0, np.inf, epsabs=0, epsrel=1e-13, limit=200)
                    cart[ia, ib, ic, id_] = 2.0 / math.sqrt(math.pi) * (v1 + v2)
    Ca, Cb, Cc, Cd = real_solid_poly(la), real_solid_poly(lb), real_solid_poly(lc), real_solid_poly(ld)
    return np.einsum("ai,bj,ck,dl,ijkl->abcd", Ca, Cb, Cc, Cd, cart)
