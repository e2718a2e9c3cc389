"""Oracle: plain, slow CPU reference for SHGO nuclear-attraction integrals (test infrastructure).

Only the test suite, the smoke check and the bench's CPU-baseline leg may import this package.
The library it loads (``liboracle.so``, built from ``shgo_oracle.cpp`` by ``build_oracle.py``)
shares no code with the GPU path. Every function cites, in the C++ source, the passage of the
paper (arXiv:2404.16245) it follows.

Precision argument: 0 = double (the oracle proper), 1 = long double, 2 = __float128 (used only
to certify the double oracle's rounding error).
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        lib = ctypes.CDLL(build_oracle.LIB)
        lib.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _d]
        lib.oracle_solid_complex.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _d]
        lib.oracle_solid_real.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _d]
        lib.oracle_cg.argtypes = [ctypes.c_int] * 6
        lib.oracle_cg.restype = ctypes.c_double
        lib.oracle_eps.argtypes = [ctypes.c_int] * 4
        lib.oracle_eps.restype = ctypes.c_double
        lib.oracle_shift_matrix.argtypes = [ctypes.c_int, ctypes.c_double, _d, _d]
        lib.oracle_one_center.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _d, _d]
        basis_args = [ctypes.c_int, _d, _i32, _i32, _i64, _d, _d]
        lib.oracle_blocks.argtypes = ([ctypes.c_int] + basis_args + [ctypes.c_int, _d, _d, ctypes.c_int64, _i32, _i32,
                                                                    ctypes.c_double, _d, ctypes.c_int])
        lib.oracle_blocks.restype = ctypes.c_int
        lib.oracle_matrix.argtypes = [ctypes.c_int] + basis_args + [ctypes.c_int, _d, _d, ctypes.c_double, _d, ctypes.c_int]
        lib.oracle_matrix.restype = ctypes.c_int
        lib.oracle_grad.argtypes = (basis_args + [ctypes.c_int, _d, _d, ctypes.c_double, _d, _d, _d, _d, ctypes.c_int])
        lib.oracle_grad.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ptr):
    return a.ctypes.data_as(ptr)


def _basis_args(basis):
    c = np.ascontiguousarray(basis.center, dtype=np.float64)
    l = np.ascontiguousarray(basis.l, dtype=np.int32)
    k = np.ascontiguousarray(basis.nprim, dtype=np.int32)
    o = np.ascontiguousarray(basis.prim_off, dtype=np.int64)
    e = np.ascontiguousarray(basis.expo, dtype=np.float64)
    d = np.ascontiguousarray(basis.coef, dtype=np.float64)
    keep = (c, l, k, o, e, d)
    return keep, [basis.n_shells, _p(c, _d), _p(l, _i32), _p(k, _i32), _p(o, _i64), _p(e, _d), _p(d, _d)]


def _nuc_args(nuclei):
    pos = np.ascontiguousarray(nuclei.pos, dtype=np.float64).reshape(-1, 3)
    Z = np.ascontiguousarray(nuclei.Z, dtype=np.float64)
    return (pos, Z), [int(Z.shape[0]), _p(pos, _d), _p(Z, _d)]


def boys(mmax, t, precision=0):
    """F_0..F_mmax at t (Boys function, the radial factor of Eq. 12)."""
    out = np.zeros(mmax + 1)
    _load().oracle_boys(precision, mmax, float(t), _p(out, _d))
    return out


def solid_complex(lmax, x, y, z):
    """Complex regular solid harmonics (Eq. 2), index l*l + m + l."""
    out = np.zeros(2 * (lmax + 1) ** 2)
    _load().oracle_solid_complex(lmax, float(x), float(y), float(z), _p(out, _d))
    return out[0::2] + 1j * out[1::2]


def solid_real(lmax, x, y, z):
    """Real solid harmonics, order m = -l..l, index l*l + m + l."""
    out = np.zeros((lmax + 1) ** 2)
    _load().oracle_solid_real(lmax, float(x), float(y), float(z), _p(out, _d))
    return out


def cg(j1, m1, j2, m2, J, M):
    return _load().oracle_cg(j1, m1, j2, m2, J, M)


def eps(l1, l2, m1, m2):
    """Vector-coupling coefficient of Eq. 8."""
    return _load().oracle_eps(l1, l2, m1, m2)


def shift_matrix(la, s, R):
    """Complex shift matrix of Eq. 7 (sign-corrected): (2la+1) x (la+1)^2."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    out = np.zeros(2 * (2 * la + 1) * (la + 1) ** 2)
    _load().oracle_shift_matrix(la, float(s), _p(R, _d), _p(out, _d))
    return (out[0::2] + 1j * out[1::2]).reshape(2 * la + 1, (la + 1) ** 2)


def one_center(la, lb, p, C, precision=0):
    """Complex one-center Coulomb table I(l1 m1, l2 m2), shape ((la+1)^2, (lb+1)^2)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    out = np.zeros(2 * (la + 1) ** 2 * (lb + 1) ** 2)
    _load().oracle_one_center(precision, la, lb, float(p), _p(C, _d), _p(out, _d))
    return (out[0::2] + 1j * out[1::2]).reshape((la + 1) ** 2, (lb + 1) ** 2)


def block_sizes(basis, pa, pb):
    la = basis.l[pa].astype(np.int64)
    lb = basis.l[pb].astype(np.int64)
    return (2 * la + 1) * (2 * lb + 1)


def nuc_blocks(basis, nuclei, pa, pb, screen=0.0, precision=0, nthreads=0):
    """Concatenated real blocks V[a, b] (row-major (2la+1)x(2lb+1)) for the listed shell pairs."""
    pa = np.ascontiguousarray(pa, dtype=np.int32)
    pb = np.ascontiguousarray(pb, dtype=np.int32)
    out = np.zeros(int(block_sizes(basis, pa, pb).sum()))
    keep, bargs = _basis_args(basis)
    nkeep, nargs = _nuc_args(nuclei)
    rc = _load().oracle_blocks(precision, *bargs, *nargs, len(pa), _p(pa, _i32), _p(pb, _i32), float(screen),
                               _p(out, _d), int(nthreads))
    if rc:
        raise ValueError("oracle: invalid basis")
    return out


def overlap_blocks(basis, pa, pb, precision=0, nthreads=0):
    """Concatenated real overlap blocks S[a, b] (Eqs. 9-10, sign-corrected)."""
    pa = np.ascontiguousarray(pa, dtype=np.int32)
    pb = np.ascontiguousarray(pb, dtype=np.int32)
    out = np.zeros(int(block_sizes(basis, pa, pb).sum()))
    keep, bargs = _basis_args(basis)
    dummy = np.zeros(3)
    rc = _load().oracle_blocks(precision, *bargs, -1, _p(dummy, _d), _p(dummy, _d), len(pa), _p(pa, _i32),
                               _p(pb, _i32), 0.0, _p(out, _d), int(nthreads))
    if rc:
        raise ValueError("oracle: invalid basis")
    return out


def nuc_matrix(basis, nuclei, screen=0.0, precision=0, nthreads=0):
    """Full symmetric nbf x nbf nuclear-attraction matrix."""
    nbf = basis.nbf()
    V = np.zeros((nbf, nbf))
    keep, bargs = _basis_args(basis)
    nkeep, nargs = _nuc_args(nuclei)
    rc = _load().oracle_matrix(precision, *bargs, *nargs, float(screen), _p(V, _d), int(nthreads))
    if rc:
        raise ValueError("oracle: invalid basis")
    return V


def grad(basis, nuclei, D, screen=0.0, nthreads=0):
    """Analytic gradient of E = sum_ij D_ij V_ij by dual numbers.

    Returns (dE/d nuclear positions [n_nuc, 3], dE/d shell centers [n_shells, 3], E)."""
    nbf = basis.nbf()
    D = np.ascontiguousarray(D, dtype=np.float64)
    assert D.shape == (nbf, nbf)
    dn = np.zeros((nuclei.n, 3))
    dc = np.zeros((basis.n_shells, 3))
    e = np.zeros(1)
    keep, bargs = _basis_args(basis)
    nkeep, nargs = _nuc_args(nuclei)
    rc = _load().oracle_grad(*bargs, *nargs, float(screen), _p(D, _d), _p(dn, _d), _p(dc, _d), _p(e, _d),
                             int(nthreads))
    if rc:
        raise ValueError("oracle: invalid basis")
    return dn, dc, float(e[0])


def split_blocks(flat, basis, pa, pb):
    """Split concatenated blocks into a list of 2-D arrays."""
    sizes = block_sizes(basis, pa, pb)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return [flat[offs[i]:offs[i + 1]].reshape(2 * basis.l[pa[i]] + 1, 2 * basis.l[pb[i]] + 1)
            for i in range(len(pa))]
