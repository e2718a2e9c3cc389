// Oracle: plain, slow CPU evaluation of one-electron nuclear-attraction integrals over
// contracted solid-harmonic Gaussian orbitals (SHGOs), following the vector-coupling route of
// Hu, Peslherbe, Ooi and Hu, "Computationally Efficient Molecular Integrals of Solid Harmonic
// Gaussian Orbitals Using Quantum Entanglement of Angular Momentum" (arXiv:2404.16245).
//
// TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg of the
// bench load this library. It shares no code, header, table or constant with the GPU path.
//
// Route (every step in the paper's order and notation, with two corrections that are listed
// as readings in the design notes):
//   1. SHGO primitive N(l,a) Y^l_m(r-A) exp(-a|r-A|^2)                          (Eq. 1)
//   2. complex regular solid harmonics, Racah normalisation, Condon-Shortley      (Eq. 2)
//   3. Gaussian product: p = a+b, P = (aA+bB)/p, K = exp(-ab/p |A-B|^2)           (Eq. 5)
//   4. shift of both harmonics to P with the vector-coupling coefficients eps     (Eqs. 7, 8)
//      -- reading: the shift vector is P-A = (b/p)(B-A) (and P-B = (a/p)(A-B)); the printed
//         Eq. 7 carries (A-B), which flips the sign of odd l_a-l_1 terms.
//   5. one-center Coulomb integral at P for nucleus c                             (Eq. 11)
//      -- reading: the product of the two harmonics at P is first coupled with the product
//         rule (Clebsch-Gordan form of the supplement's Eq. 4); each r^{2k} Y^L_M term is then
//         integrated with Hobson's theorem and the Boys function (Eq. 12 holds for k = 0, and
//         r^{2k} exp(-p r^2) = (-d/dp)^k exp(-p r^2) gives the k > 0 terms).
//   6. sum over nuclei with charge Z_c and sign -1, contraction over primitives, and the
//      unitary map from complex to real solid harmonics (real output basis).
//
// Parity pins (tests/test_oracle_*.py): Boys against mpmath, harmonics against sympy, CG
// against sympy, the addition theorem and the product rule at random points, one-center
// integrals and full matrices against an independent Gaussian-transform quadrature and an
// independent Cartesian McMurchie-Davidson route, rotation/translation invariance, symmetry,
// unit self-overlap, and the oracle's own rounding error via long double / __float128.
//
// Scalar types: double (the oracle), long double and __float128 (to certify the double
// oracle's rounding), and a forward-mode dual number (analytic gradient, independent of any
// hand-written adjoint).

#include <quadmath.h>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ------------------------------------------------------------------------------------------
// Scalar support
// ------------------------------------------------------------------------------------------
// Forward-mode dual number with one derivative component.
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual& operator/=(Dual& a, Dual b) { a = a / b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }

inline double val(double x) { return x; }
inline double val(long double x) { return (double)x; }
inline double val(__float128 x) { return (double)x; }
inline double val(Dual x) { return x.v; }

inline double t_exp(double x) { return std::exp(x); }
inline long double t_exp(long double x) { return expl(x); }
inline __float128 t_exp(__float128 x) { return expq(x); }
inline Dual t_exp(Dual x) { double e = std::exp(x.v); return Dual(e, e * x.d); }

inline double t_sqrt(double x) { return std::sqrt(x); }
inline long double t_sqrt(long double x) { return sqrtl(x); }
inline __float128 t_sqrt(__float128 x) { return sqrtq(x); }
inline Dual t_sqrt(Dual x) { double s = std::sqrt(x.v); return Dual(s, s > 0 ? x.d / (2 * s) : 0.0); }

template <class T> T t_pi();
template <> double t_pi<double>() { return 3.14159265358979323846; }
template <> long double t_pi<long double>() { return 3.141592653589793238462643383279502884L; }
template <> __float128 t_pi<__float128>() { return M_PIq; }
template <> Dual t_pi<Dual>() { return Dual(3.14159265358979323846); }

// Relative tolerance for series truncation, per type.
template <class T> double t_eps();
template <> double t_eps<double>() { return 1e-18; }
template <> double t_eps<long double>() { return 1e-21; }
template <> double t_eps<__float128>() { return 1e-36; }
template <> double t_eps<Dual>() { return 1e-18; }

// Minimal complex number over any scalar (std::complex is unspecified for non-standard types).
template <class T> struct Cx {
  T re, im;
  Cx() : re(0), im(0) {}
  Cx(T r) : re(r), im(0) {}
  Cx(T r, T i) : re(r), im(i) {}
};
template <class T> inline Cx<T> operator+(Cx<T> a, Cx<T> b) { return Cx<T>(a.re + b.re, a.im + b.im); }
template <class T> inline Cx<T> operator-(Cx<T> a, Cx<T> b) { return Cx<T>(a.re - b.re, a.im - b.im); }
template <class T> inline Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return Cx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T> inline Cx<T> operator*(T s, Cx<T> a) { return Cx<T>(s * a.re, s * a.im); }
template <class T> inline Cx<T> conj(Cx<T> a) { return Cx<T>(a.re, T(0) - a.im); }

// Factorials as T (exact up to 22! in double; fine for the precisions used).
template <class T> T fact(int n) {
  T f = T(1);
  for (int i = 2; i <= n; ++i) f = f * T(i);
  return f;
}
template <class T> T binom(int n, int k) {
  if (k < 0 || k > n || n < 0) return T(0);
  return fact<T>(n) / (fact<T>(k) * fact<T>(n - k));
}
template <class T> T dfact(int n) {  // n!!, with (-1)!! = 1
  T f = T(1);
  for (int i = n; i > 1; i -= 2) f = f * T(i);
  return f;
}

// ------------------------------------------------------------------------------------------
// Boys function F_m(t) = int_0^1 u^{2m} exp(-t u^2) du  (the radial factor of Eq. 12)
// ------------------------------------------------------------------------------------------
// t <= 40: the convergent series F_m = exp(-t) sum_i (2t)^i / ((2m+1)(2m+3)...(2m+2i+1)),
// all terms positive.  t > 40: F_0 = sqrt(pi/t)/2 * erf(sqrt t), with erfc(sqrt t) from
// Laplace's continued fraction, then the upward recursion F_{m+1} = ((2m+1)F_m - e^{-t})/(2t),
// which loses no accuracy when t exceeds m.
template <class T> T erfc_large(T x) {
  // erfc(x) = exp(-x^2)/sqrt(pi) * 1/(x + (1/2)/(x + 1/(x + (3/2)/(x + 2/(x + ...)))))
  T frac = x;
  for (int n = 400; n >= 1; --n) frac = x + T(0.5 * n) / frac;
  return t_exp(T(0) - x * x) / (t_sqrt(t_pi<T>()) * frac);
}

template <class T> void boys(int mmax, T t, T* F) {
  if (val(t) <= 40.0) {
    T et = t_exp(T(0) - t);
    for (int m = 0; m <= mmax; ++m) {
      T term = T(1) / T(2 * m + 1);
      T sum = term;
      for (int i = 1; i < 2000; ++i) {
        term = term * (T(2) * t) / T(2 * m + 2 * i + 1);
        sum = sum + term;
        if (val(term) <= t_eps<T>() * val(sum)) break;
      }
      F[m] = et * sum;
    }
  } else {
    T x = t_sqrt(t);
    T f0 = t_sqrt(t_pi<T>()) / (T(2) * x) * (T(1) - erfc_large(x));
    T et = t_exp(T(0) - t);
    F[0] = f0;
    for (int m = 0; m < mmax; ++m) F[m + 1] = (T(2 * m + 1) * F[m] - et) / (T(2) * t);
  }
}

// Dual-number Boys function: value from the double routine, derivative dF_m/dt = -F_{m+1}.
template <> void boys<Dual>(int mmax, Dual t, Dual* F) {
  std::vector<double> f(mmax + 2);
  boys<double>(mmax + 1, t.v, f.data());
  for (int m = 0; m <= mmax; ++m) F[m] = Dual(f[m], -f[m + 1] * t.d);
}

// ------------------------------------------------------------------------------------------
// Complex regular solid harmonics Y^l_m(x,y,z) = sqrt(4pi/(2l+1)) r^l Y_lm  (Eq. 2)
// ------------------------------------------------------------------------------------------
// For m >= 0 the textbook polynomial
//   Y^l_m = sqrt((l+m)!(l-m)!) sum_k (-(x+iy)/2)^{m+k} ((x-iy)/2)^k z^{l-m-2k} / ((m+k)! k! (l-m-2k)!)
// and Y^l_{-m} = (-1)^m conj(Y^l_m).  Output index: l*l + (m + l).
template <class T> void solid_complex(int lmax, T x, T y, T z, Cx<T>* Y) {
  const int n = 2 * lmax + 2;
  std::vector<Cx<T>> wp(n + 1), vp(n + 1);
  std::vector<T> zp(n + 1);
  Cx<T> w(T(0) - x / T(2), T(0) - y / T(2));
  Cx<T> v(x / T(2), T(0) - y / T(2));
  wp[0] = Cx<T>(T(1));
  vp[0] = Cx<T>(T(1));
  zp[0] = T(1);
  for (int i = 1; i <= n; ++i) {
    wp[i] = wp[i - 1] * w;
    vp[i] = vp[i - 1] * v;
    zp[i] = zp[i - 1] * z;
  }
  for (int l = 0; l <= lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      Cx<T> s;
      for (int k = 0; 2 * k <= l - m; ++k) {
        T c = T(1) / (fact<T>(m + k) * fact<T>(k) * fact<T>(l - m - 2 * k));
        s = s + (c * zp[l - m - 2 * k]) * (wp[m + k] * vp[k]);
      }
      s = t_sqrt(fact<T>(l + m) * fact<T>(l - m)) * s;
      Y[l * l + (m + l)] = s;
      if (m > 0) {
        Cx<T> c = conj(s);
        if (m & 1) c = Cx<T>(T(0) - c.re, T(0) - c.im);
        Y[l * l + (-m + l)] = c;
      }
    }
  }
}

// Unitary map to real solid harmonics, S^l = U_l Y^l (real order m = -l..l):
//   S^l_0 = Y^l_0;  S^l_m = ((-1)^m Y^l_m + Y^l_{-m})/sqrt2;  S^l_{-m} = i(Y^l_{-m} - (-1)^m Y^l_m)/sqrt2.
// U is stored (2l+1) x (2l+1), row = real index m'+l, column = complex index m+l.
template <class T> void real_map(int l, Cx<T>* U) {
  const int d = 2 * l + 1;
  for (int i = 0; i < d * d; ++i) U[i] = Cx<T>();
  T h = T(1) / t_sqrt(T(2));
  U[l * d + l] = Cx<T>(T(1));
  for (int m = 1; m <= l; ++m) {
    T sg = (m & 1) ? T(-1) : T(1);
    U[(m + l) * d + (m + l)] = Cx<T>(sg * h);
    U[(m + l) * d + (-m + l)] = Cx<T>(h);
    U[(-m + l) * d + (-m + l)] = Cx<T>(T(0), h);
    U[(-m + l) * d + (m + l)] = Cx<T>(T(0), T(0) - sg * h);
  }
}

// ------------------------------------------------------------------------------------------
// Vector-coupling coefficients (Eq. 8) and Clebsch-Gordan coefficients (Racah formula)
// ------------------------------------------------------------------------------------------
template <class T> T eps_coef(int l1, int l2, int m1, int m2) {
  // sqrt( C(l1+m1, l2+m2) C(l1-m1, l2-m2) ), zero when a lower index leaves [0, upper].
  T b1 = binom<T>(l1 + m1, l2 + m2);
  T b2 = binom<T>(l1 - m1, l2 - m2);
  return t_sqrt(b1 * b2);
}

template <class T> T clebsch(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M) return T(0);
  if (J < std::abs(j1 - j2) || J > j1 + j2) return T(0);
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return T(0);
  T pre = T(2 * J + 1) * fact<T>(J + j1 - j2) * fact<T>(J - j1 + j2) * fact<T>(j1 + j2 - J) /
          fact<T>(j1 + j2 + J + 1);
  pre = pre * fact<T>(J + M) * fact<T>(J - M) * fact<T>(j1 - m1) * fact<T>(j1 + m1) *
        fact<T>(j2 - m2) * fact<T>(j2 + m2);
  T s = T(0);
  for (int k = 0; k <= j1 + j2 + J; ++k) {
    int a1 = j1 + j2 - J - k, a2 = j1 - m1 - k, a3 = j2 + m2 - k, a4 = J - j2 + m1 + k,
        a5 = J - j1 - m2 + k;
    if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0 || a5 < 0) continue;
    T term = T(1) / (fact<T>(k) * fact<T>(a1) * fact<T>(a2) * fact<T>(a3) * fact<T>(a4) * fact<T>(a5));
    s = (k & 1) ? s - term : s + term;
  }
  return t_sqrt(pre) * s;
}

// Product rule of complex solid harmonics (supplement Eq. 4 in Clebsch-Gordan form):
//   Y^{l1}_{m1} Y^{l2}_{m2} = sum_L <l1 0 l2 0|L 0><l1 m1 l2 m2|L M> r^{l1+l2-L} Y^L_M.
template <class T> struct Coupling {
  int lmax;
  std::vector<T> g;  // indexed [l1][m1][l2][m2][L]
  explicit Coupling(int lm) : lmax(lm) {
    int d = 2 * lm + 1, nl = lm + 1, nL = 2 * lm + 1;
    g.assign((size_t)nl * d * nl * d * nL, T(0));
    for (int l1 = 0; l1 <= lm; ++l1)
      for (int m1 = -l1; m1 <= l1; ++m1)
        for (int l2 = 0; l2 <= lm; ++l2)
          for (int m2 = -l2; m2 <= l2; ++m2)
            for (int L = std::abs(l1 - l2); L <= l1 + l2; L += 2) {
              int M = m1 + m2;
              if (std::abs(M) > L) continue;
              g[idx(l1, m1, l2, m2, L)] = clebsch<T>(l1, 0, l2, 0, L, 0) * clebsch<T>(l1, m1, l2, m2, L, M);
            }
  }
  size_t idx(int l1, int m1, int l2, int m2, int L) const {
    int d = 2 * lmax + 1, nl = lmax + 1, nL = 2 * lmax + 1;
    return ((((size_t)l1 * d + (m1 + lmax)) * nl + l2) * d + (m2 + lmax)) * nL + L;
  }
};

// ------------------------------------------------------------------------------------------
// One-center Coulomb integral at P (last line of Eq. 11):
//   I(l1 m1, l2 m2) = int Y^{l1}_{m1}(rho) Y^{l2}_{m2}(rho) exp(-p rho^2) / |rho - C| d^3rho
// with rho = r - P and C = c - P.  Product rule, then for each r^{2k} Y^L_M term
//   int rho^{2k} Y^L_M(rho) exp(-p rho^2)/|rho - C| = Y^L_M(C) * 2 pi k!/p^{k+1} sum_j T^j/j! F_{L+j}(T)
// with T = p |C|^2 (Hobson's theorem plus the Boys function; the k > 0 terms follow from
// r^{2k} exp(-p r^2) = (-d/dp)^k exp(-p r^2) and dF_m/dT = -F_{m+1}).
// Output: I[(l1*l1 + m1 + l1) * (lb+1)^2 + (l2*l2 + m2 + l2)], complex.
// ------------------------------------------------------------------------------------------
template <class T>
void one_center(int la, int lb, T p, T Cx_, T Cy_, T Cz_, const Coupling<T>& cp, Cx<T>* I) {
  const int Lmax = la + lb;
  std::vector<Cx<T>> YC((Lmax + 1) * (Lmax + 1));
  solid_complex<T>(Lmax, Cx_, Cy_, Cz_, YC.data());
  T t = p * (Cx_ * Cx_ + Cy_ * Cy_ + Cz_ * Cz_);
  std::vector<T> F(Lmax + 1);
  boys<T>(Lmax, t, F.data());
  // J[L][k]
  const int kmax = std::min(la, lb);
  std::vector<T> J((Lmax + 1) * (kmax + 1), T(0));
  for (int L = 0; L <= Lmax; ++L)
    for (int k = 0; k <= kmax && L + 2 * k <= Lmax; ++k) {
      T s = T(0), tj = T(1);
      for (int j = 0; j <= k; ++j) {
        s = s + tj / fact<T>(j) * F[L + j];
        tj = tj * t;
      }
      T pk = p;
      for (int j = 0; j < k; ++j) pk = pk * p;
      J[L * (kmax + 1) + k] = T(2) * t_pi<T>() * fact<T>(k) / pk * s;
    }
  const int nb = (lb + 1) * (lb + 1);
  for (int l1 = 0; l1 <= la; ++l1)
    for (int m1 = -l1; m1 <= l1; ++m1)
      for (int l2 = 0; l2 <= lb; ++l2)
        for (int m2 = -l2; m2 <= l2; ++m2) {
          Cx<T> s;
          int M = m1 + m2;
          for (int L = std::abs(l1 - l2); L <= l1 + l2; L += 2) {
            if (std::abs(M) > L) continue;
            int k = (l1 + l2 - L) / 2;
            T g = cp.g[cp.idx(l1, m1, l2, m2, L)];
            s = s + (g * J[L * (kmax + 1) + k]) * YC[L * L + M + L];
          }
          I[(l1 * l1 + m1 + l1) * nb + (l2 * l2 + m2 + l2)] = s;
        }
}

// Shift matrix of Eq. 7 (sign-corrected): Y^{la}_{ma}(r - A) = sum_{l1 m1} S[ma][l1 m1] Y^{l1}_{m1}(r - P)
// with S[ma][l1 m1] = eps_{la l1 ma m1} (b/p)^{la-l1} Y^{la-l1}_{ma-m1}(B - A).
// Arguments: s = b/p, (Rx,Ry,Rz) = B - A.  Output (2la+1) x (la+1)^2.
template <class T> void shift_matrix(int la, T s, T Rx, T Ry, T Rz, Cx<T>* S) {
  std::vector<Cx<T>> YR((la + 1) * (la + 1));
  solid_complex<T>(la, Rx, Ry, Rz, YR.data());
  const int na = (la + 1) * (la + 1);
  for (int ma = -la; ma <= la; ++ma)
    for (int l1 = 0; l1 <= la; ++l1)
      for (int m1 = -l1; m1 <= l1; ++m1) {
        int lam = la - l1, mu = ma - m1;
        Cx<T> v;
        if (std::abs(mu) <= lam) {
          T sp = T(1);
          for (int j = 0; j < lam; ++j) sp = sp * s;
          v = (eps_coef<T>(la, l1, ma, m1) * sp) * YR[lam * lam + mu + lam];
        }
        S[(ma + la) * na + (l1 * l1 + m1 + l1)] = v;
      }
}

// Complex primitive integral (unnormalised, no conjugation) for one nucleus at c:
//   N(ma, mb) = int Y^{la}_{ma}(r-A) e^{-a|r-A|^2} Y^{lb}_{mb}(r-B) e^{-b|r-B|^2} / |r-c|   (Eq. 11)
// accumulated as out += w * N.  Output (2la+1) x (2lb+1).
template <class T>
void prim_nuc(int la, int lb, T a, const T* A, T b, const T* B, const T* c, T w, const Coupling<T>& cp,
              Cx<T>* out) {
  T p = a + b;
  T P[3], R[3], mR[3];
  for (int i = 0; i < 3; ++i) {
    P[i] = (a * A[i] + b * B[i]) / p;
    R[i] = B[i] - A[i];
    mR[i] = A[i] - B[i];
  }
  T mu = a * b / p;
  T K = t_exp(T(0) - mu * (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]));  // Eq. 5
  const int na = (la + 1) * (la + 1), nb = (lb + 1) * (lb + 1);
  std::vector<Cx<T>> Sa((2 * la + 1) * na), Sb((2 * lb + 1) * nb), I(na * nb);
  shift_matrix<T>(la, b / p, R[0], R[1], R[2], Sa.data());
  shift_matrix<T>(lb, a / p, mR[0], mR[1], mR[2], Sb.data());
  one_center<T>(la, lb, p, c[0] - P[0], c[1] - P[1], c[2] - P[2], cp, I.data());
  // N = K * Sa * I * Sb^T  (plain matrix products, Eq. 11 double sum)
  std::vector<Cx<T>> X((2 * la + 1) * nb);
  for (int i = 0; i < 2 * la + 1; ++i)
    for (int q = 0; q < nb; ++q) {
      Cx<T> s;
      for (int r = 0; r < na; ++r) s = s + Sa[i * na + r] * I[r * nb + q];
      X[i * nb + q] = s;
    }
  T wk = w * K;
  for (int i = 0; i < 2 * la + 1; ++i)
    for (int j = 0; j < 2 * lb + 1; ++j) {
      Cx<T> s;
      for (int q = 0; q < nb; ++q) s = s + X[i * nb + q] * Sb[j * nb + q];
      out[i * (2 * lb + 1) + j] = out[i * (2 * lb + 1) + j] + wk * s;
    }
}

// Complex primitive overlap (Eqs. 9, 10 with the sign correction): the one-center overlap
//   int Y^{l1}_{m1}(rho) Y^{l2}_{m2}(rho) e^{-p rho^2} = <l1 0 l2 0|00><l1 m1 l2 m2|00> (2k+1)!! pi^{3/2}/(2^k p^{k+3/2})
// with k = l1 = l2 (only the L = 0 term of the product rule survives the angular integral).
template <class T>
void prim_ovl(int la, int lb, T a, const T* A, T b, const T* B, T w, const Coupling<T>& cp, Cx<T>* out) {
  T p = a + b;
  T R[3], mR[3];
  for (int i = 0; i < 3; ++i) {
    R[i] = B[i] - A[i];
    mR[i] = A[i] - B[i];
  }
  T mu = a * b / p;
  T K = t_exp(T(0) - mu * (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]));
  const int na = (la + 1) * (la + 1), nb = (lb + 1) * (lb + 1);
  std::vector<Cx<T>> Sa((2 * la + 1) * na), Sb((2 * lb + 1) * nb), I(na * nb);
  shift_matrix<T>(la, b / p, R[0], R[1], R[2], Sa.data());
  shift_matrix<T>(lb, a / p, mR[0], mR[1], mR[2], Sb.data());
  T pi32 = t_pi<T>() * t_sqrt(t_pi<T>());
  for (int l1 = 0; l1 <= la; ++l1)
    for (int m1 = -l1; m1 <= l1; ++m1)
      for (int l2 = 0; l2 <= lb; ++l2)
        for (int m2 = -l2; m2 <= l2; ++m2) {
          Cx<T> v;
          if (l1 == l2 && m1 + m2 == 0) {
            int k = l1;
            T pk = t_sqrt(p) * p;
            for (int j = 0; j < k; ++j) pk = pk * (T(2) * p);
            v = Cx<T>(cp.g[cp.idx(l1, m1, l2, m2, 0)] * dfact<T>(2 * k + 1) * pi32 / pk);
          }
          I[(l1 * l1 + m1 + l1) * nb + (l2 * l2 + m2 + l2)] = v;
        }
  T wk = w * K;
  for (int i = 0; i < 2 * la + 1; ++i)
    for (int j = 0; j < 2 * lb + 1; ++j) {
      Cx<T> s;
      for (int r = 0; r < na; ++r)
        for (int q = 0; q < nb; ++q) s = s + Sa[i * na + r] * I[r * nb + q] * Sb[j * nb + q];
      out[i * (2 * lb + 1) + j] = out[i * (2 * lb + 1) + j] + wk * s;
    }
}

// ------------------------------------------------------------------------------------------
// Basis handling: normalisation N(l,a) and contraction (Eq. 1; the paper leaves N implicit)
// ------------------------------------------------------------------------------------------
//   N(l,a)^2 = 2^l (2a)^{l+3/2} / ((2l-1)!! pi^{3/2})   (unit self-overlap of a primitive)
//   chi = sum_k dhat_k N_k S^l_m(r-A) e^{-a_k |r-A|^2},  dhat = d / sqrt(sum d_k d_k' <phi_k|phi_k'>)
//   <phi_k|phi_k'> = N_k N_k' (2l-1)!! pi^{3/2} / (2^l (a_k + a_k')^{l+3/2})
template <class T> T prim_norm(int l, T a) {
  T x = t_sqrt(T(2) * a);  // (2a)^{1/2}
  T pw = x * x * x;        // (2a)^{3/2}
  for (int j = 0; j < l; ++j) pw = pw * T(2) * a;
  for (int j = 0; j < l; ++j) pw = pw * T(2);
  T pi32 = t_pi<T>() * t_sqrt(t_pi<T>());
  return t_sqrt(pw / (dfact<T>(2 * l - 1) * pi32));
}

struct Basis {
  int n_shells;
  const double* center;
  const int32_t* l;
  const int32_t* nprim;
  const int64_t* prim_off;
  const double* expo;
  const double* coef;
};

template <class T> struct ShellT {
  int l, K;
  T A[3];
  std::vector<T> a, w;  // exponents and dhat_k * N_k
};

template <class T> ShellT<T> make_shell(const Basis& bs, int s, const T* center_override) {
  ShellT<T> sh;
  sh.l = bs.l[s];
  sh.K = bs.nprim[s];
  for (int i = 0; i < 3; ++i) sh.A[i] = center_override ? center_override[i] : T(bs.center[3 * s + i]);
  const int64_t o = bs.prim_off[s];
  std::vector<T> N(sh.K), d(sh.K);
  sh.a.resize(sh.K);
  sh.w.resize(sh.K);
  for (int k = 0; k < sh.K; ++k) {
    sh.a[k] = T(bs.expo[o + k]);
    d[k] = T(bs.coef[o + k]);
    N[k] = prim_norm<T>(sh.l, sh.a[k]);
  }
  T pi32 = t_pi<T>() * t_sqrt(t_pi<T>());
  T ss = T(0);
  for (int k = 0; k < sh.K; ++k)
    for (int q = 0; q < sh.K; ++q) {
      T ap = sh.a[k] + sh.a[q];
      T pw = t_sqrt(ap) * ap;
      for (int j = 0; j < sh.l; ++j) pw = pw * ap * T(2);
      ss = ss + d[k] * d[q] * N[k] * N[q] * dfact<T>(2 * sh.l - 1) * pi32 / pw;
    }
  T inv = T(1) / t_sqrt(ss);
  for (int k = 0; k < sh.K; ++k) sh.w[k] = d[k] * inv * N[k];
  return sh;
}

// Real block (2la+1) x (2lb+1) for shells a, b, summing nuclei with -Z (or the overlap when
// nuc == nullptr).  Primitive pairs with exp(-mu R^2) <= screen are dropped (screen = 0 keeps all).
template <class T>
void shell_block(const ShellT<T>& sa, const ShellT<T>& sb, int n_nuc, const T* nuc_pos, const T* nuc_Z,
                 bool overlap, double screen, const Coupling<T>& cp, T* out_real) {
  const int la = sa.l, lb = sb.l, da = 2 * la + 1, db = 2 * lb + 1;
  std::vector<Cx<T>> acc(da * db);
  T R2 = T(0);
  for (int i = 0; i < 3; ++i) R2 = R2 + (sb.A[i] - sa.A[i]) * (sb.A[i] - sa.A[i]);
  for (int k = 0; k < sa.K; ++k)
    for (int q = 0; q < sb.K; ++q) {
      T a = sa.a[k], b = sb.a[q];
      if (screen > 0.0) {
        double Kv = std::exp(-val(a) * val(b) / (val(a) + val(b)) * val(R2));
        if (!(Kv > screen)) continue;
      }
      T w = sa.w[k] * sb.w[q];
      if (overlap) {
        prim_ovl<T>(la, lb, a, sa.A, b, sb.A, w, cp, acc.data());
      } else {
        for (int c = 0; c < n_nuc; ++c)
          prim_nuc<T>(la, lb, a, sa.A, b, sb.A, nuc_pos + 3 * c, T(0) - nuc_Z[c] * w, cp, acc.data());
      }
    }
  // complex -> real: V_real = U_a acc U_b^T (no conjugation: the real functions are real)
  std::vector<Cx<T>> Ua(da * da), Ub(db * db);
  real_map<T>(la, Ua.data());
  real_map<T>(lb, Ub.data());
  for (int i = 0; i < da; ++i)
    for (int j = 0; j < db; ++j) {
      Cx<T> s;
      for (int u = 0; u < da; ++u)
        for (int v = 0; v < db; ++v) s = s + Ua[i * da + u] * acc[u * db + v] * Ub[j * db + v];
      out_real[i * db + j] = s.re;
    }
}

template <class T>
int run_blocks(const Basis& bs, int n_nuc, const double* nuc_pos, const double* nuc_Z, int64_t n_pairs,
               const int32_t* pa, const int32_t* pb, double screen, bool overlap, double* out, int nthreads) {
  int lmax = 0;
  for (int s = 0; s < bs.n_shells; ++s) lmax = std::max(lmax, (int)bs.l[s]);
  Coupling<T> cp(lmax);
  std::vector<T> np(3 * n_nuc), nz(n_nuc);
  for (int i = 0; i < 3 * n_nuc; ++i) np[i] = T(nuc_pos[i]);
  for (int i = 0; i < n_nuc; ++i) nz[i] = T(nuc_Z[i]);
  std::vector<int64_t> off(n_pairs + 1, 0);
  for (int64_t i = 0; i < n_pairs; ++i)
    off[i + 1] = off[i] + (int64_t)(2 * bs.l[pa[i]] + 1) * (2 * bs.l[pb[i]] + 1);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_pairs; ++i) {
    ShellT<T> sa = make_shell<T>(bs, pa[i], nullptr), sb = make_shell<T>(bs, pb[i], nullptr);
    int da = 2 * sa.l + 1, db = 2 * sb.l + 1;
    std::vector<T> blk(da * db);
    shell_block<T>(sa, sb, n_nuc, np.data(), nz.data(), overlap, screen, cp, blk.data());
    for (int j = 0; j < da * db; ++j) out[off[i] + j] = val(blk[j]);
  }
  return 0;
}

// Gradient of E = sum_ij D_ij V_ij (V the full symmetric matrix) with respect to the nuclear
// positions and the shell centers, by forward-mode dual numbers (Eq. 11 differentiated through
// every step of the route, Boys included via dF_m/dT = -F_{m+1}). For each shell pair a <= b the
// pair's energy is sum D~ V_ab with D~ = D_ab + D_ba^T (a != b) or D_aa (a = b); each center
// coordinate is seeded in its own evaluation of the whole block, each nuclear coordinate in an
// evaluation of that nucleus's term only. The screening decision uses the plain values, so the
// surviving primitive pairs stay those of the reference geometry.
int grad_pairs(const Basis& bs, int n_nuc, const double* nuc_pos, const double* nuc_Z, const double* D, double screen,
               double* dnuc, double* dcen, double* energy, int nthreads) {
  int lmax = 0;
  for (int s = 0; s < bs.n_shells; ++s) lmax = std::max(lmax, (int)bs.l[s]);
  Coupling<Dual> cp(lmax);
  std::vector<int64_t> so(bs.n_shells + 1, 0);
  for (int s = 0; s < bs.n_shells; ++s) so[s + 1] = so[s] + 2 * bs.l[s] + 1;
  const int64_t nbf = so[bs.n_shells];
  std::vector<int32_t> pa, pb;
  for (int a = 0; a < bs.n_shells; ++a)
    for (int b = a; b < bs.n_shells; ++b) {
      pa.push_back(a);
      pb.push_back(b);
    }
  std::vector<Dual> npos(3 * n_nuc), nz(n_nuc);
  for (int i = 0; i < 3 * n_nuc; ++i) npos[i] = Dual(nuc_pos[i]);
  for (int i = 0; i < n_nuc; ++i) nz[i] = Dual(nuc_Z[i]);
  for (int i = 0; i < 3 * n_nuc; ++i) dnuc[i] = 0.0;
  for (int i = 0; i < 3 * bs.n_shells; ++i) dcen[i] = 0.0;
  double e_tot = 0.0;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
    std::vector<double> dn(3 * n_nuc, 0.0), dc(3 * bs.n_shells, 0.0);
    double e_loc = 0.0;
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < (int64_t)pa.size(); ++i) {
      const int a = pa[i], b = pb[i];
      const int da = 2 * bs.l[a] + 1, db = 2 * bs.l[b] + 1;
      std::vector<double> Dt(da * db);
      for (int x = 0; x < da; ++x)
        for (int y = 0; y < db; ++y)
          Dt[x * db + y] = D[(so[a] + x) * nbf + so[b] + y] + (a != b ? D[(so[b] + y) * nbf + so[a] + x] : 0.0);
      bool any = false;
      for (double v : Dt) any = any || v != 0.0;
      if (!any) continue;  // a zero density block contributes nothing to E or its gradient
      const ShellT<Dual> sa = make_shell<Dual>(bs, a, nullptr), sb = make_shell<Dual>(bs, b, nullptr);
      std::vector<Dual> blk(da * db);
      auto pair_energy = [&](const ShellT<Dual>& A, const ShellT<Dual>& B, int nn, const Dual* pos, const Dual* Z) {
        shell_block<Dual>(A, B, nn, pos, Z, false, screen, cp, blk.data());
        Dual e;
        for (int j = 0; j < da * db; ++j) e = e + Dual(Dt[j]) * blk[j];
        return e;
      };
      e_loc += pair_energy(sa, sb, n_nuc, npos.data(), nz.data()).v;
      for (int x = 0; x < 3; ++x) {
        ShellT<Dual> sa2 = sa, sb2 = sb;
        sa2.A[x].d = 1.0;
        if (a == b) sb2.A[x].d = 1.0;  // one shell: its center appears on both sides
        dc[3 * a + x] += pair_energy(sa2, sb2, n_nuc, npos.data(), nz.data()).d;
        if (a != b) {
          ShellT<Dual> sa3 = sa, sb3 = sb;
          sb3.A[x].d = 1.0;
          dc[3 * b + x] += pair_energy(sa3, sb3, n_nuc, npos.data(), nz.data()).d;
        }
      }
      for (int c = 0; c < n_nuc; ++c)
        for (int x = 0; x < 3; ++x) {
          Dual pc[3] = {npos[3 * c], npos[3 * c + 1], npos[3 * c + 2]};
          pc[x].d = 1.0;
          dn[3 * c + x] += pair_energy(sa, sb, 1, pc, &nz[c]).d;
        }
    }
#pragma omp critical
    {
      for (int j = 0; j < 3 * n_nuc; ++j) dnuc[j] += dn[j];
      for (int j = 0; j < 3 * bs.n_shells; ++j) dcen[j] += dc[j];
      e_tot += e_loc;
    }
  }
  if (energy) *energy = e_tot;
  return 0;
}

int check_basis(const Basis& bs) {
  for (int s = 0; s < bs.n_shells; ++s) {
    if (bs.l[s] < 0 || bs.l[s] > 8 || bs.nprim[s] < 1) return 1;
    for (int k = 0; k < bs.nprim[s]; ++k)
      if (!(bs.expo[bs.prim_off[s] + k] > 0)) return 1;
  }
  return 0;
}

}  // namespace

extern "C" {

// Boys function F_0..F_mmax at t. precision: 0 double, 1 long double, 2 __float128.
void oracle_boys(int precision, int mmax, double t, double* F) {
  if (precision == 0) {
    boys<double>(mmax, t, F);
  } else if (precision == 1) {
    std::vector<long double> f(mmax + 1);
    boys<long double>(mmax, (long double)t, f.data());
    for (int m = 0; m <= mmax; ++m) F[m] = (double)f[m];
  } else {
    std::vector<__float128> f(mmax + 1);
    boys<__float128>(mmax, (__float128)t, f.data());
    for (int m = 0; m <= mmax; ++m) F[m] = (double)f[m];
  }
}

// Complex solid harmonics Y^l_m for l <= lmax; out[2*(l*l+m+l)] = re, [+1] = im.
void oracle_solid_complex(int lmax, double x, double y, double z, double* out) {
  std::vector<Cx<double>> Y((lmax + 1) * (lmax + 1));
  solid_complex<double>(lmax, x, y, z, Y.data());
  for (size_t i = 0; i < Y.size(); ++i) {
    out[2 * i] = Y[i].re;
    out[2 * i + 1] = Y[i].im;
  }
}

// Real solid harmonics S^l_m for l <= lmax; out[l*l+m+l].
void oracle_solid_real(int lmax, double x, double y, double z, double* out) {
  std::vector<Cx<double>> Y((lmax + 1) * (lmax + 1));
  solid_complex<double>(lmax, x, y, z, Y.data());
  for (int l = 0; l <= lmax; ++l) {
    int d = 2 * l + 1;
    std::vector<Cx<double>> U(d * d);
    real_map<double>(l, U.data());
    for (int i = 0; i < d; ++i) {
      Cx<double> s;
      for (int j = 0; j < d; ++j) s = s + U[i * d + j] * Y[l * l + j];
      out[l * l + i] = s.re;
    }
  }
}

double oracle_cg(int j1, int m1, int j2, int m2, int J, int M) { return clebsch<double>(j1, m1, j2, m2, J, M); }
double oracle_eps(int l1, int l2, int m1, int m2) { return eps_coef<double>(l1, l2, m1, m2); }

// Shift matrix of Eq. 7 (sign-corrected), complex, (2la+1) x (la+1)^2 interleaved re/im.
void oracle_shift_matrix(int la, double s, const double* R, double* out) {
  int na = (la + 1) * (la + 1);
  std::vector<Cx<double>> S((2 * la + 1) * na);
  shift_matrix<double>(la, s, R[0], R[1], R[2], S.data());
  for (size_t i = 0; i < S.size(); ++i) {
    out[2 * i] = S[i].re;
    out[2 * i + 1] = S[i].im;
  }
}

// One-center Coulomb table I(l1 m1, l2 m2) for l1 <= la, l2 <= lb (complex, interleaved).
void oracle_one_center(int precision, int la, int lb, double p, const double* C, double* out) {
  int na = (la + 1) * (la + 1), nb = (lb + 1) * (lb + 1);
  int lm = std::max(la, lb);
  auto run = [&](auto tag) {
    using T = decltype(tag);
    Coupling<T> cp(lm);
    std::vector<Cx<T>> I(na * nb);
    one_center<T>(la, lb, T(p), T(C[0]), T(C[1]), T(C[2]), cp, I.data());
    for (int i = 0; i < na * nb; ++i) {
      out[2 * i] = val(I[i].re);
      out[2 * i + 1] = val(I[i].im);
    }
  };
  if (precision == 0) run(double());
  else if (precision == 1) run((long double)0);
  else run((__float128)0);
}

// Blocks of V (or of the overlap S when n_nuc < 0) for an explicit list of shell pairs.
// Block i is (2 l[pa[i]] + 1) x (2 l[pb[i]] + 1), row-major, stored back to back in pair order.
// Returns 0 on success, 1 on invalid basis.
int oracle_blocks(int precision, int n_shells, const double* center, const int32_t* l, const int32_t* nprim,
                  const int64_t* prim_off, const double* expo, const double* coef, int n_nuc,
                  const double* nuc_pos, const double* nuc_Z, int64_t n_pairs, const int32_t* pa,
                  const int32_t* pb, double screen, double* out, int nthreads) {
  Basis bs{n_shells, center, l, nprim, prim_off, expo, coef};
  if (check_basis(bs)) return 1;
  bool ovl = n_nuc < 0;
  int nn = ovl ? 0 : n_nuc;
  if (precision == 0)
    return run_blocks<double>(bs, nn, nuc_pos, nuc_Z, n_pairs, pa, pb, screen, ovl, out, nthreads);
  if (precision == 1)
    return run_blocks<long double>(bs, nn, nuc_pos, nuc_Z, n_pairs, pa, pb, screen, ovl, out, nthreads);
  return run_blocks<__float128>(bs, nn, nuc_pos, nuc_Z, n_pairs, pa, pb, screen, ovl, out, nthreads);
}

// Full symmetric matrix (nbf x nbf, row-major; basis index = shell offset + m + l).
int oracle_matrix(int precision, int n_shells, const double* center, const int32_t* l, const int32_t* nprim,
                  const int64_t* prim_off, const double* expo, const double* coef, int n_nuc,
                  const double* nuc_pos, const double* nuc_Z, double screen, double* V, int nthreads) {
  std::vector<int32_t> pa, pb;
  for (int a = 0; a < n_shells; ++a)
    for (int b = a; b < n_shells; ++b) {
      pa.push_back(a);
      pb.push_back(b);
    }
  std::vector<int64_t> boff(pa.size() + 1, 0);
  for (size_t i = 0; i < pa.size(); ++i) boff[i + 1] = boff[i] + (int64_t)(2 * l[pa[i]] + 1) * (2 * l[pb[i]] + 1);
  std::vector<double> blocks(boff.back());
  int rc = oracle_blocks(precision, n_shells, center, l, nprim, prim_off, expo, coef, n_nuc, nuc_pos, nuc_Z,
                         (int64_t)pa.size(), pa.data(), pb.data(), screen, blocks.data(), nthreads);
  if (rc) return rc;
  std::vector<int64_t> so(n_shells + 1, 0);
  for (int s = 0; s < n_shells; ++s) so[s + 1] = so[s] + 2 * l[s] + 1;
  int64_t nbf = so[n_shells];
  for (size_t i = 0; i < pa.size(); ++i) {
    int a = pa[i], b = pb[i], da = 2 * l[a] + 1, db = 2 * l[b] + 1;
    for (int x = 0; x < da; ++x)
      for (int y = 0; y < db; ++y) {
        double v = blocks[boff[i] + x * db + y];
        V[(so[a] + x) * nbf + so[b] + y] = v;
        V[(so[b] + y) * nbf + so[a] + x] = v;
      }
  }
  return 0;
}

// dE/d(nuclear positions) [n_nuc][3], dE/d(shell centers) [n_shells][3] and E itself for
// E = sum_ij D_ij V_ij, D an nbf x nbf row-major matrix. Returns 0, or 1 on an invalid basis.
int oracle_grad(int n_shells, const double* center, const int32_t* l, const int32_t* nprim, const int64_t* prim_off,
                const double* expo, const double* coef, int n_nuc, const double* nuc_pos, const double* nuc_Z,
                double screen, const double* D, double* dnuc, double* dcen, double* energy, int nthreads) {
  Basis bs{n_shells, center, l, nprim, prim_off, expo, coef};
  if (check_basis(bs)) return 1;
  return grad_pairs(bs, n_nuc, nuc_pos, nuc_Z, D, screen, dnuc, dcen, energy, nthreads);
}

}  // extern "C"
