// The oracle (oracle/shgo_oracle.cpp) under AddressSanitizer and UBSan: a small contracted molecule
// with every l up to 6, evaluated through each of its C entry points in every scalar type (double,
// long double, __float128), the overlap blocks, a screened evaluation and the dual-number gradient,
// with one and with several OpenMP threads. Exit status 0 when every result is finite and the
// matrix is symmetric; the sanitizers abort on any invalid access or undefined operation.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void oracle_boys(int precision, int mmax, double t, double* F);
int oracle_blocks(int precision, int n_shells, const double* center, const int32_t* l, const int32_t* nprim,
                  const int64_t* prim_off, const double* expo, const double* coef, int n_nuc, const double* nuc_pos,
                  const double* nuc_Z, int64_t n_pairs, const int32_t* pa, const int32_t* pb, double screen,
                  double* out, int nthreads);
int oracle_matrix(int precision, int n_shells, const double* center, const int32_t* l, const int32_t* nprim,
                  const int64_t* prim_off, const double* expo, const double* coef, int n_nuc, const double* nuc_pos,
                  const double* nuc_Z, double screen, double* V, int nthreads);
int oracle_grad(int n_shells, const double* center, const int32_t* l, const int32_t* nprim, const int64_t* prim_off,
                const double* expo, const double* coef, int n_nuc, const double* nuc_pos, const double* nuc_Z,
                double screen, const double* D, double* dnuc, double* dcen, double* energy, int nthreads);
}

static int fails = 0;
#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "failed at line %d: %s\n", __LINE__, #c); \
      ++fails;                                                        \
    }                                                                 \
  } while (0)

int main() {
  // seven shells l = 0..6 on three centers, K = 1..3 primitives, two nuclei (one on a center)
  const int ns = 7;
  std::vector<double> center = {0, 0, 0, 0, 0, 0, 1.1, -0.4, 0.7, 1.1, -0.4, 0.7, -0.8, 0.9, 0.3, 0, 0, 0, -0.8, 0.9, 0.3};
  std::vector<int32_t> l = {0, 1, 2, 3, 4, 5, 6}, nprim = {3, 2, 1, 2, 3, 1, 2};
  std::vector<int64_t> off(ns);
  std::vector<double> expo, coef;
  for (int s = 0; s < ns; ++s) {
    off[s] = (int64_t)expo.size();
    for (int k = 0; k < nprim[s]; ++k) {
      expo.push_back(0.3 + 1.7 * k + 0.11 * s);
      coef.push_back(0.4 + 0.2 * k);
    }
  }
  std::vector<double> npos = {0.2, 0.1, -0.3, 1.1, -0.4, 0.7}, nz = {3.0, 1.0};
  int nbf = 0;
  for (int s = 0; s < ns; ++s) nbf += 2 * l[s] + 1;
  double F[15];
  for (int p = 0; p < 3; ++p)
    for (double t : {0.0, 1e-9, 0.5, 17.0, 39.9, 40.1, 300.0}) {
      oracle_boys(p, 14, t, F);
      for (double f : F) EXPECT(std::isfinite(f) && f > 0);
    }
  for (int threads : {1, 3}) {
    std::vector<double> V((size_t)nbf * nbf, 0.0);
    EXPECT(oracle_matrix(0, ns, center.data(), l.data(), nprim.data(), off.data(), expo.data(), coef.data(), 2,
                         npos.data(), nz.data(), 0.0, V.data(), threads) == 0);
    for (int i = 0; i < nbf; ++i)
      for (int j = 0; j < nbf; ++j) EXPECT(std::isfinite(V[i * nbf + j]) && V[i * nbf + j] == V[j * nbf + i]);
    std::vector<int32_t> pa = {6, 0, 5, 3}, pb = {6, 6, 2, 3};
    int64_t sz = 0;
    for (size_t i = 0; i < pa.size(); ++i) sz += (int64_t)(2 * l[pa[i]] + 1) * (2 * l[pb[i]] + 1);
    for (int prec = 0; prec < 3; ++prec) {
      std::vector<double> out((size_t)sz, 0.0);
      EXPECT(oracle_blocks(prec, ns, center.data(), l.data(), nprim.data(), off.data(), expo.data(), coef.data(), 2,
                           npos.data(), nz.data(), (int64_t)pa.size(), pa.data(), pb.data(), 1e-3, out.data(),
                           threads) == 0);
      for (double v : out) EXPECT(std::isfinite(v));
      // overlap blocks (no nuclei)
      EXPECT(oracle_blocks(prec, ns, center.data(), l.data(), nprim.data(), off.data(), expo.data(), coef.data(), -1,
                           npos.data(), nz.data(), (int64_t)pa.size(), pa.data(), pb.data(), 0.0, out.data(),
                           threads) == 0);
      for (double v : out) EXPECT(std::isfinite(v));
    }
    std::vector<double> D((size_t)nbf * nbf), dn(6), dc(3 * ns), e(1);
    for (int i = 0; i < nbf; ++i)
      for (int j = 0; j < nbf; ++j) D[i * nbf + j] = std::sin(0.1 * (i + 1) * (j + 1));
    EXPECT(oracle_grad(ns, center.data(), l.data(), nprim.data(), off.data(), expo.data(), coef.data(), 2, npos.data(),
                       nz.data(), 1e-12, D.data(), dn.data(), dc.data(), e.data(), threads) == 0);
    for (double v : dn) EXPECT(std::isfinite(v));
    for (double v : dc) EXPECT(std::isfinite(v));
  }
  // an invalid basis is refused, not read out of bounds
  std::vector<int32_t> bad_l = l;
  bad_l[2] = -1;
  std::vector<double> V((size_t)nbf * nbf);
  EXPECT(oracle_matrix(0, ns, center.data(), bad_l.data(), nprim.data(), off.data(), expo.data(), coef.data(), 2,
                       npos.data(), nz.data(), 0.0, V.data(), 1) != 0);
  std::printf(fails ? "FAILED\n" : "ok\n");
  return fails ? 1 : 0;
}
