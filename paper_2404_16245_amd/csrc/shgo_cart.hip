// The Cartesian route to the same V on MI355X (gfx950): McMurchie-Davidson over Cartesian
// Gaussians, then the Cartesian-to-real-harmonic transform -- the textbook method the paper sets
// its solid-harmonic route against (Table 1, Cartesian column), run on the same GPU for a
// like-for-like comparison. It reads the plan's class-sorted pairs, normalised primitive weights
// and screening like the integral kernel, and writes V in the same layout.
//
// Per primitive pair (p, P, mu) of a shell pair:
//   V_cart(a, b) = -(2 pi / p) e^{-mu R^2} sum_c Z_c sum_tuv E^x_t E^y_u E^z_v R_tuv(p, P - c),
// with the Hermite expansion coefficients E of the two Cartesian factors about P and the Hermite
// Coulomb integrals R_tuv = d^t/dX^t d^u/dY^u d^v/dZ^v F_0(p |P - c|^2). The nucleus sum is taken
// first, W_tuv = sum_c Z_c R_tuv, so that the contraction with E runs once per primitive pair.
// Then V(ma, mb) += w_a w_b sum C_a[ma][qa] C_b[mb][qb] V_cart(qa, qb), C the coefficients of the
// real solid harmonics S^l_m over the Cartesian monomials.
//
// One wavefront per shell pair: its lanes take the nuclei (each lane a partial W in registers),
// the partial sums are reduced through LDS, and the lanes then share the contraction and the
// transform. One kernel per (la, lb) class, la, lb <= kCartLmax.
#include "shgo_internal.h"

#include "generated/shgo_cart.inc"

namespace shgo_impl {
namespace {

constexpr int kCartThreads = 256;
constexpr int kCartWavesPerGroup = kCartThreads / 64;
constexpr int kRedChunk = 16;  // W entries reduced per pass through LDS

SHGO_HD constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

template <int LA, int LB>
struct CartLds {  // per-wavefront LDS, in doubles
  static constexpr int L = LA + LB, NT = CartR<L>::NT, NA = 2 * LA + 1, NB = 2 * LB + 1;
  static constexpr int NCA = ncart(LA), NCB = ncart(LB);
  static constexpr int NE = (LA + 1) * (LB + 1) * (L + 1);  // per dimension
  static constexpr int W = 0;
  static constexpr int E = W + NT;
  static constexpr int VC = E + 3 * NE;
  static constexpr int T1 = VC + NCA * NCB;
  static constexpr int ACC = T1 + NA * NCB;
  static constexpr int RED = ACC + NA * NB;
  static constexpr int SIZE = RED + 64 * kRedChunk;
};

// Registers of the partial W decide the occupancy: two waves per SIMD up to L = 4 (35 entries),
// one above (84 to 165 entries).
template <int L>
struct CartWaves {
  static constexpr int value = L <= 4 ? 2 : 1;
};

// Cartesian monomial q of degree l (cart_monomials order): s = j + k, q = s(s+1)/2 + k.
__device__ __forceinline__ void cart_exps(int l, int q, int& i, int& j, int& k) {
  int s = 0;
  while ((s + 1) * (s + 2) / 2 <= q) ++s;
  k = q - s * (s + 1) / 2;
  j = s - k;
  i = l - s;
}
// Hermite index of (t, u, v) (tuv_list order).
__device__ __forceinline__ int tuv_index(int t, int u, int v) {
  const int N = t + u + v, s = u + v;
  return N * (N + 1) * (N + 2) / 6 + s * (s + 1) / 2 + v;
}

// The real-harmonic coefficients of degree l, row-major [2l+1][ncart(l)].
template <int l>
__device__ __forceinline__ const double* cart_table() {
  static_assert(l <= kCartLmax && kCartLmax == 4, "cart_table lists the coefficient tables of l = 0..4");
  if constexpr (l == 0) return &kCartSph0[0][0];
  else if constexpr (l == 1) return &kCartSph1[0][0];
  else if constexpr (l == 2) return &kCartSph2[0][0];
  else if constexpr (l == 3) return &kCartSph3[0][0];
  else return &kCartSph4[0][0];
}

template <int LA, int LB>
__global__ void __launch_bounds__(kCartThreads) __attribute__((amdgpu_waves_per_eu(CartWaves<LA + LB>::value)))
k_cart(DevBasis bs, DevPairs pr, const Nuc* __restrict__ nucs, int n_nuc, const double* __restrict__ boys_tab,
       double* __restrict__ out) {
  using LY = CartLds<LA, LB>;
  const double* __restrict__ Ca = cart_table<LA>();
  const double* __restrict__ Cb = cart_table<LB>();
  constexpr int L = LY::L, NT = LY::NT, NA = LY::NA, NB = LY::NB, NCA = LY::NCA, NCB = LY::NCB, NE = LY::NE;
  __shared__ double s_lds[kCartWavesPerGroup * LY::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* const sm = s_lds + wave * LY::SIZE;
  constexpr int cls = class_id(LA, LB);
  const int start = pr.key_off[cls * kKeysPerClass], end = pr.key_off[(cls + 1) * kKeysPerClass];
  const int nwaves = gridDim.x * kCartWavesPerGroup;
  for (int slot = start + blockIdx.x * kCartWavesPerGroup + wave; slot < end; slot += nwaves) {
    const int s1 = pr.s1[slot], s2 = pr.s2[slot];
    double A[3], B[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      A[x] = bs.center[3 * s1 + x];
      B[x] = bs.center[3 * s2 + x];
    }
    const double R2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    for (int e = lane; e < NA * NB; e += 64) sm[LY::ACC + e] = 0.0;
    const int64_t o1 = bs.prim_off[s1], o2 = bs.prim_off[s2];
    const int K1 = bs.nprim[s1], K2 = bs.nprim[s2];
    for (int pi = 0; pi < K1; ++pi)
      for (int pj = 0; pj < K2; ++pj) {
        const double a = bs.expo[o1 + pi], b = bs.expo[o2 + pj];
        if (!keep_prim(a, b, R2, pr.screen)) continue;
        const double p = a + b, ip = 1.0 / p;
        const double P[3] = {(a * A[0] + b * B[0]) * ip, (a * A[1] + b * B[1]) * ip, (a * A[2] + b * B[2]) * ip};
        // W_tuv partial over this lane's nuclei
        double Wp[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) Wp[k] = 0.0;
        for (int c = lane; c < n_nuc; c += 64) {
          const Nuc nc = nucs[c];
          const double X = P[0] - nc.x, Y = P[1] - nc.y, Z = P[2] - nc.z;
          const double T = p * fma(X, X, fma(Y, Y, Z * Z));
          double row[kBoysRowLoad];
          {
            const double* __restrict__ r = boys_row_ptr(boys_tab, L, boys_index(T));
#pragma unroll
            for (int k = 0; k < kBoysRowLoad; ++k) row[k] = r[k];
          }
          double F[L + 1];
          boys_row<L>(T, row, F);
          double g[L + 1];
          double m2p = 1.0;
#pragma unroll
          for (int n = 0; n <= L; ++n) {
            g[n] = m2p * F[n];
            m2p *= -2.0 * p;
          }
          CartR<L>::step(Wp, X, Y, Z, nc.Z, g);
        }
        // reduce the 64 partials of each entry: chunks of kRedChunk entries through LDS, lane
        // (quarter q, entry e) summing 16 lanes' values, then the four quarters by shuffles
        double* const red = sm + LY::RED;
#pragma unroll
        for (int k0 = 0; k0 < NT; k0 += kRedChunk) {
#pragma unroll
          for (int e = 0; e < kRedChunk; ++e)
            if (k0 + e < NT) red[e * 64 + lane] = Wp[k0 + e];
          wave_sync();
          const int e = lane & (kRedChunk - 1), q = lane >> 4;
          double s = 0.0;
#pragma unroll
          for (int r = 0; r < 16; ++r) s += red[e * 64 + q * 16 + r];
          s += __shfl_xor(s, 16);
          s += __shfl_xor(s, 32);
          if (q == 0 && k0 + e < NT) sm[LY::W + k0 + e] = s;
          wave_sync();
        }
        // Hermite expansion coefficients E^{i j}_t of each dimension (lanes 0..2), without e^{-mu R^2}
        if (lane < 3) {
          const double Pd = lane == 0 ? P[0] : lane == 1 ? P[1] : P[2];
          const double xa = Pd - (lane == 0 ? A[0] : lane == 1 ? A[1] : A[2]);
          const double xb = Pd - (lane == 0 ? B[0] : lane == 1 ? B[1] : B[2]), h = 0.5 * ip;
          double* const E = sm + LY::E + lane * NE;
          auto at = [&](int i, int j, int t) -> double& { return E[(i * (LB + 1) + j) * (L + 1) + t]; };
          for (int k = 0; k < NE; ++k) E[k] = 0.0;
          at(0, 0, 0) = 1.0;
          for (int i = 0; i <= LA; ++i)
            for (int j = 0; j <= LB; ++j) {
              if (i == 0 && j == 0) continue;
              const bool up_i = i > 0;
              const int pi2 = up_i ? i - 1 : i, pj2 = up_i ? j : j - 1;
              const double x = up_i ? xa : xb;
              const int tmax = i + j;
              for (int t = 0; t <= tmax; ++t) {
                double v = x * at(pi2, pj2, t);
                if (t > 0) v = fma(h, at(pi2, pj2, t - 1), v);
                if (t + 1 <= tmax - 1) v = fma((double)(t + 1), at(pi2, pj2, t + 1), v);
                at(i, j, t) = v;
              }
            }
        }
        wave_sync();
        // V_cart(qa, qb) = sum_tuv E^x E^y E^z W_tuv, lanes over the Cartesian pairs
        for (int q = lane; q < NCA * NCB; q += 64) {
          const int qa = q / NCB, qb = q - qa * NCB;
          int ia, ja, ka, ib, jb, kb;
          cart_exps(LA, qa, ia, ja, ka);
          cart_exps(LB, qb, ib, jb, kb);
          const double* Ex = sm + LY::E + (ia * (LB + 1) + ib) * (L + 1);
          const double* Ey = sm + LY::E + NE + (ja * (LB + 1) + jb) * (L + 1);
          const double* Ez = sm + LY::E + 2 * NE + (ka * (LB + 1) + kb) * (L + 1);
          double s = 0.0;
          for (int t = 0; t <= ia + ib; ++t)
            for (int u = 0; u <= ja + jb; ++u) {
              const double exy = Ex[t] * Ey[u];
              double sz = 0.0;
              for (int v = 0; v <= ka + kb; ++v) sz = fma(Ez[v], sm[LY::W + tuv_index(t, u, v)], sz);
              s = fma(exy, sz, s);
            }
          sm[LY::VC + q] = s;
        }
        wave_sync();
        // to the real harmonics: T1 = C_a V_cart, then acc += pre T1 C_b^T
        for (int q = lane; q < NA * NCB; q += 64) {
          const int ma = q / NCB, qb = q - ma * NCB;
          double s = 0.0;
          for (int qa = 0; qa < NCA; ++qa) s = fma(Ca[ma * NCA + qa], sm[LY::VC + qa * NCB + qb], s);
          sm[LY::T1 + q] = s;
        }
        wave_sync();
        const double pre = -6.283185307179586477 * ip * exp_neg(a * b * ip * R2) * bs.w[o1 + pi] * bs.w[o2 + pj];
        for (int e = lane; e < NA * NB; e += 64) {
          const int ma = e / NB, mb = e - ma * NB;
          double s = 0.0;
          for (int qb = 0; qb < NCB; ++qb) s = fma(sm[LY::T1 + ma * NCB + qb], Cb[mb * NCB + qb], s);
          sm[LY::ACC + e] = fma(pre, s, sm[LY::ACC + e]);
        }
        wave_sync();
      }
    // the block into V, as the integral kernel writes it
    const int64_t d0 = pr.dst0[slot], d1 = pr.dst1[slot];
    if (pr.full) {
      const int64_t n = bs.nbf;
      for (int pass = 0; pass < 2; ++pass)
        for (int e = lane; e < NA * NB; e += 64) {
          int i, col;
          if (pass == 0) {
            i = e / NB;
            col = e - i * NB;
          } else {
            col = e / NA;
            i = e - col * NA;
          }
          const int64_t o = out_index_matrix(pass, d0, d1, i, col, n);
          if (o >= 0) out[o] = sm[LY::ACC + i * NB + col];
        }
    } else {
      for (int e = lane; e < NA * NB; e += 64) out[d0 + e] = sm[LY::ACC + list_source_entry(e, d1 != 0, NA, NB)];
    }
    wave_sync();
  }
}

template <int LA, int LB>
hipError_t cart_class(const shgo_plan* p, double* out, hipStream_t st) {
  const int c = class_id(LA, LB);
  if (p->class_cand[c] == 0) return hipSuccess;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cart<LA, LB>, kCartThreads, 0) !=
      hipSuccess)
    per_cu = 1;
  const int64_t need = (p->class_cand[c] + kCartWavesPerGroup - 1) / kCartWavesPerGroup;
  // eight rounds of resident workgroups, which the hardware balances over the pairs' uneven costs
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)8 * std::max(1, per_cu) * p->ctx->n_cu));
  hipLaunchKernelGGL((k_cart<LA, LB>), dim3(blocks), dim3(kCartThreads), 0, st, p->bs, p->pr, p->nuc, p->n_nuc,
                     p->ctx->boys_tab, out);
  return hipGetLastError();
}

template <int LA, int LB>
hipError_t cart_all(const shgo_plan* p, double* out, hipStream_t st) {
  if constexpr (LA <= kCartLmax) {
    const hipError_t e = cart_class<LA, LB>(p, out, st);
    if (e != hipSuccess) return e;
    if constexpr (LB < LA)
      return cart_all<LA, LB + 1>(p, out, st);
    else
      return cart_all<LA + 1, 0>(p, out, st);
  }
  return hipSuccess;
}

}  // namespace

int cart_lmax() { return kCartLmax; }

hipError_t launch_cartesian(const shgo_plan* p, double* out, hipStream_t st) { return cart_all<0, 0>(p, out, st); }

}  // namespace shgo_impl
