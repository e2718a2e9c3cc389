// Two-electron Coulomb integrals (ab|cd) on MI355X (gfx950) by the solid-harmonic route
// (Eqs. 13-15: the four-center integral reduced to a two-center one between the Gaussian
// products at P and Q, with solid-harmonic derivatives and the product rule).
//
// Each pair is worked as in the nuclear-attraction kernel: Gaussian product (Eq. 5), shifts to P
// in the pair frame (Eq. 7), product rule (Supplement Eq. 4), so that the pair's charge
// distribution of block entry (ma, mb) is sum_w B[(ma,mb)][w] |u|^{2k} S^L_M(u) e^{-p u^2},
// w = (L, M, k), u = r - P; B is rotated to the laboratory frame (W blocks and block rows, with the
// rotations of the integral kernel). Hobson's theorem turns S^L(u) e^{-p u^2} into
// (2p)^{-L} S^L(grad_P) e^{-p u^2}, and |u|^{2k} into sum_j gamma_{L,k,j} p^{-(k+j)} (grad_P^2)^j,
// so B becomes B' over w = (L, M, j). The two-center integral of two such terms is
//   I[w1][w2] = (-1)^{L2} sum_{L,M} g(L1 M1, L2 M2; L M) S^L_M(P - Q) h_{L, j1 + j2 + kappa},
//   h_{L,0} = c (-2 alpha)^L F_L(T),  h_{L,n>0} = c (-2 alpha)^L alpha^n P_{L,n}(T) e^{-T},
// c = 2 pi^{5/2} / (p q sqrt(p+q)), alpha = pq/(p+q), T = alpha |P - Q|^2, kappa = (L1+L2-L)/2,
// g the real Gaunt coefficients (the product rule applied to the gradients), and the primitive
// block is K_ab K_cd B'_bra I B'_ket^T.
//
// One wavefront per shell quartet, its lanes over the entries of the LDS matrices; shells up to
// l = kEriLmax. The tables come from gen_classes.py (generated/shgo_eri.inc).
#include "shgo_internal.h"

#include "generated/shgo_rot.inc"
#include "generated/shgo_eri.inc"

namespace shgo_impl {
namespace {

constexpr int kEriThreads = 256;
constexpr int kEriWavesPerGroup = kEriThreads / 64;
constexpr int kNabMax = (2 * kEriLmax + 1) * (2 * kEriLmax + 1);
constexpr int kNwMax = 35;  // W entries of the (2, 2) pair class
constexpr int kNS = (kEriLT + 1) * (kEriLT + 1);
constexpr int kNH = (kEriLT + 1) * (kEriNmax + 1);

struct EriLds {  // per-wavefront LDS, in doubles
  static constexpr int BB = 0;
  static constexpr int BK = BB + kNabMax * kNwMax;
  static constexpr int I = BK + kNabMax * kNwMax;
  static constexpr int T = I + kNwMax * kNwMax;
  static constexpr int ACC = T + kNabMax * kNwMax;
  static constexpr int SR = ACC + kNabMax * kNabMax;
  static constexpr int H = SR + kNS;
  static constexpr int F = H + kNH;
  static constexpr int SIZE = F + kEriLT + 2;
};

struct Angles {
  double cth[kEriLmax * 2 + 1], sth[kEriLmax * 2 + 1], cph[kEriLmax * 2 + 1], sph[kEriLmax * 2 + 1];
};

// v <- D^T v for the (2L+1)-vector at p[idx[i]] or p[i * stride]
template <int L>
__device__ __forceinline__ void rot_at(double* p, const int* idx, int stride, const Angles& an) {
  double v[2 * L + 1];
#pragma unroll
  for (int i = 0; i <= 2 * L; ++i) v[i] = p[idx ? idx[i] : i * stride];
  Rot<L>::apply(v, an.cth, an.sth, an.cph, an.sph);
#pragma unroll
  for (int i = 0; i <= 2 * L; ++i) p[idx ? idx[i] : i * stride] = v[i];
}
__device__ __forceinline__ void rot_dispatch(int L, double* p, const int* idx, int stride, const Angles& an) {
  static_assert(2 * kEriLmax == 4, "rot_dispatch covers L = 0..4");
  switch (L) {
    case 0: rot_at<0>(p, idx, stride, an); break;
    case 1: rot_at<1>(p, idx, stride, an); break;
    case 2: rot_at<2>(p, idx, stride, an); break;
    case 3: rot_at<3>(p, idx, stride, an); break;
    default: rot_at<4>(p, idx, stride, an); break;
  }
}

// Real solid harmonics S^L_M(x, y, z), L <= LM, by the sectoral and vertical recurrences
// (Racah normalisation), out[L L + M + L].
template <int LM>
__device__ void solid_harmonics(double x, double y, double z, double* out) {
  const double r2 = x * x + y * y + z * z;
  out[0] = 1.0;
  double sc = 1.0, ss = 0.0;
  for (int l = 0; l < LM; ++l) {
    const double f = l == 0 ? 1.0 : sqrt((2.0 * l + 1.0) / (2.0 * l + 2.0));
    const double nc = f * (x * sc - y * ss), ns = f * (y * sc + x * ss);
    sc = nc;
    ss = ns;
    out[(l + 1) * (l + 1) + 2 * (l + 1)] = sc;
    out[(l + 1) * (l + 1)] = ss;
  }
  for (int m = 0; m <= LM; ++m)
    for (int sg = 0; sg < (m == 0 ? 1 : 2); ++sg) {
      const int mm = sg == 0 ? m : -m;
      double prev = 0.0, cur = out[m * m + mm + m];
      for (int l = m; l < LM; ++l) {
        const double den = sqrt((double)((l + m + 1) * (l - m + 1)));
        const double a = (2.0 * l + 1.0) / den, b = sqrt((double)((l + m) * (l - m))) / den;
        const double nxt = a * z * cur - b * r2 * prev;
        out[(l + 1) * (l + 1) + mm + l + 1] = nxt;
        prev = cur;
        cur = nxt;
      }
    }
}

// B' of one primitive pair of class (LA, LB) (LA >= LB) into Bx [NA NB][NW]: coupling terms,
// rotation of the W blocks and of the block rows to the laboratory frame, then the gradient form.
__device__ void build_side(double* Bx, int cls, int LA, int LB, double ta, double tb, double p, const Angles& an,
                           int lane) {
  const int NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB, NW = kEriNW[cls], base = kEriEntBase[cls];
  for (int i = lane; i < NAB * NW; i += 64) Bx[i] = 0.0;
  wave_sync();
  const double tap[3] = {1.0, ta, ta * ta}, tbp[3] = {1.0, tb, tb * tb};
  for (int w = lane; w < NW; w += 64)
    for (int t = kEriTermOff[base + w]; t < kEriTermOff[base + w + 1]; ++t) {
      const EriTerm T = kEriTerm[t];
      Bx[T.e * NW + w] = fma(T.coef * tap[T.pa], tbp[T.pb], Bx[T.e * NW + w]);
    }
  wave_sync();
  const int b0 = kEriBlkBase[cls], nblk = kEriBlkBase[cls + 1] - b0;
  for (int it = lane; it < NAB * nblk; it += 64) {
    const int e = it / nblk, b = it - e * nblk;
    rot_dispatch(kEriBlk[b0 + b][0], Bx + e * NW, kEriBlkW + kEriBlk[b0 + b][2], 0, an);
  }
  wave_sync();
  for (int it = lane; it < NW * NA; it += 64) {
    const int w = it / NA, ma = it - w * NA;
    rot_dispatch(LB, Bx + ma * NB * NW + w, nullptr, NW, an);
  }
  wave_sync();
  for (int it = lane; it < NW * NB; it += 64) {
    const int w = it / NB, mb = it - w * NB;
    rot_dispatch(LA, Bx + mb * NW + w, nullptr, NB * NW, an);
  }
  wave_sync();
  const int g0 = kEriGrpBase[cls], ngrp = kEriGrpBase[cls + 1] - g0;
  const double ip = 1.0 / p;
  for (int it = lane; it < NAB * ngrp; it += 64) {
    const int e = it / ngrp, gi = it - e * ngrp;
    const int L = kEriGrp[g0 + gi][0], nk = kEriGrp[g0 + gi][1];
    const int* ws = kEriGrpW + kEriGrp[g0 + gi][2];
    double v[kEriLmax + 1];
    for (int k = 0; k < nk; ++k) v[k] = Bx[e * NW + ws[k]];
    double pl = 1.0;
    for (int i = 0; i < L; ++i) pl *= 0.5 * ip;  // (2p)^{-L}
    for (int j = 0; j < nk; ++j) {
      double s = 0.0, pk = 1.0;
      for (int i = 0; i < 2 * j; ++i) pk *= ip;  // p^{-(k+j)} from k = j
      for (int k = j; k < nk; ++k) {
        s = fma(kEriGamma[L][k][j] * pk, v[k], s);
        pk *= ip;
      }
      Bx[e * NW + ws[j]] = pl * s;
    }
  }
  wave_sync();
}

__global__ void __launch_bounds__(kEriThreads) k_eri(DevBasis bs, int64_t n_quartets, const int32_t* __restrict__ quartets,
                                                     const int64_t* __restrict__ offsets,
                                                     const double* __restrict__ boys_tab, double* __restrict__ out) {
  __shared__ double s_lds[kEriWavesPerGroup * EriLds::SIZE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* const sm = s_lds + wave * EriLds::SIZE;
  const int64_t nw_total = (int64_t)gridDim.x * kEriWavesPerGroup;
  for (int64_t q = (int64_t)blockIdx.x * kEriWavesPerGroup + wave; q < n_quartets; q += nw_total) {
    int s[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s[i] = quartets[4 * q + i];
      l[i] = bs.l[s[i]];
    }
    // pair classes (higher l first) and whether each listed pair is swapped
    const bool swb = l[0] < l[1], swk = l[2] < l[3];
    const int sa = swb ? s[1] : s[0], sb = swb ? s[0] : s[1], sc = swk ? s[3] : s[2], sd = swk ? s[2] : s[3];
    const int LA = bs.l[sa], LB = bs.l[sb], LC = bs.l[sc], LD = bs.l[sd];
    const int cb = class_id(LA, LB), ck = class_id(LC, LD);
    const int NB = 2 * LB + 1, ND = 2 * LD + 1, NAB = (2 * LA + 1) * NB, NCD = (2 * LC + 1) * ND;
    const int NW1 = kEriNW[cb], NW2 = kEriNW[ck], base1 = kEriEntBase[cb], base2 = kEriEntBase[ck];
    PairState pb, pk;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      pb.A[x] = bs.center[3 * sa + x];
      pb.B[x] = bs.center[3 * sb + x];
      pk.A[x] = bs.center[3 * sc + x];
      pk.B[x] = bs.center[3 * sd + x];
    }
    frame_of(pb);
    frame_of(pk);
    Angles anb, ank;
    angles<2 * kEriLmax>(pb.ct, pb.st, anb.cth, anb.sth);
    angles<2 * kEriLmax>(pb.cp, pb.sp, anb.cph, anb.sph);
    angles<2 * kEriLmax>(pk.ct, pk.st, ank.cth, ank.sth);
    angles<2 * kEriLmax>(pk.cp, pk.sp, ank.cph, ank.sph);
    for (int i = lane; i < NAB * NCD; i += 64) sm[EriLds::ACC + i] = 0.0;
    const int64_t oa = bs.prim_off[sa], ob = bs.prim_off[sb], oc = bs.prim_off[sc], od = bs.prim_off[sd];
    const int Ka = bs.nprim[sa], Kb = bs.nprim[sb], Kc = bs.nprim[sc], Kd = bs.nprim[sd];
    const int LT = LA + LB + LC + LD;
    for (int i = 0; i < Ka; ++i)
      for (int j = 0; j < Kb; ++j) {
        const double a = bs.expo[oa + i], b = bs.expo[ob + j], p = a + b, ip = 1.0 / p;
        double P[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) P[x] = (a * pb.A[x] + b * pb.B[x]) * ip;
        const double Kab = exp_neg(a * b * ip * pb.R * pb.R) * bs.w[oa + i] * bs.w[ob + j];
        build_side(sm + EriLds::BB, cb, LA, LB, b * pb.R * ip, -a * pb.R * ip, p, anb, lane);
        for (int k = 0; k < Kc; ++k)
          for (int m = 0; m < Kd; ++m) {
            const double c = bs.expo[oc + k], d = bs.expo[od + m], qq = c + d, iq = 1.0 / qq;
            double R[3];
#pragma unroll
            for (int x = 0; x < 3; ++x) R[x] = P[x] - (c * pk.A[x] + d * pk.B[x]) * iq;
            const double Kcd = exp_neg(c * d * iq * pk.R * pk.R) * bs.w[oc + k] * bs.w[od + m];
            build_side(sm + EriLds::BK, ck, LC, LD, d * pk.R * iq, -c * pk.R * iq, qq, ank, lane);
            const double alpha = p * qq / (p + qq);
            const double T = alpha * (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
            const double cpre = 2.0 * 17.493418327624862846 * ip * iq / sqrt(p + qq);  // 2 pi^{5/2} / (p q sqrt(p+q))
            if (lane == 0) {
              double row[kBoysRowLoad];
              const double* __restrict__ r = boys_row_ptr(boys_tab, kEriLT, boys_index(T));
#pragma unroll
              for (int u = 0; u < kBoysRowLoad; ++u) row[u] = r[u];
              double F[kEriLT + 1];
              boys_row<kEriLT>(T, row, F);
#pragma unroll
              for (int u = 0; u <= kEriLT; ++u) sm[EriLds::F + u] = F[u];
              sm[EriLds::F + kEriLT + 1] = exp_neg(T);
              solid_harmonics<kEriLT>(R[0], R[1], R[2], sm + EriLds::SR);
            }
            wave_sync();
            // h[L][n] for L <= LT and the orders n the quartet reaches (at most LT / 2 + LA... <= kEriNmax)
            for (int it = lane; it < (LT + 1) * (kEriNmax + 1); it += 64) {
              const int L = it / (kEriNmax + 1), n = it - L * (kEriNmax + 1);
              double base = cpre;
              for (int u = 0; u < L; ++u) base *= -2.0 * alpha;
              double v;
              if (n == 0) {
                v = sm[EriLds::F + L];
              } else {
                double poly = 0.0;
                for (int u = n - 1; u >= 0; --u) poly = fma(poly, T, kEriP[L][n][u]);
                double an = 1.0;
                for (int u = 0; u < n; ++u) an *= alpha;
                v = an * poly * sm[EriLds::F + kEriLT + 1];
              }
              sm[EriLds::H + it] = base * v;
            }
            wave_sync();
            // two-center matrix I[w1][w2]
            for (int it = lane; it < NW1 * NW2; it += 64) {
              const int w1 = it / NW2, w2 = it - w1 * NW2;
              const int L1 = kEriEnt[base1 + w1][0], M1 = kEriEnt[base1 + w1][1], j1 = kEriEnt[base1 + w1][2];
              const int L2 = kEriEnt[base2 + w2][0], M2 = kEriEnt[base2 + w2][1], j2 = kEriEnt[base2 + w2][2];
              const int i12 = (L1 * L1 + M1 + L1) * (kEriL12 + 1) * (kEriL12 + 1) + L2 * L2 + M2 + L2;
              double sacc = 0.0;
              for (int t = kEriGOff[i12]; t < kEriGOff[i12 + 1]; ++t) {
                const EriGaunt G = kEriG[t];
                int L = 0;
                while ((L + 1) * (L + 1) <= G.I) ++L;
                const int n = j1 + j2 + (L1 + L2 - L) / 2;
                sacc = fma(G.g * sm[EriLds::SR + G.I], sm[EriLds::H + L * (kEriNmax + 1) + n], sacc);
              }
              sm[EriLds::I + it] = (L2 & 1) ? -sacc : sacc;
            }
            wave_sync();
            // T = B'_bra I, then ACC += K_ab K_cd T B'_ket^T
            for (int it = lane; it < NAB * NW2; it += 64) {
              const int e1 = it / NW2, w2 = it - e1 * NW2;
              double sacc = 0.0;
              for (int w1 = 0; w1 < NW1; ++w1)
                sacc = fma(sm[EriLds::BB + e1 * NW1 + w1], sm[EriLds::I + w1 * NW2 + w2], sacc);
              sm[EriLds::T + it] = sacc;
            }
            wave_sync();
            const double pre = Kab * Kcd;
            for (int it = lane; it < NAB * NCD; it += 64) {
              const int e1 = it / NCD, e2 = it - e1 * NCD;
              double sacc = 0.0;
              for (int w2 = 0; w2 < NW2; ++w2)
                sacc = fma(sm[EriLds::T + e1 * NW2 + w2], sm[EriLds::BK + e2 * NW2 + w2], sacc);
              sm[EriLds::ACC + it] = fma(pre, sacc, sm[EriLds::ACC + it]);
            }
            wave_sync();
          }
      }
    // the block in the listed order: entry ((i0 N1 + i1) N2 + i2) N3 + i3
    const int N1 = 2 * l[1] + 1, N2 = 2 * l[2] + 1, N3 = 2 * l[3] + 1;
    const int64_t o = offsets[q];
    for (int it = lane; it < NAB * NCD; it += 64) {
      const int e1 = it / NCD, e2 = it - e1 * NCD;
      const int ma = e1 / NB, mb = e1 - ma * NB, mc = e2 / ND, md = e2 - mc * ND;
      const int i0 = swb ? mb : ma, i1 = swb ? ma : mb, i2 = swk ? md : mc, i3 = swk ? mc : md;
      out[o + ((int64_t)(i0 * N1 + i1) * N2 + i2) * N3 + i3] = sm[EriLds::ACC + it];
    }
    wave_sync();
  }
}

}  // namespace

int eri_lmax() { return kEriLmax; }

hipError_t launch_eri(const shgo_plan* p, int64_t n_quartets, const int32_t* quartets, const int64_t* offsets,
                      double* out, hipStream_t st) {
  if (n_quartets <= 0) return hipSuccess;
  const int64_t need = (n_quartets + kEriWavesPerGroup - 1) / kEriWavesPerGroup;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)4 * p->ctx->n_cu));
  hipLaunchKernelGGL(k_eri, dim3(blocks), dim3(kEriThreads), 0, st, p->bs, n_quartets, quartets, offsets,
                     p->ctx->boys_tab, out);
  return hipGetLastError();
}

}  // namespace shgo_impl
