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
// k_eri_pairs: one wavefront per distinct shell pair of the quartet list builds B' of each of its
// primitive pairs once (with p, P and K_ab) into a workspace of pair records. k_eri: one wavefront
// per shell quartet, its lanes over the entries of the LDS matrices, reads the two pairs' records
// and forms the two-center matrix and its product with the ket per primitive quartet, the bra's
// product once per bra primitive pair; it runs as two instances sized for their quartets'
// matrices (pairs up to (2,1), and the rest), each over its quartets costliest first. Shells up to l = kEriLmax. The tables come from gen_classes.py
// (generated/shgo_eri.inc).
#include "shgo_internal.h"

#include "generated/shgo_rot.inc"
#include "generated/shgo_eri.inc"

#include <algorithm>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace shgo_impl {
namespace {

constexpr int kEriThreads = 256;
constexpr int kEriWavesPerGroup = kEriThreads / 64;
constexpr int kNabMax = (2 * kEriLmax + 1) * (2 * kEriLmax + 1);
constexpr int kNwMax = kEriNwMax;
constexpr int kNS = (kEriLT + 1) * (kEriLT + 1);
constexpr int kNH = (kEriLT + 1) * (kEriNmax + 1);
constexpr int kEriHdr = 8;                                   // p, P (3), K_ab w_a w_b, padding
// the small instance of k_eri: pair classes up to (2,1), NAB <= 15 and NW <= 20
constexpr int kNabSmall = 15, kNwSmall = 20;
static_assert(kEriGTerms <= 4096 && kEriGmax < 32, "Gaunt list offsets take 12 bits, counts 5");
static_assert(kNS <= 256 && kNH <= 256, "Gaunt term indices take 8 bits each");

// The largest la + lb of a pair class with at most nabm block entries and shells up to kEriLmax.
__host__ __device__ constexpr int eri_max_lsum(int nabm) {
  int best = 0;
  for (int la = 0; la <= kEriLmax; ++la)
    for (int lb = 0; lb <= la; ++lb)
      if ((2 * la + 1) * (2 * lb + 1) <= nabm && la + lb > best) best = la + lb;
  return best;
}

// Per-wavefront LDS of k_eri for blocks of at most NABM entries and NWM two-center entries, in
// doubles: the bra's and the ket's B' of the current primitive pairs, the two-center matrix I
// (after a bra primitive pair's kets, Y^T [NCD][NW1]), the Boys values and solid harmonics of
// kSlots primitive quartets (one slot each: F_0..F_LTM, e^{-T}, then S^L_M for L <= LTM), and the
// h table. The 2 x 2 tiles may read past a ragged last row or column without keeping the result:
// each of BB, BK and I is followed by at least NWM doubles, and Y^T's reads stay inside I and the
// slots.
template <int NABM, int NWM>
struct EriLds {
  static constexpr int LTM = 2 * eri_max_lsum(NABM);         // the largest LA + LB + LC + LD
  static constexpr int kFS = LTM + 2;                        // F_0..F_LTM and e^{-T}
  static constexpr int kSlot = kFS + (LTM + 1) * (LTM + 1);  // and the solid harmonics
  static constexpr int kSlots = NABM * NWM / kSlot;
  static constexpr int BB = 0;
  static constexpr int BK = BB + NABM * NWM;
  static constexpr int I = BK + NABM * NWM;
  static constexpr int STG = I + NWM * NWM;
  static constexpr int H = STG + kSlots * kSlot;
  static constexpr int SIZE = H + kNH;
  static constexpr int kAccPerLane = (((NABM + 1) / 2) * ((NABM + 1) / 2) + 63) / 64;  // 2 x 2 block tiles per lane
  static constexpr int kIPerLane = (NWM * NWM + 63) / 64;                               // two-center entries per lane
  static constexpr int kYPerLane = (((NWM + 1) / 2) * ((NABM + 1) / 2) + 63) / 64;    // 2 x 2 tiles of Y per lane
  static_assert(kSlots >= 1 && kSlots <= 64 && kSlots * kSlot >= NWM, "room after I for the tiles' reads");
  static_assert((NABM + 1) * NWM <= NWM * NWM + kSlots * kSlot, "Y^T's tiles read inside I and the slots");
  static_assert(kNH >= 1 && LTM <= kEriLT, "the h table and the Boys orders");
};

// The distinct pairs of a quartet list and each quartet's pairs; every pointer is device memory.
struct EriWork {
  int64_t n_pairs, n_quartets;
  const int32_t* pairs;     // [n_pairs][2] shells (a, b) of each pair, l_a >= l_b
  const int64_t* pair_off;  // [n_pairs] first double of the pair's records in rec
  const int32_t* quart;     // [n_quartets][4] bra pair, ket pair, swaps (1: bra, 2: ket), unused
  const int64_t* out_off;   // [n_quartets] first double of the quartet's block in out
  double* rec;              // per primitive pair i Kb + j: kEriHdr doubles, then B' [NAB][NW]
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
// (Racah normalisation), out[L L + M + L]; unrolled, so that the coefficients are constants.
template <int LM>
__device__ __forceinline__ void solid_harmonics(double x, double y, double z, double* out) {
  const double r2 = x * x + y * y + z * z;
  out[0] = 1.0;
  double sc = 1.0, ss = 0.0;
#pragma unroll
  for (int l = 0; l < LM; ++l) {
    const double f = l == 0 ? 1.0 : sqrt((2.0 * l + 1.0) / (2.0 * l + 2.0));
    const double nc = f * (x * sc - y * ss), ns = f * (y * sc + x * ss);
    sc = nc;
    ss = ns;
    out[(l + 1) * (l + 1) + 2 * (l + 1)] = sc;
    out[(l + 1) * (l + 1)] = ss;
  }
#pragma unroll
  for (int m = 0; m <= LM; ++m)
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      if (m == 0 && sg == 1) continue;
      const int mm = sg == 0 ? m : -m;
      double prev = 0.0, cur = out[m * m + mm + m];
#pragma unroll
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

// F_0..F_LT(T) into fb, e^{-T} into *fexp and S^L_M(R), L <= LT, into sr (the lane's slot)
template <int LT>
__device__ __forceinline__ void boys_and_harmonics(double T, const double* R, const double* __restrict__ boys_tab,
                                                   double* fb, double* fexp, double* sr) {
  double row[kBoysRowLoad];
  const double* __restrict__ r = boys_row_ptr(boys_tab, LT, boys_index(T));
#pragma unroll
  for (int u = 0; u < kBoysRowLoad; ++u) row[u] = r[u];
  double F[LT + 1];
  boys_row<LT>(T, row, F);
#pragma unroll
  for (int u = 0; u <= LT; ++u) fb[u] = F[u];
  *fexp = exp_neg(T);
  solid_harmonics<LT>(R[0], R[1], R[2], sr);
}
// LT = LA + LB + LC + LD up to LTMAX (the instance's largest quartet)
template <int LTMAX>
__device__ void boys_and_harmonics_lt(int LT, double T, const double* R, const double* __restrict__ boys_tab, double* fb,
                                      double* fexp, double* sr) {
  static_assert(LTMAX <= kEriLT && kEriLT == 8, "the dispatch covers LT = 0..8");
  switch (LT < LTMAX ? LT : LTMAX) {
    case 0: boys_and_harmonics<0>(T, R, boys_tab, fb, fexp, sr); break;
    case 1: boys_and_harmonics<1>(T, R, boys_tab, fb, fexp, sr); break;
    case 2: boys_and_harmonics<2>(T, R, boys_tab, fb, fexp, sr); break;
    case 3: boys_and_harmonics<3>(T, R, boys_tab, fb, fexp, sr); break;
    case 4: boys_and_harmonics<4>(T, R, boys_tab, fb, fexp, sr); break;
    case 5: boys_and_harmonics<5>(T, R, boys_tab, fb, fexp, sr); break;
    case 6: boys_and_harmonics<6>(T, R, boys_tab, fb, fexp, sr); break;
    case 7: if constexpr (LTMAX >= 7) boys_and_harmonics<7>(T, R, boys_tab, fb, fexp, sr); break;
    default: if constexpr (LTMAX >= 8) boys_and_harmonics<8>(T, R, boys_tab, fb, fexp, sr); break;
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

// One wavefront per distinct pair: B' of each primitive pair, in the pair's records.
__global__ void __launch_bounds__(kEriThreads) k_eri_pairs(DevBasis bs, EriWork wk) {
  __shared__ double s_bx[kEriWavesPerGroup][kNabMax * kNwMax];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* const bx = s_bx[wave];
  for (int64_t u = (int64_t)blockIdx.x * kEriWavesPerGroup + wave; u < wk.n_pairs;
       u += (int64_t)gridDim.x * kEriWavesPerGroup) {
    const int sa = wk.pairs[2 * u], sb = wk.pairs[2 * u + 1];
    const int LA = bs.l[sa], LB = bs.l[sb], cls = class_id(LA, LB);
    const int n = (2 * LA + 1) * (2 * LB + 1) * kEriNW[cls], stride = kEriHdr + n;
    PairState ps;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      ps.A[x] = bs.center[3 * sa + x];
      ps.B[x] = bs.center[3 * sb + x];
    }
    frame_of(ps);
    Angles an;
    angles<2 * kEriLmax>(ps.ct, ps.st, an.cth, an.sth);
    angles<2 * kEriLmax>(ps.cp, ps.sp, an.cph, an.sph);
    const int64_t oa = bs.prim_off[sa], ob = bs.prim_off[sb];
    const int Ka = bs.nprim[sa], Kb = bs.nprim[sb];
    for (int i = 0; i < Ka; ++i)
      for (int j = 0; j < Kb; ++j) {
        const double a = bs.expo[oa + i], b = bs.expo[ob + j], p = a + b, ip = 1.0 / p;
        build_side(bx, cls, LA, LB, b * ps.R * ip, -a * ps.R * ip, p, an, lane);
        double* const rec = wk.rec + wk.pair_off[u] + (int64_t)(i * Kb + j) * stride;
        if (lane < kEriHdr) {
          double v = 0.0;
          if (lane == 0) v = p;
          else if (lane <= 3) v = (a * ps.A[lane - 1] + b * ps.B[lane - 1]) * ip;
          else if (lane == 4) v = exp_neg(a * b * ip * ps.R * ps.R) * bs.w[oa + i] * bs.w[ob + j];
          rec[lane] = v;
        }
        for (int t = lane; t < n; t += 64) rec[kEriHdr + t] = bx[t];
        wave_sync();
      }
  }
}

// One wavefront per quartet. For each bra primitive pair: the Boys values and solid harmonics of
// P - Q for up to kSlots ket primitive pairs at once (a lane each), then for each ket primitive
// pair the h table, the two-center matrix I and Y += K_cd I B'_ket^T (the ket contracted first,
// in registers); then the block += K_ab B'_bra Y,
// accumulated in registers (2 x 2 tiles lane + 64 k of the pair-ordered block). NABM and NWM bound
// the quartet's block and two-center entries per side; WPE is the occupancy (wavefronts per SIMD)
// the instance is compiled for.
template <int NABM, int NWM, int WPE>
__global__ void __launch_bounds__(kEriThreads) __attribute__((amdgpu_waves_per_eu(WPE)))
k_eri(DevBasis bs, EriWork wk, const double* __restrict__ boys_tab, double* __restrict__ out) {
  using Lds = EriLds<NABM, NWM>;
  constexpr int kAccPerLane = Lds::kAccPerLane, kIPerLane = Lds::kIPerLane, kYPerLane = Lds::kYPerLane;
  __shared__ double s_lds[kEriWavesPerGroup * Lds::SIZE];
  // the Gaunt terms, shared by the workgroup: coefficient, and (L, M) index | h offset << 8
  __shared__ double s_gg[kEriGTerms];
  __shared__ int s_gpk[kEriGTerms];
  for (int t = threadIdx.x; t < kEriGTerms; t += kEriThreads) {
    s_gg[t] = kEriG[t].g;
    s_gpk[t] = kEriG[t].I | kEriG[t].h << 8;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* const sm = s_lds + wave * Lds::SIZE;
  for (int64_t q = (int64_t)blockIdx.x * kEriWavesPerGroup + wave; q < wk.n_quartets;
       q += (int64_t)gridDim.x * kEriWavesPerGroup) {
    const int ub = wk.quart[4 * q], uk = wk.quart[4 * q + 1], fl = wk.quart[4 * q + 2];
    const int sa = wk.pairs[2 * ub], sb = wk.pairs[2 * ub + 1], sc = wk.pairs[2 * uk], sd = wk.pairs[2 * uk + 1];
    const int LA = bs.l[sa], LB = bs.l[sb], LC = bs.l[sc], LD = bs.l[sd];
    const int cb = class_id(LA, LB), ck = class_id(LC, LD);
    const int NB = 2 * LB + 1, ND = 2 * LD + 1, NAB = (2 * LA + 1) * NB, NCD = (2 * LC + 1) * ND;
    const int NW1 = kEriNW[cb], NW2 = kEriNW[ck], base1 = kEriEntBase[cb], base2 = kEriEntBase[ck];
    const int nb = bs.nprim[sa] * bs.nprim[sb], nk = bs.nprim[sc] * bs.nprim[sd];
    const int strb = kEriHdr + NAB * NW1, strk = kEriHdr + NCD * NW2;
    const double* const recb = wk.rec + wk.pair_off[ub];
    const double* const reck = wk.rec + wk.pair_off[uk];
    const int LT = LA + LB + LC + LD;
    // the lane's two-center entries (class-pair data, the same for every primitive quartet): the
    // first Gaunt term (12 bits), their count (5), j1 + j2 (3) and the sign (-1)^{L2} (1)
    uint32_t ient[kIPerLane];
#pragma unroll
    for (int k = 0; k < kIPerLane; ++k) {
      const int it = lane + 64 * k;
      uint32_t word = 0;
      if (it < NW1 * NW2) {
        const int w1 = it / NW2, w2 = it - w1 * NW2;
        const int L1 = kEriEnt[base1 + w1][0], M1 = kEriEnt[base1 + w1][1], j1 = kEriEnt[base1 + w1][2];
        const int L2 = kEriEnt[base2 + w2][0], M2 = kEriEnt[base2 + w2][1], j2 = kEriEnt[base2 + w2][2];
        const int i12 = (L1 * L1 + M1 + L1) * (kEriL12 + 1) * (kEriL12 + 1) + L2 * L2 + M2 + L2;
        const int g0 = kEriGOff[i12], gn = kEriGOff[i12 + 1] - g0;
        word = (uint32_t)g0 | (uint32_t)gn << 12 | (uint32_t)(j1 + j2) << 17 | (uint32_t)(L2 & 1) << 20;
      }
      ient[k] = word;
    }

    // the lane's entry of the h table: (L, n) with n <= (LT - L) / 2 (the orders the Gaunt terms
    // reach), and the coefficients of P_{L,n} (zero above its degree n - 1)
    int hL = -1, hn = 0;
    {
      int it = lane;
      for (int L = 0; L <= LT && hL < 0; ++L) {
        const int c = (LT - L) / 2 + 1;
        if (it < c) {
          hL = L;
          hn = it;
        } else {
          it -= c;
        }
      }
    }
    double hp[kEriNmax];
#pragma unroll
    for (int u = 0; u < kEriNmax; ++u) hp[u] = hL >= 0 ? kEriP[hL][hn][u] : 0.0;
    // the block in 2 x 2 tiles (e1, e1 + 1) x (e2, e2 + 1), tile lane + 64 k of nt1 x nt2
    const int nt1 = (NAB + 1) / 2, nt2 = (NCD + 1) / 2, ny1 = (NW1 + 1) / 2;
    double acc[kAccPerLane][4], y[kYPerLane][4];
#pragma unroll
    for (int k = 0; k < kAccPerLane; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[k][c] = 0.0;
#pragma unroll
    for (int k = 0; k < kYPerLane; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) y[k][c] = 0.0;
    for (int r1 = 0; r1 < nb; ++r1) {
      const double* const rb = recb + (int64_t)r1 * strb;
      const double p = rb[0], Kab = rb[4];
      const double P[3] = {rb[1], rb[2], rb[3]};
      for (int t = lane; t < NAB * NW1; t += 64) sm[Lds::BB + t] = rb[kEriHdr + t];
      for (int c0 = 0; c0 < nk; c0 += Lds::kSlots) {
        // the Boys values and solid harmonics of the next kSlots ket primitive pairs, a lane each
        if (lane < Lds::kSlots && c0 + lane < nk) {
          const double* const rk = reck + (int64_t)(c0 + lane) * strk;
          const double qq = rk[0];
          const double R[3] = {P[0] - rk[1], P[1] - rk[2], P[2] - rk[3]};
          const double T = p * qq / (p + qq) * (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
          double* const f = sm + Lds::STG + lane * Lds::kSlot;
          boys_and_harmonics_lt<Lds::LTM>(LT, T, R, boys_tab, f, f + Lds::LTM + 1, f + Lds::kFS);
        }
        wave_sync();
        for (int r2 = c0; r2 < nk && r2 < c0 + Lds::kSlots; ++r2) {
          const double* const rk = reck + (int64_t)r2 * strk;
          const double qq = rk[0], Kcd = rk[4];
          const double R[3] = {P[0] - rk[1], P[1] - rk[2], P[2] - rk[3]};
          for (int t = lane; t < NCD * NW2; t += 64) sm[Lds::BK + t] = rk[kEriHdr + t];
          const double alpha = p * qq / (p + qq);
          const double T = alpha * (R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
          const double cpre = 2.0 * 17.493418327624862846 / (p * qq * sqrt(p + qq));  // 2 pi^{5/2} / (p q sqrt(p+q))
          const double* const f = sm + Lds::STG + (r2 - c0) * Lds::kSlot;
          // h[L][n]: the lane's entry
          if (hL >= 0) {
            double base = cpre;
            for (int u = 0; u < hL; ++u) base *= -2.0 * alpha;
            double v;
            if (hn == 0) {
              v = f[hL];
            } else {
              double poly = 0.0;
#pragma unroll
              for (int u = kEriNmax - 1; u >= 0; --u) poly = fma(poly, T, hp[u]);
              double an = 1.0;
              for (int u = 0; u < hn; ++u) an *= alpha;
              v = an * poly * f[Lds::LTM + 1];
            }
            sm[Lds::H + hL * (kEriNmax + 1) + hn] = base * v;
          }
          wave_sync();
          // two-center matrix I[w1][w2]
#pragma unroll
          for (int k = 0; k < kIPerLane; ++k) {
            const int it = lane + 64 * k;
            if (it < NW1 * NW2) {
              const uint32_t wd = ient[k];
              const int g0 = (int)(wd & 4095u), gn = (int)((wd >> 12) & 31u), js = (int)((wd >> 17) & 7u);
              double sacc = 0.0;
              for (int t = g0; t < g0 + gn; ++t) {
                const int pk = s_gpk[t];
                sacc = fma(s_gg[t] * f[Lds::kFS + (pk & 255)], sm[Lds::H + (pk >> 8) + js], sacc);
              }
              sm[Lds::I + it] = ((wd >> 20) & 1u) ? -sacc : sacc;
            }
          }
          wave_sync();
          // Y += K_cd I B'_ket^T, in 2 x 2 tiles (rows w1, w1 + 1; columns e2, e2 + 1) held in
          // registers over the ket's primitive pairs; reads past the last row or column stay inside
          // the wavefront's LDS and their results are not kept
#pragma unroll
          for (int k = 0; k < kYPerLane; ++k) {
            const int tt = lane + 64 * k;
            if (tt < ny1 * nt2) {
              const int w1 = 2 * (tt / nt2), e2 = 2 * (tt - (tt / nt2) * nt2);
              double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
              const double* const i0 = sm + Lds::I + w1 * NW2;
              const double* const k0 = sm + Lds::BK + e2 * NW2;
              for (int w2 = 0; w2 < NW2; ++w2) {
                const double x0 = i0[w2], x1 = i0[NW2 + w2], y0 = k0[w2], y1 = k0[NW2 + w2];
                s00 = fma(x0, y0, s00);
                s01 = fma(x0, y1, s01);
                s10 = fma(x1, y0, s10);
                s11 = fma(x1, y1, s11);
              }
              y[k][0] = fma(Kcd, s00, y[k][0]);
              y[k][1] = fma(Kcd, s01, y[k][1]);
              y[k][2] = fma(Kcd, s10, y[k][2]);
              y[k][3] = fma(Kcd, s11, y[k][3]);
            }
          }
          wave_sync();
        }
      }
      // Y^T [e2][w1] into the I region, then the block += K_ab B'_bra Y
#pragma unroll
      for (int k = 0; k < kYPerLane; ++k) {
        const int tt = lane + 64 * k;
        if (tt < ny1 * nt2) {
          const int w1 = 2 * (tt / nt2), e2 = 2 * (tt - (tt / nt2) * nt2);
          double* const yt = sm + Lds::I + e2 * NW1 + w1;
          const bool w_in = w1 + 1 < NW1, e_in = e2 + 1 < NCD;
          yt[0] = y[k][0];
          if (w_in) yt[1] = y[k][2];
          if (e_in) {
            yt[NW1] = y[k][1];
            if (w_in) yt[NW1 + 1] = y[k][3];
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) y[k][c] = 0.0;
        }
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < kAccPerLane; ++k) {
        const int tt = lane + 64 * k;
        if (tt < nt1 * nt2) {
          const int e1 = 2 * (tt / nt2), e2 = 2 * (tt - (tt / nt2) * nt2);
          double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
          const double* const b0 = sm + Lds::BB + e1 * NW1;
          const double* const y0p = sm + Lds::I + e2 * NW1;
          for (int w1 = 0; w1 < NW1; ++w1) {
            const double x0 = b0[w1], x1 = b0[NW1 + w1], y0 = y0p[w1], y1 = y0p[NW1 + w1];
            s00 = fma(x0, y0, s00);
            s01 = fma(x0, y1, s01);
            s10 = fma(x1, y0, s10);
            s11 = fma(x1, y1, s11);
          }
          acc[k][0] = fma(Kab, s00, acc[k][0]);
          acc[k][1] = fma(Kab, s01, acc[k][1]);
          acc[k][2] = fma(Kab, s10, acc[k][2]);
          acc[k][3] = fma(Kab, s11, acc[k][3]);
        }
      }
      wave_sync();
    }
    // the block in the listed order: entry ((i0 N1 + i1) N2 + i2) N3 + i3
    const bool swb = fl & 1, swk = fl & 2;
    const int N1 = swb ? 2 * LA + 1 : NB, N2 = swk ? ND : 2 * LC + 1, N3 = swk ? 2 * LC + 1 : ND;
    const int64_t o = wk.out_off[q];
#pragma unroll
    for (int k = 0; k < kAccPerLane; ++k) {
      const int tt = lane + 64 * k;
      if (tt < nt1 * nt2) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int e1 = 2 * (tt / nt2) + (c >> 1), e2 = 2 * (tt - (tt / nt2) * nt2) + (c & 1);
          if (e1 < NAB && e2 < NCD) {
            const int ma = e1 / NB, mb = e1 - ma * NB, mc = e2 / ND, md = e2 - mc * ND;
            const int i0 = swb ? mb : ma, i1 = swb ? ma : mb, i2 = swk ? md : mc, i3 = swk ? mc : md;
            out[o + ((int64_t)(i0 * N1 + i1) * N2 + i2) * N3 + i3] = acc[k][c];
          }
        }
      }
    }
  }
}

}  // namespace

int eri_lmax() { return kEriLmax; }

// Make *buf at least `need` bytes (device memory, or pinned host memory), in whole MiB; the old
// contents are not kept. No stream may still use the old buffer.
static hipError_t grow_buffer(void** buf, size_t* have, size_t need, bool pinned_host) {
  if (*have >= need && *buf) return hipSuccess;
  if (*buf) (void)(pinned_host ? hipHostFree(*buf) : hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  const size_t mib = (size_t)1 << 20, bytes = std::max(mib, (need + mib - 1) / mib * mib);
  const hipError_t e = pinned_host ? hipHostMalloc(buf, bytes, hipHostMallocDefault) : hipMalloc(buf, bytes);
  if (e != hipSuccess) {
    *buf = nullptr;
    return e;
  }
  *have = bytes;
  return hipSuccess;
}

hipError_t run_eri(const shgo_plan* p, const shgo_basis* basis, int64_t n_quartets, const int32_t* quartets,
                   const int64_t* offsets, double* out, hipStream_t st) {
  if (n_quartets <= 0) return hipSuccess;
  // the distinct pairs, each with its higher l first (listed order where the l are equal); a
  // dense index of the n_shells^2 ordered pairs where that is small, else a hash map
  const int nsh = basis->n_shells;
  const bool dense = (int64_t)nsh * nsh <= ((int64_t)1 << 22);
  std::vector<int32_t> dense_index(dense ? (size_t)nsh * nsh : 0, -1);
  std::unordered_map<int64_t, int32_t> index;
  std::vector<int32_t> pairs;
  std::vector<int64_t> pair_off;
  // per distinct pair: primitive pairs, block entries, two-center entries, and whether it fits the
  // small instance of k_eri
  struct PairSize {
    int32_t k, nab, nw;
    bool small;
  };
  std::vector<PairSize> psize;
  int64_t rec_size = 0;
  auto pair_of = [&](int32_t x, int32_t y, bool& swapped) {
    swapped = basis->l[x] < basis->l[y];
    const int32_t a = swapped ? y : x, b = swapped ? x : y;
    const int64_t key = (int64_t)a * nsh + b;
    if (dense) {
      if (dense_index[(size_t)key] >= 0) return dense_index[(size_t)key];
    } else {
      auto it = index.find(key);
      if (it != index.end()) return it->second;
    }
    const int32_t u = (int32_t)(pairs.size() / 2);
    if (dense)
      dense_index[(size_t)key] = u;
    else
      index.emplace(key, u);
    pairs.push_back(a);
    pairs.push_back(b);
    pair_off.push_back(rec_size);
    const int la = basis->l[a], lb = basis->l[b];
    const int nab = (2 * la + 1) * (2 * lb + 1), nw = kEriNWHost[class_id(la, lb)];
    const int32_t k = basis->n_prim[a] * basis->n_prim[b];
    psize.push_back({k, nab, nw, nab <= kNabSmall && nw <= kNwSmall});
    rec_size += (int64_t)k * (kEriHdr + nab * nw);
    return u;
  };
  // One pass over the quartets: their pairs and swaps, and the sort key: the quartets whose two
  // pairs fit the small instance of k_eri first, then the rest, and within each the costliest
  // first (primitive quartets times the matrices' sizes, in buckets of a quarter octave: a
  // counting sort), so that the wavefronts striding over the list take the long quartets early.
  constexpr int kCostBuckets = 256;
  shgo_context* const ctx = p->ctx;
  if (ctx->eri_tmp.size() < (size_t)5 * n_quartets) ctx->eri_tmp.resize((size_t)5 * n_quartets);
  int32_t* const quart = ctx->eri_tmp.data();
  int32_t* const qkey = quart + (size_t)4 * n_quartets;
  std::vector<int64_t> count(2 * kCostBuckets + 1, 0);
  int64_t n_small = 0;
  for (int64_t q = 0; q < n_quartets; ++q) {
    bool sw1 = false, sw2 = false;
    const int32_t ub = pair_of(quartets[4 * q], quartets[4 * q + 1], sw1);
    const int32_t uk = pair_of(quartets[4 * q + 2], quartets[4 * q + 3], sw2);
    quart[4 * q] = ub;
    quart[4 * q + 1] = uk;
    quart[4 * q + 2] = (sw1 ? 1 : 0) | (sw2 ? 2 : 0);
    quart[4 * q + 3] = 0;
    const PairSize &pb = psize[(size_t)ub], &pk = psize[(size_t)uk];
    const uint64_t cost = (uint64_t)pb.k * (uint64_t)pk.k *
                          (uint64_t)(pb.nw * pk.nw + pb.nab * pk.nw + pb.nab * pk.nab + 200);
    const int oct = 63 - __builtin_clzll(cost);                          // floor(log2 cost)
    const int quarter = oct >= 2 ? (int)((cost >> (oct - 2)) & 3u) : 0;  // the next two bits
    const int bucket = std::min(kCostBuckets - 1, 4 * oct + quarter);
    const bool small = pb.small && pk.small;
    n_small += small;
    const int32_t key = (small ? 0 : kCostBuckets) + (kCostBuckets - 1 - bucket);
    qkey[q] = key;
    ++count[(size_t)key + 1];
  }
  const int64_t n_pairs = (int64_t)pair_off.size();
  for (int k = 0; k < 2 * kCostBuckets; ++k) count[(size_t)k + 1] += count[(size_t)k];
  // one workspace: pairs, pair offsets, quartets, output offsets (the index part, staged in
  // pinned host memory and uploaded by one copy), then the records; each 256-byte aligned
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t b_pairs = up(8 * n_pairs), b_poff = up(8 * n_pairs), b_quart = up(16 * n_quartets),
                b_ooff = up(8 * n_quartets), b_rec = up(8 * rec_size);
  const int64_t b_index = b_pairs + b_poff + b_quart + b_ooff;
  hipError_t e = grow_buffer(&ctx->eri_dev, &ctx->eri_dev_bytes, (size_t)(b_index + b_rec), false);
  if (e == hipSuccess) e = grow_buffer(&ctx->eri_pin, &ctx->eri_pin_bytes, (size_t)b_index, true);
  if (e != hipSuccess) return e;  // nothing of this call is on the stream yet
  char* const ws = (char*)ctx->eri_dev;
  char* const hs = (char*)ctx->eri_pin;
  std::memcpy(hs, pairs.data(), (size_t)8 * n_pairs);
  std::memcpy(hs + b_pairs, pair_off.data(), (size_t)8 * n_pairs);
  int32_t* const quart_sorted = (int32_t*)(hs + b_pairs + b_poff);
  int64_t* const off_sorted = (int64_t*)(hs + b_pairs + b_poff + b_quart);
  for (int64_t q = 0; q < n_quartets; ++q) {
    const int64_t k = count[(size_t)qkey[q]]++;
    for (int i = 0; i < 4; ++i) quart_sorted[4 * k + i] = quart[4 * q + i];
    off_sorted[k] = offsets[q];
  }
  EriWork wk;
  wk.n_pairs = n_pairs;
  wk.n_quartets = n_quartets;
  wk.pairs = (const int32_t*)ws;
  wk.pair_off = (const int64_t*)(ws + b_pairs);
  wk.quart = (const int32_t*)(ws + b_pairs + b_poff);
  wk.out_off = (const int64_t*)(ws + b_pairs + b_poff + b_quart);
  wk.rec = (double*)(ws + b_index);
  e = hipMemcpyAsync(ws, hs, (size_t)b_index, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    auto grid = [&](int64_t waves, int per_cu) {
      const int64_t cap = (int64_t)4 * per_cu * p->ctx->n_cu;
      return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + kEriWavesPerGroup - 1) / kEriWavesPerGroup, cap)));
    };
    hipLaunchKernelGGL(k_eri_pairs, grid(n_pairs, 1), dim3(kEriThreads), 0, st, p->bs, wk);
    // the small instance: 11 KB of matrices per wavefront, two workgroups and wavefronts per SIMD;
    // the large one (pair class (2,2) on either side): 31 KB, one
    EriWork ws_small = wk, ws_large = wk;
    ws_small.n_quartets = n_small;
    ws_large.n_quartets = n_quartets - n_small;
    ws_large.quart = wk.quart + 4 * n_small;
    ws_large.out_off = wk.out_off + n_small;
    if (ws_small.n_quartets > 0)
      hipLaunchKernelGGL((k_eri<kNabSmall, kNwSmall, 2>), grid(ws_small.n_quartets, 2), dim3(kEriThreads), 0, st, p->bs,
                         ws_small, p->ctx->boys_tab, out);
    if (ws_large.n_quartets > 0)
      hipLaunchKernelGGL((k_eri<kNabMax, kNwMax, 1>), grid(ws_large.n_quartets, 1), dim3(kEriThreads), 0, st, p->bs,
                         ws_large, p->ctx->boys_tab, out);
    e = hipGetLastError();
  }
  // the staged host copy and the workspace are reused by the next call: wait for the stream
  const hipError_t e2 = hipStreamSynchronize(st);
  if (e == hipSuccess) e = e2;
  return e;
}

}  // namespace shgo_impl
