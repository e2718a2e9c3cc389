// Host-side plan logic of the nuclear-attraction library, in plain C++ (no HIP): input validation,
// the counts a plan is sized by (candidate and screened shell pairs, integrals, output size), the
// layout of the plan's one device workspace, and the default schedule. shgo_api.hip uses it; the
// CPU test harness compiles it with g++ under AddressSanitizer and UBSan.
//
// Inputs follow the statement of the problem (Eq. 1: shells as center, l, exponents and
// contraction coefficients; Eq. 11: point nuclei with charges). Screening (not in the paper) drops
// a primitive pair when exp(-ab/(a+b) |A-B|^2) <= screen, and a shell pair with none left.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "shgo.h"
#include "schedule.h"
#include "generated/shgo_meta.inc"

namespace shgo_host {

using namespace shgo_sched;

inline shgo_status bad(std::string* msg, shgo_status s, const char* what) {
  if (msg) *msg = what;
  return s;
}

// Every check a plan performs before any device work; nothing is written on failure.
inline shgo_status validate_inputs(const shgo_basis* b, const shgo_nuclei* n, double screen, std::string* msg) {
  if (!b || !n) return bad(msg, SHGO_ERR_INVALID_ARG, "null basis or nuclei");
  if (b->n_shells < 0 || n->n_nuclei < 0) return bad(msg, SHGO_ERR_INVALID_ARG, "negative count");
  if (b->n_shells > 0 && (!b->center || !b->l || !b->n_prim || !b->prim_offset || !b->exponent || !b->coef))
    return bad(msg, SHGO_ERR_INVALID_ARG, "null basis array");
  if (n->n_nuclei > 0 && (!n->position || !n->charge)) return bad(msg, SHGO_ERR_INVALID_ARG, "null nuclei array");
  if (!std::isfinite(screen) || screen < 0.0) return bad(msg, SHGO_ERR_INVALID_ARG, "screen must be finite and >= 0");
  for (int s = 0; s < b->n_shells; ++s) {
    if (b->l[s] < 0 || b->l[s] > SHGO_LMAX) return bad(msg, SHGO_ERR_UNSUPPORTED_L, "shell l out of range 0..SHGO_LMAX");
    if (b->n_prim[s] < 1 || b->prim_offset[s] < 0) return bad(msg, SHGO_ERR_INVALID_ARG, "shell with no primitives");
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(b->center[3 * s + x])) return bad(msg, SHGO_ERR_NOT_FINITE, "non-finite shell center");
    for (int k = 0; k < b->n_prim[s]; ++k) {
      const double a = b->exponent[b->prim_offset[s] + k], d = b->coef[b->prim_offset[s] + k];
      if (!std::isfinite(a) || !std::isfinite(d)) return bad(msg, SHGO_ERR_NOT_FINITE, "non-finite exponent or coefficient");
      if (!(a > 0.0)) return bad(msg, SHGO_ERR_INVALID_ARG, "exponent must be > 0");
    }
  }
  for (int c = 0; c < n->n_nuclei; ++c) {
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(n->position[3 * c + x])) return bad(msg, SHGO_ERR_NOT_FINITE, "non-finite nucleus position");
    if (!std::isfinite(n->charge[c])) return bad(msg, SHGO_ERR_NOT_FINITE, "non-finite nuclear charge");
  }
  return SHGO_OK;
}

// Pair-list checks of shgo_plan_pairs and the size limits of both plan kinds.
inline shgo_status validate_pairs(const shgo_basis* b, int full, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                                  std::string* msg) {
  if (!full) {
    if (n_pairs < 0 || (n_pairs > 0 && (!pa || !pb))) return bad(msg, SHGO_ERR_INVALID_ARG, "bad pair list");
    for (int64_t i = 0; i < n_pairs; ++i)
      if (pa[i] < 0 || pa[i] >= b->n_shells || pb[i] < 0 || pb[i] >= b->n_shells)
        return bad(msg, SHGO_ERR_INVALID_ARG, "pair index out of range");
    if (n_pairs > (int64_t)INT32_MAX) return bad(msg, SHGO_ERR_INVALID_ARG, "too many pairs");
  } else if ((int64_t)b->n_shells * (b->n_shells + 1) / 2 > (int64_t)INT32_MAX) {
    return bad(msg, SHGO_ERR_INVALID_ARG, "too many shells");
  }
  return SHGO_OK;
}

// exp(-mu |A-B|^2) > screen for one primitive pair (every pair survives when screen <= 0).
inline bool keeps(double a, double b, double R2, double screen) {
  return !(screen > 0.0) || std::exp(-(a * b / (a + b)) * R2) > screen;
}

// What a plan is sized by.
struct PlanCounts {
  int64_t nbf = 0, n_prims = 0, n_cand = 0, out_size = 0;
  int64_t kept_pairs = 0;       // shell pairs that keep at least one primitive pair
  int64_t kept_prim_pairs = 0;  // primitive pairs that survive screening
  int64_t integrals = 0;        // sum of (2la+1)(2lb+1) over the kept shell pairs
  int64_t class_cand[kNumClasses] = {0};
  std::vector<int64_t> bf_off;  // first basis function of each shell
  std::vector<int32_t> by_l;    // [kLmax + 2] first entry of each l, then the shells by l, then primitive count
  std::vector<int64_t> blk_off; // output offset of each listed pair (pair plans)
};

inline void count_pair(const shgo_basis* b, int a, int c, double screen, PlanCounts& pc) {
  double R2 = 0.0;
  for (int x = 0; x < 3; ++x) {
    const double d = b->center[3 * a + x] - b->center[3 * c + x];
    R2 += d * d;
  }
  int64_t kept = 0;
  for (int i = 0; i < b->n_prim[a]; ++i)
    for (int j = 0; j < b->n_prim[c]; ++j)
      kept += keeps(b->exponent[b->prim_offset[a] + i], b->exponent[b->prim_offset[c] + j], R2, screen);
  pc.kept_prim_pairs += kept;
  if (kept > 0) {
    pc.kept_pairs++;
    pc.integrals += (int64_t)(2 * b->l[a] + 1) * (2 * b->l[c] + 1);
  }
}

// Counts of a matrix plan (full != 0: every a <= b) or a pair plan; inputs already validated.
inline PlanCounts plan_counts(const shgo_basis* b, int full, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                              double screen) {
  PlanCounts pc;
  pc.bf_off.resize((size_t)b->n_shells);
  for (int s = 0; s < b->n_shells; ++s) {
    pc.bf_off[(size_t)s] = pc.nbf;
    pc.nbf += 2 * b->l[s] + 1;
    pc.n_prims = std::max<int64_t>(pc.n_prims, b->prim_offset[s] + b->n_prim[s]);
  }
  // the shells of each l, by primitive count and then index (so that neighbouring pairs of a
  // class have alike contraction lengths), after the kLmax + 2 offsets of the l
  pc.by_l.assign((size_t)b->n_shells + kLmax + 2, 0);
  for (int s = 0; s < b->n_shells; ++s) pc.by_l[(size_t)b->l[s] + 1]++;
  for (int l = 0; l <= kLmax; ++l) pc.by_l[(size_t)l + 1] += pc.by_l[(size_t)l];
  {
    std::vector<int32_t> next(pc.by_l.begin(), pc.by_l.begin() + kLmax + 1);
    for (int s = 0; s < b->n_shells; ++s) pc.by_l[(size_t)kLmax + 2 + next[(size_t)b->l[s]]++] = s;
    for (int l = 0; l <= kLmax; ++l)
      std::stable_sort(pc.by_l.begin() + kLmax + 2 + pc.by_l[(size_t)l], pc.by_l.begin() + kLmax + 2 + pc.by_l[(size_t)l + 1],
                       [&](int32_t x, int32_t y) { return b->n_prim[x] < b->n_prim[y]; });
  }
  auto cls = [](int la, int lb) { return class_id(std::max(la, lb), std::min(la, lb)); };
  if (full) {
    pc.n_cand = (int64_t)b->n_shells * (b->n_shells + 1) / 2;
    pc.out_size = pc.nbf * pc.nbf;
    for (int a = 0; a < b->n_shells; ++a)
      for (int c = a; c < b->n_shells; ++c) {
        pc.class_cand[cls(b->l[a], b->l[c])]++;
        count_pair(b, a, c, screen, pc);
      }
  } else {
    pc.n_cand = n_pairs;
    pc.blk_off.resize((size_t)n_pairs);
    int64_t o = 0;
    for (int64_t i = 0; i < n_pairs; ++i) {
      pc.blk_off[(size_t)i] = o;
      o += (int64_t)(2 * b->l[pa[i]] + 1) * (2 * b->l[pb[i]] + 1);
      pc.class_cand[cls(b->l[pa[i]], b->l[pb[i]])]++;
      count_pair(b, pa[i], pb[i], screen, pc);
    }
    pc.out_size = o;
  }
  return pc;
}

// A work item holds its tile block in 24 bits (class << 24 | block).
inline shgo_status check_class_sizes(const PlanCounts& pc, std::string* msg) {
  for (int c = 0; c < kNumClasses; ++c)
    if ((pc.class_cand[c] + kTile - 1) / kTile >= ((int64_t)1 << 24))
      return bad(msg, SHGO_ERR_INVALID_ARG, "more than 2^30 shell pairs in one (la, lb) class");
  return SHGO_OK;
}

// The plan's device workspace: one block carved into every array the kernels use, each at a
// 256-byte boundary. Offsets in bytes from the block's start.
enum Buf {
  kCenter, kL, kNprim, kPoff, kBfOff, kByL, kExpo, kCoef, kW, kNuc, kPa, kPb, kBlk, kKey, kS1, kS2, kOrig, kNsurv, kRank,
  kKeyCount, kKeyOff, kDst0, kDst1, kQueue, kItemOff, kItems, kArgs, kEnergy, kNumBufs
};
struct PlanLayout {
  size_t off[kNumBufs] = {0};
  size_t bytes[kNumBufs] = {0};
  size_t total = 0;
};
inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Upper bound of the work items of a plan: one per tile of every class.
inline int64_t item_capacity(const PlanCounts& pc) {
  int64_t cap = 0;
  for (int c = 0; c < kNumClasses; ++c) cap += (pc.class_cand[c] + kTile - 1) / kTile;
  return std::max<int64_t>(cap, 1);
}

// nuc_bytes: bytes per nucleus on the device; args_bytes: bytes of the integral kernel's arguments.
inline PlanLayout plan_layout(const PlanCounts& pc, int32_t n_shells, int32_t n_nuclei, int full, size_t nuc_bytes,
                              size_t args_bytes) {
  PlanLayout L;
  const size_t ns = (size_t)n_shells, np = (size_t)pc.n_prims, nc = (size_t)pc.n_cand;
  const size_t nl = full ? 0 : nc;
  L.bytes[kCenter] = 24 * ns;
  L.bytes[kL] = 4 * ns;
  L.bytes[kNprim] = 4 * ns;
  L.bytes[kPoff] = 8 * ns;
  L.bytes[kBfOff] = 8 * ns;
  L.bytes[kByL] = 4 * (ns + kLmax + 2);
  L.bytes[kExpo] = 8 * np;
  L.bytes[kCoef] = 8 * np;
  L.bytes[kW] = 8 * np;
  L.bytes[kNuc] = nuc_bytes * (size_t)n_nuclei;
  L.bytes[kPa] = 4 * nl;
  L.bytes[kPb] = 4 * nl;
  L.bytes[kBlk] = 8 * nl;
  for (Buf b : {kKey, kS1, kS2, kOrig, kNsurv, kRank}) L.bytes[b] = 4 * nc;
  L.bytes[kKeyCount] = 4 * (size_t)kNumKeys;
  L.bytes[kKeyOff] = 4 * ((size_t)kNumKeys + 1);
  L.bytes[kDst0] = 8 * nc;
  L.bytes[kDst1] = 8 * nc;
  L.bytes[kQueue] = 4;
  L.bytes[kItemOff] = 4 * ((size_t)kNumClasses + 1);
  L.bytes[kItems] = 4 * (size_t)item_capacity(pc);
  L.bytes[kArgs] = args_bytes;
  L.bytes[kEnergy] = 8;
  size_t o = 0;
  for (int i = 0; i < kNumBufs; ++i) {
    L.off[i] = o;
    o += round_up(std::max<size_t>(L.bytes[i], 8), 256);
  }
  L.total = o;
  return L;
}

// Default tiles per work item of class c, within LDS: the fewest tiles that give the eight
// wavefronts eight (tile, slice, group) tasks. `slices` is the class's mean over its candidate
// pairs of ceil(K_a K_b / kSliceIters), capped at 8 (screening only lowers it). Where every pair
// has one slice the task counts are exact, and a smaller tile count is taken when it keeps the
// wavefronts busier over the item's task rounds (tasks / (kWaves * ceil(tasks / kWaves))): three
// groups take two tiles (six tasks in one round) rather than three (nine tasks, two rounds).
inline int default_tiles(int c, double slices) {
  const double tasks_per_tile = kClassGroups[c] * std::max(1.0, slices);
  const int t0 = std::max(1, std::min(class_max_tiles(c), (int)std::ceil(8.0 / tasks_per_tile - 1e-9)));
  if (slices > 1.0) return t0;
  int best = t0;
  double best_eff = 0.0;
  for (int t = t0; t >= 1; --t) {
    const int tasks = t * kClassGroups[c];
    const double eff = (double)tasks / (kWaves * ((tasks + kWaves - 1) / kWaves));
    if (eff > best_eff + 1e-12) {
      best = t;
      best_eff = eff;
    }
  }
  return best;
}

// Mean primitive-pair slices per candidate pair of each class, before screening (the matrix
// plan's pairs a <= b counted from a histogram of shells by l and primitive count).
inline void mean_slices(const shgo_basis* b, int full, int64_t n_pairs, const int32_t* pa, const int32_t* pb,
                        double* mean) {
  double sum[kNumClasses] = {0}, cnt[kNumClasses] = {0};
  auto sl = [](int64_t ka, int64_t kb) { return (double)std::min<int64_t>(8, (ka * kb + kSliceIters - 1) / kSliceIters); };
  auto cls = [](int la, int lb) { return class_id(std::max(la, lb), std::min(la, lb)); };
  if (full) {
    constexpr int kK = 64;  // primitive counts above this have the capped slice count too
    std::vector<double> h((size_t)(SHGO_LMAX + 1) * (kK + 1), 0.0);
    for (int s = 0; s < b->n_shells; ++s) h[(size_t)b->l[s] * (kK + 1) + std::min(b->n_prim[s], kK)] += 1.0;
    for (int la = 0; la <= SHGO_LMAX; ++la)
      for (int lb = 0; lb <= la; ++lb)
        for (int ka = 1; ka <= kK; ++ka)
          for (int kb = 1; kb <= kK; ++kb) {
            const double na = h[(size_t)la * (kK + 1) + ka], nb = h[(size_t)lb * (kK + 1) + kb];
            if (na == 0.0 || nb == 0.0) continue;
            double n;
            if (la != lb)
              n = na * nb;
            else if (ka < kb)
              n = na * nb;
            else if (ka == kb)
              n = na * (na + 1.0) / 2.0;
            else
              continue;
            sum[cls(la, lb)] += n * sl(ka, kb);
            cnt[cls(la, lb)] += n;
          }
  } else {
    for (int64_t i = 0; i < n_pairs; ++i) {
      const int c = cls(b->l[pa[i]], b->l[pb[i]]);
      sum[c] += sl(b->n_prim[pa[i]], b->n_prim[pb[i]]);
      cnt[c] += 1.0;
    }
  }
  for (int c = 0; c < kNumClasses; ++c) mean[c] = cnt[c] > 0.0 ? sum[c] / cnt[c] : 1.0;
}

// Checks of the single-call options beyond the inputs: the precision, the scratch limit against
// the workspace the call would allocate (0 = no limit).
inline shgo_status validate_options(const shgo_options* o, std::string* msg) {
  if (!o) return SHGO_OK;
  if (o->precision != SHGO_PREC_FP64 && o->precision != SHGO_PREC_MIXED)
    return bad(msg, SHGO_ERR_INVALID_ARG, "unknown precision");
  if (!std::isfinite(o->screen_threshold) || o->screen_threshold < 0.0)
    return bad(msg, SHGO_ERR_INVALID_ARG, "screen_threshold must be finite and >= 0");
  return SHGO_OK;
}

}  // namespace shgo_host
