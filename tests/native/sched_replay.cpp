// CPU replay of the integral kernel's schedule and layout arithmetic (csrc/schedule.h) and of the
// plan's host logic (csrc/plan_host.h), built with g++ under AddressSanitizer and UBSan.
//
// For one workload (a basis, a screening threshold, a matrix plan or a pair list) it replays, in
// plain loops, what the device does with the same functions:
//   pair build   candidate i -> (a, b) (tri_pair), its class and surviving primitive pairs, its
//                key, the counting sort into slots, each slot's output destination
//   work items   per class the items of T tiles, their cost buckets and the bucket sort
//   each item    tile geometry, per-tile iterations, the (tile, slice, group) tasks handed out
//                by the first-task rule and the LDS counter, the lanes' pair slots, the LDS
//                offsets of accumulators, frames and staged destinations, the output phase
// and asserts every index against its buffer, and that every item, task, slot and output element
// is covered exactly once (a diagonal element of a shell's block with itself is written by both
// output passes, from the same accumulator entry).
//
// Input file (whitespace-separated):
//   full n_shells n_nuclei screen n_pairs
//   per shell: l nprim prim_offset cx cy cz
//   n_prims, then per primitive: exponent coef
//   per nucleus: x y z Z
//   per listed pair (pair plans): a b
//   n_schedules, then per schedule kNumClasses tiles
// Output: one line "ok items=... tasks=... writes=..." per schedule; exit status 1 on a failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan_host.h"
#include "schedule.h"

using namespace shgo_sched;

#define CHECK(cond, ...)                                                            \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      std::fprintf(stderr, "CHECK failed at line %d: %s -- ", __LINE__, #cond);   \
      std::fprintf(stderr, __VA_ARGS__);                                            \
      std::fprintf(stderr, "\n");                                                   \
      std::exit(1);                                                                 \
    }                                                                               \
  } while (0)

struct Workload {
  int full = 1;
  double screen = 0.0;
  int n_shells = 0, n_nuc = 0;
  std::vector<int32_t> l, nprim;
  std::vector<int64_t> poff;
  std::vector<double> center, expo, coef, npos, nz;
  std::vector<int32_t> pa, pb;
  std::vector<std::vector<int32_t>> schedules;
};

static Workload read_input(const char* path) {
  FILE* f = std::fopen(path, "r");
  CHECK(f, "cannot open %s", path);
  Workload w;
  long long n_pairs = 0;
  CHECK(std::fscanf(f, "%d %d %d %lf %lld", &w.full, &w.n_shells, &w.n_nuc, &w.screen, &n_pairs) == 5, "header");
  w.l.resize(w.n_shells);
  w.nprim.resize(w.n_shells);
  w.poff.resize(w.n_shells);
  w.center.resize(3 * (size_t)w.n_shells);
  for (int s = 0; s < w.n_shells; ++s) {
    long long o = 0;
    CHECK(std::fscanf(f, "%d %d %lld %lf %lf %lf", &w.l[s], &w.nprim[s], &o, &w.center[3 * s], &w.center[3 * s + 1],
                      &w.center[3 * s + 2]) == 6,
          "shell %d", s);
    w.poff[s] = o;
  }
  long long np = 0;
  CHECK(std::fscanf(f, "%lld", &np) == 1, "primitive count");
  w.expo.resize(np);
  w.coef.resize(np);
  for (long long k = 0; k < np; ++k) CHECK(std::fscanf(f, "%lf %lf", &w.expo[k], &w.coef[k]) == 2, "primitive");
  w.npos.resize(3 * (size_t)w.n_nuc);
  w.nz.resize(w.n_nuc);
  for (int c = 0; c < w.n_nuc; ++c)
    CHECK(std::fscanf(f, "%lf %lf %lf %lf", &w.npos[3 * c], &w.npos[3 * c + 1], &w.npos[3 * c + 2], &w.nz[c]) == 4,
          "nucleus");
  w.pa.resize(n_pairs);
  w.pb.resize(n_pairs);
  for (long long i = 0; i < n_pairs; ++i) CHECK(std::fscanf(f, "%d %d", &w.pa[i], &w.pb[i]) == 2, "pair");
  int ns = 0;
  CHECK(std::fscanf(f, "%d", &ns) == 1, "schedule count");
  for (int k = 0; k < ns; ++k) {
    std::vector<int32_t> t(kNumClasses);
    for (int c = 0; c < kNumClasses; ++c) CHECK(std::fscanf(f, "%d", &t[c]) == 1, "tiles");
    w.schedules.push_back(t);
  }
  std::fclose(f);
  return w;
}

int main(int argc, char** argv) {
  CHECK(argc == 2, "usage: sched_replay INPUT");
  Workload w = read_input(argv[1]);
  shgo_basis b{w.n_shells, w.center.data(), w.l.data(), w.nprim.data(), w.poff.data(), w.expo.data(), w.coef.data()};
  shgo_nuclei nu{w.n_nuc, w.npos.data(), w.nz.data()};
  const int64_t n_pairs = (int64_t)w.pa.size();
  std::string msg;
  CHECK(shgo_host::validate_inputs(&b, &nu, w.screen, &msg) == SHGO_OK, "inputs: %s", msg.c_str());
  CHECK(shgo_host::validate_pairs(&b, w.full, n_pairs, w.pa.data(), w.pb.data(), &msg) == SHGO_OK, "pairs: %s",
        msg.c_str());
  const shgo_host::PlanCounts pc = shgo_host::plan_counts(&b, w.full, n_pairs, w.pa.data(), w.pb.data(), w.screen);
  CHECK(shgo_host::check_class_sizes(pc, &msg) == SHGO_OK, "sizes");

  // ---- the plan's workspace layout: disjoint, aligned, inside the block
  const shgo_host::PlanLayout lay = shgo_host::plan_layout(pc, w.n_shells, w.n_nuc, w.full, 32, 1024);
  for (int i = 0; i < shgo_host::kNumBufs; ++i) {
    CHECK(lay.off[i] % 256 == 0, "buffer %d misaligned", i);
    const size_t end = lay.off[i] + lay.bytes[i];
    CHECK(end <= (i + 1 < shgo_host::kNumBufs ? lay.off[i + 1] : lay.total), "buffer %d overlaps the next", i);
  }

  // ---- default schedule
  double slices[kNumClasses];
  shgo_host::mean_slices(&b, w.full, n_pairs, w.pa.data(), w.pb.data(), slices);
  std::vector<int32_t> def(kNumClasses);
  for (int c = 0; c < kNumClasses; ++c) {
    def[c] = shgo_host::default_tiles(c, slices[c]);
    CHECK(def[c] >= 1 && def[c] <= class_max_tiles(c), "default tiles of class %d", c);
  }
  w.schedules.insert(w.schedules.begin(), def);

  // ---- pair build (k_classify, k_scan_keys' key scan, k_scatter)
  const int64_t n_cand = pc.n_cand;
  CHECK(n_cand <= (int64_t)INT32_MAX, "candidates");
  std::vector<int32_t> key(n_cand), rank(n_cand), key_count(kNumKeys, 0);
  std::vector<uint8_t> seen_pair;
  if (w.full) seen_pair.assign((size_t)w.n_shells * w.n_shells, 0);
  int64_t kept_pairs = 0, kept_prims = 0, integrals = 0;
  for (int64_t i = 0; i < n_cand; ++i) {
    int a, c;
    if (w.full) {
      tri_pair(i, w.n_shells, a, c);
      CHECK(a >= 0 && a <= c && c < w.n_shells, "tri_pair(%lld) = (%d, %d)", (long long)i, a, c);
      CHECK(!seen_pair[(size_t)a * w.n_shells + c], "tri_pair repeats (%d, %d)", a, c);
      seen_pair[(size_t)a * w.n_shells + c] = 1;
    } else {
      a = w.pa[i];
      c = w.pb[i];
    }
    const int s1 = w.l[a] >= w.l[c] ? a : c, s2 = w.l[a] >= w.l[c] ? c : a;
    double R2 = 0.0;
    for (int x = 0; x < 3; ++x) {
      const double d = w.center[3 * s2 + x] - w.center[3 * s1 + x];
      R2 += d * d;
    }
    int ns = 0;
    for (int p = 0; p < w.nprim[s1]; ++p)
      for (int q = 0; q < w.nprim[s2]; ++q)
        ns += shgo_host::keeps(w.expo[w.poff[s1] + p], w.expo[w.poff[s2] + q], R2, w.screen);
    kept_prims += ns;
    if (ns > 0) {
      kept_pairs++;
      integrals += (int64_t)(2 * w.l[a] + 1) * (2 * w.l[c] + 1);
    }
    key[i] = pair_key(class_id(w.l[s1], w.l[s2]), ns);
    CHECK(key[i] >= 0 && key[i] < kNumKeys, "key %d", key[i]);
    rank[i] = key_count[key[i]]++;
  }
  CHECK(kept_pairs == pc.kept_pairs && kept_prims == pc.kept_prim_pairs && integrals == pc.integrals,
        "screened counts differ from the plan's");
  std::vector<int32_t> key_off(kNumKeys + 1, 0);
  for (int k = 0; k < kNumKeys; ++k) key_off[k + 1] = key_off[k] + key_count[k];
  CHECK(key_off[kNumKeys] == n_cand, "key scan total");
  for (int c = 0; c < kNumClasses; ++c)
    CHECK(key_off[(c + 1) * kKeysPerClass] - key_off[c * kKeysPerClass] == pc.class_cand[c], "class %d count", c);
  std::vector<int32_t> s1v(n_cand, -1), s2v(n_cand), nsurv(n_cand);
  std::vector<int64_t> dst0(n_cand), dst1(n_cand);
  for (int64_t i = 0; i < n_cand; ++i) {
    int a, c;
    if (w.full)
      tri_pair(i, w.n_shells, a, c);
    else {
      a = w.pa[i];
      c = w.pb[i];
    }
    const int64_t slot = (int64_t)key_off[key[i]] + rank[i];
    CHECK(slot >= 0 && slot < n_cand && s1v[slot] < 0, "slot %lld", (long long)slot);
    const bool sw = w.l[a] < w.l[c];
    s1v[slot] = sw ? c : a;
    s2v[slot] = sw ? a : c;
    nsurv[slot] = key_survivors(key[i]);
    if (w.full) {
      dst0[slot] = pc.bf_off[sw ? c : a];
      dst1[slot] = pc.bf_off[sw ? a : c];
    } else {
      dst0[slot] = pc.blk_off[i];
      dst1[slot] = sw ? 1 : 0;
    }
  }

  // ---- every schedule: items, tasks, LDS offsets, output
  const int64_t out_size = pc.out_size;
  for (const std::vector<int32_t>& tiles : w.schedules) {
    float weight[kNumClasses];
    for (int c = 0; c < kNumClasses; ++c) {
      CHECK(tiles[c] >= 1 && tiles[c] <= class_max_tiles(c), "tiles[%d] = %d", c, tiles[c]);
      weight[c] = (float)(1 + 37 * c % 1000);
    }
    // k_scan_keys: items per class, first item of each class, buckets, counting sort
    int32_t ioff[kNumClasses + 1];
    ioff[0] = 0;
    for (int c = 0; c < kNumClasses; ++c)
      ioff[c + 1] = ioff[c] + class_items(key_off[(c + 1) * kKeysPerClass] - key_off[c * kKeysPerClass], tiles[c]);
    const int total = ioff[kNumClasses];
    CHECK(total <= shgo_host::item_capacity(pc), "items %d exceed the capacity", total);
    std::vector<int> bucket(total), bcount(kCostBuckets, 0);
    for (int i = 0; i < total; ++i) {
      const int c = class_of_item(i, ioff);
      CHECK(i >= ioff[c] && i < ioff[c + 1], "class_of_item(%d) = %d", i, c);
      const int blk = i - ioff[c];
      const ItemGeom g = item_geom(key_off.data(), c, tiles[c], blk);
      const int m = item_iters(key_off.data(), c, g);
      const float cost = item_cost(weight[c], m, g.nt, item_tasks(g.nt, kClassGroups[c], m));
      int bk = 0;
      if (cost >= 1.0f) bk = imin(kCostBuckets - 1, (int)(4.0f * std::log2(cost)));
      CHECK(bk >= 0 && bk < kCostBuckets, "bucket %d", bk);
      bucket[i] = bk;
      bcount[bk]++;
    }
    std::vector<int> bstart(kCostBuckets);
    int run = 0;
    for (int r = 0; r < kCostBuckets; ++r) {
      bstart[kCostBuckets - 1 - r] = run;
      run += bcount[kCostBuckets - 1 - r];
    }
    std::vector<int32_t> items(total, -1);
    for (int i = 0; i < total; ++i) {
      const int c = class_of_item(i, ioff);
      const int pos = bstart[bucket[i]]++;
      CHECK(pos >= 0 && pos < total && items[pos] < 0, "item position %d", pos);
      items[pos] = (c << 24) | (i - ioff[c]);
    }
    // process_block of every item
    std::vector<uint8_t> slot_done(n_cand, 0);
    std::vector<uint8_t> writes(out_size, 0);
    std::vector<int64_t> source(out_size, -1);
    int64_t n_tasks = 0, n_writes = 0;
    for (int q = 0; q < total; ++q) {
      const int c = items[q] >> 24, blk = items[q] & 0xffffff;
      CHECK(c >= 0 && c < kNumClasses && blk < ioff[c + 1] - ioff[c], "item %d", q);
      const int LA = class_la(c), LB = class_lb(c), NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB;
      const int Q = kClassGroups[c];
      const ItemGeom ig = item_geom(key_off.data(), c, tiles[c], blk);
      CHECK(ig.nt >= 1 && ig.nt <= tiles[c] && ig.t0 >= 0 && ig.t0 + ig.nt <= ig.tiles && ig.nt <= kWaves,
            "item geometry c=%d blk=%d", c, blk);
      const int lds = item_lds_doubles(NAB, ig.nt);
      CHECK(lds <= kLdsDoubles, "LDS %d doubles", lds);
      const int frm = frames_offset(NAB, ig.nt);
      CHECK(frm + 4 * kTile * ig.nt <= lds, "frames");
      CHECK(2 * kTile * ig.nt <= 4 * kTile * ig.nt, "staged destinations exceed the frames area");
      // per-tile iterations (wavefront t < nt), and every lane's pair slot
      int iters[kMaxTilesPerItem] = {0};
      for (int t = 0; t < ig.nt; ++t)
        for (int lane = 0; lane < kTile; ++lane) {
          const int slot = ig.start + (ig.t0 + t) * kTile + lane;
          const bool active = slot < ig.end;
          const int sl = active ? slot : ig.end - 1;
          CHECK(sl >= ig.start && sl < ig.end, "lane slot %d of [%d, %d)", sl, ig.start, ig.end);
          if (active) iters[t] = imax(iters[t], pair_iters(nsurv[slot], w.nprim[s1v[slot]], w.nprim[s2v[slot]]));
          // accumulator entries of this lane, the frames of its tile
          CHECK(acc_offset(NAB, t) + (NAB - 1) * kAccStride + lane < frm, "accumulator");
          CHECK(frm + t * 4 * kTile + 3 * kTile + lane < lds, "frame entry");
        }
      // tasks: wavefront w takes task w first, then tasks from the counter (starting at kWaves)
      std::vector<std::vector<std::pair<int, int>>> ranges((size_t)ig.nt * Q);
      int counter = kWaves;
      for (int wave = 0; wave < kWaves; ++wave) {
        int task = wave;
        while (true) {
          int t, g, it0, it1;
          if (!decode_task(task, Q, ig.nt, iters, t, g, it0, it1)) break;
          CHECK(t >= 0 && t < ig.nt && g >= 0 && g < Q && it0 >= 0 && it1 <= imax(iters[t], 0) + 0 &&
                    it1 - it0 <= kSliceIters,
                "task %d -> (%d, %d, [%d, %d))", task, t, g, it0, it1);
          ranges[(size_t)t * Q + g].push_back({it0, it1});
          n_tasks++;
          task = counter++;
        }
      }
      for (int t = 0; t < ig.nt; ++t)
        for (int g = 0; g < Q; ++g) {
          std::vector<std::pair<int, int>>& r = ranges[(size_t)t * Q + g];
          CHECK(!r.empty(), "tile %d group %d never ran", t, g);
          std::sort(r.begin(), r.end());
          int at = 0;
          for (const auto& x : r) {
            CHECK(x.first == at && x.second >= x.first, "iterations of tile %d group %d not covered once", t, g);
            at = x.second;
          }
          CHECK(at == iters[t], "tile %d group %d ran %d of %d iterations", t, g, at, iters[t]);
          CHECK(r.size() == (size_t)slices_of(iters[t]), "slices of tile %d", t);
        }
      // rotations back: (tile, row) and (tile, column) tasks
      for (int k = 0; k < ig.nt * NA; ++k) {
        const int t = k / NA, r = k - t * NA;
        CHECK((t * NAB + r * NB + NB - 1) * kAccStride + kTile - 1 < frm, "row rotation");
      }
      for (int k = 0; k < ig.nt * NB; ++k) {
        const int t = k / NB, col = k - t * NB;
        CHECK((t * NAB + (NA - 1) * NB + col) * kAccStride + kTile - 1 < frm, "column rotation");
      }
      // output phase
      const int base = ig.start + ig.t0 * kTile;
      const int n_out = ig.nt * kTile * NAB;
      for (int pass = 0; pass < (w.full ? 2 : 1); ++pass)
        for (int j = 0; j < n_out; ++j) {
          const int tp = j / NAB, e = j - tp * NAB;
          const int slot = base + tp;
          if (slot >= ig.end) continue;
          if (pass == 0 && e == 0) {
            CHECK(!slot_done[slot], "slot %d output twice", slot);
            slot_done[slot] = 1;
          }
          int i, col, src;
          int64_t o;
          if (w.full) {
            if (pass == 0) {
              i = e / NB;
              col = e - i * NB;
            } else {
              col = e / NA;
              i = e - col * NA;
            }
            src = i * NB + col;
            o = out_index_matrix(pass, dst0[slot], dst1[slot], i, col, (int64_t)pc.nbf);
          } else {
            src = list_source_entry(e, dst1[slot] != 0, NA, NB);
            o = dst0[slot] + e;
          }
          CHECK(src >= 0 && src < NAB, "block entry %d", src);
          CHECK(acc_entry(NAB, tp, src) < frm, "accumulator read %d", acc_entry(NAB, tp, src));
          if (o < 0) continue;
          CHECK(o < out_size, "output index %lld of %lld", (long long)o, (long long)out_size);
          const int64_t tag = (int64_t)slot * 256 + src;
          if (writes[o]) {
            CHECK(writes[o] == 1 && source[o] == tag, "output %lld written twice from different entries", (long long)o);
          }
          writes[o]++;
          source[o] = tag;
          n_writes++;
        }
    }
    for (int64_t s = 0; s < n_cand; ++s) CHECK(slot_done[s], "slot %lld never output", (long long)s);
    for (int64_t o = 0; o < out_size; ++o) CHECK(writes[o] >= 1, "output %lld never written", (long long)o);
    std::printf("ok items=%d tasks=%lld writes=%lld\n", total, (long long)n_tasks, (long long)n_writes);
  }
  return 0;
}
