// Schedule and layout arithmetic of the integral kernel, shared by the device code and by host
// code (plan sizing, the autotuner, and the CPU replay harness under tests/ that checks every
// index against its buffer). Plain integer arithmetic only: no HIP types, no device intrinsics.
//
// Terms:
//   class   c = la(la+1)/2 + lb for la >= lb (the shell with the higher l comes first)
//   key     c * kKeysPerClass + min(surviving primitive pairs, kKeysPerClass - 1); shell pairs are
//           counting-sorted by key, so a class's pairs are contiguous and ascending in survivors
//   tile    kTile consecutive class-sorted pairs, one per lane of a wavefront
//   item    a block of T consecutive tiles of one class (T = tiles[c]); one workgroup runs it
//   task    (tile, slice, group) of an item: a slice is at most kSliceIters primitive-pair
//           iterations of the tile, a group is one of the class's register groups of W
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define SHGO_HD __host__ __device__ __forceinline__
#else
#define SHGO_HD inline
#endif

namespace shgo_sched {

constexpr int kLmax = 7;                                         // highest shell l
constexpr int kNumClasses = (kLmax + 1) * (kLmax + 2) / 2;       // (la, lb) with la >= lb
constexpr int kKeysPerClass = 256;
constexpr int kNumKeys = kNumClasses * kKeysPerClass;
constexpr int kTile = 64;                                        // shell pairs per tile
constexpr int kIntegralThreads = 512;                            // one workgroup per CU
constexpr int kWaves = kIntegralThreads / 64;                    // wavefronts of a workgroup
constexpr int kMaxTilesPerItem = 8;
constexpr int kAccStride = kTile + 1;                            // doubles between accumulator entries
constexpr int kFrameDoubles = 4 * kTile;                         // cos/sin of theta and phi per pair
// Dynamic LDS of a work item, in doubles; the kernel's static LDS fits in the last 256 bytes of
// the CU's 160 KB.
constexpr int kLdsBytes = 163840;
constexpr int kStaticLdsReserve = 256;
constexpr int kLdsDoubles = (kLdsBytes - kStaticLdsReserve) / 8;
constexpr int kSliceIters = 2;                                   // primitive-pair iterations per slice
constexpr int kCostBuckets = 128;                                // 4 per octave of the item estimate

SHGO_HD constexpr int imin(int a, int b) { return a < b ? a : b; }
SHGO_HD constexpr int imax(int a, int b) { return a > b ? a : b; }

SHGO_HD constexpr int class_id(int la, int lb) { return la * (la + 1) / 2 + lb; }
SHGO_HD constexpr int class_la(int c) {
  int la = 0;
  while ((la + 1) * (la + 2) / 2 <= c) ++la;
  return la;
}
SHGO_HD constexpr int class_lb(int c) { return c - class_la(c) * (class_la(c) + 1) / 2; }
SHGO_HD constexpr int class_nab(int c) { return (2 * class_la(c) + 1) * (2 * class_lb(c) + 1); }

// LDS of one tile of class c: the accumulator [NA*NB][kAccStride] and the frames [4][kTile].
SHGO_HD constexpr int class_tile_doubles(int c) { return class_nab(c) * kAccStride + kFrameDoubles; }
SHGO_HD constexpr int class_max_tiles(int c) {
  return imin(kMaxTilesPerItem, kLdsDoubles / class_tile_doubles(c));
}
// Offsets (doubles) inside a work item's dynamic LDS of nt tiles.
SHGO_HD constexpr int acc_offset(int nab, int t) { return t * nab * kAccStride; }
SHGO_HD constexpr int frames_offset(int nab, int nt) { return nt * nab * kAccStride; }
SHGO_HD constexpr int item_lds_doubles(int nab, int nt) { return nt * (nab * kAccStride + kFrameDoubles); }

// Sort key of a shell pair of class c with ns surviving primitive pairs; the survivors a key
// records (saturated at kKeysPerClass - 1); the primitive-pair iterations the kernel runs for a
// pair of K1 x K2 primitives with that record (a saturated record visits every candidate pair
// and skips the screened ones).
SHGO_HD constexpr int pair_key(int c, int ns) { return c * kKeysPerClass + imin(ns, kKeysPerClass - 1); }
SHGO_HD constexpr int key_survivors(int key) { return key % kKeysPerClass; }
SHGO_HD constexpr int pair_iters(int survivors, int K1, int K2) {
  return survivors >= kKeysPerClass - 1 ? K1 * K2 : survivors;
}

SHGO_HD constexpr int slices_of(int iters) { return imax(1, (iters + kSliceIters - 1) / kSliceIters); }

// Tiles of a work item: class pairs [start, end) of the sorted list, the item's first tile t0 and
// its tile count nt (the last item of a class may hold fewer than T).
struct ItemGeom {
  int start, end, tiles, t0, nt;
};
SHGO_HD ItemGeom item_geom(const int32_t* key_off, int c, int T, int blk) {
  ItemGeom g;
  g.start = key_off[c * kKeysPerClass];
  g.end = key_off[(c + 1) * kKeysPerClass];
  g.tiles = (g.end - g.start + kTile - 1) / kTile;
  g.t0 = blk * T;
  g.nt = imin(T, g.tiles - g.t0);
  return g;
}

// (a, b) with a <= b from the linear index i of the upper triangle of an n x n matrix in
// row-major order (a matrix plan's candidate pair i).
SHGO_HD void tri_pair(int64_t i, int n, int& a, int& b) {
  const int64_t m = (int64_t)n * (n + 1) / 2;
  const int64_t j = m - 1 - i;
  int64_t r = (int64_t)((sqrt(8.0 * (double)j + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= j) ++r;
  while (r * (r + 1) / 2 > j) --r;
  a = n - 1 - (int)r;
  b = n - 1 - (int)(j - r * (r + 1) / 2);
}

// Work items of class c with `pairs` sorted pairs and T tiles per item.
SHGO_HD constexpr int class_items(int pairs, int T) { return ((pairs + kTile - 1) / kTile + T - 1) / T; }

// The last class whose first item index is <= i (ioff[c] = first item of class c, ascending).
SHGO_HD int class_of_item(int i, const int32_t* ioff) {
  int lo = 0, hi = kNumClasses - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ioff[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Surviving primitive pairs of the item's longest tile: the key of its last pair (keys ascend in
// a class), found by bisection over the class's key offsets; at least 1.
SHGO_HD int item_iters(const int32_t* key_off, int c, const ItemGeom& g) {
  const int last = imin(g.start + (g.t0 + g.nt) * kTile, g.end) - 1;
  int lo = 0, hi = kKeysPerClass - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key_off[c * kKeysPerClass + mid] <= last)
      lo = mid;
    else
      hi = mid - 1;
  }
  return imax(lo, 1);
}

// Tasks of an item whose longest tile runs m iterations, and the item's cost estimate
// weight x m x nt / (wavefronts its tasks keep busy).
SHGO_HD int item_tasks(int nt, int groups, int m) { return nt * groups * slices_of(m); }
SHGO_HD float item_cost(float weight, int m, int nt, int tasks) {
  return weight * (float)m * (float)nt / (float)imin(kWaves, tasks);
}

// Decode a task index of an item with nt tiles of per-tile iteration counts iters[t] and Q
// groups: tasks are tile-major from the item's last tile to its first (a class's pairs ascend in
// surviving primitive pairs, so the longest tasks are handed out first and the short ones fill the
// end), then slice, then group (groups are generated heaviest first). Returns false once the index
// lies past the item's last task; else the tile t, the group g and the iteration range [it0, it1).
SHGO_HD bool decode_task(int task, int Q, int nt, const int* iters, int& t, int& g, int& it0, int& it1) {
  int u = task / Q;
  g = task - u * Q;
  int m = 0;
  for (t = nt - 1; t >= 0; --t) {
    m = iters[t];
    const int s = slices_of(m);
    if (u < s) break;
    u -= s;
  }
  if (t < 0) return false;
  it0 = u * kSliceIters;
  it1 = imin(m, it0 + kSliceIters);
  return true;
}

// Output phase: entry j of the item's nt * kTile * NAB outputs is entry e of the block of pair
// tp (tile tp / kTile, lane tp % kTile); the accumulator holds V(i, col) of that pair at
// acc_entry(nab, tp, i * NB + col).
SHGO_HD constexpr int acc_entry(int nab, int tp, int e) { return ((tp >> 6) * nab + e) * kAccStride + (tp & 63); }
static_assert(kTile == 64, "acc_entry splits a pair index into tile and lane by shifts");

// Output element of entry (i, col) of a pair's block. Matrix output (nbf x nbf, row-major), the
// pair's rows starting at basis function r0 and its columns at c0: pass 0 writes the block,
// pass 1 its mirror; a shell with itself (r0 == c0) writes only i <= col in each pass, so that a
// diagonal element is written twice with the same value and the others once. Returns -1 where
// nothing is written.
SHGO_HD int64_t out_index_matrix(int pass, int64_t r0, int64_t c0, int i, int col, int64_t nbf) {
  if (r0 == c0 && i > col) return -1;
  return pass == 0 ? (r0 + i) * nbf + c0 + col : (c0 + col) * nbf + r0 + i;
}
// Pair-list output: the block of NA x NB entries at offset bo, row-major in the listed orientation;
// sw != 0 when the listed pair is (s2, s1), whose output entry e = col NA + i holds V(i, col).
// Returns the block entry i NB + col that output entry e takes.
SHGO_HD int list_source_entry(int e, bool sw, int NA, int NB) {
  if (!sw) return e;
  const int col = e / NA, i = e - col * NA;
  return i * NB + col;
}

}  // namespace shgo_sched
