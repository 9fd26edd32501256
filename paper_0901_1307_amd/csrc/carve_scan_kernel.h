// The signature/probe scan kernel and the tile spaces it walks (one image, or
// a batch of images), Section 3.1: the djb2 signature of each 512-byte sector
// (Eq. (1), 64-bit) and its lookup among the master signatures of the
// sector's cluster position. Device code only; included by carve.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "carve_device.h"

namespace carve {

constexpr int kScanThreads = 256;
constexpr int kScanWaves = kScanThreads / (int)kWave;
// kFlags: hit words and the matched slot of each flagged sector (for
// confirmation); kFlagBits: hit words only; kSigs: the signatures themselves.
enum { kFlags = 0, kSigs = 1, kFlagBits = 2 };

// ------------------------------------------------------------ images
// One image of a scan. tile_begin: its first tile in the scan's tile space.
struct ImageDesc {
  const uint8_t* base;
  uint64_t n_sectors;
  uint64_t tile_begin;
  uint32_t tau0;      // cluster position of the image's first sector
  uint32_t any_tau;   // 1: match at any cluster position
};

// Where a tile's sectors are.
struct TileRef {
  const uint8_t* base;   // its first sector
  uint32_t n_valid;      // 1..64 sectors
  uint32_t tau_first;    // cluster position of its first sector
  uint32_t any_tau;
  uint32_t image;
};

__device__ __forceinline__ TileRef tile_of(const ImageDesc& d, uint64_t g, uint32_t image) {
  const uint64_t first = (g - d.tile_begin) * kTileSectors;
  const uint64_t rem = d.n_sectors - first;
  return TileRef{d.base + first * kSectorBytes, rem >= kTileSectors ? kTileSectors : (uint32_t)rem,
                 (uint32_t)((first + d.tau0) & (kClusterSectors - 1)), d.any_tau, image};
}

// A scan of one image: the descriptor travels by value. Units are sectors:
// unit j is bytes [512j, 512j + 512) of its image.
struct OneImage {
  static constexpr uint32_t kUnitBytes = kSectorBytes, kUnitStride = kSectorBytes;
  static constexpr bool kAnyPosition = false;   // the image's own rule applies
  ImageDesc d;
  __device__ __forceinline__ uint64_t n_tiles() const { return (d.n_sectors + kTileSectors - 1) / kTileSectors; }
  // `cursor` is the image of the previous lookup (tiles are visited in increasing order)
  __device__ __forceinline__ TileRef tile(uint64_t g, uint32_t&) const { return tile_of(d, g, 0); }
  __device__ __forceinline__ const ImageDesc& image(uint32_t) const { return d; }
  __device__ __forceinline__ uint32_t image_of_tile(uint64_t) const { return 0; }
};

// A batch: descriptors in device memory, n + 1 of them (the last one only
// carries the total tile count in tile_begin).
struct ManyImages {
  static constexpr uint32_t kUnitBytes = kSectorBytes, kUnitStride = kSectorBytes;
  static constexpr bool kAnyPosition = false;
  const ImageDesc* __restrict__ d;
  uint32_t n;
  __device__ __forceinline__ uint64_t n_tiles() const { return d[n].tile_begin; }
  __device__ __forceinline__ TileRef tile(uint64_t g, uint32_t& cursor) const {
    // The image holding tile g is the last i with d[i].tile_begin <= g
    // (empty images are skipped). A wave's tiles are a stride of the grid
    // apart, which can pass several small images: the next 8 starts are
    // read at once (independent loads, one wait), not one after another.
    while (true) {
      uint32_t step = 0;
#pragma unroll
      for (uint32_t k = 1; k <= 8; ++k) {
        const uint32_t i = cursor + k < n ? cursor + k : n;   // d[n] (the total) ends every walk
        step += g >= d[i].tile_begin ? 1u : 0u;
      }
      cursor += step;
      if (step < 8) break;
    }
    return tile_of(d[cursor], g, cursor);
  }
  __device__ __forceinline__ const ImageDesc& image(uint32_t i) const { return d[i]; }
  __device__ __forceinline__ uint32_t image_of_tile(uint64_t g) const {   // last i with d[i].tile_begin <= g
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (d[mid].tile_begin <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
  }
};

// ------------------------------------------------------------------ scan
// Persistent grid over the tile space: wave q takes chunks q, q + W, ... of
// `chunk` consecutive tiles (W = waves in the grid). 4 waves per SIMD (at
// most 128 VGPRs): the more waves, the more sector loads in flight per CU.
// kSig: kSigDjb2 (wt = the digit-plane weight table) or kSigCrc64 (no table;
// wt unused). kLayout: the index's probe layout (kFlags only).
template <int kMode, int kSig, class Src, int kLayout = kLayoutBucketed>
__global__ __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_scan(
    Src src, uint32_t chunk, IndexView ix, uint64_t wt, uint64_t* __restrict__ out, uint32_t* __restrict__ hit_slot) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kScanWaves * kTileLds];
  const uint32_t w = threadIdx.x / kWave;
  const uint32_t l = lane_id();
  uint8_t* my = lds + w * kTileLds;
  const uint64_t n_tiles = src.n_tiles();
  const uint64_t n_waves = (uint64_t)gridDim.x * kScanWaves;
  uint64_t g = ((uint64_t)blockIdx.x * kScanWaves + w) * chunk;
  if (g >= n_tiles) return;
  auto next_of = [&](uint64_t t) {
    return ((t + 1) % chunk != 0) ? t + 1 : t + 1 + (n_waves - 1) * chunk;
  };
  uint32_t cur = 0;
  TileRef tr = src.tile(g, cur);
  PhaseRegs A, B;
  load_phase<true>(ContiguousRows{tr.base, tr.n_valid}, 0, A);
  while (true) {
    const uint64_t gn = next_of(g);
    const bool more = gn < n_tiles;
    uint32_t cur_n = cur;
    TileRef tn = tr;
    // The next tile's first phase is loaded while this tile's last one is
    // hashed. Unconditionally (the last tile reloads itself): a load under a
    // branch would make the compiler wait for every load at the join. The
    // next tile is looked up only here, with this tile's last phase in
    // flight: in a batch the lookup walks the image descriptors (dependent
    // loads), which must not hold back this tile's own loads.
    auto prefetch = [&](PhaseRegs& R) {
      if (more) tn = src.tile(gn, cur_n);
      load_phase<true>(ContiguousRows{tn.base, tn.n_valid}, 0, R);
    };
    uint64_t h;
    if constexpr (kSig == kSigCrc64)
      h = tile_crc_pipelined<true>(ContiguousRows{tr.base, tr.n_valid}, my, A, B, prefetch);
    else
      h = tile_signature_pipelined<true>(ContiguousRows{tr.base, tr.n_valid}, my, wt, A, B, prefetch);
    if constexpr (kMode == kFlags || kMode == kFlagBits) {
      const uint32_t tau = (tr.tau_first + l) & (kClusterSectors - 1);
      uint64_t hits = tile_probe<kLayout, 1, kMode == kFlags>(
          ix, h, tau, tr.any_tau != 0, kMode == kFlags ? hit_slot + g * kTileSectors : nullptr, ix.bloom,
          ix.log2_bloom_words);
      if (tr.n_valid < kTileSectors) hits &= (1ull << tr.n_valid) - 1ull;
      if (l == 0) out[g] = hits;
    } else {
      if (l < tr.n_valid) out[g * kTileSectors + l] = h;   // one image: tile g holds sectors 64g..
    }
    if (!more) break;
    g = gn;
    cur = cur_n;
    tr = tn;
  }
}

// ------------------------------------------------- position-split scan
// One image, per-cluster rule, split by cluster position. Workgroups are
// dispatched to the chip's 8 XCDs in turn (block b runs on XCD b mod 8), so
// block b scans the sectors at position p = b mod 8 and probes position p's
// slice of the Bloom filter: each XCD's L2 holds one eighth of the filter
// instead of all of it (until the last tiles, which go to whichever waves are
// free; see the work sharing below). Tile k of position p is the sectors
// j = 8(64k + i) + r (i = 0..63, r = (p - tau0) mod 8), 512 B each, one
// cluster apart; its 64 hit bits go to tau_words[p * words_per_pos + k]
// (lane i = bit i), to be merged into the ordinary bitmap afterwards.
constexpr uint32_t kPositions = kClusterSectors;

__device__ __forceinline__ uint64_t position_count(uint64_t n_sectors, uint32_t r) {
  return n_sectors > r ? (n_sectors - r + kPositions - 1) / kPositions : 0;
}

// Work sharing of the position-split scan. A position's tiles go in runs of
// `chunk`. The first 7/8 of them are fixed: in round k, wave q of the
// position (of W) takes run kW + q. The rest are handed out by the
// position's counter (32 bits at the start of the p-th 256-byte line of ctr,
// zero at launch): a claim that returns c takes run KW + c (K = the fixed
// rounds). A wave whose position has no run left claims from the next
// positions in turn, so an XCD that finishes early takes over tiles of one
// that lags. On the 64 GiB large image with fixed shares only, the waves'
// finishing times spread over about 1 ms (even XCDs about 0.45 ms behind odd
// ones, and 0.65 ms within an XCD) and the kernel ended with the last; this
// scheme took it from 10.58-10.84 to 10.40-10.42 ms with runs of 2 tiles (the
// same scheme with every run claimed: 10.9-12.0 ms, because adds on one
// counter serialize at about 22 per microsecond; 3/4 or 15/16 fixed: no better).
constexpr uint32_t kCtrStride = 32;
constexpr uint32_t kTauCounters = kPositions * kCtrStride;

struct TauPos {
  uint32_t p;         // cluster position (its slice of the filter, its hit words)
  uint32_t r;         // its first sector: j = 8k + r
  uint64_t count;     // its sectors
  uint64_t n_tiles;
  uint64_t n_static;  // rounds of fixed runs (one run per wave of the position each)
};

__device__ __forceinline__ TauPos tau_pos(uint32_t p, uint64_t n_sectors, uint32_t tau0, uint64_t round_tiles) {
  TauPos t;
  t.p = p;
  t.r = (p - tau0) & (kPositions - 1);
  t.count = position_count(n_sectors, t.r);
  t.n_tiles = (t.count + kTileSectors - 1) / kTileSectors;
  t.n_static = t.n_tiles * 7 / (8 * round_tiles);   // 7/8 of the tiles in fixed runs
  return t;
}

// Lane 0 increments position p's counter (32 bits at the start of its line);
// the result is read later with tau_claim_read, so the atomic's latency hides
// behind the tile in flight. An increment, not an add: the compiler turns an
// add into a wave-wide atomic whose result it broadcasts, and waits for, at
// once.
__device__ __forceinline__ uint32_t tau_claim_issue(unsigned int* ctr, uint32_t p, uint32_t l) {
  uint32_t v = 0;
  if (l == 0) v = atomicInc(ctr + p * (2 * kCtrStride), 0xFFFFFFFFu);
  return v;
}
__device__ __forceinline__ uint64_t tau_claim_read(uint32_t v) {   // lane 0's value, to every lane
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// kSlots = false: no slot records (hit_slot unused).
template <int kSig, int kLayout = kLayoutBucketed, bool kSlots = true>
__global__ __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_scan_tau(
    const uint8_t* __restrict__ image, uint64_t n_sectors, uint32_t tau0, uint64_t words_per_pos, uint32_t chunk,
    IndexView ix, uint64_t wt, uint64_t* __restrict__ tau_words, uint32_t* __restrict__ hit_slot,
    unsigned int* __restrict__ ctr) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kScanWaves * kTileLds];
  // the wave's index, uniform (so tile addresses stay in scalar registers)
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const uint32_t l = lane_id();
  uint8_t* my = lds + w * kTileLds;
  const uint64_t n_waves = (uint64_t)(gridDim.x / kPositions) * kScanWaves;   // per position
  const uint64_t q = (uint64_t)(blockIdx.x / kPositions) * kScanWaves + w;
  auto rows_of = [&](const TauPos& t, uint64_t k) {
    const uint64_t first = k * kTileSectors;   // its first cluster among the position's
    const uint64_t rem = t.count - first;
    return ClusterStrideRows{image + (first * kPositions + t.r) * kSectorBytes,
                             rem >= kTileSectors ? kTileSectors : (uint32_t)rem};
  };
  // A run claimed from position t's counter (c) or, once t has none left,
  // from the next positions; false when every position is done.
  const uint64_t round_tiles = n_waves * chunk;
  uint32_t visited = 1;
  auto claim_from = [&](TauPos& t, uint64_t c, uint64_t& g, uint64_t& end) {
    while (true) {
      g = (t.n_static * n_waves + c) * chunk;
      end = g + chunk;
      if (g < t.n_tiles) return true;
      if (visited == kPositions) return false;
      t = tau_pos((t.p + 1) & (kPositions - 1), n_sectors, tau0, round_tiles);
      ++visited;
      c = tau_claim_read(tau_claim_issue(ctr, t.p, l));
    }
  };
  TauPos cur = tau_pos(blockIdx.x % kPositions, n_sectors, tau0, round_tiles);
  uint64_t k = 0;          // the wave's fixed run of its own position
  bool fixed = cur.n_static > 0;
  uint64_t g = q * chunk, end = g + chunk;
  if (!fixed && !claim_from(cur, tau_claim_read(tau_claim_issue(ctr, cur.p, l)), g, end)) return;
  ClusterStrideRows tr = rows_of(cur, g);
  PhaseRegs A, B;
  load_phase<true>(tr, 0, A);
  while (true) {
    // the next tile: the rest of this run, else the wave's next fixed run,
    // else a claim issued now and read when the next tile's first loads are due
    const bool in_run = g + 1 < end && g + 1 < cur.n_tiles;
    const bool next_fixed = !in_run && fixed && k + 1 < cur.n_static;
    const bool claim = !in_run && !next_fixed;
    const uint32_t pending = claim ? tau_claim_issue(ctr, cur.p, l) : 0u;
    TauPos nxt = cur;
    uint64_t gn = g + 1, end_n = end;
    bool more = true;
    ClusterStrideRows tn = tr;
    auto prefetch = [&](PhaseRegs& R) {   // unconditionally, as in k_scan
      if (next_fixed) {
        gn = ((k + 1) * n_waves + q) * chunk;
        end_n = gn + chunk;
      } else if (claim) {
        // an empty asm that takes the claim's register here, so the compiler
        // waits for the atomic at this point and not where it was issued
        uint32_t c = pending;
        asm volatile("" : "+v"(c));
        more = claim_from(nxt, tau_claim_read(c), gn, end_n);
      }
      if (more) tn = rows_of(nxt, gn);
      load_phase<true>(tn, 0, R);
    };
    uint64_t h;
    if constexpr (kSig == kSigCrc64)
      h = tile_crc_pipelined<true>(tr, my, A, B, prefetch);
    else
      h = tile_signature_pipelined<true>(tr, my, wt, A, B, prefetch);
    // this position's slice of the filter
    const uint64_t* bloom = ix.bloom_tau ? ix.bloom_tau + ((uint64_t)cur.p << ix.log2_bloom_tau) : ix.bloom;
    const uint32_t log2_bloom = ix.bloom_tau ? ix.log2_bloom_tau : ix.log2_bloom_words;
    uint64_t hits = tile_probe<kLayout, kPositions, kSlots>(
        ix, h, cur.p, false, kSlots ? hit_slot + (g * kTileSectors * kPositions + cur.r) : nullptr, bloom, log2_bloom);
    if (tr.n_valid < kTileSectors) hits &= (1ull << tr.n_valid) - 1ull;
    if (l == 0) tau_words[cur.p * words_per_pos + g] = hits;
    if (!more) break;
    if (next_fixed) ++k;
    if (claim) fixed = false;
    cur = nxt;
    g = gn;
    end = end_n;
    tr = tn;
  }
}

}  // namespace carve
