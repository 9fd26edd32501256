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
// block b scans only the sectors at position p = b mod 8 and probes only
// position p's slice of the Bloom filter: each XCD's L2 holds one eighth of
// the filter instead of all of it. Tile k of position p is the sectors
// j = 8(64k + i) + r (i = 0..63, r = (p - tau0) mod 8), 512 B each, one
// cluster apart; its 64 hit bits go to tau_words[p * words_per_pos + k]
// (lane i = bit i), to be merged into the ordinary bitmap afterwards.
constexpr uint32_t kPositions = kClusterSectors;

__device__ __forceinline__ uint64_t position_count(uint64_t n_sectors, uint32_t r) {
  return n_sectors > r ? (n_sectors - r + kPositions - 1) / kPositions : 0;
}

// kSlots = false: no slot records (hit_slot unused).
template <int kSig, int kLayout = kLayoutBucketed, bool kSlots = true>
__global__ __launch_bounds__(kScanThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_scan_tau(
    const uint8_t* __restrict__ image, uint64_t n_sectors, uint32_t tau0, uint64_t words_per_pos, uint32_t chunk,
    IndexView ix, uint64_t wt, uint64_t* __restrict__ tau_words, uint32_t* __restrict__ hit_slot) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kScanWaves * kTileLds];
  // the wave's index, uniform (so tile addresses stay in scalar registers)
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const uint32_t l = lane_id();
  uint8_t* my = lds + w * kTileLds;
  const uint32_t p = blockIdx.x % kPositions;
  const uint32_t r = (p - tau0) & (kPositions - 1);
  const uint64_t count = position_count(n_sectors, r);
  const uint64_t n_tiles = (count + kTileSectors - 1) / kTileSectors;
  // this position's slice of the filter
  const uint64_t* bloom = ix.bloom_tau ? ix.bloom_tau + ((uint64_t)p << ix.log2_bloom_tau) : ix.bloom;
  const uint32_t log2_bloom = ix.bloom_tau ? ix.log2_bloom_tau : ix.log2_bloom_words;
  const uint64_t n_waves = (uint64_t)(gridDim.x / kPositions) * kScanWaves;
  uint64_t g = ((uint64_t)(blockIdx.x / kPositions) * kScanWaves + w) * chunk;
  if (g >= n_tiles) return;
  auto next_of = [&](uint64_t t) {
    return ((t + 1) % chunk != 0) ? t + 1 : t + 1 + (n_waves - 1) * chunk;
  };
  auto rows_of = [&](uint64_t k) {
    const uint64_t first = k * kTileSectors;   // its first cluster among this position's
    const uint64_t rem = count - first;
    return ClusterStrideRows{image + (first * kPositions + r) * kSectorBytes,
                             rem >= kTileSectors ? kTileSectors : (uint32_t)rem};
  };
  ClusterStrideRows tr = rows_of(g);
  PhaseRegs A, B;
  load_phase<true>(tr, 0, A);
  while (true) {
    const uint64_t gn = next_of(g);
    const bool more = gn < n_tiles;
    const ClusterStrideRows tn = more ? rows_of(gn) : tr;
    auto prefetch = [&](PhaseRegs& R) { load_phase<true>(tn, 0, R); };   // unconditionally, as in k_scan
    uint64_t h;
    if constexpr (kSig == kSigCrc64)
      h = tile_crc_pipelined<true>(tr, my, A, B, prefetch);
    else
      h = tile_signature_pipelined<true>(tr, my, wt, A, B, prefetch);
    uint64_t hits = tile_probe<kLayout, kPositions, kSlots>(
        ix, h, p, false, kSlots ? hit_slot + (g * kTileSectors * kPositions + r) : nullptr, bloom, log2_bloom);
    if (tr.n_valid < kTileSectors) hits &= (1ull << tr.n_valid) - 1ull;
    if (l == 0) tau_words[p * words_per_pos + g] = hits;
    if (!more) break;
    g = gn;
    tr = tn;
  }
}

}  // namespace carve
