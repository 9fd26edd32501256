// Kernels and C-ABI host runtime of the carving library (gfx950).
//
// A scan covers one image or a batch of images. Their sectors form one tile
// space: image after image, each padded to whole 64-sector tiles. Every
// kernel below indexes that space, so a batch of uneven images costs no more
// launches than one image. A fragment scan (Section 5) uses the same space
// with 64-byte windows at 4-byte steps as its units.
//
// Pipeline of a scan (Sections 3.1-3.2):
//   k_scan<kFlags>    sector loads -> djb2-64 or CRC-64 -> cluster position ->
//                     index probe (bucketed, linear or sorted layout, Bloom
//                     prefilter) -> one 64-bit hit word per tile (ballot); the
//                     matched slot of each flagged sector is recorded
//                     (carve_scan_kernel.h; k_frag_scan in
//                     carve_fragment_kernel.h for fragments)
//   k_reduce / k_scan_blocks / k_apply<EmitIds>   popcount prefix ->
//                     ascending flagged ids (per image, image order)
//   k_image_offsets   (batches) where each image's ids start
// Confirmation (Section 3.1), from the slot each flagged unit matched:
//   k_confirm_count   byte comparison with every compatible candidate
//   prefix sum        output offsets (counts read on the device)
//   k_confirm_emit    ordered match records
//   k_stage_out       (server) counts, ids and records into pinned host memory
// Index build (Section 3.1, Eq. (3)):
//   k_master_meta, k_scan<kSigs> / k_frag_sigs, k_insert, k_narrow_masks,
//   k_scatter, k_sort_segments, k_bloom_build; k_occupied, k_insert_linear and
//   a radix sort for the other layouts; k_lds_filter_build for fragments.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "../../include/carve.h"
#include "carve_device.h"
#include "carve_internal.h"
#include "carve_scan_kernel.h"
#include "carve_fragment_kernel.h"

using namespace carve;

// Work buffers of scan_image_noalloc, for callers that cannot allocate: hit
// words (and the position-split scan's per-position words) of images up to
// 2^27 sectors, and the compaction's chunk sums. Every GPU that runs the
// library holds its own copy until the process ends. In host code this name
// is a host-side stand-in, never a device address: kernels get the address
// that noalloc_scratch() looks up per device.
constexpr uint64_t kNoAllocMaxSectors = 1ull << 27;                        // 64 GiB of image
constexpr uint64_t kNoAllocMaxWords = kNoAllocMaxSectors / kTileSectors;    // 2^21 hit words
constexpr uint64_t kNoAllocMaxChunks = kNoAllocMaxWords / 1024;             // compaction chunks of 1024 words
constexpr uint64_t kNoAllocCounters = 256;   // the position-split scan's work-sharing counters
constexpr uint64_t kScratchWords = 2 * kNoAllocMaxWords + 2 * kNoAllocMaxChunks + kNoAllocCounters;   // 32 MiB + 34 KiB
static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace {

constexpr int kBlockThreads = 256;
constexpr int kItemsPerThread = 4;
constexpr int kItemsPerBlock = kBlockThreads * kItemsPerThread;   // 1024
static_assert(kNoAllocMaxChunks * kItemsPerBlock == kNoAllocMaxWords, "scratch holds every chunk sum");
static_assert(kNoAllocCounters == carve::kTauCounters, "scratch holds the split scan's counters");
static_assert((2 * kNoAllocMaxWords + 2 * kNoAllocMaxChunks) % carve::kCtrStride == 0, "counters on 256-byte lines");

constexpr uint32_t kNoSlot = 0xFFFFFFFFu;   // master whose key could not be placed

// A scan object's device counters: [0] flagged units, [1] confirmed records,
// [kConfirmedWord] 1 once a confirmation ran after the latest scan. Every
// scan's compaction clears the marker on the device, so a scan replayed from a
// captured graph (which runs no host code) still invalidates an earlier
// confirmation; the host checks it before reusing one.
constexpr uint32_t kConfirmedWord = 2;

// Timed launches whose kernel durations a scan object keeps (the most recent).
constexpr uint64_t kTimedRing = 256;

// -------------------------------------------------------- prefix sums
// An item count known on the host (dev == null) or read on the device, so work
// sized by a count the host has not seen can be enqueued without waiting.
struct Count {
  uint64_t v;            // the count, or with dev: the most the buffers have room for
  const uint64_t* dev;
  __device__ __forceinline__ uint64_t get() const {
    if (!dev) return v;
    const uint64_t n = *dev;
    return n < v ? n : v;
  }
};

struct U32Items {
  const uint32_t* v;
  __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return v[i]; }
};
struct PopcountItems {
  const uint64_t* words;
  __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return (uint64_t)__popcll(words[i]); }
};
// After a position-split scan: hit word w of the image (sectors 64w..64w+63)
// gathered from the per-position words. Sector 64w + 8m + r sits at position
// (r + tau0) mod 8, in that position's tile w/8, bit 8(w mod 8) + m: byte
// w mod 8 of the 8 positions' words, an 8 x 8 bit matrix, transposed. Writes
// the word to the bitmap (the last one cut at the image's end) and counts it.
struct TauMergeItems {
  const uint64_t* tau_words;
  uint64_t words_per_pos;
  uint64_t* bitmap;
  uint64_t n_words;
  uint32_t tau0;
  uint32_t last_bits;   // valid bits of the last word, 0 = all 64
  __device__ __forceinline__ uint64_t operator()(uint64_t w) const {
    const uint64_t k = w / 8;
    const uint32_t sh = 8u * (uint32_t)(w % 8);
    uint64_t x = 0;
#pragma unroll
    for (uint32_t r = 0; r < 8; ++r) {
      const uint32_t p = (r + tau0) & 7u;
      x |= ((tau_words[p * words_per_pos + k] >> sh) & 0xFFull) << (8 * r);
    }
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;   // bit 8r + m -> bit 8m + r
    x ^= t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x ^= t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x ^= t ^ (t << 28);
    if (w == n_words - 1 && last_bits) x &= (1ull << last_bits) - 1ull;
    bitmap[w] = x;
    return (uint64_t)__popcll(x);
  }
};

// Items are taken in chunks of kItemsPerBlock, chunk c = items [c kItemsPerBlock,
// (c + 1) kItemsPerBlock); a block handles chunks blockIdx.x, + gridDim.x, ...
// so a grid sized for a count read on the device need not cover its upper
// bound. Chunks past the count are not touched (their sums are not scanned).
// Within a chunk, consecutive threads take consecutive items (the sum does not
// depend on the order), so every load instruction is coalesced.
template <class Items>
__global__ __launch_bounds__(kBlockThreads) void k_reduce(Items items, Count count, uint64_t* __restrict__ blk_sums) {
  __shared__ uint64_t lds_w[kBlockThreads / kWave];
  const uint64_t n = count.get();
  for (uint64_t c = blockIdx.x; c * kItemsPerBlock < n; c += gridDim.x) {
    const uint64_t base = c * kItemsPerBlock + threadIdx.x;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const uint64_t i = base + (uint64_t)k * kBlockThreads;
      if (i < n) s += items(i);
    }
    uint64_t total;
    block_exclusive_scan<kBlockThreads>(s, lds_w, &total);
    if (threadIdx.x == 0) blk_sums[c] = total;
  }
}

// One block: exclusive offsets of the block sums; total into *total. Only
// the blocks that hold items are scanned (a count read on the device can be
// far below the capacity the launches were sized for). A scan's compaction
// also clears its confirmation marker (*clear, see kConfirmedWord). Each
// thread takes a run of kScanRun consecutive sums per pass, its loads issued
// together, so a pass of 4096 sums costs one memory round trip (a pass of 256,
// one sum per thread, made the 8192 sums of a 2 GiB fragment image 23 us).
constexpr int kScanRun = 16;
__global__ __launch_bounds__(kBlockThreads) void k_scan_blocks(const uint64_t* __restrict__ blk_sums, Count items,
                                                              uint64_t* __restrict__ blk_off,
                                                              uint64_t* __restrict__ total,
                                                              uint64_t* __restrict__ clear = nullptr) {
  __shared__ uint64_t lds_w[kBlockThreads / kWave];
  const uint64_t n_blk = (items.get() + kItemsPerBlock - 1) / kItemsPerBlock;
  uint64_t carry = 0;
  for (uint64_t b0 = 0; b0 < n_blk; b0 += (uint64_t)kBlockThreads * kScanRun) {
    const uint64_t first = b0 + (uint64_t)threadIdx.x * kScanRun;
    uint64_t v[kScanRun];
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) v[k] = first + k < n_blk ? blk_sums[first + k] : 0;
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) run += v[k];
    uint64_t t;
    uint64_t off = carry + block_exclusive_scan<kBlockThreads>(run, lds_w, &t);
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) {
      if (first + k < n_blk) blk_off[first + k] = off;
      off += v[k];
    }
    carry += t;
  }
  if (threadIdx.x == 0) {
    *total = carry;
    if (clear) *clear = 0;
  }
}

// Hit words -> ascending ids of the flagged sectors, relative to their image
// (and, for batches, the image of each); ids at positions cap and beyond are
// not written (the count is still complete). An Emit type gives k_apply an item's
// raw value (load), its count (count_of; 0 for the value 0) and what to write
// for it at its exclusive position (emit); finish(n, end) runs once per scan
// of n items, with end = the total.
template <class Src>
struct EmitIds {
  static constexpr bool kDenseOut = false;   // a variable number of records per item
  Src src;
  const uint64_t* words;
  uint64_t* ids;
  uint32_t* img_of;   // null for one image
  uint64_t cap;       // room in ids (and img_of)
  __device__ __forceinline__ uint64_t load(uint64_t i) const { return words[i]; }
  __device__ __forceinline__ uint64_t count_of(uint64_t x) const { return (uint64_t)__popcll(x); }
  __device__ __forceinline__ void emit(uint64_t i, uint64_t x, uint64_t pos) const {
    if (!x || pos >= cap) return;
    const uint32_t im = src.image_of_tile(i);
    const uint64_t first = (i - src.image(im).tile_begin) * kTileSectors;
    while (x && pos < cap) {
      const int b = __ffsll((long long)x) - 1;
      ids[pos] = first + (uint64_t)b;
      if (img_of) img_of[pos] = im;
      ++pos;
      x &= x - 1;
    }
  }
  __device__ __forceinline__ void finish(uint64_t, uint64_t) const {}
};
// u32 counts -> exclusive offsets (out[n] = total).
template <class T>
struct EmitOffsets {
  static constexpr bool kDenseOut = true;   // out[i] for every item i: k_apply stores it coalesced
  const uint32_t* v;
  T* out;
  __device__ __forceinline__ uint64_t load(uint64_t i) const { return v[i]; }
  __device__ __forceinline__ uint64_t count_of(uint64_t x) const { return x; }
  __device__ __forceinline__ void emit(uint64_t i, uint64_t, uint64_t pos) const { out[i] = (T)pos; }
  __device__ __forceinline__ void finish(uint64_t n, uint64_t end) const { out[n] = (T)end; }
};

// A chunk's items go through LDS: loaded coalesced (consecutive threads,
// consecutive items), then each thread takes its kItemsPerThread consecutive
// items for the ordered scan. One pad word per 32 spreads a thread's reads
// over the LDS banks.
__device__ __forceinline__ uint32_t stage_index(uint32_t j) { return j + (j >> 5); }
constexpr uint32_t kStageWords = kItemsPerBlock + kItemsPerBlock / 32;

// Chunks as in k_reduce.
template <class Emit>
__global__ __launch_bounds__(kBlockThreads) void k_apply(Emit e, Count count, const uint64_t* __restrict__ blk_off) {
  __shared__ uint64_t lds_w[kBlockThreads / kWave];
  __shared__ uint64_t stage[kStageWords];
  const uint64_t n = count.get();
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) e.finish(0, 0);
    return;
  }
  for (uint64_t ch = blockIdx.x; ch * kItemsPerBlock < n; ch += gridDim.x) {
    const uint64_t c0 = ch * kItemsPerBlock;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      const uint32_t j = (uint32_t)k * kBlockThreads + threadIdx.x;
      stage[stage_index(j)] = c0 + j < n ? e.load(c0 + j) : 0;
    }
    __syncthreads();
    const uint32_t j0 = threadIdx.x * kItemsPerThread;
    uint64_t x[kItemsPerThread], c[kItemsPerThread];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItemsPerThread; ++k) {
      x[k] = stage[stage_index(j0 + k)];
      c[k] = e.count_of(x[k]);
      s += c[k];
    }
    // (the scan's barriers also keep the next chunk's stores behind these reads)
    uint64_t total;
    uint64_t pos = blk_off[ch] + block_exclusive_scan<kBlockThreads>(s, lds_w, &total);
    if constexpr (Emit::kDenseOut) {
      // one output per item: the positions go back through LDS (every thread
      // has read its items: the scan's barriers) and out in item order
#pragma unroll
      for (int k = 0; k < kItemsPerThread; ++k) {
        stage[stage_index(j0 + k)] = pos;
        if (c0 + j0 + k == n - 1) e.finish(n, pos + c[k]);
        pos += c[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kItemsPerThread; ++k) {
        const uint32_t j = (uint32_t)k * kBlockThreads + threadIdx.x;
        if (c0 + j < n) e.emit(c0 + j, 0, stage[stage_index(j)]);
      }
      __syncthreads();   // before the next chunk's loads overwrite the stage
    } else {
#pragma unroll
      for (int k = 0; k < kItemsPerThread; ++k) {
        const uint64_t i = c0 + j0 + k;
        if (i < n) {
          e.emit(i, x[k], pos);
          pos += c[k];
          if (i == n - 1) e.finish(n, pos);
        }
      }
    }
  }
}

// Batches: first flagged-id position of each image (img_off[n] = total), from
// the block offsets of the compaction and the words of the image's block that
// precede its first tile. One wave per image: its lanes popcount those words
// (at most kItemsPerBlock - 1) in strides of the wave, then add up.
__global__ void k_image_offsets(ManyImages src, const uint64_t* __restrict__ words,
                                const uint64_t* __restrict__ blk_off, const uint64_t* __restrict__ total,
                                uint64_t* __restrict__ img_off) {
  const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;   // uniform in the wave
  const uint32_t lane = threadIdx.x % kWave;
  if (i > src.n) return;
  const uint64_t w = src.d[i].tile_begin;
  if (w >= src.d[src.n].tile_begin) {
    if (lane == 0) img_off[i] = *total;
    return;
  }
  const uint64_t b = w / kItemsPerBlock;
  uint32_t c = 0;
  for (uint64_t k = b * kItemsPerBlock + lane; k < w; k += kWave) c += (uint32_t)__popcll(words[k]);
  for (int o = kWave / 2; o; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o);
  if (lane == 0) img_off[i] = blk_off[b] + c;
}

// Batches, for callers that cannot wait: totals, per-image offsets, ids and
// records written straight into host-visible memory, each up to its capacity.
// Records are copied as 64-bit words (a record is three of them).
__global__ void k_stage_out(const uint64_t* __restrict__ counts, int with_matches, uint32_t n_images,
                            const uint64_t* __restrict__ img_off, const uint64_t* __restrict__ ids,
                            const uint64_t* __restrict__ rec_words, uint64_t rec_room, uint64_t* totals,
                            uint64_t* h_off, uint64_t* h_ids, uint64_t ids_cap, uint64_t* h_rec_words,
                            uint64_t rec_cap) {
  static_assert(sizeof(carve_batch_match) == 24, "a batch record is three 64-bit words");
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t nf = counts[0];
  const uint64_t nm = with_matches ? counts[1] : 0;
  if (t == 0) {
    totals[0] = nf;
    totals[1] = nm;
  }
  for (uint64_t i = t; i <= n_images; i += stride) h_off[i] = img_off[i];
  const uint64_t kf = nf < ids_cap ? nf : ids_cap;
  for (uint64_t i = t; i < kf; i += stride) h_ids[i] = ids[i];
  uint64_t km = nm < rec_room ? nm : rec_room;
  if (km > rec_cap) km = rec_cap;
  for (uint64_t i = t; i < 3 * km; i += stride) h_rec_words[i] = rec_words[i];
}

// A fill kernel rather than hipMemsetAsync, so the scan sequence can be
// captured in a HIP graph.
__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

struct NonEmptyLists {
  const uint32_t* off;
  __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return off[i + 1] != off[i] ? 1u : 0u; }
};

// ------------------------------------------------------------ build
__global__ void k_master_meta(const uint64_t* __restrict__ off, uint32_t n_files, uint64_t n_masters,
                              uint32_t* __restrict__ m_file, uint32_t* __restrict__ m_k) {
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_masters) return;
  uint32_t lo = 0, hi = n_files - 1;   // last f with off[f] <= m
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= m) lo = mid; else hi = mid - 1;
  }
  m_file[m] = lo;
  m_k[m] = (uint32_t)(m - off[lo]);
}

// Insert every master signature (Eq. (3) at bucket granularity): first free
// slot of the home bucket, else of the next bucket, and so on. Equal
// signatures share one slot. Records the slot of each master, the cluster
// positions present per slot and the number of masters per slot.
__global__ void k_insert(const uint64_t* __restrict__ sig, const uint32_t* __restrict__ m_k, uint64_t n_masters,
                         uint64_t* keys, uint32_t log2_buckets, uint32_t* tau_mask, uint32_t* cnt,
                         uint32_t* __restrict__ m_slot, uint32_t* overflow, uint32_t* failed) {
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_masters) return;
  const uint64_t h = sig[m];
  const uint64_t n_slots = (uint64_t)kBucketSlots << log2_buckets;
  uint64_t slot = n_slots;   // side slot of signature 0
  if (h != kEmptyKey) {
    const uint32_t nb_mask = (1u << log2_buckets) - 1u;
    const uint32_t home = bucket_of(h, log2_buckets);
    uint32_t b = home;
    bool placed = false;
    for (uint32_t it = 0; it <= nb_mask && !placed; ++it) {
      for (uint32_t sl = 0; sl < kBucketSlots; ++sl) {
        unsigned long long* p = (unsigned long long*)(keys + (uint64_t)b * kBucketSlots + sl);
        unsigned long long cur = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == kEmptyKey) cur = atomicCAS(p, (unsigned long long)kEmptyKey, (unsigned long long)h);
        if (cur == kEmptyKey || cur == h) {   // claimed it, or it already holds h
          slot = (uint64_t)b * kBucketSlots + sl;
          placed = true;
          break;
        }
      }
      if (!placed) b = (b + 1) & nb_mask;
    }
    if (!placed) {   // only possible with a full table; the load ceiling rules it out
      atomicAdd(failed, 1u);
      m_slot[m] = kNoSlot;
      return;
    }
    if (b != home) atomicAdd(overflow, 1u);
  }
  m_slot[m] = (uint32_t)slot;
  atomicOr(&tau_mask[slot], 1u << (m_k[m] & (kClusterSectors - 1)));
  atomicAdd(&cnt[slot], 1u);
}

// Bloom filter of the table's keys (signature 0 is kept apart and not in it).
__global__ void k_bloom_build(const uint64_t* __restrict__ keys, uint64_t n_slots, uint32_t log2_words,
                              uint64_t* bloom) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const uint64_t h = keys[i];
  if (h == kEmptyKey) return;
  uint32_t w;
  uint64_t bits;
  bloom_place(h, log2_words, &w, &bits);
  atomicOr((unsigned long long*)(bloom + w), (unsigned long long)bits);
}

// The filter split by cluster position: slice t holds the keys with a master
// at position t (placed like the whole filter, in 2^log2_words words). Built
// for every sector index with a filter. A filter of 2^kSplitMinLog2 words
// (4 MiB) or more cannot stay in an XCD's 4 MB L2 beside the streamed image,
// so per-cluster scans of one image run position-split (k_scan_tau) by
// default, each XCD holding one eighth; smaller filters stay in L2 whole and
// the contiguous scan is faster with them (1.29 vs 1.35 ms on the 8 GiB mid
// workload, 2 MiB filter; the split took the 64 GiB large workload, 8 MiB
// filter, from 11.79 to 10.86 ms). carve_scan_config.split overrides it.
constexpr uint32_t kSplitMinLog2 = 19;
__global__ void k_bloom_tau_build(const uint64_t* __restrict__ keys, const uint8_t* __restrict__ tau_mask,
                                  uint64_t n_slots, uint32_t log2_words, uint64_t* bloom_tau) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slots) return;
  const uint64_t h = keys[i];
  if (h == kEmptyKey) return;
  uint32_t w;
  uint64_t bits;
  bloom_place(h, log2_words, &w, &bits);
  for (uint32_t m = tau_mask[i]; m; m &= m - 1u)
    atomicOr((unsigned long long*)(bloom_tau + ((uint64_t)__builtin_ctz(m) << log2_words) + w),
             (unsigned long long)bits);
}

// The fragment scan's two filters (placed by frag_lds_place and
// frag_bloom_place from a signature's filter key; 32-bit words), from the
// table's keys; with_zero: signature 0 is a master's too (it has no slot), so
// the bits of its key are set as well.
__global__ void k_lds_filter_build(const uint64_t* __restrict__ keys, uint64_t n_slots, uint32_t n_words,
                                   uint32_t with_zero, uint32_t* filter) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t w, bits;
  if (i == 0 && with_zero) {
    frag_lds_place(frag_filter_key(0), n_words, &w, &bits);
    atomicOr(&filter[w], bits);
  }
  if (i >= n_slots || keys[i] == kEmptyKey) return;
  frag_lds_place(frag_filter_key(keys[i]), n_words, &w, &bits);
  atomicOr(&filter[w], bits);
}
__global__ void k_frag_bloom_build(const uint64_t* __restrict__ keys, uint64_t n_slots, uint32_t log2_words,
                                   uint32_t with_zero, uint32_t* bloom) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t w, bits;
  if (i == 0 && with_zero) {
    frag_bloom_place(frag_filter_key(0), log2_words, &w, &bits);
    atomicOr(&bloom[w], bits);
  }
  if (i >= n_slots || keys[i] == kEmptyKey) return;
  frag_bloom_place(frag_filter_key(keys[i]), log2_words, &w, &bits);
  atomicOr(&bloom[w], bits);
}

// Other probe layouts. The distinct signatures of the table with their slots
// (any order).
__global__ void k_occupied(const uint64_t* __restrict__ keys, uint64_t n_slots, uint64_t* __restrict__ out_keys,
                           uint32_t* __restrict__ out_slots, unsigned long long* __restrict__ count) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_slots || keys[t] == kEmptyKey) return;
  const unsigned long long i = atomicAdd(count, 1ull);
  out_keys[i] = keys[t];
  out_slots[i] = (uint32_t)t;
}

// The paper's table (Eq. (3)): a key goes to the slot given by its w low bits,
// or the first free slot after it. Keys are distinct, so a slot taken by
// another key only means: try the next one.
__global__ void k_insert_linear(const uint64_t* __restrict__ in_keys, const uint32_t* __restrict__ in_slots, uint64_t n,
                                uint64_t* lin_keys, uint32_t* __restrict__ lin_slot, uint32_t log2_lin) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t h = in_keys[t];
  const uint64_t mask = (1ull << log2_lin) - 1ull;
  uint64_t s = h & mask;
  for (uint64_t it = 0; it <= mask; ++it) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&lin_keys[s], (unsigned long long)kEmptyKey, (unsigned long long)h);
    if (prev == kEmptyKey) {
      lin_slot[s] = in_slots[t];
      return;
    }
    s = (s + 1) & mask;
  }
}

__global__ void k_narrow_masks(const uint32_t* __restrict__ m32, uint64_t n, uint8_t* __restrict__ m8) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m8[i] = (uint8_t)m32[i];
}

__global__ void k_scatter(const uint32_t* __restrict__ m_slot, uint64_t n_masters, const uint32_t* __restrict__ cand_off,
                          uint32_t* cursor, uint32_t* __restrict__ unsorted) {
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_masters) return;
  const uint32_t s = m_slot[m];
  if (s == kNoSlot) return;
  unsorted[cand_off[s] + atomicAdd(&cursor[s], 1u)] = (uint32_t)m;
}

// Candidate lists in ascending master order (so matches come out ordered by
// file, then sector in file): one wave per list; each element goes to its
// rank among the list's (distinct) elements, from `unsorted` into `cand`.
__global__ __launch_bounds__(kBlockThreads) void k_sort_segments(const uint32_t* __restrict__ cand_off, uint64_t n_lists,
                                                                const uint32_t* __restrict__ unsorted,
                                                                uint32_t* __restrict__ cand) {
  const uint32_t l = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (kBlockThreads / kWave);
  for (uint64_t s = (uint64_t)blockIdx.x * (kBlockThreads / kWave) + threadIdx.x / kWave; s < n_lists; s += waves) {
    const uint32_t a = cand_off[s], e = cand_off[s + 1];
    for (uint32_t i = a + l; i < e; i += kWave) {
      const uint32_t v = unsorted[i];
      uint32_t rank = 0;
      for (uint32_t j = a; j < e; ++j) rank += unsorted[j] < v;
      cand[a + rank] = v;
    }
  }
}

// -------------------------------------------------------- confirmation
struct ConfirmView {
  const uint32_t* cand_off;   // n_slots + 2: candidate list of each slot (+ signature 0)
  const uint32_t* cand;       // master sector ids, ascending within each list
  const uint32_t* m_file;     // file of each master sector
  const uint32_t* m_k;        // sector in file of each master sector
  const uint8_t* masters;     // packed master sectors
};

// Lanes per flagged unit in the confirmation count: 8 x 64 B for a sector;
// one lane for a 64-byte window. The time goes to a chain of dependent loads
// (id -> slot -> candidate list -> master), so more units in flight per wave
// beat spreading one compare over more lanes.
template <class Src>
constexpr uint32_t confirm_lanes() {
  return Src::kUnitBytes == kSectorBytes ? 8u : 1u;
}

// The match mask of a flagged unit: bit r = the r-th compatible candidate is
// equal, for the first kMaskRanks of them (later ones are compared again when
// emitted). Windows (any position: every candidate is compatible) with at
// most 32 candidates use a short form instead: bit 63 set, the list's first
// index in bits 32-62, the equality mask of the whole list in bits 0-31; so
// emitting needs neither the slot nor the list offsets.
template <class Src>
constexpr uint32_t mask_ranks() {
  return Src::kUnitBytes == kSectorBytes ? 64u : 63u;
}
constexpr uint64_t kShortMask = 1ull << 63;
constexpr uint32_t kShortMaxList = 32;

__device__ __forceinline__ bool compatible(const ConfirmView& cv, uint32_t m, uint32_t tau, uint32_t any_tau) {
  return any_tau || (cv.m_k[m] & (kClusterSectors - 1)) == tau;
}

// The i-th flagged sector of a scan: its bytes, cluster position, rule and slot.
struct Flagged {
  const uint8_t* bytes;
  uint64_t j;       // sector id in its image
  uint32_t image;
  uint32_t tau;
  uint32_t any_tau;
  uint32_t slot;
};

template <class Src>
__device__ __forceinline__ Flagged flagged(const Src& src, const uint64_t* ids, const uint32_t* img_of,
                                           const uint32_t* hit_slot, uint64_t i) {
  const uint32_t im = img_of ? img_of[i] : 0u;
  const ImageDesc& d = src.image(im);
  const uint64_t j = ids[i];
  return Flagged{d.base + j * Src::kUnitStride, j, im, (uint32_t)((j + d.tau0) & (kClusterSectors - 1)),
                 Src::kAnyPosition ? 1u : d.any_tau, hit_slot[d.tile_begin * kTileSectors + j]};
}

// A group of lanes per flagged sector (8), or one lane per flagged window:
// compare its bytes with every candidate master unit of its slot at a
// compatible cluster position. Records the number of equal ones and the match
// mask (mask_ranks).
template <class Src>
__global__ __launch_bounds__(kBlockThreads) void k_confirm_count(Src src, const uint64_t* __restrict__ ids,
                                                                const uint32_t* __restrict__ img_of,
                                                                Count count,
                                                                const uint32_t* __restrict__ hit_slot, ConfirmView cv,
                                                                uint32_t* __restrict__ n_match,
                                                                uint64_t* __restrict__ match_mask,
                                                                uint64_t* __restrict__ confirmed) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *confirmed = 1;   // stream order: after the scan that cleared it
  constexpr uint32_t kLanes = confirm_lanes<Src>();
  constexpr uint64_t kGroupMask = (1ull << kLanes) - 1ull;
  const uint64_t n_flagged = count.get();
  if constexpr (kLanes == 1) {   // 64-byte windows (4-byte aligned) against 64-byte aligned master fragments
    static_assert(Src::kUnitBytes == 64, "one lane per unit only for 64-byte units");
    for (uint64_t i = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x; i < n_flagged;
         i += (uint64_t)gridDim.x * kBlockThreads) {
      const Flagged f = flagged(src, ids, img_of, hit_slot, i);
      uint32_t w[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) w[k] = ((const uint32_t*)f.bytes)[k];
      static_assert(Src::kAnyPosition, "windows match at any position");
      uint32_t cnt = 0, rank = 0;
      uint64_t mask = 0;
      const uint32_t c0 = cv.cand_off[f.slot], e = cv.cand_off[f.slot + 1];
      for (uint32_t c = c0; c < e; ++c) {   // every candidate is compatible: rank = c - c0
        const uint32_t m = cv.cand[c];
        const u32x4* q = (const u32x4*)(cv.masters + (uint64_t)m * Src::kUnitBytes);
        uint32_t x = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const u32x4 v = q[k];
          x |= (v.x ^ w[4 * k]) | (v.y ^ w[4 * k + 1]) | (v.z ^ w[4 * k + 2]) | (v.w ^ w[4 * k + 3]);
        }
        if (x == 0) {
          ++cnt;
          if (rank < mask_ranks<Src>()) mask |= 1ull << rank;
        }
        ++rank;
      }
      if (e - c0 <= kShortMaxList && c0 < (1u << 31)) mask |= kShortMask | ((uint64_t)c0 << 32);
      n_match[i] = cnt;
      match_mask[i] = mask;
    }
  } else {   // sectors: lane gl of a group compares the 16-byte chunks gl, gl + kLanes, ...
    static_assert(Src::kUnitBytes == kSectorBytes, "lane groups only for sectors");
    constexpr uint32_t kChunks = kSectorBytes / 16 / kLanes;
    const uint32_t l = lane_id();
    const uint32_t g = l / kLanes, gl = l % kLanes;
    const uint64_t per_block = kBlockThreads / kLanes;
    const uint64_t n_groups = (uint64_t)gridDim.x * per_block;
    for (uint64_t i = (uint64_t)blockIdx.x * per_block + threadIdx.x / kLanes; i < n_flagged; i += n_groups) {
      const Flagged f = flagged(src, ids, img_of, hit_slot, i);
      const u32x4* d = (const u32x4*)f.bytes + gl;
      u32x4 dv[kChunks];
#pragma unroll
      for (uint32_t k = 0; k < kChunks; ++k) dv[k] = d[k * kLanes];
      uint32_t cnt = 0, rank = 0;
      uint64_t mask = 0;
      for (uint32_t c = cv.cand_off[f.slot], e = cv.cand_off[f.slot + 1]; c < e; ++c) {
        const uint32_t m = cv.cand[c];
        if (!compatible(cv, m, f.tau, f.any_tau)) continue;   // same decision in all lanes of the group
        const u32x4* q = (const u32x4*)(cv.masters + (uint64_t)m * kSectorBytes) + gl;
        u32x4 x = dv[0] ^ q[0];
#pragma unroll
        for (uint32_t k = 1; k < kChunks; ++k) x |= dv[k] ^ q[k * kLanes];
        const uint64_t diff = ballot((x.x | x.y | x.z | x.w) != 0);
        if (((diff >> (g * kLanes)) & kGroupMask) == 0) {
          ++cnt;
          if (rank < mask_ranks<Src>()) mask |= 1ull << rank;
        }
        ++rank;
      }
      if (gl == 0) {
        n_match[i] = cnt;
        match_mask[i] = mask;
      }
    }
  }
}

template <uint32_t kBytes>
__device__ __forceinline__ bool units_equal(const uint8_t* a, const uint8_t* b) {
  const uint32_t* x = (const uint32_t*)a;   // 4-byte aligned (windows start on 4-byte boundaries)
  const uint32_t* y = (const uint32_t*)b;
  for (uint32_t k = 0; k < kBytes / 4; ++k)
    if (x[k] != y[k]) return false;
  return true;
}

__device__ __forceinline__ void put_record(carve_match* out, uint64_t pos, uint64_t j, uint32_t f, uint32_t k,
                                           uint32_t) {
  carve_match r;
  r.disk_sector = j;
  r.file_id = f;
  r.sector_in_file = k;
  out[pos] = r;
}
__device__ __forceinline__ void put_record(carve_batch_match* out, uint64_t pos, uint64_t j, uint32_t f, uint32_t k,
                                           uint32_t image) {
  carve_batch_match r;
  r.disk_sector = j;
  r.file_id = f;
  r.sector_in_file = k;
  r.image = image;
  r.reserved = 0;
  out[pos] = r;
}

// Thread per flagged sector (grid-stride): its confirmed matches, in
// candidate (= file, sector-in-file) order, at its offset of the output;
// records past `cap` are counted but not written.
template <class Src, class Rec>
__global__ void k_confirm_emit(Src src, const uint64_t* __restrict__ ids, const uint32_t* __restrict__ img_of,
                               Count count, const uint32_t* __restrict__ hit_slot, ConfirmView cv,
                               const uint64_t* __restrict__ match_mask, const uint64_t* __restrict__ out_off,
                               Rec* __restrict__ out, uint64_t cap) {
  const uint64_t n_flagged = count.get();
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_flagged;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t pos = out_off[i];
    if (pos >= cap) continue;
    const uint64_t mask = match_mask[i];
    if constexpr (Src::kUnitBytes != kSectorBytes) {
      if (mask & kShortMask) {   // the list start and its equality mask
        const uint32_t c0 = (uint32_t)(mask >> 32) & 0x7FFFFFFFu;
        const uint64_t j = ids[i];
        const uint32_t im = img_of ? img_of[i] : 0u;
        for (uint32_t bits = (uint32_t)mask; bits && pos < cap; bits &= bits - 1u) {
          const uint32_t m = cv.cand[c0 + (uint32_t)__builtin_ctz(bits)];
          put_record(out, pos++, j, cv.m_file[m], cv.m_k[m], im);
        }
        continue;
      }
    }
    const Flagged f = flagged(src, ids, img_of, hit_slot, i);
    uint32_t rank = 0;
    for (uint32_t c = cv.cand_off[f.slot], e = cv.cand_off[f.slot + 1]; c < e && pos < cap; ++c) {
      const uint32_t m = cv.cand[c];
      if (!compatible(cv, m, f.tau, f.any_tau)) continue;
      const bool eq = rank < mask_ranks<Src>()
                          ? ((mask >> rank) & 1u) != 0
                          : units_equal<Src::kUnitBytes>(f.bytes, cv.masters + (uint64_t)m * Src::kUnitBytes);
      ++rank;
      if (eq) put_record(out, pos++, f.j, cv.m_file[m], cv.m_k[m], f.image);
    }
  }
}

// Copies ids [0, min(*count, cap)); cap is at most the ids the scan has room for.
__global__ void k_copy_ids(const uint64_t* __restrict__ ids, const uint64_t* __restrict__ count, uint64_t cap,
                           uint64_t* __restrict__ out) {
  const uint64_t n = *count < cap ? *count : cap;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = ids[i];
}

// ============================================================ host side
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(CARVE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CARVE_TRY(expr)            \
  do {                             \
    int r_ = (expr);               \
    if (r_ != CARVE_OK) return r_; \
  } while (0)

// Device buffer that grows on demand (contents not preserved).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int reserve(size_t need) {
    if (need <= bytes) return CARVE_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t sz = need < 256 ? 256 : need;
    if (hipMalloc(&p, sz) != hipSuccess) return fail(CARVE_ENOMEM, "hipMalloc(%zu) failed", sz);
    bytes = sz;
    return CARVE_OK;
  }
  template <class T>
  T* as() const { return (T*)p; }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Pinned host buffer that grows on demand.
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int reserve(size_t need) {
    if (need <= bytes) return CARVE_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    size_t sz = need < 256 ? 256 : need;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return fail(CARVE_ENOMEM, "hipHostMalloc failed");
    bytes = sz;
    return CARVE_OK;
  }
  template <class T>
  T* as() const { return (T*)p; }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Device address, on the current device, of djb2's digit-plane weight table
// (0 on failure).
uint64_t weight_table() {
  static uint64_t ptr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_weights)) != hipSuccess) return 0;
    ptr[dev] = (uint64_t)(uintptr_t)p;
  }
  return ptr[dev];
}

// The table argument of the scan kernel for a signature kind: djb2's weights;
// the CRC needs none. Returns false when the table is unavailable.
bool sig_table(uint32_t kind, uint64_t* wt) {
  *wt = kind == CARVE_SIG_CRC64_ISO ? 0 : weight_table();
  return kind == CARVE_SIG_CRC64_ISO || *wt != 0;
}

// One scan kernel launch for the signature kind chosen at run time.
template <int kMode, class Src>
int launch_k_scan(uint32_t kind, const Src& src, uint64_t n_tiles, uint32_t chunk, uint32_t per_cu_cap,
                  const IndexView& ix, uint64_t wt, uint64_t* out, uint32_t* hit_slot, hipStream_t s,
                  uint32_t layout = CARVE_LAYOUT_BUCKETED);

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

// Resident blocks per CU of a kernel at a block size, queried once per
// (kernel, block size, device): the query costs more host time than a launch.
struct OccupancyEntry {
  const void* fn;
  int threads;
  int device;
  int per_cu;
};
std::mutex g_occ_mu;
std::vector<OccupancyEntry> g_occ;

template <class Kernel>
int blocks_per_cu(Kernel kernel, int threads) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const void* fn = (const void*)kernel;
  std::lock_guard<std::mutex> lock(g_occ_mu);
  for (const OccupancyEntry& e : g_occ)
    if (e.fn == fn && e.threads == threads && e.device == dev) return e.per_cu;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  g_occ.push_back(OccupancyEntry{fn, threads, dev, per_cu});
  return per_cu;
}

// Blocks of a persistent grid: as many as stay resident at once (capped by
// `per_cu_cap` when non-zero) so no block waits for a second round, and no
// more than the work needs.
template <class Kernel>
int resident_grid(Kernel kernel, int threads, uint64_t want, uint32_t per_cu_cap = 0) {
  int per_cu = blocks_per_cu(kernel, threads);
  if (per_cu_cap && (uint32_t)per_cu > per_cu_cap) per_cu = (int)per_cu_cap;
  const uint64_t cap = (uint64_t)device_cus() * (uint64_t)per_cu;
  return (int)(want < cap ? (want ? want : 1) : cap);
}

// Exclusive scan of n u32 counts into out[0..n] (out[n] = total); total also
// left in *d_total. ws holds the block sums and offsets. With n_dev, the count
// is read on the device and n is only its upper bound.
template <class T>
int scan_counts(const uint32_t* in, T* out, uint64_t n, uint64_t* d_total, DevBuf& ws, hipStream_t s,
                const uint64_t* n_dev = nullptr) {
  const uint64_t nb = cdiv(n ? n : 1, kItemsPerBlock);
  CARVE_TRY(ws.reserve(2 * nb * sizeof(uint64_t)));
  uint64_t* sums = ws.as<uint64_t>();
  uint64_t* offs = sums + nb;
  // a count read on the device is often far below n: a resident grid strides
  // over the chunks it has instead of launching a block per possible chunk
  const uint64_t g_red = n_dev ? (uint64_t)resident_grid(k_reduce<U32Items>, kBlockThreads, nb) : nb;
  const uint64_t g_app = n_dev ? (uint64_t)resident_grid(k_apply<EmitOffsets<T>>, kBlockThreads, nb) : nb;
  k_reduce<<<g_red, kBlockThreads, 0, s>>>(U32Items{in}, Count{n, n_dev}, sums);
  k_scan_blocks<<<1, kBlockThreads, 0, s>>>(sums, Count{n, n_dev}, offs, d_total);
  k_apply<<<g_app, kBlockThreads, 0, s>>>(EmitOffsets<T>{in, out}, Count{n, n_dev}, offs);   // also out[count]
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

template <int kMode, int kSig, int kLayout, class Src>
void launch_k_scan_as(const Src& src, uint64_t want, uint32_t chunk, uint32_t per_cu_cap, const IndexView& ix,
                      uint64_t wt, uint64_t* out, uint32_t* hit_slot, hipStream_t s) {
  const int grid = resident_grid(k_scan<kMode, kSig, Src, kLayout>, kScanThreads, want, per_cu_cap);
  k_scan<kMode, kSig, Src, kLayout><<<grid, kScanThreads, 0, s>>>(src, chunk, ix, wt, out, hit_slot);
}

template <int kMode, int kSig, class Src>
void launch_k_scan_sig(uint32_t layout, const Src& src, uint64_t want, uint32_t chunk, uint32_t per_cu_cap,
                       const IndexView& ix, uint64_t wt, uint64_t* out, uint32_t* hit_slot, hipStream_t s) {
  if constexpr (kMode == kFlags || kMode == kFlagBits) {
    if (layout == CARVE_LAYOUT_LINEAR)
      return launch_k_scan_as<kMode, kSig, kLayoutLinear>(src, want, chunk, per_cu_cap, ix, wt, out, hit_slot, s);
    if (layout == CARVE_LAYOUT_SORTED)
      return launch_k_scan_as<kMode, kSig, kLayoutSorted>(src, want, chunk, per_cu_cap, ix, wt, out, hit_slot, s);
  }
  launch_k_scan_as<kMode, kSig, kLayoutBucketed>(src, want, chunk, per_cu_cap, ix, wt, out, hit_slot, s);
}

template <int kMode, class Src>
int launch_k_scan(uint32_t kind, const Src& src, uint64_t n_tiles, uint32_t chunk, uint32_t per_cu_cap,
                  const IndexView& ix, uint64_t wt, uint64_t* out, uint32_t* hit_slot, hipStream_t s,
                  uint32_t layout) {
  const uint64_t want = cdiv(cdiv(n_tiles, chunk), kScanWaves);
  if (kind == CARVE_SIG_CRC64_ISO)
    launch_k_scan_sig<kMode, kSigCrc64>(layout, src, want, chunk, per_cu_cap, ix, wt, out, hit_slot, s);
  else
    launch_k_scan_sig<kMode, kSigDjb2>(layout, src, want, chunk, per_cu_cap, ix, wt, out, hit_slot, s);
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

// The position-split scan of one image (k_scan_tau): a persistent grid whose
// size is a multiple of 8, one eighth of it per cluster position.
template <int kSig, int kLayout, bool kSlots>
void launch_k_scan_tau_as(const ImageDesc& d, uint64_t words_per_pos, uint32_t chunk, uint32_t per_cu_cap,
                          const IndexView& ix, uint64_t wt, uint64_t* tau_words, uint32_t* hit_slot, uint64_t* ctr,
                          hipStream_t s) {
  const uint64_t want = kPositions * cdiv(cdiv(words_per_pos, chunk), kScanWaves);
  int grid = resident_grid(k_scan_tau<kSig, kLayout, kSlots>, kScanThreads, want, per_cu_cap);
  grid = grid < (int)kPositions ? (int)kPositions : grid - grid % (int)kPositions;
  k_fill_u64<<<1, 256, 0, s>>>(ctr, kTauCounters, 0);   // the work-sharing counters start at zero
  k_scan_tau<kSig, kLayout, kSlots><<<grid, kScanThreads, 0, s>>>(d.base, d.n_sectors, d.tau0, words_per_pos, chunk,
                                                                   ix, wt, tau_words, hit_slot,
                                                                   (unsigned int*)ctr);
}

template <int kSig, bool kSlots>
void launch_k_scan_tau_sig(uint32_t layout, const ImageDesc& d, uint64_t words_per_pos, uint32_t chunk,
                           uint32_t per_cu_cap, const IndexView& ix, uint64_t wt, uint64_t* tau_words,
                           uint32_t* hit_slot, uint64_t* ctr, hipStream_t s) {
  if (layout == CARVE_LAYOUT_LINEAR)
    return launch_k_scan_tau_as<kSig, kLayoutLinear, kSlots>(d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                              hit_slot, ctr, s);
  if (layout == CARVE_LAYOUT_SORTED)
    return launch_k_scan_tau_as<kSig, kLayoutSorted, kSlots>(d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                              hit_slot, ctr, s);
  launch_k_scan_tau_as<kSig, kLayoutBucketed, kSlots>(d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                       hit_slot, ctr, s);
}

// The position-split scan's work-sharing counters sit behind its hit words,
// on a 256-byte boundary.
uint64_t tau_counter_offset(uint64_t n_words) {
  return cdiv(kPositions * cdiv(n_words, kPositions), kCtrStride) * kCtrStride;
}
uint64_t* tau_counters(uint64_t* tau_words, uint64_t n_words) {
  return tau_words + tau_counter_offset(n_words);
}

// hit_slot null: no slot records (the flags are not confirmed afterwards). ctr: kTauCounters
// words, 256-byte aligned, for the work-sharing counters (cleared here).
int launch_k_scan_tau(uint32_t kind, uint32_t layout, const ImageDesc& d, uint64_t words_per_pos, uint32_t chunk,
                      uint32_t per_cu_cap, const IndexView& ix, uint64_t wt, uint64_t* tau_words, uint32_t* hit_slot,
                      uint64_t* ctr, hipStream_t s) {
  const bool crc = kind == CARVE_SIG_CRC64_ISO;
  if (hit_slot) {
    if (crc) launch_k_scan_tau_sig<kSigCrc64, true>(layout, d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                     hit_slot, ctr, s);
    else launch_k_scan_tau_sig<kSigDjb2, true>(layout, d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                hit_slot, ctr, s);
  } else {
    if (crc) launch_k_scan_tau_sig<kSigCrc64, false>(layout, d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                      nullptr, ctr, s);
    else launch_k_scan_tau_sig<kSigDjb2, false>(layout, d, words_per_pos, chunk, per_cu_cap, ix, wt, tau_words,
                                                 nullptr, ctr, s);
  }
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

}  // namespace

// ================================================================ objects
struct carve_index {
  int device = 0;
  uint64_t n_masters = 0;
  uint32_t n_files = 0;
  const uint8_t* masters = nullptr;
  uint32_t log2_buckets = 1;
  uint64_t n_slots = 0;
  uint32_t zero_sig_mask = 0;
  uint64_t n_unique = 0;
  uint64_t n_overflow = 0;
  uint64_t weights = 0;     // djb2's weight table (0 for the CRC)
  uint32_t sig_kind = CARVE_SIG_DJB2_64;
  uint32_t unit_bytes = kSectorBytes;   // master units: sectors, or 64-byte fragments
  uint32_t log2_bloom_words = 0;
  carve_scan_config cfg{};
  DevBuf keys, tau_mask, cand_off, cand, m_file, m_k, bloom;   // tau_mask: one byte per slot
  uint32_t layout = CARVE_LAYOUT_BUCKETED;
  DevBuf lin_keys, lin_slot, sorted_keys, sorted_slot;          // probe structures of the other layouts
  uint32_t log2_lin = 0, n_sorted = 0;
  DevBuf lds_filter;                                            // fragment indexes: first-level filter
  uint32_t lds_words = 0;
  DevBuf bloom_tau;                                             // sector indexes: the filter split by position
  uint32_t log2_bloom_tau = 0;
  IndexView view() const {
    return IndexView{keys.as<uint64_t>(), tau_mask.as<uint8_t>(), bloom.bytes ? bloom.as<uint64_t>() : nullptr,
                     log2_buckets, log2_bloom_words, zero_sig_mask, (uint32_t)n_slots,
                     lin_keys.as<uint64_t>(), lin_slot.as<uint32_t>(), log2_lin, n_sorted,
                     sorted_keys.as<uint64_t>(), sorted_slot.as<uint32_t>(), lds_filter.as<uint32_t>(),
                     lds_words, bloom_tau.bytes ? bloom_tau.as<uint64_t>() : nullptr, log2_bloom_tau};
  }
  ConfirmView cview() const {
    return ConfirmView{cand_off.as<uint32_t>(), cand.as<uint32_t>(), m_file.as<uint32_t>(), m_k.as<uint32_t>(),
                       masters};
  }
};

// Results of one scan (one image, or a batch of them).
struct carve_scan {
  int device = 0;
  hipStream_t stream = nullptr;
  const carve_index* idx = nullptr;
  bool batch = false;
  bool fragments = false;        // units are the 64-byte windows of one image
  uint64_t n_dwords = 0;         // fragments: whole 4-byte words of the image
  std::vector<ImageDesc> desc;   // n_images + 1 (the last: total tiles)
  uint32_t n_images = 0;
  uint64_t n_tiles = 0;
  uint64_t max_sectors = 0;      // largest id space of one image, for flagged_sectors' copy kernel
  uint32_t grid_per_cu = 0;      // scan blocks per CU for this object's launches; 0: the index's setting
  DevBuf d_desc;                 // batches: the descriptors on the device
  HostBuf h_desc;                // pinned staging for their upload
  std::vector<ImageDesc> uploaded;
  DevBuf bitmap, ws, ids, img_of, count, hit_slot, img_off;   // hit_slot: matched slot of each flagged sector
  DevBuf tau_words;   // one image, per-cluster rule: the hit words of the position-split scan
  HostBuf h_small, h_img_off;                                 // pinned readbacks
  // confirmation: records go to `matches` (rec_cap of them) or to a caller's
  // device buffer (conf_dest, conf_dest_cap records)
  DevBuf n_match, match_mask, out_off, matches, cws;
  uint64_t conf_room = 0;        // flagged units the last enqueued confirmation had room for
  uint64_t conf_need = 0;        // the most flagged units a confirmation of this object has met
  bool confirm_enqueued = false;
  uint64_t rec_cap = 0;
  void* conf_dest = nullptr;
  uint64_t conf_dest_cap = 0;
  // timing: launch k brackets its scan kernel with ev[2 (k mod kTimedRing)]
  // and ev[2 (k mod kTimedRing) + 1]; n_timed launches so far
  std::vector<hipEvent_t> ev;
  hipEvent_t kernel_done = nullptr;   // recorded after each scan kernel, before the compaction (scan_wait_kernel)
  uint64_t n_timed = 0;
  bool timing = false, timed = false;
};
struct carve_batch : carve_scan {};

namespace {

OneImage one_image(const carve_scan* sc) { return OneImage{sc->desc[0]}; }

// Whether a scan of one image under rule any_tau runs position-split
// (k_scan_tau): never for the any-position rule or without the split filter;
// else as the index's scan config says (automatic: filters of 4 MiB and more).
bool use_split(const carve_index* idx, uint32_t any_tau);
FragmentWindows fragment_windows(const carve_scan* sc) { return FragmentWindows{sc->desc[0]}; }
ManyImages many_images(const carve_scan* sc) {
  return ManyImages{sc->d_desc.as<ImageDesc>(), sc->n_images};
}

bool use_split(const carve_index* idx, uint32_t any_tau) {
  if (any_tau || !idx->bloom_tau.bytes) return false;
  if (idx->cfg.split == CARVE_SPLIT_ON) return true;
  if (idx->cfg.split == CARVE_SPLIT_OFF) return false;
  return idx->log2_bloom_words >= kSplitMinLog2;
}

// n (at most 8) consecutive device words, in one copy.
int read_words(carve_scan* sc, const uint64_t* d, uint32_t n, uint64_t* h) {
  CARVE_TRY(sc->h_small.reserve(64));
  HIP_TRY(hipMemcpyAsync(sc->h_small.p, d, 8 * n, hipMemcpyDeviceToHost, sc->stream));
  HIP_TRY(hipStreamSynchronize(sc->stream));
  for (uint32_t i = 0; i < n; ++i) h[i] = sc->h_small.as<uint64_t>()[i];
  return CARVE_OK;
}
int read_u64(carve_scan* sc, const uint64_t* d, uint64_t* h) { return read_words(sc, d, 1, h); }

// Memory a kernel may read: device (or managed) memory, not host memory.
bool gpu_readable(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // unknown to the runtime: plain host memory
    return false;
  }
  return a.type != hipMemoryTypeUnregistered && a.type != hipMemoryTypeHost;
}

// Device memory the kernels can write directly (else: staging + copy).
bool is_device_memory(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // plain host memory: clear the sticky error
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

bool same_desc(const std::vector<ImageDesc>& a, const std::vector<ImageDesc>& b) {
  return a.size() == b.size() && (a.empty() || memcmp(a.data(), b.data(), a.size() * sizeof(ImageDesc)) == 0);
}

int validate_image(const void* image, uint64_t n_bytes, uint32_t tau0, uint32_t tau_mode, const char* who,
                   long which) {
  char tag[64] = "";
  if (which >= 0) snprintf(tag, sizeof tag, " (image %ld)", which);
  if (tau0 > 7) return fail(CARVE_EINVAL, "%s: tau0 %u > 7%s", who, tau0, tag);
  if (tau_mode != CARVE_TAU_PER_CLUSTER && tau_mode != CARVE_TAU_ANY)
    return fail(CARVE_EINVAL, "%s: bad tau_mode %u%s", who, tau_mode, tag);
  if (n_bytes / kSectorBytes && !image) return fail(CARVE_EINVAL, "%s: null image%s", who, tag);
  if ((uintptr_t)image % 16) return fail(CARVE_EINVAL, "%s: image not 16-byte aligned%s", who, tag);
  return CARVE_OK;
}

// Launch the scan kernel, the compaction and (batches) the per-image offsets.
template <class Src>
int launch_scan(carve_scan* sc, const Src& src) {
  const carve_index* idx = sc->idx;
  hipStream_t s = sc->stream;
  const uint32_t per_cu = sc->grid_per_cu ? sc->grid_per_cu : idx->cfg.blocks_per_cu;
  const uint64_t n_words = sc->n_tiles;
  uint64_t* d_count = sc->count.as<uint64_t>();
  if (n_words == 0) {   // nothing to scan: the count is zero (and the confirmation marker cleared)
    k_fill_u64<<<1, 64, 0, s>>>(d_count, kConfirmedWord + 1, 0);
    if (sc->batch) k_fill_u64<<<1, 256, 0, s>>>(sc->img_off.as<uint64_t>(), sc->n_images + 1, 0);
    HIP_TRY(hipGetLastError());
    return CARVE_OK;
  }
  // one image of sectors under the per-cluster rule: the position-split scan
  bool split = false;
  ImageDesc one{};
  if constexpr (std::is_same<Src, OneImage>::value) {
    one = src.d;
    split = use_split(idx, one.any_tau);
  }
  const uint64_t slot = 2 * (sc->n_timed % kTimedRing);
  if (sc->timing) HIP_TRY(hipEventRecord(sc->ev[slot], s));
  if constexpr (std::is_same<Src, FragmentWindows>::value) {
    const uint64_t n_tasks = cdiv(src.d.n_sectors, kWaveWindows);
    const IndexView ix = idx->view();
    if (ix.bloom) {
      const int grid = resident_grid(k_frag_scan<true>, kFragThreads, cdiv(n_tasks, kFragWaves), per_cu);
      k_frag_scan<true><<<grid, kFragThreads, 0, s>>>((const uint32_t*)src.d.base, src.d.n_sectors, sc->n_dwords,
                                                      ix, sc->bitmap.as<uint64_t>(), sc->hit_slot.as<uint32_t>());
    } else {
      const int grid = resident_grid(k_frag_scan<false>, kFragThreads, cdiv(n_tasks, kFragWaves), per_cu);
      k_frag_scan<false><<<grid, kFragThreads, 0, s>>>((const uint32_t*)src.d.base, src.d.n_sectors, sc->n_dwords,
                                                       ix, sc->bitmap.as<uint64_t>(), sc->hit_slot.as<uint32_t>());
    }
    HIP_TRY(hipGetLastError());
  } else if (split) {
    const uint32_t chunk = idx->cfg.tiles_per_chunk ? idx->cfg.tiles_per_chunk : 1;
    CARVE_TRY(launch_k_scan_tau(idx->sig_kind, idx->layout, one, cdiv(n_words, kPositions), chunk,
                                per_cu, idx->view(), idx->weights, sc->tau_words.as<uint64_t>(),
                                sc->hit_slot.as<uint32_t>(), tau_counters(sc->tau_words.as<uint64_t>(), n_words),
                                s));
  } else {
    const uint32_t chunk = idx->cfg.tiles_per_chunk ? idx->cfg.tiles_per_chunk : 1;
    CARVE_TRY(launch_k_scan<kFlags>(idx->sig_kind, src, n_words, chunk, per_cu, idx->view(),
                                     idx->weights, sc->bitmap.as<uint64_t>(), sc->hit_slot.as<uint32_t>(), s,
                                     idx->layout));
  }
  if (sc->timing) {
    HIP_TRY(hipEventRecord(sc->ev[slot + 1], s));
    ++sc->n_timed;
    sc->timed = true;
  }
  HIP_TRY(hipEventRecord(sc->kernel_done, s));
  const uint64_t nb = cdiv(n_words, kItemsPerBlock);
  uint64_t* sums = sc->ws.as<uint64_t>();
  uint64_t* offs = sums + nb;
  if (split)   // the position-split scan's words, merged into the bitmap while counting
    k_reduce<<<nb, kBlockThreads, 0, s>>>(
        TauMergeItems{sc->tau_words.as<uint64_t>(), cdiv(n_words, kPositions), sc->bitmap.as<uint64_t>(), n_words,
                      one.tau0, (uint32_t)(one.n_sectors % kTileSectors)},
        Count{n_words, nullptr}, sums);
  else
    k_reduce<<<nb, kBlockThreads, 0, s>>>(PopcountItems{sc->bitmap.as<uint64_t>()}, Count{n_words, nullptr}, sums);
  k_scan_blocks<<<1, kBlockThreads, 0, s>>>(sums, Count{n_words, nullptr}, offs, d_count, d_count + kConfirmedWord);
  k_apply<<<nb, kBlockThreads, 0, s>>>(
      EmitIds<Src>{src, sc->bitmap.as<uint64_t>(), sc->ids.as<uint64_t>(), sc->batch ? sc->img_of.as<uint32_t>() : nullptr,
                   ~0ull},
      Count{n_words, nullptr}, offs);
  if constexpr (std::is_same<Src, ManyImages>::value) {
    const uint64_t per_block = kBlockThreads / kWave;
    k_image_offsets<<<cdiv(sc->n_images + 1, per_block), kBlockThreads, 0, s>>>(
        src, sc->bitmap.as<uint64_t>(), offs, d_count, sc->img_off.as<uint64_t>());
  }
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

// The events around timed scan kernels. They carry timestamps only (read
// after the host has waited for the stream), so they skip the system-scope
// fence that writes back and invalidates the caches at every record.
int create_timing_ring(carve_scan* sc) {
  sc->ev.assign(2 * kTimedRing, nullptr);
  for (hipEvent_t& e : sc->ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return CARVE_OK;
}

// Buffers for a tile space of n_tiles tiles.
int reserve_scan(carve_scan* sc) {
  const uint64_t n_words = sc->n_tiles ? sc->n_tiles : 1;
  const uint64_t nb = cdiv(n_words, kItemsPerBlock);
  CARVE_TRY(sc->bitmap.reserve(n_words * 8));
  CARVE_TRY(sc->ws.reserve(2 * nb * 8));
  CARVE_TRY(sc->ids.reserve(n_words * kTileSectors * 8));
  // a single image of sectors may be scanned split by position (k_scan_tau):
  // its tiles of 64 clusters reach slot 512 * ceil(n_words / 8)
  const bool split = !sc->batch && !sc->fragments && sc->idx && use_split(sc->idx, sc->desc[0].any_tau);
  const uint64_t tau_tiles = cdiv(n_words, kPositions);
  CARVE_TRY(sc->hit_slot.reserve((split ? tau_tiles * kPositions : n_words) * kTileSectors * 4));
  if (split) CARVE_TRY(sc->tau_words.reserve((tau_counter_offset(n_words) + kTauCounters) * 8));
  CARVE_TRY(sc->count.reserve(64));
  if (sc->batch) {
    CARVE_TRY(sc->img_of.reserve(n_words * kTileSectors * 4));
    CARVE_TRY(sc->img_off.reserve((sc->n_images + 1) * 8));
  }
  if (sc->timing && sc->ev.empty()) CARVE_TRY(create_timing_ring(sc));
  // an ordering point for other streams only (no host read, no data handed
  // over), so without the system-scope fence that writes back and invalidates
  // the caches at every record
  if (!sc->kernel_done)
    HIP_TRY(hipEventCreateWithFlags(&sc->kernel_done, hipEventDisableTiming | hipEventDisableSystemFence));
  return CARVE_OK;
}

// The scan's counts in one readback: flagged units, confirmed records, and
// the marker (1: a confirmation ran after the latest scan).
int read_counts(carve_scan* sc, uint64_t c[3]) {
  static_assert(kConfirmedWord == 2, "the counts and the marker are read in one copy");
  return read_words(sc, sc->count.as<uint64_t>(), 3, c);
}

// Confirmation buffers for up to cap_f flagged units. Records: room for
// about one per eighth of the units (more are counted, and produced again
// with their exact count when they are copied out). Returns the record room.
template <class Rec>
int reserve_confirm(carve_scan* sc, uint64_t cap_f, uint64_t* rec_room) {
  CARVE_TRY(sc->n_match.reserve(cap_f * 4));
  CARVE_TRY(sc->match_mask.reserve(cap_f * 8));
  CARVE_TRY(sc->out_off.reserve((cap_f + 1) * 8));
  CARVE_TRY(sc->cws.reserve(2 * cdiv(cap_f ? cap_f : 1, kItemsPerBlock) * sizeof(uint64_t)));
  uint64_t rec_cap = sc->matches.bytes / sizeof(Rec);
  if (rec_cap < cap_f / 8 + 4096) rec_cap = cap_f / 8 + 4096;
  CARVE_TRY(sc->matches.reserve(rec_cap * sizeof(Rec)));
  *rec_room = rec_cap;
  return CARVE_OK;
}

// Enqueue the confirmation of every flagged unit of the scan: the equal
// counts and masks (k_confirm_count), their offsets, the records
// (k_confirm_emit). The number of flagged units is not read back: the kernels
// take it from the device, and buffers are sized for the most there can be,
// so nothing here waits. Records go to the scan's own buffer, or (dest !=
// null: device memory of the caller, dest_cap records) straight to their
// destination.
template <class Src, class Rec>
int confirm_enqueue_impl(const carve_index* idx, carve_scan* sc, const Src& src, Rec* dest = nullptr,
                         uint64_t dest_cap = 0) {
  hipStream_t s = sc->stream;
  sc->confirm_enqueued = true;
  sc->rec_cap = 0;
  sc->conf_dest = dest;
  sc->conf_dest_cap = dest ? dest_cap : 0;
  if (sc->n_tiles == 0) return CARVE_OK;
  // Flagged units are at most `most`. A sector scan's per-flagged arrays have
  // room for all of them; a fragment scan's for an eighth of its windows (at
  // least 2^20), or for what an earlier confirmation of this object met: the
  // kernels stop at the room, and confirm_all redoes a confirmation that ran
  // short (a window scan would otherwise keep about 20 bytes per window here).
  const uint64_t most = sc->n_tiles * kTileSectors;
  uint64_t cap_f = most;
  if (sc->fragments) {
    uint64_t room = most / 8 > (1ull << 20) ? most / 8 : (1ull << 20);
    if (room < sc->conf_need) room = sc->conf_need;
    if (room < cap_f) cap_f = room;
  }
  sc->conf_room = cap_f;
  const uint64_t* d_count = sc->count.as<uint64_t>();
  uint64_t rec_cap = 0;
  CARVE_TRY(reserve_confirm<Rec>(sc, cap_f, &rec_cap));
  sc->rec_cap = dest ? 0 : rec_cap;
  const ConfirmView cv = idx->cview();
  const uint32_t* img_of = sc->batch ? sc->img_of.as<uint32_t>() : nullptr;
  const uint64_t per_block = kBlockThreads / confirm_lanes<Src>();
  const Count nf{cap_f, d_count};
  k_confirm_count<Src><<<resident_grid(k_confirm_count<Src>, kBlockThreads, cdiv(cap_f, per_block)), kBlockThreads,
                         0, s>>>(src, sc->ids.as<uint64_t>(), img_of, nf, sc->hit_slot.as<uint32_t>(), cv,
                                 sc->n_match.as<uint32_t>(), sc->match_mask.as<uint64_t>(),
                                 sc->count.as<uint64_t>() + kConfirmedWord);
  uint64_t* d_total = sc->count.as<uint64_t>() + 1;
  CARVE_TRY(scan_counts<uint64_t>(sc->n_match.as<uint32_t>(), sc->out_off.as<uint64_t>(), cap_f, d_total, sc->cws, s,
                                  d_count));
  k_confirm_emit<Src, Rec><<<resident_grid(k_confirm_emit<Src, Rec>, 256, cdiv(cap_f, 256)), 256, 0, s>>>(
      src, sc->ids.as<uint64_t>(), img_of, nf, sc->hit_slot.as<uint32_t>(), cv, sc->match_mask.as<uint64_t>(),
      sc->out_off.as<uint64_t>(), dest ? dest : sc->matches.as<Rec>(), dest ? dest_cap : rec_cap);
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

// Confirmed records of the scan into `out` (host or device): one readback of
// the counts (enqueueing the confirmation first unless it already is), then
// at most a copy. Records already written to `out` by the enqueued
// confirmation are not copied again.
template <class Src, class Rec>
int confirm_all(const carve_index* idx, carve_scan* sc, const Src& src, Rec* out, uint64_t cap, uint64_t* n_out) {
  hipStream_t s = sc->stream;
  *n_out = 0;
  const bool to_device = cap && is_device_memory(out);
  if (!sc->confirm_enqueued)   // a device destination gets its records directly
    CARVE_TRY((confirm_enqueue_impl<Src, Rec>(idx, sc, src, to_device ? out : nullptr, cap)));
  if (sc->n_tiles == 0) return CARVE_OK;
  uint64_t c[3];
  CARVE_TRY(read_counts(sc, c));
  // not confirmed since the scan (a scan replayed from a graph after the
  // enqueue), or room for fewer flagged units than there are: again
  if (!c[kConfirmedWord] || c[0] > sc->conf_room) {
    if (c[0] > sc->conf_room) sc->conf_need = c[0];
    CARVE_TRY((confirm_enqueue_impl<Src, Rec>(idx, sc, src, to_device ? out : nullptr, cap)));
    CARVE_TRY(read_counts(sc, c));
  }
  const uint64_t nf = c[0], nm = c[1];
  *n_out = nm;
  const uint64_t k = nm < cap ? nm : cap;
  const bool in_place = sc->conf_dest == (void*)out && k <= sc->conf_dest_cap;
  if (k && !in_place) {
    if (sc->conf_dest || k > sc->rec_cap) {   // records elsewhere, or past the room: produced again, all of them
      if (k > sc->rec_cap) CARVE_TRY(sc->matches.reserve(k * sizeof(Rec)));
      sc->rec_cap = sc->matches.bytes / sizeof(Rec);
      sc->conf_dest = nullptr;
      sc->conf_dest_cap = 0;
      k_confirm_emit<Src, Rec><<<resident_grid(k_confirm_emit<Src, Rec>, 256, cdiv(nf, 256)), 256, 0, s>>>(
          src, sc->ids.as<uint64_t>(), sc->batch ? sc->img_of.as<uint32_t>() : nullptr, Count{nf, nullptr},
          sc->hit_slot.as<uint32_t>(), idx->cview(), sc->match_mask.as<uint64_t>(), sc->out_off.as<uint64_t>(),
          sc->matches.as<Rec>(), sc->rec_cap);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(out, sc->matches.p, k * sizeof(Rec), hipMemcpyDefault, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (nm > cap) return fail(CARVE_ETRUNC, "confirm: %llu matches, capacity %llu", (unsigned long long)nm,
                            (unsigned long long)cap);
  return CARVE_OK;
}

// min(count, cap) ids starting at `first` of the scan's id list into `out`.
int copy_ids(carve_scan* sc, uint64_t first, uint64_t n, uint64_t* out, uint64_t cap) {
  const uint64_t k = n < cap ? n : cap;
  if (!k) return CARVE_OK;
  HIP_TRY(hipMemcpyAsync(out, sc->ids.as<uint64_t>() + first, k * 8, hipMemcpyDefault, sc->stream));
  HIP_TRY(hipStreamSynchronize(sc->stream));
  return CARVE_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" const char* carve_last_error(void) { return g_err.c_str(); }

CARVE_HIDDEN int carve_fail_msg(int code, const char* msg) {
  return fail(code, "%s", msg);
}

extern "C" int sector_signatures_kind(uint32_t sig_kind, const void* sectors, uint64_t n_sectors, uint64_t* sigs,
                                      void* stream) {
  if (sig_kind != CARVE_SIG_DJB2_64 && sig_kind != CARVE_SIG_CRC64_ISO)
    return fail(CARVE_EINVAL, "sector_signatures: unknown sig_kind %u", sig_kind);
  if (n_sectors == 0) return CARVE_OK;
  if (!sectors || !sigs) return fail(CARVE_EINVAL, "sector_signatures: null pointer");
  if ((uintptr_t)sectors % 16) return fail(CARVE_EINVAL, "sector_signatures: sectors not 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  uint64_t wt = 0;
  if (!sig_table(sig_kind, &wt)) return fail(CARVE_EDEVICE, "sector_signatures: weight table unavailable");
  const OneImage src{ImageDesc{(const uint8_t*)sectors, n_sectors, 0, 0, 0}};
  return launch_k_scan<kSigs>(sig_kind, src, cdiv(n_sectors, kTileSectors), 1, 0, IndexView{}, wt, sigs, nullptr, s);
}

extern "C" int sector_signatures(const void* sectors, uint64_t n_sectors, uint64_t* sigs, void* stream) {
  return sector_signatures_kind(CARVE_SIG_DJB2_64, sectors, n_sectors, sigs, stream);
}

extern "C" void free_index(carve_index* idx) {
  if (!idx) return;
  idx->keys.release();
  idx->tau_mask.release();
  idx->cand_off.release();
  idx->cand.release();
  idx->m_file.release();
  idx->m_k.release();
  idx->bloom.release();
  idx->lin_keys.release();
  idx->lin_slot.release();
  idx->sorted_keys.release();
  idx->sorted_slot.release();
  idx->lds_filter.release();
  idx->bloom_tau.release();
  delete idx;
}

namespace {
// The probe structure of the linear or sorted layout, from the n_keys
// distinct signatures held in the finished table's slots (signature 0 has no
// slot). Built even when there are none, so that a probe always finds a table.
int build_layout(carve_index* ix, const carve_index_params& p, uint64_t n_keys, hipStream_t s) {
  struct Temps {
    DevBuf list_keys, list_slots, counter, tmp;
    ~Temps() {
      list_keys.release();
      list_slots.release();
      counter.release();
      tmp.release();
    }
  } t;
  DevBuf &list_keys = t.list_keys, &list_slots = t.list_slots, &counter = t.counter, &tmp = t.tmp;
  CARVE_TRY(list_keys.reserve((n_keys ? n_keys : 1) * 8));
  CARVE_TRY(list_slots.reserve((n_keys ? n_keys : 1) * 4));
  CARVE_TRY(counter.reserve(8));
  HIP_TRY(hipMemsetAsync(counter.p, 0, 8, s));
  k_occupied<<<cdiv(ix->n_slots, 256), 256, 0, s>>>(ix->keys.as<uint64_t>(), ix->n_slots, list_keys.as<uint64_t>(),
                                                    list_slots.as<uint32_t>(),
                                                    (unsigned long long*)counter.as<uint64_t>());
  HIP_TRY(hipGetLastError());
  uint64_t listed = 0;
  HIP_TRY(hipMemcpyAsync(&listed, counter.p, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (listed != n_keys)
    return fail(CARVE_EDEVICE, "build_master_index: %llu table keys listed, %llu expected", (unsigned long long)listed,
                (unsigned long long)n_keys);
  if (p.layout == CARVE_LAYOUT_LINEAR) {
    uint32_t w = 1;
    while ((double)(1ull << w) * p.max_load < (double)n_keys) ++w;
    if (w > 32) return fail(CARVE_EUNSUPPORTED, "build_master_index: linear table too large");
    CARVE_TRY(ix->lin_keys.reserve(8ull << w));
    CARVE_TRY(ix->lin_slot.reserve(4ull << w));
    HIP_TRY(hipMemsetAsync(ix->lin_keys.p, 0, 8ull << w, s));
    ix->log2_lin = w;
    if (n_keys)
      k_insert_linear<<<cdiv(n_keys, 256), 256, 0, s>>>(list_keys.as<uint64_t>(), list_slots.as<uint32_t>(), n_keys,
                                                        ix->lin_keys.as<uint64_t>(), ix->lin_slot.as<uint32_t>(), w);
    HIP_TRY(hipGetLastError());
  } else if (n_keys) {
    CARVE_TRY(ix->sorted_keys.reserve(n_keys * 8));
    CARVE_TRY(ix->sorted_slot.reserve(n_keys * 4));
    size_t bytes = 0;
    HIP_TRY(rocprim::radix_sort_pairs(nullptr, bytes, list_keys.as<uint64_t>(), ix->sorted_keys.as<uint64_t>(),
                                      list_slots.as<uint32_t>(), ix->sorted_slot.as<uint32_t>(), (size_t)n_keys, 0,
                                      64, s));
    CARVE_TRY(tmp.reserve(bytes));
    HIP_TRY(rocprim::radix_sort_pairs(tmp.p, bytes, list_keys.as<uint64_t>(), ix->sorted_keys.as<uint64_t>(),
                                      list_slots.as<uint32_t>(), ix->sorted_slot.as<uint32_t>(), (size_t)n_keys, 0,
                                      64, s));
    ix->n_sorted = (uint32_t)n_keys;
  }
  HIP_TRY(hipStreamSynchronize(s));   // before the temporaries are freed
  return CARVE_OK;
}
}  // namespace

namespace {
// One thread per master fragment: its djb2 over 64 bytes.
__global__ void k_frag_sigs(const uint32_t* __restrict__ fragments, uint64_t n, uint64_t* __restrict__ sig) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  uint32_t w[16];
  const u32x4* p = (const u32x4*)(fragments + t * 16);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const u32x4 v = p[k];
    w[4 * k] = v.x;
    w[4 * k + 1] = v.y;
    w[4 * k + 2] = v.z;
    w[4 * k + 3] = v.w;
  }
  sig[t] = fragment_signature(w);
}

int build_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                const carve_index_params* params, void* stream, carve_index** out, uint32_t unit);
}  // namespace

extern "C" int build_master_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                                  const carve_index_params* params, void* stream, carve_index** out) {
  return build_index(master_sectors, file_sector_offsets, n_files, params, stream, out, kSectorBytes);
}

extern "C" int build_fragment_index(const void* master_fragments, const uint64_t* file_fragment_offsets,
                                    uint32_t n_files, const carve_index_params* params, void* stream,
                                    carve_index** out) {
  if (params && (params->sig_kind != CARVE_SIG_DJB2_64 || params->layout != CARVE_LAYOUT_BUCKETED))
    return fail(CARVE_EUNSUPPORTED, "build_fragment_index: fragments use djb2-64 and the bucketed layout");
  return build_index(master_fragments, file_fragment_offsets, n_files, params, stream, out, kFragBytes);
}

namespace {
int build_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                const carve_index_params* params, void* stream, carve_index** out, uint32_t unit) {
  if (!out) return fail(CARVE_EINVAL, "build_master_index: out is null");
  *out = nullptr;
  if (!file_sector_offsets && n_files) return fail(CARVE_EINVAL, "build_master_index: null offsets");
  carve_index_params p{};
  p.max_load = 0.5f;
  if (params) {
    p = *params;
    if (p.max_load == 0.f) p.max_load = 0.5f;
    for (uint32_t r : p.reserved)
      if (r) return fail(CARVE_EINVAL, "build_master_index: reserved params must be zero");
  }
  if (p.sig_kind != CARVE_SIG_DJB2_64 && p.sig_kind != CARVE_SIG_CRC64_ISO)
    return fail(CARVE_EUNSUPPORTED, "build_master_index: unknown sig_kind %u", p.sig_kind);
  if (!(p.max_load > 0.f && p.max_load <= 0.9f)) return fail(CARVE_EINVAL, "build_master_index: max_load out of (0, 0.9]");
  if (p.layout > CARVE_LAYOUT_SORTED) return fail(CARVE_EINVAL, "build_master_index: unknown layout %u", p.layout);
  if (p.bloom_bits_per_key != 0 && p.bloom_bits_per_key != CARVE_BLOOM_OFF &&
      (p.bloom_bits_per_key < 4 || p.bloom_bits_per_key > 64))
    return fail(CARVE_EINVAL, "build_master_index: bloom_bits_per_key %u out of 4..64", p.bloom_bits_per_key);
  uint64_t n_masters = 0;
  if (n_files) {
    if (file_sector_offsets[0] != 0) return fail(CARVE_EINVAL, "build_master_index: offsets[0] != 0");
    for (uint32_t f = 0; f < n_files; ++f)
      if (file_sector_offsets[f + 1] < file_sector_offsets[f])
        return fail(CARVE_EINVAL, "build_master_index: offsets not ascending at file %u", f);
    n_masters = file_sector_offsets[n_files];
  }
  if (n_masters >= 0xFFFFFFFFull) return fail(CARVE_EUNSUPPORTED, "build_master_index: too many master sectors");
  if (n_masters && !master_sectors) return fail(CARVE_EINVAL, "build_master_index: null master_sectors");
  if ((uintptr_t)master_sectors % 16) return fail(CARVE_EINVAL, "build_master_index: masters not 16-byte aligned");

  hipStream_t s = (hipStream_t)stream;
  carve_index* ix = new carve_index();
  auto bail = [&](int code) {
    free_index(ix);
    return code;
  };
  (void)hipGetDevice(&ix->device);
  ix->n_masters = n_masters;
  ix->n_files = n_files;
  ix->masters = (const uint8_t*)master_sectors;
  ix->unit_bytes = unit;
  ix->sig_kind = p.sig_kind;
  if (!sig_table(p.sig_kind, &ix->weights))
    return bail(fail(CARVE_EDEVICE, "build_master_index: weight table unavailable"));
  ix->layout = p.layout;
  // the bucketed table holds the candidate lists in every layout; max_load
  // sizes the layout that is probed
  const float bucket_load = p.layout == CARVE_LAYOUT_BUCKETED ? p.max_load : 0.5f;
  uint32_t lb = 1;
  while (((uint64_t)kBucketSlots << lb) * bucket_load < (double)n_masters) ++lb;
  if (lb > 27) return bail(fail(CARVE_EUNSUPPORTED, "build_master_index: table too large"));   // slots fit 32 bits
  ix->log2_buckets = lb;
  ix->n_slots = (uint64_t)kBucketSlots << lb;
  const uint64_t n_lists = ix->n_slots + 1;   // + side slot of signature 0

  int rc;
  if ((rc = ix->keys.reserve(ix->n_slots * 8)) || (rc = ix->tau_mask.reserve(n_lists)) ||
      (rc = ix->cand_off.reserve((n_lists + 1) * 4)) || (rc = ix->cand.reserve((n_masters ? n_masters : 1) * 4)) ||
      (rc = ix->m_file.reserve((n_masters ? n_masters : 1) * 4)) || (rc = ix->m_k.reserve((n_masters ? n_masters : 1) * 4)))
    return bail(rc);
  DevBuf d_off, sig, cnt, m_slot, tmp, ws, misc, mask32;
  auto cleanup = [&]() {
    mask32.release();
    d_off.release();
    sig.release();
    cnt.release();
    m_slot.release();
    tmp.release();
    ws.release();
    misc.release();
  };
  auto bail2 = [&](int code) {
    cleanup();
    return bail(code);
  };
  if ((rc = d_off.reserve((n_files + 1) * 8)) || (rc = sig.reserve((n_masters ? n_masters : 1) * 8)) ||
      (rc = cnt.reserve(n_lists * 4)) || (rc = m_slot.reserve((n_masters ? n_masters : 1) * 4)) ||
      (rc = tmp.reserve((n_masters ? n_masters : 1) * 4)) || (rc = misc.reserve(64)) ||
      (rc = mask32.reserve(n_lists * 4)))
    return bail2(rc);
  uint32_t* d_overflow = misc.as<uint32_t>();
  uint32_t* d_failed = d_overflow + 1;
  uint64_t* d_total = misc.as<uint64_t>() + 1;
#define BUILD_TRY(expr)                                                                            \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return bail2(fail(CARVE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_))); \
  } while (0)
  BUILD_TRY(hipMemsetAsync(ix->keys.p, 0, ix->n_slots * 8, s));
  BUILD_TRY(hipMemsetAsync(mask32.p, 0, n_lists * 4, s));
  BUILD_TRY(hipMemsetAsync(cnt.p, 0, n_lists * 4, s));
  BUILD_TRY(hipMemsetAsync(misc.p, 0, 64, s));
  if (n_masters) {
    BUILD_TRY(hipMemcpyAsync(d_off.p, file_sector_offsets, (n_files + 1) * 8, hipMemcpyHostToDevice, s));
    const uint32_t nbk = (uint32_t)cdiv(n_masters, 256);
    k_master_meta<<<nbk, 256, 0, s>>>(d_off.as<uint64_t>(), n_files, n_masters, ix->m_file.as<uint32_t>(),
                                     ix->m_k.as<uint32_t>());
    if (unit == kFragBytes) {
      k_frag_sigs<<<nbk, 256, 0, s>>>((const uint32_t*)ix->masters, n_masters, sig.as<uint64_t>());
    } else {
      const uint64_t n_tiles = cdiv(n_masters, kTileSectors);
      const OneImage src{ImageDesc{ix->masters, n_masters, 0, 0, 0}};
      if ((rc = launch_k_scan<kSigs>(ix->sig_kind, src, n_tiles, 1, 0, IndexView{}, ix->weights, sig.as<uint64_t>(),
                                     nullptr, s)))
        return bail2(rc);
    }
    k_insert<<<nbk, 256, 0, s>>>(sig.as<uint64_t>(), ix->m_k.as<uint32_t>(), n_masters, ix->keys.as<uint64_t>(), lb,
                                mask32.as<uint32_t>(), cnt.as<uint32_t>(), m_slot.as<uint32_t>(), d_overflow,
                                d_failed);
    BUILD_TRY(hipGetLastError());
  }
  k_narrow_masks<<<cdiv(n_lists, 256), 256, 0, s>>>(mask32.as<uint32_t>(), n_lists, ix->tau_mask.as<uint8_t>());
  if ((rc = scan_counts<uint32_t>(cnt.as<uint32_t>(), ix->cand_off.as<uint32_t>(), n_lists, d_total, ws, s)))
    return bail2(rc);
  if (n_masters) {
    BUILD_TRY(hipMemsetAsync(cnt.p, 0, n_lists * 4, s));   // reused as scatter cursors
    const uint32_t nbk = (uint32_t)cdiv(n_masters, 256);
    k_scatter<<<nbk, 256, 0, s>>>(m_slot.as<uint32_t>(), n_masters, ix->cand_off.as<uint32_t>(), cnt.as<uint32_t>(),
                                 tmp.as<uint32_t>());
    k_sort_segments<<<device_cus() * 8, kBlockThreads, 0, s>>>(ix->cand_off.as<uint32_t>(), n_lists,
                                                                tmp.as<uint32_t>(), ix->cand.as<uint32_t>());
    BUILD_TRY(hipGetLastError());
  }
  {   // distinct signatures = non-empty candidate lists
    const uint64_t nb = cdiv(n_lists, kItemsPerBlock);
    if ((rc = ws.reserve(2 * nb * 8))) return bail2(rc);
    k_reduce<<<nb, kBlockThreads, 0, s>>>(NonEmptyLists{ix->cand_off.as<uint32_t>()}, Count{n_lists, nullptr},
                                          ws.as<uint64_t>());
    k_scan_blocks<<<1, kBlockThreads, 0, s>>>(ws.as<uint64_t>(), Count{n_lists, nullptr}, ws.as<uint64_t>() + nb,
                                              d_total + 1);
    BUILD_TRY(hipGetLastError());
  }
  uint32_t h_misc[2] = {0, 0};
  uint64_t h_unique = 0;
  uint32_t zmask = 0;
  BUILD_TRY(hipMemcpyAsync(h_misc, misc.p, 8, hipMemcpyDeviceToHost, s));
  BUILD_TRY(hipMemcpyAsync(&h_unique, d_total + 1, 8, hipMemcpyDeviceToHost, s));
  BUILD_TRY(hipMemcpyAsync(&zmask, mask32.as<uint32_t>() + ix->n_slots, 4, hipMemcpyDeviceToHost, s));
  BUILD_TRY(hipStreamSynchronize(s));
#undef BUILD_TRY
  if (h_misc[1]) return bail2(fail(CARVE_EDEVICE, "build_master_index: %u keys could not be placed", h_misc[1]));
  ix->n_overflow = h_misc[0];
  ix->zero_sig_mask = zmask;
  ix->n_unique = h_unique;
  {   // prefilter: words of 64 bits, a power of two of them
    // Automatic size (measured on 1M, 4M and 16M signatures): at least 4 bits
    // per signature, then as large as 4 MiB and 16 bits per signature allow.
    // A filter word per sector costs less traffic than a bucket line even
    // where the filter no longer fits in L2.
    // Fragment indexes (32-bit words of 3 bits, which fill less evenly) aim
    // at twice the bits.
    constexpr uint64_t kAutoBytes = 4ull << 20;
    const uint64_t keys_n = h_unique ? h_unique : 1;
    const uint64_t aim = unit == kFragBytes ? 32 : 16;
    uint32_t lw = 0;
    if (p.bloom_bits_per_key == 0) {
      while ((64ull << lw) < 4 * keys_n) ++lw;
      while ((8ull << (lw + 1)) <= kAutoBytes && (64ull << lw) < aim * keys_n) ++lw;
    } else if (p.bloom_bits_per_key != CARVE_BLOOM_OFF) {
      while ((64ull << lw) < (uint64_t)p.bloom_bits_per_key * keys_n) ++lw;
    }
    if (unit == kFragBytes && lw > 29) lw = 29;   // fragment filters: at most 2^30 words of 32 bits
    if (lw > 0 && lw <= 32) {
      if ((rc = ix->bloom.reserve(8ull << lw))) return bail2(rc);
      ix->log2_bloom_words = lw;
      if (hipMemsetAsync(ix->bloom.p, 0, 8ull << lw, s) != hipSuccess)
        return bail2(fail(CARVE_EDEVICE, "build_master_index: bloom memset failed"));
      if (unit == kFragBytes)   // the same bytes as 2^(lw+1) words of 32 bits, 3 bits per signature
        k_frag_bloom_build<<<cdiv(ix->n_slots, 256), 256, 0, s>>>(ix->keys.as<uint64_t>(), ix->n_slots, lw + 1,
                                                                   zmask ? 1u : 0u, ix->bloom.as<uint32_t>());
      else
        k_bloom_build<<<cdiv(ix->n_slots, 256), 256, 0, s>>>(ix->keys.as<uint64_t>(), ix->n_slots, lw,
                                                            ix->bloom.as<uint64_t>());
      // The filter split by position (sector indexes): slice t holds the keys
      // with a master at position t, about an eighth of them, and each XCD of a
      // position-split scan keeps only its slice in L2, so the slices are sized
      // apart from the whole filter: automatically 16 bits per key of a slice,
      // up to 4 MiB per slice (on the 64 GiB large workload, 16M keys: 10.57 ms
      // at 16 bits per key against 10.82 ms at the whole filter's 4, whose
      // false positives send 16% of the sectors to the table); else the
      // requested bits per key. At least 2 words per slice (bloom_place needs
      // log2_words >= 1: its shift by 64 - log2_words).
      if (unit == kSectorBytes) {
        constexpr uint64_t kSliceAutoBytes = 4ull << 20;
        const uint64_t per_slice = cdiv(keys_n, kPositions);
        const uint64_t bits = p.bloom_bits_per_key ? p.bloom_bits_per_key : 16;
        uint32_t ls = 1;
        while (ls < 32 && (64ull << ls) < bits * per_slice &&
               (p.bloom_bits_per_key || (8ull << (ls + 1)) <= kSliceAutoBytes))
          ++ls;
        if ((rc = ix->bloom_tau.reserve((8ull * kPositions) << ls))) return bail2(rc);
        ix->log2_bloom_tau = ls;
        if (hipMemsetAsync(ix->bloom_tau.p, 0, (8ull * kPositions) << ls, s) != hipSuccess)
          return bail2(fail(CARVE_EDEVICE, "build_master_index: bloom memset failed"));
        k_bloom_tau_build<<<cdiv(ix->n_slots, 256), 256, 0, s>>>(ix->keys.as<uint64_t>(), ix->tau_mask.as<uint8_t>(),
                                                                ix->n_slots, ls, ix->bloom_tau.as<uint64_t>());
      }
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return bail2(fail(CARVE_EDEVICE, "build_master_index: bloom build failed"));
    }
  }
  if (p.layout != CARVE_LAYOUT_BUCKETED) {
    // the distinct signatures counted above include signature 0, which has no slot
    if ((rc = build_layout(ix, p, h_unique - (zmask ? 1 : 0), s))) return bail2(rc);
  }
  if (unit == kFragBytes) {   // first-level filter: about 16 bits per signature, 1-160 KiB (always present)
    const uint64_t want = cdiv(16 * h_unique, 32 * 256) * 256;   // words, a multiple of 256
    const uint32_t lw = (uint32_t)(want < 256 ? 256 : (want > kLdsFilterMaxWords ? kLdsFilterMaxWords : want));
    if ((rc = ix->lds_filter.reserve(4ull * lw))) return bail2(rc);
    ix->lds_words = lw;
    if (hipMemsetAsync(ix->lds_filter.p, 0, 4ull * lw, s) != hipSuccess)
      return bail2(fail(CARVE_EDEVICE, "build_fragment_index: filter memset failed"));
    k_lds_filter_build<<<cdiv(ix->n_slots, 256), 256, 0, s>>>(ix->keys.as<uint64_t>(), ix->n_slots, lw,
                                                             zmask ? 1u : 0u, ix->lds_filter.as<uint32_t>());
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return bail2(fail(CARVE_EDEVICE, "build_fragment_index: filter build failed"));
  }
  cleanup();
  *out = ix;
  return CARVE_OK;
}
}  // namespace

extern "C" int index_stats(const carve_index* idx, carve_index_stats* out) {
  if (!idx || !out) return fail(CARVE_EINVAL, "index_stats: null argument");
  out->n_master_sectors = idx->n_masters;
  out->n_unique_signatures = idx->n_unique;
  out->n_buckets = 1ull << idx->log2_buckets;
  out->n_overflow_keys = idx->n_overflow;
  out->device_bytes = idx->keys.bytes + idx->tau_mask.bytes + idx->cand_off.bytes + idx->cand.bytes +
                      idx->m_file.bytes + idx->m_k.bytes + idx->bloom.bytes + idx->lin_keys.bytes + idx->bloom_tau.bytes +
                      idx->lin_slot.bytes + idx->sorted_keys.bytes + idx->sorted_slot.bytes + idx->lds_filter.bytes;
  out->bloom_bytes = idx->bloom.bytes;
  return CARVE_OK;
}

extern "C" int index_set_scan_config(carve_index* idx, const carve_scan_config* cfg) {
  if (!idx || !cfg) return fail(CARVE_EINVAL, "index_set_scan_config: null argument");
  if (cfg->reserved) return fail(CARVE_EINVAL, "index_set_scan_config: reserved must be zero");
  if (cfg->blocks_per_cu > 64 || cfg->tiles_per_chunk > (1u << 20) || cfg->split > CARVE_SPLIT_ON)
    return fail(CARVE_EINVAL, "index_set_scan_config: out of range");
  idx->cfg = *cfg;
  return CARVE_OK;
}

extern "C" int index_get_scan_config(const carve_index* idx, carve_scan_config* cfg) {
  if (!idx || !cfg) return fail(CARVE_EINVAL, "index_get_scan_config: null argument");
  *cfg = idx->cfg;
  return CARVE_OK;
}

extern "C" void free_scan(carve_scan* sc) {
  if (!sc) return;
  (void)hipStreamSynchronize(sc->stream);
  for (DevBuf* b : {&sc->d_desc, &sc->bitmap, &sc->ids, &sc->img_of, &sc->count, &sc->hit_slot, &sc->img_off,
                    &sc->tau_words, &sc->ws, &sc->n_match, &sc->match_mask, &sc->out_off,
                    &sc->matches, &sc->cws})
    b->release();
  sc->h_desc.release();
  sc->h_small.release();
  sc->h_img_off.release();
  for (hipEvent_t e : sc->ev) (void)hipEventDestroy(e);
  if (sc->kernel_done) (void)hipEventDestroy(sc->kernel_done);
  if (sc->batch) delete static_cast<carve_batch*>(sc);
  else delete sc;
}

extern "C" void free_batch(carve_batch* b) { free_scan(b); }

extern "C" int scan_image(const carve_index* idx, const void* image, uint64_t n_bytes, uint32_t tau0,
                          uint32_t tau_mode, void* stream, carve_scan** io) {
  if (!idx || !io) return fail(CARVE_EINVAL, "scan_image: null idx or io");
  if (idx->unit_bytes != kSectorBytes)
    return fail(CARVE_EINVAL, "scan_image: a fragment index (use scan_fragments)");
  CARVE_TRY(validate_image(image, n_bytes, tau0, tau_mode, "scan_image", -1));
  if (n_bytes >= kSectorBytes && !gpu_readable(image))
    return fail(CARVE_EINVAL, "scan_image: image is not in device memory");
  if (*io && (*io)->batch) return fail(CARVE_EINVAL, "scan_image: io is a batch object");
  carve_scan* sc = *io;
  const bool created = !sc;
  if (created) {
    sc = new carve_scan();
    (void)hipGetDevice(&sc->device);
  }
  const uint64_t n_sectors = n_bytes / kSectorBytes;
  sc->stream = (hipStream_t)stream;
  sc->idx = idx;
  sc->n_images = 1;
  sc->n_tiles = cdiv(n_sectors, kTileSectors);
  sc->max_sectors = n_sectors;
  sc->desc.assign(2, ImageDesc{});
  sc->desc[0] = ImageDesc{(const uint8_t*)image, n_sectors, 0, tau0, tau_mode == CARVE_TAU_ANY ? 1u : 0u};
  sc->desc[1].tile_begin = sc->n_tiles;
  sc->fragments = false;
  sc->timed = false;
  sc->confirm_enqueued = false;
  int rc = reserve_scan(sc);
  if (rc == CARVE_OK) rc = launch_scan(sc, one_image(sc));
  if (rc != CARVE_OK) {
    if (created) free_scan(sc);
    return rc;
  }
  *io = sc;
  return CARVE_OK;
}

namespace {
std::mutex g_scratch_mu;
uint64_t* g_scratch_dev[64] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current (each GPU has its own copy of the array).
int noalloc_scratch(uint64_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(CARVE_EUNSUPPORTED, "scan_image_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    uint64_t* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CARVE_EDEVICE, "scan_image_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return CARVE_OK;
}
}  // namespace

extern "C" int scan_image_noalloc(const carve_index* idx, const void* image, uint64_t n_bytes, uint32_t tau0,
                                  uint32_t tau_mode, void* stream, uint64_t* ids, uint64_t cap, uint64_t* count) {
  if (!idx || !count) return fail(CARVE_EINVAL, "scan_image_noalloc: null idx or count");
  if (cap && !ids) return fail(CARVE_EINVAL, "scan_image_noalloc: null ids with cap > 0");
  const uint64_t n_sectors = n_bytes / kSectorBytes;
  if (n_sectors > kNoAllocMaxSectors)
    return fail(CARVE_EINVAL, "scan_image_noalloc: %llu sectors, at most %llu (64 GiB) without allocation",
                (unsigned long long)n_sectors, (unsigned long long)kNoAllocMaxSectors);
  if (idx->unit_bytes != kSectorBytes) return fail(CARVE_EINVAL, "scan_image_noalloc: a fragment index");
  CARVE_TRY(validate_image(image, n_bytes, tau0, tau_mode, "scan_image_noalloc", -1));
  if (n_sectors && !gpu_readable(image)) return fail(CARVE_EINVAL, "scan_image_noalloc: image is not in device memory");
  if ((uintptr_t)count % 8 || (uintptr_t)ids % 8)
    return fail(CARVE_EINVAL, "scan_image_noalloc: ids and count must be 8-byte aligned");
  if (!is_device_memory(count) || (cap && !is_device_memory(ids)))
    return fail(CARVE_EINVAL, "scan_image_noalloc: ids and count must be device memory");
  uint64_t* sw = nullptr;
  CARVE_TRY(noalloc_scratch(&sw));
  hipStream_t s = (hipStream_t)stream;
  const uint64_t n_words = cdiv(n_sectors, kTileSectors);
  if (n_words == 0) {
    k_fill_u64<<<1, 64, 0, s>>>(count, 1, 0);
    HIP_TRY(hipGetLastError());
    return CARVE_OK;
  }
  // every word read below is written first by this call's own kernels
  uint64_t* bitmap = sw;
  uint64_t* tau_words = sw + kNoAllocMaxWords;
  uint64_t* sums = sw + 2 * kNoAllocMaxWords;
  uint64_t* offs = sums + kNoAllocMaxChunks;
  const OneImage src{ImageDesc{(const uint8_t*)image, n_sectors, 0, tau0, tau_mode == CARVE_TAU_ANY ? 1u : 0u}};
  const uint32_t per_cu = idx->cfg.blocks_per_cu;
  const uint32_t chunk = idx->cfg.tiles_per_chunk ? idx->cfg.tiles_per_chunk : 1;
  const uint64_t nb = cdiv(n_words, kItemsPerBlock);
  if (use_split(idx, src.d.any_tau)) {   // as scan_image: the position-split scan
    CARVE_TRY(launch_k_scan_tau(idx->sig_kind, idx->layout, src.d, cdiv(n_words, kPositions), chunk, per_cu,
                                idx->view(), idx->weights, tau_words, nullptr, offs + kNoAllocMaxChunks, s));
    k_reduce<<<nb, kBlockThreads, 0, s>>>(TauMergeItems{tau_words, cdiv(n_words, kPositions), bitmap, n_words,
                                                        tau0, (uint32_t)(n_sectors % kTileSectors)},
                                          Count{n_words, nullptr}, sums);
  } else {
    CARVE_TRY(launch_k_scan<kFlagBits>(idx->sig_kind, src, n_words, chunk, per_cu, idx->view(), idx->weights, bitmap,
                                        nullptr, s, idx->layout));
    k_reduce<<<nb, kBlockThreads, 0, s>>>(PopcountItems{bitmap}, Count{n_words, nullptr}, sums);
  }
  k_scan_blocks<<<1, kBlockThreads, 0, s>>>(sums, Count{n_words, nullptr}, offs, count);
  k_apply<<<nb, kBlockThreads, 0, s>>>(EmitIds<OneImage>{src, bitmap, ids, nullptr, cap}, Count{n_words, nullptr},
                                       offs);
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

extern "C" int scan_fragments(const carve_index* idx, const void* image, uint64_t n_bytes, void* stream,
                              carve_scan** io) {
  if (!idx || !io) return fail(CARVE_EINVAL, "scan_fragments: null idx or io");
  if (idx->unit_bytes != kFragBytes)
    return fail(CARVE_EINVAL, "scan_fragments: a sector index (build it with build_fragment_index)");
  if (n_bytes >= kFragBytes && !image) return fail(CARVE_EINVAL, "scan_fragments: null image");
  if ((uintptr_t)image % 16) return fail(CARVE_EINVAL, "scan_fragments: image not 16-byte aligned");
  if (n_bytes >= kFragBytes && !gpu_readable(image))
    return fail(CARVE_EINVAL, "scan_fragments: image is not in device memory");
  if (*io && (*io)->batch) return fail(CARVE_EINVAL, "scan_fragments: io is a batch object");
  carve_scan* sc = *io;
  const bool created = !sc;
  if (created) {
    sc = new carve_scan();
    (void)hipGetDevice(&sc->device);
  }
  const uint64_t n_windows = n_bytes < kFragBytes ? 0 : (n_bytes - kFragBytes) / kWindowStride + 1;
  sc->stream = (hipStream_t)stream;
  sc->idx = idx;
  sc->n_images = 1;
  sc->n_tiles = cdiv(n_windows, kTileSectors);
  sc->max_sectors = n_windows;
  sc->n_dwords = n_bytes / 4;
  sc->desc.assign(2, ImageDesc{});
  sc->desc[0] = ImageDesc{(const uint8_t*)image, n_windows, 0, 0, 1u};
  sc->desc[1].tile_begin = sc->n_tiles;
  sc->fragments = true;
  sc->timed = false;
  sc->confirm_enqueued = false;
  int rc = reserve_scan(sc);
  if (rc == CARVE_OK) rc = launch_scan(sc, fragment_windows(sc));
  if (rc != CARVE_OK) {
    if (created) free_scan(sc);
    return rc;
  }
  *io = sc;
  return CARVE_OK;
}

extern "C" int scan_batch(const carve_index* idx, const carve_image_desc* images, uint32_t n_images, void* stream,
                          carve_batch** io) {
  if (!idx || !io || (n_images && !images)) return fail(CARVE_EINVAL, "scan_batch: null argument");
  if (idx->unit_bytes != kSectorBytes) return fail(CARVE_EINVAL, "scan_batch: a fragment index");
  std::vector<ImageDesc> desc(n_images + 1);
  uint64_t tiles = 0, max_sectors = 0;
  for (uint32_t i = 0; i < n_images; ++i) {
    const carve_image_desc& d = images[i];
    CARVE_TRY(validate_image(d.image, d.n_bytes, d.tau0, d.tau_mode, "scan_batch", (long)i));
    const uint64_t n = d.n_bytes / kSectorBytes;
    desc[i] = ImageDesc{(const uint8_t*)d.image, n, tiles, d.tau0, d.tau_mode == CARVE_TAU_ANY ? 1u : 0u};
    tiles += cdiv(n, kTileSectors);
    if (n > max_sectors) max_sectors = n;
  }
  desc[n_images] = ImageDesc{nullptr, 0, tiles, 0, 0};
  carve_batch* b = *io;
  const bool created = !b;
  if (created) {
    b = new carve_batch();
    b->batch = true;
    (void)hipGetDevice(&b->device);
  }
  auto bail = [&](int code) {
    if (created) free_batch(b);
    return code;
  };
  b->stream = (hipStream_t)stream;
  b->idx = idx;
  b->n_images = n_images;
  b->n_tiles = tiles;
  b->max_sectors = max_sectors;
  b->desc = desc;
  b->timed = false;
  b->confirm_enqueued = false;
  int rc;
  if ((rc = reserve_scan(b))) return bail(rc);
  if (!same_desc(desc, b->uploaded)) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(b->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return bail(fail(CARVE_EINVAL, "scan_batch: new image descriptors while the stream is being captured"));
    const size_t bytes = desc.size() * sizeof(ImageDesc);
    // the staging buffer may still feed the previous upload
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(fail(CARVE_EDEVICE, "scan_batch: sync failed"));
    if ((rc = b->d_desc.reserve(bytes)) || (rc = b->h_desc.reserve(bytes))) return bail(rc);
    memcpy(b->h_desc.p, desc.data(), bytes);
    if (hipMemcpyAsync(b->d_desc.p, b->h_desc.p, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      return bail(fail(CARVE_EDEVICE, "scan_batch: descriptor upload failed"));
    b->uploaded = desc;
  }
  if ((rc = launch_scan(b, many_images(b)))) return bail(rc);
  *io = b;
  return CARVE_OK;
}

CARVE_HIDDEN int carve_batch_set_grid(carve_batch* b, uint32_t blocks_per_cu) {
  if (!b || !b->batch) return fail(CARVE_EINVAL, "carve_batch_set_grid: not a batch");
  b->grid_per_cu = blocks_per_cu;
  return CARVE_OK;
}

CARVE_HIDDEN uint32_t carve_batch_scan_blocks_per_cu(void) {
  return (uint32_t)blocks_per_cu(k_scan<kFlags, kSigDjb2, ManyImages, kLayoutBucketed>, kScanThreads);
}

extern "C" int scan_set_timing(carve_scan* sc, int enable) {
  if (!sc) return fail(CARVE_EINVAL, "scan_set_timing: null scan");
  if (enable && sc->ev.empty()) CARVE_TRY(create_timing_ring(sc));
  if (enable && !sc->timing) {   // a new timed series
    sc->n_timed = 0;
    sc->timed = false;
  }
  sc->timing = enable != 0;
  return CARVE_OK;
}

extern "C" int scan_kernel_ms(carve_scan* sc, float* ms) {
  if (!sc || !ms) return fail(CARVE_EINVAL, "scan_kernel_ms: null argument");
  if (!sc->timed) return fail(CARVE_EINVAL, "scan_kernel_ms: the last scan was not timed");
  const uint64_t slot = 2 * ((sc->n_timed - 1) % kTimedRing);
  HIP_TRY(hipEventSynchronize(sc->ev[slot + 1]));
  HIP_TRY(hipEventElapsedTime(ms, sc->ev[slot], sc->ev[slot + 1]));
  return CARVE_OK;
}

extern "C" int scan_kernel_ms_recent(carve_scan* sc, float* ms, uint32_t n, uint32_t* n_out) {
  if (!sc || !n_out || (n && !ms)) return fail(CARVE_EINVAL, "scan_kernel_ms_recent: null argument");
  *n_out = 0;
  const uint64_t have = sc->n_timed < kTimedRing ? sc->n_timed : kTimedRing;
  const uint32_t k = (uint32_t)(n < have ? n : have);
  if (!k) return CARVE_OK;
  HIP_TRY(hipEventSynchronize(sc->ev[2 * ((sc->n_timed - 1) % kTimedRing) + 1]));   // the latest ends last
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t slot = 2 * ((sc->n_timed - k + i) % kTimedRing);
    HIP_TRY(hipEventElapsedTime(&ms[i], sc->ev[slot], sc->ev[slot + 1]));
  }
  *n_out = k;
  return CARVE_OK;
}

namespace {
// Enqueue the copy of min(count, cap) flagged ids into the caller's device memory.
int enqueue_id_copy(carve_scan* sc, uint64_t* out, uint64_t cap) {
  const uint64_t most = cap < sc->max_sectors ? cap : sc->max_sectors;   // ids of one image: at most its units
  const uint64_t blocks = cdiv(most ? most : 1, 256);
  k_copy_ids<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, sc->stream>>>(
      sc->ids.as<uint64_t>(), sc->count.as<uint64_t>(), most, out);
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}
}  // namespace

extern "C" int flagged_sectors(carve_scan* sc, uint64_t* out, uint64_t cap, uint64_t* n_out) {
  if (!sc || !n_out) return fail(CARVE_EINVAL, "flagged_sectors: null argument");
  if (sc->batch) return fail(CARVE_EINVAL, "flagged_sectors: a batch object (use batch_flagged_sectors)");
  if (cap && !out) return fail(CARVE_EINVAL, "flagged_sectors: null out with cap > 0");
  uint64_t n = 0;
  if (cap && sc->n_tiles && is_device_memory(out)) {   // copy on the device, then one synchronization
    CARVE_TRY(enqueue_id_copy(sc, out, cap));
    CARVE_TRY(read_u64(sc, sc->count.as<uint64_t>(), &n));
  } else {
    CARVE_TRY(read_u64(sc, sc->count.as<uint64_t>(), &n));
    CARVE_TRY(copy_ids(sc, 0, n, out, cap));
  }
  *n_out = n;
  if (n > cap) return fail(CARVE_ETRUNC, "flagged_sectors: %llu flagged, capacity %llu", (unsigned long long)n,
                           (unsigned long long)cap);
  return CARVE_OK;
}

extern "C" int flagged_sectors_enqueue(carve_scan* sc, uint64_t* out, uint64_t cap) {
  if (!sc) return fail(CARVE_EINVAL, "flagged_sectors_enqueue: null scan");
  if (sc->batch) return fail(CARVE_EINVAL, "flagged_sectors_enqueue: a batch object");
  if (cap && !out) return fail(CARVE_EINVAL, "flagged_sectors_enqueue: null out with cap > 0");
  if (cap && !is_device_memory(out)) return fail(CARVE_EINVAL, "flagged_sectors_enqueue: out is not device memory");
  if (!cap || !sc->n_tiles) return CARVE_OK;
  return enqueue_id_copy(sc, out, cap);
}

extern "C" int scan_wait_kernel(carve_scan* sc, void* stream) {
  if (!sc) return fail(CARVE_EINVAL, "scan_wait_kernel: null scan");
  if (!sc->kernel_done) return CARVE_OK;   // no scan kernel enqueued yet
  HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, sc->kernel_done, 0));
  return CARVE_OK;
}

extern "C" int scan_counts(carve_scan* sc, uint64_t* n_flagged, uint64_t* n_confirmed) {
  if (!sc || !n_flagged || !n_confirmed) return fail(CARVE_EINVAL, "scan_counts: null argument");
  if (!sc->n_tiles) {   // nothing was scanned: no kernel ran
    *n_flagged = 0;
    *n_confirmed = sc->confirm_enqueued ? 0 : CARVE_NOT_CONFIRMED;
    return CARVE_OK;
  }
  uint64_t c[3];
  CARVE_TRY(read_counts(sc, c));
  *n_flagged = c[0];
  *n_confirmed = c[kConfirmedWord] ? c[1] : CARVE_NOT_CONFIRMED;
  return CARVE_OK;
}

extern "C" int confirm_matches(const carve_index* idx, carve_scan* sc, carve_match* out, uint64_t cap,
                               uint64_t* n_out) {
  if (!idx || !sc || !n_out) return fail(CARVE_EINVAL, "confirm_matches: null argument");
  if (sc->batch) return fail(CARVE_EINVAL, "confirm_matches: a batch object (use batch_confirm_matches)");
  if (cap && !out) return fail(CARVE_EINVAL, "confirm_matches: null out with cap > 0");
  if (sc->idx != idx) return fail(CARVE_EINVAL, "confirm_matches: scan was made with another index");
  if (sc->fragments) return confirm_all(idx, sc, fragment_windows(sc), out, cap, n_out);
  return confirm_all(idx, sc, one_image(sc), out, cap, n_out);
}

extern "C" int confirm_enqueue(const carve_index* idx, carve_scan* sc) {
  if (!idx || !sc) return fail(CARVE_EINVAL, "confirm_enqueue: null argument");
  if (sc->batch) return fail(CARVE_EINVAL, "confirm_enqueue: a batch object (use batch_confirm_enqueue)");
  if (sc->idx != idx) return fail(CARVE_EINVAL, "confirm_enqueue: scan was made with another index");
  if (sc->fragments) return confirm_enqueue_impl<FragmentWindows, carve_match>(idx, sc, fragment_windows(sc));
  return confirm_enqueue_impl<OneImage, carve_match>(idx, sc, one_image(sc));
}

extern "C" int confirm_enqueue_to(const carve_index* idx, carve_scan* sc, carve_match* out, uint64_t cap) {
  if (!idx || !sc) return fail(CARVE_EINVAL, "confirm_enqueue_to: null argument");
  if (sc->batch) return fail(CARVE_EINVAL, "confirm_enqueue_to: a batch object (use batch_confirm_enqueue)");
  if (sc->idx != idx) return fail(CARVE_EINVAL, "confirm_enqueue_to: scan was made with another index");
  if (cap && !out) return fail(CARVE_EINVAL, "confirm_enqueue_to: null out with cap > 0");
  if (cap && !is_device_memory(out)) return fail(CARVE_EINVAL, "confirm_enqueue_to: out is not device memory");
  carve_match* dest = cap ? out : nullptr;
  if (sc->fragments)
    return confirm_enqueue_impl<FragmentWindows, carve_match>(idx, sc, fragment_windows(sc), dest, cap);
  return confirm_enqueue_impl<OneImage, carve_match>(idx, sc, one_image(sc), dest, cap);
}

extern "C" int batch_confirm_enqueue(const carve_index* idx, carve_batch* b) {
  if (!idx || !b) return fail(CARVE_EINVAL, "batch_confirm_enqueue: null argument");
  if (b->idx != idx) return fail(CARVE_EINVAL, "batch_confirm_enqueue: batch was made with another index");
  return confirm_enqueue_impl<ManyImages, carve_batch_match>(idx, b, many_images(b));
}

namespace {
int read_img_off(carve_batch* b) {
  CARVE_TRY(b->h_img_off.reserve((b->n_images + 1) * 8));
  HIP_TRY(hipMemcpyAsync(b->h_img_off.p, b->img_off.p, (b->n_images + 1) * 8, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return CARVE_OK;
}
}  // namespace

extern "C" int batch_flag_counts(carve_batch* b, uint64_t* counts, uint32_t n_images) {
  if (!b || (n_images && !counts)) return fail(CARVE_EINVAL, "batch_flag_counts: null argument");
  if (n_images != b->n_images) return fail(CARVE_EINVAL, "batch_flag_counts: the batch has %u images", b->n_images);
  if (!n_images) return CARVE_OK;
  CARVE_TRY(read_img_off(b));
  const uint64_t* off = b->h_img_off.as<uint64_t>();
  for (uint32_t i = 0; i < n_images; ++i) counts[i] = off[i + 1] - off[i];
  return CARVE_OK;
}

extern "C" int batch_flagged_sectors(carve_batch* b, uint32_t image, uint64_t* out, uint64_t cap, uint64_t* n_out) {
  if (!b || !n_out) return fail(CARVE_EINVAL, "batch_flagged_sectors: null argument");
  const bool all = image == CARVE_ALL_IMAGES;
  if (!all && image >= b->n_images) return fail(CARVE_EINVAL, "batch_flagged_sectors: image %u of %u", image,
                                                b->n_images);
  if (cap && !out) return fail(CARVE_EINVAL, "batch_flagged_sectors: null out with cap > 0");
  uint64_t first = 0, n = 0;
  if (all) {
    if (b->n_tiles) CARVE_TRY(read_u64(b, b->count.as<uint64_t>(), &n));
  } else {
    CARVE_TRY(read_img_off(b));
    const uint64_t* off = b->h_img_off.as<uint64_t>();
    first = off[image];
    n = off[image + 1] - off[image];
  }
  CARVE_TRY(copy_ids(b, first, n, out, cap));
  *n_out = n;
  if (n > cap) return fail(CARVE_ETRUNC, "batch_flagged_sectors: %llu flagged, capacity %llu",
                           (unsigned long long)n, (unsigned long long)cap);
  return CARVE_OK;
}

extern "C" int batch_confirm_matches(const carve_index* idx, carve_batch* b, carve_batch_match* out, uint64_t cap,
                                     uint64_t* n_out) {
  if (!idx || !b || !n_out) return fail(CARVE_EINVAL, "batch_confirm_matches: null argument");
  if (cap && !out) return fail(CARVE_EINVAL, "batch_confirm_matches: null out with cap > 0");
  if (b->idx != idx) return fail(CARVE_EINVAL, "batch_confirm_matches: batch was made with another index");
  return confirm_all(idx, b, many_images(b), out, cap, n_out);
}

// ------------------------------------------------------------ server hooks
CARVE_HIDDEN int carve_batch_reserve(const carve_index* idx, carve_batch** io, uint64_t n_sectors,
                                     uint32_t n_images, void* stream) {
  if (!idx || !io) return fail(CARVE_EINVAL, "carve_batch_reserve: null argument");
  carve_batch* b = *io;
  const bool created = !b;
  if (created) {
    b = new carve_batch();
    b->batch = true;
    (void)hipGetDevice(&b->device);
    b->stream = (hipStream_t)stream;
    b->idx = idx;
  }
  // every image may end in a partial tile
  const uint64_t tiles = cdiv(n_sectors, kTileSectors) + n_images;
  const uint64_t keep_tiles = b->n_tiles;
  const uint32_t keep_images = b->n_images;
  b->n_tiles = tiles;
  b->n_images = n_images;
  uint64_t room = 0;
  const size_t desc_bytes = ((size_t)n_images + 1) * sizeof(ImageDesc);
  int rc = reserve_scan(b);
  if (rc == CARVE_OK) rc = reserve_confirm<carve_batch_match>(b, tiles * kTileSectors, &room);
  if (rc == CARVE_OK) rc = b->d_desc.reserve(desc_bytes);
  if (rc == CARVE_OK) rc = b->h_desc.reserve(desc_bytes);
  b->n_tiles = keep_tiles;
  b->n_images = keep_images;
  if (rc != CARVE_OK) {
    if (created) free_batch(b);
    return rc;
  }
  *io = b;
  return CARVE_OK;
}

CARVE_HIDDEN int carve_batch_stage_out(carve_batch* b, int with_matches, const carve_stage_out* st,
                                       uint64_t* match_room) {
  if (!b || !st || !match_room || !st->totals || !st->img_off || (st->ids_cap && !st->ids) ||
      (st->match_cap && !st->matches))
    return fail(CARVE_EINVAL, "carve_batch_stage_out: null argument");
  if (with_matches && !b->confirm_enqueued)
    return fail(CARVE_EINVAL, "carve_batch_stage_out: confirmation was not enqueued");
  // an empty tile space writes no counts: stage zeros (the offsets are zero-filled)
  const bool counted = b->n_tiles != 0;
  if (!counted) k_fill_u64<<<1, 64, 0, b->stream>>>(b->count.as<uint64_t>(), 2, 0);
  const uint64_t room = with_matches && counted ? b->rec_cap : 0;
  *match_room = room;
  const uint64_t most = st->ids_cap + 3 * st->match_cap + b->n_images + 1;
  const uint64_t want = cdiv(most, 256);
  k_stage_out<<<(unsigned)(want < 1024 ? (want ? want : 1) : 1024), 256, 0, b->stream>>>(
      b->count.as<uint64_t>(), with_matches, b->n_images, b->img_off.as<uint64_t>(), b->ids.as<uint64_t>(),
      b->matches.as<uint64_t>(), room, st->totals, st->img_off, st->ids, st->ids_cap, (uint64_t*)st->matches,
      st->match_cap);
  HIP_TRY(hipGetLastError());
  return CARVE_OK;
}

namespace {
// Mean kernel time of the scan of a sample image with the index's current
// launch shape: one warm-up run, then at least 5 timed runs and about 8 ms of
// kernel time (a small sample needs more runs to rank shapes). *sc is reused.
int time_scan(carve_index* idx, const void* sample, uint64_t n_bytes, void* stream, carve_scan** sc, float* mean) {
  float total = 0.f;
  int timed = 0;
  for (int rep = 0;; ++rep) {
    CARVE_TRY(scan_image(idx, sample, n_bytes, 0, CARVE_TAU_PER_CLUSTER, stream, sc));
    if (rep == 0) {
      CARVE_TRY(scan_set_timing(*sc, 1));   // the first run only warms up
      continue;
    }
    float ms = 0.f;
    CARVE_TRY(scan_kernel_ms(*sc, &ms));
    total += ms;
    ++timed;
    if (timed >= 5 && (total >= 8.f || timed >= 64)) break;
  }
  *mean = total / (float)timed;
  return CARVE_OK;
}

// Mean kernel time of the batch scan (the kernel batches and the server run)
// over the sample cut into 16 images of uneven sizes (piece i about (i + 1)/136
// of it, cluster-aligned), timed as time_scan does. *b is reused.
int time_batch(carve_index* idx, const void* sample, uint64_t n_bytes, void* stream, carve_batch** b, float* mean) {
  constexpr uint32_t kPieces = 16;
  const uint64_t n_sec = n_bytes / kSectorBytes;
  carve_image_desc d[kPieces];
  uint64_t at = 0;
  for (uint32_t i = 0; i < kPieces; ++i) {
    uint64_t len = n_sec * (i + 1) / (kPieces * (kPieces + 1) / 2);
    len -= len % kClusterSectors;
    if (i == kPieces - 1 || at + len > n_sec) len = n_sec - at;
    d[i] = carve_image_desc{(const uint8_t*)sample + at * kSectorBytes, len * kSectorBytes, 0, CARVE_TAU_PER_CLUSTER};
    at += len;
  }
  float total = 0.f;
  int timed = 0;
  for (int rep = 0;; ++rep) {
    CARVE_TRY(scan_batch(idx, d, kPieces, stream, b));
    if (rep == 0) {
      CARVE_TRY(scan_set_timing(*b, 1));
      continue;
    }
    float ms = 0.f;
    CARVE_TRY(scan_kernel_ms(*b, &ms));
    total += ms;
    ++timed;
    if (timed >= 5 && (total >= 8.f || timed >= 64)) break;
  }
  *mean = total / (float)timed;
  return CARVE_OK;
}

// time_scan, or time_batch for an index that will serve batches.
int time_walk(carve_index* idx, const void* sample, uint64_t n_bytes, void* stream, bool batches, carve_scan** sc,
              float* mean) {
  if (!batches) return time_scan(idx, sample, n_bytes, stream, sc, mean);
  carve_batch* b = (*sc && (*sc)->batch) ? static_cast<carve_batch*>(*sc) : nullptr;
  if (*sc && !(*sc)->batch) {
    free_scan(*sc);
    *sc = nullptr;
  }
  const int rc = time_batch(idx, sample, n_bytes, stream, &b, mean);
  *sc = b;
  return rc;
}

// The walks a per-cluster scan of one image can take with this index.
std::vector<uint32_t> split_modes(const carve_index* idx, bool contiguous_only) {
  if (!idx->bloom_tau.bytes || contiguous_only) return {CARVE_SPLIT_OFF};
  return {CARVE_SPLIT_OFF, CARVE_SPLIT_ON};
}

// Every launch shape (blocks per CU x tiles per chunk x walk) timed on the
// sample (contiguous_only: the batch kernel, on the sample cut into images);
// the index keeps the fastest. *best_ms receives its mean kernel time.
int tune_shapes(carve_index* idx, const void* sample, uint64_t n_bytes, void* stream, bool contiguous_only,
                carve_scan_config* best, float* best_ms) {
  const carve_scan_config saved = idx->cfg;
  carve_scan* sc = nullptr;
  carve_scan_config winner = saved;
  float winner_ms = 1e30f;
  const uint32_t blocks[] = {0, 3, 2};
  const uint32_t chunks[] = {1, 2, 4, 8, 16};
  int rc = CARVE_OK;
  for (uint32_t sp : split_modes(idx, contiguous_only)) {
    for (uint32_t bpc : blocks) {
      for (uint32_t ch : chunks) {
        idx->cfg = carve_scan_config{bpc, ch, sp, 0};
        float mean = 0.f;
        if ((rc = time_walk(idx, sample, n_bytes, stream, contiguous_only, &sc, &mean)) != CARVE_OK) break;
        if (mean < winner_ms) {
          winner_ms = mean;
          winner = idx->cfg;
        }
      }
      if (rc != CARVE_OK) break;
    }
    if (rc != CARVE_OK) break;
  }
  free_scan(sc);
  idx->cfg = rc == CARVE_OK ? winner : saved;
  if (rc == CARVE_OK) {
    if (best) *best = winner;
    if (best_ms) *best_ms = winner_ms;
  }
  return rc;
}

int check_sample(const carve_index* idx, const void* sample, uint64_t n_bytes, const char* who) {
  if (idx && idx->unit_bytes != kSectorBytes) return fail(CARVE_EINVAL, "%s: a fragment index", who);
  if (n_bytes < kSectorBytes) return fail(CARVE_EINVAL, "%s: the sample needs at least one sector", who);
  CARVE_TRY(validate_image(sample, n_bytes, 0, CARVE_TAU_PER_CLUSTER, who, -1));
  if (!gpu_readable(sample)) return fail(CARVE_EINVAL, "%s: the sample is not in device memory", who);
  return CARVE_OK;
}
}  // namespace

extern "C" int autotune_scan(carve_index* idx, const void* sample_image, uint64_t n_bytes, void* stream,
                             carve_scan_config* best) {
  if (!idx) return fail(CARVE_EINVAL, "autotune_scan: null index");
  CARVE_TRY(check_sample(idx, sample_image, n_bytes, "autotune_scan"));
  return tune_shapes(idx, sample_image, n_bytes, stream, false, best, nullptr);
}

// ------------------------------------------------------------ index autotuner
namespace {
struct TunePick {
  carve_index_params params;
  carve_scan_config cfg;
  float ms;
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, TunePick>> g_tune_cache;

// The cache key: the device's architecture, the signature kind, the master
// count's power-of-two class, the load ceiling and the candidate space.
int tune_key(const carve_index_params& base, const carve_tune_space& sp, uint64_t n_masters, std::string* key) {
  int dev = 0;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  uint32_t cls = 0;
  while ((1ull << cls) < n_masters) ++cls;
  char buf[512];
  int n = snprintf(buf, sizeof buf, "%s|sig%u|m2^%u|load%.3f|lay%x|flags%x|bloom", prop.gcnArchName, base.sig_kind, cls,
                   (double)base.max_load, sp.layouts, sp.flags & ~(uint32_t)CARVE_TUNE_NO_CACHE);
  for (uint32_t i = 0; i < sp.n_bloom && n > 0 && n < (int)sizeof buf; ++i)
    n += snprintf(buf + n, sizeof buf - n, ",%u", sp.bloom_bits[i]);
  *key = buf;
  return CARVE_OK;
}
}  // namespace

extern "C" int autotune_index(const void* master_sectors, const uint64_t* file_sector_offsets, uint32_t n_files,
                              const carve_index_params* base, const carve_tune_space* space, const void* sample_image,
                              uint64_t n_bytes, void* stream, carve_index** out, carve_tune_result* result) {
  if (!out) return fail(CARVE_EINVAL, "autotune_index: out is null");
  *out = nullptr;
  CARVE_TRY(check_sample(nullptr, sample_image, n_bytes, "autotune_index"));
  carve_index_params b{};
  if (base) b = *base;
  carve_tune_space sp{};
  if (space) sp = *space;
  if (sp.n_bloom > 8 || sp.reserved[0] || sp.reserved[1] || (sp.layouts & ~7u))
    return fail(CARVE_EINVAL, "autotune_index: bad tuning space");
  if (sp.flags & ~(uint32_t)(CARVE_TUNE_NO_CACHE | CARVE_TUNE_CONTIGUOUS))
    return fail(CARVE_EINVAL, "autotune_index: unknown flags");
  if (!sp.layouts) sp.layouts = 7u;
  if (!sp.n_bloom) {   // the automatic size, then 8, 16 and 32 bits per signature
    const uint32_t dflt[] = {0, 8, 16, 32};
    sp.n_bloom = 4;
    for (uint32_t i = 0; i < 4; ++i) sp.bloom_bits[i] = dflt[i];
  }
  if (b.max_load == 0.f) b.max_load = 0.5f;
  const bool contiguous = (sp.flags & CARVE_TUNE_CONTIGUOUS) != 0;
  const uint64_t n_masters = n_files && file_sector_offsets ? file_sector_offsets[n_files] : 0;
  std::string key;
  CARVE_TRY(tune_key(b, sp, n_masters, &key));
  carve_tune_result res{};
  if (!(sp.flags & CARVE_TUNE_NO_CACHE)) {
    TunePick hit{};
    bool found = false;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      for (const auto& e : g_tune_cache)
        if (e.first == key) {
          hit = e.second;
          found = true;
        }
    }
    if (found) {   // the pick of an earlier tuning of this class: build it, no timing
      carve_index* ix = nullptr;
      CARVE_TRY(build_master_index(master_sectors, file_sector_offsets, n_files, &hit.params, stream, &ix));
      ix->cfg = hit.cfg;
      res.params = hit.params;
      res.config = hit.cfg;
      res.kernel_ms = hit.ms;
      res.from_cache = 1;
      if (result) *result = res;
      *out = ix;
      return CARVE_OK;
    }
  }
  // Stage 1: every (layout, filter) candidate at one launch shape, each walk,
  // the first candidate of the space (the default, bucketed with the
  // automatic filter, when the space holds it) first; a later candidate
  // replaces the best only when it is more than 1% faster: on a sample,
  // differences below that are noise and do not carry over to the images.
  // Stage 2: the picked candidate's full launch-shape sweep.
  constexpr float kClearGain = 0.99f;
  carve_index* best = nullptr;
  carve_index_params best_p{};
  float best_ms = 1e30f;
  carve_scan* sc = nullptr;
  int rc = CARVE_OK;
  for (uint32_t layout = 0; layout < 3 && rc == CARVE_OK; ++layout) {
    if (!((sp.layouts >> layout) & 1u)) continue;
    for (uint32_t i = 0; i < sp.n_bloom && rc == CARVE_OK; ++i) {
      carve_index_params p = b;
      p.layout = layout;
      p.bloom_bits_per_key = sp.bloom_bits[i];
      carve_index* ix = nullptr;
      if ((rc = build_master_index(master_sectors, file_sector_offsets, n_files, &p, stream, &ix)) != CARVE_OK) break;
      ++res.candidates;
      float cand_ms = 1e30f;
      for (uint32_t w : split_modes(ix, contiguous)) {
        ix->cfg = carve_scan_config{2, 1, w, 0};
        float ms = 0.f;
        if ((rc = time_walk(ix, sample_image, n_bytes, stream, contiguous, &sc, &ms)) != CARVE_OK) break;
        if (ms < cand_ms) cand_ms = ms;
      }
      free_scan(sc);   // a scan object belongs to one index
      sc = nullptr;
      if (rc == CARVE_OK && (!best || cand_ms < best_ms * kClearGain)) {
        free_index(best);
        best = ix;
        best_p = p;
        best_ms = cand_ms;
      } else {
        free_index(ix);
      }
    }
  }
  if (rc == CARVE_OK && !best) rc = fail(CARVE_EINVAL, "autotune_index: no candidate");
  carve_scan_config cfg{};
  if (rc == CARVE_OK) rc = tune_shapes(best, sample_image, n_bytes, stream, contiguous, &cfg, &best_ms);
  if (rc != CARVE_OK) {
    free_index(best);
    return rc;
  }
  res.params = best_p;
  res.config = cfg;
  res.kernel_ms = best_ms;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    bool replaced = false;
    for (auto& e : g_tune_cache)
      if (e.first == key) {
        e.second = TunePick{best_p, cfg, best_ms};
        replaced = true;
      }
    if (!replaced) g_tune_cache.emplace_back(key, TunePick{best_p, cfg, best_ms});
  }
  if (result) *result = res;
  *out = best;
  return CARVE_OK;
}

CARVE_HIDDEN uint32_t carve_index_unit_bytes(const carve_index* idx) { return idx ? idx->unit_bytes : 0; }
