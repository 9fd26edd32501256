// Fragment scan (Section 5): every 64-byte window of an image that starts on
// a 4-byte boundary (window j = bytes [4j, 4j + 64)), hashed with djb2 over
// its 64 bytes (Eq. (1)), looked up among the signatures of the master files'
// 64-byte fragments at any position. Device code only; included by carve.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "carve_device.h"
#include "carve_scan_kernel.h"

namespace carve {

constexpr uint32_t kFragBytes = 64;                          // a master fragment, an image window
constexpr uint32_t kWindowStride = 4;                        // windows start on 4-byte boundaries
constexpr uint32_t kFragThreads = 1024;                      // one block per CU: its LDS holds the filter
constexpr uint32_t kFragWaves = kFragThreads / kWave;
constexpr uint32_t kLaneWindows = 16;                        // consecutive windows per lane
constexpr uint32_t kWaveWindows = kWave * kLaneWindows;      // 1024 windows = 4 KiB of image per wave task
constexpr uint32_t kFragRowDw = kLaneWindows;                // a lane's own 64 bytes, in dwords
constexpr uint32_t kLdsFilterMaxWords = 40960;               // 160 KiB, all of a CU's LDS: the first filter
constexpr int kDppWaveShl1 = 0x130;                          // DPP control: lane i takes lane i + 1's value
// Buffer descriptor word 3 for raw (unformatted, unswizzled) dword access on
// gfx9-family chips: data format 32 in bits 15-18 (value 4), the rest 0.
constexpr int kRawBufferFlags = 0x00020000;

// The two filters of a fragment index, both of 32-bit words, are placed from
// a 32-bit key: k = H mod 2^32, the low half of the window's data part H (its
// signature minus the constant 5381*33^64, below). Eq. (1) reduced modulo 2^32
// is the same recurrence (reduction modulo 2^32 respects sums and products),
// so the scan rolls k with 32-bit arithmetic alone, and equal signatures give
// equal keys; the full 64-bit signature is formed only for the rare windows
// that pass both filters. Rolling H rather than the signature drops the
// constant term from every step.
// Each level takes one 32 x 32 -> 64-bit product of the key (a = k * kFragMulA,
// b = k * kFragMulB; one multiply-add instruction each, the only full 32-bit
// multiplies of a lookup):
// * first level, in LDS: the word from the low 24 bits of a's high half scaled
//   to the word count (a 24-bit multiply, which need not be a power of two),
//   2 bit positions from bits 24-28 of a's high and of a's low half;
// * second level, the Bloom filter in L2: the word from the top bits of b's
//   low half, 3 bit positions from bits 0-4, 16-20 and 24-28 of b's high half.
// Bit positions sit at byte and half-word boundaries so that the scan's shifts
// take them straight from the product's register (sub-dword operand selects).
// A simulation of the logos set's filters on random keys: both levels pass
// 0.033% of windows; 3 Bloom bits keep the exact path rare for two
// instructions fewer than 4. Only windows that pass the first level read the
// second. Key 0 is placed like any other; when a master's whole signature is
// 0 (it lives beside the table, not in it) the build sets the bits of its key
// in both filters, so no value needs special handling in the scan.
constexpr uint32_t kFragMulA = 0x9E3779B1u;
constexpr uint32_t kFragMulB = 0x85EBCA77u;
// A first-level lookup: the word and the 2 bit positions (each < 32).
struct FragLdsProbe {
  uint32_t word, p0, p1;
};
// n_words in 1..kLdsFilterMaxWords (so n_words * 256 < 2^24).
__device__ __forceinline__ FragLdsProbe frag_lds_probe(uint32_t key, uint32_t n_words) {
  const uint64_t a = (uint64_t)key * kFragMulA;
  const uint32_t hi = (uint32_t)(a >> 32), lo = (uint32_t)a;
  FragLdsProbe r;
  const uint32_t n8 = (n_words << 8) & 0xFFFFFFu;   // both factors 24-bit: a 24-bit multiply
  r.word = (uint32_t)(((uint64_t)(hi & 0xFFFFFFu) * n8) >> 32);   // < n_words
  r.p0 = (hi >> 24) & 31u;
  r.p1 = (lo >> 24) & 31u;
  return r;
}
// A second-level lookup: the word's byte offset and the 3 bit positions.
struct FragBloomProbe {
  uint32_t byte_off, p0, p1, p2;
};
// log2_words in 1..30 (the filter has 2 to 2^30 words).
__device__ __forceinline__ FragBloomProbe frag_bloom_probe(uint32_t key, uint32_t log2_words) {
  const uint64_t b = (uint64_t)key * kFragMulB;
  const uint32_t hi = (uint32_t)(b >> 32), lo = (uint32_t)b;
  FragBloomProbe r;
  r.byte_off = (lo >> (30 - log2_words)) & ~3u;   // the word (top log2_words bits of lo) times 4
  r.p0 = hi & 31u;
  r.p1 = (hi >> 16) & 31u;
  r.p2 = (hi >> 24) & 31u;
  return r;
}
// The build's view: the word and its bits.
__device__ __forceinline__ void frag_lds_place(uint32_t key, uint32_t n_words, uint32_t* word, uint32_t* bits) {
  const FragLdsProbe r = frag_lds_probe(key, n_words);
  *word = r.word;
  *bits = (1u << r.p0) | (1u << r.p1);
}
__device__ __forceinline__ void frag_bloom_place(uint32_t key, uint32_t log2_words, uint32_t* word, uint32_t* bits) {
  const FragBloomProbe r = frag_bloom_probe(key, log2_words);
  *word = r.byte_off >> 2;
  *bits = (1u << r.p0) | (1u << r.p1) | (1u << r.p2);
}
// The scan's view: 1 when all of a probe's bits are set in the filter word x
// (the word shifted by each position and the low bits combined: fewer
// instructions than a mask built and compared).
__device__ __forceinline__ uint32_t frag_lds_has(uint32_t x, const FragLdsProbe& r) {
  return (x >> r.p0) & (x >> r.p1) & 1u;
}
__device__ __forceinline__ uint32_t frag_bloom_has(uint32_t x, const FragBloomProbe& r) {
  return (x >> r.p0) & (x >> r.p1) & (x >> r.p2) & 1u;
}

// Rolling Eq. (1) over a 64-byte window by 4 bytes. With the window's data
// part H(j) = sum_{i<64} s[4j+i] 33^(63-i) (its signature is 5381*33^64 + H)
// and D(w) = b0 33^3 + b1 33^2 + b2 33 + b3 for the bytes of word w in address
// order (D < 2^24):
//   H(j+1) = H(j) 33^4 - 33^64 D(j) + D(j+16)        (mod 2^64)
// and the first window is Horner over its 16 words: H = H 33^4 + D(k). On the
// signatures themselves, sig(j) = 5381*33^64 + H(j):
//   sig(j+1) = sig(j) 33^4 + D(j+16) + [5381*33^64 (1 - 33^4) - 33^64 D(j)]
// where the bracket is one multiply-add of D(j) with constants.
constexpr uint64_t kPow4 = pow33(4);
constexpr uint64_t kPow64 = pow33(kFragBytes);
constexpr uint64_t kFragInit = 5381ull * pow33(kFragBytes);
constexpr uint64_t kRollAdd = kFragInit - kFragInit * kPow4;   // mod 2^64
constexpr uint64_t kNegPow64 = 0ull - kPow64;                  // mod 2^64
// the constants modulo 2^32 that roll the filter key H mod 2^32
constexpr uint32_t kPow4Lo = (uint32_t)kPow4;
constexpr uint32_t kFragInitLo = (uint32_t)kFragInit;
constexpr uint32_t kNegPow64Lo = (uint32_t)kNegPow64;
// The filter key of a signature: its data part modulo 2^32.
__device__ __forceinline__ uint32_t frag_filter_key(uint64_t sig) { return (uint32_t)sig - kFragInitLo; }

// The byte weights of D in dot4 form: D = dot(word, low bytes of 33^(3-i))
// + 256 dot(word, second bytes of 33^(3-i)) (33^3 < 2^16).
constexpr uint32_t word_weights(uint32_t shift) {
  uint32_t w = 0;
  for (uint32_t k = 0; k < 4; ++k) w |= (uint32_t)((pow33(3 - k) >> shift) & 0xFFu) << (8 * k);
  return w;
}
constexpr uint32_t kWordWeightsLo = word_weights(0);
constexpr uint32_t kWordWeightsHi = word_weights(8);

__device__ __forceinline__ uint32_t word_djb2(uint32_t x) {
  return __builtin_amdgcn_udot4(x, kWordWeightsLo, 0u, false) +
         (__builtin_amdgcn_udot4(x, kWordWeightsHi, 0u, false) << 8);
}

// Signature of a whole 64-byte fragment (16 words, little-endian dwords).
__device__ __forceinline__ uint64_t fragment_signature(const uint32_t* w) {
  uint64_t H = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) H = H * kPow4 + word_djb2(w[k]);
  return kFragInit + H;
}

// The windows of one image as a tile space for compaction and confirmation:
// unit j is bytes [4j, 4j + 64); d.n_sectors holds the number of windows.
struct FragmentWindows {
  static constexpr uint32_t kUnitBytes = kFragBytes, kUnitStride = kWindowStride;
  static constexpr bool kAnyPosition = true;
  ImageDesc d;
  __device__ __forceinline__ uint64_t n_tiles() const { return (d.n_sectors + kTileSectors - 1) / kTileSectors; }
  __device__ __forceinline__ const ImageDesc& image(uint32_t) const { return d; }
  __device__ __forceinline__ uint32_t image_of_tile(uint64_t) const { return 0; }
};

// find_slot reading each bucket as two 64-byte halves in turn. k_insert
// claims a bucket's slots in order (and nothing is ever removed), so the
// occupied slots of a bucket are a prefix of it: a free slot in the first
// half ends the search there. At load 1/2 or less most probes read one half
// (a fragment index: about 91% of buckets hold at most 8 keys).
__device__ __forceinline__ int64_t find_slot_halves(const IndexView& ix, uint64_t h) {
  constexpr uint32_t kHalf = kBucketSlots / 2;
  const uint32_t nb_mask = (1u << ix.log2_buckets) - 1u;
  uint32_t b = bucket_of(h, ix.log2_buckets);
  for (uint32_t it = 0; it <= nb_mask; ++it) {
#pragma unroll
    for (uint32_t half = 0; half < 2; ++half) {
      const uint64_t first = (uint64_t)b * kBucketSlots + half * kHalf;
      const u64x2* p = (const u64x2*)(ix.keys + first);
      u64x2 kv[kHalf / 2];
#pragma unroll
      for (int c = 0; c < (int)(kHalf / 2); ++c) kv[c] = p[c];
      int64_t found = -1;
      bool any_empty = false;
#pragma unroll
      for (int c = 0; c < (int)(kHalf / 2); ++c) {
        if (kv[c].x == h) found = (int64_t)(first + 2 * c);
        if (kv[c].y == h) found = (int64_t)(first + 2 * c + 1);
        any_empty |= (kv[c].x == kEmptyKey) | (kv[c].y == kEmptyKey);
      }
      if (found >= 0) return found;
      if (any_empty) return -1;
    }
    b = (b + 1) & nb_mask;
  }
  return -1;
}

// A task's image words for lane l: its 16 own dwords (dwords 16l..16l+15 of
// the task) and, in lanes 0-15, dword 1024 + (l mod 16) (the next task's first
// words, which lane 63's windows reach). Every task but the image's last lies
// wholly inside the image (n_dwords >= n_windows + 15) and uses 16-byte loads;
// the last task clamps every dword to the image's last one (only windows past
// the end read the repeated words).
struct TaskWords {
  u32x4 v[kFragRowDw / 4];
  uint32_t x;
};
// The inside task's words come by buffer loads from a descriptor based at
// the task (scalar base, 32-bit lane offsets: less address arithmetic than
// 64-bit global addresses), streaming and system-scoped (cache policy nt, sc1):
// on the 2 GiB logos workload 1.187 vs 1.211 ms for non-temporal global loads,
// and 74 MB less fetched per launch. The image is only read, so the policy
// affects speed alone.
constexpr int kImagePolicy = 2 | 16;   // nt | sc1
__device__ __forceinline__ void load_task_inside(const uint32_t* __restrict__ image, uint64_t t, uint32_t l,
                                                 TaskWords& T) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(image + t * kWaveWindows), (short)0, 0x7FFFFFFF, kRawBufferFlags);
#pragma unroll
  for (uint32_t q = 0; q < kFragRowDw / 4; ++q) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((l * kFragRowDw + 4 * q) * 4), 0, kImagePolicy);
    T.v[q] = u32x4{v[0], v[1], v[2], v[3]};
  }
  T.x = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)((kWaveWindows + (l % kFragRowDw)) * 4), 0, kImagePolicy);
}
__device__ __forceinline__ void load_task_clamped(const uint32_t* __restrict__ image, uint64_t n_dwords, uint64_t t,
                                                  uint32_t l, TaskWords& T) {
  const uint64_t dw0 = t * kWaveWindows;
#pragma unroll
  for (uint32_t k = 0; k < kFragRowDw; ++k) {
    const uint64_t g = dw0 + (uint64_t)l * kFragRowDw + k;
    T.v[k / 4][k % 4] = image[g < n_dwords ? g : n_dwords - 1];
  }
  const uint64_t g = dw0 + kWaveWindows + (l % kFragRowDw);
  T.x = image[g < n_dwords ? g : n_dwords - 1];
}

// One task of a wave (see k_frag_scan). kBloom: the index has the second
// filter (a compile-time choice: no branch around the filter's loads).
template <bool kBloom>
__device__ __forceinline__ void frag_task(uint64_t n_windows, uint64_t n_words, const IndexView& ix,
                                          const uint32_t* lfilter, uint32_t lw, uint64_t t, uint32_t l,
                                          const TaskWords& cur, uint64_t* __restrict__ out,
                                          uint32_t* __restrict__ hit_slot) {
  const char* bloom = (const char*)ix.bloom;   // fragment indexes: 32-bit words
  const uint32_t lwb = ix.log2_bloom_words + 1;
  // Wave priority by stage: a wave whose image words have arrived goes first
  // until its Bloom loads are issued (3), then the Bloom check and the exact
  // path (1), then the store (0), so the waves' long filter lookups start as
  // early as possible: 1.136 vs 1.191 ms on the 2 GiB logos workload (3
  // through the Bloom issue and 0 after it: 1.139-1.147 ms; 3 only around
  // the Bloom issue: 1.156-1.164 ms; 3 around the image loads: no change).
  __builtin_amdgcn_s_setprio(3);
  // d[k] = D(dword 16l + k) of the task; dx = D of dword 1024 + (l % 16)
  uint32_t d[kFragRowDw];
#pragma unroll
  for (uint32_t k = 0; k < kFragRowDw; ++k) d[k] = word_djb2(cur.v[k / 4][k % 4]);
  const uint32_t dx = word_djb2(cur.x);
  // nx[k] = D(dword 16l + 16 + k): the next lane's d[k]; for lane 63, lane
  // k's dx (the whole wave runs this code, so every source lane is active).
  // Lane 63's value arrives first by a permute (lane 63 reads lane k; the
  // other lanes read lanes below 31 and are overwritten), then a wave-wide
  // shift by one lane moves d[k] down into lanes 0-62 and leaves lane 63,
  // which has no source, as it was: one vector instruction per word.
  const uint32_t ext_from = l == kWave - 1 ? 0u : 4u * (l % kFragRowDw);   // byte address of a lane
  uint32_t nx[kFragRowDw];
#pragma unroll
  for (uint32_t k = 0; k < kFragRowDw; ++k) {
    const int ext = __builtin_amdgcn_ds_bpermute((int)(ext_from + 4u * k), (int)dx);
    nx[k] = (uint32_t)__builtin_amdgcn_update_dpp(ext, (int)d[k], kDppWaveShl1, 0xF, 0xF, false);
  }
  const uint64_t j0 = t * kWaveWindows + (uint64_t)l * kLaneWindows;
  const uint32_t valid = j0 >= n_windows ? 0u : (n_windows - j0 >= kLaneWindows ? kLaneWindows
                                                                                 : (uint32_t)(n_windows - j0));
  // filter keys (H mod 2^32) of the lane's 16 windows: Horner over the first
  // window's words, then the rolling update modulo 2^32
  uint32_t s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kFragRowDw; ++k) s = s * kPow4Lo + d[k];
  uint32_t h[kLaneWindows];
#pragma unroll
  for (uint32_t w = 0; w < kLaneWindows; ++w) {
    h[w] = s;
    s = s * kPow4Lo + kNegPow64Lo * d[w] + nx[w];   // unused after the last window
  }
  // windows still candidates after both filters
  uint32_t pend = valid >= 16 ? 0xFFFFu : (1u << valid) - 1u;
  uint32_t pass = 0;
#pragma unroll
  for (uint32_t w = 0; w < kLaneWindows; ++w) {
    const FragLdsProbe r = frag_lds_probe(h[w], lw);
    pass |= frag_lds_has(lfilter[r.word], r) << w;
  }
  pend &= pass;
  // the Bloom words, all in flight together: a window that failed the LDS
  // filter reads the filter's first word, the same address in every such
  // lane, and its bits are dropped (no branches)
  if constexpr (kBloom) {
    FragBloomProbe r[kLaneWindows];
    uint32_t fw[kLaneWindows];
#pragma unroll
    for (uint32_t w = 0; w < kLaneWindows; ++w) {
      r[w] = frag_bloom_probe(h[w], lwb);
      const uint32_t keep = 0u - ((pend >> w) & 1u);   // all ones or zero
      fw[w] = *(const uint32_t*)(bloom + (r[w].byte_off & keep));
    }
    __builtin_amdgcn_s_setprio(1);
    pass = 0;
#pragma unroll
    for (uint32_t w = 0; w < kLaneWindows; ++w) pass |= frag_bloom_has(fw[w], r[w]) << w;
    pend &= pass;
  } else {
    __builtin_amdgcn_s_setprio(1);
  }
  // The candidates (rare: about one window in 3000 of random data, besides
  // the true hits) take the exact test with the full 64-bit signature,
  // rolled across the lane's 16 windows in the lanes that have one.
  uint32_t mask = 0;
  if (pend) {
    uint64_t H = 0;
#pragma unroll
    for (uint32_t k = 0; k < kFragRowDw; ++k) H = H * kPow4 + d[k];
    uint64_t sig = kFragInit + H;
#pragma unroll
    for (uint32_t w = 0; w < kLaneWindows; ++w) {
      if ((pend >> w) == 0u) break;   // no candidate left in this lane
      if ((pend >> w) & 1u) {
        int64_t slot = -1;
        if (sig == kEmptyKey) {
          if (ix.zero_sig_mask) slot = ix.zero_slot;
        } else {
          slot = find_slot_halves(ix, sig);   // any position: every occupied slot has masters
        }
        if (slot >= 0) {
          mask |= 1u << w;
          hit_slot[j0 + w] = (uint32_t)slot;
        }
      }
      sig = sig * kPow4 + (kRollAdd + kNegPow64 * d[w]) + nx[w];
    }
  }
  __builtin_amdgcn_s_setprio(0);
  // four lanes' 16-bit masks make one 64-bit hit word
  const uint32_t m1 = (uint32_t)__shfl_down((int)mask, 1, kWave);
  const uint32_t m2 = (uint32_t)__shfl_down((int)mask, 2, kWave);
  const uint32_t m3 = (uint32_t)__shfl_down((int)mask, 3, kWave);
  const uint64_t wi = t * (kWaveWindows / kTileSectors) + l / 4;
  if ((l & 3u) == 0 && wi < n_words)
    out[wi] = (uint64_t)(mask | (m1 << 16)) | ((uint64_t)(m2 | (m3 << 16)) << 32);
}

// Persistent grid of one block per CU; wave q takes tasks q, q + W, ...
// (W = waves in the grid). Task t: windows [1024t, 1024t + 1024); lane l
// rolls over windows 16l..16l+15 of it, and lanes 4m..4m+3 make hit word
// 16t + m (bit b = window 64(16t+m)+b). For each hit the matched table slot
// goes to hit_slot[window]. The block's LDS holds only the first filter; the
// image goes straight to registers. Requesting the next task's words ahead,
// behind the current task's Bloom words, was measured slower (1.34 vs
// 1.23 ms on the 2 GiB logos workload, and 0.47 GB more fetched): the extra
// image data in flight displaced Bloom words from L2.
template <bool kBloom>
__global__ __launch_bounds__(kFragThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_frag_scan(
    const uint32_t* __restrict__ image, uint64_t n_windows, uint64_t n_dwords, IndexView ix,
    uint64_t* __restrict__ out, uint32_t* __restrict__ hit_slot) {
  __shared__ uint32_t lfilter[kLdsFilterMaxWords];
  const uint32_t lw = ix.lds_words;   // at most kLdsFilterMaxWords
  for (uint32_t i = threadIdx.x; i < lw; i += kFragThreads) lfilter[i] = ix.lds_filter[i];
  __syncthreads();   // before any wave of the block can leave
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const uint32_t l = lane_id();
  const uint64_t n_tasks = (n_windows + kWaveWindows - 1) / kWaveWindows;
  const uint64_t n_words = (n_windows + kTileSectors - 1) / kTileSectors;
  const uint64_t n_waves = (uint64_t)gridDim.x * kFragWaves;
  const uint64_t last = n_tasks - 1;   // n_windows >= 1 (the host launches nothing otherwise)
  for (uint64_t t = (uint64_t)blockIdx.x * kFragWaves + wv; t < n_tasks; t += n_waves) {
    TaskWords cur;
    if (t < last) load_task_inside(image, t, l, cur);   // uniform branch
    else load_task_clamped(image, n_dwords, t, l, cur);
    frag_task<kBloom>(n_windows, n_words, ix, lfilter, lw, t, l, cur, out, hit_slot);
  }
}

}  // namespace carve
