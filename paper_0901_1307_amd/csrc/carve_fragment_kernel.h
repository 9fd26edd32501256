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

// The two filters of a fragment index, both of 32-bit words. Their positions
// come from two 32 x 32 -> 64-bit products of the signature's halves,
// a = hi * kFragMulA and b = lo * kFragMulB (one multiply-add instruction
// each); a word index comes from the top bits of a product's low half
// (multiplicative hashing), bit positions are 5-bit fields of its high half:
// * first level, in LDS: word from a (the low half scaled to the word count,
//   which need not be a power of two), 2 bits from a's high half;
// * second level, the Bloom filter in L2: word from b, 4 bits from b's high half.
// Only windows that pass the first level read the second.
constexpr uint32_t kFragMulA = 0x9E3779B1u;
constexpr uint32_t kFragMulB = 0x85EBCA77u;
__device__ __forceinline__ void frag_lds_place(uint64_t h, uint32_t n_words, uint32_t* word, uint32_t* bits) {
  const uint64_t a = (uint64_t)(uint32_t)(h >> 32) * kFragMulA;
  const uint32_t a_hi = (uint32_t)(a >> 32);
  *word = (uint32_t)(((uint64_t)(uint32_t)a * n_words) >> 32);   // < n_words
  *bits = (1u << (a_hi & 31u)) | (1u << ((a_hi >> 5) & 31u));
}
__device__ __forceinline__ void frag_bloom_place(uint64_t h, uint32_t log2_words, uint32_t* word, uint32_t* bits) {
  const uint64_t b = (uint64_t)(uint32_t)h * kFragMulB;
  const uint32_t b_hi = (uint32_t)(b >> 32);
  *word = log2_words ? (uint32_t)b >> (32 - log2_words) : 0u;   // log2_words in 0..32
  *bits = (1u << (b_hi & 31u)) | (1u << ((b_hi >> 5) & 31u)) | (1u << ((b_hi >> 10) & 31u)) |
          (1u << ((b_hi >> 15) & 31u));
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

// Persistent grid of one block per CU; wave q takes tasks q, q + W, ...
// (W = waves in the grid). Task t: windows [1024t, 1024t + 1024); lane l
// rolls over windows 16l..16l+15 of it, and lanes 4m..4m+3 make hit word
// 16t + m (bit b = window 64(16t+m)+b). For each hit the matched table slot
// goes to hit_slot[window]. The block's LDS holds only the first filter; the
// image goes straight to registers.
__global__ __launch_bounds__(kFragThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_frag_scan(
    const uint32_t* __restrict__ image, uint64_t n_windows, uint64_t n_dwords, IndexView ix,
    uint64_t* __restrict__ out, uint32_t* __restrict__ hit_slot) {
  __shared__ uint32_t lfilter[kLdsFilterMaxWords];
  const uint32_t lw = ix.lds_words;   // at most kLdsFilterMaxWords
  for (uint32_t i = threadIdx.x; i < lw; i += kFragThreads) lfilter[i] = ix.lds_filter[i];
  __syncthreads();   // before any wave of the block can leave
  const uint32_t wv = threadIdx.x / kWave;
  const uint32_t l = lane_id();
  const uint64_t n_tasks = (n_windows + kWaveWindows - 1) / kWaveWindows;
  const uint64_t n_words = (n_windows + kTileSectors - 1) / kTileSectors;
  const uint64_t n_waves = (uint64_t)gridDim.x * kFragWaves;
  for (uint64_t t = (uint64_t)blockIdx.x * kFragWaves + wv; t < n_tasks; t += n_waves) {
    // Lane l's windows read dwords [16l, 16l + 32) of the task (dword dw0 =
    // window 1024t): its own 16 and the next lane's. Lane 63's second 16 are
    // the next task's first words, which lanes 0-15 load. Only the words' D
    // values are kept. Inside the image these are 16-byte loads; the last
    // task clamps every dword to the image's last one (only windows past the
    // end read the repeated words).
    const uint64_t dw0 = t * kWaveWindows;
    // d[k] = D(dword 16l + k), dx = D of dword 1024 + (l % 16) of the task
    uint32_t d[kFragRowDw], dx;
    if (dw0 + kWaveWindows + kFragRowDw <= n_dwords) {
      const uint32_t* src = image + dw0 + (uint64_t)l * kFragRowDw;
#pragma unroll
      for (uint32_t q = 0; q < kFragRowDw / 4; ++q) {
        const u32x4 v = __builtin_nontemporal_load((const u32x4*)(src + 4 * q));
        d[4 * q] = word_djb2(v.x), d[4 * q + 1] = word_djb2(v.y);
        d[4 * q + 2] = word_djb2(v.z), d[4 * q + 3] = word_djb2(v.w);
      }
      dx = word_djb2(__builtin_nontemporal_load(image + dw0 + kWaveWindows + (l % kFragRowDw)));
    } else {
#pragma unroll
      for (uint32_t k = 0; k < kFragRowDw; ++k) {
        const uint64_t g = dw0 + (uint64_t)l * kFragRowDw + k;
        d[k] = word_djb2(image[g < n_dwords ? g : n_dwords - 1]);
      }
      const uint64_t g = dw0 + kWaveWindows + (l % kFragRowDw);
      dx = word_djb2(image[g < n_dwords ? g : n_dwords - 1]);
    }
    // D of word 16 + k of lane l's stream: the next lane's d[k]; for lane 63,
    // lane k's dx (the whole wave runs this code, so every source lane is active)
    auto d_second = [&](uint32_t k) {
      const uint32_t next_lane = (uint32_t)__shfl_down((int)d[k], 1, kWave);
      const uint32_t from_ext = (uint32_t)__builtin_amdgcn_readlane((int)dx, (int)k);
      return l == kWave - 1 ? from_ext : next_lane;
    };
    const uint64_t j0 = dw0 + (uint64_t)l * kLaneWindows;
    const uint32_t valid = j0 >= n_windows ? 0u : (n_windows - j0 >= kLaneWindows ? kLaneWindows
                                                                                   : (uint32_t)(n_windows - j0));
    uint64_t H = 0;
#pragma unroll
    for (uint32_t k = 0; k < kFragRowDw; ++k) H = H * kPow4 + d[k];
    uint64_t sig = kFragInit + H;   // window 16l of the task
    const uint32_t* bloom = (const uint32_t*)ix.bloom;   // fragment indexes: 32-bit words
    const uint32_t lwb = ix.log2_bloom_words + 1;
    uint32_t mask = 0;
    // batches of 8 windows: 8 signatures; the LDS filter; Bloom words only for
    // the windows that pass it, in flight together; then the (rare) windows
    // that pass both go through the table probe
#pragma unroll
    for (uint32_t b = 0; b < kLaneWindows; b += 8) {
      uint64_t h[8];
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t w = b + i;
        h[i] = sig;
        // roll to window w + 1 (after the last window the result is unused)
        sig = sig * kPow4 + (kRollAdd + kNegPow64 * d[w]) + d_second(w);
      }
      uint32_t pend = valid <= b ? 0u : (valid - b >= 8 ? 0xFFu : (1u << (valid - b)) - 1u);
#pragma unroll
      for (int i = 0; i < 8; ++i) {   // no branches: every window reads its LDS word
        uint32_t wi, bits;
        frag_lds_place(h[i], lw, &wi, &bits);
        const bool out = (lfilter[wi] & bits) != bits && h[i] != kEmptyKey;
        pend &= ~((uint32_t)out << i);
      }
      if (bloom) {
        uint32_t bits[8], fw[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          uint32_t wi;
          frag_bloom_place(h[i], lwb, &wi, &bits[i]);
          fw[i] = ((pend >> i) & 1u) ? bloom[wi] : ~0u;
        }
        uint32_t pass = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) pass |= (uint32_t)(h[i] == kEmptyKey || (fw[i] & bits[i]) == bits[i]) << i;
        pend &= pass;
      }
      while (pend) {
        const int i = __builtin_ctz(pend);
        pend &= pend - 1u;
        uint64_t hv = h[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) hv = i == k ? h[k] : hv;
        int64_t slot = -1;
        if (hv == kEmptyKey) {
          if (ix.zero_sig_mask) slot = ix.zero_slot;
        } else {
          slot = find_slot(ix, hv);   // any position: every occupied slot has masters
        }
        if (slot >= 0) {
          mask |= 1u << (b + i);
          hit_slot[j0 + b + i] = (uint32_t)slot;
        }
      }
    }
    // four lanes' 16-bit masks make one 64-bit hit word
    const uint32_t m1 = (uint32_t)__shfl_down((int)mask, 1, kWave);
    const uint32_t m2 = (uint32_t)__shfl_down((int)mask, 2, kWave);
    const uint32_t m3 = (uint32_t)__shfl_down((int)mask, 3, kWave);
    const uint64_t wi = t * (kWaveWindows / kTileSectors) + l / 4;
    if ((l & 3u) == 0 && wi < n_words)
      out[wi] = (uint64_t)(mask | (m1 << 16)) | ((uint64_t)(m2 | (m3 << 16)) << 32);
  }
}

}  // namespace carve
