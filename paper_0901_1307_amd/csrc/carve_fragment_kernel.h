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
constexpr uint32_t kLdsFilterMaxWords = 1u << 15;            // 128 KiB: the first filter, in LDS

// First-level filter: a bitmap of 32-bit words in LDS; a signature sets 2 bits
// of one word, placed by a multiplicative hash independent of the Bloom
// filter's. Only windows that pass it read the (L2-resident) Bloom filter.
constexpr uint64_t kLdsFilterMul = 0x9FB21C651E98DF25ull;
__device__ __forceinline__ void lds_filter_place(uint64_t h, uint32_t log2_words, uint32_t* word, uint32_t* bits) {
  const uint64_t p = h * kLdsFilterMul;
  *word = (uint32_t)(p >> (64 - log2_words));
  const uint32_t f = (uint32_t)(p >> (54 - log2_words));   // 10 bits below the word index
  *bits = (1u << (f & 31u)) | (1u << ((f >> 5) & 31u));
}

// Rolling Eq. (1) over a 64-byte window by 4 bytes. With the window's data
// part H(j) = sum_{i<64} s[4j+i] 33^(63-i) (its signature is 5381*33^64 + H)
// and D(w) = b0 33^3 + b1 33^2 + b2 33 + b3 for the bytes of word w in address
// order (D < 2^24):
//   H(j+1) = H(j) 33^4 - 33^64 D(j) + D(j+16)        (mod 2^64)
// and the first window is Horner over its 16 words: H = H 33^4 + D(k).
constexpr uint64_t kPow4 = pow33(4);
constexpr uint64_t kPow64 = pow33(kFragBytes);
constexpr uint64_t kFragInit = 5381ull * pow33(kFragBytes);

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
  const uint32_t lw = ix.log2_lds_words;
  for (uint32_t i = threadIdx.x; i < (1u << lw); i += kFragThreads) lfilter[i] = ix.lds_filter[i];
  __syncthreads();   // before any wave of the block can leave
  const uint32_t wv = threadIdx.x / kWave;
  const uint32_t l = lane_id();
  const uint64_t n_tasks = (n_windows + kWaveWindows - 1) / kWaveWindows;
  const uint64_t n_words = (n_windows + kTileSectors - 1) / kTileSectors;
  const uint64_t n_waves = (uint64_t)gridDim.x * kFragWaves;
  for (uint64_t t = (uint64_t)blockIdx.x * kFragWaves + wv; t < n_tasks; t += n_waves) {
    // Lane l's windows read dwords [16l, 16l + 32) of the task (dword dw0 =
    // window 1024t): its own 16 (own[k] = dword 16l + k) and the next lane's.
    // Lane 63's second 16 are the next task's first words, which lanes 0-15
    // load (ext). Inside the image these are 16-byte loads; the last task
    // clamps every dword to the image's last one (only windows past the end
    // read the repeated words).
    const uint64_t dw0 = t * kWaveWindows;
    uint32_t own[kFragRowDw], ext;
    if (dw0 + kWaveWindows + kFragRowDw <= n_dwords) {
      const uint32_t* src = image + dw0 + (uint64_t)l * kFragRowDw;
#pragma unroll
      for (uint32_t q = 0; q < kFragRowDw / 4; ++q) {
        const u32x4 v = __builtin_nontemporal_load((const u32x4*)(src + 4 * q));
        own[4 * q] = v.x, own[4 * q + 1] = v.y, own[4 * q + 2] = v.z, own[4 * q + 3] = v.w;
      }
      ext = __builtin_nontemporal_load(image + dw0 + kWaveWindows + (l % kFragRowDw));
    } else {
#pragma unroll
      for (uint32_t k = 0; k < kFragRowDw; ++k) {
        const uint64_t g = dw0 + (uint64_t)l * kFragRowDw + k;
        own[k] = image[g < n_dwords ? g : n_dwords - 1];
      }
      const uint64_t g = dw0 + kWaveWindows + (l % kFragRowDw);
      ext = image[g < n_dwords ? g : n_dwords - 1];
    }
    // word 16 + k of lane l's stream: the next lane's own[k]; for lane 63,
    // lane k's ext (the whole wave runs this code, so every source lane is active)
    auto second = [&](uint32_t k) {
      const uint32_t next_lane = (uint32_t)__shfl_down((int)own[k], 1, kWave);
      const uint32_t from_ext = (uint32_t)__builtin_amdgcn_readlane((int)ext, (int)k);
      return l == kWave - 1 ? from_ext : next_lane;
    };
    const uint64_t j0 = dw0 + (uint64_t)l * kLaneWindows;
    const uint32_t valid = j0 >= n_windows ? 0u : (n_windows - j0 >= kLaneWindows ? kLaneWindows
                                                                                   : (uint32_t)(n_windows - j0));
    uint64_t H = 0;
#pragma unroll
    for (uint32_t k = 0; k < kFragRowDw; ++k) H = H * kPow4 + word_djb2(own[k]);
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
        h[i] = kFragInit + H;
        // roll to window w + 1 (after the last window the result is unused)
        H = H * kPow4 - kPow64 * word_djb2(own[w]) + word_djb2(second(w));
      }
      uint32_t pend = valid <= b ? 0u : (valid - b >= 8 ? 0xFFu : (1u << (valid - b)) - 1u);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        uint32_t wi, bits;
        lds_filter_place(h[i], lw, &wi, &bits);
        if (h[i] != kEmptyKey && (lfilter[wi] & bits) != bits) pend &= ~(1u << i);
      }
      if (ix.bloom) {
        uint64_t bits[8], fw[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          uint32_t wi;
          bloom_place(h[i], ix.log2_bloom_words, &wi, &bits[i]);
          fw[i] = ((pend >> i) & 1u) ? ix.bloom[wi] : ~0ull;
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
          slot = find_slot(ix, hv);
          if (slot >= 0 && ix.tau_mask[slot] == 0) slot = -1;
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
