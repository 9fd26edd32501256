// Device-side building blocks of the carving scan for gfx950 (wave64).
//
// Signature: djb2 with a 64-bit accumulator (Eq. (1), Section 2.2; 64-bit
// accumulator, Section 4). The recurrence is linear modulo 2^64, so for a
// 512-byte sector s_0..s_511 it unrolls to
//     h = 5381*33^512 + sum_b s_b * 33^(511-b)            (mod 2^64).
// Each weight 33^(511-b) mod 2^64 is split into 8 base-256 digits; with the
// sector bytes also 8-bit, each digit plane q accumulates
//     acc_q = sum_b s_b * digit_q(33^(511-b))
// with v_dot4_u32_u8 (four byte products per instruction, no carry chain:
// acc_q <= 512*255*255 < 2^25), and h = 5381*33^512 + sum_q acc_q << 8q.
// The digits are compile-time constants (they become SGPR literals).
//
// Lane mapping: a wave hashes a tile of 64 sectors, one sector per lane, like
// the paper's cohorts (Section 3.2) but 64 wide. Global loads are coalesced:
// 8 lanes read 128 contiguous bytes of one sector (16 B each), so one load
// instruction covers 8 full 128-byte lines. The bytes go through a per-wave
// LDS staging area with a padded row pitch (the job Fig. 9's skewed tile did
// for a 16-bank shared memory) and each lane reads back its own sector.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace carve {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t kSectorBytes = 512;
constexpr uint32_t kClusterSectors = 8;
constexpr uint32_t kWave = 64;
constexpr uint32_t kTileSectors = 64;                       // one sector per lane
constexpr uint32_t kPhaseBytes = 128;                       // bytes per sector staged at once
constexpr uint32_t kPhases = kSectorBytes / kPhaseBytes;    // 4
constexpr uint32_t kRowPitch = kPhaseBytes + 16;            // padding spreads rows over banks
constexpr uint32_t kTileLds = kTileSectors * kRowPitch;     // 9216 B per wave
constexpr uint32_t kBucketSlots = 16;                       // 16 x 8 B keys = one 128-B line
constexpr uint64_t kEmptyKey = 0;                           // a real signature 0 lives in a side slot
constexpr uint64_t kBucketMul = 0x9E3779B97F4A7C15ull;      // Fibonacci hashing of the signature

// ---------------------------------------------------------------- weights
constexpr uint64_t pow33(uint32_t e) {
  uint64_t r = 1, b = 33;
  while (e) {
    if (e & 1u) r *= b;
    b *= b;
    e >>= 1;
  }
  return r;
}

constexpr uint64_t kInitTerm = 5381ull * pow33(kSectorBytes);   // wraps modulo 2^64

// Digit plane q of the weights of bytes 4d..4d+3, packed little-endian like
// the data dword (byte 4d is the dword's low byte).
constexpr uint32_t weight_dword(uint32_t d, uint32_t q) {
  uint32_t w = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    uint64_t wb = pow33(kSectorBytes - 1 - (4 * d + k));
    w |= (uint32_t)((wb >> (8 * q)) & 0xFFu) << (8 * k);
  }
  return w;
}

// ------------------------------------------------------------ static for
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, uint32_t src) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl((int)lo, (int)src, kWave);
  hi = (uint32_t)__shfl((int)hi, (int)src, kWave);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Byte g of x non-zero -> bit g of the result (x is wave-uniform).
__device__ __forceinline__ uint32_t bytes_nonzero(uint64_t x) {
  uint32_t r = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g) r |= ((x >> (8 * g)) & 0xFFu) ? (1u << g) : 0u;
  return r;
}

// ------------------------------------------------------------ tile hash
// Sector addresses of a tile. Contiguous: sector s is base + s*512 and is
// valid for s < n_valid. Gathered: each lane holds its own sector pointer
// (null = invalid) and the others read it with a cross-lane shuffle.
struct ContiguousRows {
  const uint8_t* base;
  uint32_t n_valid;
  __device__ __forceinline__ const uint8_t* row(uint32_t s) const { return base + (uint64_t)s * kSectorBytes; }
  __device__ __forceinline__ bool valid(uint32_t s) const { return s < n_valid; }
};

struct GatheredRows {
  uint64_t mine;   // this lane's sector address, 0 if none
  __device__ __forceinline__ const uint8_t* row(uint32_t s) const {
    return (const uint8_t*)shfl_u64(mine, s);
  }
  __device__ __forceinline__ bool valid(uint32_t s) const { return row(s) != nullptr; }
};

template <bool kNonTemporal>
__device__ __forceinline__ u32x4 load16(const uint8_t* p) {
  if constexpr (kNonTemporal) return __builtin_nontemporal_load((const u32x4*)p);
  else return *(const u32x4*)p;
}

// Returns, in lane l, the djb2-64 signature of sector l of the tile.
// lds: this wave's kTileLds-byte staging area.
template <bool kNonTemporal, class Rows>
__device__ __forceinline__ uint64_t tile_signature(const Rows& rows, uint8_t* lds) {
  const uint32_t l = lane_id();
  const uint32_t col = (l & 7u) * 16u;
  uint32_t acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0;

  // instruction i of a phase: lane l loads 16 B of sector 8i + l/8
  const uint8_t* src[8];
  bool ok[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t s = 8u * i + (l >> 3);
    ok[i] = rows.valid(s);
    src[i] = rows.row(s) + col;
  }

  u32x4 cur[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) cur[i] = ok[i] ? load16<kNonTemporal>(src[i]) : u32x4{0, 0, 0, 0};

  static_for<kPhases>([&](auto P) {
    constexpr int p = decltype(P)::value;
    // stage: row s = 8i + l/8, column l%8
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *(u32x4*)(lds + (8u * i + (l >> 3)) * kRowPitch + col) = cur[i];
    wave_sync_lds();
    // next phase's loads are in flight while this phase is hashed
    if constexpr (p + 1 < (int)kPhases) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        cur[i] = ok[i] ? load16<kNonTemporal>(src[i] + (p + 1) * kPhaseBytes) : u32x4{0, 0, 0, 0};
    }
    static_for<8>([&](auto C) {
      constexpr int c = decltype(C)::value;
      const u32x4 r = *(const u32x4*)(lds + l * kRowPitch + c * 16);
      static_for<4>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr uint32_t d = p * (kPhaseBytes / 4) + c * 4 + k;
        const uint32_t x = r[k];
        static_for<8>([&](auto Q) {
          constexpr int q = decltype(Q)::value;
          constexpr uint32_t w = weight_dword(d, q);
          acc[q] = __builtin_amdgcn_udot4(x, w, acc[q], false);
        });
      });
    });
    wave_sync_lds();
  });

  uint64_t h = kInitTerm;
#pragma unroll
  for (int q = 0; q < 8; ++q) h += (uint64_t)acc[q] << (8 * q);
  return h;
}

// ---------------------------------------------------------------- index
struct IndexView {
  const uint64_t* keys;       // n_buckets * 16 slots, kEmptyKey = free
  const uint32_t* tau_mask;   // per slot (+1: the side slot of signature 0), bit t = present at position t
  uint32_t log2_buckets;
  uint32_t zero_sig_mask;     // tau mask of signature 0 (the side slot)
};

__device__ __forceinline__ uint32_t bucket_of(uint64_t h, uint32_t log2_buckets) {
  return (uint32_t)((h * kBucketMul) >> (64 - log2_buckets));
}

// Slot of key h (h != kEmptyKey) or -1. Linear probing over buckets: a key
// lives in its home bucket or, if that bucket filled up first, a later one
// (Eq. (3) at bucket granularity); a bucket with a free slot ends the search.
__device__ __forceinline__ int64_t find_slot(const IndexView& ix, uint64_t h) {
  const uint32_t nb_mask = (1u << ix.log2_buckets) - 1u;
  uint32_t b = bucket_of(h, ix.log2_buckets);
  for (uint32_t it = 0; it <= nb_mask; ++it) {
    const u64x2* p = (const u64x2*)(ix.keys + (uint64_t)b * kBucketSlots);
    bool any_empty = false;
#pragma unroll
    for (int c = 0; c < (int)(kBucketSlots / 2); ++c) {
      const u64x2 kv = p[c];
      if (kv.x == h) return (int64_t)b * kBucketSlots + 2 * c;
      if (kv.y == h) return (int64_t)b * kBucketSlots + 2 * c + 1;
      any_empty |= (kv.x == kEmptyKey) | (kv.y == kEmptyKey);
    }
    if (any_empty) return -1;
    b = (b + 1) & nb_mask;
  }
  return -1;
}

__device__ __forceinline__ bool tau_ok(uint32_t mask, uint32_t tau, bool any_tau) {
  return any_tau ? (mask != 0) : (((mask >> tau) & 1u) != 0);
}

// Membership of the 64 lane signatures, cooperatively: in round r, the 8 lanes
// of group g read the 128-byte home bucket of sector 8r+g (16 B each), so a
// round is one load instruction over 8 whole lines. Returns the 64-bit hit
// mask of the tile (bit l = sector l). tau: this lane's cluster position.
__device__ __forceinline__ uint64_t tile_probe(const IndexView& ix, uint64_t h, uint32_t tau, bool any_tau) {
  const uint32_t l = lane_id();
  const uint32_t bkt = bucket_of(h, ix.log2_buckets);
  uint64_t hits = 0, unresolved = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t s = 8u * r + (l >> 3);
    const uint64_t hs = shfl_u64(h, s);
    const uint32_t bs = (uint32_t)__shfl((int)bkt, (int)s, kWave);
    const uint32_t ts = (uint32_t)__shfl((int)tau, (int)s, kWave);
    const uint64_t slot0 = (uint64_t)bs * kBucketSlots + 2u * (l & 7u);
    const u64x2 kv = *(const u64x2*)(ix.keys + slot0);
    const bool live = hs != kEmptyKey;
    const bool m0 = live && kv.x == hs;
    const bool m1 = live && kv.y == hs;
    const bool empty = !live || kv.x == kEmptyKey || kv.y == kEmptyKey;
    bool ok = false;
    if (m0 | m1) ok = tau_ok(ix.tau_mask[slot0 + (m1 ? 1 : 0)], ts, any_tau);
    const uint64_t b_ok = ballot(ok);
    const uint64_t b_done = ballot(m0 | m1 | empty);
    hits |= (uint64_t)bytes_nonzero(b_ok) << (8 * r);
    unresolved |= (uint64_t)(~bytes_nonzero(b_done) & 0xFFu) << (8 * r);
  }
  // rare: the home bucket was full and did not hold the key
  bool ok_more = false;
  if ((unresolved >> l) & 1u) {
    const int64_t slot = find_slot(ix, h);
    ok_more = slot >= 0 && tau_ok(ix.tau_mask[slot], tau, any_tau);
  }
  // signature 0 cannot be stored in the table (it marks free slots)
  const bool ok_zero = (h == kEmptyKey) && tau_ok(ix.zero_sig_mask, tau, any_tau);
  return hits | ballot(ok_more) | ballot(ok_zero);
}

// -------------------------------------------------------- block scans
// Exclusive prefix sum over a 256-thread block; returns this thread's prefix
// and writes the block total to *total (all threads).
template <int kThreads>
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* lds_w, uint64_t* total) {
  const uint32_t l = lane_id();
  const uint32_t w = threadIdx.x / kWave;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < (int)kWave; o <<= 1) {
    const uint64_t y = shfl_u64(x, l >= (uint32_t)o ? l - o : l);
    if (l >= (uint32_t)o) x += y;
  }
  if (l == kWave - 1) lds_w[w] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kThreads / (int)kWave; ++i) {
    const uint64_t t = lds_w[i];
    before += (i < (int)w) ? t : 0;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

}  // namespace carve
