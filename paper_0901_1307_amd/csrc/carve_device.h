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

// All 128 x 8 weight words. They are read from device memory with uniform
// addresses, i.e. by scalar loads of 16 words at a time; as literals they would
// cost one scalar move per dot product, as many scalar instructions as vector ones.
struct WeightTable {
  uint32_t w[kSectorBytes / 4][8];
};
constexpr WeightTable make_weight_table() {
  WeightTable t{};
  for (uint32_t d = 0; d < kSectorBytes / 4; ++d)
    for (uint32_t q = 0; q < 8; ++q) t.w[d][q] = weight_dword(d, q);
  return t;
}
__device__ WeightTable g_weights = make_weight_table();

// Kernels take the table's address as an integer and read it through a
// constant-address-space pointer: uniform loads from that space are scalar loads.
typedef const __attribute__((address_space(4))) WeightTable* WeightPtr;

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

// Byte g of x non-zero -> bit g of the result (x is wave-uniform): fold each
// byte onto its low bit, then gather bits 0, 8, ..., 56 with one multiply
// (the partial products land on distinct bits, so nothing carries).
__device__ __forceinline__ uint32_t bytes_nonzero(uint64_t x) {
  x |= x >> 4;
  x |= x >> 2;
  x |= x >> 1;
  x &= 0x0101010101010101ull;
  return (uint32_t)((x * 0x0102040810204080ull) >> 56);
}

// ------------------------------------------------------------ tile hash
// Sector addresses of a tile: sector s is base + s*512; sectors past n_valid
// are replaced by the last valid one (their hash is discarded), so every load
// stays inside the image without a branch.
struct ContiguousRows {
  const uint8_t* base;
  uint32_t n_valid;   // 1..64
  __device__ __forceinline__ const uint8_t* row(uint32_t s) const {
    return base + (uint64_t)(s < n_valid ? s : n_valid - 1) * kSectorBytes;
  }
};
// A tile of one cluster position: sector s is base + s*4096 (the same
// position in 64 consecutive clusters); past n_valid, the last valid one.
struct ClusterStrideRows {
  const uint8_t* base;
  uint32_t n_valid;   // 1..64
  __device__ __forceinline__ const uint8_t* row(uint32_t s) const {
    return base + (uint64_t)(s < n_valid ? s : n_valid - 1) * (kClusterSectors * kSectorBytes);
  }
};

template <bool kNonTemporal>
__device__ __forceinline__ u32x4 load16(const uint8_t* p) {
  if constexpr (kNonTemporal) return __builtin_nontemporal_load((const u32x4*)p);
  else return *(const u32x4*)p;
}

// Phase p of a tile: instruction i, lane l loads 16 B of sector 8i + l/8 at
// byte 128p + 16(l%8); one instruction covers 8 whole 128-byte lines.
struct PhaseRegs {
  u32x4 v[8];
};

template <bool kNonTemporal, class Rows>
__device__ __forceinline__ void load_phase(const Rows& rows, uint32_t p, PhaseRegs& r) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int i = 0; i < 8; ++i) r.v[i] = load16<kNonTemporal>(rows.row(8u * i + (l >> 3)) + p * kPhaseBytes + (l & 7u) * 16u);
}

// Stage phase P through this wave's LDS area and fold its 128 bytes per
// sector into the 8 digit-plane accumulators of lane l's sector.
template <int P>
__device__ __forceinline__ void hash_phase(const PhaseRegs& r, uint8_t* lds, uint64_t wt, uint32_t (&acc)[8]) {
  // the loads issued before this call stay above it
  __builtin_amdgcn_sched_barrier(0);
  // The weights are loop-invariant; hiding the pointer's identity per phase
  // keeps the compiler from hoisting all 1024 of them into scalar registers.
  WeightPtr w = (WeightPtr)wt;
  asm volatile("" : "+s"(w));
  const uint32_t l = lane_id();
  const uint32_t col = (l & 7u) * 16u;
#pragma unroll
  for (int i = 0; i < 8; ++i) *(u32x4*)(lds + (8u * i + (l >> 3)) * kRowPitch + col) = r.v[i];
  wave_sync_lds();
  static_for<8>([&](auto C) {
    constexpr int c = decltype(C)::value;
    // one 16-byte column (32 weights) at a time, or the weight loads of the
    // whole phase get hoisted and overflow the scalar registers
    __builtin_amdgcn_sched_barrier(0);
    const u32x4 x4 = *(const u32x4*)(lds + l * kRowPitch + c * 16);
    static_for<4>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr uint32_t d = P * (kPhaseBytes / 4) + c * 4 + k;
      const uint32_t x = x4[k];
      static_for<8>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        acc[q] = __builtin_amdgcn_udot4(x, w->w[d][q], acc[q], false);
      });
    });
  });
  // The accumulators must be final here: an empty asm that "modifies" them
  // is a side effect, so neither this phase's math can sink below the next
  // phase's LDS stores nor can those stores rise above it.
  asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
               "+v"(acc[6]), "+v"(acc[7]));
  wave_sync_lds();
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ uint64_t finish_signature(const uint32_t (&acc)[8]) {
  uint64_t h = kInitTerm;
#pragma unroll
  for (int q = 0; q < 8; ++q) h += (uint64_t)acc[q] << (8 * q);
  return h;
}

// Signature of every sector of a tile (lane l = sector l). A and B are the
// two register buffers of the load pipeline: on entry A holds (or is
// receiving) phase 0; phase p+1 loads are issued before phase p is hashed,
// and `prefetch` (called before the last phase is hashed) may start the next
// tile's phase 0 into A.
template <bool kNonTemporal, class Rows, class Prefetch>
__device__ __forceinline__ uint64_t tile_signature_pipelined(const Rows& rows, uint8_t* lds, uint64_t wt,
                                                             PhaseRegs& A, PhaseRegs& B, Prefetch&& prefetch) {
  uint32_t acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0;
  load_phase<kNonTemporal>(rows, 1, B);
  hash_phase<0>(A, lds, wt, acc);
  load_phase<kNonTemporal>(rows, 2, A);
  hash_phase<1>(B, lds, wt, acc);
  load_phase<kNonTemporal>(rows, 3, B);
  hash_phase<2>(A, lds, wt, acc);
  prefetch(A);
  hash_phase<3>(B, lds, wt, acc);
  return finish_signature(acc);
}

// ---------------------------------------------------------------- CRC-64
// The other signature of Section 2.1: a 64-bit CRC, read as CRC-64/GO-ISO
// (generator x^64 + x^4 + x^3 + x + 1, bytes entering least significant bit
// first, register preset to all ones, result complemented).
//
// No table: this generator lets the register absorb a 32-bit word with shifts
// and xors. In the right-shifting (reflected) register a feedback term enters
// at bit 59 or above, so within any 32 steps the bits tested are exactly the
// input bits. Absorbing the little-endian word d (bytes in address order) is
// then, with x = crc ^ d and u = x mod 2^32,
//   crc' = (x >> 32) ^ (u << 28) ^ (u << 29) ^ (u << 31) ^ (u << 32),
// x >> 32 xor the carry-less product of u with the generator's terms below x^64
// (0x1B: bits 0, 1, 3, 4), placed 28 bits up. About 11 VALU operations per word.
enum : int { kSigDjb2 = 0, kSigCrc64 = 1 };   // the values of carve_sig_kind

// The same, on the register's 32-bit halves (full-rate 32-bit shifts):
// the low half becomes hi ^ u<<28 ^ u<<29 ^ u<<31, the high half
// u ^ u>>1 ^ u>>3 ^ u>>4 (the bits the 64-bit shifts carry across).
// a ^ b ^ c in one instruction: gfx950's three-input bit operation with the
// truth table of xor3 (0x96: set where an odd number of inputs is set).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void crc_word(uint32_t& lo, uint32_t& hi, uint32_t d) {
  const uint32_t u = lo ^ d;
  lo = xor3(hi, u << 28, u << 29) ^ (u << 31);
  hi = xor3(u, u >> 1, u >> 3) ^ (u >> 4);
}

// Stage a phase through this wave's LDS area, then run lane l's register over
// the 128 bytes of its sector, in address order.
__device__ __forceinline__ void crc_phase(const PhaseRegs& r, uint8_t* lds, uint32_t& lo, uint32_t& hi) {
  __builtin_amdgcn_sched_barrier(0);
  const uint32_t l = lane_id();
  const uint32_t col = (l & 7u) * 16u;
#pragma unroll
  for (int i = 0; i < 8; ++i) *(u32x4*)(lds + (8u * i + (l >> 3)) * kRowPitch + col) = r.v[i];
  wave_sync_lds();
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const u32x4 x4 = *(const u32x4*)(lds + l * kRowPitch + c * 16);
#pragma unroll
    for (int k = 0; k < 4; ++k) crc_word(lo, hi, x4[k]);
  }
  asm volatile("" : "+v"(lo), "+v"(hi));
  wave_sync_lds();
  __builtin_amdgcn_sched_barrier(0);
}

// CRC-64 of every sector of a tile, with the same load pipeline as the djb2 path.
template <bool kNonTemporal, class Rows, class Prefetch>
__device__ __forceinline__ uint64_t tile_crc_pipelined(const Rows& rows, uint8_t* lds, PhaseRegs& A, PhaseRegs& B,
                                                       Prefetch&& prefetch) {
  uint32_t lo = ~0u, hi = ~0u;   // preset: all ones
  load_phase<kNonTemporal>(rows, 1, B);
  crc_phase(A, lds, lo, hi);
  load_phase<kNonTemporal>(rows, 2, A);
  crc_phase(B, lds, lo, hi);
  load_phase<kNonTemporal>(rows, 3, B);
  crc_phase(A, lds, lo, hi);
  prefetch(A);
  crc_phase(B, lds, lo, hi);
  return ~(((uint64_t)hi << 32) | lo);   // complemented
}

// ---------------------------------------------------------------- index
struct IndexView {
  const uint64_t* keys;      // n_buckets * 16 slots, kEmptyKey = free
  const uint8_t* tau_mask;   // per slot, bit t = a master with this signature sits at position t
  const uint64_t* bloom;     // blocked Bloom filter of the table's keys, or null
  uint32_t log2_buckets;
  uint32_t log2_bloom_words;
  uint32_t zero_sig_mask;    // positions of signature 0, which has no slot in the table
  uint32_t zero_slot;        // candidate-list id of signature 0 (= number of table slots)
  // other probe layouts, mapping a signature to its slot of the table above
  const uint64_t* lin_keys;  // linear probing per slot from the signature's low bits: 2^log2_lin keys
  const uint32_t* lin_slot;  //   and the table slot of each
  uint32_t log2_lin;
  uint32_t n_sorted;         // sorted distinct signatures (binary search)
  const uint64_t* sorted_keys;
  const uint32_t* sorted_slot;
  const uint32_t* lds_filter;  // fragment indexes: the first-level filter copied into LDS (lds_words words)
  uint32_t lds_words;
  // sector indexes: the Bloom filter split by cluster position, slice t (2^log2_bloom_tau
  // words at bloom_tau + t 2^log2_bloom_tau) holding the keys present at position t; or null
  const uint64_t* bloom_tau;
  uint32_t log2_bloom_tau;
};

// Probe layouts (the values of carve_index_layout).
enum : int { kLayoutBucketed = 0, kLayoutLinear = 1, kLayoutSorted = 2 };

// Register-blocked Bloom filter: a key owns one 64-bit word and sets 4 of
// its bits. Word and bit positions come from the high half of a second
// multiplicative hash (djb2's low bits are weak: 33 = 1 mod 32).
// log2_words must be in 1..40: the word index is a shift by 64 - log2_words,
// and a shift by 64 is not a shift by 64 on this chip (its amount is taken
// mod 64), so a one-word filter would index far past its end.
constexpr uint64_t kBloomMul = 0xD6E8FEB86659FD93ull;
__device__ __forceinline__ void bloom_place(uint64_t h, uint32_t log2_words, uint32_t* word, uint64_t* bits) {
  const uint64_t p = h * kBloomMul;
  *word = (uint32_t)(p >> (64 - log2_words));
  const uint32_t f = (uint32_t)(p >> (40 - log2_words));   // 24 bits below the word index
  *bits = (1ull << (f & 63)) | (1ull << ((f >> 6) & 63)) | (1ull << ((f >> 12) & 63)) | (1ull << ((f >> 18) & 63));
}

__device__ __forceinline__ uint32_t bucket_of(uint64_t h, uint32_t log2_buckets) {
  return (uint32_t)((h * kBucketMul) >> (64 - log2_buckets));
}

// Slot of key h (h != kEmptyKey) or -1. Linear probing over buckets: a key
// lives in its home bucket or, if that bucket filled up first, a later one
// (Eq. (3) at bucket granularity); a bucket with a free slot ends the search.
// The whole 128-byte bucket is loaded before any key is compared: one memory
// round trip per bucket (keys are distinct, so at most one slot matches).
__device__ __forceinline__ int64_t find_slot(const IndexView& ix, uint64_t h) {
  const uint32_t nb_mask = (1u << ix.log2_buckets) - 1u;
  uint32_t b = bucket_of(h, ix.log2_buckets);
  for (uint32_t it = 0; it <= nb_mask; ++it) {
    const u64x2* p = (const u64x2*)(ix.keys + (uint64_t)b * kBucketSlots);
    u64x2 kv[kBucketSlots / 2];
#pragma unroll
    for (int c = 0; c < (int)(kBucketSlots / 2); ++c) kv[c] = p[c];
    int64_t found = -1;
    bool any_empty = false;
#pragma unroll
    for (int c = 0; c < (int)(kBucketSlots / 2); ++c) {
      if (kv[c].x == h) found = (int64_t)b * kBucketSlots + 2 * c;
      if (kv[c].y == h) found = (int64_t)b * kBucketSlots + 2 * c + 1;
      any_empty |= (kv[c].x == kEmptyKey) | (kv[c].y == kEmptyKey);
    }
    if (found >= 0) return found;
    if (any_empty) return -1;
    b = (b + 1) & nb_mask;
  }
  return -1;
}

// The paper's layout (Eq. (3)): home slot = the w low bits of the signature,
// then the next slots in turn until the key or a free slot. Returns the
// table slot or -1.
__device__ __forceinline__ int64_t find_slot_linear(const IndexView& ix, uint64_t h) {
  const uint64_t mask = (1ull << ix.log2_lin) - 1ull;
  uint64_t s = h & mask;
  for (uint64_t it = 0; it <= mask; ++it) {
    const uint64_t k = ix.lin_keys[s];
    if (k == h) return (int64_t)ix.lin_slot[s];
    if (k == kEmptyKey) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

// Sorted distinct signatures: lower bound by halving with no data-dependent
// branch (every lane takes the same ceil(log2 n) steps). Returns the table
// slot or -1.
__device__ __forceinline__ int64_t find_slot_sorted(const IndexView& ix, uint64_t h) {
  uint64_t base = 0, n = ix.n_sorted;
  if (n == 0) return -1;
  while (n > 1) {
    const uint64_t half = n >> 1;
    base = ix.sorted_keys[base + half] <= h ? base + half : base;
    n -= half;
  }
  return ix.sorted_keys[base] == h ? (int64_t)ix.sorted_slot[base] : -1;
}

template <int kLayout>
__device__ __forceinline__ int64_t find_slot_in(const IndexView& ix, uint64_t h) {
  if constexpr (kLayout == kLayoutLinear) return find_slot_linear(ix, h);
  else if constexpr (kLayout == kLayoutSorted) return find_slot_sorted(ix, h);
  else return find_slot(ix, h);
}

__device__ __forceinline__ bool tau_ok(uint32_t mask, uint32_t tau, bool any_tau) {
  return any_tau ? (mask != 0) : (((mask >> tau) & 1u) != 0);
}

// Membership of the 64 lane signatures. With a Bloom filter (kept small
// enough to stay in L2): one 8-byte filter word per sector, and only the
// sectors that pass probe the table, each lane its own. Without one: a
// cooperative probe in which, in round r, the 8 lanes of group g read the
// 128-byte home bucket of sector 8r+g (16 B each) and its 16 position masks
// (2 B each); all 16 loads are issued before any is used, so the tile pays
// one memory latency. Returns the tile's hit mask (bit l = sector l); tau is
// this lane's cluster position. For each hit, the slot that matched is
// stored in slot_out[sector * kSlotStride] (the candidate list that
// confirmation walks; the stride is 8 for a tile of one cluster position).
// The linear and sorted layouts probe lane by lane, after the filter if there
// is one.
// bloom / log2_bloom: the filter to consult (the index's, or one position's
// slice of it), or null. kSlots = false records no slots (slot_out unused),
// for scans whose flags are not confirmed afterwards.
template <int kLayout = kLayoutBucketed, uint32_t kSlotStride = 1, bool kSlots = true>
__device__ __forceinline__ uint64_t tile_probe(const IndexView& ix, uint64_t h, uint32_t tau, bool any_tau,
                                               uint32_t* __restrict__ slot_out, const uint64_t* bloom,
                                               uint32_t log2_bloom) {
  const uint32_t l = lane_id();
  // signature 0 cannot be stored in the table (it marks free slots)
  const bool ok_zero = (h == kEmptyKey) && tau_ok(ix.zero_sig_mask, tau, any_tau);
  if (kSlots && ok_zero) slot_out[l * kSlotStride] = ix.zero_slot;
  if (kLayout != kLayoutBucketed || bloom) {
    bool maybe = h != kEmptyKey;
    if (bloom) {
      uint32_t w;
      uint64_t bits;
      bloom_place(h, log2_bloom, &w, &bits);
      maybe = maybe && (bloom[w] & bits) == bits;
    }
    bool ok = false;
    if (maybe) {
      const int64_t slot = find_slot_in<kLayout>(ix, h);
      ok = slot >= 0 && tau_ok(ix.tau_mask[slot], tau, any_tau);
      if (kSlots && ok) slot_out[l * kSlotStride] = (uint32_t)slot;
    }
    return ballot(ok) | ballot(ok_zero);
  }
  const uint32_t bkt = bucket_of(h, ix.log2_buckets);
  // per round: the bucket's slots 2(l%8), 2(l%8)+1 and their masks
  u64x2 kv[8];
  uint32_t mk[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t s = 8u * r + (l >> 3);
    const uint32_t slot0 = (uint32_t)__shfl((int)bkt, (int)s, kWave) * kBucketSlots + 2u * (l & 7u);
    kv[r] = *(const u64x2*)(ix.keys + slot0);
    mk[r] = *(const uint16_t*)(ix.tau_mask + slot0);
  }
  uint64_t hits = 0, unresolved = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    // the round's sector, fetched again rather than kept live across the loads
    const uint32_t s = 8u * r + (l >> 3);
    const uint64_t hs = shfl_u64(h, s);
    const uint32_t ts = (uint32_t)__shfl((int)tau, (int)s, kWave);
    const bool live = hs != kEmptyKey;
    const bool m0 = live && kv[r].x == hs;
    const bool m1 = live && kv[r].y == hs;
    const bool empty = !live || kv[r].x == kEmptyKey || kv[r].y == kEmptyKey;
    const uint32_t mask = m0 ? (mk[r] & 0xFFu) : (mk[r] >> 8);
    const bool ok = (m0 | m1) && tau_ok(mask, ts, any_tau);
    // cross-lane reads only with every lane active: lane s may be idle inside `if (ok)`
    const uint32_t slot0 = (uint32_t)__shfl((int)bkt, (int)s, kWave) * kBucketSlots + 2u * (l & 7u);
    if (kSlots && ok) slot_out[s * kSlotStride] = slot0 + (m1 ? 1u : 0u);
    hits |= (uint64_t)bytes_nonzero(ballot(ok)) << (8 * r);
    unresolved |= (uint64_t)(~bytes_nonzero(ballot(m0 | m1 | empty)) & 0xFFu) << (8 * r);
  }
  // rare: the home bucket was full and did not hold the key
  bool ok_more = false;
  if ((unresolved >> l) & 1u) {
    const int64_t slot = find_slot(ix, h);
    ok_more = slot >= 0 && tau_ok(ix.tau_mask[slot], tau, any_tau);
    if (kSlots && ok_more) slot_out[l * kSlotStride] = (uint32_t)slot;
  }
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
