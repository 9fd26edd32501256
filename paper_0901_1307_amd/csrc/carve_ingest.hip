// Host ingest (Section 3.1, Fig. 7): scanning an image that lives in host
// memory, by chunks through a pair of device buffers {g0, g1}. While one chunk
// crosses PCIe into g_b on the copy stream, the compute stream scans (and
// confirms) the chunk in the other buffer; a chunk's results are collected two
// chunks later, just before its buffer is refilled. A pageable image is first
// copied by CPU threads into a pair of pinned staging buffers {h0, h1} (the
// paper's host double buffers); a pinned one is transferred directly.
// Host code only, over the public scan API.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "../../include/carve.h"
#include "carve_internal.h"

namespace {
constexpr uint64_t kSector = 512;
constexpr uint64_t kCluster = 4096;
constexpr uint64_t kDefaultChunk = 256ull << 20;

bool is_pinned(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // plain pageable memory: clear the sticky error
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

void parallel_copy(void* dst, const void* src, uint64_t n, uint32_t threads) {
  if (threads <= 1 || n < (8ull << 20)) {
    memcpy(dst, src, n);
    return;
  }
  std::vector<std::thread> pool;
  const uint64_t part = (n / threads + 4095) / 4096 * 4096;
  for (uint32_t t = 0; t < threads; ++t) {
    const uint64_t lo = std::min<uint64_t>(n, t * part), hi = std::min<uint64_t>(n, lo + part);
    if (lo >= hi) break;
    pool.emplace_back([=] { memcpy((char*)dst + lo, (const char*)src + lo, hi - lo); });
  }
  for (auto& th : pool) th.join();
}
}  // namespace

struct carve_ingest {
  const carve_index* idx = nullptr;
  carve_ingest_params p{};
  void* g[2] = {nullptr, nullptr};      // device chunk buffers
  void* h[2] = {nullptr, nullptr};      // pinned staging for pageable images
  hipStream_t copy = nullptr, comp = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr};
  carve_scan* scan[2] = {nullptr, nullptr};
  bool busy[2] = {false, false};
  uint64_t first_sector[2] = {0, 0};    // of the chunk in each buffer
  std::vector<uint64_t> ids;
  std::vector<carve_match> matches;
  std::vector<uint64_t> tmp_ids;
  std::vector<carve_match> tmp_matches;
  carve_ingest_stats st{};
};

namespace {
// Results of the chunk in buffer b (waits for its scan), ids made image-relative.
int collect(carve_ingest* in, int b) {
  if (!in->busy[b]) return CARVE_OK;
  in->busy[b] = false;
  if (hipEventSynchronize(in->done[b]) != hipSuccess) return carve_fail_msg(CARVE_EDEVICE, "ingest: sync failed");
  uint64_t n = 0;
  int rc = flagged_sectors(in->scan[b], nullptr, 0, &n);
  if (rc != CARVE_OK && rc != CARVE_ETRUNC) return rc;
  in->tmp_ids.resize(n);
  if (n && (rc = flagged_sectors(in->scan[b], in->tmp_ids.data(), n, &n)) != CARVE_OK) return rc;
  const uint64_t base = in->first_sector[b];
  for (uint64_t v : in->tmp_ids) in->ids.push_back(v + base);
  if (in->p.confirm && n) {
    uint64_t m = 0;
    in->tmp_matches.resize(n + n / 8 + 64);
    rc = confirm_matches(in->idx, in->scan[b], in->tmp_matches.data(), in->tmp_matches.size(), &m);
    if (rc == CARVE_ETRUNC) {
      in->tmp_matches.resize(m);
      rc = confirm_matches(in->idx, in->scan[b], in->tmp_matches.data(), m, &m);
    }
    if (rc != CARVE_OK) return rc;
    for (uint64_t i = 0; i < m; ++i) {
      carve_match r = in->tmp_matches[i];
      r.disk_sector += base;
      in->matches.push_back(r);
    }
  }
  return CARVE_OK;
}
}  // namespace

extern "C" int ingest_create(const carve_index* idx, const carve_ingest_params* params, carve_ingest** out) {
  if (!idx || !out) return carve_fail_msg(CARVE_EINVAL, "ingest_create: null argument");
  if (carve_index_unit_bytes(idx) != kSector) return carve_fail_msg(CARVE_EINVAL, "ingest_create: a fragment index");
  carve_ingest_params p{};
  if (params) p = *params;
  for (uint32_t r : p.reserved)
    if (r) return carve_fail_msg(CARVE_EINVAL, "ingest_create: reserved params must be zero");
  if (!p.chunk_bytes) p.chunk_bytes = kDefaultChunk;
  if (p.chunk_bytes % kCluster) return carve_fail_msg(CARVE_EINVAL, "ingest_create: chunk_bytes not a multiple of 4096");
  if (!p.copy_threads) p.copy_threads = 8;
  if (p.copy_threads > 64) return carve_fail_msg(CARVE_EINVAL, "ingest_create: at most 64 copy threads");
  carve_ingest* in = new carve_ingest();
  in->idx = idx;
  in->p = p;
  bool ok = hipStreamCreateWithFlags(&in->copy, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&in->comp, hipStreamNonBlocking) == hipSuccess;   // default priority
  for (int b = 0; ok && b < 2; ++b)
    ok = hipMalloc(&in->g[b], p.chunk_bytes) == hipSuccess &&
         hipHostMalloc(&in->h[b], p.chunk_bytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&in->copied[b], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&in->done[b], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    ingest_free(in);
    return carve_fail_msg(CARVE_ENOMEM, "ingest_create: buffer, stream or event creation failed");
  }
  *out = in;
  return CARVE_OK;
}

extern "C" int ingest_scan(carve_ingest* in, const void* host_image, uint64_t n_bytes, uint32_t tau0,
                           uint32_t tau_mode) {
  if (!in) return carve_fail_msg(CARVE_EINVAL, "ingest_scan: null ingest");
  if (n_bytes >= kSector && !host_image) return carve_fail_msg(CARVE_EINVAL, "ingest_scan: null image");
  if (tau0 > 7 || (tau_mode != CARVE_TAU_PER_CLUSTER && tau_mode != CARVE_TAU_ANY))
    return carve_fail_msg(CARVE_EINVAL, "ingest_scan: bad tau0 or tau_mode");
  const auto t0 = std::chrono::steady_clock::now();
  in->ids.clear();
  in->matches.clear();
  const uint64_t scanned = n_bytes - n_bytes % kSector;   // a trailing partial sector is not scanned
  const bool pinned = scanned && is_pinned(host_image);
  const uint64_t C = in->p.chunk_bytes;
  const uint64_t n_chunks = (scanned + C - 1) / C;
  int rc = CARVE_OK;
  for (uint64_t i = 0; i < n_chunks && rc == CARVE_OK; ++i) {
    const int b = (int)(i & 1);
    if ((rc = collect(in, b)) != CARVE_OK) break;   // chunk i - 2: its buffers are free afterwards
    const uint64_t off = i * C, len = std::min(C, scanned - off);
    const void* src = (const uint8_t*)host_image + off;
    if (!pinned) {
      parallel_copy(in->h[b], src, len, in->p.copy_threads);
      src = in->h[b];
    }
    if (hipMemcpyAsync(in->g[b], src, len, hipMemcpyHostToDevice, in->copy) != hipSuccess ||
        hipEventRecord(in->copied[b], in->copy) != hipSuccess ||
        hipStreamWaitEvent(in->comp, in->copied[b], 0) != hipSuccess) {
      rc = carve_fail_msg(CARVE_EDEVICE, "ingest_scan: transfer failed");
      break;
    }
    // chunks start on cluster boundaries, so every chunk keeps the image's tau0
    rc = scan_image(in->idx, in->g[b], len, tau0, tau_mode, in->comp, &in->scan[b]);
    if (rc == CARVE_OK && in->p.confirm) rc = confirm_enqueue(in->idx, in->scan[b]);
    if (rc == CARVE_OK && hipEventRecord(in->done[b], in->comp) != hipSuccess)
      rc = carve_fail_msg(CARVE_EDEVICE, "ingest_scan: event record failed");
    if (rc == CARVE_OK) {
      in->busy[b] = true;
      in->first_sector[b] = off / kSector;
    }
  }
  // the last two chunks, in order
  if (rc == CARVE_OK && n_chunks >= 2) rc = collect(in, (int)(n_chunks & 1));
  if (rc == CARVE_OK) rc = collect(in, (int)((n_chunks + 1) & 1));
  if (rc != CARVE_OK) {   // leave nothing in flight
    (void)hipStreamSynchronize(in->copy);
    (void)hipStreamSynchronize(in->comp);
    in->busy[0] = in->busy[1] = false;
    return rc;
  }
  in->st.bytes = scanned;
  in->st.chunks = n_chunks;
  in->st.pinned_source = pinned ? 1 : 0;
  in->st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return CARVE_OK;
}

extern "C" int ingest_flagged_sectors(const carve_ingest* in, uint64_t* out, uint64_t cap, uint64_t* n_out) {
  if (!in || !n_out || (cap && !out)) return carve_fail_msg(CARVE_EINVAL, "ingest_flagged_sectors: null argument");
  *n_out = in->ids.size();
  const uint64_t k = std::min<uint64_t>(cap, in->ids.size());
  if (k) memcpy(out, in->ids.data(), k * sizeof(uint64_t));
  return in->ids.size() > cap ? carve_fail_msg(CARVE_ETRUNC, "ingest_flagged_sectors: capacity too small")
                              : CARVE_OK;
}

extern "C" int ingest_matches(const carve_ingest* in, carve_match* out, uint64_t cap, uint64_t* n_out) {
  if (!in || !n_out || (cap && !out)) return carve_fail_msg(CARVE_EINVAL, "ingest_matches: null argument");
  *n_out = in->matches.size();
  const uint64_t k = std::min<uint64_t>(cap, in->matches.size());
  if (k) memcpy(out, in->matches.data(), k * sizeof(carve_match));
  return in->matches.size() > cap ? carve_fail_msg(CARVE_ETRUNC, "ingest_matches: capacity too small") : CARVE_OK;
}

extern "C" int ingest_stats(const carve_ingest* in, carve_ingest_stats* out) {
  if (!in || !out) return carve_fail_msg(CARVE_EINVAL, "ingest_stats: null argument");
  *out = in->st;
  return CARVE_OK;
}

extern "C" void ingest_free(carve_ingest* in) {
  if (!in) return;
  if (in->copy) (void)hipStreamSynchronize(in->copy);
  if (in->comp) (void)hipStreamSynchronize(in->comp);
  for (int b = 0; b < 2; ++b) {
    free_scan(in->scan[b]);
    if (in->g[b]) (void)hipFree(in->g[b]);
    if (in->h[b]) (void)hipHostFree(in->h[b]);
    if (in->copied[b]) (void)hipEventDestroy(in->copied[b]);
    if (in->done[b]) (void)hipEventDestroy(in->done[b]);
  }
  if (in->copy) (void)hipStreamDestroy(in->copy);
  if (in->comp) (void)hipStreamDestroy(in->comp);
  delete in;
}
