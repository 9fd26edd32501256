// Serving runtime: admission by byte budget and continuous batching of scan
// jobs over stream lanes, built on the public batch API of the library (the
// scans themselves are the kernels of carve.hip). Host code only.
//
// A lane is a HIP stream with its own batch object and completion event.
// server_poll first retires lanes whose event has completed, then fills every
// free lane with the queued jobs that fit the budget, oldest first, as one
// batch. Behind a batch's scan the lane enqueues its confirmation and a
// stage-out kernel that writes the batch's counts, flagged ids and confirmed
// matches straight into pinned host buffers, so retiring a batch reads host
// memory and waits on nothing: no lane's readback queues behind another lane's
// scan. The buffers are shared by the batch's jobs (each keeps its slice) and
// recycled once every job of the batch is released. Each lane's device
// workspace is sized at creation for its share of the budget, so serving
// allocates and frees nothing (both synchronize the whole device) unless a
// batch outgrows it.
//
// Jobs may also live in host memory (Section 3.1: sectors arrive from disks
// through host memory). At launch such a job's whole sectors are copied into
// the lane's device arena on the lane's stream, ahead of the scan; pinned
// memory makes the copy asynchronous, pageable memory blocks the caller for
// it. The arena is allocated on the first host job, sized to the lane's share.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/carve.h"
#include "carve_internal.h"

namespace {

uint64_t pow2_at_least(uint64_t n) {
  uint64_t p = 1024;
  while (p < n) p <<= 1;
  return p;
}

// Pinned host array, grown on demand to a power of two. The CPU writes every
// page once when it is allocated: the pages of a fresh pinned allocation are
// mapped for the CPU on first touch, and a first read of a batch's records
// in retire() then took page faults on the serving thread (about 8 ms per
// large batch, measured in a kernel trace as idle gaps between batches in the
// first closed-loop pass after small ones).
template <class T>
struct Pinned {
  T* p = nullptr;
  size_t cap = 0;
  bool reserve(size_t n) {
    if (n <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = pow2_at_least(n);
    if (hipHostMalloc((void**)&p, want * sizeof(T), hipHostMallocDefault) != hipSuccess) return false;
    memset((void*)p, 0, want * sizeof(T));
    cap = want;
    return true;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Results of one retired batch, shared by its jobs.
struct Results {
  Pinned<uint64_t> ids;
  Pinned<carve_batch_match> matches;
};

struct Job {
  carve_image_desc desc{};
  uint64_t bytes = 0;
  bool host = false;   // the image is in host memory (copied to the lane's arena at launch)
  int state = 0;   // 0 queued, 1 running, 2 done (reported), 3 done (to report)
  int32_t status = CARVE_OK;
  std::shared_ptr<Results> res;
  uint64_t flag_at = 0, n_flags = 0, match_at = 0, n_matches = 0;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  carve_batch* batch = nullptr;
  std::vector<uint64_t> jobs;
  uint64_t bytes = 0;
  bool busy = false;
  Pinned<uint64_t> stage;         // [0] flagged, [1] matches, then n_images + 1 id offsets
  void* arena = nullptr;          // device copies of the batch's host-memory jobs
  uint64_t arena_cap = 0;
  std::shared_ptr<Results> res;   // ids and records of the batch in flight
  uint64_t match_room = 0;        // records the device held for the stage-out
};

// Results room for a batch of `sectors` sectors: one flagged sector in eight
// (more take the synchronous path at retirement).
uint64_t results_room(uint64_t sectors) { return sectors / 8 + 4096; }

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct carve_server {
  const carve_index* idx = nullptr;
  carve_server_params p{};
  std::vector<Lane> lanes;
  std::deque<uint64_t> queue;
  std::deque<uint64_t> to_report;
  std::unordered_map<uint64_t, Job> jobs;
  uint64_t next_id = 1;
  uint64_t in_flight = 0;
  uint64_t batches = 0, completed = 0;
  double t_launch = 0, t_retire = 0;
  std::vector<carve_image_desc> descs;
  std::vector<uint64_t> counts;
  uint32_t scan_per_cu = 1;   // scan blocks per CU that stay resident (the batch scan kernel's occupancy)
  uint32_t fail_launches = 0;  // server_fail_next_launches: launches still to fail after enqueuing their work
  std::vector<std::unique_ptr<Results>> spare;   // recycled result buffers

  // Recycled buffers with room for `n` ids and records: the smallest spare
  // that fits, else the largest spare grown (or a new one).
  std::shared_ptr<Results> new_results(uint64_t n, int* rc) {
    size_t pick = spare.size();
    for (size_t i = 0; i < spare.size(); ++i) {
      const Results& r = *spare[i];
      if (r.ids.cap >= n && r.matches.cap >= n && (pick == spare.size() || r.ids.cap < spare[pick]->ids.cap)) pick = i;
    }
    if (pick == spare.size())
      for (size_t i = 0; i < spare.size(); ++i)
        if (pick == spare.size() || spare[i]->ids.cap > spare[pick]->ids.cap) pick = i;
    Results* r;
    if (pick < spare.size()) {
      r = spare[pick].release();
      spare.erase(spare.begin() + (ptrdiff_t)pick);
    } else {
      r = new Results();
    }
    if (!r->ids.reserve(n) || !r->matches.reserve(n))
      *rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
    return std::shared_ptr<Results>(r, [this](Results* x) { spare.emplace_back(x); });
  }
  ~carve_server() {
    for (Lane& ln : lanes) ln.res.reset();
    jobs.clear();   // returns every Results to `spare`
    for (auto& r : spare) {
      r->ids.release();
      r->matches.release();
    }
  }
};

namespace {

// Retire a lane whose batch has completed: per-job results, budget back.
// The stage-out has already put everything in host memory unless a result
// outgrew its room; only then are ids or records fetched synchronously.
int retire(carve_server* s, Lane& ln) {
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t n = (uint32_t)ln.jobs.size();
  int rc = CARVE_OK;
  std::shared_ptr<Results> res = std::move(ln.res);
  const uint64_t* st = ln.stage.p;
  const uint64_t total = st[0];
  const uint64_t* off = st + 2;
  uint64_t nm = s->p.confirm ? st[1] : 0;
  if (total > res->ids.cap) {
    uint64_t got = 0;
    if (!res->ids.reserve(total)) rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
    else rc = batch_flagged_sectors(ln.batch, CARVE_ALL_IMAGES, res->ids.p, res->ids.cap, &got);
  }
  const uint64_t staged = ln.match_room < res->matches.cap ? ln.match_room : res->matches.cap;
  if (rc == CARVE_OK && nm > staged) {
    if (!res->matches.reserve(nm)) rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
    else rc = batch_confirm_matches(s->idx, ln.batch, res->matches.p, res->matches.cap, &nm);
  }
  // slices: the ids of image i are [off[i], off[i+1]); matches are ordered by image
  uint64_t m = 0;
  for (uint32_t i = 0; i < n; ++i) {
    Job& j = s->jobs[ln.jobs[i]];
    j.state = 3;
    j.status = rc;
    if (rc == CARVE_OK) {
      j.res = res;
      j.flag_at = off[i];
      j.n_flags = off[i + 1] - off[i];
      j.match_at = m;
      while (m < nm && res->matches.p[m].image == i) ++m;
      j.n_matches = m - j.match_at;
    }
    s->to_report.push_back(ln.jobs[i]);
  }
  s->completed += n;
  s->in_flight -= ln.bytes;
  ln.jobs.clear();
  ln.bytes = 0;
  ln.busy = false;
  s->t_retire += seconds_since(t0);
  return rc;
}

// Host-memory jobs of the batch being launched: their whole sectors go to the
// lane's arena (4 KiB-aligned slots) on the lane's stream, and their
// descriptors point there.
int stage_host_jobs(carve_server* s, Lane& ln) {
  constexpr uint64_t kAlign = 4096;
  uint64_t need = 0;
  for (uint64_t id : ln.jobs) {
    const Job& j = s->jobs[id];
    if (j.host) need += (j.bytes + kAlign - 1) / kAlign * kAlign;
  }
  if (!need) return CARVE_OK;
  if (need > ln.arena_cap) {
    const uint64_t share = s->p.budget_bytes / s->lanes.size();
    const uint64_t cap = std::max(need, (share + kAlign - 1) / kAlign * kAlign);
    if (ln.arena) (void)hipFree(ln.arena);
    ln.arena = nullptr;
    ln.arena_cap = 0;
    if (hipMalloc(&ln.arena, cap) != hipSuccess) return carve_fail_msg(CARVE_ENOMEM, "server: arena allocation failed");
    ln.arena_cap = cap;
  }
  uint64_t at = 0;
  for (size_t i = 0; i < ln.jobs.size(); ++i) {
    const Job& j = s->jobs[ln.jobs[i]];
    if (!j.host) continue;
    uint8_t* dst = (uint8_t*)ln.arena + at;
    if (j.bytes && hipMemcpyAsync(dst, j.desc.image, j.bytes, hipMemcpyHostToDevice, ln.stream) != hipSuccess)
      return carve_fail_msg(CARVE_EDEVICE, "server: host job copy failed");
    s->descs[i].image = dst;
    s->descs[i].n_bytes = j.bytes;
    at += (j.bytes + kAlign - 1) / kAlign * kAlign;
  }
  return CARVE_OK;
}

// Fill a free lane with queued jobs, oldest first, within the budget. A lane
// takes at most its share of the budget (a job larger than that goes alone),
// so at saturation the lanes' batches overlap instead of one lane holding it all.
int launch(carve_server* s, Lane& ln) {
  const auto t0 = std::chrono::steady_clock::now();
  s->descs.clear();
  const uint64_t share = s->p.budget_bytes / s->lanes.size();
  while (!s->queue.empty() && ln.jobs.size() < s->p.max_jobs_per_batch) {
    Job& j = s->jobs[s->queue.front()];
    if (s->in_flight + j.bytes > s->p.budget_bytes) break;   // admission: wait for budget
    if (!ln.jobs.empty() && ln.bytes + j.bytes > share) break;
    s->in_flight += j.bytes;
    ln.bytes += j.bytes;
    j.state = 1;
    ln.jobs.push_back(s->queue.front());
    s->descs.push_back(j.desc);
    s->queue.pop_front();
  }
  if (ln.jobs.empty()) return CARVE_OK;
  // A lane that starts while another lane's batch runs takes half of the
  // CUs' scan slots: two persistent grids then stay resident together instead
  // of one waiting for the other's blocks to drain. Alone it takes them all.
  bool others = false;
  for (const Lane& o : s->lanes) others = others || (&o != &ln && o.busy);
  const uint32_t half = s->scan_per_cu > 1 ? s->scan_per_cu / 2 : 1;
  int rc = carve_batch_set_grid(ln.batch, others ? half : 0);
  if (rc == CARVE_OK) rc = stage_host_jobs(s, ln);
  if (rc == CARVE_OK) rc = scan_batch(s->idx, s->descs.data(), (uint32_t)s->descs.size(), ln.stream, &ln.batch);
  if (rc == CARVE_OK && s->p.confirm) rc = batch_confirm_enqueue(s->idx, ln.batch);
  if (rc == CARVE_OK) ln.res = s->new_results(results_room(ln.bytes / 512), &rc);
  if (rc == CARVE_OK && !ln.stage.reserve(ln.jobs.size() + 3))
    rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
  if (rc == CARVE_OK) {
    const carve_stage_out st{ln.stage.p, ln.stage.p + 2, ln.res->ids.p, ln.res->ids.cap, ln.res->matches.p,
                             ln.res->matches.cap};
    rc = carve_batch_stage_out(ln.batch, s->p.confirm ? 1 : 0, &st, &ln.match_room);
  }
  if (rc == CARVE_OK && s->fail_launches > 0) {   // a failure after every step above was enqueued
    --s->fail_launches;
    rc = carve_fail_msg(CARVE_EDEVICE, "server: injected launch failure (server_fail_next_launches)");
  }
  if (rc == CARVE_OK && hipEventRecord(ln.done, ln.stream) != hipSuccess)
    rc = carve_fail_msg(CARVE_EDEVICE, "server: event record failed");
  if (rc != CARVE_OK) {   // the jobs fail with the batch's error
    // Work enqueued before the failure (host-job copies, the scan, the
    // confirmation, the stage-out) may still read the jobs' images and write
    // the results buffer: wait for it before the jobs and the buffer are
    // handed back.
    (void)hipStreamSynchronize(ln.stream);
    ln.res.reset();
    for (uint64_t id : ln.jobs) {
      Job& j = s->jobs[id];
      j.state = 3;
      j.status = rc;
      s->to_report.push_back(id);
    }
    s->in_flight -= ln.bytes;
    ln.jobs.clear();
    ln.bytes = 0;
  } else {
    ln.busy = true;
    ++s->batches;
  }
  s->t_launch += seconds_since(t0);
  return rc;
}

}  // namespace

extern "C" int server_create(const carve_index* idx, const carve_server_params* params, carve_server** out) {
  if (!idx || !out) return carve_fail_msg(CARVE_EINVAL, "server_create: null argument");
  if (carve_index_unit_bytes(idx) != 512) return carve_fail_msg(CARVE_EINVAL, "server_create: a fragment index");
  carve_server_params p{};
  if (params) p = *params;
  for (uint32_t r : p.reserved)
    if (r) return carve_fail_msg(CARVE_EINVAL, "server_create: reserved params must be zero");
  if (!p.n_streams) p.n_streams = 2;
  if (!p.max_jobs_per_batch) p.max_jobs_per_batch = 4096;
  if (!p.budget_bytes) p.budget_bytes = 32ull << 30;
  if (p.n_streams > 64) return carve_fail_msg(CARVE_EINVAL, "server_create: at most 64 streams");
  if (p.max_jobs_per_batch > 65536) return carve_fail_msg(CARVE_EINVAL, "server_create: at most 65536 jobs per batch");
  carve_server* s = new carve_server();
  s->idx = idx;
  s->p = p;
  s->scan_per_cu = carve_batch_scan_blocks_per_cu();
  s->lanes.resize(p.n_streams);
  // each lane sized for its share of the budget (a larger single job grows it)
  const uint64_t share_sectors = p.budget_bytes / p.n_streams / 512;
  for (Lane& ln : s->lanes) {
    // default-priority streams only
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
      server_free(s);
      return carve_fail_msg(CARVE_EDEVICE, "server_create: stream or event creation failed");
    }
    int rc = carve_batch_reserve(idx, &ln.batch, share_sectors, p.max_jobs_per_batch, ln.stream);
    if (rc == CARVE_OK && !ln.stage.reserve((uint64_t)p.max_jobs_per_batch + 3))
      rc = carve_fail_msg(CARVE_ENOMEM, "server_create: pinned allocation failed");
    if (rc != CARVE_OK) {
      server_free(s);
      return rc;
    }
  }
  // Warm result buffers, two per lane: a retired batch's buffer stays with its
  // jobs until they are released, and by then the lane already runs its next
  // batch. Pinned allocation (and freeing) stalls the device, so serving at
  // saturation must find them ready.
  {
    std::vector<std::shared_ptr<Results>> warm;
    int rc = CARVE_OK;
    for (size_t i = 0; i < 2 * s->lanes.size() && rc == CARVE_OK; ++i)
      warm.push_back(s->new_results(results_room(share_sectors), &rc));
    warm.clear();   // into the spare pool
    if (rc != CARVE_OK) {
      server_free(s);
      return rc;
    }
  }
  *out = s;
  return CARVE_OK;
}

namespace {
// Checks one job descriptor; `which` >= 0 names it in the message.
int check_job(const carve_server* s, const carve_image_desc* job, long which) {
  char msg[128];
  const char* why = nullptr;
  int code = CARVE_EINVAL;
  if (job->tau0 > 7 || (job->tau_mode != CARVE_TAU_PER_CLUSTER && job->tau_mode != CARVE_TAU_ANY)) {
    why = "bad tau0 or tau_mode";
  } else if ((job->n_bytes >= 512 && !job->image) || (uintptr_t)job->image % 16) {
    why = "null or misaligned image";
  } else if (job->n_bytes - job->n_bytes % 512 > s->p.budget_bytes) {
    why = "job exceeds the budget";
    code = CARVE_EUNSUPPORTED;
  }
  if (!why) return CARVE_OK;
  if (which >= 0) snprintf(msg, sizeof msg, "server_submit: %s (job %ld)", why, which);
  else snprintf(msg, sizeof msg, "server_submit: %s", why);
  return carve_fail_msg(code, msg);
}

// Host memory: pinned (hipHostMalloc) or plain pageable memory, which the
// runtime reports as unregistered (or does not know at all).
bool in_host_memory(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // clear the sticky error
    return true;
  }
  return a.type == hipMemoryTypeUnregistered || a.type == hipMemoryTypeHost;
}

uint64_t enqueue_job(carve_server* s, const carve_image_desc* job) {
  const uint64_t id = s->next_id++;
  Job& j = s->jobs[id];
  j.desc = *job;
  j.bytes = job->n_bytes - job->n_bytes % 512;
  j.host = j.bytes && in_host_memory(job->image);
  s->queue.push_back(id);
  return id;
}
}  // namespace

extern "C" int server_submit(carve_server* s, const carve_image_desc* job, uint64_t* job_id) {
  if (!s || !job || !job_id) return carve_fail_msg(CARVE_EINVAL, "server_submit: null argument");
  const int rc = check_job(s, job, -1);
  if (rc != CARVE_OK) return rc;
  *job_id = enqueue_job(s, job);
  return CARVE_OK;
}

extern "C" int server_submit_many(carve_server* s, const carve_image_desc* jobs, uint32_t n, uint64_t* job_ids) {
  if (!s || (n && (!jobs || !job_ids))) return carve_fail_msg(CARVE_EINVAL, "server_submit_many: null argument");
  for (uint32_t i = 0; i < n; ++i) {
    const int rc = check_job(s, &jobs[i], (long)i);
    if (rc != CARVE_OK) return rc;
  }
  s->jobs.reserve(s->jobs.size() + n);
  for (uint32_t i = 0; i < n; ++i) job_ids[i] = enqueue_job(s, &jobs[i]);
  return CARVE_OK;
}

extern "C" int server_poll(carve_server* s, carve_job_done* done, uint32_t cap, uint32_t* n_done) {
  if (!s || !n_done || (cap && !done)) return carve_fail_msg(CARVE_EINVAL, "server_poll: null argument");
  // A batch that fails in retire() or launch() reports each of its jobs with
  // the error as its status; only a failure that leaves jobs unreported (an
  // event query that fails: the lane stays busy) is the call's own error.
  int rc = CARVE_OK;
  for (Lane& ln : s->lanes) {
    if (!ln.busy) continue;
    const hipError_t q = hipEventQuery(ln.done);
    if (q == hipErrorNotReady) continue;
    if (q == hipSuccess) (void)retire(s, ln);
    else if (rc == CARVE_OK) rc = carve_fail_msg(CARVE_EDEVICE, "server_poll: event query failed");
  }
  for (Lane& ln : s->lanes) {
    if (s->queue.empty()) break;
    if (!ln.busy) (void)launch(s, ln);
  }
  uint32_t k = 0;
  while (k < cap && !s->to_report.empty()) {
    const uint64_t id = s->to_report.front();
    s->to_report.pop_front();
    Job& j = s->jobs[id];
    j.state = 2;
    done[k++] = carve_job_done{id, j.n_flags, j.n_matches, j.status, 0};
  }
  *n_done = k;
  return rc;
}

namespace {
Job* finished(carve_server* s, uint64_t id) {
  auto it = s->jobs.find(id);
  return (it != s->jobs.end() && it->second.state >= 2) ? &it->second : nullptr;
}
}  // namespace

extern "C" int server_job_flags(carve_server* s, uint64_t job_id, uint64_t* out, uint64_t cap, uint64_t* n_out) {
  if (!s || !n_out || (cap && !out)) return carve_fail_msg(CARVE_EINVAL, "server_job_flags: null argument");
  Job* j = finished(s, job_id);
  if (!j) return carve_fail_msg(CARVE_EINVAL, "server_job_flags: no such completed job");
  if (j->status != CARVE_OK) return carve_fail_msg(j->status, "server_job_flags: the job failed (see its status)");
  *n_out = j->n_flags;
  const uint64_t k = j->n_flags < cap ? j->n_flags : cap;
  if (k) memcpy(out, j->res->ids.p + j->flag_at, k * 8);
  return j->n_flags > cap ? carve_fail_msg(CARVE_ETRUNC, "server_job_flags: capacity too small") : CARVE_OK;
}

extern "C" int server_job_matches(carve_server* s, uint64_t job_id, carve_match* out, uint64_t cap, uint64_t* n_out) {
  if (!s || !n_out || (cap && !out)) return carve_fail_msg(CARVE_EINVAL, "server_job_matches: null argument");
  Job* j = finished(s, job_id);
  if (!j) return carve_fail_msg(CARVE_EINVAL, "server_job_matches: no such completed job");
  if (j->status != CARVE_OK) return carve_fail_msg(j->status, "server_job_matches: the job failed (see its status)");
  *n_out = j->n_matches;
  const uint64_t k = j->n_matches < cap ? j->n_matches : cap;
  for (uint64_t i = 0; i < k; ++i) {
    const carve_batch_match& r = j->res->matches.p[j->match_at + i];
    out[i] = carve_match{r.disk_sector, r.file_id, r.sector_in_file};
  }
  return j->n_matches > cap ? carve_fail_msg(CARVE_ETRUNC, "server_job_matches: capacity too small") : CARVE_OK;
}

extern "C" int server_release(carve_server* s, uint64_t job_id) {
  if (!s) return carve_fail_msg(CARVE_EINVAL, "server_release: null server");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end() || it->second.state != 2)   // unknown, running or not yet reported
    return carve_fail_msg(CARVE_EINVAL, "server_release: no such reported job");
  s->jobs.erase(it);
  return CARVE_OK;
}

extern "C" int server_release_many(carve_server* s, const uint64_t* job_ids, uint32_t n) {
  if (!s || (n && !job_ids)) return carve_fail_msg(CARVE_EINVAL, "server_release_many: null argument");
  for (uint32_t i = 0; i < n; ++i) {
    const int rc = server_release(s, job_ids[i]);
    if (rc != CARVE_OK) return rc;
  }
  return CARVE_OK;
}

extern "C" int server_fail_next_launches(carve_server* s, uint32_t n) {
  if (!s) return carve_fail_msg(CARVE_EINVAL, "server_fail_next_launches: null server");
  s->fail_launches = n;
  return CARVE_OK;
}

extern "C" int server_stats(const carve_server* s, carve_server_stats* out) {
  if (!s || !out) return carve_fail_msg(CARVE_EINVAL, "server_stats: null argument");
  carve_server_stats st{};
  st.queued_jobs = s->queue.size();
  for (const Lane& ln : s->lanes) st.running_jobs += ln.jobs.size();
  for (const auto& kv : s->jobs) st.done_jobs += kv.second.state >= 2;
  st.in_flight_bytes = s->in_flight;
  st.batches_launched = s->batches;
  st.jobs_completed = s->completed;
  st.host_launch_s = s->t_launch;
  st.host_retire_s = s->t_retire;
  *out = st;
  return CARVE_OK;
}

extern "C" void server_free(carve_server* s) {
  if (!s) return;
  for (Lane& ln : s->lanes) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    free_batch(ln.batch);
    ln.stage.release();
    if (ln.arena) (void)hipFree(ln.arena);
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  delete s;
}
