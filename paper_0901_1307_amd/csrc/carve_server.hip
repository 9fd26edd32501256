// Serving runtime: admission by byte budget and continuous batching of scan
// jobs over stream lanes, built on the public batch API of the library (the
// scans themselves are the kernels of carve.hip). Host code only.
//
// A lane is a HIP stream with its own batch object and completion event.
// server_poll first retires lanes whose event has completed, then fills every
// free lane with the queued jobs that fit the budget, oldest first, as one
// batch. A retired batch's flagged ids and confirmed matches are copied in two
// transfers into pinned host buffers that its jobs share (each job keeps its
// slice) and that are recycled once every job of the batch is released.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <memory>
#include <unordered_map>
#include <vector>

#include "../../include/carve.h"

// Records a message for carve_last_error() (defined with the other entry points).
extern "C" __attribute__((visibility("hidden"))) int carve_fail_msg(int code, const char* msg);

namespace {

// Pinned host array, grown on demand.
template <class T>
struct Pinned {
  T* p = nullptr;
  size_t cap = 0;
  bool reserve(size_t n) {
    if (n <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t want = n < 1024 ? 1024 : n + n / 2;
    if (hipHostMalloc((void**)&p, want * sizeof(T), hipHostMallocDefault) != hipSuccess) return false;
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
};

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
  std::vector<std::unique_ptr<Results>> spare;   // recycled result buffers

  std::shared_ptr<Results> new_results() {
    Results* r;
    if (!spare.empty()) {
      r = spare.back().release();
      spare.pop_back();
    } else {
      r = new Results();
    }
    return std::shared_ptr<Results>(r, [this](Results* x) { spare.emplace_back(x); });
  }
  ~carve_server() {
    jobs.clear();   // returns every Results to `spare`
    for (auto& r : spare) {
      r->ids.release();
      r->matches.release();
    }
  }
};

namespace {

// Retire a lane whose batch has completed: per-job results, budget back.
int retire(carve_server* s, Lane& ln) {
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t n = (uint32_t)ln.jobs.size();
  int rc = CARVE_OK;
  std::shared_ptr<Results> res = s->new_results();
  s->counts.assign(n, 0);
  if (n) rc = batch_flag_counts(ln.batch, s->counts.data(), n);
  uint64_t total = 0;
  for (uint64_t c : s->counts) total += c;
  uint64_t got = 0;
  if (rc == CARVE_OK && total) {
    if (!res->ids.reserve(total)) rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
    else rc = batch_flagged_sectors(ln.batch, CARVE_ALL_IMAGES, res->ids.p, total, &got);
  }
  uint64_t nm = 0;
  if (rc == CARVE_OK && s->p.confirm && total) {
    // about one match per flagged sector: room for that avoids a second pass
    if (!res->matches.reserve(total + total / 8 + 64)) rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
    if (rc == CARVE_OK) rc = batch_confirm_matches(s->idx, ln.batch, res->matches.p, res->matches.cap, &nm);
    if (rc == CARVE_ETRUNC) {
      if (!res->matches.reserve(nm)) rc = carve_fail_msg(CARVE_ENOMEM, "server: pinned allocation failed");
      else rc = batch_confirm_matches(s->idx, ln.batch, res->matches.p, res->matches.cap, &nm);
    }
  }
  // slices: the ids of image i follow those of images 0..i-1; matches are
  // ordered by image
  uint64_t at = 0, m = 0;
  for (uint32_t i = 0; i < n; ++i) {
    Job& j = s->jobs[ln.jobs[i]];
    j.state = 3;
    j.status = rc;
    if (rc == CARVE_OK) {
      j.res = res;
      j.flag_at = at;
      j.n_flags = s->counts[i];
      at += s->counts[i];
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
  int rc = scan_batch(s->idx, s->descs.data(), (uint32_t)s->descs.size(), ln.stream, &ln.batch);
  // confirmation queued right behind the scan: at retirement only copies remain,
  // and no lane's readback waits for kernels queued behind another lane's scan
  if (rc == CARVE_OK && s->p.confirm) rc = batch_confirm_enqueue(s->idx, ln.batch);
  if (rc == CARVE_OK && hipEventRecord(ln.done, ln.stream) != hipSuccess)
    rc = carve_fail_msg(CARVE_EDEVICE, "server: event record failed");
  if (rc != CARVE_OK) {   // the jobs fail with the batch's error
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
  carve_server_params p{};
  if (params) p = *params;
  for (uint32_t r : p.reserved)
    if (r) return carve_fail_msg(CARVE_EINVAL, "server_create: reserved params must be zero");
  if (!p.n_streams) p.n_streams = 4;
  if (!p.max_jobs_per_batch) p.max_jobs_per_batch = 4096;
  if (!p.budget_bytes) p.budget_bytes = 32ull << 30;
  if (p.n_streams > 64) return carve_fail_msg(CARVE_EINVAL, "server_create: at most 64 streams");
  carve_server* s = new carve_server();
  s->idx = idx;
  s->p = p;
  s->lanes.resize(p.n_streams);
  for (Lane& ln : s->lanes) {
    // default-priority streams only
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
      server_free(s);
      return carve_fail_msg(CARVE_EDEVICE, "server_create: stream or event creation failed");
    }
  }
  *out = s;
  return CARVE_OK;
}

extern "C" int server_submit(carve_server* s, const carve_image_desc* job, uint64_t* job_id) {
  if (!s || !job || !job_id) return carve_fail_msg(CARVE_EINVAL, "server_submit: null argument");
  if (job->tau0 > 7 || (job->tau_mode != CARVE_TAU_PER_CLUSTER && job->tau_mode != CARVE_TAU_ANY))
    return carve_fail_msg(CARVE_EINVAL, "server_submit: bad tau0 or tau_mode");
  if ((job->n_bytes >= 512 && !job->image) || (uintptr_t)job->image % 16)
    return carve_fail_msg(CARVE_EINVAL, "server_submit: null or misaligned image");
  const uint64_t bytes = job->n_bytes - job->n_bytes % 512;
  if (bytes > s->p.budget_bytes) return carve_fail_msg(CARVE_EUNSUPPORTED, "server_submit: job exceeds the budget");
  const uint64_t id = s->next_id++;
  Job& j = s->jobs[id];
  j.desc = *job;
  j.bytes = bytes;
  s->queue.push_back(id);
  *job_id = id;
  return CARVE_OK;
}

extern "C" int server_poll(carve_server* s, carve_job_done* done, uint32_t cap, uint32_t* n_done) {
  if (!s || !n_done || (cap && !done)) return carve_fail_msg(CARVE_EINVAL, "server_poll: null argument");
  int rc = CARVE_OK;
  for (Lane& ln : s->lanes) {
    if (!ln.busy) continue;
    const hipError_t q = hipEventQuery(ln.done);
    if (q == hipErrorNotReady) continue;
    const int r = q == hipSuccess ? retire(s, ln) : carve_fail_msg(CARVE_EDEVICE, "server_poll: event query failed");
    if (r != CARVE_OK && rc == CARVE_OK) rc = r;
  }
  for (Lane& ln : s->lanes) {
    if (s->queue.empty()) break;
    if (ln.busy) continue;
    const int r = launch(s, ln);
    if (r != CARVE_OK && rc == CARVE_OK) rc = r;
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
  *n_out = j->n_flags;
  const uint64_t k = j->n_flags < cap ? j->n_flags : cap;
  if (k) memcpy(out, j->res->ids.p + j->flag_at, k * 8);
  return j->n_flags > cap ? carve_fail_msg(CARVE_ETRUNC, "server_job_flags: capacity too small") : CARVE_OK;
}

extern "C" int server_job_matches(carve_server* s, uint64_t job_id, carve_match* out, uint64_t cap, uint64_t* n_out) {
  if (!s || !n_out || (cap && !out)) return carve_fail_msg(CARVE_EINVAL, "server_job_matches: null argument");
  Job* j = finished(s, job_id);
  if (!j) return carve_fail_msg(CARVE_EINVAL, "server_job_matches: no such completed job");
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
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  delete s;
}
