// Serving loop of the polar SCL decoder (declarations and contracts in
// include/polar_scl.h): continuous batching over a set of HIP streams, each
// slot with its own work area so that admitted batches run concurrently.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "../../include/polar_scl.h"
#include "batch.h"

struct polar_server_s {
  polar_server_config cfg{};
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint32_t* work = nullptr;
    char* spill = nullptr;  // depth-1 slots of spilled layouts, grown on demand
    uint64_t spill_bytes = 0;
    bool busy = false;
    uint32_t frames = 0;
    uint64_t tag = 0;
  };
  std::vector<Slot> slots;
  uint32_t inflight = 0;
};

namespace {

void release(polar_server s) {
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.work) (void)hipFree(sl.work);
    if (sl.spill) (void)hipFree(sl.spill);
  }
  delete s;
}

}  // namespace

extern "C" {

int polar_server_create(const polar_server_config* cfg, polar_server* out) {
  if (!cfg || !out || cfg->n_slots == 0 || cfg->n_slots > 64 || cfg->max_batch == 0 ||
      cfg->max_inflight == 0)
    return POLAR_EINVAL;
  *out = nullptr;
  polar_server s = new (std::nothrow) polar_server_s;
  if (!s) return POLAR_ENOMEM;
  s->cfg = *cfg;
  s->slots.resize(cfg->n_slots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      release(s);
      return POLAR_EHIP;
    }
    if (hipMalloc(&sl.work, polar::work_words(cfg->max_batch) * sizeof(uint32_t)) != hipSuccess) {
      release(s);
      return POLAR_ENOMEM;
    }
  }
  *out = s;
  return POLAR_OK;
}

int polar_server_submit(polar_server s, const polar_plan* plans, uint32_t n_plans,
                        const polar_frame* d_frames, uint32_t first, uint32_t count,
                        const void* d_llr, uint32_t* d_info, polar_status* d_status,
                        uint64_t tag, uint32_t* slot) {
  if (!s || !d_frames || count == 0 || count > s->cfg.max_batch) return POLAR_EINVAL;
  if (s->inflight + count > s->cfg.max_inflight) return POLAR_EAGAIN;
  uint32_t i = 0;
  while (i < s->slots.size() && s->slots[i].busy) ++i;
  if (i == s->slots.size()) return POLAR_EAGAIN;
  polar::Batch b;
  int rc = polar::prepare(plans, n_plans, d_frames + first, count, d_llr, d_info,
                          d_status ? d_status + first : nullptr, nullptr, nullptr, &b);
  if (rc) return rc;
  auto& sl = s->slots[i];
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return POLAR_EHIP;
  const uint64_t sp = polar::spill_need(b, cus);
  if (sp > sl.spill_bytes) {  // the slot is idle: nothing of it is in flight
    if (sl.spill) (void)hipFree(sl.spill);
    sl.spill = nullptr;
    sl.spill_bytes = 0;
    if (hipMalloc(&sl.spill, sp) != hipSuccess) return POLAR_ENOMEM;
    sl.spill_bytes = sp;
  }
  polar::Work w = polar::work_view(sl.work, s->cfg.max_batch);
  w.spill = sl.spill;
  w.spill_bytes = sl.spill_bytes;
  rc = polar::launch_batch(b, 0, w, sl.stream, false, false);
  if (rc) return rc;
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return POLAR_EHIP;
  sl.busy = true;
  sl.frames = count;
  sl.tag = tag;
  s->inflight += count;
  if (slot) *slot = i;
  return POLAR_OK;
}

int polar_server_poll(polar_server s, uint64_t* tags, uint32_t max, uint32_t* n) {
  if (!s || !n || (max && !tags)) return POLAR_EINVAL;
  *n = 0;
  for (auto& sl : s->slots) {
    if (!sl.busy || *n >= max) continue;
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return POLAR_EHIP;
    sl.busy = false;
    s->inflight -= sl.frames;
    tags[(*n)++] = sl.tag;
  }
  return POLAR_OK;
}

int polar_server_inflight(polar_server s, uint32_t* frames) {
  if (!s || !frames) return POLAR_EINVAL;
  *frames = s->inflight;
  return POLAR_OK;
}

int polar_server_destroy(polar_server s) {
  if (!s) return POLAR_OK;
  release(s);
  return POLAR_OK;
}

int polar_serve_replay(polar_server s, const polar_plan* plans, uint32_t n_plans,
                       const polar_frame* d_frames, uint32_t n_req, const double* arrival_us,
                       const void* d_llr, uint32_t* d_info, polar_status* d_status,
                       double* complete_us, double* stats) {
  if (!s || !plans || !d_frames || !arrival_us || !complete_us || !d_status) return POLAR_EINVAL;
  if (n_req == 0) return POLAR_OK;
  if (s->inflight) return POLAR_EINVAL;  // the session owns the server
  for (uint32_t r = 1; r < n_req; ++r)
    if (arrival_us[r] < arrival_us[r - 1]) return POLAR_EINVAL;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_us = [&]() {
    return std::chrono::duration<double, std::micro>(clk::now() - t0).count();
  };
  std::vector<uint64_t> tags(s->slots.size());
  uint32_t next = 0, done = 0, batches = 0, peak = 0;
  double frames_sum = 0;
  int rc = POLAR_OK;
  while (done < n_req) {
    const double t = now_us();
    // admit every released request (one batch), as budget and slots allow
    if (next < n_req && arrival_us[next] <= t) {
      const uint32_t released =
          (uint32_t)(std::upper_bound(arrival_us + next, arrival_us + n_req, t) - arrival_us);
      uint32_t count = std::min(released - next, s->cfg.max_batch);
      count = std::min(count, s->cfg.max_inflight - std::min(s->cfg.max_inflight, s->inflight));
      if (count) {
        rc = polar_server_submit(s, plans, n_plans, d_frames, next, count, d_llr, d_info,
                                 d_status, ((uint64_t)next << 32) | count, nullptr);
        if (rc == POLAR_OK) {
          next += count;
          ++batches;
          frames_sum += count;
          peak = std::max(peak, s->inflight);
        } else if (rc != POLAR_EAGAIN) {
          break;
        }
        rc = POLAR_OK;
      }
    }
    uint32_t n = 0;
    rc = polar_server_poll(s, tags.data(), (uint32_t)tags.size(), &n);
    if (rc) break;
    if (n) {
      const double tc = now_us();
      for (uint32_t k = 0; k < n; ++k) {
        const uint32_t lo = (uint32_t)(tags[k] >> 32), cnt = (uint32_t)tags[k];
        for (uint32_t r = lo; r < lo + cnt; ++r) complete_us[r] = tc;
        done += cnt;
      }
    }
  }
  if (rc) {
    for (auto& sl : s->slots) (void)hipStreamSynchronize(sl.stream);
    uint32_t n = 0;
    (void)polar_server_poll(s, tags.data(), (uint32_t)tags.size(), &n);
    return rc;
  }
  if (stats) {
    stats[0] = batches;
    stats[1] = batches ? frames_sum / batches : 0.0;
    stats[2] = peak;
    stats[3] = now_us();
  }
  return POLAR_OK;
}

}  // extern "C"
