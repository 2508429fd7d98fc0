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
    char* spill = nullptr;  // spill regions of the slot's launches (fixed size)
    uint64_t spill_bytes = 0;
    bool busy = false;
    uint32_t frames = 0;
    uint64_t bytes = 0;  // charged to the byte budget
    uint64_t tag = 0;
  };
  std::vector<Slot> slots;
  uint32_t inflight = 0;
  uint64_t inflight_bytes = 0;
  int cus = 1;
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
  if (s->cfg.slot_spill_bytes == 0) s->cfg.slot_spill_bytes = 64ull << 20;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete s;
    return POLAR_EHIP;
  }
  s->slots.resize(cfg->n_slots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      release(s);
      return POLAR_EHIP;
    }
    // every device buffer of the slot is allocated here, none in submit
    if (hipMalloc(&sl.work, polar::work_words(cfg->max_batch) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&sl.spill, s->cfg.slot_spill_bytes) != hipSuccess) {
      release(s);
      return POLAR_ENOMEM;
    }
    sl.spill_bytes = s->cfg.slot_spill_bytes;
  }
  *out = s;
  return POLAR_OK;
}

int polar_server_submit(polar_server s, const polar_plan* plans, uint32_t n_plans,
                        const polar_frame* d_frames, uint32_t first, uint32_t count,
                        const uint32_t* h_plan_idx, const void* d_llr, uint32_t* d_info,
                        polar_status* d_status, uint64_t tag, uint32_t* slot) {
  if (!s || !plans || n_plans == 0 || !d_frames || count == 0 || count > s->cfg.max_batch)
    return POLAR_EINVAL;
  if (s->inflight + count > s->cfg.max_inflight) return POLAR_EAGAIN;
  // bytes the batch is charged: per frame, its plan's figure (the largest of
  // the list without host plan indices)
  uint64_t bytes = 0;
  if (s->cfg.budget_bytes) {
    std::vector<uint64_t> cost(n_plans, 0);
    for (uint32_t p = 0; p < n_plans; ++p)
      if (polar_plan_frame_bytes(plans[p], &cost[p]) != POLAR_OK) return POLAR_EINVAL;
    if (h_plan_idx) {
      for (uint32_t i = 0; i < count; ++i) {
        if (h_plan_idx[i] >= n_plans) return POLAR_EINVAL;
        bytes += cost[h_plan_idx[i]];
      }
    } else {
      bytes = (uint64_t)count * *std::max_element(cost.begin(), cost.end());
    }
    if (s->inflight_bytes + bytes > s->cfg.budget_bytes) return POLAR_EAGAIN;
  }
  uint32_t i = 0;
  while (i < s->slots.size() && s->slots[i].busy) ++i;
  if (i == s->slots.size()) return POLAR_EAGAIN;
  polar::Batch b;
  int rc = polar::prepare(plans, n_plans, d_frames + first, count, d_llr, d_info,
                          d_status ? d_status + first : nullptr, nullptr, nullptr, &b);
  if (rc) return rc;
  auto& sl = s->slots[i];
  // persistent grids cut to the slot's fixed spill area
  b.spill_cap = sl.spill_bytes;
  if (polar::spill_need(b, s->cus) > sl.spill_bytes) return POLAR_EUNSUP;
  polar::Work w = polar::work_view(sl.work, s->cfg.max_batch);
  w.spill = sl.spill;
  w.spill_bytes = sl.spill_bytes;
  rc = polar::launch_batch(b, 0, w, sl.stream, false, false);
  if (rc) return rc;
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return POLAR_EHIP;
  sl.busy = true;
  sl.frames = count;
  sl.bytes = bytes;
  sl.tag = tag;
  s->inflight += count;
  s->inflight_bytes += bytes;
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
    s->inflight_bytes -= sl.bytes;
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
                       const uint32_t* h_plan_of, const void* d_llr, uint32_t* d_info,
                       polar_status* d_status, double* complete_us, double* stats) {
  if (!s || !plans || !d_frames || !arrival_us || !complete_us || !d_status) return POLAR_EINVAL;
  if (n_req == 0) return POLAR_OK;
  if (s->inflight) return POLAR_EINVAL;  // the session owns the server
  for (uint32_t r = 1; r < n_req; ++r)
    if (arrival_us[r] < arrival_us[r - 1]) return POLAR_EINVAL;
  // cumulative bytes of the requests, for admission by the byte budget
  std::vector<uint64_t> cum;
  if (s->cfg.budget_bytes) {
    std::vector<uint64_t> cost(n_plans, 0);
    for (uint32_t p = 0; p < n_plans; ++p)
      if (polar_plan_frame_bytes(plans[p], &cost[p]) != POLAR_OK) return POLAR_EINVAL;
    const uint64_t top = *std::max_element(cost.begin(), cost.end());
    cum.assign(n_req + 1, 0);
    for (uint32_t r = 0; r < n_req; ++r) {
      if (h_plan_of && h_plan_of[r] >= n_plans) return POLAR_EINVAL;
      cum[r + 1] = cum[r] + (h_plan_of ? cost[h_plan_of[r]] : top);
    }
  }
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto now_us = [&]() {
    return std::chrono::duration<double, std::micro>(clk::now() - t0).count();
  };
  std::vector<uint64_t> tags(s->slots.size());
  uint32_t next = 0, done = 0, batches = 0, peak = 0;
  uint64_t peak_bytes = 0;
  double frames_sum = 0;
  int rc = POLAR_OK;
  while (done < n_req) {
    const double t = now_us();
    // admit the released requests (one batch), as slots and budget allow
    if (next < n_req && arrival_us[next] <= t) {
      const uint32_t released =
          (uint32_t)(std::upper_bound(arrival_us + next, arrival_us + n_req, t) - arrival_us);
      uint32_t count = std::min(released - next, s->cfg.max_batch);
      count = std::min(count, s->cfg.max_inflight - std::min(s->cfg.max_inflight, s->inflight));
      if (s->cfg.budget_bytes && count) {
        const uint64_t room = s->cfg.budget_bytes - std::min(s->cfg.budget_bytes, s->inflight_bytes);
        const uint32_t fit = (uint32_t)(std::upper_bound(cum.begin() + next, cum.begin() + next + count + 1,
                                                         cum[next] + room) -
                                        (cum.begin() + next)) - 1u;
        count = std::min(count, fit);
      }
      if (count) {
        rc = polar_server_submit(s, plans, n_plans, d_frames, next, count,
                                 h_plan_of ? h_plan_of + next : nullptr, d_llr, d_info, d_status,
                                 ((uint64_t)next << 32) | count, nullptr);
        if (rc == POLAR_OK) {
          next += count;
          ++batches;
          frames_sum += count;
          peak = std::max(peak, s->inflight);
          peak_bytes = std::max(peak_bytes, s->inflight_bytes);
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
    stats[4] = (double)peak_bytes;
  }
  return POLAR_OK;
}

}  // extern "C"
