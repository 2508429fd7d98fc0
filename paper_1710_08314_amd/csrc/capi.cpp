// C ABI of the polar SCL decoder (declarations and contracts in
// include/polar_scl.h).  Host-side validation, plan upload and launches.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/polar_scl.h"
#include "kernels.h"
#include "plan.h"

struct polar_plan_s {
  polar::HostPlan hp;
  int device = 0;
  polar::DevPlan* d_blob = nullptr;
  const polar::DevPlan** d_self = nullptr;  // one-entry device plan table
};

namespace {

std::mutex g_mu;
// per-device escalation queue of the tiered schedule (grown on demand)
struct Scratch {
  uint32_t* q = nullptr;
  size_t cap = 0;  // frame slots
  int cus = 0;
};
std::map<int, Scratch> g_scratch;
thread_local size_t g_cap_current = 0;

int device_scratch(size_t frames, uint32_t** q, int* cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch& sc = g_scratch[dev];
  if (sc.cus == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return POLAR_EHIP;
    sc.cus = v > 0 ? v : 1;
  }
  if (sc.cap < frames) {
    if (sc.q) {
      // the previous queue may still be in use by work queued on any stream
      if (hipDeviceSynchronize() != hipSuccess) return POLAR_EHIP;
      (void)hipFree(sc.q);
      sc.q = nullptr;
      sc.cap = 0;
    }
    const size_t want = frames < 4096 ? 4096 : frames;
    // two queues of (want + 2) words each
    if (hipMalloc(&sc.q, 2 * (want + 2) * sizeof(uint32_t)) != hipSuccess) return POLAR_ENOMEM;
    sc.cap = want;
  }
  *q = sc.q;
  *cus = sc.cus;
  g_cap_current = sc.cap;
  return POLAR_OK;
}

// events of the last timed call on this host thread: before the first
// kernel, after the SC tier, after list tier A, after list tier B; and which
// ran (plain schedule: [0] .. [3] bracket the one kernel)
struct TierTiming {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ran[3] = {false, false, false};
  bool plain = false, valid = false;
};
thread_local TierTiming g_timing;

hipEvent_t* timing_events() {
  for (auto& e : g_timing.ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return nullptr;
  return g_timing.ev;
}

// capacity (frame slots) of the queues returned by the last device_scratch()
size_t device_queue_cap() { return g_cap_current; }
// device plan tables of multi-plan batches, keyed by the plan list
std::map<std::vector<polar_plan>, const polar::DevPlan**> g_tables;

int hip_ok(hipError_t e) { return e == hipSuccess ? POLAR_OK : POLAR_EHIP; }

const polar::DevPlan* const* plan_table(const polar_plan* plans, uint32_t n, int* rc) {
  *rc = POLAR_OK;
  if (n == 1) return plans[0]->d_self;
  std::vector<polar_plan> key(plans, plans + n);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) return it->second;
  std::vector<const polar::DevPlan*> h(n);
  for (uint32_t i = 0; i < n; ++i) h[i] = plans[i]->d_blob;
  const polar::DevPlan** d = nullptr;
  if (hipMalloc(&d, n * sizeof(void*)) != hipSuccess) {
    *rc = POLAR_ENOMEM;
    return nullptr;
  }
  if (hipMemcpy(d, h.data(), n * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    *rc = POLAR_EHIP;
    return nullptr;
  }
  g_tables.emplace(std::move(key), d);
  return d;
}

void forget_tables(polar_plan p) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto it = g_tables.begin(); it != g_tables.end();) {
    bool uses = false;
    for (auto q : it->first) uses |= (q == p);
    if (uses) {
      (void)hipFree(it->second);
      it = g_tables.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace

extern "C" {

int polar_scl_plan(const polar_plan_desc* desc, polar_plan* out) {
  if (!desc || !out) return POLAR_EINVAL;
  polar_plan p = new (std::nothrow) polar_plan_s;
  if (!p) return POLAR_ENOMEM;
  int rc = polar::make_plan(*desc, p->hp);
  if (rc) {
    delete p;
    return rc;
  }
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return POLAR_EHIP;
  }
  const size_t bytes = p->hp.blob.size() * 4;
  if (hipMalloc(&p->d_blob, bytes) != hipSuccess) {
    delete p;
    return POLAR_ENOMEM;
  }
  if (hipMalloc(&p->d_self, sizeof(void*)) != hipSuccess) {
    (void)hipFree(p->d_blob);
    delete p;
    return POLAR_ENOMEM;
  }
  const polar::DevPlan* self = p->d_blob;
  if (hipMemcpy(p->d_blob, p->hp.blob.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_self, &self, sizeof(void*), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->d_blob);
    (void)hipFree(p->d_self);
    delete p;
    return POLAR_EHIP;
  }
  *out = p;
  return POLAR_OK;
}

int polar_plan_destroy(polar_plan p) {
  if (!p) return POLAR_OK;
  forget_tables(p);
  int rc = POLAR_OK;
  if (p->d_blob && hipFree(p->d_blob) != hipSuccess) rc = POLAR_EHIP;
  if (p->d_self && hipFree(p->d_self) != hipSuccess) rc = POLAR_EHIP;
  delete p;
  return rc;
}

namespace {
void fill_info(const polar::HostPlan& hp, polar_plan_info* o) {
  const polar::DevPlan& h = hp.hdr;
  std::memset(o, 0, sizeof(*o));
  o->N = h.N;
  o->K = h.K;
  o->crc_len = h.c;
  o->n_tx = h.n_tx;
  o->k_data = h.k_data;
  o->info_words = h.info_words;
  o->code_words = h.code_words;
  o->llr_bytes = h.n_tx * polar::elem_bytes(h.quant);
  o->max_list = h.max_list;
  o->n_ops = h.n_ops;
  o->n_r0 = hp.counts.r0;
  o->n_r1 = hp.counts.r1;
  o->n_rep = hp.counts.rep;
  o->n_spc = hp.counts.spc;
  o->n_leaf_frozen = hp.counts.leaf_f;
  o->n_leaf_info = hp.counts.leaf_i;
  o->lds_bytes = h.lds_max;
}
}  // namespace

int polar_plan_get_info(polar_plan p, polar_plan_info* o) {
  if (!p || !o) return POLAR_EINVAL;
  fill_info(p->hp, o);
  return POLAR_OK;
}

int polar_plan_query(const polar_plan_desc* desc, polar_plan_info* info, uint32_t* frozen_words) {
  if (!desc || !info) return POLAR_EINVAL;
  polar::HostPlan hp;
  const int rc = polar::make_plan(*desc, hp);
  if (rc) return rc;
  fill_info(hp, info);
  if (frozen_words) std::memcpy(frozen_words, hp.frozen.data(), hp.frozen.size() * 4);
  return POLAR_OK;
}

int polar_plan_get_frozen(polar_plan p, uint32_t* fw) {
  if (!p || !fw) return POLAR_EINVAL;
  std::memcpy(fw, p->hp.frozen.data(), p->hp.frozen.size() * 4);
  return POLAR_OK;
}

int polar_scl_decode_batch(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
                           uint32_t n_frames, const void* d_llr, uint32_t* d_info,
                           polar_status* d_status, uint32_t* d_pm_lists,
                           const polar_decode_opts* opts, void* stream) {
  if (!plans || n_plans == 0) return POLAR_EINVAL;
  for (uint32_t i = 0; i < n_plans; ++i)
    if (!plans[i]) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (!d_llr || !d_info || !d_status) return POLAR_EINVAL;
  if (!d_frames && n_plans != 1) return POLAR_EINVAL;
  const uint32_t quant = plans[0]->hp.hdr.quant;
  uint32_t lds = 0, pm_stride = 0;
  for (uint32_t i = 0; i < n_plans; ++i) {
    const polar::DevPlan& h = plans[i]->hp.hdr;
    if (h.quant != quant) return POLAR_EINVAL;
    lds = h.lds_max > lds ? h.lds_max : lds;
    pm_stride = h.max_list > pm_stride ? h.max_list : pm_stride;
  }
  int rc = POLAR_OK;
  polar::KArgs A{};
  A.plans = plan_table(plans, n_plans, &rc);
  if (rc) return rc;
  A.frames = d_frames;
  A.n_frames = n_frames;
  A.llr = static_cast<const char*>(d_llr);
  A.llr_bytes = plans[0]->hp.hdr.n_tx * polar::elem_bytes(quant);
  A.info_words = plans[0]->hp.hdr.info_words;
  A.info = d_info;
  A.status = d_status;
  A.pm_lists = d_pm_lists;
  A.pm_stride = pm_stride;
  A.times = opts ? opts->d_times : nullptr;
  const uint32_t grid = n_frames < 0x7FFFFFFFu ? n_frames : 0x7FFFFFFFu;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t schedule = opts ? opts->schedule : 0;
  const bool timed = opts && (opts->flags & POLAR_OPT_TIER_TIMING);
  hipEvent_t* ev = timed ? timing_events() : nullptr;
  if (timed && !ev) return POLAR_EHIP;
  if (schedule == 1) {
    if (ev) (void)hipEventRecord(ev[0], st);
    rc = polar::launch_decode_plain(quant, A, lds, grid, st);
    if (ev) {
      (void)hipEventRecord(ev[3], st);
      g_timing.plain = true;
      g_timing.valid = rc == POLAR_OK;
    }
    return rc;
  }
  if (schedule != 0) return POLAR_EINVAL;
  // tiered schedule: SC tier if any plan starts at L = 1; list tier A if any
  // plan has a stage of list size 2..4; list tier B if any plan has a stage
  // above 4 (the stages of a plan: SC {1}, CA {L}, PA {1, L_max}, FA {1, 2,
  // 4, ..., L_max})
  polar::TierPlan tp{};
  uint32_t lds_sc = 0, lds_a = 0;
  for (uint32_t i = 0; i < n_plans; ++i) {
    const polar::DevPlan& h = plans[i]->hp.hdr;
    if (h.first_stage == 1) tp.run_sc = true;
    const bool fa = h.algo == POLAR_FA_SCL;
    const bool has_a = (h.first_stage > 1 && h.first_stage <= polar::kTierALmax) ||
                       (h.first_stage == 1 && h.max_list > 1 &&
                        (fa || h.max_list <= polar::kTierALmax));
    // list tier A is used for single-plan batches only: a batch of several
    // plans goes from the SC tier straight to list tier B (which then runs
    // every remaining stage)
    if (has_a && n_plans == 1) {
      tp.run_a = true;
      const uint32_t la = h.max_list < polar::kTierALmax ? h.max_list : polar::kTierALmax;
      const uint32_t b = polar::plan_lds_bytes(h, la);
      lds_a = b > lds_a ? b : lds_a;
    }
    if (h.max_list > polar::kTierALmax || (n_plans > 1 && h.max_list > 1)) tp.run_b = true;
    const uint32_t l1 = polar::sc_lds_bytes(h.N, polar::elem_bytes(h.quant));
    lds_sc = l1 > lds_sc ? l1 : lds_sc;
  }
  uint32_t* q = nullptr;
  int cus = 1;
  rc = device_scratch(n_frames, &q, &cus);
  if (rc) return rc;
  auto persistent = [&](uint32_t lds_wg, uint32_t max_per_cu) {
    uint32_t per_cu = polar::kLdsLimit / (lds_wg ? lds_wg : 1);
    per_cu = per_cu < 1 ? 1 : (per_cu > max_per_cu ? max_per_cu : per_cu);
    const uint64_t g = (uint64_t)cus * per_cu;
    return (uint32_t)(g < n_frames ? g : n_frames);
  };
  tp.lds_sc = lds_sc;
  tp.grid_sc = grid;
  tp.lds_a = lds_a;
  tp.grid_a = persistent(lds_a, 16);
  tp.lds_b = lds;
  tp.grid_b = persistent(lds, 4);
  rc = polar::launch_decode_tiered(quant, A, tp, q, q + 2 + device_queue_cap(), st, ev);
  if (ev) {
    g_timing.ran[0] = tp.run_sc;
    g_timing.ran[1] = tp.run_a;
    g_timing.ran[2] = tp.run_b;
    g_timing.plain = false;
    g_timing.valid = rc == POLAR_OK;
  }
  return rc;
}

int polar_last_tier_ms(float ms[4]) {
  if (!ms || !g_timing.valid) return POLAR_EINVAL;
  for (int i = 0; i < 4; ++i) ms[i] = 0.f;
  float v = 0.f;
  if (g_timing.plain) {
    if (hipEventSynchronize(g_timing.ev[3]) != hipSuccess ||
        hipEventElapsedTime(&v, g_timing.ev[0], g_timing.ev[3]) != hipSuccess)
      return POLAR_EHIP;
    ms[3] = v;
    return POLAR_OK;
  }
  if (hipEventSynchronize(g_timing.ev[3]) != hipSuccess) return POLAR_EHIP;
  for (int i = 0; i < 3; ++i) {
    if (!g_timing.ran[i]) continue;
    if (hipEventElapsedTime(&v, g_timing.ev[i], g_timing.ev[i + 1]) != hipSuccess)
      return POLAR_EHIP;
    ms[i] = v;
  }
  return POLAR_OK;
}

int polar_encode(polar_plan p, const uint32_t* d_data, uint32_t* d_code, uint32_t n_frames,
                 void* stream) {
  if (!p || (n_frames && (!d_data || !d_code))) return POLAR_EINVAL;
  return polar::launch_encode(p->d_blob, p->hp.hdr, d_data, d_code, n_frames,
                              static_cast<hipStream_t>(stream));
}

int polar_gen_data(polar_plan p, uint64_t seed, uint64_t frame0, uint32_t n_frames,
                   uint32_t* d_data, void* stream) {
  if (!p || (n_frames && !d_data)) return POLAR_EINVAL;
  return polar::launch_gen_data(p->hp.hdr, seed, frame0, n_frames, d_data,
                                static_cast<hipStream_t>(stream));
}

int polar_channel(polar_plan p, const uint32_t* d_code, uint32_t n_frames, float ebn0_db,
                  int32_t frac_bits, uint64_t seed, uint64_t frame0, void* d_llr, void* stream) {
  if (!p || (n_frames && (!d_code || !d_llr))) return POLAR_EINVAL;
  if (frac_bits < 0 || frac_bits > 14) return POLAR_EINVAL;
  return polar::launch_channel(p->hp.hdr, d_code, n_frames, ebn0_db, frac_bits, seed, frame0,
                               d_llr, static_cast<hipStream_t>(stream));
}

int polar_plan_stage_work(polar_plan p, uint32_t L, uint64_t* ops) {
  if (!p || !ops || L == 0 || L > polar::kMaxL || (L & (L - 1))) return POLAR_EINVAL;
  *ops = polar::stage_work(p->hp, L);
  return POLAR_OK;
}

int polar_device_clock_khz(uint32_t* khz) {
  if (!khz) return POLAR_EINVAL;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return POLAR_EHIP;
  *khz = (uint32_t)v;
  return POLAR_OK;
}

const char* polar_strerror(int err) {
  switch (err) {
    case POLAR_OK: return "success";
    case POLAR_EINVAL: return "invalid argument";
    case POLAR_EUNSUP: return "unsupported configuration";
    case POLAR_ENOMEM: return "out of memory";
    case POLAR_EHIP: return "HIP runtime error";
    case POLAR_ENOTSYS: return "frozen set not usable for systematic encoding";
    default: return "unknown error";
  }
}

const char* polar_version(void) { return "polar-scl-gfx950 0.1"; }

}  // extern "C"
