// C ABI of the polar SCL decoder (declarations and contracts in
// include/polar_scl.h).  Host-side validation, plan upload and launches.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <iterator>
#include <string>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/polar_scl.h"
#include "batch.h"
#include "kernels.h"
#include "plan.h"

struct polar_plan_s {
  polar::HostPlan hp;
  uint64_t frame_bytes = 0;  // device bytes an in-flight frame is charged (serving budget)
  int device = 0;
  polar::DevPlan* d_blob = nullptr;
  const polar::DevPlan** d_self = nullptr;  // one-entry device plan table
};

namespace {

std::mutex g_mu;

using polar::Work;
using polar::work_view;
using polar::work_words;
using polar::Batch;

// per-device shared work area (grown on demand) and compute-unit count
struct Scratch {
  uint32_t* q = nullptr;
  size_t cap = 0;  // frame slots
  int cus = 0;
};
std::map<int, Scratch> g_scratch;

int device_cus(int dev, int* cus) {
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch& sc = g_scratch[dev];
  if (sc.cus == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return POLAR_EHIP;
    sc.cus = v > 0 ? v : 1;
  }
  *cus = sc.cus;
  return POLAR_OK;
}

int device_scratch(size_t frames, Work* w) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  Scratch& sc = g_scratch[dev];
  if (sc.cap < frames) {
    if (sc.q) {
      // the previous area may still be in use by work queued on any stream
      if (hipDeviceSynchronize() != hipSuccess) return POLAR_EHIP;
      (void)hipFree(sc.q);
      sc.q = nullptr;
      sc.cap = 0;
    }
    const size_t want = frames < 4096 ? 4096 : frames;
    if (hipMalloc(&sc.q, work_words(want) * sizeof(uint32_t)) != hipSuccess) return POLAR_ENOMEM;
    sc.cap = want;
  }
  *w = work_view(sc.q, sc.cap);
  return POLAR_OK;
}

// per-device buffer for the depth-1 slots of spilled layouts (grown on demand)
struct SpillBuf {
  char* p = nullptr;
  uint64_t bytes = 0;
};
std::map<int, SpillBuf> g_spill;

int device_spill(uint64_t bytes, Work* w) {
  if (bytes == 0) return POLAR_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  SpillBuf& sb = g_spill[dev];
  if (sb.bytes < bytes) {
    if (sb.p) {
      if (hipDeviceSynchronize() != hipSuccess) return POLAR_EHIP;
      (void)hipFree(sb.p);
      sb.p = nullptr;
      sb.bytes = 0;
    }
    if (hipMalloc(&sb.p, bytes) != hipSuccess) return POLAR_ENOMEM;
    sb.bytes = bytes;
  }
  w->spill = sb.p;
  w->spill_bytes = sb.bytes;
  return POLAR_OK;
}

// events of the last timed call on this host thread: [0] before the first
// kernel, [1] after the SC tier, [2] after list tier A, [3] after list tier B
// (plain schedule: [0] and [3] bracket the one kernel); [4], [5] bracket the
// kernels of the class schedule
struct TierTiming {
  hipEvent_t ev[6] = {};
  bool ran[3] = {false, false, false};
  bool plain = false, classes = false, valid = false;
};
thread_local TierTiming g_timing;

hipEvent_t* timing_events() {
  for (auto& e : g_timing.ev)
    if (!e && hipEventCreate(&e) != hipSuccess) return nullptr;
  return g_timing.ev;
}

// kernel attributes are set once per device, outside any capture
std::map<int, bool> g_attr_done;
int ensure_attributes(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_attr_done[dev]) return POLAR_OK;
  const int rc = polar::init_kernel_attributes();
  if (rc == POLAR_OK) g_attr_done[dev] = true;
  return rc;
}

// class-schedule choices, per plan list
struct ClassConfig {
  uint32_t l8_kernel = polar::CK_W2_L8;  // kernel of the L = 5..8 plans
  uint32_t split_n = 1;                   // classes split by code length
  bool tuned = false;
};
std::map<std::vector<polar_plan>, ClassConfig> g_sched;

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
  for (auto it = g_sched.begin(); it != g_sched.end();) {
    bool uses = false;
    for (auto q : it->first) uses |= (q == p);
    it = uses ? g_sched.erase(it) : std::next(it);
  }
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
  char* area = nullptr;  // set-up of the allocation-free entry point on this device
  if (hipGetDevice(&p->device) != hipSuccess || ensure_attributes(p->device) != POLAR_OK ||
      polar::noalloc_area(&area) != POLAR_OK) {
    delete p;
    return POLAR_EHIP;
  }
  {
    // LLRs, outputs, status, work-area words, and the decoder state of the
    // largest stage of the schedule (its layout's LDS and global parts)
    const polar::DevPlan& h = p->hp.hdr;
    const uint32_t E = polar::elem_bytes(h.quant);
    uint64_t state = 0;
    for (uint32_t L = h.first_stage;; L = polar::stage_after(h.algo == POLAR_PA_SCL, h.L_max, L)) {
      const polar::LdsLayout lay = polar::lds_layout(h.N, h.n, E, L, polar::key_bytes(h.quant));
      const uint64_t v = (uint64_t)lay.total + lay.gbytes;
      state = v > state ? v : state;
      if (L >= h.L_max) break;
    }
    p->frame_bytes = (uint64_t)h.n_tx * E + 4ull * h.info_words + sizeof(polar_status) + 8 + state;
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

int polar_plan_frame_bytes(polar_plan p, uint64_t* bytes) {
  if (!p || !bytes) return POLAR_EINVAL;
  *bytes = p->frame_bytes;
  return POLAR_OK;
}

int polar_plan_get_frozen(polar_plan p, uint32_t* fw) {
  if (!p || !fw) return POLAR_EINVAL;
  std::memcpy(fw, p->hp.frozen.data(), p->hp.frozen.size() * 4);
  return POLAR_OK;
}

}  // extern "C"

namespace polar {

size_t work_words(size_t cap) { return 2 * cap + 1 + 2 * kClaimSegs + kMaxClasses; }

Work work_view(uint32_t* base, size_t cap) {
  Work w;
  w.state = base;
  w.tier_heads = base + cap;
  w.heads = base + cap + 2 * kClaimSegs;
  w.xlist = w.heads + kMaxClasses;
  return w;
}

// The list layouts of a batch's stages with list size in [lo, hi] (every
// stage of every plan's schedule in that range): the largest LDS footprint
// and the largest spill region per workgroup.
StageSpan stage_span(const Batch& b, uint32_t lo, uint32_t hi) {
  StageSpan r{0, 0};
  for (polar_plan p : b.plans) {
    const DevPlan& h = p->hp.hdr;
    for (uint32_t L = h.first_stage;; L = stage_after(h.algo == POLAR_PA_SCL, h.L_max, L)) {
      if (L >= lo && L <= hi) {
        const LdsLayout lay = lds_layout(h.N, h.n, elem_bytes(h.quant), L, key_bytes(h.quant));
        r.lds = lay.total > r.lds ? lay.total : r.lds;
        r.spill = lay.gbytes > r.spill ? lay.gbytes : r.spill;
      }
      if (L >= h.L_max) break;
    }
  }
  return r;
}

}  // namespace polar

namespace {
using polar::launch_batch;
using polar::prepare;
}  // namespace

namespace polar {

int prepare(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
            uint32_t n_frames, const void* d_llr, uint32_t* d_info, polar_status* d_status,
            uint32_t* d_pm_lists, const polar_decode_opts* opts, Batch* b, bool upload_table) {
  if (!plans || n_plans == 0) return POLAR_EINVAL;
  for (uint32_t i = 0; i < n_plans; ++i)
    if (!plans[i]) return POLAR_EINVAL;
  if (!d_llr || !d_info || !d_status) return POLAR_EINVAL;
  if (!d_frames && n_plans != 1) return POLAR_EINVAL;
  b->quant = plans[0]->hp.hdr.quant;
  uint32_t pm_stride = 0;
  bool mixed = false;
  for (uint32_t i = 0; i < n_plans; ++i) {
    const polar::DevPlan& h = plans[i]->hp.hdr;
    mixed = mixed || h.quant != b->quant;
    b->lds = h.lds_max > b->lds ? h.lds_max : b->lds;
    pm_stride = h.max_list > pm_stride ? h.max_list : pm_stride;
    if (h.algo != POLAR_SC && h.algo != POLAR_CA_SCL) b->fixed_list = false;
  }
  // plans of different LLR types in one decode: the class schedule (fixed
  // lists, frame descriptors, automatic schedule), whose classes each take
  // one type
  if (mixed && (!b->fixed_list || !d_frames || n_plans < 2 || (opts && opts->schedule != 0)))
    return POLAR_EINVAL;
  b->plans.assign(plans, plans + n_plans);
  int rc = POLAR_OK;
  polar::KArgs& A = b->A;
  if (upload_table || n_plans == 1) {
    A.plans = plan_table(plans, n_plans, &rc);
    if (rc) return rc;
  }
  A.frames = d_frames;
  A.n_frames = n_frames;
  A.llr = static_cast<const char*>(d_llr);
  A.llr_bytes = plans[0]->hp.hdr.n_tx * polar::elem_bytes(b->quant);
  A.info_words = plans[0]->hp.hdr.info_words;
  A.info = d_info;
  A.status = d_status;
  A.pm_lists = d_pm_lists;
  A.pm_stride = pm_stride;
  A.times = opts ? opts->d_times : nullptr;
  return POLAR_OK;
}

}  // namespace polar

namespace {

bool uses_classes(const Batch& b, uint32_t schedule) {
  return schedule == 0 && b.fixed_list && b.plans.size() > 1 && b.A.frames != nullptr;
}

// persistent grid: as many workgroups as the CUs hold (LDS-limited, at most
// `max_per_cu`), never more than frames
uint32_t persistent_grid(int cus, uint32_t lds_wg, uint32_t max_per_cu, uint32_t n_frames) {
  uint32_t per_cu = polar::kLdsLimit / (lds_wg ? lds_wg : 1);
  per_cu = per_cu < 1 ? 1 : (per_cu > max_per_cu ? max_per_cu : per_cu);
  const uint64_t g = (uint64_t)cus * per_cu;
  return (uint32_t)(g < n_frames ? g : n_frames);
}

// Classes of a fixed-list batch: kernel by list size, then (optionally) by
// code length, each with the LDS of its largest member.
int build_classes(const Batch& b, const ClassConfig& cfg, int cus,
                  std::vector<polar::ClassLaunch>* out) {
  static const uint32_t nb_split[5] = {0, 256, 512, 1024, polar::kMaxN};
  static const uint32_t nb_one[2] = {0, polar::kMaxN};
  const uint32_t* nb = cfg.split_n ? nb_split : nb_one;
  const uint32_t n_nc = cfg.split_n ? 4 : 1;
  auto kernel_of = [&](uint32_t L) -> uint32_t {
    if (L <= 1) return polar::CK_SC;
    if (L <= 4) return polar::CK_W1_L4;
    if (L <= 8) return cfg.l8_kernel;
    return polar::CK_W4_L32;
  };
  // [quant][kernel][n class] -> lds, spill bytes per workgroup
  uint32_t lds[3][4][4] = {};
  uint64_t spill[3][4][4] = {};
  bool used[3][4][4] = {};
  for (polar_plan p : b.plans) {
    const polar::DevPlan& h = p->hp.hdr;
    const uint32_t qt = h.quant;
    const uint32_t k = kernel_of(h.first_stage);
    uint32_t c = 0;
    while (c + 1 < n_nc && h.N > nb[c + 1]) ++c;
    uint32_t need;
    uint64_t gb = 0;
    if (k == polar::CK_SC) {
      need = polar::sc_lds_bytes(h.N, polar::elem_bytes(h.quant));
    } else {
      const polar::LdsLayout lay = polar::lds_layout(h.N, h.n, polar::elem_bytes(h.quant),
                                                     h.first_stage, polar::key_bytes(h.quant));
      need = lay.total;
      gb = lay.gbytes;
    }
    used[qt][k][c] = true;
    lds[qt][k][c] = need > lds[qt][k][c] ? need : lds[qt][k][c];
    spill[qt][k][c] = gb > spill[qt][k][c] ? gb : spill[qt][k][c];
  }
  out->clear();
  const uint32_t n_frames = b.A.n_frames;
  for (uint32_t qt = 0; qt < 3; ++qt)
  for (uint32_t k = 0; k < 4; ++k)
    for (uint32_t c = 0; c < n_nc; ++c) {
      if (!used[qt][k][c]) continue;
      polar::ClassLaunch cl{};
      cl.kernel = k;
      cl.sel.on = 1;
      cl.sel.quant = qt;
      cl.sel.nmin = nb[c] + 1;
      cl.sel.nmax = nb[c + 1];
      if (k == polar::CK_SC) {
        cl.sel.lmin = cl.sel.lmax = 1;
      } else if (k == polar::CK_W1_L4) {
        cl.sel.lmin = 2;
        cl.sel.lmax = 4;
      } else if (k == polar::CK_W2_L8) {
        cl.sel.lmin = 5;
        cl.sel.lmax = 8;
      } else {
        cl.sel.lmin = cfg.l8_kernel == polar::CK_W4_L32 ? 5 : 9;
        cl.sel.lmax = polar::kMaxL;
      }
      cl.lds = lds[qt][k][c];
      cl.spill = spill[qt][k][c];
      if (k == polar::CK_SC)
        cl.grid = n_frames;  // one wave per frame, frames outside the class exit at once
      else
        cl.grid = polar::cap_grid(
            persistent_grid(cus, cl.lds, k == polar::CK_W1_L4 ? 32 : (k == polar::CK_W2_L8 ? 8 : 4),
                            (n_frames + 63) / 64 * 64),
            cl.spill, b.spill_cap);
      out->push_back(cl);
    }
  return out->size() <= polar::kMaxClasses ? POLAR_OK : POLAR_EUNSUP;
}

// Tiered schedule: SC tier if any plan starts at L = 1; list tier A if any
// plan has a stage of list size 2..4; list tier B if any plan has a stage
// above 4 (the stages of a plan: SC {1}, CA {L}, PA {1, L_max}, FA {1, 2, 4,
// ..., L_max}).
int plan_tiers(const Batch& b, polar::TierPlan* out) {
  const uint32_t n_frames = b.A.n_frames;
  polar::TierPlan tp{};
  uint32_t lds_sc = 0;
  for (polar_plan p : b.plans) {
    const polar::DevPlan& h = p->hp.hdr;
    if (h.first_stage == 1) tp.run_sc = true;
    const bool fa = h.algo == POLAR_FA_SCL;
    const bool has_a = (h.first_stage > 1 && h.first_stage <= polar::kTierALmax) ||
                       (h.first_stage == 1 && h.max_list > 1 &&
                        (fa || h.max_list <= polar::kTierALmax));
    if (has_a) tp.run_a = true;
    if (h.max_list > polar::kTierALmax) tp.run_b = true;
    const uint32_t l1 = polar::sc_lds_bytes(h.N, polar::elem_bytes(h.quant));
    lds_sc = l1 > lds_sc ? l1 : lds_sc;
  }
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  const int rc = device_cus(dev, &cus);
  if (rc) return rc;
  const polar::StageSpan sa = polar::stage_span(b, 2, polar::kTierALmax);
  const polar::StageSpan sb =
      polar::stage_span(b, tp.run_a ? polar::kTierALmax + 1 : 2, polar::kMaxL);
  // the SC tier reads the channel LLRs in place (no root in LDS) for a
  // uniform batch of a code that sends all N >= 256 positions, starts with f
  // and has 4-byte aligned frames
  if (!b.A.frames && b.plans.size() == 1) {
    const polar::HostPlan& hp = b.plans[0]->hp;
    const polar::DevPlan& h = hp.hdr;
    if (h.n_punct == 0 && h.n_tx == h.N && h.N >= 256 && !hp.prog.empty() &&
        polar::op_code(hp.prog[0]) == polar::OP_F && (((uintptr_t)b.A.llr) & 3u) == 0 &&
        (b.A.llr_bytes & 3u) == 0) {
      tp.sc_groot = 1;
      lds_sc = polar::sc_lds_bytes(h.N, polar::elem_bytes(h.quant), 1);
      // int8 with 16-byte aligned frames: one frame per lane, a persistent
      // grid of as many waves as a CU holds (at most 16: its registers; its
      // LDS), each with its own region
      if (h.quant == POLAR_I8 && (((uintptr_t)b.A.llr) & 15u) == 0 &&
          (b.A.llr_bytes & 15u) == 0 && b.A.llr_bytes >= h.N) {
        const uint32_t groups = (n_frames + 63) / 64;
        const uint32_t per_cu = polar::kLdsLimit / polar::kScxLds;
        const uint32_t cap = (per_cu < 16u ? per_cu : 16u) * (uint32_t)cus;
        const uint32_t rounds = groups > cap ? (groups + cap - 1) / cap : 1u;
        tp.sc_x = 1;
        tp.spill_sc = polar::scx_region_bytes(h.N);
        tp.grid_scx = polar::cap_grid(groups ? (groups + rounds - 1) / rounds : 1u, tp.spill_sc,
                                      b.spill_cap);
        // the L = 2 stage the same way, when the schedule has one and every
        // REP / SPC node fits the register levels (<= 32 positions)
        const bool fa = h.algo == POLAR_FA_SCL;
        const bool stage2 = h.first_stage == 2 ||
                            (h.first_stage == 1 && h.max_list >= 2 && (fa || h.max_list == 2));
        bool small = true;
        for (uint32_t w : hp.prog) {
          const uint32_t op = polar::op_code(w);
          if ((op == polar::OP_REP || op == polar::OP_SPC) && (h.N >> polar::op_depth(w)) > 32)
            small = false;
        }
        // (waves per CU that its registers allow: 3 per SIMD); the
        // path-per-lane stages below replace it when they cover every list
        // stage of the plan
        const uint32_t cap2 = 12u * (uint32_t)cus;
        // N = 512, 1024 or 2048 with REP / SPC nodes in the register levels:
        // four lanes per frame, the state in registers (waves per SIMD that
        // its registers allow: 2 at N = 2048, 3 below)
        if (small && h.n >= 9 && h.n <= 11) {
          const uint32_t g16 = (n_frames + 15) / 16;
          const uint32_t capq = (h.n <= 10 ? 12u : 8u) * (uint32_t)cus;
          tp.sc_q = h.n;
          tp.n_ops = h.n_sc_ops;  // LDS for the longer program (the lists' is shorter)
          tp.grid_q = g16 < capq ? (g16 ? g16 : 1u) : capq;
        }
        if (stage2 && small) {
          tp.run_x2 = 1;
          tp.spill_x2 = polar::listx_region_bytes(h.N, 2);
          tp.grid_x2 = polar::cap_grid(groups < cap2 ? (groups ? groups : 1u) : cap2, tp.spill_x2,
                                       b.spill_cap);
        }
        // list stages: one path per lane when each of them is 2, 4, 8, 16 or
        // 32 (then also in place of the frame-per-lane L = 2 stage; waves per
        // CU that the registers allow: 4 per SIMD at L <= 8 and 32, 3 at 16)
        uint32_t st = h.first_stage, np = 0, pst[5] = {0, 0, 0, 0, 0};
        bool fits = small;
        for (int guard = 0; guard < 8; ++guard) {
          if (st >= 2) {
            if ((st == 2 || st == 4 || st == 8 || st == 16 || st == 32) && np < 5)
              pst[np++] = st;
            else
              fits = false;
          }
          if (st >= h.L_max && st >= h.first_stage) break;
          st = polar::stage_after(h.algo == POLAR_PA_SCL, h.L_max, st);
        }
        if (fits && np > 0) {
          tp.run_x2 = 0;
          tp.run_p = 1;
          tp.n_p = np;
          tp.spill_p = polar::scx_region_bytes(h.N);
          // the L = 32 stage's short lists: the region in LDS, as many waves
          // per CU as its LDS holds (1 at N = 2048, 2 at N = 1024)
          const uint32_t lds_w = (uint32_t)tp.spill_p + polar::listp_static_lds();
          if (lds_w <= polar::kLdsLimit) {
            tp.lds_pl = (uint32_t)tp.spill_p;
            tp.grid_pl = (polar::kLdsLimit / lds_w) * (uint32_t)cus;
          }
          for (uint32_t i = 0; i < np; ++i) {
            const uint32_t fw = 64u / pst[i];
            const uint32_t need = (n_frames + fw - 1) / fw;
            const uint32_t capp = (pst[i] <= 8 || pst[i] == 32 ? 16u : 12u) * (uint32_t)cus;
            tp.p_stage[i] = pst[i];
            tp.grid_p[i] = polar::cap_grid(need < capp ? (need ? need : 1u) : capp, tp.spill_p,
                                           b.spill_cap);
            if (pst[i] == 32) {
              // lists of up to 3 waves per SIMD: the form with no register bound
              const uint32_t cm = 12u * (uint32_t)cus;
              tp.grid_pm = tp.grid_p[i] < cm ? tp.grid_p[i] : cm;
            }
            // four lanes per path: 16 / L frames per wave, 2 waves per SIMD
            const uint32_t nq = (n_frames + 16u / pst[i] - 1u) / (16u / pst[i] < 1u ? 1u : 16u / pst[i]);
            const uint32_t capq = 8u * (uint32_t)cus;
            tp.grid_ql[i] = nq < capq ? (nq ? nq : 1u) : capq;
          }
        }
      }
    }
  }
  tp.lds_sc = lds_sc;
  tp.grid_sc = n_frames < 0x7FFFFFFFu ? n_frames : 0x7FFFFFFFu;
  tp.lds_a = sa.lds;
  tp.spill_a = sa.spill;
  tp.grid_a = polar::cap_grid(persistent_grid(cus, sa.lds, 32, n_frames), sa.spill, b.spill_cap);
  tp.lds_b = b.lds;
  tp.spill_b = sb.spill;
  tp.grid_b = polar::cap_grid(persistent_grid(cus, b.lds, 8, n_frames), sb.spill, b.spill_cap);
  // frames claimed at a time: about n / (32 workgroups' worth), so that the
  // frames a tier has to decode spread evenly over its workgroups; at most 64
  // (one wave's worth of state words), at least 1
  auto chunk_of = [&](uint32_t grid) {
    const uint64_t c = n_frames / ((uint64_t)(grid ? grid : 1) * 32);
    return (uint32_t)(c < 1 ? 1 : (c > 64 ? 64 : c));
  };
  tp.chunk_a = chunk_of(tp.grid_a);
  tp.chunk_b = chunk_of(tp.grid_b);
  *out = tp;
  return POLAR_OK;
}

// Grid of the plain schedule: one workgroup per frame, or a persistent grid
// (one spill region per workgroup) when a stage spills.
uint32_t plain_grid(const Batch& b, int cus, uint64_t spill) {
  const uint32_t n = b.A.n_frames;
  return spill ? polar::cap_grid(persistent_grid(cus, b.lds, polar::kLdsLimit, n), spill, b.spill_cap)
               : (n < 0x7FFFFFFFu ? n : 0x7FFFFFFFu);
}

const char* kernel_name(uint32_t k) {
  switch (k) {
    case polar::CK_SC: return "sc";
    case polar::CK_W1_L4: return "w1_l4";
    case polar::CK_W2_L8: return "w2_l8";
    default: return "w4_l32";
  }
}

ClassConfig cached_config(const std::vector<polar_plan>& key, bool* found) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_sched.find(key);
  *found = it != g_sched.end();
  return *found ? it->second : ClassConfig{};
}

// The class schedule; with `autotune` and no cached choice, every candidate
// is timed on this batch and the fastest is cached (and its outputs kept).
int run_classes(const Batch& b, const Work& w, hipStream_t st, bool autotune, hipEvent_t ev0,
                hipEvent_t ev1) {
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  int rc = device_cus(dev, &cus);
  if (rc) return rc;
  bool found = false;
  ClassConfig cfg = cached_config(b.plans, &found);
  std::vector<polar::ClassLaunch> cls;
  if (autotune && !found) {
    static const ClassConfig cands[4] = {{polar::CK_W2_L8, 1, true},
                                         {polar::CK_W4_L32, 1, true},
                                         {polar::CK_W2_L8, 0, true},
                                         {polar::CK_W4_L32, 0, true}};
    hipEvent_t e[2] = {nullptr, nullptr};
    if (hipEventCreate(&e[0]) != hipSuccess || hipEventCreate(&e[1]) != hipSuccess) {
      if (e[0]) (void)hipEventDestroy(e[0]);
      return POLAR_EHIP;
    }
    float best = 1e30f;
    uint32_t best_i = 0;
    for (uint32_t i = 0; i < 4 && rc == POLAR_OK; ++i) {
      rc = build_classes(b, cands[i], cus, &cls);
      if (rc) break;
      rc = polar::launch_decode_classes(b.A, cls.data(), (uint32_t)cls.size(), w.heads,
                                        st, e[0], e[1]);
      float ms = 0.f;
      if (rc == POLAR_OK && (hipEventSynchronize(e[1]) != hipSuccess ||
                             hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess))
        rc = POLAR_EHIP;
      if (rc == POLAR_OK && ms < best) {
        best = ms;
        best_i = i;
      }
    }
    (void)hipEventDestroy(e[0]);
    (void)hipEventDestroy(e[1]);
    if (rc) return rc;
    cfg = cands[best_i];
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_sched[b.plans] = cfg;
    }
  }
  rc = build_classes(b, cfg, cus, &cls);
  if (rc) return rc;
  return polar::launch_decode_classes(b.A, cls.data(), (uint32_t)cls.size(), w.heads, st,
                                      ev0, ev1);
}

}  // namespace

namespace polar {

uint64_t spill_need(const Batch& b, int cus) {
  uint64_t need = 0;
  auto upd = [&](uint64_t grid, uint64_t stride) {
    if (grid * stride > need) need = grid * stride;
  };
  TierPlan tp{};
  if (plan_tiers(b, &tp) == POLAR_OK) {
    if (tp.run_sc && tp.sc_x && !tp.sc_q) upd(tp.grid_scx, tp.spill_sc);
    if (tp.run_x2) upd(tp.grid_x2, tp.spill_x2);
    for (uint32_t i = 0; tp.run_p && i < tp.n_p; ++i)
      if (!(tp.sc_q && tp.p_stage[i] <= 16)) upd(tp.grid_p[i], tp.spill_p);
    if (tp.run_a) upd(tp.grid_a, tp.spill_a);
    if (tp.run_b) upd(tp.grid_b, tp.spill_b);
  }
  const uint64_t sp = stage_span(b, 1, kMaxL).spill;
  upd(plain_grid(b, cus, sp), sp);
  if (uses_classes(b, 0)) {
    static const ClassConfig cfgs[4] = {{CK_W2_L8, 1, true},
                                        {CK_W4_L32, 1, true},
                                        {CK_W2_L8, 0, true},
                                        {CK_W4_L32, 0, true}};
    std::vector<ClassLaunch> cls;
    for (const ClassConfig& cfg : cfgs) {
      if (build_classes(b, cfg, cus, &cls) != POLAR_OK) continue;
      for (const ClassLaunch& cl : cls) upd(cl.grid, cl.spill);
    }
  }
  return need;
}

constexpr uint32_t kTinyAdaptive = 32;

// Launch one decode of a prepared batch on `st` with work area `w`.
int launch_batch(const Batch& b_in, uint32_t schedule, const Work& w, hipStream_t st, bool timed,
                 bool autotune) {
  Batch b = b_in;
  polar::KArgs& A = b.A;
  const uint32_t n_frames = A.n_frames;
  hipEvent_t* ev = timed ? timing_events() : nullptr;
  if (timed && !ev) return POLAR_EHIP;
  int rc = POLAR_OK;
  int dev0 = 0, cus0 = 1;
  if (hipGetDevice(&dev0) != hipSuccess) return POLAR_EHIP;
  rc = device_cus(dev0, &cus0);
  if (rc) return rc;
  // spilled layouts: one region per workgroup of each launch (each launch
  // sets its own stride); every launch's grid times stride fits the area
  const uint64_t need = polar::spill_need(b, cus0);
  if (need) {
    if (!w.spill || w.spill_bytes < need) return POLAR_EINVAL;
    A.spill = w.spill;
  }
  // A batch of fewer than kTinyAdaptive frames with an adaptive plan runs
  // the plain form: one launch instead of the tier chain, whose launches
  // would each hold a handful of frames (and one-frame batches once hung in
  // that chain without a cause found).
  if (schedule == 0 && !b.fixed_list && n_frames < kTinyAdaptive) schedule = 1;
  if (schedule == 1) {
    A.spill_stride = polar::stage_span(b, 1, polar::kMaxL).spill;
    const uint32_t grid = plain_grid(b, cus0, A.spill_stride);
    if (ev) (void)hipEventRecord(ev[0], st);
    rc = polar::launch_decode_plain(b.quant, A, b.lds, grid, st);
    if (ev) {
      (void)hipEventRecord(ev[3], st);
      g_timing.plain = true;
      g_timing.classes = false;
      g_timing.valid = rc == POLAR_OK;
    }
    return rc;
  }
  if (schedule != 0) return POLAR_EINVAL;
  if (uses_classes(b, schedule)) {
    rc = run_classes(b, w, st, autotune, ev ? ev[4] : nullptr, ev ? ev[5] : nullptr);
    if (ev) {
      g_timing.plain = false;
      g_timing.classes = true;
      g_timing.valid = rc == POLAR_OK;
    }
    return rc;
  }
  polar::TierPlan tp{};
  rc = plan_tiers(b, &tp);
  if (rc) return rc;
  rc = polar::launch_decode_tiered(b.quant, A, tp, w.state, w.tier_heads, w.xlist, st, ev);
  if (ev) {
    g_timing.ran[0] = tp.run_sc;
    g_timing.ran[1] = tp.run_a;
    g_timing.ran[2] = tp.run_b;
    g_timing.plain = false;
    g_timing.classes = false;
    g_timing.valid = rc == POLAR_OK;
  }
  return rc;
}

}  // namespace

extern "C" {

int polar_scl_decode_batch(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
                           uint32_t n_frames, const void* d_llr, uint32_t* d_info,
                           polar_status* d_status, uint32_t* d_pm_lists,
                           const polar_decode_opts* opts, void* stream) {
  if (!plans || n_plans == 0) return POLAR_EINVAL;
  if (n_frames == 0) {
    for (uint32_t i = 0; i < n_plans; ++i)
      if (!plans[i]) return POLAR_EINVAL;
    return POLAR_OK;
  }
  Batch b;
  int rc = prepare(plans, n_plans, d_frames, n_frames, d_llr, d_info, d_status, d_pm_lists, opts,
                   &b);
  if (rc) return rc;
  const uint32_t schedule = opts ? opts->schedule : 0;
  if (schedule > 1) return POLAR_EINVAL;
  Work w;
  if (schedule == 0) {
    rc = device_scratch(n_frames, &w);
    if (rc) return rc;
  }
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  rc = device_cus(dev, &cus);
  if (rc) return rc;
  rc = device_spill(polar::spill_need(b, cus), &w);
  if (rc) return rc;
  const uint32_t flags = opts ? opts->flags : 0;
  return launch_batch(b, schedule, w, static_cast<hipStream_t>(stream),
                      (flags & POLAR_OPT_TIER_TIMING) != 0, (flags & POLAR_OPT_AUTOTUNE) != 0);
}

int polar_scl_decode_batch_noalloc(const polar_plan* plans, uint32_t n_plans,
                                   const polar_frame* d_frames, uint32_t n_frames,
                                   const void* d_llr, uint32_t* d_info, polar_status* d_status,
                                   uint32_t* d_pm_lists, const polar_decode_opts* opts,
                                   void* stream) {
  if (!plans || n_plans == 0) return POLAR_EINVAL;
  for (uint32_t i = 0; i < n_plans; ++i)
    if (!plans[i]) return POLAR_EINVAL;
  const uint32_t flags = opts ? opts->flags : 0;
  // timing and autotuning create events: not for callers that cannot allocate
  if (flags & (POLAR_OPT_TIER_TIMING | POLAR_OPT_AUTOTUNE)) return POLAR_EINVAL;
  const uint32_t schedule = opts ? opts->schedule : 0;
  if (schedule > 1) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (n_frames > polar::kNoAllocMaxFrames || n_plans > polar::kNoAllocMaxPlans)
    return POLAR_ESCRATCH;
  char* base = nullptr;
  int rc = polar::noalloc_area(&base);
  if (rc) return rc;
  Batch b;
  rc = prepare(plans, n_plans, d_frames, n_frames, d_llr, d_info, d_status, d_pm_lists, opts, &b,
               false);
  if (rc) return rc;
  // area: [plan table (multi-plan batches)] [work area] [spill regions], each 256-byte aligned
  auto up256 = [](uint64_t v) { return (v + 255u) & ~(uint64_t)255u; };
  const uint64_t tab_bytes = n_plans > 1 ? up256((uint64_t)n_plans * sizeof(void*)) : 0;
  const uint64_t work_bytes = up256(polar::work_words(n_frames) * sizeof(uint32_t));
  if (tab_bytes + work_bytes >= polar::kNoAllocBytes) return POLAR_ESCRATCH;
  Work w = work_view(reinterpret_cast<uint32_t*>(base + tab_bytes), n_frames);
  b.spill_cap = polar::kNoAllocBytes - tab_bytes - work_bytes;
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  rc = device_cus(dev, &cus);
  if (rc) return rc;
  // every grid is cut to the spill room; a single region larger than it fails
  const uint64_t need = polar::spill_need(b, cus);
  if (need > b.spill_cap) return POLAR_ESCRATCH;
  if (need) {
    w.spill = base + tab_bytes + work_bytes;
    w.spill_bytes = b.spill_cap;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (n_plans > 1) {
    const void* h[256];
    const polar::DevPlan** tab = reinterpret_cast<const polar::DevPlan**>(base);
    for (uint32_t i = 0; i < n_plans; i += 256) {
      const uint32_t m = n_plans - i < 256 ? n_plans - i : 256;
      for (uint32_t j = 0; j < m; ++j) h[j] = plans[i + j]->d_blob;
      rc = polar::launch_store_ptrs(reinterpret_cast<const void**>(tab + i), h, m, st);
      if (rc) return rc;
    }
    b.A.plans = tab;
  }
  return launch_batch(b, schedule, w, st, false, false);
}

int polar_last_tier_ms(float ms[5]) {
  if (!ms || !g_timing.valid) return POLAR_EINVAL;
  for (int i = 0; i < 5; ++i) ms[i] = 0.f;
  float v = 0.f;
  hipEvent_t* ev = g_timing.ev;
  if (g_timing.classes) {
    if (hipEventSynchronize(ev[5]) != hipSuccess || hipEventElapsedTime(&v, ev[4], ev[5]) != hipSuccess)
      return POLAR_EHIP;
    ms[4] = v;
    return POLAR_OK;
  }
  if (hipEventSynchronize(ev[3]) != hipSuccess) return POLAR_EHIP;
  if (g_timing.plain) {
    if (hipEventElapsedTime(&v, ev[0], ev[3]) != hipSuccess) return POLAR_EHIP;
    ms[3] = v;
    return POLAR_OK;
  }
  for (int i = 0; i < 3; ++i) {
    if (!g_timing.ran[i]) continue;
    if (hipEventElapsedTime(&v, ev[i], ev[i + 1]) != hipSuccess) return POLAR_EHIP;
    ms[i] = v;
  }
  return POLAR_OK;
}

int polar_schedule_describe(const polar_plan* plans, uint32_t n_plans, char* buf, uint32_t len) {
  if (!plans || n_plans == 0 || !buf || len == 0) return POLAR_EINVAL;
  for (uint32_t i = 0; i < n_plans; ++i)
    if (!plans[i]) return POLAR_EINVAL;
  Batch b;
  b.plans.assign(plans, plans + n_plans);
  for (polar_plan p : b.plans) {
    const polar::DevPlan& h = p->hp.hdr;
    if (h.algo != POLAR_SC && h.algo != POLAR_CA_SCL) b.fixed_list = false;
  }
  if (!b.fixed_list || n_plans < 2) return POLAR_EINVAL;
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EHIP;
  int rc = device_cus(dev, &cus);
  if (rc) return rc;
  bool found = false;
  const ClassConfig cfg = cached_config(b.plans, &found);
  b.A.n_frames = 1u << 20;  // grid sizes for a large batch
  std::vector<polar::ClassLaunch> cls;
  rc = build_classes(b, cfg, cus, &cls);
  if (rc) return rc;
  std::string t = "classes=" + std::to_string(cls.size()) +
                  " l8=" + kernel_name(cfg.l8_kernel) + " split_n=" + std::to_string(cfg.split_n) +
                  " tuned=" + std::to_string(found && cfg.tuned ? 1 : 0);
  for (const auto& c : cls)
    t += "; " + std::string(kernel_name(c.kernel)) + " q" + std::to_string(c.sel.quant) + " L" +
         std::to_string(c.sel.lmin) + "-" +
         std::to_string(c.sel.lmax) + " N" + std::to_string(c.sel.nmin) + "-" +
         std::to_string(c.sel.nmax) + " lds=" + std::to_string(c.lds) + " wg=" + std::to_string(c.grid);
  std::snprintf(buf, len, "%s", t.c_str());
  return POLAR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- graphs
struct polar_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t* work = nullptr;
  char* spill = nullptr;
};

extern "C" {

int polar_graph_destroy(polar_graph g) {
  if (!g) return POLAR_OK;
  int rc = POLAR_OK;
  if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) rc = POLAR_EHIP;
  if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) rc = POLAR_EHIP;
  if (g->work && hipFree(g->work) != hipSuccess) rc = POLAR_EHIP;
  if (g->spill && hipFree(g->spill) != hipSuccess) rc = POLAR_EHIP;
  delete g;
  return rc;
}

int polar_graph_create(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
                       uint32_t n_frames, const void* d_llr, uint32_t* d_info,
                       polar_status* d_status, uint32_t* d_pm_lists,
                       const polar_decode_opts* opts, polar_graph* out) {
  if (!out || n_frames == 0) return POLAR_EINVAL;
  *out = nullptr;
  const uint32_t flags = opts ? opts->flags : 0;
  if (flags & (POLAR_OPT_TIER_TIMING | POLAR_OPT_AUTOTUNE)) return POLAR_EINVAL;
  const uint32_t schedule = opts ? opts->schedule : 0;
  if (schedule > 1) return POLAR_EINVAL;
  Batch b;
  int rc = prepare(plans, n_plans, d_frames, n_frames, d_llr, d_info, d_status, d_pm_lists, opts,
                   &b);
  if (rc) return rc;
  polar_graph g = new (std::nothrow) polar_graph_s;
  if (!g) return POLAR_ENOMEM;
  if (hipMalloc(&g->work, work_words(n_frames) * sizeof(uint32_t)) != hipSuccess) {
    delete g;
    return POLAR_ENOMEM;
  }
  Work w = work_view(g->work, n_frames);
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess || device_cus(dev, &cus) != POLAR_OK) {
    (void)polar_graph_destroy(g);
    return POLAR_EHIP;
  }
  const uint64_t sp = polar::spill_need(b, cus);
  if (sp) {
    if (hipMalloc(&g->spill, sp) != hipSuccess) {
      (void)polar_graph_destroy(g);
      return POLAR_ENOMEM;
    }
    w.spill = g->spill;
    w.spill_bytes = sp;
  }
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)polar_graph_destroy(g);
    return POLAR_EHIP;
  }
  rc = POLAR_OK;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = POLAR_EHIP;
  if (rc == POLAR_OK) {
    const int lr = launch_batch(b, schedule, w, s, false, false);
    const hipError_t ec = hipStreamEndCapture(s, &g->graph);
    rc = lr ? lr : (ec == hipSuccess ? POLAR_OK : POLAR_EHIP);
  }
  if (rc == POLAR_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = POLAR_EHIP;
  (void)hipStreamDestroy(s);
  if (rc) {
    (void)polar_graph_destroy(g);
    return rc;
  }
  *out = g;
  return POLAR_OK;
}

int polar_graph_launch(polar_graph g, void* stream) {
  if (!g || !g->exec) return POLAR_EINVAL;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? POLAR_OK
                                                                                   : POLAR_EHIP;
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

int polar_quantize(const float* d_llr, uint32_t n, int32_t quant, int32_t frac_bits, void* d_out,
                   void* stream) {
  if (n && (!d_llr || !d_out)) return POLAR_EINVAL;
  if (quant < POLAR_F32 || quant > POLAR_I8 || frac_bits < 0 || frac_bits > 14) return POLAR_EINVAL;
  return polar::launch_quantize(d_llr, n, (uint32_t)quant, frac_bits, d_out,
                                static_cast<hipStream_t>(stream));
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
    case POLAR_EAGAIN: return "no free serving slot or budget; poll and retry";
    case POLAR_ESCRATCH:
      return "batch exceeds the fixed device area of the allocation-free entry point";
    default: return "unknown error";
  }
}

const char* polar_version(void) { return "polar-scl-gfx950 0.1"; }

}  // extern "C"
