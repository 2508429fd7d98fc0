// Host-side batch launch shared by the C ABI entry points (capi.cpp) and the
// serving loop (server.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/polar_scl.h"
#include "kernels.h"

namespace polar {

// Work area of one decode: the per-frame state words of the tiered schedule
// (cap words), its list-tier claim counters (kClaimSegs per tier) and the
// per-class claim counters of the class schedule.  Decodes that may run at the same time need
// work areas of their own.
struct Work {
  uint32_t* state = nullptr;
  uint32_t* tier_heads = nullptr;
  uint32_t* heads = nullptr;  // class schedule
  uint32_t* xlist = nullptr;  // count + frame indices of the frame-per-lane L = 2 stage
  char* spill = nullptr;      // LLR buffers of spilled layouts (spill_need bytes)
  uint64_t spill_bytes = 0;
};
size_t work_words(size_t cap);                // words of a work area for `cap` frames
Work work_view(uint32_t* base, size_t cap);  // the regions of an area at `base`

// A validated batch: kernel arguments and what the schedules need.
struct Batch {
  KArgs A{};
  uint32_t quant = 0, lds = 0;
  bool fixed_list = true;  // every plan has one stage (SC or CA-SCL)
  uint64_t spill_cap = 0;  // nonzero: each launch's persistent grid is cut so that its
                           // grid times its spill bytes per workgroup stays within this
  std::vector<polar_plan> plans;
};

// Grid of a launch whose workgroups each own `stride` bytes of spill area,
// cut to what `cap` bytes hold (cap 0: no limit; at least 1).
inline uint32_t cap_grid(uint32_t grid, uint64_t stride, uint64_t cap) {
  if (!cap || !stride) return grid;
  const uint64_t m = cap / stride;
  return m == 0 ? 1u : (grid < m ? grid : (uint32_t)m);
}

// Validate the arguments of polar_scl_decode_batch and fill `b`.  With
// `upload_table` (the default) a multi-plan batch gets the cached device plan
// table of its plan list (uploaded when the list is new, so not under graph
// capture); without it b->A.plans is left null for such a batch and the
// caller provides the table.
int prepare(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
            uint32_t n_frames, const void* d_llr, uint32_t* d_info, polar_status* d_status,
            uint32_t* d_pm_lists, const polar_decode_opts* opts, Batch* b,
            bool upload_table = true);

// The fixed device area of polar_scl_decode_batch_noalloc (noalloc.hip): one
// copy per GPU, held until the process ends.  Laid out per call as the plan
// table (multi-plan batches), the work area, then spill regions.
constexpr uint64_t kNoAllocBytes = 96ull << 20;
constexpr uint32_t kNoAllocMaxFrames = 1u << 21;
constexpr uint32_t kNoAllocMaxPlans = 16384;
// This device's copy of the area (its address is looked up once per device,
// with that device current).
int noalloc_area(char** base);
// Write n device pointers from host memory to dst with kernel launches on s
// (no copy engine, no staging buffer).
int launch_store_ptrs(const void** dst, const void* const* src, uint32_t n, hipStream_t s);

// Largest LDS footprint and spill region per workgroup among the list
// layouts of the batch's stages with list size in [lo, hi].
struct StageSpan {
  uint32_t lds;
  uint64_t spill;
};
StageSpan stage_span(const Batch& b, uint32_t lo, uint32_t hi);

// Global memory the batch's spilled layouts need in a work area (0: none):
// the largest, over every launch any schedule may make for the batch, of
// its grid times its spill bytes per workgroup.
uint64_t spill_need(const Batch& b, int cus);

// Enqueue one decode of `b` on `st` using work area `w` (schedule 0 automatic,
// 1 plain; `timed`: tier events of this host thread; `autotune`: see
// POLAR_OPT_AUTOTUNE).
int launch_batch(const Batch& b, uint32_t schedule, const Work& w, hipStream_t st, bool timed,
                 bool autotune);

}  // namespace polar
