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
  std::vector<polar_plan> plans;
};

// Validate the arguments of polar_scl_decode_batch and fill `b` (uploads the
// device plan table of a new plan list, so not under graph capture).
int prepare(const polar_plan* plans, uint32_t n_plans, const polar_frame* d_frames,
            uint32_t n_frames, const void* d_llr, uint32_t* d_info, polar_status* d_status,
            uint32_t* d_pm_lists, const polar_decode_opts* opts, Batch* b);

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
