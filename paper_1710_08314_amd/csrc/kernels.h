// Kernel arguments and launchers (device side in decode.hip / gen.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/polar_scl.h"
#include "polar_internal.h"

namespace polar {

struct KArgs {
  const DevPlan* const* plans;  // device array of device plan blobs
  const polar_frame* frames;    // NULL: uniform batch of plans[0]
  uint32_t n_frames;
  const char* llr;
  uint32_t llr_bytes;   // uniform batch: bytes per frame
  uint32_t info_words;  // uniform batch: output words per frame
  uint32_t* info;
  polar_status* status;
  uint32_t* pm_lists;   // nullable
  uint32_t pm_stride;   // entries per frame in pm_lists
  uint64_t* times;      // nullable: realtime stamps, start and end per frame
};

// One generic launch: each workgroup decodes whole frames (every stage of
// the schedule in place).  `lds` = dynamic LDS bytes per workgroup.
int launch_decode_plain(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid,
                        hipStream_t s);

// Tiered schedule.  SC tier: one wave per frame with the L = 1 footprint,
// pushing the CRC failures of adaptive plans (and untouched fixed-list
// frames) to queue 1.  List tier A: one wave per frame with the L = 4
// footprint, stages of L <= 4, failures to queue 2.  List tier B: several
// waves per frame with the largest footprint, the remaining stages.  Each
// tier's kernel is persistent and drains its input queue; a tier whose
// predecessors did not run takes every frame directly.
constexpr int kListWaves = 4;       // waves per frame in list tier B
constexpr uint32_t kTierALmax = 4;  // largest list size of list tier A

struct TierPlan {
  bool run_sc, run_a, run_b;
  uint32_t lds_sc, lds_a, lds_b, grid_sc, grid_a, grid_b;
};
// ev (nullable): 4 events recorded before the first tier and after the SC
// tier, list tier A and list tier B.
int launch_decode_tiered(uint32_t quant, const KArgs& A, const TierPlan& tp, uint32_t* q1,
                         uint32_t* q2, hipStream_t s, hipEvent_t* ev);
// The SC tier kernel alone (sc.hip); `lds` = sc_lds_bytes of the largest N.
// With `sel` on, the kernel decodes only the frames of its class and skips
// the others (no queue); otherwise frames of plans whose first stage is not
// L = 1 are queued untouched.
struct ClassSel {
  uint32_t on;
  uint32_t lmin, lmax;  // the plan's first stage (list size) in [lmin, lmax]
  uint32_t nmin, nmax;  // the plan's code length in [nmin, nmax]
};
int launch_decode_sc(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid, uint32_t* queue,
                     const ClassSel& sel, hipStream_t s);

// Class schedule of a batch of fixed-list plans (no escalation): the frames
// are split into classes by list size and code length, and each class is
// decoded by its own persistent kernel that walks the frame descriptors,
// picks the frames of its class and runs their single stage.  No frame is
// handed between kernels.  Kernel variants (waves per frame, largest list):
enum ClassKernel : uint32_t {
  CK_SC = 0,      // k_sc: L = 1, one wave per frame
  CK_W1_L4 = 1,   // one wave, L <= 4
  CK_W2_L8 = 2,   // two waves, L <= 8
  CK_W4_L32 = 3,  // four waves, L <= 32
};
struct ClassLaunch {
  uint32_t kernel;  // ClassKernel
  ClassSel sel;
  uint32_t lds, grid;
};
constexpr uint32_t kMaxClasses = 16;
// heads: one counter per class, cleared by the first kernel of the launch.
int launch_decode_classes(uint32_t quant, const KArgs& A, const ClassLaunch* cls, uint32_t n_cls,
                          uint32_t* heads, hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end);
// Allow every decoder kernel the whole LDS of a CU (called once, outside any
// graph capture); launches then pass their actual footprint.
int init_kernel_attributes();

// Encoder, data generator and channel (gen.hip).
int launch_encode(const DevPlan* dplan, const DevPlan& h, const uint32_t* d_data,
                  uint32_t* d_code, uint32_t n_frames, hipStream_t s);
int launch_gen_data(const DevPlan& h, uint64_t seed, uint64_t frame0, uint32_t n_frames,
                    uint32_t* d_data, hipStream_t s);
int launch_channel(const DevPlan& h, const uint32_t* d_code, uint32_t n_frames, float ebn0_db,
                   int32_t frac_bits, uint64_t seed, uint64_t frame0, void* d_llr, hipStream_t s);

}  // namespace polar
