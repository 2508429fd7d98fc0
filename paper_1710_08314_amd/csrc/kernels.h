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
  char* spill;          // nullable: LLR buffers of spilled layouts (lds_layout), one region
  uint64_t spill_stride;  // of spill_stride bytes per workgroup, indexed by blockIdx.x
  uint32_t sc_groot;      // 1: the SC tier reads the channel LLRs from global memory (every
                          // plan sends all N positions, frames 4-byte aligned; no root in LDS)
};

// One generic launch: each workgroup decodes whole frames (every stage of
// the schedule in place).  `lds` = dynamic LDS bytes per workgroup.
int launch_decode_plain(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid,
                        hipStream_t s);

// Tiered schedule.  A per-frame state word holds the list size of each
// frame's next stage, initialised to its plan's first stage; a finished
// frame's word is 0 (list tiers) or stays 1 (SC tier), which no list tier
// takes.  SC tier: two frames per wave (k_sc), or one frame per lane for a
// uniform int8 batch (k_scx), decodes the frames whose plan starts at L = 1.
// List tier A: one wave per frame with the L = 4 footprint, the frames whose
// next stage is 2..4, up to L = 4.  List tier B: several waves per frame
// with the largest footprint, the frames whose next stage is above A's
// range, to the end.  The list tiers are persistent kernels that scan the state words 64 frames at a
// time; a frame that leaves a tier unfinished carries its next stage in its
// state word, so escalation needs no host round trip and no frame list.
constexpr int kListWaves = 4;       // waves per frame in list tier B
constexpr uint32_t kTierALmax = 4;  // largest list size of list tier A

struct TierPlan {
  bool run_sc, run_a, run_b;
  uint32_t lds_sc, lds_a, lds_b, grid_sc, grid_a, grid_b;
  uint32_t chunk_a, chunk_b;  // frames a list-tier workgroup claims at a time (1..64)
  uint64_t spill_a, spill_b;  // spill bytes per workgroup of the list tiers
  uint32_t sc_groot;          // the SC tier reads the channel LLRs from global memory
  uint32_t sc_x;              // the SC tier runs one frame per lane (k_scx)
  uint32_t grid_scx;          // its persistent grid (waves)
  uint64_t spill_sc;          // its region bytes per wave (scx_region_bytes)
  uint32_t run_x2;            // the L = 2 stage runs one frame per lane first (k_listx<2>)
  uint32_t grid_x2;           // its persistent grid (waves)
  uint64_t spill_x2;          // its region bytes per wave (listx_region_bytes)
  uint32_t run_p;             // the list stages (2, 4, 8, 16, 32) run one path per lane
                              // (k_listp) in place of list tiers A and B
  uint32_t p_stage[5], grid_p[5], n_p;  // those stages in order and their grids (waves)
  uint64_t spill_p;           // region bytes per wave (scx_region_bytes)
  uint32_t grid_pl, lds_pl;   // the L = 32 stage's LDS form for short lists: grid (waves)
                              // and region bytes in LDS (0: not used)
  uint32_t grid_pm;           // its unbounded-register form for lists up to one pass
  uint32_t sc_q;              // nonzero: log2 N (9, 10 or 11); the L = 1 stage runs four
                              // lanes per frame, its state in registers (k_rq), in
                              // place of k_scx
  uint32_t grid_q;            // its persistent grid (waves)
  uint32_t n_ops;             // program words of the batch's plan (uniform batches)
  uint32_t grid_ql[5];        // with sc_q: grids of the list stages L <= 16, which then run
                              // four lanes per path (k_rq) in place of k_listp
};
// state: n_frames words; heads: 2 x kClaimSegs claim counters (tier A, then
// tier B), cleared by a kernel launched before the state init.
constexpr uint32_t kClaimSegs = 32;  // claim counters per list tier
// ev (nullable): 4 events recorded before the first tier and after the SC
// tier, list tier A and list tier B.
// xl: the frame list of the frame-per-lane L = 2 stage (n_frames + 1 words).
int launch_decode_tiered(uint32_t quant, const KArgs& A, const TierPlan& tp, uint32_t* state,
                         uint32_t* heads, uint32_t* xl, hipStream_t s, hipEvent_t* ev);

#if defined(__HIPCC__)
// First stage of a frame's schedule (Sec. II-B5) above L_done: the plan's
// first stage if not yet run, else L_max (partially adaptive) or 2 L_done
// (fully adaptive).
__device__ __forceinline__ uint32_t next_stage(const DevPlan* P, uint32_t L_done) {
  if (P->first_stage > L_done) return P->first_stage;
  if (P->algo == POLAR_PA_SCL) return P->L_max;
  return 2 * L_done;
}
#endif

// The SC tier kernel alone (sc.hip); `lds` = sc_lds_bytes of the largest N.
// With `sel` on, the kernel decodes only the frames of its class and skips
// the others (no state); otherwise it decodes the frames of plans that start
// at L = 1 and records their state.
struct ClassSel {
  uint32_t on;
  uint32_t lmin, lmax;  // the plan's first stage (list size) in [lmin, lmax]
  uint32_t nmin, nmax;  // the plan's code length in [nmin, nmax]
  uint32_t quant;       // the plan's LLR type (polar_quant)
};
int launch_decode_sc(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid, uint32_t* state,
                     const ClassSel& sel, hipStream_t s);

// The L = 1 tier with one frame per lane (scx.hip), for a uniform int8
// batch of a code with N >= 256 that sends every position, whose program
// starts with f and whose frames are 16-byte aligned: a persistent grid of
// `grid` waves, each with a region of scx_region_bytes(N) at
// A.spill + blockIdx.x * A.spill_stride.
uint64_t scx_region_bytes(uint32_t N);
constexpr uint32_t kScxLds = 4 * 1024;  // its LDS per wave (level 6)
// The stage of size L = 2 with one frame per lane (scx.hip) for the same
// batches, when the plan's REP and SPC nodes have at most 32 positions:
// a gather kernel lists the frames whose next stage is L in xl (xl[0] =
// count), then a persistent grid of `grid` waves decodes them, each wave
// with a region of listx_region_bytes(N, L) at A.spill + blockIdx.x *
// A.spill_stride.  Finished frames get state 0, the others their next stage.
uint64_t listx_region_bytes(uint32_t N, uint32_t L);
int launch_decode_listx(const KArgs& A, uint32_t grid, uint32_t* state, uint32_t* xl,
                        hipStream_t s);
// The stages of size L = 2, 4, 8, 16, 32 with one path per lane (scx.hip), 64 / L
// frames per wave, for the same batches: the frames whose next stage is L
// are listed in xl as above, then decoded by a persistent grid of `grid`
// waves, each with a region of scx_region_bytes(N).  At L = 32 the list's
// group count picks one of three forms: with grid_lds > 0 and lds > 0, up to
// grid_lds groups go to grid_lds waves whose regions are `lds` bytes of
// dynamic LDS (scx_region_bytes(N) <= lds, lds + listp_static_lds() <= the
// LDS of a CU); then up to grid_mid groups to grid_mid waves with no register
// bound (grid_mid <= grid: their regions are the first grid_mid of the
// global ones); longer lists to the `grid` waves held to 4 per SIMD.
int launch_decode_listp(uint32_t L, const KArgs& A, uint32_t grid, uint32_t grid_mid,
                        uint32_t grid_lds, uint32_t lds, uint32_t* state, uint32_t* xl,
                        hipStream_t s);
uint32_t listp_static_lds();
int listp_set_attributes(uint32_t lds);
int launch_decode_scx(const KArgs& A, uint32_t grid, uint32_t* state, hipStream_t s);
// The L = 1 stage with four lanes per frame and the decoder state in
// registers (rq.hip), for the batches of k_scx with N = 2^nl, nl = 9, 10 or
// 11, whose REP and SPC nodes have at most 32 positions: 16 frames per wave,
// a persistent grid of `grid` waves, no spill region; the plan's program
// (n_ops words) is staged in LDS.
int launch_decode_rq1(uint32_t nl, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                      hipStream_t s);
// The list stage of size L = 2, 4, 8 or 16 the same way (rq.hip), 16 / L
// frames per wave, for the frames whose next stage is L (listed in xl by
// launch_gather first).  Finished frames get state 0, the others their next
// stage.
int launch_decode_rqL(uint32_t nl, uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid,
                      uint32_t* state, uint32_t* xl, hipStream_t s);
// the same per code length (rq9.hip, rq10.hip, rq.hip)
int launch_rq1_n9(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s);
int launch_rq1_n10(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s);
int launch_rq1_n11(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s);
int launch_rqL_n9(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                  uint32_t* xl, hipStream_t s);
int launch_rqL_n10(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                   uint32_t* xl, hipStream_t s);
int launch_rqL_n11(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                   uint32_t* xl, hipStream_t s);
// The frames whose next stage is L, listed in xl (xl[0] = count, then their
// indices in no set order; scx.hip).
int launch_gather(uint32_t n_frames, uint32_t L, const uint32_t* state, uint32_t* xl, hipStream_t s);

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
  uint64_t spill;  // spill bytes per workgroup
};
constexpr uint32_t kMaxClasses = 48;  // 3 quantisations x 4 kernels x 4 code lengths
// heads: one counter per class, cleared by the first kernel of the launch;
// each class is launched for its own quantisation, so one decode may mix
// plans of different LLR types.
int launch_decode_classes(const KArgs& A, const ClassLaunch* cls, uint32_t n_cls, uint32_t* heads,
                          hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end);
// Allow every decoder kernel the whole LDS of a CU (called once, outside any
// graph capture); launches then pass their actual footprint.
int init_kernel_attributes();

// Encoder, data generator and channel (gen.hip).
int launch_encode(const DevPlan* dplan, const DevPlan& h, const uint32_t* d_data,
                  uint32_t* d_code, uint32_t n_frames, hipStream_t s);
int launch_gen_data(const DevPlan& h, uint64_t seed, uint64_t frame0, uint32_t n_frames,
                    uint32_t* d_data, hipStream_t s);
int launch_quantize(const float* d_llr, uint32_t n, uint32_t quant, int32_t frac_bits, void* d_out,
                    hipStream_t s);
int launch_channel(const DevPlan& h, const uint32_t* d_code, uint32_t n_frames, float ebn0_db,
                   int32_t frac_bits, uint64_t seed, uint64_t frame0, void* d_llr, hipStream_t s);

}  // namespace polar
