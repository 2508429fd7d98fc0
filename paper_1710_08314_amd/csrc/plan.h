// Host planner interface (see plan.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/polar_scl.h"
#include "polar_internal.h"

namespace polar {

struct NodeCounts {
  uint32_t r0 = 0, r1 = 0, rep = 0, spc = 0, leaf_f = 0, leaf_i = 0;
};

struct HostPlan {
  polar_plan_desc desc{};        // copy of the descriptor (frozen pointer cleared)
  DevPlan hdr{};                 // header as uploaded
  std::vector<uint32_t> blob;    // header + tables (32-bit words)
  std::vector<uint32_t> prog;    // node program
  std::vector<uint32_t> sc_prog;  // node program with fused steps (single-path tier)
  std::vector<uint32_t> q_prog;   // the same with OP_PAIR steps (register stages)
  std::vector<uint32_t> frozen;  // frozen mask, bw words
  NodeCounts counts;
};

// log-domain Bhattacharyya parameters of the 2^n channels from log Z0.
std::vector<double> bhattacharyya_log(uint32_t n, double lz0);

// Validate the descriptor and build every plan table.  Returns POLAR_OK or
// a negative POLAR_E* code.
int make_plan(const polar_plan_desc& d, HostPlan& hp);

// Algorithmic element operations of one decoding stage at list size L.
uint64_t stage_work(const HostPlan& hp, uint32_t L);

// LDS bytes of one frame of this plan at list size L.
uint32_t plan_lds_bytes(const DevPlan& h, uint32_t L);

}  // namespace polar
