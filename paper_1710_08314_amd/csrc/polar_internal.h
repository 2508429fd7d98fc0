// Internal layout shared by the host planner and the gfx950 kernels of the
// polar SCL decoder: the device plan blob, the node-program encoding and the
// per-frame LDS layout.  Not part of the public C ABI.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define POLAR_HD __host__ __device__
#else
#define POLAR_HD
#endif

namespace polar {

constexpr uint32_t kMaxN = 2048;
constexpr uint32_t kMaxLogN = 11;
constexpr uint32_t kMaxL = 32;
constexpr uint32_t kLdsLimit = 160 * 1024;  // LDS of one gfx950 compute unit

// ---------------------------------------------------------------------------
// Node program: the pre-order walk of the pruned decoding tree (Algorithm 1
// with the dedicated nodes of Sec. II-B3), one 32-bit word per step:
//   bits 0..3   opcode
//   bits 4..7   depth d of the node (node size m = N >> d)
//   bits 8..23  first leaf (u-index) of the node = partial-sum bit offset
// F/G read the node's LLRs at depth d and write its child's at depth d + 1;
// H combines the children's partial sums in place; the node ops read the
// node's LLRs at depth d, update path metrics, fork paths, and write the
// node's partial sums.
// ---------------------------------------------------------------------------
enum Op : uint32_t {
  OP_F = 0,
  OP_G = 1,
  OP_H = 2,
  OP_R0 = 3,
  OP_R1 = 4,
  OP_REP = 5,
  OP_SPC = 6,
  OP_LF = 7,  // frozen leaf
  OP_LI = 8,  // information leaf
  // Fused steps of the L = 1 program (a node program of its own, decoded
  // by the single-path tier): the node's opcode in bits 24..27.
  OP_FN = 9,    // f at depth d, then the left child: a node (size <= 64)
  OP_GNH = 10,  // g at depth d, the right child: a node (size <= 64), then h at d
  // The register stages' program merges an OP_FN and the OP_GNH of the same
  // node that follows it: the left child's opcode in bits 16..19, the right
  // child's in bits 20..23 (in place of the node offset, which those stages
  // do not read), bits 24..31 zero.
  OP_PAIR = 11,
};

POLAR_HD inline uint32_t op_make(uint32_t op, uint32_t d, uint32_t o) {
  return (op & 15u) | ((d & 15u) << 4) | ((o & 0xFFFFu) << 8);
}
POLAR_HD inline uint32_t op_code(uint32_t w) { return w & 15u; }
POLAR_HD inline uint32_t op_depth(uint32_t w) { return (w >> 4) & 15u; }
POLAR_HD inline uint32_t op_off(uint32_t w) { return (w >> 8) & 0xFFFFu; }
POLAR_HD inline uint32_t op_sub(uint32_t w) { return (w >> 24) & 15u; }
POLAR_HD inline uint32_t pair_left(uint32_t w) { return (w >> 16) & 15u; }
POLAR_HD inline uint32_t pair_right(uint32_t w) { return (w >> 20) & 15u; }

// ---------------------------------------------------------------------------
// Device plan blob: a header followed by tables, all 32-bit words, offsets
// in words from the blob start.
// ---------------------------------------------------------------------------
struct DevPlan {
  uint32_t N, n, K, c;                // code length, log2 N, |A|, CRC length
  uint32_t n_tx, k_data, quant, algo;  // sent positions, K - c, polar_quant, polar_algo
  uint32_t L, L_max, n_ops, bw;       // list sizes, program length, bit words per path
  uint32_t info_words, code_words, max_list, lds_max;
  uint32_t off_prog;      // n_ops program words
  uint32_t off_infomask;  // bw words: positions in A
  uint32_t off_datamask;  // bw words: the first K - c positions of A
  uint32_t off_dataprefix;  // bw words: data positions before word w
  uint32_t off_crccol;    // N words: CRC syndrome column of codeword position j
  uint32_t off_crcpos;    // c words: codeword positions of the CRC bits
  uint32_t first_stage;   // list size of the first stage of the schedule
  uint32_t off_crcnib;    // ceil(N/4) x 16 words: XOR of the CRC columns of every
                          // 4-bit pattern at each nibble position of the codeword
  uint32_t n_punct;       // P: codeword positions [0, P) not sent (LLR 0); the sent
                          // positions are [P, P + n_tx)
  uint32_t off_sc_prog;   // n_sc_ops words: the program with fused steps (OP_FN,
  uint32_t n_sc_ops;      // OP_GNH) for the single-path tier
  uint32_t off_datacomp;  // bw x 8 words, for word w: its data mask, the five move
                          // masks that gather the mask's bits to the low end, the
                          // data positions before w and the data positions in w
  uint32_t off_q_prog;    // n_q_ops words: the fused program with OP_PAIR steps
  uint32_t n_q_ops;       // (the register stages)
  uint32_t pad[2];
};
static_assert(sizeof(DevPlan) == 32 * 4, "DevPlan header is 32 words");

POLAR_HD inline const uint32_t* plan_tab(const DevPlan* p, uint32_t off) {
  return reinterpret_cast<const uint32_t*>(p) + off;
}

// ---------------------------------------------------------------------------
// LDS layout of one frame at list size L (element size E bytes, path-metric
// key size KB bytes).  Byte offsets; every region 16-byte aligned.
//   root    N LLRs (channel; shared by every path, never written by f/g)
//   stage d (1..n): L slots of max(N >> d, 1) LLRs, slot padded to 4 bytes;
//           the path of rank r reads depth-d LLRs from slot ptr[d][r] and
//           writes depth d + 1 to its own slot r (index indirection)
//   bits    L x bw words of partial sums, statically owned by rank (copied
//           on fork)
//   ptr     12 x 32 bytes: slot of each (depth, rank)
//   pm      32 path metrics
//   cand    8 L candidate keys;  sel: L sorted keys
//   cpos    L x 4 least-reliable positions (u16) of the current node
//   tabs    12 stage bases + 12 slot strides
//   syn, ord, out, misc
// ---------------------------------------------------------------------------
struct LdsLayout {
  uint32_t root, stages, bits, ptr, pm, cand, sel, cpos, tabs, syn, ord, out, misc, total;
  uint32_t spill;  // S: the slots of depths 1..S live in global memory
  uint32_t groot;  // 1: the root (channel LLRs) lives in global memory too
  // global bytes per workgroup: root (if groot, 16-byte padded), then the
  // slots of depths 1..S
  uint32_t gbytes;
};

// LDS a decoder workgroup may use for its frame (the CU's LDS less room for
// the kernels' static variables).
constexpr uint32_t kLdsBudget = kLdsLimit - 1024;

POLAR_HD inline uint32_t ru16(uint32_t x) { return (x + 15u) & ~15u; }
POLAR_HD inline uint32_t ru4(uint32_t x) { return (x + 3u) & ~3u; }

POLAR_HD inline uint32_t slot_bytes(uint32_t N, uint32_t d, uint32_t E) {
  uint32_t m = N >> d;
  if (m < 1) m = 1;
  return ru4(m * E);
}

POLAR_HD inline LdsLayout lds_layout_s(uint32_t N, uint32_t n, uint32_t E, uint32_t L, uint32_t KB,
                                       uint32_t spill, uint32_t groot = 0) {
  LdsLayout l{};
  l.spill = spill;
  l.groot = groot;
  l.gbytes = groot ? ru16(N * E) : 0u;
  for (uint32_t d = 1; d <= spill; ++d) l.gbytes += L * slot_bytes(N, d, E);
  uint32_t cur = 0;
  l.root = cur;
  if (!groot) cur += ru16(N * E);
  l.stages = cur;
  for (uint32_t d = spill + 1; d <= n; ++d) cur += L * slot_bytes(N, d, E);
  cur = ru16(cur);
  const uint32_t bw = N >= 32 ? N / 32 : 1;
  l.bits = cur;
  cur += ru16(L * bw * 4);
  l.ptr = cur;
  cur += 12 * 32;
  l.pm = cur;
  cur += 32 * 4;
  l.cand = cur;
  cur += ru16(8 * L * KB);
  l.sel = cur;
  cur += ru16(L * KB);
  l.cpos = cur;
  cur += ru16(L * 4 * 2);
  l.tabs = cur;
  cur += 24 * 4;
  l.syn = cur;
  cur += 32 * 4;
  l.ord = cur;
  cur += 32 * 4;
  l.out = cur;
  cur += 64 * 4;
  l.misc = cur;
  cur += 16 * 4;
  l.total = ru16(cur);
  return l;
}

// Spill policy: which LLR buffers of a frame live in a per-workgroup region
// of global memory instead of LDS.  Only a handful of ops (f and g at the
// top depths, a node as large as the code) touch them; moving them out
// multiplies the workgroups a CU holds, which hides the LDS latency chains
// of the list decoder.
//   * Small lists (L <= kSmallListMax) of codes with N >= 1024: the root and
//     the slots of depths 1 and 2.
//   * Large lists: the slots of the top depths, at most kMaxSpill of them
//     (N >= 512), always when the state would not fit a CU's LDS (float32
//     at N = 2048, L = 32 needs 272 KB) and at L >= kSpillMinL whenever it
//     exceeds kLdsTarget.
// Spilled depths hold nodes of at least 64 elements.
constexpr uint32_t kSmallListMax = 4;
constexpr uint32_t kLdsTarget = 32 * 1024;
constexpr uint32_t kSpillMinL = 16;
constexpr uint32_t kMaxSpill = 3;

POLAR_HD inline LdsLayout lds_layout(uint32_t N, uint32_t n, uint32_t E, uint32_t L, uint32_t KB) {
  if (L <= kSmallListMax && N >= 1024) return lds_layout_s(N, n, E, L, KB, 2, 1);
  LdsLayout l = lds_layout_s(N, n, E, L, KB, 0);
  uint32_t s = 0;
  while (s < kMaxSpill && N >= 512 &&
         (l.total > kLdsBudget || (L >= kSpillMinL && l.total > kLdsTarget))) {
    ++s;
    l = lds_layout_s(N, n, E, L, KB, s);
  }
  return l;
}

// LDS layout of the L = 1 tier for one frame: root N LLRs (absent with gr:
// the channel LLRs are then read from global memory), the LLRs of the nodes
// of size >= 128 at depths 1, 2, ... (depth d at root_bytes +
// E (N - N / 2^(d-1))), partial sums (N bits), output staging.
POLAR_HD inline uint32_t sc_root_bytes(uint32_t N, uint32_t E, uint32_t gr = 0) {
  return gr ? 0u : ru16(N * E);
}
POLAR_HD inline uint32_t sc_stage_base(uint32_t N, uint32_t d, uint32_t E, uint32_t gr = 0) {
  return sc_root_bytes(N, E, gr) + E * (N - (N >> (d - 1)));
}
POLAR_HD inline uint32_t sc_bits_off(uint32_t N, uint32_t E, uint32_t gr = 0) {
  return ru16(sc_root_bytes(N, E, gr) + E * N);
}
POLAR_HD inline uint32_t sc_out_off(uint32_t N, uint32_t E, uint32_t gr = 0) {
  return sc_bits_off(N, E, gr) + ru16((N >= 64 ? N / 8 : 8));
}
POLAR_HD inline uint32_t sc_lds_bytes(uint32_t N, uint32_t E, uint32_t gr = 0) {
  return sc_out_off(N, E, gr) + 64 * 4;
}

// List size of the stage after stage L of a schedule (Sec. II-B5): the
// first stage, then L_max (partially adaptive) or 2 L (fully adaptive); the
// last stage is the first with L >= L_max.
POLAR_HD inline uint32_t stage_after(uint32_t algo_pa, uint32_t L_max, uint32_t L) {
  return algo_pa ? L_max : 2 * L;
}

POLAR_HD inline uint32_t elem_bytes(uint32_t quant) { return quant == 0 ? 4u : (quant == 1 ? 2u : 1u); }
POLAR_HD inline uint32_t key_bytes(uint32_t quant) { return quant == 0 ? 8u : 4u; }

}  // namespace polar
