// The decoder's stages for uniform int8 batches on gfx950, with the lanes of
// a wave spread over frames (L = 1) or over the paths of a list:
//   * k_scx: the L = 1 stage, successive cancellation over the pruned tree
//     (Sec. II-B1, II-B3) with the CRC check of the adaptive schedules
//     (Sec. II-B5), one frame per lane;
//   * k_listx<L>: a list stage with a frame's L paths in one lane (kept for
//     L = 2 where the path-per-lane stages do not apply);
//   * k_listp<L>: a list stage (L = 2 .. 32) with one path per lane and
//     64 / L frames per wave;
//   * k_gather: the list of frames whose next stage is L.
// This comment describes the L = 1 kernel; each list kernel has its own.
//
// Every frame of a uniform batch runs the same node program, and a list of
// one path takes the same steps whatever the LLRs are, so a wave decodes 64
// frames in lockstep: the program walk, its dispatch and every loop bound
// are scalar, and every lane of every vector instruction does a frame's
// arithmetic: the inter-frame use of SIMD that Sec. IV-A sets against the
// intra-frame one, which leaves most lanes idle near the leaves.  The
// frame-per-half tier (sc.hip) decodes everything else.
//
// Per lane (frame):
//   * the LLRs of the current node at each level k <= 5 (at most 32 of
//     them) live in registers, packed four int8 per 32-bit word;
//   * the LLRs of the current node of level 6 live in LDS, those of each
//     level 7 <= k < n in a per-wave region of global memory; both hold
//     16-byte chunks interleaved over the 64 lanes (chunk c of lane l at
//     16 (64 c + l)), so every access of the wave is one contiguous
//     kilobyte (conflict-free in LDS);
//   * the root is the channel LLR buffer itself (frame-major);
//   * partial sums of levels >= 6 are N bits per frame in the same region,
//     word w of lane l at 4 (64 w + l); those of a node of level <= 5 stay in
//     a register until its parent consumes them.
// The decisions are those of the frame-per-half tier and of a list of one
// under the list decoder's selection rule: the hard decision wins a tie, the
// all-zero REP candidate wins a tie, SPC flips the first least reliable
// position; integer metrics stay 0 at L = 1, so only the REP decision needs
// its (saturated) penalties.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/polar_scl.h"
#include "device_common.h"
#include "kernels.h"
#include "polar_internal.h"

namespace polar {

namespace {

constexpr int kQ = VT<int8_t>::Q;  // saturation of the int8 LLRs

struct Chunk {
  uint32_t w[4];  // 16 packed LLRs
};
__device__ __forceinline__ Chunk ldc(const char* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return Chunk{{v.x, v.y, v.z, v.w}};
}
__device__ __forceinline__ void stc(char* p, const Chunk& c) {
  *reinterpret_cast<uint4*>(p) = make_uint4(c.w[0], c.w[1], c.w[2], c.w[3]);
}
__device__ __forceinline__ uint32_t hd16(const Chunk& c) {
  return hd4(c.w[0]) | (hd4(c.w[1]) << 4) | (hd4(c.w[2]) << 8) | (hd4(c.w[3]) << 12);
}

// --------------------------------------------------------- register levels
struct XR {
  uint32_t x5[8], x4[4], x3[2], x2, x1, x0;  // LLRs of the current nodes of levels 5..0
  uint32_t b;    // partial sums of the last finished node of level <= 5 (2^k bits)
  uint32_t lft;  // left-child partial sums of the split nodes of levels 1..5: those of
                 // level K (2^(K-1) bits) at bit 2^(K-1) - 1
  uint32_t l6;   // left-child partial sums of the split node of level 6
};

// words of level K (K <= 5): element i in word i / 4, byte i % 4
template <int K>
__device__ __forceinline__ uint32_t& xw(XR& R, int j) {
  if constexpr (K == 5) return R.x5[j];
  else if constexpr (K == 4) return R.x4[j];
  else if constexpr (K == 3) return R.x3[j];
  else if constexpr (K == 2) return R.x2;
  else if constexpr (K == 1) return R.x1;
  else return R.x0;
}

// f (G = false) or g (G = true) of a split node of level K in 1..5: the
// child (level K - 1) gets element i from elements i and i + 2^(K-1)
template <int K, bool G>
__device__ __forceinline__ void reg_fg(XR& R) {
  constexpr uint32_t h = 1u << (K - 1);
  if constexpr (G) {
    const uint32_t hm = (1u << h) - 1u;
    R.lft = (R.lft & ~(hm << (h - 1))) | ((R.b & hm) << (h - 1));
  }
  if constexpr (K >= 3) {
    constexpr int W = (int)h / 4;  // words of the child
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const uint32_t a = xw<K>(R, j), c = xw<K>(R, j + W);
      xw<K - 1>(R, j) = G ? g4(a, c, (R.b >> (4 * j)) & 15u) : f4(a, c);
    }
  } else {
    // K = 2: bytes 0, 1 against 2, 3; K = 1: byte 0 against byte 1
    const uint32_t a = xw<K>(R, 0), c = a >> (8 * h);
    const uint32_t keep = (1u << (8 * h)) - 1u;
    xw<K - 1>(R, 0) = (G ? g4(a, c, R.b & ((1u << h) - 1u)) : f4(a, c)) & keep;
  }
}

// h of a split node of level K in 1..5: beta = [left ^ right, right]
template <int K>
__device__ __forceinline__ void reg_h(XR& R) {
  constexpr uint32_t h = 1u << (K - 1);
  const uint32_t left = (R.lft >> (h - 1)) & ((1u << h) - 1u);
  R.b = (left ^ R.b) | (R.b << h);
}

// a dedicated node or leaf of level K <= 5
template <int K>
__device__ __forceinline__ void reg_node(XR& R, uint32_t opc) {
  constexpr uint32_t M = 1u << K;
  constexpr int W = M >= 4 ? (int)M / 4 : 1;
  constexpr uint32_t full = M == 32 ? 0xFFFFFFFFu : ((1u << (M & 31u)) - 1u);
  if (opc == OP_R0 || opc == OP_LF) {
    R.b = 0u;
    return;
  }
  uint32_t hd = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) hd |= hd4(xw<K>(R, j)) << (4 * j);
  hd &= full;
  if (opc == OP_R1 || opc == OP_LI) {
    R.b = hd;
    return;
  }
  if (opc == OP_REP) {
    int p0 = 0, p1 = 0;
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * j + i < (int)M) {
          const int v = sx8(xw<K>(R, j), i);
          if (v < 0)
            p0 -= v;
          else
            p1 += v;
        }
    R.b = min(p1, kQ) < min(p0, kQ) ? full : 0u;
    return;
  }
  // SPC: odd parity flips the least reliable position (smallest index on ties)
  if (__popc(hd) & 1u) {
    uint32_t key = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * j + i < (int)M) {
          const uint32_t kk = ((uint32_t)abs(sx8(xw<K>(R, j), i)) << 6) | (uint32_t)(4 * j + i);
          key = min(key, kk);
        }
    hd ^= 1u << (key & 63u);
  }
  R.b = hd;
}

// ---------------------------------------------------------- memory levels
// The current node of level k >= 7: its LLRs are the channel LLRs (k = n:
// lane base llr + N f, chunk stride 16) or level k's buffer (lane base
// buf_k + 16 l, chunk stride 1024).
struct Src {
  const char* p;
  uint32_t cs;
};

struct Ctx {
  char* region;       // this wave's region
  const char* root;   // this lane's channel LLRs
  uint32_t n, lane;
  uint32_t* bits;     // partial-sum words of this lane: word w at bits[64 w]
  uint4* l6;          // this lane's level-6 chunks in LDS: chunk c at l6[64 c]
};

__device__ __forceinline__ char* level_buf(const Ctx& C, uint32_t k) {
  // levels 7 .. n-1, level k at 64 (2^k - 128) bytes
  return C.region + (size_t)64u * ((1u << k) - 128u);
}
// chunk c of a lane's LDS buffer whose chunk 0 is at p
__device__ __forceinline__ Chunk ldl(const uint4* p, uint32_t c) {
  const uint4 v = p[64u * c];
  return Chunk{{v.x, v.y, v.z, v.w}};
}
__device__ __forceinline__ void stl(uint4* p, uint32_t c, const Chunk& x) {
  p[64u * c] = make_uint4(x.w[0], x.w[1], x.w[2], x.w[3]);
}
__device__ __forceinline__ Chunk ld6(const Ctx& C, uint32_t c) { return ldl(C.l6, c); }
__device__ __forceinline__ Src src_of(const Ctx& C, uint32_t k) {
  if (k == C.n) return Src{C.root, 16u};
  return Src{level_buf(C, k) + 16u * C.lane, 1024u};
}

// f / g of a split node of level k >= 7 (child level k - 1 >= 6: LDS for
// k = 7 (L6), global memory above)
template <bool G, bool L6>
__device__ __forceinline__ void mem_fg(const Ctx& C, uint32_t k, uint32_t o) {
  const Src s = src_of(C, k);
  const uint32_t nc = 1u << (k - 5);  // chunks of the child (h / 16)
  const char* pa = s.p;
  const char* pb = s.p + (size_t)nc * s.cs;
  char* dst = L6 ? nullptr : level_buf(C, k - 1) + 16u * C.lane;
  const uint32_t* lb = C.bits + (size_t)64u * (o >> 5);
  for (uint32_t c = 0; c < nc; c += 2) {
    const Chunk a0 = ldc(pa + (size_t)c * s.cs), b0 = ldc(pb + (size_t)c * s.cs);
    const Chunk a1 = ldc(pa + (size_t)(c + 1) * s.cs), b1 = ldc(pb + (size_t)(c + 1) * s.cs);
    Chunk r0, r1;
    if constexpr (G) {
      const uint32_t sw = lb[64u * (c >> 1)];  // left partial sums of elements 16c .. 16c+31
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = g4(a0.w[j], b0.w[j], (sw >> (4 * j)) & 15u);
        r1.w[j] = g4(a1.w[j], b1.w[j], (sw >> (16 + 4 * j)) & 15u);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = f4(a0.w[j], b0.w[j]);
        r1.w[j] = f4(a1.w[j], b1.w[j]);
      }
    }
    if constexpr (L6) {
      C.l6[64u * c] = make_uint4(r0.w[0], r0.w[1], r0.w[2], r0.w[3]);
      C.l6[64u * (c + 1)] = make_uint4(r1.w[0], r1.w[1], r1.w[2], r1.w[3]);
    } else {
      stc(dst + (size_t)c * 1024u, r0);
      stc(dst + (size_t)(c + 1) * 1024u, r1);
    }
  }
}

// f / g of a split node of level 6: the child (level 5) goes to registers
template <bool G>
__device__ __forceinline__ void mem_fg6(const Ctx& C, XR& R) {
  const Chunk a0 = ld6(C, 0), a1 = ld6(C, 1), b0 = ld6(C, 2), b1 = ld6(C, 3);
  if constexpr (G) R.l6 = R.b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (G) {
      R.x5[j] = g4(a0.w[j], b0.w[j], (R.b >> (4 * j)) & 15u);
      R.x5[j + 4] = g4(a1.w[j], b1.w[j], (R.b >> (16 + 4 * j)) & 15u);
    } else {
      R.x5[j] = f4(a0.w[j], b0.w[j]);
      R.x5[j + 4] = f4(a1.w[j], b1.w[j]);
    }
  }
}

// h of a split node of level k >= 6 at leaf offset o
__device__ __forceinline__ void mem_h(const Ctx& C, XR& R, uint32_t k, uint32_t o) {
  uint32_t* w = C.bits + (size_t)64u * (o >> 5);
  if (k == 6) {
    w[0] = R.l6 ^ R.b;
    w[64] = R.b;
    return;
  }
  const uint32_t nw = 1u << (k - 6);  // words of each half
  uint32_t* r = w + (size_t)64u * nw;
  for (uint32_t q = 0; q < nw; ++q) w[64u * q] ^= r[64u * q];
}

// a dedicated node of level k >= 6 at leaf offset o; rd(c) reads chunk c of
// its LLRs
template <class RD>
__device__ __forceinline__ void mem_node_t(const Ctx& C, uint32_t opc, uint32_t k, uint32_t o,
                                           const RD& rd) {
  uint32_t* w = C.bits + (size_t)64u * (o >> 5);
  const uint32_t nw = 1u << (k - 5);  // 32-bit words of partial sums
  if (opc == OP_R0) {
    for (uint32_t q = 0; q < nw; ++q) w[64u * q] = 0u;
    return;
  }
  if (opc == OP_REP) {
    int p0 = 0, p1 = 0;
    for (uint32_t c = 0; c < 2 * nw; ++c) {
      const Chunk x = rd(c);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int v = sx8(x.w[j], i);
          if (v < 0)
            p0 -= v;
          else
            p1 += v;
        }
    }
    const uint32_t v = min(p1, kQ) < min(p0, kQ) ? 0xFFFFFFFFu : 0u;
    for (uint32_t q = 0; q < nw; ++q) w[64u * q] = v;
    return;
  }
  // R1 / SPC: hard decisions, word q from chunks 2q, 2q + 1
  uint32_t par = 0, key = 0xFFFFFFFFu;
  for (uint32_t q = 0; q < nw; ++q) {
    const Chunk x0 = rd(2 * q), x1 = rd(2 * q + 1);
    const uint32_t hw = hd16(x0) | (hd16(x1) << 16);
    w[64u * q] = hw;
    if (opc == OP_SPC) {
      par ^= hw;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t e = 32u * q + 4u * j + i;
          key = min(key, ((uint32_t)abs(sx8(x0.w[j], i)) << 12) | e);
          key = min(key, ((uint32_t)abs(sx8(x1.w[j], i)) << 12) | (e + 16u));
        }
    }
  }
  if (opc == OP_SPC && (__popc(par) & 1u)) {
    const uint32_t e = key & 0xFFFu;
    w[64u * (e >> 5)] ^= 1u << (e & 31u);
  }
}
__device__ __forceinline__ void mem_node(const Ctx& C, uint32_t opc, uint32_t k, uint32_t o) {
  if (k == 6) {
    mem_node_t(C, opc, k, o, [&](uint32_t c) { return ld6(C, c); });
  } else {
    const Src s = src_of(C, k);
    mem_node_t(C, opc, k, o, [&](uint32_t c) { return ldc(s.p + (size_t)c * s.cs); });
  }
}

// ------------------------------------------------------- the op dispatch
__device__ __forceinline__ void reg_op(XR& R, uint32_t opc, uint32_t k) {
  // split-node steps of levels 1..5 and nodes of levels 0..5
  if (opc == OP_F || opc == OP_G || opc == OP_H) {
    const bool g = opc == OP_G;
    if (opc == OP_H) {
      switch (k) {
        case 5: reg_h<5>(R); break;
        case 4: reg_h<4>(R); break;
        case 3: reg_h<3>(R); break;
        case 2: reg_h<2>(R); break;
        default: reg_h<1>(R); break;
      }
      return;
    }
    switch (k) {
      case 5: g ? reg_fg<5, true>(R) : reg_fg<5, false>(R); break;
      case 4: g ? reg_fg<4, true>(R) : reg_fg<4, false>(R); break;
      case 3: g ? reg_fg<3, true>(R) : reg_fg<3, false>(R); break;
      case 2: g ? reg_fg<2, true>(R) : reg_fg<2, false>(R); break;
      default: g ? reg_fg<1, true>(R) : reg_fg<1, false>(R); break;
    }
    return;
  }
  switch (k) {
    case 5: reg_node<5>(R, opc); break;
    case 4: reg_node<4>(R, opc); break;
    case 3: reg_node<3>(R, opc); break;
    case 2: reg_node<2>(R, opc); break;
    case 1: reg_node<1>(R, opc); break;
    default: reg_node<0>(R, opc); break;
  }
}

// ===================================================== L = 2: one frame per lane
// A list stage of size L (Algorithm 1 with the dedicated nodes of Sec.
// II-B3 and the selection of Sec. II-B2) for the frames of a uniform int8
// batch whose next stage is L; written for L <= 4, launched for L = 2.  Each lane holds its frame's L paths;
// the number of active paths grows the same way in every frame (a <-
// min(L, a C) at a node with C candidates per path), so it is scalar.
//   * Register levels (<= 32 positions) per path, as in the L = 1 kernel.
//   * Levels >= 6: L slots per level (LDS for level 6, the wave's region
//     above); the path of rank r reads its node from the slot its slot bit
//     names and writes its child to slot r (index indirection: a fork copies
//     no LLRs).
//   * Partial sums of levels >= 6: one N-bit array per path in the region,
//     copied from the parent when a selection moves a path.
// Candidates follow the list decoder: a leaf or REP node offers 0 and 1, a
// Rate-1 node the Chase-2 flips of its two least reliable positions, an SPC
// node the flips of its four least reliable positions whose weight has the
// parity of the hard decisions; a candidate's metric is the parent's plus
// the flipped magnitudes, saturated at Q; the L smallest keys (metric,
// parent, local index) survive and metrics are normalised to the best.
// The caller admits plans whose REP and SPC nodes fit in registers.

template <int L>
struct PS {  // the paths of a lane
  XR R[L];
  int pm[L];
  uint32_t P[L];  // slot of each level k >= 6 of the path's buffers: 2 bits at 2 (k - 6)
};

template <int L>
struct CtxL {
  char* region;      // this wave's region
  const char* root;  // this lane's channel LLRs
  uint32_t n, lane;
  uint32_t* bits[L];  // partial-sum words of path r: word w at bits[r][64 w]
  uint4* l6[L];       // LDS slot s of level 6 for this lane: chunk c at l6[s][64 c]
};

// level k in 7 .. n-1: L slots of 64 2^k bytes, at 64 L (2^k - 128)
template <int L>
__device__ __forceinline__ char* lbuf(const CtxL<L>& C, uint32_t k, uint32_t s) {
  return C.region + (size_t)(64u * L) * ((1u << k) - 128u) + (size_t)s * (64u << k) + 16u * C.lane;
}
__device__ __forceinline__ uint32_t slot_of(uint32_t Pr, uint32_t k) { return (Pr >> (2 * (k - 6))) & 3u; }
__device__ __forceinline__ uint32_t set_slot(uint32_t Pr, uint32_t k, uint32_t r) {
  return (Pr & ~(3u << (2 * (k - 6)))) | (r << (2 * (k - 6)));
}
// the node of level k >= 7 of a path with slot bits Pr
template <int L>
__device__ __forceinline__ Src srcL(const CtxL<L>& C, uint32_t Pr, uint32_t k) {
  if (k == C.n) return Src{C.root, 16u};
  return Src{lbuf<L>(C, k, slot_of(Pr, k)), 1024u};
}
template <int L>
__device__ __forceinline__ const uint4* l6of(const CtxL<L>& C, uint32_t Pr) {
  const uint32_t s = slot_of(Pr, 6);
  const uint4* p = C.l6[0];
#pragma unroll
  for (int i = 1; i < L; ++i) p = s == (uint32_t)i ? C.l6[i] : p;
  return p;
}

// f / g of path r's split node of level k >= 7 into its own slot of level k - 1
template <int L, bool G, bool DL>
__device__ __forceinline__ void fgL(const CtxL<L>& C, uint32_t Pr, uint32_t r, uint32_t k,
                                    uint32_t o) {
  const Src s = srcL<L>(C, Pr, k);
  const uint32_t nc = 1u << (k - 5);
  const char* pa = s.p;
  const char* pb = s.p + (size_t)nc * s.cs;
  char* dst = DL ? nullptr : lbuf<L>(C, k - 1, r);
  uint4* dl = C.l6[r];
  const uint32_t* lb = C.bits[r] + (size_t)64u * (o >> 5);
  for (uint32_t c = 0; c < nc; c += 2) {
    const Chunk a0 = ldc(pa + (size_t)c * s.cs), b0 = ldc(pb + (size_t)c * s.cs);
    const Chunk a1 = ldc(pa + (size_t)(c + 1) * s.cs), b1 = ldc(pb + (size_t)(c + 1) * s.cs);
    Chunk r0, r1;
    if constexpr (G) {
      const uint32_t sw = lb[64u * (c >> 1)];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = g4(a0.w[j], b0.w[j], (sw >> (4 * j)) & 15u);
        r1.w[j] = g4(a1.w[j], b1.w[j], (sw >> (16 + 4 * j)) & 15u);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = f4(a0.w[j], b0.w[j]);
        r1.w[j] = f4(a1.w[j], b1.w[j]);
      }
    }
    if constexpr (DL) {
      stl(dl, c, r0);
      stl(dl, c + 1, r1);
    } else {
      stc(dst + (size_t)c * 1024u, r0);
      stc(dst + (size_t)(c + 1) * 1024u, r1);
    }
  }
}

// f / g of a path's split node of level 6 into its level-5 registers
template <int L, bool G>
__device__ __forceinline__ void fg6L(const CtxL<L>& C, uint32_t Pr, XR& R) {
  const uint4* l = l6of<L>(C, Pr);
  const Chunk a0 = ldl(l, 0), a1 = ldl(l, 1), b0 = ldl(l, 2), b1 = ldl(l, 3);
  if constexpr (G) R.l6 = R.b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (G) {
      R.x5[j] = g4(a0.w[j], b0.w[j], (R.b >> (4 * j)) & 15u);
      R.x5[j + 4] = g4(a1.w[j], b1.w[j], (R.b >> (16 + 4 * j)) & 15u);
    } else {
      R.x5[j] = f4(a0.w[j], b0.w[j]);
      R.x5[j + 4] = f4(a1.w[j], b1.w[j]);
    }
  }
}

// h of path r's split node of level k >= 6
template <int L>
__device__ __forceinline__ void hL(const CtxL<L>& C, uint32_t r, const XR& R, uint32_t k,
                                   uint32_t o) {
  uint32_t* w = C.bits[r] + (size_t)64u * (o >> 5);
  if (k == 6) {
    w[0] = R.l6 ^ R.b;
    w[64] = R.b;
    return;
  }
  const uint32_t nw = 1u << (k - 6);
  uint32_t* q = w + (size_t)64u * nw;
  for (uint32_t i = 0; i < nw; ++i) w[64u * i] ^= q[64u * i];
}

// keep the L smallest keys, ascending
template <int L>
__device__ __forceinline__ void insL(uint32_t key, uint32_t (&kk)[L]) {
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const uint32_t lo = min(key, kk[t]);
    key = max(key, kk[t]);
    kk[t] = lo;
  }
}
__device__ __forceinline__ uint32_t ckey(int pm, uint32_t pen, uint32_t r, uint32_t local) {
  const int v = min(pm + (int)pen, kQ);
  return ((uint32_t)v << 8) | (r << 4) | local;
}
template <int L>
__device__ __forceinline__ void normalise(PS<L>& S, uint32_t a) {
  int mn = S.pm[0];
#pragma unroll
  for (int r = 1; r < L; ++r)
    if ((uint32_t)r < a) mn = min(mn, S.pm[r]);
#pragma unroll
  for (int r = 0; r < L; ++r) S.pm[r] -= mn;
}
// element i of a small per-path array by a lane-varying index
template <int L, class V>
__device__ __forceinline__ V pick(const V (&v)[L], uint32_t i) {
  V x = v[0];
#pragma unroll
  for (int t = 1; t < L; ++t) x = i == (uint32_t)t ? v[t] : x;
  return x;
}

// The survivors (keys kk[0 .. keep)) replace the paths: registers, metrics
// and slot bits from their parents, and the partial-sum words [0, W) of
// levels >= 6 copied where a path's parent is another rank.
template <int L>
__device__ __forceinline__ void take(PS<L>& S, const CtxL<L>& C, const uint32_t (&kk)[L],
                                     uint32_t keep, uint32_t W) {
  uint32_t p[L];
  bool moved = false;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    p[j] = (uint32_t)j < keep ? (kk[j] >> 4) & 3u : (uint32_t)j;
    moved = moved || p[j] != (uint32_t)j;
  }
  XR old[L];
  uint32_t oP[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    old[i] = S.R[i];
    oP[i] = S.P[i];
  }
#pragma unroll
  for (int j = 0; j < L; ++j) {
    XR t = old[0];
#pragma unroll
    for (int i = 1; i < L; ++i)
      if (p[j] == (uint32_t)i) t = old[i];
    S.R[j] = t;
    S.P[j] = pick<L>(oP, p[j]);
    S.pm[j] = (uint32_t)j < keep ? (int)(kk[j] >> 8) - (int)(kk[0] >> 8) : 0;
  }
  if (moved) {
    for (uint32_t w = 0; w < W; ++w) {
      uint32_t x[L];
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] = C.bits[i][64u * w];
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (p[j] != (uint32_t)j) C.bits[j][64u * w] = pick<L>(x, p[j]);
    }
  }
}

// the T = 4 least reliable positions (|alpha|, then index) of a register
// node, as keys |alpha| << 5 | index in ascending order
template <int K>
__device__ __forceinline__ void least4(XR& R, uint32_t s[4]) {
  constexpr uint32_t M = 1u << K;
  constexpr int W = M >= 4 ? (int)M / 4 : 1;
  s[0] = s[1] = s[2] = s[3] = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < W; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * j + i < (int)M) {
        uint32_t v = ((uint32_t)abs(sx8(xw<K>(R, j), i)) << 5) | (uint32_t)(4 * j + i);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const uint32_t lo = min(v, s[t]);
          v = max(v, s[t]);
          s[t] = lo;
        }
      }
}

// candidates per path of a forking node
__device__ __forceinline__ uint32_t n_cands(uint32_t opc) {
  return opc == OP_SPC ? 8u : (opc == OP_R1 ? 4u : 2u);
}

// a dedicated node or leaf of level K <= 5 over the a active paths
template <int L, int K>
__device__ __forceinline__ void node_regL(PS<L>& S, const CtxL<L>& C, uint32_t opc, uint32_t o,
                                          uint32_t& a) {
  constexpr uint32_t M = 1u << K;
  constexpr int W = M >= 4 ? (int)M / 4 : 1;
  constexpr uint32_t full = M == 32 ? 0xFFFFFFFFu : ((1u << (M & 31u)) - 1u);
  uint32_t hd[L], pos[L], kk[L];
#pragma unroll
  for (int r = 0; r < L; ++r) {
    hd[r] = pos[r] = 0u;
    kk[r] = 0xFFFFFFFFu;
  }
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)L; ++r) {
    if (r >= a) break;
    XR& R = S.R[r];
    int p0 = 0, p1 = 0;  // disagreement with all-0 / all-1
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * j + i < (int)M) {
          const int v = sx8(xw<K>(R, j), i);
          if (v < 0)
            p0 -= v;
          else
            p1 += v;
        }
    uint32_t h = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) h |= hd4(xw<K>(R, j)) << (4 * j);
    hd[r] = h & full;
    if (opc == OP_R0 || opc == OP_LF) {
      S.pm[r] = min(S.pm[r] + p0, kQ);
      R.b = 0u;
    } else if (opc == OP_LI || opc == OP_REP) {
      insL<L>(ckey(S.pm[r], (uint32_t)p0, r, 0u), kk);
      insL<L>(ckey(S.pm[r], (uint32_t)p1, r, 1u), kk);
    } else {
      uint32_t s4[4];
      least4<K>(R, s4);
      pos[r] = (s4[0] & 31u) | ((s4[1] & 31u) << 5) | ((s4[2] & 31u) << 10) | ((s4[3] & 31u) << 15);
      const uint32_t m0 = s4[0] >> 5, m1 = s4[1] >> 5, m2 = s4[2] >> 5, m3 = s4[3] >> 5;
      if (opc == OP_R1) {
#pragma unroll
        for (uint32_t mk = 0; mk < 4; ++mk)
          insL<L>(ckey(S.pm[r], ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u), r, mk), kk);
      } else {
        const uint32_t par = __popc(hd[r]) & 1u;
#pragma unroll
        for (uint32_t mk = 0; mk < 16; ++mk) {
          if ((__popc(mk) & 1u) != par) continue;
          const uint32_t pen = ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u) +
                               ((mk & 4u) ? m2 : 0u) + ((mk & 8u) ? m3 : 0u);
          insL<L>(ckey(S.pm[r], pen, r, mk), kk);
        }
      }
    }
  }
  if (opc == OP_R0 || opc == OP_LF) {
    normalise<L>(S, a);
    return;
  }
  const uint32_t keep = min((uint32_t)L, a * n_cands(opc));
  uint32_t nb[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const uint32_t pj = (kk[j] >> 4) & 3u, lj = kk[j] & 15u;
    if (opc == OP_LI || opc == OP_REP) {
      nb[j] = lj ? full : 0u;
    } else {
      const uint32_t ps = pick<L>(pos, pj);
      uint32_t fl = 0;
#pragma unroll
      for (uint32_t t = 0; t < 4; ++t) fl |= ((lj >> t) & 1u) << ((ps >> (5 * t)) & 31u);
      nb[j] = pick<L>(hd, pj) ^ fl;
    }
  }
  take<L>(S, C, kk, keep, (o >> 6) << 1);  // words below the level-6 ancestor
  a = keep;
#pragma unroll
  for (int j = 0; j < L; ++j) S.R[j].b = nb[j];
}

// a Rate-0 or Rate-1 node of level k >= 6 over the a active paths
template <int L>
__device__ __forceinline__ void node_memL(PS<L>& S, const CtxL<L>& C, uint32_t opc, uint32_t k,
                                          uint32_t o, uint32_t& a) {
  const uint32_t nw = 1u << (k - 5);
  uint32_t kk[L], pos[L];
#pragma unroll
  for (int r = 0; r < L; ++r) {
    kk[r] = 0xFFFFFFFFu;
    pos[r] = 0u;
  }
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)L; ++r) {
    if (r >= a) break;
    const uint32_t Pr = S.P[r];
    const Src s = k == 6 ? Src{nullptr, 0u} : srcL<L>(C, Pr, k);
    const uint4* l = l6of<L>(C, Pr);
    uint32_t* w = C.bits[r] + (size_t)64u * (o >> 5);
    int p0 = 0;
    uint32_t s0 = 0xFFFFFFFFu, s1 = 0xFFFFFFFFu;
    for (uint32_t q = 0; q < nw; ++q) {
      const Chunk x0 = k == 6 ? ldl(l, 2 * q) : ldc(s.p + (size_t)(2 * q) * s.cs);
      const Chunk x1 = k == 6 ? ldl(l, 2 * q + 1) : ldc(s.p + (size_t)(2 * q + 1) * s.cs);
      if (opc == OP_R0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            p0 += max(-sx8(x0.w[j], i), 0);
            p0 += max(-sx8(x1.w[j], i), 0);
          }
        w[64u * q] = 0u;
      } else {
        w[64u * q] = hd16(x0) | (hd16(x1) << 16);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t e = 32u * q + 4u * j + i;
            uint32_t v = ((uint32_t)abs(sx8(x0.w[j], i)) << 12) | e;
            uint32_t lo = min(v, s0);
            v = max(v, s0);
            s0 = lo;
            s1 = min(v, s1);
            v = ((uint32_t)abs(sx8(x1.w[j], i)) << 12) | (e + 16u);
            lo = min(v, s0);
            v = max(v, s0);
            s0 = lo;
            s1 = min(v, s1);
          }
      }
    }
    if (opc == OP_R0) {
      S.pm[r] = min(S.pm[r] + p0, kQ);
    } else {
      pos[r] = (s0 & 0xFFFu) | ((s1 & 0xFFFu) << 16);
      const uint32_t m0 = s0 >> 12, m1 = s1 >> 12;
#pragma unroll
      for (uint32_t mk = 0; mk < 4; ++mk)
        insL<L>(ckey(S.pm[r], ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u), r, mk), kk);
    }
  }
  if (opc == OP_R0) {
    normalise<L>(S, a);
    return;
  }
  const uint32_t keep = min((uint32_t)L, a * 4u);
  uint32_t ps[L], lj[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    ps[j] = pick<L>(pos, (kk[j] >> 4) & 3u);
    lj[j] = kk[j] & 15u;
  }
  take<L>(S, C, kk, keep, (o >> 5) + nw);
  a = keep;
#pragma unroll
  for (uint32_t j = 0; j < (uint32_t)L; ++j) {
    if (j >= keep) break;
#pragma unroll
    for (uint32_t t = 0; t < 2; ++t)
      if ((lj[j] >> t) & 1u) {
        const uint32_t e = o + ((ps[j] >> (16 * t)) & 0xFFFu);
        C.bits[j][64u * (e >> 5)] ^= 1u << (e & 31u);
      }
  }
}

template <int L>
__device__ __forceinline__ void nodeL(PS<L>& S, const CtxL<L>& C, uint32_t opc, uint32_t k,
                                      uint32_t o, uint32_t& a) {
  switch (k) {
    case 5: node_regL<L, 5>(S, C, opc, o, a); break;
    case 4: node_regL<L, 4>(S, C, opc, o, a); break;
    case 3: node_regL<L, 3>(S, C, opc, o, a); break;
    case 2: node_regL<L, 2>(S, C, opc, o, a); break;
    case 1: node_regL<L, 1>(S, C, opc, o, a); break;
    case 0: node_regL<L, 0>(S, C, opc, o, a); break;
    default: node_memL<L>(S, C, opc, k, o, a); break;
  }
}

// ================================================= L = 2..32: one path per lane
// The list stages of size L >= 2 (Algorithm 1 with the dedicated nodes of
// Sec. II-B3 and the selection of Sec. II-B2) for the frames of a uniform
// int8 batch whose next stage is L: 64 / L frames per wave, lane g L + r
// holding path r of frame g.  Every lane runs its path's steps as in the
// L = 1 kernel; a lane's buffers of levels >= 6 are the slots of the list:
// a path reads its node from the lane its slot number names and writes its
// child to its own lane (index indirection).  At a forking node every path
// offers its candidates (as in the list decoder), a candidate's rank among
// the frame's L C keys (metric, parent, local index) is counted across its
// lanes, the L best are scattered through LDS to their new ranks, and each
// new path takes its parent's registers and slot numbers by lane
// permutation and copies its partial sums below the node.

struct PP {  // one path of a lane
  XR R;
  int pm;
  uint32_t P;  // lane holding this path's buffer of level k (6 .. 10): 6 bits at 6 (k - 6)
};

struct CtxP {
  char* region;      // this wave's region (as the L = 1 kernel's)
  const char* root;  // this lane's channel LLRs
  uint32_t n, lane, bw;
  uint32_t* bits0;  // partial-sum word w of lane s at bits0[64 w + s]
  uint4* l60;       // level-6 chunk c of lane s at l60[64 c + s] (LDS)
  uint32_t* sel;    // LDS: 64 words of selection scratch
};

__device__ __forceinline__ uint32_t pslot(uint32_t P, uint32_t k) { return (P >> (6 * (k - 6))) & 63u; }
__device__ __forceinline__ uint32_t pset(uint32_t P, uint32_t k, uint32_t s) {
  return (P & ~(63u << (6 * (k - 6)))) | (s << (6 * (k - 6)));
}
__device__ __forceinline__ char* pbuf(const CtxP& C, uint32_t k, uint32_t s) {
  return C.region + (size_t)64u * ((1u << k) - 128u) + 16u * s;  // levels 7 .. n-1
}
__device__ __forceinline__ Src psrc(const CtxP& C, uint32_t P, uint32_t k) {
  if (k == C.n) return Src{C.root, 16u};
  return Src{pbuf(C, k, pslot(P, k)), 1024u};
}
__device__ __forceinline__ uint32_t* pcol(const CtxP& C, uint32_t s) { return C.bits0 + s; }

template <bool G, bool DL>
__device__ __forceinline__ void fgP(const CtxP& C, uint32_t P, uint32_t k, uint32_t o) {
  const Src s = psrc(C, P, k);
  const uint32_t nc = 1u << (k - 5);
  const char* pa = s.p;
  const char* pb = s.p + (size_t)nc * s.cs;
  char* dst = DL ? nullptr : pbuf(C, k - 1, C.lane);
  uint4* dl = C.l60 + C.lane;
  const uint32_t* lb = pcol(C, C.lane) + (size_t)64u * (o >> 5);
  for (uint32_t c = 0; c < nc; c += 2) {
    const Chunk a0 = ldc(pa + (size_t)c * s.cs), b0 = ldc(pb + (size_t)c * s.cs);
    const Chunk a1 = ldc(pa + (size_t)(c + 1) * s.cs), b1 = ldc(pb + (size_t)(c + 1) * s.cs);
    Chunk r0, r1;
    if constexpr (G) {
      const uint32_t sw = lb[64u * (c >> 1)];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = g4(a0.w[j], b0.w[j], (sw >> (4 * j)) & 15u);
        r1.w[j] = g4(a1.w[j], b1.w[j], (sw >> (16 + 4 * j)) & 15u);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        r0.w[j] = f4(a0.w[j], b0.w[j]);
        r1.w[j] = f4(a1.w[j], b1.w[j]);
      }
    }
    if constexpr (DL) {
      stl(dl, c, r0);
      stl(dl, c + 1, r1);
    } else {
      stc(dst + (size_t)c * 1024u, r0);
      stc(dst + (size_t)(c + 1) * 1024u, r1);
    }
  }
}

template <bool G>
__device__ __forceinline__ void fg6P(const CtxP& C, uint32_t P, XR& R) {
  const uint4* l = C.l60 + pslot(P, 6);
  const Chunk a0 = ldl(l, 0), a1 = ldl(l, 1), b0 = ldl(l, 2), b1 = ldl(l, 3);
  if constexpr (G) R.l6 = R.b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (G) {
      R.x5[j] = g4(a0.w[j], b0.w[j], (R.b >> (4 * j)) & 15u);
      R.x5[j + 4] = g4(a1.w[j], b1.w[j], (R.b >> (16 + 4 * j)) & 15u);
    } else {
      R.x5[j] = f4(a0.w[j], b0.w[j]);
      R.x5[j + 4] = f4(a1.w[j], b1.w[j]);
    }
  }
}

__device__ __forceinline__ void hP(const CtxP& C, const XR& R, uint32_t k, uint32_t o) {
  uint32_t* w = pcol(C, C.lane) + (size_t)64u * (o >> 5);
  if (k == 6) {
    w[0] = R.l6 ^ R.b;
    w[64] = R.b;
    return;
  }
  const uint32_t nw = 1u << (k - 6);
  uint32_t* q = w + (size_t)64u * nw;
  for (uint32_t i = 0; i < nw; ++i) w[64u * i] ^= q[64u * i];
}

__device__ __forceinline__ XR bperm_xr(const XR& R, uint32_t src) {
  XR o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o.x5[j] = bperm(R.x5[j], src);
#pragma unroll
  for (int j = 0; j < 4; ++j) o.x4[j] = bperm(R.x4[j], src);
  o.x3[0] = bperm(R.x3[0], src);
  o.x3[1] = bperm(R.x3[1], src);
  o.x2 = bperm(R.x2, src);
  o.x1 = bperm(R.x1, src);
  o.x0 = bperm(R.x0, src);
  o.b = bperm(R.b, src);
  o.lft = bperm(R.lft, src);
  o.l6 = bperm(R.l6, src);
  return o;
}

// smallest value over the L lanes of the caller's frame
template <int L>
__device__ __forceinline__ int group_min(int v, uint32_t lane) {
#pragma unroll
  for (uint32_t s = 1; s < (uint32_t)L; s <<= 1) v = min(v, (int)bperm((uint32_t)v, lane ^ s));
  return v;
}

// Keys: metric << 9 | parent rank << 4 | local index (unique in a frame).
__device__ __forceinline__ uint32_t pkey(int pm, uint32_t pen, uint32_t r, uint32_t local) {
  return ((uint32_t)min(pm + (int)pen, kQ) << 9) | (r << 4) | local;
}

// The L best of the frame's candidates (kc[0 .. C) per lane, ~0 where
// absent) become the new paths: returns this lane's new key (~0 when the
// lane holds no path afterwards) and its parent's lane.
template <int L, int C>
__device__ __forceinline__ uint32_t select_p(const CtxP& C_, const uint32_t (&kc)[C], uint32_t keep,
                                             uint32_t& parent_lane, uint32_t& best) {
  const uint32_t lane = C_.lane, g0 = lane & ~(uint32_t)(L - 1);
  uint32_t rk[C];
#pragma unroll
  for (int c = 0; c < C; ++c) rk[c] = 0;
  for (uint32_t t = 0; t < (uint32_t)L; ++t) {
#pragma unroll
    for (int c2 = 0; c2 < C; ++c2) {
      const uint32_t o = bperm(kc[c2], g0 + t);
#pragma unroll
      for (int c = 0; c < C; ++c) rk[c] += o < kc[c] ? 1u : 0u;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (kc[c] != 0xFFFFFFFFu && rk[c] < keep) C_.sel[g0 + rk[c]] = kc[c];
  __syncthreads();
  const uint32_t r = lane - g0;
  const uint32_t nk = r < keep ? C_.sel[lane] : 0xFFFFFFFFu;
  best = C_.sel[g0];
  __syncthreads();
  // a lane left without a path keeps its own state (and reads only its own column)
  parent_lane = nk == 0xFFFFFFFFu ? lane : g0 + ((nk >> 4) & 31u);
  return nk;
}

// new paths take their parents' state; partial-sum words [0, W) follow the parent
__device__ __forceinline__ void adopt(PP& S, const CtxP& C, uint32_t nk, uint32_t pl, uint32_t best,
                                      uint32_t W) {
  S.R = bperm_xr(S.R, pl);
  S.P = bperm(S.P, pl);
  S.pm = nk == 0xFFFFFFFFu ? 0 : (int)(nk >> 9) - (int)(best >> 9);
  const bool mv = nk != 0xFFFFFFFFu && pl != C.lane;
  if (__ballot(mv) == 0ull) return;
  uint32_t* src = pcol(C, pl);
  uint32_t* dst = pcol(C, C.lane);
  // every lane reads word w before any lane overwrites it (a parent's column
  // may be another new path's own)
  for (uint32_t w = 0; w < W; ++w) {
    const uint32_t x = src[64u * w];
    __syncthreads();
    if (mv) dst[64u * w] = x;
  }
}

// a dedicated node or leaf of level K <= 5; r: this lane's path rank, a: active paths
template <int L, int K>
__device__ __forceinline__ void node_regP(PP& S, const CtxP& C, uint32_t opc, uint32_t o, uint32_t r,
                                          uint32_t& a) {
  constexpr uint32_t M = 1u << K;
  constexpr int W = M >= 4 ? (int)M / 4 : 1;
  constexpr uint32_t full = M == 32 ? 0xFFFFFFFFu : ((1u << (M & 31u)) - 1u);
  const bool act = r < a;
  XR& R = S.R;
  int p0 = 0, p1 = 0;
#pragma unroll
  for (int j = 0; j < W; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * j + i < (int)M) {
        const int v = sx8(xw<K>(R, j), i);
        if (v < 0)
          p0 -= v;
        else
          p1 += v;
      }
  uint32_t hd = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) hd |= hd4(xw<K>(R, j)) << (4 * j);
  hd &= full;
  if (opc == OP_R0 || opc == OP_LF) {
    S.pm = min(S.pm + p0, kQ);
    R.b = 0u;
    const int mn = group_min<L>(act ? S.pm : 0x7FFFFFFF, C.lane);
    S.pm -= mn;
    return;
  }
  uint32_t nk, pl, best;
  uint32_t pos = 0;
  if (opc == OP_LI || opc == OP_REP) {
    uint32_t kc[2] = {act ? pkey(S.pm, (uint32_t)p0, r, 0u) : 0xFFFFFFFFu,
                      act ? pkey(S.pm, (uint32_t)p1, r, 1u) : 0xFFFFFFFFu};
    nk = select_p<L, 2>(C, kc, min((uint32_t)L, a * 2u), pl, best);
    a = min((uint32_t)L, a * 2u);
  } else {
    uint32_t s4[4];
    least4<K>(R, s4);
    pos = (s4[0] & 31u) | ((s4[1] & 31u) << 5) | ((s4[2] & 31u) << 10) | ((s4[3] & 31u) << 15);
    const uint32_t m0 = s4[0] >> 5, m1 = s4[1] >> 5, m2 = s4[2] >> 5, m3 = s4[3] >> 5;
    if (opc == OP_R1) {
      uint32_t kc[4];
#pragma unroll
      for (uint32_t mk = 0; mk < 4; ++mk)
        kc[mk] = act ? pkey(S.pm, ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u), r, mk) : 0xFFFFFFFFu;
      nk = select_p<L, 4>(C, kc, min((uint32_t)L, a * 4u), pl, best);
      a = min((uint32_t)L, a * 4u);
    } else {
      // the eight masks whose weight has the parity of the hard decisions
      // (nibble i of 0xFCA96530: the even ones, of 0xEDB87421: the odd ones)
      const uint32_t masks = (__popc(hd) & 1u) ? 0xEDB87421u : 0xFCA96530u;
      uint32_t kc[8];
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t mk = (masks >> (4 * i)) & 15u;
        const uint32_t pen = ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u) + ((mk & 4u) ? m2 : 0u) +
                             ((mk & 8u) ? m3 : 0u);
        kc[i] = act ? pkey(S.pm, pen, r, mk) : 0xFFFFFFFFu;
      }
      nk = select_p<L, 8>(C, kc, min((uint32_t)L, a * 8u), pl, best);
      a = min((uint32_t)L, a * 8u);
    }
  }
  const uint32_t hdp = bperm(hd, pl), posp = bperm(pos, pl);
  adopt(S, C, nk, pl, best, (o >> 6) << 1);
  const uint32_t lj = nk & 15u;
  if (opc == OP_LI || opc == OP_REP) {
    S.R.b = lj ? full : 0u;
  } else {
    uint32_t fl = 0;
#pragma unroll
    for (uint32_t t = 0; t < 4; ++t) fl |= ((lj >> t) & 1u) << ((posp >> (5 * t)) & 31u);
    S.R.b = hdp ^ fl;
  }
}

// a Rate-0 or Rate-1 node of level k >= 6
template <int L>
__device__ __forceinline__ void node_memP(PP& S, const CtxP& C, uint32_t opc, uint32_t k, uint32_t o,
                                          uint32_t r, uint32_t& a) {
  const uint32_t nw = 1u << (k - 5);
  const bool act = r < a;
  const Src s = k == 6 ? Src{nullptr, 0u} : psrc(C, S.P, k);
  const uint4* l = C.l60 + pslot(S.P, 6);
  uint32_t* w = pcol(C, C.lane) + (size_t)64u * (o >> 5);
  int p0 = 0;
  uint32_t s0 = 0xFFFFFFFFu, s1 = 0xFFFFFFFFu;
  for (uint32_t q = 0; q < nw; ++q) {
    const Chunk x0 = k == 6 ? ldl(l, 2 * q) : ldc(s.p + (size_t)(2 * q) * s.cs);
    const Chunk x1 = k == 6 ? ldl(l, 2 * q + 1) : ldc(s.p + (size_t)(2 * q + 1) * s.cs);
    if (opc == OP_R0) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          p0 += max(-sx8(x0.w[j], i), 0);
          p0 += max(-sx8(x1.w[j], i), 0);
        }
      w[64u * q] = 0u;
    } else {
      w[64u * q] = hd16(x0) | (hd16(x1) << 16);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t e = 32u * q + 4u * j + i;
          uint32_t v = ((uint32_t)abs(sx8(x0.w[j], i)) << 12) | e;
          uint32_t lo = min(v, s0);
          v = max(v, s0);
          s0 = lo;
          s1 = min(v, s1);
          v = ((uint32_t)abs(sx8(x1.w[j], i)) << 12) | (e + 16u);
          lo = min(v, s0);
          v = max(v, s0);
          s0 = lo;
          s1 = min(v, s1);
        }
    }
  }
  if (opc == OP_R0) {
    S.pm = min(S.pm + p0, kQ);
    const int mn = group_min<L>(act ? S.pm : 0x7FFFFFFF, C.lane);
    S.pm -= mn;
    return;
  }
  const uint32_t pos = (s0 & 0xFFFu) | ((s1 & 0xFFFu) << 16);
  const uint32_t m0 = s0 >> 12, m1 = s1 >> 12;
  uint32_t kc[4];
#pragma unroll
  for (uint32_t mk = 0; mk < 4; ++mk)
    kc[mk] = act ? pkey(S.pm, ((mk & 1u) ? m0 : 0u) + ((mk & 2u) ? m1 : 0u), r, mk) : 0xFFFFFFFFu;
  uint32_t pl, best;
  const uint32_t nk = select_p<L, 4>(C, kc, min((uint32_t)L, a * 4u), pl, best);
  a = min((uint32_t)L, a * 4u);
  const uint32_t posp = bperm(pos, pl);
  adopt(S, C, nk, pl, best, (o >> 5) + nw);
  const uint32_t lj = nk & 15u;
  if (nk != 0xFFFFFFFFu) {
#pragma unroll
    for (uint32_t t = 0; t < 2; ++t)
      if ((lj >> t) & 1u) {
        const uint32_t e = o + ((posp >> (16 * t)) & 0xFFFu);
        pcol(C, C.lane)[64u * (e >> 5)] ^= 1u << (e & 31u);
      }
  }
}

template <int L>
__device__ __forceinline__ void nodeP(PP& S, const CtxP& C, uint32_t opc, uint32_t k, uint32_t o,
                                      uint32_t r, uint32_t& a) {
  switch (k) {
    case 5: node_regP<L, 5>(S, C, opc, o, r, a); break;
    case 4: node_regP<L, 4>(S, C, opc, o, r, a); break;
    case 3: node_regP<L, 3>(S, C, opc, o, r, a); break;
    case 2: node_regP<L, 2>(S, C, opc, o, r, a); break;
    case 1: node_regP<L, 1>(S, C, opc, o, r, a); break;
    case 0: node_regP<L, 0>(S, C, opc, o, r, a); break;
    default: node_memP<L>(S, C, opc, k, o, r, a); break;
  }
}

}  // namespace

// A persistent grid: wave g decodes the groups of 64 frames g, g + G, ...
// (frame 64 q + lane; lanes past the batch decode its last frame and drop
// the result).  Every frame of the batch starts at L = 1 (the caller checks
// the plan); a frame whose CRC fails gets its next list size in state[f],
// the others are finished here.
__global__ __launch_bounds__(64) void k_scx(KArgs A, uint32_t* state) {
  __shared__ uint4 lds6[4 * 64];  // level 6: 4 chunks per lane
  static_assert(sizeof(lds6) == kScxLds, "LDS per wave");
  const uint32_t lane = threadIdx.x;
  const DevPlan* P = uni_ptr(A.plans[0]);
  const uint32_t N = uni(P->N), n = uni(P->n), n_ops = uni(P->n_ops), bw = uni(P->bw);
  const uint32_t iw = uni(A.info_words), L_max = uni(P->L_max), c_len = uni(P->c);
  const uint32_t* prog = uni_ptr(plan_tab(P, uni(P->off_prog)));
  const uint32_t* imask = uni_ptr(plan_tab(P, uni(P->off_infomask)));
  const uint32_t* nib = uni_ptr(plan_tab(P, uni(P->off_crcnib)));
  const uint32_t* dmask = uni_ptr(plan_tab(P, uni(P->off_datamask)));
  char* region = A.spill + (size_t)blockIdx.x * A.spill_stride;
  const uint32_t n_groups = (A.n_frames + 63u) / 64u;
  for (uint32_t q = blockIdx.x; q < n_groups; q += gridDim.x) {
    const uint32_t f = 64u * q + lane;
    const bool valid = f < A.n_frames;
    const uint32_t fi = valid ? f : A.n_frames - 1u;
    if (valid && A.times) A.times[2 * (size_t)f] = wall_clock64();
    Ctx C;
    C.region = region;
    C.root = A.llr + (size_t)fi * A.llr_bytes;
    C.n = n;
    C.lane = lane;
    C.bits = reinterpret_cast<uint32_t*>(region + (size_t)64u * (N - 128u)) + lane;
    C.l6 = lds6 + lane;
    XR R;
#pragma unroll
    for (int j = 0; j < 8; ++j) R.x5[j] = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) R.x4[j] = 0u;
    R.x3[0] = R.x3[1] = R.x2 = R.x1 = R.x0 = 0u;
    R.b = R.lft = R.l6 = 0u;
    uint32_t w_next = prog[0];
    for (uint32_t pc = 0; pc < n_ops; ++pc) {
      const uint32_t w = uni(w_next);
      if (pc + 1 < n_ops) w_next = prog[pc + 1];
      const uint32_t opc = op_code(w), k = n - op_depth(w), o = op_off(w);
      if (k <= 5) {
        reg_op(R, opc, k);
      } else if (opc == OP_F) {
        if (k == 6)
          mem_fg6<false>(C, R);
        else if (k == 7)
          mem_fg<false, true>(C, k, o);
        else
          mem_fg<false, false>(C, k, o);
      } else if (opc == OP_G) {
        if (k == 6)
          mem_fg6<true>(C, R);
        else if (k == 7)
          mem_fg<true, true>(C, k, o);
        else
          mem_fg<true, false>(C, k, o);
      } else if (opc == OP_H) {
        mem_h(C, R, k, o);
      } else {
        mem_node(C, opc, k, o);
      }
    }
    // ---- CRC syndrome of the codeword estimate through the nibble table
    uint32_t syn = 0;
    if (c_len > 0) {
      for (uint32_t wd = 0; wd < bw; ++wd) {
        const uint32_t im = imask[wd];
        if (!im) continue;
        const uint32_t v = C.bits[64u * wd] & im;
        for (uint32_t t = 0; t < 8; ++t)
          if ((im >> (4 * t)) & 15u) syn ^= nib[((wd * 8 + t) << 4) + ((v >> (4 * t)) & 15u)];
      }
    }
    const bool ok = syn == 0u;
    const bool esc = valid && !ok && L_max > 1;
    if (esc) state[f] = next_stage(P, 1);
    const bool fin = valid && !esc;
    // ---- information bits: the data positions of A in ascending order
    uint32_t* out = A.info + (size_t)fi * iw;
    uint32_t cur = 0, pos = 0, ow = 0;
    for (uint32_t wd = 0; wd < bw; ++wd) {
      uint32_t dm = dmask[wd];
      if (!dm) continue;
      const uint32_t x = C.bits[64u * wd];
      uint32_t v = 0, cnt = 0;
      while (dm) {
        const uint32_t b = __ffs(dm) - 1;
        v |= ((x >> b) & 1u) << cnt;
        ++cnt;
        dm &= dm - 1u;
      }
      cur |= v << pos;
      if (pos + cnt >= 32) {
        if (fin) out[ow] = cur;
        ++ow;
        cur = pos ? v >> (32 - pos) : 0u;
      }
      pos = (pos + cnt) & 31u;
    }
    if (pos && fin) out[ow] = cur;
    if (fin) {
      polar_status st;
      st.crc_ok = ok ? 1 : 0;
      st.L_used = 1;
      st.n_paths = 1;
      st.flags = 0;
      st.pm = 0u;
      A.status[f] = st;
      if (A.pm_lists)
        for (uint32_t t = 0; t < A.pm_stride; ++t)
          A.pm_lists[(size_t)f * A.pm_stride + t] = t == 0 ? 0u : 0xFFFFFFFFu;
      if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
    }
  }
}

// Bytes of one wave's region for a code of length N (levels 7 .. n-1, then
// the partial sums), 256-byte aligned.
uint64_t scx_region_bytes(uint32_t N) {
  const uint64_t b = 64ull * (N - 128u) + 8ull * N;
  return (b + 255u) & ~255ull;
}

int launch_decode_scx(const KArgs& A, uint32_t grid, uint32_t* state, hipStream_t s) {
  hipLaunchKernelGGL(k_scx, dim3(grid > 0 ? grid : 1), dim3(64), 0, s, A, state);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

// Frames whose next stage is L, listed for the frame-per-lane list kernel:
// xl[0] counts them (zeroed by k_xreset first), xl[1 ..] holds their indices
// (in no set order).
__global__ void k_xreset(uint32_t* xl) {
  if (threadIdx.x == 0) xl[0] = 0u;
}
__global__ __launch_bounds__(256) void k_gather(uint32_t n_frames, uint32_t L, const uint32_t* state,
                                                uint32_t* xl) {
  // each wave takes chunks of kGatherGroups groups of 64 frames: it counts
  // the chunk's frames, reserves their places with one atomic, then writes
  // them (the chunk's state words are read twice, the second time from cache)
  constexpr uint32_t kGatherGroups = 16;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
  const uint32_t n_groups = (n_frames + 63u) / 64u;
  for (uint32_t c = w0; kGatherGroups * c < n_groups; c += nw) {
    const uint32_t g_end = min(n_groups, kGatherGroups * (c + 1u));
    uint32_t tot = 0;
    for (uint32_t g = kGatherGroups * c; g < g_end; ++g) {
      const uint32_t f = 64u * g + lane;
      tot += (uint32_t)__popcll(__ballot(f < n_frames && (state[f] & 0xFFu) == L));
    }
    if (!tot) continue;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&xl[0], tot);
    base = __shfl(base, 0, 64);
    for (uint32_t g = kGatherGroups * c; g < g_end; ++g) {
      const uint32_t f = 64u * g + lane;
      const bool take = f < n_frames && (state[f] & 0xFFu) == L;
      const uint64_t bal = __ballot(take);
      if (take) xl[1 + base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = f;
      base += (uint32_t)__popcll(bal);
    }
  }
}

// The stage of size L of the listed frames, 64 per wave (persistent grid,
// wave g takes the groups g, g + G, ...).  A frame whose CRC passes, or whose
// plan ends at L, is finished (bits, status, metric list, end stamp; state
// 0); the others get their next stage.
template <int L>
__global__ __launch_bounds__(64) void k_listx(KArgs A, uint32_t* state, const uint32_t* xl) {
  __shared__ uint4 lds6x[L * 4 * 64];  // level 6: L slots of 4 chunks per lane
  const uint32_t lane = threadIdx.x;
  const DevPlan* P = uni_ptr(A.plans[0]);
  const uint32_t N = uni(P->N), n = uni(P->n), n_ops = uni(P->n_ops), bw = uni(P->bw);
  const uint32_t iw = uni(A.info_words), L_max = uni(P->L_max), c_len = uni(P->c);
  const uint32_t* prog = uni_ptr(plan_tab(P, uni(P->off_prog)));
  const uint32_t* imask = uni_ptr(plan_tab(P, uni(P->off_infomask)));
  const uint32_t* nib = uni_ptr(plan_tab(P, uni(P->off_crcnib)));
  const uint32_t* dmask = uni_ptr(plan_tab(P, uni(P->off_datamask)));
  char* region = A.spill + (size_t)blockIdx.x * A.spill_stride;
  // the count through a vector load at device scope, not the scalar cache;
  // a list never holds more frames than the batch, and the list's capacity
  // is the batch size, so a count above it is never trusted
  const uint32_t count0 =
      uni(__hip_atomic_load(&xl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  const uint32_t count = count0 < A.n_frames ? count0 : A.n_frames;
  const uint32_t n_groups = (count + 63u) / 64u;
  for (uint32_t q = blockIdx.x; q < n_groups; q += gridDim.x) {
    const uint32_t idx = 64u * q + lane;
    const bool valid = idx < count;
    const uint32_t f0 = xl[1 + (valid ? idx : 64u * q)];
    const uint32_t f = f0 < A.n_frames ? f0 : A.n_frames - 1u;
    CtxL<L> C;
    C.region = region;
    C.root = A.llr + (size_t)f * A.llr_bytes;
    C.n = n;
    C.lane = lane;
    uint32_t* bb = reinterpret_cast<uint32_t*>(region + (size_t)(64u * L) * (N - 128u)) + lane;
    PS<L> S;
#pragma unroll
    for (int r = 0; r < L; ++r) {
      C.bits[r] = bb + (size_t)r * 64u * bw;
      C.l6[r] = lds6x + r * 4 * 64 + lane;
#pragma unroll
      for (int j = 0; j < 8; ++j) S.R[r].x5[j] = 0u;
#pragma unroll
      for (int j = 0; j < 4; ++j) S.R[r].x4[j] = 0u;
      S.R[r].x3[0] = S.R[r].x3[1] = S.R[r].x2 = S.R[r].x1 = S.R[r].x0 = 0u;
      S.R[r].b = S.R[r].lft = S.R[r].l6 = 0u;
      S.pm[r] = 0;
      S.P[r] = 0u;
    }
    uint32_t a = 1;
    uint32_t w_next = prog[0];
    for (uint32_t pc = 0; pc < n_ops; ++pc) {
      const uint32_t w = uni(w_next);
      if (pc + 1 < n_ops) w_next = prog[pc + 1];
      const uint32_t opc = op_code(w), k = n - op_depth(w), o = op_off(w);
      if (opc == OP_F || opc == OP_G || opc == OP_H) {
        const bool g = opc == OP_G;
#pragma unroll
        for (uint32_t r = 0; r < (uint32_t)L; ++r) {
          if (r >= a) break;
          if (k <= 5) {
            reg_op(S.R[r], opc, k);
          } else if (opc == OP_H) {
            hL<L>(C, r, S.R[r], k, o);
          } else if (k == 6) {
            g ? fg6L<L, true>(C, S.P[r], S.R[r]) : fg6L<L, false>(C, S.P[r], S.R[r]);
          } else {
            if (k == 7)
              g ? fgL<L, true, true>(C, S.P[r], r, k, o) : fgL<L, false, true>(C, S.P[r], r, k, o);
            else
              g ? fgL<L, true, false>(C, S.P[r], r, k, o) : fgL<L, false, false>(C, S.P[r], r, k, o);
            S.P[r] = set_slot(S.P[r], k - 1, r);
          }
        }
      } else {
        nodeL<L>(S, C, opc, k, o, a);
      }
    }
    // ---- CRC of each path, in metric order (rank breaks ties)
    uint32_t syn[L], ord[L];
#pragma unroll
    for (int r = 0; r < L; ++r) {
      syn[r] = 0u;
      ord[r] = 0xFFFFFFFFu;
    }
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)L; ++r)
      if (r < a) insL<L>(((uint32_t)S.pm[r] << 2) | r, ord);
    if (c_len > 0) {
      for (uint32_t wd = 0; wd < bw; ++wd) {
        const uint32_t im = imask[wd];
        if (!im) continue;
        uint32_t v[L];
#pragma unroll
        for (int r = 0; r < L; ++r) v[r] = C.bits[r][64u * wd] & im;
        for (uint32_t t = 0; t < 8; ++t)
          if ((im >> (4 * t)) & 15u) {
            const uint32_t base = (wd * 8 + t) << 4;
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)L; ++r)
              if (r < a) syn[r] ^= nib[base + ((v[r] >> (4 * t)) & 15u)];
          }
      }
    }
    uint32_t ch = ord[0] & 3u;
    bool ok = false;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
      const uint32_t r = ord[t] & 3u;
      if ((uint32_t)t < a && pick<L>(syn, r) == 0u) {
        ch = r;
        ok = true;
      }
    }
    const bool fin = valid && (ok || L_max <= (uint32_t)L);
    if (valid && !fin) state[f] = next_stage(P, L);
    // ---- outputs of a finished frame: the chosen path's data bits
    uint32_t* out = A.info + (size_t)f * iw;
    const uint32_t* xb = pick<L>(C.bits, ch);
    uint32_t cur = 0, pos = 0, ow = 0;
    for (uint32_t wd = 0; wd < bw; ++wd) {
      uint32_t dm = dmask[wd];
      if (!dm) continue;
      const uint32_t x = xb[64u * wd];
      uint32_t v = 0, cnt = 0;
      while (dm) {
        const uint32_t b = __ffs(dm) - 1;
        v |= ((x >> b) & 1u) << cnt;
        ++cnt;
        dm &= dm - 1u;
      }
      cur |= v << pos;
      if (pos + cnt >= 32) {
        if (fin) out[ow] = cur;
        ++ow;
        cur = pos ? v >> (32 - pos) : 0u;
      }
      pos = (pos + cnt) & 31u;
    }
    if (pos && fin) out[ow] = cur;
    if (fin) {
      polar_status st;
      st.crc_ok = ok ? 1 : 0;
      st.L_used = (uint8_t)L;
      st.n_paths = (uint8_t)a;
      st.flags = 0;
      st.pm = (uint32_t)pick<L>(S.pm, ch);
      A.status[f] = st;
      if (A.pm_lists)
        for (uint32_t t = 0; t < A.pm_stride; ++t) {
          uint32_t v = 0xFFFFFFFFu;
          if (t < a) v = pick<L>(ord, t) >> 2;
          A.pm_lists[(size_t)f * A.pm_stride + t] = v;
        }
      if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
      state[f] = 0u;
    }
  }
}

// Bytes of one wave's region of the list kernel of size L for a code of
// length N (L slots of levels 7 .. n-1, then L partial-sum arrays),
// 256-byte aligned.
uint64_t listx_region_bytes(uint32_t N, uint32_t L) {
  const uint64_t b = 64ull * L * (N - 128u) + 8ull * L * N;
  return (b + 255u) & ~255ull;
}

int launch_decode_listx(const KArgs& A, uint32_t grid, uint32_t* state, uint32_t* xl,
                        hipStream_t s) {
  const uint32_t gb = (A.n_frames + 255u) / 256u < 1024u ? (A.n_frames + 255u) / 256u : 1024u;
  hipLaunchKernelGGL(k_xreset, dim3(1), dim3(64), 0, s, xl);
  hipLaunchKernelGGL(k_gather, dim3(gb > 0 ? gb : 1), dim3(256), 0, s, A.n_frames, 2u,
                     (const uint32_t*)state, xl);
  hipLaunchKernelGGL(k_listx<2>, dim3(grid > 0 ? grid : 1), dim3(64), 0, s, A, state,
                     (const uint32_t*)xl);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

// The stage of size L >= 2 of the listed frames, 64 / L per wave
// (persistent grid, wave q takes the groups q, q + G, ...).  A frame whose
// CRC passes, or whose plan ends at L, is finished (bits, status, metric
// list, end stamp; state 0); the others get their next stage.  `region` is
// the wave's region (levels 7 .. n-1 and the partial sums): global memory,
// or LDS in the form for short lists.  Of the forms launched for a stage,
// the one whose range lo < groups <= hi holds the list's group count takes
// it; the others return at once.
template <int L>
__device__ __forceinline__ void listp_run(const KArgs& A, uint32_t* state, const uint32_t* xl,
                                          char* region, uint4* lds6p, uint32_t* selp,
                                          uint32_t lo, uint32_t hi) {
  constexpr uint32_t FW = 64u / L;  // frames per wave
  const uint32_t lane = threadIdx.x, gi = lane / L, r = lane % L, g0 = lane - r;
  const DevPlan* P = uni_ptr(A.plans[0]);
  const uint32_t N = uni(P->N), n = uni(P->n), n_ops = uni(P->n_ops), bw = uni(P->bw);
  const uint32_t iw = uni(A.info_words), L_max = uni(P->L_max), c_len = uni(P->c);
  const uint32_t* prog = uni_ptr(plan_tab(P, uni(P->off_prog)));
  const uint32_t* imask = uni_ptr(plan_tab(P, uni(P->off_infomask)));
  const uint32_t* nib = uni_ptr(plan_tab(P, uni(P->off_crcnib)));
  const uint32_t* dmask = uni_ptr(plan_tab(P, uni(P->off_datamask)));
  // the count through a vector load at device scope, not the scalar cache;
  // a list never holds more frames than the batch, and the list's capacity
  // is the batch size, so a count above it is never trusted
  const uint32_t count0 =
      uni(__hip_atomic_load(&xl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  const uint32_t count = count0 < A.n_frames ? count0 : A.n_frames;
  const uint32_t n_groups = (count + FW - 1u) / FW;
  if (n_groups <= lo || n_groups > hi) return;
  for (uint32_t q = blockIdx.x; q < n_groups; q += gridDim.x) {
    const uint32_t idx = FW * q + gi;
    const bool valid = idx < count;
    const uint32_t f0 = xl[1 + (valid ? idx : FW * q)];
    const uint32_t f = f0 < A.n_frames ? f0 : A.n_frames - 1u;
    CtxP C;
    C.region = region;
    C.root = A.llr + (size_t)f * A.llr_bytes;
    C.n = n;
    C.lane = lane;
    C.bw = bw;
    C.bits0 = reinterpret_cast<uint32_t*>(region + (size_t)64u * (N - 128u));
    C.l60 = lds6p;
    C.sel = selp;
    PP S;
#pragma unroll
    for (int j = 0; j < 8; ++j) S.R.x5[j] = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) S.R.x4[j] = 0u;
    S.R.x3[0] = S.R.x3[1] = S.R.x2 = S.R.x1 = S.R.x0 = 0u;
    S.R.b = S.R.lft = S.R.l6 = 0u;
    S.pm = 0;
    S.P = 0u;
    uint32_t a = 1;
    uint32_t w_next = prog[0];
    for (uint32_t pc = 0; pc < n_ops; ++pc) {
      const uint32_t w = uni(w_next);
      if (pc + 1 < n_ops) w_next = prog[pc + 1];
      const uint32_t opc = op_code(w), k = n - op_depth(w), o = op_off(w);
      if (opc == OP_F || opc == OP_G || opc == OP_H) {
        const bool g = opc == OP_G;
        if (k <= 5) {
          reg_op(S.R, opc, k);
        } else if (opc == OP_H) {
          hP(C, S.R, k, o);
        } else if (k == 6) {
          g ? fg6P<true>(C, S.P, S.R) : fg6P<false>(C, S.P, S.R);
        } else {
          if (k == 7)
            g ? fgP<true, true>(C, S.P, k, o) : fgP<false, true>(C, S.P, k, o);
          else
            g ? fgP<true, false>(C, S.P, k, o) : fgP<false, false>(C, S.P, k, o);
          S.P = pset(S.P, k - 1, lane);
        }
      } else {
        nodeP<L>(S, C, opc, k, o, r, a);
      }
    }
    // ---- order of the paths (metric, rank), CRC of each, first passing wins
    const bool act = r < a;
    const uint32_t okey = act ? (((uint32_t)S.pm << 6) | r) : 0xFFFFFFFFu;
    uint32_t ordr = 0;
    for (uint32_t t = 0; t < (uint32_t)L; ++t) ordr += bperm(okey, g0 + t) < okey ? 1u : 0u;
    uint32_t syn = 0;
    if (c_len > 0) {
      const uint32_t* col = pcol(C, lane);
      for (uint32_t wd = 0; wd < bw; ++wd) {
        const uint32_t im = imask[wd];
        if (!im) continue;
        const uint32_t v = col[64u * wd] & im;
        for (uint32_t t = 0; t < 8; ++t)
          if ((im >> (4 * t)) & 15u) syn ^= nib[((wd * 8 + t) << 4) + ((v >> (4 * t)) & 15u)];
      }
    }
    const int first = group_min<L>(act && syn == 0u ? (int)ordr : 255, lane);
    const bool ok = first < 255;
    const uint32_t cho = ok ? (uint32_t)first : 0u;
    const bool ch = act && ordr == cho;
    const bool fin = valid && (ok || L_max <= (uint32_t)L);
    if (r == 0 && valid) state[f] = fin ? 0u : next_stage(P, L);
    // ---- outputs of a finished frame from its chosen path's lane
    uint32_t* out = A.info + (size_t)f * iw;
    const uint32_t* xb = pcol(C, lane);
    const bool wr = fin && ch;
    uint32_t cur = 0, pos = 0, ow = 0;
    for (uint32_t wd = 0; wd < bw; ++wd) {
      uint32_t dm = dmask[wd];
      if (!dm) continue;
      const uint32_t x = xb[64u * wd];
      uint32_t v = 0, cnt = 0;
      while (dm) {
        const uint32_t b = __ffs(dm) - 1;
        v |= ((x >> b) & 1u) << cnt;
        ++cnt;
        dm &= dm - 1u;
      }
      cur |= v << pos;
      if (pos + cnt >= 32) {
        if (wr) out[ow] = cur;
        ++ow;
        cur = pos ? v >> (32 - pos) : 0u;
      }
      pos = (pos + cnt) & 31u;
    }
    if (pos && wr) out[ow] = cur;
    if (wr) {
      polar_status st;
      st.crc_ok = ok ? 1 : 0;
      st.L_used = (uint8_t)L;
      st.n_paths = (uint8_t)a;
      st.flags = 0;
      st.pm = (uint32_t)S.pm;
      A.status[f] = st;
      if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
    }
    // metric list in order: each path's metric to its order's place
    if (act) selp[g0 + ordr] = (uint32_t)S.pm;
    __syncthreads();
    const uint32_t mine = r < a ? selp[lane] : 0xFFFFFFFFu;
    __syncthreads();
    if (fin && A.pm_lists)
      for (uint32_t t = r; t < A.pm_stride; t += L)
        A.pm_lists[(size_t)f * A.pm_stride + t] = t == r ? mine : 0xFFFFFFFFu;
  }
}

// L = 32 is held to 128 VGPRs (4 waves per SIMD): at the busiest point its
// frames then fit the chip in one pass.
template <int L>
__global__ __launch_bounds__(64, (L == 32 ? 4 : 1)) void k_listp(KArgs A, uint32_t* state,
                                                                 const uint32_t* xl, uint32_t lo,
                                                                 uint32_t hi) {
  __shared__ uint4 lds6p[4 * 64];  // level 6: 4 chunks per lane
  __shared__ uint32_t selp[64];
  listp_run<L>(A, state, xl, A.spill + (size_t)blockIdx.x * A.spill_stride, lds6p, selp, lo, hi);
}

// The same stage with no register bound (160 VGPRs at L = 32, 3 waves per
// SIMD): for lists that fit the chip in one pass at that occupancy, where
// each wave's own latency sets the time.
template <int L>
__global__ __launch_bounds__(64) void k_listp_mid(KArgs A, uint32_t* state, const uint32_t* xl,
                                                  uint32_t lo, uint32_t hi) {
  __shared__ uint4 lds6p[4 * 64];
  __shared__ uint32_t selp[64];
  listp_run<L>(A, state, xl, A.spill + (size_t)blockIdx.x * A.spill_stride, lds6p, selp, lo, hi);
}

// The same stage with the wave's region in dynamic LDS (scx_region_bytes(N)
// bytes): for short lists, whose few waves would otherwise wait on global
// memory at every level >= 7.
template <int L>
__global__ __launch_bounds__(64, 1) void k_listp_lds(KArgs A, uint32_t* state, const uint32_t* xl,
                                                     uint32_t lo, uint32_t hi) {
  __shared__ uint4 lds6p[4 * 64];
  __shared__ uint32_t selp[64];
  extern __shared__ uint4 lds_region[];
  listp_run<L>(A, state, xl, reinterpret_cast<char*>(lds_region), lds6p, selp, lo, hi);
}

uint32_t listp_static_lds() { return (uint32_t)(4 * 64 * sizeof(uint4) + 64 * sizeof(uint32_t)); }

int listp_set_attributes(uint32_t lds) {
  return hipFuncSetAttribute((const void*)k_listp_lds<32>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess
             ? POLAR_OK
             : POLAR_EHIP;
}

int launch_gather(uint32_t n_frames, uint32_t L, const uint32_t* state, uint32_t* xl, hipStream_t s) {
  const uint32_t gb = (n_frames + 255u) / 256u < 1024u ? (n_frames + 255u) / 256u : 1024u;
  hipLaunchKernelGGL(k_xreset, dim3(1), dim3(64), 0, s, xl);
  hipLaunchKernelGGL(k_gather, dim3(gb > 0 ? gb : 1), dim3(256), 0, s, n_frames, L, state, xl);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_decode_listp(uint32_t L, const KArgs& A, uint32_t grid, uint32_t grid_mid,
                        uint32_t grid_lds, uint32_t lds, uint32_t* state, uint32_t* xl,
                        hipStream_t s) {
  const uint32_t gb = (A.n_frames + 255u) / 256u < 1024u ? (A.n_frames + 255u) / 256u : 1024u;
  hipLaunchKernelGGL(k_xreset, dim3(1), dim3(64), 0, s, xl);
  hipLaunchKernelGGL(k_gather, dim3(gb > 0 ? gb : 1), dim3(256), 0, s, A.n_frames, L,
                     (const uint32_t*)state, xl);
  const dim3 gr(grid > 0 ? grid : 1);
  const uint32_t* cxl = xl;
  if (L != 32) {
    const uint32_t lo = 0, hi = 0xFFFFFFFFu;
    if (L == 2)
      hipLaunchKernelGGL(k_listp<2>, gr, dim3(64), 0, s, A, state, cxl, lo, hi);
    else if (L == 4)
      hipLaunchKernelGGL(k_listp<4>, gr, dim3(64), 0, s, A, state, cxl, lo, hi);
    else if (L == 8)
      hipLaunchKernelGGL(k_listp<8>, gr, dim3(64), 0, s, A, state, cxl, lo, hi);
    else
      hipLaunchKernelGGL(k_listp<16>, gr, dim3(64), 0, s, A, state, cxl, lo, hi);
    return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
  }
  // L = 32: up to grid_lds groups in LDS (one pass), then up to grid_mid
  // (the one-pass capacity at 3 waves per SIMD) unbounded, the rest bounded
  const uint32_t h_lds = grid_lds > 0 && lds > 0 ? grid_lds : 0u;
  const uint32_t h_mid = grid_mid > h_lds ? grid_mid : h_lds;
  if (h_lds)
    hipLaunchKernelGGL(k_listp_lds<32>, dim3(grid_lds), dim3(64), lds, s, A, state, cxl, 0u,
                       h_lds);
  if (h_mid > h_lds)
    hipLaunchKernelGGL(k_listp_mid<32>, dim3(grid_mid), dim3(64), 0, s, A, state, cxl, h_lds,
                       h_mid);
  hipLaunchKernelGGL(k_listp<32>, gr, dim3(64), 0, s, A, state, cxl, h_mid, 0xFFFFFFFFu);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

}  // namespace polar
