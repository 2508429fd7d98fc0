// L = 1 tier of the decoder on gfx950: successive cancellation over the
// pruned tree (Sec. II-B1, II-B3) for every frame, with the CRC check of the
// fully / partially adaptive schedules (Sec. II-B5) and a per-frame state
// word for the frames that need a list.  (Uniform int8 batches of codes
// that send every position run one frame per lane instead: scx.hip.)
//
// A list of one path never forks, so this tier keeps no candidate lists, no
// path copies and no slot indirection.  One wave decodes two frames of the
// same plan, one per half (32 lanes each): the node program, its dispatch
// and every uniform value are shared by the pair, and a register op serves
// both frames.  Its layout follows the shape of the tree:
//   * nodes of size >= 128 keep their LLRs in LDS (one region per frame);
//   * every subtree of size <= 64 runs in registers: the nodes of size
//     2^k <= 16 on the current path share one register, level k in lanes
//     [2^k, 2^(k+1)) of the half, the node of size 32 has a register of its
//     own (lane = element) and the node of size 64 two (elements l, l + 32);
//     partial sums are one bit per lane in the same places, so an op at any
//     register level is one code path (operands move between levels by lane
//     permutation) and the op word is dispatched on its opcode alone;
//   * a dedicated node decides with a ballot (Rate-1: hard decision; SPC:
//     hard decision with the least reliable position flipped on odd parity)
//     or a lane reduction (REP: the two disagreement penalties).
// The decisions are those of a list of one under the selection rule of the
// list decoder (candidate key = metric, parent rank, local index): the
// hard-decision candidate wins a tie, the all-zero REP candidate wins a tie,
// and float32 metrics are summed in the stride-halving order.  Integer metrics
// are normalised after every update, so they stay 0 at L = 1; only the REP
// decision needs its saturated penalties.  In float32 every forking decision
// also compares the best candidate metric with the runner-up's: a gap
// within 1e-4 relative flags the frame as a near-tie (bit 0 of its status
// flags, or bit 8 of its state word when it moves on to a list).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/polar_scl.h"
#include "device_common.h"
#include "kernels.h"
#include "polar_internal.h"

namespace polar {

namespace {

template <typename T>
struct Lane {  // register type of one LLR
  using V = int;
};
template <>
struct Lane<float> {
  using V = float;
};

template <typename T>
__device__ __forceinline__ typename Lane<T>::V fv(typename Lane<T>::V a, typename Lane<T>::V b) {
  if constexpr (VT<T>::INT)
    return f_opi(a, b);
  else
    return f_op(a, b);
}
template <typename T>
__device__ __forceinline__ typename Lane<T>::V gv(typename Lane<T>::V a, typename Lane<T>::V b,
                                                  uint32_t s) {
  if constexpr (VT<T>::INT)
    return g_opi<VT<T>::Q>(a, b, s);
  else
    return g_op(a, b, s);
}
template <typename T>
__device__ __forceinline__ typename VT<T>::Acc magv(typename Lane<T>::V v) {
  if constexpr (VT<T>::INT)
    return abs(v);
  else
    return fabsf(v);
}

// Near-tie test of a selection (float32): the kept candidate's metric lo and
// the best rejected one's hi (lo <= hi) within 1e-4 relative, in double.
__device__ __forceinline__ uint32_t tie_gap(float lo, float hi) {
  return (double)hi - (double)lo <= 1e-4 * fmax(1.0, fabs((double)lo)) ? 1u : 0u;
}

// Decision of a REP node at L = 1: the all-one candidate wins only when its
// metric is strictly smaller.  Returns v and updates the (float) metric and
// near-tie flag.
template <typename T>
__device__ __forceinline__ uint32_t rep_decide(typename VT<T>::Acc p0, typename VT<T>::Acc p1,
                                               typename VT<T>::Acc& pm, uint32_t& tie) {
  if constexpr (VT<T>::INT) {
    const int q0 = min(p0, VT<T>::Q), q1 = min(p1, VT<T>::Q);
    return q1 < q0 ? 1u : 0u;
  } else {
    const float a0 = pm + p0, a1 = pm + p1;
    const uint32_t v = a1 < a0 ? 1u : 0u;
    pm = v ? a1 : a0;
    tie |= v ? tie_gap(a1, a0) : tie_gap(a0, a1);
    return v;
  }
}

// Float32 near-tie of a Rate-1 node or information leaf at L = 1 (metric pm
// before the node): the hard decision (penalty 0) against the Chase flip of
// the least reliable position (penalty mn = its |alpha|).
__device__ __forceinline__ uint32_t r1_tie(float pm, float mn) { return tie_gap(pm + 0.f, pm + mn); }
// ... of an SPC node: with even parity the hard decision against the flip of
// the two least reliable positions (m1 <= m2); with odd parity the flip of the
// least reliable against that of the second.
__device__ __forceinline__ uint32_t spc_tie(float pm, uint32_t odd, float m1, float m2) {
  return odd ? tie_gap(pm + m1, pm + m2) : tie_gap(pm + 0.f, pm + ((0.f + m1) + m2));
}

// Butterfly reduction over aligned segments of M <= 32 lanes (stride-halving
// order for sums); every lane of a segment ends with its segment's result.
template <typename A>
__device__ __forceinline__ A seg_sum(A v, uint32_t M, uint32_t lane) {
  for (uint32_t s = M >> 1; s >= 1; s >>= 1) v = v + bperm(v, lane ^ s);
  return v;
}
__device__ __forceinline__ uint64_t bperm64(uint64_t v, uint32_t src) {
  return ((uint64_t)bperm((uint32_t)(v >> 32), src) << 32) | bperm((uint32_t)v, src);
}
__device__ __forceinline__ uint64_t seg_min64(uint64_t v, uint32_t M, uint32_t lane) {
  for (uint32_t s = M >> 1; s >= 1; s >>= 1) {
    const uint64_t o = bperm64(v, lane ^ s);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ float seg_minf(float v, uint32_t M, uint32_t lane) {
  for (uint32_t s = M >> 1; s >= 1; s >>= 1) v = fminf(v, bperm(v, lane ^ s));
  return v;
}
// The two smallest magnitudes (m1 <= m2) over aligned segments of M lanes,
// each lane offering the key k = (|alpha| bits << 6) | position (unique per
// position; ~0 for none): every lane ends with its segment's pair.
__device__ __forceinline__ void seg_two_smallest(uint64_t k, uint32_t M, uint32_t lane, float& m1,
                                                 float& m2) {
  const uint64_t k1 = seg_min64(k, M, lane);
  const uint64_t k2 = seg_min64(k == k1 ? ~0ull : k, M, lane);
  m1 = __uint_as_float((uint32_t)(k1 >> 6));
  m2 = __uint_as_float((uint32_t)(k2 >> 6));
}
// bits of the calling lane's half in a wave ballot
__device__ __forceinline__ uint32_t half_bits(uint64_t bal, uint32_t hb) {
  return (uint32_t)(bal >> hb);
}

// ------------------------------------------------------- register levels
template <typename T>
struct Regs {
  typename Lane<T>::V xs, x5, x6a, x6b;  // LLRs: levels 0..4, 5, 6 (elements l, l + 32)
  uint32_t bs, b5, b6a, b6b;             // partial sums of the last finished nodes
  uint32_t ls, l6, l7a, l7b;             // left children of the nodes being decoded
  uint32_t tie;                          // float32: a decision of the frame was a near-tie
};

template <typename T>
__device__ __forceinline__ void reg_load_root(uint32_t K, Regs<T>& R, const char* fs, uint32_t l) {
  using V = typename Lane<T>::V;
  const T* root = reinterpret_cast<const T*>(fs);
  const uint32_t M = 1u << K, j = l - M;
  V a = (V)0, b = (V)0, c = (V)0;
  if (K >= 5) a = (V)root[l];
  if (K == 6) b = (V)root[l + 32];
  if (K < 5 && j < M) c = (V)root[j];
  R.x6a = K == 6 ? a : R.x6a;
  R.x6b = K == 6 ? b : R.x6b;
  R.x5 = K == 5 ? a : R.x5;
  R.xs = (K < 5 && j < M) ? c : R.xs;
}

template <typename T>
__device__ __forceinline__ void reg_store_root(uint32_t K, Regs<T>& R, char* fs, uint32_t N,
                                               uint32_t lane) {
  const uint32_t hb = lane & 32u, l = lane & 31u;
  uint32_t* bits = reinterpret_cast<uint32_t*>(fs + sc_bits_off(N, VT<T>::E));
  if (K == 6) {
    const uint32_t w0 = half_bits(__ballot(R.b6a & 1u), hb), w1 = half_bits(__ballot(R.b6b & 1u), hb);
    if (l < 2) bits[l] = l ? w1 : w0;
  } else {
    const uint32_t M = 1u << K;
    const uint32_t w = K == 5 ? half_bits(__ballot(R.b5 & 1u), hb)
                              : (half_bits(__ballot(R.bs & 1u), hb) >> M) & ((1u << M) - 1u);
    if (l == 0) bits[0] = w;
  }
}

// f (G = false) or g (G = true) at level K <= 6: the child (level K - 1)
// gets element i from the node's elements i and i + 2^(K-1).
template <typename T, bool G>
__device__ __forceinline__ void reg_fg(uint32_t K, Regs<T>& R, uint32_t lane) {
  using V = typename Lane<T>::V;
  if (K == 6) {
    if constexpr (!G) {
      R.x5 = fv<T>(R.x6a, R.x6b);
    } else {
      R.x5 = gv<T>(R.x6a, R.x6b, R.b5 & 1u);
      R.l6 = R.b5;
    }
    return;
  }
  const uint32_t hb = lane & 32u, l = lane & 31u;
  const uint32_t M = 1u << K, h = M >> 1;
  const V x5v = R.x5, xsv = R.xs;  // values, not an lvalue select (keeps R in registers)
  const V x = K == 5 ? x5v : xsv;
  const uint32_t src = hb + (K == 5 ? 0u : M) + ((l - h) & (h - 1));
  const V a = bperm(x, src);
  const V b = bperm(x, src + h);
  const bool child = l - h < h;  // lanes [h, 2h) of the half: level K - 1
  if constexpr (!G) {
    const V y = fv<T>(a, b);
    if (child) R.xs = y;
  } else {
    // the left child's partial sums sit in the same lanes (level K - 1)
    const V y = gv<T>(a, b, R.bs & 1u);
    if (child) {
      R.xs = y;
      R.ls = R.bs;
    }
  }
}

// h at level K <= 6: beta_K[i] = left[i] ^ beta_{K-1}[i], beta_K[i + h] = beta_{K-1}[i]
template <typename T>
__device__ __forceinline__ void reg_h(uint32_t K, Regs<T>& R, uint32_t lane) {
  if (K == 6) {
    R.b6a = (R.l6 ^ R.b5) & 1u;
    R.b6b = R.b5;
    return;
  }
  const uint32_t hb = lane & 32u, l = lane & 31u;
  const uint32_t M = 1u << K, h = M >> 1;
  const uint32_t j = l - (K == 5 ? 0u : M);
  const uint32_t pk = (R.bs & 1u) | (((R.ls ^ R.bs) & 1u) << 1);
  const uint32_t g = bperm(pk, hb + h + (j & (h - 1)));
  const uint32_t v = j < h ? (g >> 1) : (g & 1u);
  // value selects, never a store through a selected field address (which
  // would keep R in scratch memory)
  R.b5 = K == 5 ? v : R.b5;
  R.bs = (K != 5 && j < M) ? v : R.bs;
}

// A dedicated node or leaf of size 64 (elements l and l + 32 of the half).
template <typename T>
__device__ __forceinline__ void node64(uint32_t opc, Regs<T>& R, typename VT<T>::Acc& pm,
                                       uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  const uint32_t hb = lane & 32u, l = lane & 31u;
  const V xa = R.x6a, xb = R.x6b;
  const bool na = xa < (V)0, nb = xb < (V)0;
  const Acc ma = magv<T>(xa), mb = magv<T>(xb);
  const Acc pm0 = pm;  // the metric before the node
  uint32_t ba = na ? 1u : 0u, bb = nb ? 1u : 0u;
  if (opc == OP_SPC) {
    const uint64_t pa = __ballot(na), pb = __ballot(nb);
    const uint32_t odd0 = (__popc((uint32_t)pa) + __popc((uint32_t)pb)) & 1u;
    const uint32_t odd1 = (__popc((uint32_t)(pa >> 32)) + __popc((uint32_t)(pb >> 32))) & 1u;
    const uint32_t odd = hb ? odd1 : odd0;
    if constexpr (!VT<T>::INT) {
      // the two least reliable of the 64 positions (two per lane)
      const uint64_t ka = ((uint64_t)__float_as_uint(ma) << 6) | l;
      const uint64_t kb = ((uint64_t)__float_as_uint(mb) << 6) | (l + 32);
      const uint64_t k1 = seg_min64(ka < kb ? ka : kb, 32, lane);
      const uint64_t k2 = seg_min64(ka == k1 ? kb : (kb == k1 ? ka : (ka < kb ? ka : kb)), 32, lane);
      R.tie |= spc_tie(pm0, odd, __uint_as_float((uint32_t)(k1 >> 6)),
                       __uint_as_float((uint32_t)(k2 >> 6)));
    }
    if (odd0 | odd1) {
      uint64_t ka, kb;
      if constexpr (VT<T>::INT) {
        ka = ((uint64_t)(uint32_t)ma << 6) | l;
        kb = ((uint64_t)(uint32_t)mb << 6) | (l + 32);
      } else {
        ka = ((uint64_t)__float_as_uint(ma) << 6) | l;
        kb = ((uint64_t)__float_as_uint(mb) << 6) | (l + 32);
      }
      const uint64_t key = seg_min64(ka < kb ? ka : kb, 32, lane);
      const uint32_t idx = (uint32_t)key & 63u;
      if (odd) {
        if (idx == l) ba ^= 1u;
        if (idx == l + 32) bb ^= 1u;
      }
      if constexpr (!VT<T>::INT) pm = pm + (odd ? __uint_as_float((uint32_t)(key >> 6)) : 0.f);
    } else if constexpr (!VT<T>::INT) {
      pm = pm + 0.f;
    }
  } else if (opc == OP_REP) {
    // stride-halving: element i + 32 onto i first, then across the lanes
    const Acc p0 = seg_sum<Acc>((na ? ma : (Acc)0) + (nb ? mb : (Acc)0), 32, lane);
    const Acc p1 = seg_sum<Acc>((na ? (Acc)0 : ma) + (nb ? (Acc)0 : mb), 32, lane);
    ba = bb = rep_decide<T>(p0, p1, pm, R.tie);
  } else if (opc == OP_R0 || opc == OP_LF) {
    ba = bb = 0;
    if constexpr (!VT<T>::INT) {
      const float pen = seg_sum<float>((na ? ma : 0.f) + (nb ? mb : 0.f), 32, lane);
      pm = pm + pen;
    }
  } else if constexpr (!VT<T>::INT) {
    // Rate-1: the hard decision against the flip of the least reliable
    R.tie |= r1_tie(pm0, seg_minf(fminf(ma, mb), 32, lane));
  }
  R.b6a = ba;
  R.b6b = bb;
}

// A dedicated node or leaf at level K <= 6.
template <typename T>
__device__ __forceinline__ void reg_node(uint32_t opc, uint32_t K, Regs<T>& R,
                                         typename VT<T>::Acc& pm, uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  if (K == 6) {
    node64<T>(opc, R, pm, lane);
    return;
  }
  const uint32_t hb = lane & 32u, l = lane & 31u;
  const uint32_t M = 1u << K, base = K == 5 ? 0u : M, j = l - base;
  const bool in = j < M;
  const uint32_t first = hb + base;  // the node's first lane in this half
  const V x5v = R.x5, xsv = R.xs;  // values, not an lvalue select (keeps R in registers)
  const V x = K == 5 ? x5v : xsv;
  const bool neg = x < (V)0;
  const Acc mg = magv<T>(x);
  const Acc pm0 = pm;  // the metric before the node
  uint32_t bit = neg ? 1u : 0u;  // Rate-1 / information leaf: the hard decision
  if (opc == OP_SPC) {
    const uint64_t hd = __ballot(in && neg);
    const uint32_t odd0 = __popc((uint32_t)hd) & 1u, odd1 = __popc((uint32_t)(hd >> 32)) & 1u;
    const uint32_t odd = hb ? odd1 : odd0;
    if constexpr (!VT<T>::INT) {
      float m1, m2;
      seg_two_smallest(in ? (((uint64_t)__float_as_uint(mg) << 6) | j) : ~0ull, M, lane, m1, m2);
      R.tie |= spc_tie(pm0, odd, bperm(m1, first), bperm(m2, first));
    }
    if (odd0 | odd1) {
      // least reliable position (smallest |alpha|, then smallest index)
      uint64_t key;
      if constexpr (VT<T>::INT)
        key = in ? (((uint64_t)(uint32_t)mg << 6) | j) : ~0ull;
      else
        key = in ? (((uint64_t)__float_as_uint(mg) << 6) | j) : ~0ull;
      key = bperm64(seg_min64(key, M, lane), first);
      if (odd && j == ((uint32_t)key & 63u)) bit ^= 1u;
      if constexpr (!VT<T>::INT) pm = pm + (odd ? __uint_as_float((uint32_t)(key >> 6)) : 0.f);
    } else if constexpr (!VT<T>::INT) {
      pm = pm + 0.f;
    }
  } else if (opc == OP_REP) {
    const Acc p0 = bperm(seg_sum<Acc>(in && neg ? mg : (Acc)0, M, lane), first);
    const Acc p1 = bperm(seg_sum<Acc>(in && !neg ? mg : (Acc)0, M, lane), first);
    bit = rep_decide<T>(p0, p1, pm, R.tie);
  } else if (opc == OP_R0 || opc == OP_LF) {
    bit = 0;
    if constexpr (!VT<T>::INT) pm = pm + bperm(seg_sum<float>(in && neg ? mg : 0.f, M, lane), first);
  } else if constexpr (!VT<T>::INT) {
    // Rate-1 or information leaf: the hard decision against the flip of the
    // least reliable position
    R.tie |= r1_tie(pm0, bperm(seg_minf(in ? mg : __int_as_float(0x7f800000), M, lane), first));
  }
  R.b5 = K == 5 ? bit : R.b5;
  R.bs = (K != 5 && in) ? bit : R.bs;
}

// ------------------------------------------------------------ LDS levels
// Node of size m = 2^k >= 128 at depth d of the frame whose LDS region is
// fs: its LLRs are the root (d = 0) or the depth-d stage buffer.  Lane l of
// the half holds elements l, l + 32, ...
typedef __attribute__((address_space(1))) const uint32_t gword;  // global memory

template <typename T>
__device__ __forceinline__ void lds_op(char* fs, uint32_t N, uint32_t gr, const char* llr,
                                       uint32_t opc, uint32_t d, uint32_t k, uint32_t o,
                                       Regs<T>& R, typename VT<T>::Acc& pm, uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  constexpr uint32_t E = VT<T>::E, PER = 4 / E;  // elements per 32-bit word
  const uint32_t hb = lane & 32u, l = lane & 31u;
  const uint32_t m = 1u << k, h = m >> 1;
  const T* src = reinterpret_cast<const T*>(fs + (d ? sc_stage_base(N, d, E, gr) : 0u));
  uint32_t* bits = reinterpret_cast<uint32_t*>(fs + sc_bits_off(N, E, gr));
  if (d == 0 && gr && (opc == OP_F || opc == OP_G)) {
    // f / g of the root straight from the channel LLRs in global memory
    // (the root of such codes has N >= 256, so its child stays in LDS)
    gword* sa = (gword*)(llr);
    gword* sb = (gword*)(llr + h * E);
    uint32_t* dst = reinterpret_cast<uint32_t*>(fs + sc_stage_base(N, 1, E, gr));
    for (uint32_t q = l; q < h / PER; q += 32) {
      const uint32_t wa = sa[q], wb = sb[q];
      uint32_t wo = 0;
      if (opc == OP_F) {
        f_chunk<T, PER>(&wa, &wb, &wo);
      } else {
        const uint32_t bp = o + q * PER;
        g_chunk<T, PER>(&wa, &wb, bits[bp >> 5] >> (bp & 31), &wo);
      }
      dst[q] = wo;
    }
    __syncthreads();
    return;
  }
  if (opc == OP_F || opc == OP_G) {
    if (k == 7) {
      // the child (size 64) goes to registers: elements l and l + 32
      const V a0 = (V)src[l], b0 = (V)src[l + 64], a1 = (V)src[l + 32], b1 = (V)src[l + 96];
      if (opc == OP_F) {
        R.x6a = fv<T>(a0, b0);
        R.x6b = fv<T>(a1, b1);
      } else {
        R.l7a = R.b6a;
        R.l7b = R.b6b;
        R.x6a = gv<T>(a0, b0, R.b6a & 1u);
        R.x6b = gv<T>(a1, b1, R.b6b & 1u);
      }
      return;
    }
    const uint32_t* sa = reinterpret_cast<const uint32_t*>(src);
    const uint32_t* sb = reinterpret_cast<const uint32_t*>(src + h);
    uint32_t* dst = reinterpret_cast<uint32_t*>(fs + sc_stage_base(N, d + 1, E, gr));
    for (uint32_t q = l; q < h / PER; q += 32) {
      const uint32_t wa = sa[q], wb = sb[q];
      uint32_t wo = 0;
      if (opc == OP_F) {
        f_chunk<T, PER>(&wa, &wb, &wo);
      } else {
        const uint32_t bp = o + q * PER;
        g_chunk<T, PER>(&wa, &wb, bits[bp >> 5] >> (bp & 31), &wo);
      }
      dst[q] = wo;
    }
    __syncthreads();
    return;
  }
  if (opc == OP_H) {
    if (k == 7) {
      // beta_7 = [left_7 ^ beta_6, beta_6], one word per 32 elements
      const uint64_t B0 = __ballot((R.l7a ^ R.b6a) & 1u), B1 = __ballot((R.l7b ^ R.b6b) & 1u);
      const uint64_t B2 = __ballot(R.b6a & 1u), B3 = __ballot(R.b6b & 1u);
      if (l < 4) {
        const uint64_t v = l == 0 ? B0 : (l == 1 ? B1 : (l == 2 ? B2 : B3));
        bits[(o >> 5) + l] = half_bits(v, hb);
      }
    } else {
      for (uint32_t q = l; q < (h >> 5); q += 32) bits[(o >> 5) + q] ^= bits[((o + h) >> 5) + q];
    }
    __syncthreads();
    return;
  }
  // dedicated node of size m >= 128
  const uint32_t epl = m >> 5, he = epl >> 1;
  uint32_t* nb = bits + (o >> 5);
  if (opc == OP_R0) {
    for (uint32_t q = l; q < epl; q += 32) nb[q] = 0u;
    if constexpr (!VT<T>::INT) {
      // stride-halving: the first level (element t + epl/2 onto t) while loading
      float x[32];
#pragma unroll
      for (uint32_t t = 0; t < 32; ++t) {
        if (t < he) {
          const float v0 = src[l + (t << 5)], v1 = src[l + ((t + he) << 5)];
          x[t] = (v0 < 0.f ? fabsf(v0) : 0.f) + (v1 < 0.f ? fabsf(v1) : 0.f);
        }
      }
#pragma unroll
      for (uint32_t S = 16; S >= 1; S >>= 1)
        if (S < he) {
#pragma unroll
          for (uint32_t t = 0; t < S; ++t) x[t] = x[t] + x[t + S];
        }
      pm = pm + seg_sum<float>(x[0], 32, lane);
    }
    __syncthreads();
    return;
  }
  if (opc == OP_R1 || opc == OP_SPC) {
    uint32_t par = 0, w_lo = 0, w_hi = 0;
    uint64_t key = ~0ull, key2 = ~0ull;  // the lane's two least reliable (float32 near-tie)
    const Acc pm0 = pm;
    for (uint32_t t = 0; t < epl; ++t) {
      const uint32_t e = l + (t << 5);
      const V v = (V)src[e];
      const uint32_t w = half_bits(__ballot(v < (V)0), hb);  // hard decisions of elements 32t..
      par ^= (uint32_t)__popc(w) & 1u;
      if (l == (t & 31u)) {
        if (t < 32)
          w_lo = w;
        else
          w_hi = w;
      }
      if constexpr (VT<T>::INT) {
        if (opc == OP_SPC) {
          const uint64_t kk = ((uint64_t)(uint32_t)abs(v) << 16) | e;
          key = kk < key ? kk : key;
        }
      } else {
        const uint64_t kk = ((uint64_t)__float_as_uint(fabsf(v)) << 16) | e;
        key2 = kk < key ? key : (kk < key2 ? kk : key2);
        key = kk < key ? kk : key;
      }
    }
    if constexpr (!VT<T>::INT) {
      const uint64_t k1 = seg_min64(key, 32, lane);
      const uint64_t k2 = seg_min64(key == k1 ? key2 : key, 32, lane);
      const float m1 = __uint_as_float((uint32_t)(k1 >> 16)), m2 = __uint_as_float((uint32_t)(k2 >> 16));
      R.tie |= opc == OP_SPC ? spc_tie(pm0, par, m1, m2) : r1_tie(pm0, m1);
    }
    if (l < epl) nb[l] = w_lo;
    if (l + 32 < epl) nb[l + 32] = w_hi;
    if (opc == OP_SPC) {
      if (__ballot(par != 0)) {
        key = seg_min64(key, 32, lane);
        const uint32_t idx = (uint32_t)key & 0xFFFFu;
        __syncthreads();
        if (par && l == 0) nb[idx >> 5] ^= 1u << (idx & 31);
        if constexpr (!VT<T>::INT) pm = pm + (par ? __uint_as_float((uint32_t)(key >> 16)) : 0.f);
      } else if constexpr (!VT<T>::INT) {
        pm = pm + 0.f;
      }
    }
    __syncthreads();
    return;
  }
  // OP_REP of size >= 128
  Acc p0, p1;
  if constexpr (VT<T>::INT) {
    int a0 = 0, a1 = 0;
    for (uint32_t t = 0; t < epl; ++t) {
      const int v = src[l + (t << 5)];
      if (v < 0)
        a0 += -v;
      else
        a1 += v;
    }
    p0 = seg_sum<int>(a0, 32, lane);
    p1 = seg_sum<int>(a1, 32, lane);
  } else {
    float x0[32], x1[32];
#pragma unroll
    for (uint32_t t = 0; t < 32; ++t) {
      if (t < he) {
        const float v0 = src[l + (t << 5)], v1 = src[l + ((t + he) << 5)];
        x0[t] = (v0 < 0.f ? fabsf(v0) : 0.f) + (v1 < 0.f ? fabsf(v1) : 0.f);
        x1[t] = (v0 < 0.f ? 0.f : fabsf(v0)) + (v1 < 0.f ? 0.f : fabsf(v1));
      }
    }
#pragma unroll
    for (uint32_t S = 16; S >= 1; S >>= 1)
      if (S < he) {
#pragma unroll
        for (uint32_t t = 0; t < S; ++t) {
          x0[t] = x0[t] + x0[t + S];
          x1[t] = x1[t] + x1[t + S];
        }
      }
    p0 = seg_sum<float>(x0[0], 32, lane);
    p1 = seg_sum<float>(x1[0], 32, lane);
  }
  const uint32_t v = rep_decide<T>(p0, p1, pm, R.tie);
  for (uint32_t q = l; q < epl; q += 32) nb[q] = v ? ~0u : 0u;
  __syncthreads();
}

__device__ __forceinline__ void frame_at(const KArgs& A, uint32_t f, const DevPlan*& P,
                                         const char*& llr, uint32_t& out_off) {
  if (A.frames) {
    const polar_frame fr = A.frames[f];
    P = A.plans[fr.plan_idx];
    llr = A.llr + fr.llr_off;
    out_off = fr.out_off;
  } else {
    P = A.plans[0];
    llr = A.llr + (size_t)f * A.llr_bytes;
    out_off = f * A.info_words;
  }
}

// Whether this tier decodes a frame of plan P: its class (class schedule),
// else a plan whose schedule starts at L = 1 (a list tier starts the others;
// their state already holds the first stage).
__device__ __forceinline__ bool sc_takes(const DevPlan* P, const ClassSel& sel) {
  if (sel.on)
    return P->first_stage >= sel.lmin && P->first_stage <= sel.lmax && P->N >= sel.nmin &&
           P->N <= sel.nmax && P->quant == sel.quant;
  return P->first_stage == 1;
}

// Decode plan P for the frame of each half (on: this half has one).
template <typename T>
__device__ void decode_pair(const KArgs& A, uint32_t* state, const ClassSel& sel,
                            const DevPlan* P, uint32_t f, const char* llr, uint32_t out_off,
                            bool on, char* smem, uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  constexpr uint32_t E = VT<T>::E;
  const uint32_t hb = lane & 32u, l = lane & 31u;
  P = uni_ptr(P);
  const uint32_t N = uni(P->N), n = uni(P->n), ntx = uni(P->n_tx), n_ops = uni(P->n_sc_ops),
                 np = uni(P->n_punct);
  const uint32_t* prog = uni_ptr(plan_tab(P, uni(P->off_sc_prog)));
  const uint32_t gr = A.sc_groot;
  char* fs = smem + (hb ? sc_lds_bytes(N, E, gr) : 0u);  // this frame's LDS region
  if (on && l == 0 && A.times) A.times[2 * (size_t)f] = wall_clock64();
  // ---- channel LLRs -> root: punctured head [0, P) received nothing (0),
  // sent positions [P, P + n_tx), shortened tail a zero known for certain
  T* root = reinterpret_cast<T*>(fs);
  if (on && !gr) {
    const uint32_t nbytes = ntx * E;
    if ((((uintptr_t)llr) & 15u) == 0 && (nbytes & 15u) == 0 && ((np * E) & 15u) == 0) {
      const uint4* s4 = reinterpret_cast<const uint4*>(llr);
      uint4* d4 = reinterpret_cast<uint4*>(root + np);
      for (uint32_t i = l; i < (nbytes >> 4); i += 32) d4[i] = s4[i];
    } else {
      const T* s1 = reinterpret_cast<const T*>(llr);
      for (uint32_t i = l; i < ntx; i += 32) root[np + i] = s1[i];
    }
    for (uint32_t i = l; i < np; i += 32) root[i] = (T)0;
    const T known = VT<T>::INT ? (T)VT<T>::Q : (T)1048576.0f;
    for (uint32_t i = np + ntx + l; i < N; i += 32) root[i] = known;
  }
  __syncthreads();

  Regs<T> R;
  R.xs = R.x5 = R.x6a = R.x6b = (V)0;
  R.bs = R.b5 = R.b6a = R.b6b = R.ls = R.l6 = R.l7a = R.l7b = 0u;
  R.tie = 0u;
  Acc pm = (Acc)0;
  if (N <= 64) reg_load_root<T>(n, R, fs, l);  // whole code in registers
  // the next op word is fetched while the current op runs
  uint32_t w_next = n_ops ? prog[0] : 0u;
  for (uint32_t pc = 0; pc < n_ops; ++pc) {
    const uint32_t w = uni(w_next);
    if (pc + 1 < n_ops) w_next = prog[pc + 1];
    const uint32_t opc = op_code(w), d = op_depth(w), k = n - d;
    // an if-chain in op frequency order (fused steps, f, g, h, nodes) keeps
    // the uniform control flow free of the structurizer's flag variables
    if (opc == OP_GNH) {
      // g, the right child (a node at level k - 1 <= 6), h
      if (k >= 7)
        lds_op<T>(fs, N, gr, llr, OP_G, d, k, op_off(w), R, pm, lane);
      else
        reg_fg<T, true>(k, R, lane);
      reg_node<T>(op_sub(w), k - 1, R, pm, lane);
      if (k >= 7)
        lds_op<T>(fs, N, gr, llr, OP_H, d, k, op_off(w), R, pm, lane);
      else
        reg_h<T>(k, R, lane);
    } else if (opc == OP_FN) {
      // f, the left child (a node at level k - 1 <= 6)
      if (k >= 7)
        lds_op<T>(fs, N, gr, llr, OP_F, d, k, op_off(w), R, pm, lane);
      else
        reg_fg<T, false>(k, R, lane);
      reg_node<T>(op_sub(w), k - 1, R, pm, lane);
    } else if (k >= 7) {
      lds_op<T>(fs, N, gr, llr, opc, d, k, op_off(w), R, pm, lane);
    } else if (opc == OP_F) {
      reg_fg<T, false>(k, R, lane);
    } else if (opc == OP_G) {
      reg_fg<T, true>(k, R, lane);
    } else if (opc == OP_H) {
      reg_h<T>(k, R, lane);
    } else {
      reg_node<T>(opc, k, R, pm, lane);
    }
  }
  // ---- codeword estimate in LDS bits (small codes: from the root level)
  uint32_t* bits = reinterpret_cast<uint32_t*>(fs + sc_bits_off(N, E, gr));
  if (N <= 64) reg_store_root<T>(n, R, fs, N, lane);
  __syncthreads();
  // ---- CRC syndrome through the nibble table, per half
  const uint32_t bw = uni(P->bw);
  uint32_t syn = 0;
  if (uni(P->c) > 0) {
    const uint32_t* imask = plan_tab(P, uni(P->off_infomask));
    const uint32_t* nib = plan_tab(P, uni(P->off_crcnib));
    const uint32_t nq = N >= 32 ? 8u : (N + 3) / 4;
    for (uint32_t w = l; w < bw; w += 32) {
      const uint32_t v = bits[w] & imask[w];
      for (uint32_t q = 0; q < nq; ++q) syn ^= nib[((w * 8 + q) << 4) + ((v >> (4 * q)) & 15u)];
    }
  }
  for (uint32_t s = 16; s >= 1; s >>= 1) syn ^= bperm(syn, lane ^ s);
  const bool ok = syn == 0u;
  // a frame of an adaptive plan whose L = 1 decision fails goes to the list tiers
  const uint32_t L_max = uni(P->L_max);
  const bool esc = on && !ok && L_max > 1 && !sel.on;
  if (esc && l == 0) state[f] = next_stage(P, 1) | (R.tie << 8);
  const bool fin = on && !esc;
  // ---- outputs: information bits (data positions of A, ascending)
  uint32_t* out = reinterpret_cast<uint32_t*>(fs + sc_out_off(N, E, gr));
  const uint32_t iw = uni(P->info_words);
  const uint32_t* dmask = plan_tab(P, uni(P->off_datamask));
  const uint32_t* dpre = plan_tab(P, uni(P->off_dataprefix));
  if (fin)
    for (uint32_t q = l; q < iw; q += 32) out[q] = 0u;
  __syncthreads();
  if (fin) {
    for (uint32_t w = l; w < bw; w += 32) {
      const uint32_t x = bits[w];
      uint32_t dm = dmask[w];
      const uint32_t pre = dpre[w];
      uint32_t v = 0, cnt = 0;
      while (dm) {
        const uint32_t b = __ffs(dm) - 1;
        v |= ((x >> b) & 1u) << cnt;
        ++cnt;
        dm &= dm - 1u;
      }
      if (cnt) {
        atomicOr(&out[pre >> 5], v << (pre & 31));
        if ((pre & 31) + cnt > 32) atomicOr(&out[(pre >> 5) + 1], v >> (32 - (pre & 31)));
      }
    }
  }
  __syncthreads();
  if (fin) {
    for (uint32_t q = l; q < iw; q += 32) A.info[out_off + q] = out[q];
    if (l == 0) {
      polar_status st;
      st.crc_ok = ok ? 1 : 0;
      st.L_used = 1;
      st.n_paths = 1;
      st.flags = (uint8_t)R.tie;
      if constexpr (VT<T>::INT)
        st.pm = 0u;
      else
        st.pm = __float_as_uint(pm);
      A.status[f] = st;
      if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
    }
    if (A.pm_lists) {
      for (uint32_t t = l; t < A.pm_stride; t += 32)
        A.pm_lists[(size_t)f * A.pm_stride + t] =
            t == 0 ? (VT<T>::INT ? 0u : __float_as_uint((float)pm)) : 0xFFFFFFFFu;
    }
  }
  __syncthreads();
}

}  // namespace

// One wave per pair of frames (2p, 2p + 1).  Tiered schedule (sel off): only
// frames whose plan starts at L = 1 are decoded here; a frame of an adaptive
// plan whose L = 1 decision fails the CRC gets its next list size in
// state[f] (the list tiers pick it up); every other decoded frame is
// finished here (its state keeps the value 1, which no list tier takes).
// Class schedule (sel on): only the frames of the class, no state.  Two
// frames of one plan share a pass; otherwise each gets a pass of its own
// with the other half idle.
// Occupancy: the integer kernels are held to 64 VGPRs (8 waves per SIMD; a
// few values spill, which costs less than the latency it hides); float32
// keeps its registers.
template <typename T>
__global__ __launch_bounds__(64, (VT<T>::INT ? 8 : 1)) void k_sc(KArgs A, uint32_t* state,
                                                               ClassSel sel) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const uint32_t lane = threadIdx.x, half = lane >> 5;
  const uint32_t n_pairs = (A.n_frames + 1) / 2;
  for (uint32_t pr = blockIdx.x; pr < n_pairs; pr += gridDim.x) {
    const uint32_t f0 = 2 * pr, f1 = 2 * pr + 1;
    const DevPlan *P0, *P1 = nullptr;
    const char *llr0, *llr1 = nullptr;
    uint32_t oo0, oo1 = 0;
    frame_at(A, f0, P0, llr0, oo0);
    const bool act0 = sc_takes(P0, sel);
    bool act1 = false;
    if (f1 < A.n_frames) {
      frame_at(A, f1, P1, llr1, oo1);
      act1 = sc_takes(P1, sel);
    }
    const bool together = act0 && act1 && P0 == P1;
    for (uint32_t pass = 0; pass < 2; ++pass) {
      bool on0, on1;
      if (together) {
        if (pass) break;
        on0 = on1 = true;
      } else {
        on0 = pass == 0 && act0;
        on1 = pass == 1 && act1;
      }
      if (!on0 && !on1) continue;
      // an idle half reads the active frame's LLRs (its results are dropped)
      const char* act_llr = on0 ? llr0 : llr1;
      const bool on = half ? on1 : on0;
      decode_pair<T>(A, state, sel, on0 ? P0 : P1, half ? f1 : f0,
                     on ? (half ? llr1 : llr0) : act_llr, half ? oo1 : oo0, on, smem, lane);
    }
  }
}

// `grid` and `lds`: one per frame (sc_lds_bytes); the kernel runs a wave per
// pair of frames with both frames' regions.
template <typename T>
static int launch_sc_t(const KArgs& A, uint32_t lds, uint32_t grid, uint32_t* state,
                       const ClassSel& sel, hipStream_t s) {
  const uint32_t pairs = (grid + 1) / 2;
  hipLaunchKernelGGL(k_sc<T>, dim3(pairs > 0 ? pairs : 1), dim3(64), 2 * lds, s, A, state, sel);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_decode_sc(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid, uint32_t* state,
                     const ClassSel& sel, hipStream_t s) {
  switch (quant) {
    case POLAR_F32: return launch_sc_t<float>(A, lds, grid, state, sel, s);
    case POLAR_I16: return launch_sc_t<int16_t>(A, lds, grid, state, sel, s);
    default: return launch_sc_t<int8_t>(A, lds, grid, state, sel, s);
  }
}

int sc_set_attributes(int lds) {
  const void* ks[] = {(const void*)k_sc<float>, (const void*)k_sc<int16_t>,
                      (const void*)k_sc<int8_t>};
  for (const void* k : ks)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
      return POLAR_EHIP;
  return POLAR_OK;
}

}  // namespace polar
