// L = 1 tier of the decoder on gfx950: successive cancellation over the
// pruned tree (Sec. II-B1, II-B3) for every frame, one wave per frame, with
// the CRC check of the fully / partially adaptive schedules (Sec. II-B5) and
// a per-frame state word for the frames that need a list.
//
// A list of one path never forks, so this tier keeps no candidate lists, no
// path copies and no slot indirection.  Its layout follows the shape of the
// tree instead:
//   * nodes of size >= 128 keep their LLRs in LDS and use all 64 lanes;
//   * every subtree of size <= 64 runs in registers: the nodes of size
//     2^k <= 32 on the current path share one register, level k in lanes
//     [2^k, 2^(k+1)), the node of size 64 has a register of its own, and
//     partial sums are one bit per lane in the same places; an op at any
//     register level is one code path (operands move between levels by lane
//     permutation), so the op word is dispatched on its opcode alone;
//   * a dedicated node decides with a ballot (Rate-1: hard decision; SPC:
//     hard decision with the least reliable position flipped on odd parity)
//     or a lane reduction (REP: the two disagreement penalties).
// The decisions are those of a list of one under the selection rule of the
// list decoder (candidate key = metric, parent rank, local index): the
// hard-decision candidate wins a tie, the all-zero REP candidate wins a tie,
// and float32 metrics are summed in the stride-halving order.  Integer metrics
// are normalised after every update, so they stay 0 at L = 1; only the REP
// decision needs its saturated penalties.
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

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float rflf(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int rfli(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
  return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}


// Decision of a REP node at L = 1: the all-one candidate wins only when its
// metric is strictly smaller.  Returns v and updates the (float) metric.
template <typename T>
__device__ __forceinline__ uint32_t rep_decide(typename VT<T>::Acc p0, typename VT<T>::Acc p1,
                                               typename VT<T>::Acc& pm) {
  if constexpr (VT<T>::INT) {
    const int q0 = min(p0, VT<T>::Q), q1 = min(p1, VT<T>::Q);
    return q1 < q0 ? 1u : 0u;
  } else {
    const float a0 = pm + p0, a1 = pm + p1;
    const uint32_t v = a1 < a0 ? 1u : 0u;
    pm = v ? a1 : a0;
    return v;
  }
}

// Lane-shuffle stride-halving sum over the first `w` lanes (a power of two):
// lane i holds element i; the lanes below w end with the total.
template <typename A>
__device__ __forceinline__ A lanes_sum(A v, uint32_t w) {
  for (uint32_t s = w >> 1; s >= 1; s >>= 1) v = v + __shfl_xor(v, (int)s, 64);
  return v;
}

// ------------------------------------------------------- register levels
// The nodes of size 2^k <= 32 on the current root-to-leaf path keep their
// LLRs in one register, xs, in lanes [2^k, 2^(k+1)) (level k; levels 0..5
// fill lanes 1..63), the node of size 64 in x6 (lane i = element i).
// Partial sums are one bit per lane in the same places: bs (levels 0..5)
// and b6 hold the last finished node of each size, ls (lanes [2^(k-1), 2^k))
// the left child of the level-k node being decoded, l7 the left child (size
// 64) of the size-128 node.  An op at any register level is one code path
// with the level k as a run-time value; operands move between levels by
// lane permutation.
template <typename T>
struct Regs {
  typename Lane<T>::V xs, x6;
  uint32_t bs, b6, ls, l7;
};

// Sum over the segment of M lanes holding v (aligned to M), stride-halving
// order; every lane of the segment ends with the total.
template <typename A>
__device__ __forceinline__ A seg_sum(A v, uint32_t M, uint32_t lane) {
  for (uint32_t s = M >> 1; s >= 1; s >>= 1) v = v + bperm(v, lane ^ s);
  return v;
}
__device__ __forceinline__ float lane_f(float v, uint32_t l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)l));
}
__device__ __forceinline__ int lane_i(int v, uint32_t l) { return __builtin_amdgcn_readlane(v, (int)l); }

// Level K of the register levels: its first lane, and this lane's index in
// the node (valid below 2^K).
struct RegLevel {
  uint32_t M, base, j;
  bool top, in;
  __device__ __forceinline__ RegLevel(uint32_t K, uint32_t lane) {
    M = 1u << K;
    top = K == 6;
    base = top ? 0u : M;
    j = lane - base;
    in = j < M;
  }
};

template <typename T>
__device__ __forceinline__ void reg_load_root(uint32_t K, Regs<T>& R, uint32_t lane, char* smem) {
  using V = typename Lane<T>::V;
  const RegLevel lv(K, lane);
  const V v = lv.in ? (V)reinterpret_cast<const T*>(smem)[lv.j] : (V)0;
  if (lv.top)
    R.x6 = v;
  else if (lv.in)
    R.xs = v;
}

template <typename T>
__device__ __forceinline__ void reg_store_root(uint32_t K, Regs<T>& R, uint32_t lane, char* smem) {
  const RegLevel lv(K, lane);
  const uint64_t b = (uint64_t)__ballot((lv.top ? R.b6 : R.bs) & 1u);
  const uint64_t beta = lv.top ? b : ((b >> lv.M) & ((1ull << lv.M) - 1ull));
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem + sc_bits_off(lv.M, VT<T>::E));
  if (lane < 2) bits[lane] = lane ? (uint32_t)(beta >> 32) : (uint32_t)beta;
}

// f (G = false) or g (G = true) at level K: the child (level K - 1, lanes
// [h, 2h)) gets element i from the node's elements i and i + h.
template <typename T, bool G>
__device__ __forceinline__ void reg_fg(uint32_t K, Regs<T>& R, uint32_t lane) {
  using V = typename Lane<T>::V;
  const RegLevel lv(K, lane);
  const V x = lv.top ? R.x6 : R.xs;
  const uint32_t h = lv.M >> 1, i = (lane - h) & (h - 1);
  const V a = bperm(x, lv.base + i);
  const V b = bperm(x, lv.base + h + i);
  const bool child = lane - h < h;
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

// h at level K: beta_K[i] = left[i] ^ beta_{K-1}[i], beta_K[i + h] = beta_{K-1}[i]
template <typename T>
__device__ __forceinline__ void reg_h(uint32_t K, Regs<T>& R, uint32_t lane) {
  const RegLevel lv(K, lane);
  const uint32_t h = lv.M >> 1;
  const uint32_t pk = (R.bs & 1u) | (((R.ls ^ R.bs) & 1u) << 1);
  const uint32_t g = bperm(pk, h + (lv.j & (h - 1)));
  const uint32_t v = lv.j < h ? (g >> 1) : (g & 1u);
  if (lv.top)
    R.b6 = v;
  else if (lv.in)
    R.bs = v;
}

// A dedicated node or leaf at level K.
template <typename T>
__device__ __forceinline__ void reg_node(uint32_t opc, uint32_t K, Regs<T>& R,
                                         typename VT<T>::Acc& pm, uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  const RegLevel lv(K, lane);
  const uint32_t M = lv.M, base = lv.base, j = lv.j;
  const bool in = lv.in;
  const V x = lv.top ? R.x6 : R.xs;
  const bool neg = x < (V)0;
  const Acc mg = magv<T>(x);
  uint32_t bit = neg ? 1u : 0u;  // Rate-1 / information leaf: the hard decision
  if (opc == OP_SPC) {
    const uint64_t hd = (uint64_t)__ballot(in && neg);
    if (__popcll(hd) & 1) {
      // least reliable position (smallest |alpha|, then smallest index)
      uint64_t key;
      if constexpr (VT<T>::INT)
        key = in ? (((uint64_t)(uint32_t)mg << 6) | j) : ~0ull;
      else
        key = in ? (((uint64_t)__float_as_uint(mg) << 6) | j) : ~0ull;
      for (uint32_t s = M >> 1; s >= 1; s >>= 1) {
        const uint32_t src = lane ^ s;
        const uint64_t o = ((uint64_t)bperm((uint32_t)(key >> 32), src) << 32) |
                           bperm((uint32_t)key, src);
        key = o < key ? o : key;
      }
      const uint64_t kmin =
          ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(key >> 32), (int)base) << 32) |
          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, (int)base);
      if (j == ((uint32_t)kmin & 63u)) bit ^= 1u;
      if constexpr (!VT<T>::INT) pm = pm + __uint_as_float((uint32_t)(kmin >> 6));
    } else if constexpr (!VT<T>::INT) {
      pm = pm + 0.f;
    }
  } else if (opc == OP_REP) {
    Acc p0 = seg_sum<Acc>(in && neg ? mg : (Acc)0, M, lane);
    Acc p1 = seg_sum<Acc>(in && !neg ? mg : (Acc)0, M, lane);
    if constexpr (VT<T>::INT) {
      p0 = lane_i(p0, base);
      p1 = lane_i(p1, base);
    } else {
      p0 = lane_f(p0, base);
      p1 = lane_f(p1, base);
    }
    bit = rep_decide<T>(p0, p1, pm);
  } else if (opc == OP_R0 || opc == OP_LF) {
    bit = 0;
    if constexpr (!VT<T>::INT) {
      const float pen = lane_f(seg_sum<float>(in && neg ? mg : 0.f, M, lane), base);
      pm = pm + pen;
    }
  }
  if (lv.top)
    R.b6 = bit;
  else if (in)
    R.bs = bit;
}

// ------------------------------------------------------------ LDS levels
// Node of size m = 2^k >= 128 at depth d: its LLRs are the root (d = 0) or
// the depth-d stage buffer.
template <typename T>
__device__ __forceinline__ const T* lds_node(char* smem, uint32_t N, uint32_t d) {
  return reinterpret_cast<const T*>(smem + (d ? sc_stage_base(N, d, VT<T>::E) : 0u));
}

template <typename T>
__device__ __forceinline__ void lds_op(char* smem, uint32_t N, uint32_t opc, uint32_t d, uint32_t k, uint32_t o,
                       Regs<T>& R, typename VT<T>::Acc& pm, uint32_t lane) {
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  constexpr uint32_t E = VT<T>::E, PER = 4 / E;  // elements per 32-bit word
  const uint32_t m = 1u << k, h = m >> 1;
  const T* src = lds_node<T>(smem, N, d);
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem + sc_bits_off(N, E));
  if (opc == OP_F || opc == OP_G) {
    if (k == 7) {
      // the child (size 64) goes to registers: lane i holds element i
      const V a = (V)src[lane], b = (V)src[lane + 64];
      if (opc == OP_F) {
        R.x6 = fv<T>(a, b);
      } else {
        R.l7 = R.b6;
        R.x6 = gv<T>(a, b, R.b6 & 1u);
      }
      return;
    }
    const uint32_t* sa = reinterpret_cast<const uint32_t*>(src);
    const uint32_t* sb = reinterpret_cast<const uint32_t*>(src + h);
    uint32_t* dst = reinterpret_cast<uint32_t*>(smem + sc_stage_base(N, d + 1, E));
    for (uint32_t q = lane; q < h / PER; q += 64) {
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
      const uint64_t lo = (uint64_t)__ballot((R.l7 ^ R.b6) & 1u),
                     hi = (uint64_t)__ballot(R.b6 & 1u);
      const uint32_t w0 = o >> 5;
      if (lane < 4) {
        const uint64_t v = lane < 2 ? lo : hi;
        bits[w0 + lane] = (lane & 1) ? (uint32_t)(v >> 32) : (uint32_t)v;
      }
    } else {
      for (uint32_t q = lane; q < (h >> 5); q += 64) bits[(o >> 5) + q] ^= bits[((o + h) >> 5) + q];
    }
    __syncthreads();
    return;
  }
  // dedicated node of size m >= 128: lane j holds elements j, j + 64, ...
  const uint32_t epl = m >> 6;
  uint32_t* nb = bits + (o >> 5);
  if (opc == OP_R0) {
    for (uint32_t q = lane; q < (m >> 5); q += 64) nb[q] = 0u;
    if constexpr (!VT<T>::INT) {
      float x[32];
#pragma unroll
      for (uint32_t t = 0; t < 32; ++t) {
        if (t < epl) {
          const float v = src[lane + (t << 6)];
          x[t] = v < 0.f ? fabsf(v) : 0.f;
        }
      }
#pragma unroll
      for (uint32_t S = 16; S >= 1; S >>= 1)
        if (S < epl) {
#pragma unroll
          for (uint32_t t = 0; t < S; ++t) x[t] = x[t] + x[t + S];
        }
      pm = pm + rflf(lanes_sum<float>(x[0], 64));
    }
    __syncthreads();
    return;
  }
  if (opc == OP_R1 || opc == OP_SPC) {
    uint32_t par = 0;
    uint64_t key = ~0ull;
    for (uint32_t t = 0; t < epl; ++t) {
      const uint32_t e = lane + (t << 6);
      const V v = (V)src[e];
      const uint64_t bal = (uint64_t)__ballot(v < (V)0);
      if (lane < 2) nb[2 * t + lane] = lane ? (uint32_t)(bal >> 32) : (uint32_t)bal;
      par ^= (uint32_t)__popcll(bal) & 1u;
      if (opc == OP_SPC) {
        uint64_t kk;
        if constexpr (VT<T>::INT)
          kk = ((uint64_t)(uint32_t)abs(v) << 16) | e;
        else
          kk = ((uint64_t)__float_as_uint(fabsf(v)) << 16) | e;
        key = kk < key ? kk : key;
      }
    }
    if (opc == OP_SPC) {
      if (par) {
        for (uint32_t s = 32; s >= 1; s >>= 1) {
          const uint64_t ok = shfl_xor_k(key, (int)s);
          key = ok < key ? ok : key;
        }
        key = rfl64(key);
        const uint32_t idx = (uint32_t)key & 0xFFFFu;
        __syncthreads();
        if (lane == 0) nb[idx >> 5] ^= 1u << (idx & 31);
        if constexpr (!VT<T>::INT) pm = pm + __uint_as_float((uint32_t)(key >> 16));
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
      const int v = src[lane + (t << 6)];
      if (v < 0)
        a0 += -v;
      else
        a1 += v;
    }
    p0 = rfli(lanes_sum<int>(a0, 64));
    p1 = rfli(lanes_sum<int>(a1, 64));
  } else {
    float x0[32], x1[32];
#pragma unroll
    for (uint32_t t = 0; t < 32; ++t) {
      if (t < epl) {
        const float v = src[lane + (t << 6)];
        x0[t] = v < 0.f ? fabsf(v) : 0.f;
        x1[t] = v < 0.f ? 0.f : fabsf(v);
      }
    }
#pragma unroll
    for (uint32_t S = 16; S >= 1; S >>= 1)
      if (S < epl) {
#pragma unroll
        for (uint32_t t = 0; t < S; ++t) {
          x0[t] = x0[t] + x0[t + S];
          x1[t] = x1[t] + x1[t + S];
        }
      }
    p0 = rflf(lanes_sum<float>(x0[0], 64));
    p1 = rflf(lanes_sum<float>(x1[0], 64));
  }
  const uint32_t v = rep_decide<T>(p0, p1, pm);
  for (uint32_t q = lane; q < (m >> 5); q += 64) nb[q] = v ? ~0u : 0u;
  __syncthreads();
}

}  // namespace

// One wave per frame.  Tiered schedule (sel off): only frames whose plan
// starts at L = 1 are decoded here; a frame of an adaptive plan whose L = 1
// decision fails the CRC gets its next list size in state[f] (the list tiers
// pick it up); every other decoded frame is finished here (its state keeps
// the value 1, which no list tier takes).
// Class schedule (sel on): only the frames of the class, no state.
template <typename T>
__global__ __launch_bounds__(64) void k_sc(KArgs A, uint32_t* state, ClassSel sel) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  using V = typename Lane<T>::V;
  using Acc = typename VT<T>::Acc;
  constexpr uint32_t E = VT<T>::E;
  const uint32_t lane = threadIdx.x;
  for (uint32_t f = blockIdx.x; f < A.n_frames; f += gridDim.x) {
    const DevPlan* P;
    const char* llr;
    uint32_t out_off;
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
    if (sel.on) {
      // class schedule: only this class's frames, the others are left alone
      if (P->first_stage < sel.lmin || P->first_stage > sel.lmax || P->N < sel.nmin ||
          P->N > sel.nmax)
        continue;
    } else if (P->first_stage != 1) {
      continue;  // a list tier starts it (state[f] already holds its first stage)
    }
    if (A.times && lane == 0) A.times[2 * (size_t)f] = wall_clock64();
    P = uni_ptr(P);
    const uint32_t N = uni(P->N), n = uni(P->n), ntx = uni(P->n_tx), n_ops = uni(P->n_sc_ops),
                   np = uni(P->n_punct);
    const uint32_t* prog = uni_ptr(plan_tab(P, uni(P->off_sc_prog)));
    // ---- channel LLRs -> root: punctured head [0, P) received nothing (0),
    // sent positions [P, P + n_tx), shortened tail a zero known for certain
    T* root = reinterpret_cast<T*>(smem);
    const uint32_t nbytes = ntx * E;
    if ((((uintptr_t)llr) & 15u) == 0 && (nbytes & 15u) == 0 && ((np * E) & 15u) == 0) {
      const uint4* s4 = reinterpret_cast<const uint4*>(llr);
      uint4* d4 = reinterpret_cast<uint4*>(root + np);
      for (uint32_t i = lane; i < (nbytes >> 4); i += 64) d4[i] = s4[i];
    } else {
      const T* s1 = reinterpret_cast<const T*>(llr);
      for (uint32_t i = lane; i < ntx; i += 64) root[np + i] = s1[i];
    }
    for (uint32_t i = lane; i < np; i += 64) root[i] = (T)0;
    const T known = VT<T>::INT ? (T)VT<T>::Q : (T)1048576.0f;
    for (uint32_t i = np + ntx + lane; i < N; i += 64) root[i] = known;
    __syncthreads();

    Regs<T> R;
    R.xs = (V)0;
    R.x6 = (V)0;
    R.bs = R.b6 = R.ls = R.l7 = 0u;
    Acc pm = (Acc)0;
    if (N <= 64) reg_load_root<T>(n, R, lane, smem);  // whole code in registers
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
          lds_op<T>(smem, N, OP_G, d, k, op_off(w), R, pm, lane);
        else
          reg_fg<T, true>(k, R, lane);
        reg_node<T>(op_sub(w), k - 1, R, pm, lane);
        if (k >= 7)
          lds_op<T>(smem, N, OP_H, d, k, op_off(w), R, pm, lane);
        else
          reg_h<T>(k, R, lane);
      } else if (opc == OP_FN) {
        // f, the left child (a node at level k - 1 <= 6)
        if (k >= 7)
          lds_op<T>(smem, N, OP_F, d, k, op_off(w), R, pm, lane);
        else
          reg_fg<T, false>(k, R, lane);
        reg_node<T>(op_sub(w), k - 1, R, pm, lane);
      } else if (k >= 7)
        lds_op<T>(smem, N, opc, d, k, op_off(w), R, pm, lane);
      else if (opc == OP_F)
        reg_fg<T, false>(k, R, lane);
      else if (opc == OP_G)
        reg_fg<T, true>(k, R, lane);
      else if (opc == OP_H)
        reg_h<T>(k, R, lane);
      else
        reg_node<T>(opc, k, R, pm, lane);
    }
    // ---- codeword estimate in LDS bits (small codes: from the root mask)
    uint32_t* bits = reinterpret_cast<uint32_t*>(smem + sc_bits_off(N, E));
    if (N <= 64) reg_store_root<T>(n, R, lane, smem);
    __syncthreads();
    // ---- CRC syndrome through the nibble table
    const uint32_t bw = P->bw;
    uint32_t syn = 0;
    if (P->c > 0 && lane < bw) {
      const uint32_t* imask = plan_tab(P, P->off_infomask);
      const uint32_t* nib = plan_tab(P, P->off_crcnib);
      const uint32_t v = bits[lane] & imask[lane];
      const uint32_t nq = N >= 32 ? 8u : (N + 3) / 4;
      for (uint32_t q = 0; q < nq; ++q) syn ^= nib[((lane * 8 + q) << 4) + ((v >> (4 * q)) & 15u)];
    }
    for (int s = 32; s >= 1; s >>= 1) syn ^= __shfl_xor(syn, s, 64);
    const bool ok = rfl(syn) == 0u;
    if (!ok && P->L_max > 1 && !sel.on) {
      if (lane == 0) state[f] = next_stage(P, 1);
      __syncthreads();
      continue;
    }
    // ---- outputs: information bits (data positions of A, ascending)
    uint32_t* out = reinterpret_cast<uint32_t*>(smem + sc_out_off(N, E));
    const uint32_t iw = P->info_words;
    if (lane < iw) out[lane] = 0u;
    __syncthreads();
    if (lane < bw) {
      const uint32_t x = bits[lane];
      uint32_t dm = plan_tab(P, P->off_datamask)[lane];
      const uint32_t pre = plan_tab(P, P->off_dataprefix)[lane];
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
    __syncthreads();
    if (lane < iw) A.info[out_off + lane] = out[lane];
    if (lane == 0) {
      polar_status st;
      st.crc_ok = ok ? 1 : 0;
      st.L_used = 1;
      st.n_paths = 1;
      st.flags = 0;
      if constexpr (VT<T>::INT)
        st.pm = 0u;
      else
        st.pm = __float_as_uint(pm);
      A.status[f] = st;
      if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
    }
    if (A.pm_lists) {
      for (uint32_t t = lane; t < A.pm_stride; t += 64)
        A.pm_lists[(size_t)f * A.pm_stride + t] =
            t == 0 ? (VT<T>::INT ? 0u : __float_as_uint((float)pm)) : 0xFFFFFFFFu;
    }
    __syncthreads();
  }
}

template <typename T>
static int launch_sc_t(const KArgs& A, uint32_t lds, uint32_t grid, uint32_t* state,
                       const ClassSel& sel, hipStream_t s) {
  hipLaunchKernelGGL(k_sc<T>, dim3(grid), dim3(64), lds, s, A, state, sel);
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
