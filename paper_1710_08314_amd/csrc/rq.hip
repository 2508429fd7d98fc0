// Decoder stages for uniform int8 batches on gfx950 with each path on four
// lanes (a DPP quad) and the whole decoder state in vector registers.
//
// A list of L paths per frame (Algorithm 1 with the dedicated nodes of
// Sec. II-B3, the selection of Sec. II-B2 and the CRC choice of Sec. II-B4)
// is walked by the pre-order node program; every frame of a uniform batch
// runs the same program and a list grows the same way in every frame, so a
// wave decodes 16 / L frames in lockstep, the walk and its dispatch scalar.
//
// Layout of a path on lanes q = 0..3 of its quad:
//   * the LLRs of the current node of every level K < n (2^K of them) are in
//     registers: for K >= 4 element i sits in lane (i >> 2) & 3, word i >> 4,
//     byte i & 3, so that f and g of a node of level K >= 5 combine words of
//     the same lane; a node of level K <= 3 is held whole by every lane;
//   * the root is the channel LLR buffer itself, read twice (f and g);
//   * partial sums of a node of level K >= 4 follow its elements: lane q
//     holds the bits of its elements, element i at lane bit
//     4 (i >> 4) + (i & 3); smaller nodes are held whole by every lane;
//   * the left child's partial sums of every split node on the current path
//     wait in registers until the node's h consumes them.
// A path of an int8 code of N = 2048 holds 157 words per lane (two waves
// per SIMD); below N = 2048 a single path fits three waves per SIMD.  Beside
// the registers a wave uses LDS only for a copy of the node program and to
// stage each path's codeword for the CRC and the output, and global memory
// only for the channel LLRs, the plan's tables and the outputs.
//
// Lists keep, per level, the quad whose registers hold a path's node (index
// indirection: a fork moves slot numbers and the small levels, never the
// large levels' LLRs).  Candidate keys are sorted with lane exchanges (DPP,
// row rotations and mirrors, the 16- and 32-lane swaps); a node's words in
// another quad, a survivor's key (L >= 4) and its parent's registers come
// by ds_bpermute.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/polar_scl.h"
#include "device_common.h"
#include "kernels.h"
#include "polar_internal.h"

namespace polar {

namespace {

constexpr int kQ8 = VT<int8_t>::Q;

// ------------------------------------------------------------ quad helpers
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
constexpr int kQX1 = 0xB1;  // quad_perm [1, 0, 3, 2]: the lane q ^ 1
constexpr int kQX2 = 0x4E;  // quad_perm [2, 3, 0, 1]: the lane q ^ 2
template <int I>
__device__ __forceinline__ uint32_t q_bc(uint32_t v) {  // lane I of the quad
  return dpp<I * 0x55>(v);
}
__device__ __forceinline__ uint32_t q_or(uint32_t v) {
  v |= dpp<kQX1>(v);
  return v | dpp<kQX2>(v);
}
__device__ __forceinline__ uint32_t q_xor(uint32_t v) {
  v ^= dpp<kQX1>(v);
  return v ^ dpp<kQX2>(v);
}
__device__ __forceinline__ int q_add(int v) {
  v += (int)dpp<kQX1>((uint32_t)v);
  return v + (int)dpp<kQX2>((uint32_t)v);
}
__device__ __forceinline__ uint32_t q_min(uint32_t v) {
  v = min(v, dpp<kQX1>(v));
  return min(v, dpp<kQX2>(v));
}

constexpr uint32_t lowmask(int n) { return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u); }

// a load from global memory (plan tables, channel LLRs) through a global
// rather than a flat pointer
__device__ __forceinline__ uint32_t gld(const uint32_t* p) {
  return *(const __attribute__((address_space(1))) uint32_t*)(p);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 gld4(const uint32_t* p) {
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)(p);
  return make_uint4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------- path registers
struct RQ {
  // LLRs of the current node of levels 10 .. 0 (words per lane: 2^(K-4) for
  // K >= 4; 2, 1, 1, 1 for the whole nodes of levels 3 .. 0)
  uint32_t x10[64], x9[32], x8[16], x7[8], x6[4], x5[2], x4, x3[2], x2, x1, x0;
  // partial sums of the last finished node (up to level 10: 256 bits a lane)
  uint32_t b[8];
  // left-child partial sums of the split nodes of levels 11 .. 8, and of
  // levels 7, 6, 4 (lA) and 5, 3, 2, 1 (lB) packed
  uint32_t l11[8], l10[4], l9[2], l8, lA, lB;
};

template <int K>
__device__ __forceinline__ uint32_t& X(RQ& R, int j) {
  static_assert(K >= 0 && K <= 10, "register levels");
  if constexpr (K == 10) return R.x10[j];
  else if constexpr (K == 9) return R.x9[j];
  else if constexpr (K == 8) return R.x8[j];
  else if constexpr (K == 7) return R.x7[j];
  else if constexpr (K == 6) return R.x6[j];
  else if constexpr (K == 5) return R.x5[j];
  else if constexpr (K == 4) return R.x4;
  else if constexpr (K == 3) return R.x3[j];
  else if constexpr (K == 2) return R.x2;
  else if constexpr (K == 1) return R.x1;
  else return R.x0;
}

// the LLR words of level K made opaque to the optimiser (no instruction)
template <int K>
__device__ __forceinline__ void opaque_level(RQ& R) {
  constexpr int W = K >= 4 ? (1 << (K - 4)) : (K == 3 ? 2 : 1);
#pragma unroll
  for (int j = 0; j < W; ++j) asm volatile("" : "+v"(X<K>(R, j)));
}

// partial-sum bits a lane holds for a node of level K, and their words
constexpr int nbits(int K) { return K >= 4 ? (1 << (K - 2)) : (1 << K); }
constexpr int nwords(int K) { return nbits(K) >= 32 ? nbits(K) / 32 : 1; }

// left-child partial sums of a split node of level K >= 8: words of the array
template <int K>
__device__ __forceinline__ uint32_t& LW(RQ& R, int w) {
  static_assert(K >= 8 && K <= 11, "multi-word left sums");
  if constexpr (K == 11) return R.l11[w];
  else if constexpr (K == 10) return R.l10[w];
  else if constexpr (K == 9) return R.l9[w];
  else return R.l8;
}
// ... of a split node of level K <= 7: a field of lA (word 0) or lB (word 1)
template <int K>
struct LF {
  static constexpr int w = (K == 7 || K == 6 || K == 4) ? 0 : 1;
  static constexpr int s = K == 7 ? 0 : K == 6 ? 16 : K == 4 ? 24 : K == 5 ? 0 : K == 3 ? 4 : K == 2 ? 8 : 10;
  static constexpr int n = nbits(K - 1);
};
template <int K>
__device__ __forceinline__ uint32_t lft(const RQ& R) {
  return ((LF<K>::w ? R.lB : R.lA) >> LF<K>::s) & lowmask(LF<K>::n);
}
// at g of a split node of level K: the finished left child's sums move to
// the node's left-sum registers
template <int K>
__device__ __forceinline__ void keep_left(RQ& R) {
  if constexpr (K >= 8) {
#pragma unroll
    for (int w = 0; w < nwords(K - 1); ++w) LW<K>(R, w) = R.b[w];
  } else {
    constexpr uint32_t m = lowmask(LF<K>::n) << LF<K>::s;
    uint32_t& d = LF<K>::w ? R.lB : R.lA;
    d = (d & ~m) | ((R.b[0] << LF<K>::s) & m);
  }
}
// the left partial sums of elements 16 j + 4 q + (0..3) of a child of level
// K - 1 >= 4 (bits 4 j .. 4 j + 3 of the lane's left sums)
template <int K>
__device__ __forceinline__ uint32_t sgn4(RQ& R, int j) {
  if constexpr (K >= 8)
    return (LW<K>(R, j >> 3) >> (4 * (j & 7))) & 15u;
  else
    return (lft<K>(R) >> (4 * j)) & 15u;
}

// -------------------------------------------------------- f, g and h steps
// f (G = false) or g (G = true) of a split node of level K <= 10 in registers
template <int K, bool G>
__device__ __forceinline__ void fg_reg(RQ& R, uint32_t q) {
  if constexpr (G) keep_left<K>(R);
  if constexpr (K >= 5) {
    constexpr int WC = 1 << (K - 5);  // words of the child per lane
#pragma unroll
    for (int j = 0; j < WC; ++j) {
      const uint32_t a = X<K>(R, j), c = X<K>(R, j + WC);
      X<K - 1>(R, j) = G ? g4(a, c, sgn4<K>(R, j)) : f4(a, c);
    }
  } else if constexpr (K == 4) {
    // the child (8 elements) is held whole: elements 0..3 from lanes 0 and
    // 2, elements 4..7 from lanes 1 and 3
    const uint32_t v = R.x4;
    const uint32_t a0 = q_bc<0>(v), a1 = q_bc<1>(v), c0 = q_bc<2>(v), c1 = q_bc<3>(v);
    if constexpr (G) {
      const uint32_t s = lft<4>(R);
      R.x3[0] = g4(a0, c0, s & 15u);
      R.x3[1] = g4(a1, c1, (s >> 4) & 15u);
    } else {
      R.x3[0] = f4(a0, c0);
      R.x3[1] = f4(a1, c1);
    }
  } else if constexpr (K == 3) {
    R.x2 = G ? g4(R.x3[0], R.x3[1], lft<3>(R)) : f4(R.x3[0], R.x3[1]);
  } else {
    // K = 2: bytes 0, 1 against 2, 3; K = 1: byte 0 against byte 1
    constexpr uint32_t h = 1u << (K - 1);
    const uint32_t a = X<K>(R, 0), c = a >> (8 * h);
    X<K - 1>(R, 0) = (G ? g4(a, c, lft<K>(R)) : f4(a, c)) & lowmask(8 * h);
  }
}

// f / g at the root (level NL): the child (level NL - 1) word j of lane q
// from the channel's natural words 4 j + q and 4 j + q + N / 8
template <int NL, bool G>
__device__ __forceinline__ void fg_root(RQ& R, const uint32_t* rw, uint32_t q) {
  if constexpr (G) keep_left<NL>(R);
  constexpr int WC = 1 << (NL - 5);
  constexpr int HALF = 1 << (NL - 3);  // words of half the root
  const uint32_t* rq = rw + q;
  // all loads issued together (the child's registers are free to take
  // them), one memory latency per step
#pragma unroll
  for (int j = 0; j < WC; ++j) {
    const uint32_t a = gld(rq + 4 * j), c = gld(rq + 4 * j + HALF);
    X<NL - 1>(R, j) = G ? g4(a, c, sgn4<NL>(R, j)) : f4(a, c);
  }
}

// h of a split node of level K < NL: beta = [left ^ right, right]
template <int K>
__device__ __forceinline__ void h_step(RQ& R, uint32_t q) {
  if constexpr (K >= 8) {
    constexpr int W = nwords(K - 1);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      R.b[W + w] = R.b[w];
      R.b[w] ^= LW<K>(R, w);
    }
  } else if constexpr (K == 4) {
    const uint32_t v = q < 2u ? (lft<4>(R) ^ R.b[0]) : R.b[0];
    R.b[0] = (v >> (4u * (q & 1u))) & 15u;
  } else {
    constexpr int c = nbits(K - 1);
    const uint32_t r = R.b[0] & lowmask(c);
    R.b[0] = ((lft<K>(R) ^ r) & lowmask(c)) | (r << c);
  }
}

// hard decisions of a node of level K as the lane's partial-sum words
template <int K>
__device__ __forceinline__ void hard_bits(RQ& R, uint32_t (&hd)[nwords(K)]) {
#pragma unroll
  for (int w = 0; w < nwords(K); ++w) hd[w] = 0u;
  if constexpr (K >= 4) {
#pragma unroll
    for (int j = 0; j < (1 << (K - 4)); ++j) hd[j >> 3] |= hd4(X<K>(R, j)) << (4 * (j & 7));
  } else if constexpr (K == 3) {
    hd[0] = hd4(R.x3[0]) | (hd4(R.x3[1]) << 4);
  } else {
    hd[0] = hd4(X<K>(R, 0)) & lowmask(1 << K);
  }
}

// element e of a node of level K: the lane holding it and its lane bit
template <int K>
__device__ __forceinline__ bool owns(uint32_t e, uint32_t q) {
  return K >= 4 ? ((e >> 2) & 3u) == q : true;
}
template <int K>
__device__ __forceinline__ uint32_t lane_bit(uint32_t e) {
  return K >= 4 ? ((e >> 4) << 2) | (e & 3u) : e;
}

// A dedicated node or leaf of level K for a list of one: the partial sums
// of the survivor of the list decoder's selection with L = 1 (the hard
// decision wins every tie; REP takes all ones only if its saturated penalty
// is smaller; SPC with odd parity flips the least reliable position, the
// smallest index among equals).
template <int K>
__device__ __forceinline__ void node1(RQ& R, uint32_t opc, uint32_t q) {
  constexpr int NW = nwords(K);
  constexpr uint32_t full = lowmask(nbits(K));
  if (opc == OP_R0 || opc == OP_LF) {
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = 0u;
    return;
  }
  uint32_t hd[NW];
  hard_bits<K>(R, hd);
  if (opc == OP_R1 || opc == OP_LI) {
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = hd[w];
    return;
  }
  // REP and SPC nodes of at most 32 positions (the caller admits only plans
  // whose REP and SPC nodes have levels <= 5)
  if constexpr (K > 5) {
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = hd[w];
    return;
  }
  constexpr int WX = K >= 4 ? (1 << (K >= 4 ? K - 4 : 0)) : (K == 3 ? 2 : 1);  // LLR words per lane
  constexpr int EW = K >= 2 ? 4 : (1 << K);                       // elements per word
  if (opc == OP_REP) {
    int p0 = 0, p1 = 0;
#pragma unroll
    for (int j = 0; j < WX; ++j)
#pragma unroll
      for (int i = 0; i < EW; ++i) {
        const int v = sx8(X<K>(R, j), i);
        if (v < 0)
          p0 -= v;
        else
          p1 += v;
      }
    if constexpr (K >= 4) {
      p0 = q_add(p0);
      p1 = q_add(p1);
    }
    const uint32_t v = min(p1, kQ8) < min(p0, kQ8) ? full : 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = v;
    return;
  }
  // SPC
  uint32_t par = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) par ^= hd[w];
  par = __popc(par) & 1u;
  if constexpr (K >= 4) par = q_xor(par);
  if (par) {
    // keys (|alpha| << 12) | element; a lane's elements differ only in
    // 16 j + i, so its own minimum is taken first and 4 q added after
    uint32_t key = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < WX; ++j)
#pragma unroll
      for (int i = 0; i < EW; ++i) {
        const uint32_t e = K >= 4 ? 16u * j + i : 4u * j + i;
        key = min(key, ((uint32_t)abs(sx8(X<K>(R, j), i)) << 12) | e);
      }
    if constexpr (K >= 4) key = q_min(key | (q << 2));
    const uint32_t e = key & 0xFFFu;
    if (owns<K>(e, q)) {
      const uint32_t t = lane_bit<K>(e);
#pragma unroll
      for (int w = 0; w < NW; ++w)
        if ((t >> 5) == (uint32_t)w) hd[w] ^= 1u << (t & 31u);
    }
  }
#pragma unroll
  for (int w = 0; w < NW; ++w) R.b[w] = hd[w];
}

// the T smallest of two ascending lists of T keys, ascending, in a
template <int T>
__device__ __forceinline__ void merge_top(uint32_t (&a)[T], const uint32_t (&b)[T]) {
  uint32_t m[T];
#pragma unroll
  for (int i = 0; i < T; ++i) m[i] = min(a[i], b[T - 1 - i]);  // bitonic
#pragma unroll
  for (int d = T / 2; d >= 1; d /= 2)
#pragma unroll
    for (int i = 0; i < T; ++i)
      if (!(i & d)) {
        const uint32_t lo = min(m[i], m[i + d]), hi = max(m[i], m[i + d]);
        m[i] = lo;
        m[i + d] = hi;
      }
#pragma unroll
  for (int i = 0; i < T; ++i) a[i] = m[i];
}

// ================================================================= lists
// Per path besides its registers: the metric and, per level, the quad of the
// wave whose registers hold the path's node (index indirection: a fork
// copies no LLRs and no multi-word left sums, only these slot numbers).
struct PL {
  int pm;
  uint32_t sl;  // quad holding the LLRs of level K (5 .. 10): 4 bits at 4 (K - 5)
  uint32_t sb;  // quad holding the left sums of split level K (8 .. 11): 4 bits at 4 (K - 8)
};
__device__ __forceinline__ uint32_t nib_get(uint32_t v, int i) { return (v >> (4 * i)) & 15u; }
__device__ __forceinline__ uint32_t nib_set(uint32_t v, int i, uint32_t x) {
  return (v & ~(15u << (4 * i))) | (x << (4 * i));
}

// the value of lane (lane ^ D), D a power of two below 64, without the LDS
// crossbar: quad permutes for 1 and 2; in a row of 16 lanes, a rotation by
// 8 for 8, and rotations by 12 (lane + 4) and 4 (lane - 4) for 4; the
// 16-lane and 32-lane swaps of gfx950 for 16 and 32 (their first result
// holds the lower block in both blocks, the second the upper)
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128, kRowRor12 = 0x12C;
template <uint32_t D>
__device__ __forceinline__ uint32_t xchg(uint32_t v, uint32_t lane) {
  if constexpr (D == 1) {
    return dpp<kQX1>(v);
  } else if constexpr (D == 2) {
    return dpp<kQX2>(v);
  } else if constexpr (D == 4) {
    const uint32_t up = dpp<kRowRor12>(v), dn = dpp<kRowRor4>(v);
    return (lane & 4u) ? dn : up;
  } else if constexpr (D == 8) {
    return dpp<kRowRor8>(v);
  } else if constexpr (D == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16u) ? p[0] : p[1];
  } else {
    static_assert(D == 32, "lane distance");
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32u) ? p[0] : p[1];
  }
}

// minimum over the quads of a frame (4 L lanes, aligned)
template <int L, uint32_t D = 4>
__device__ __forceinline__ uint32_t frame_min(uint32_t v, uint32_t lane) {
  if constexpr (D < 4u * L)
    return frame_min<L, 2 * D>(min(v, xchg<D>(v, lane)), lane);
  else
    return v;
}

// Ascending sort of a frame's candidate keys: 4 L elements, one per lane
// (element fl in lane fl of the frame), or 8 L with two per lane (element
// 2 fl + t in k[t]).  A bitonic network in its mirrored form: every merge
// first compares element e with e ^ (S - 1) (the block of S reversed), then
// halves the distance; the lower element of each pair keeps the minimum, so
// every block is ascending after its merge and runs that arrive sorted
// (RUN elements, aligned) skip the stages below them.
constexpr int kQMirror = 0x1B;                      // quad_perm [3, 2, 1, 0]
constexpr int kRowHalfMirror = 0x141, kRowMirror = 0x140;
// the value of lane (lane ^ (M - 1)), M a power of two from 2 to 64
template <uint32_t M>
__device__ __forceinline__ uint32_t mirror(uint32_t v, uint32_t lane) {
  if constexpr (M == 2) return dpp<kQX1>(v);
  else if constexpr (M == 4) return dpp<kQMirror>(v);
  else if constexpr (M == 8) return dpp<kRowHalfMirror>(v);
  else if constexpr (M == 16) return dpp<kRowMirror>(v);
  else if constexpr (M == 32) return xchg<16>(dpp<kRowMirror>(v), lane);
  else return xchg<32>(xchg<16>(dpp<kRowMirror>(v), lane), lane);
}
__device__ __forceinline__ uint32_t cx(uint32_t k, uint32_t p, bool keep_min) {
  return keep_min ? min(k, p) : max(k, p);
}
template <int L, bool TWO, uint32_t S, uint32_t D>
__device__ __forceinline__ void sort_half(uint32_t& k0, uint32_t& k1, uint32_t fl, uint32_t lane) {
  if constexpr (TWO && D == 1) {
    const uint32_t lo = min(k0, k1), hi = max(k0, k1);
    k0 = lo;
    k1 = hi;
  } else {
    constexpr uint32_t DL = TWO ? D / 2 : D;  // lane distance
    const bool keep = (fl & DL) == 0u;
    const uint32_t p0 = xchg<DL>(k0, lane);
    k0 = cx(k0, p0, keep);
    if constexpr (TWO) {
      const uint32_t p1 = xchg<DL>(k1, lane);
      k1 = cx(k1, p1, keep);
    }
  }
  if constexpr (D > 1) sort_half<L, TWO, S, D / 2>(k0, k1, fl, lane);
}
template <int L, bool TWO, uint32_t S>
__device__ __forceinline__ void sort_from(uint32_t& k0, uint32_t& k1, uint32_t fl, uint32_t lane) {
  constexpr uint32_t E = TWO ? 8u * L : 4u * L;
  if constexpr (TWO) {
    if constexpr (S == 2) {
      const uint32_t lo = min(k0, k1), hi = max(k0, k1);
      k0 = lo;
      k1 = hi;
    } else {
      const bool keep = (fl & (S / 4)) == 0u;
      const uint32_t p0 = mirror<S / 2>(k1, lane), p1 = mirror<S / 2>(k0, lane);
      k0 = cx(k0, p0, keep);
      k1 = cx(k1, p1, keep);
    }
  } else {
    const bool keep = (fl & (S / 2)) == 0u;
    k0 = cx(k0, mirror<S>(k0, lane), keep);
  }
  if constexpr (S >= 4) sort_half<L, TWO, S, S / 4>(k0, k1, fl, lane);
  if constexpr (S < E) sort_from<L, TWO, 2 * S>(k0, k1, fl, lane);
}
template <int L, bool TWO, uint32_t RUN>
__device__ __forceinline__ void sort_all(uint32_t& k0, uint32_t& k1, uint32_t fl, uint32_t lane) {
  sort_from<L, TWO, 2 * RUN>(k0, k1, fl, lane);
}

// candidate key: (metric, parent rank, local index) as one integer
__device__ __forceinline__ uint32_t ckey(int pm, int pen, uint32_t r, uint32_t local) {
  return ((uint32_t)min(pm + pen, kQ8) << 8) | (r << 4) | local;
}

// Lane geometry of a list of L paths: quad Q of the wave holds rank r of
// frame slot gi; g0 = Q - r is the frame's first quad; fl the lane within
// the frame's 4 L lanes.
struct Geo {
  uint32_t lane, q, Q, r, g0, fl;
};

// The survivors of a selection (sorted keys, a * C of them valid) replace
// the paths: rank r takes the r-th smallest key; its parent's slot numbers,
// whole small-level LLRs and packed left sums are copied; the node's partial
// sums are the parent's hard decisions with the candidate's flips (or all v
// for REP and information leaves).
template <int K, int L, bool TWO, int T, uint32_t RUN>
__device__ __forceinline__ void fork(RQ& R, PL& S, const Geo& G, uint32_t k0, uint32_t k1, uint32_t C,
                                     uint32_t& a, const uint32_t (&hd)[nwords(K)], uint32_t pos,
                                     bool rep) {
  constexpr int NW = nwords(K);
  constexpr uint32_t full = lowmask(nbits(K));
  uint32_t kr, kf;
  if constexpr (L == 2) {
    // the two smallest keys of the frame on every lane of it: sorted pairs
    // merged by a butterfly over its 8 lanes (the smallest of two pairs is
    // the smaller first; the second is the smaller of the larger first and
    // the smaller second)
    uint32_t m1 = TWO ? min(k0, k1) : k0, m2 = TWO ? max(k0, k1) : 0xFFFFFFFFu;
    const auto merge = [&](uint32_t o1, uint32_t o2) {
      const uint32_t n2 = min(max(m1, o1), min(m2, o2));
      m1 = min(m1, o1);
      m2 = n2;
    };
    merge(xchg<1>(m1, G.lane), xchg<1>(m2, G.lane));
    merge(xchg<2>(m1, G.lane), xchg<2>(m2, G.lane));
    merge(xchg<4>(m1, G.lane), xchg<4>(m2, G.lane));
    kr = G.r ? m2 : m1;
    kf = m1;
  } else {
    sort_all<L, TWO, RUN>(k0, k1, G.fl, G.lane);
    const uint32_t fb = G.lane - G.fl;  // the frame's first lane
    if constexpr (TWO) {
      const uint32_t x0 = bperm(k0, fb + (G.r >> 1)), x1 = bperm(k1, fb + (G.r >> 1));
      kr = (G.r & 1u) ? x1 : x0;
    } else {
      kr = bperm(k0, fb + G.r);
    }
    kf = bperm(k0, fb);
  }
  const uint32_t an = min((uint32_t)L, a * C);
  const bool alive = G.r < an;
  const uint32_t p = alive ? (kr >> 4) & 15u : G.r, local = alive ? kr & 15u : 0u;
  const uint32_t src = 4u * (G.g0 + p) + G.q;
  R.x4 = bperm(R.x4, src);
  R.x3[0] = bperm(R.x3[0], src);
  R.x3[1] = bperm(R.x3[1], src);
  R.x2 = bperm(R.x2, src);
  R.x1 = bperm(R.x1, src);
  R.x0 = bperm(R.x0, src);
  R.lA = bperm(R.lA, src);
  R.lB = bperm(R.lB, src);
  S.sl = bperm(S.sl, src);
  S.sb = bperm(S.sb, src);
  if (rep) {
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = local ? full : 0u;
  } else {
    uint32_t h[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) h[w] = bperm(hd[w], src);
    const uint32_t pp = bperm(pos, src);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (!((local >> t) & 1u)) continue;
      const uint32_t e = T == 2 ? (pp >> (16 * t)) & 0xFFFFu : (pp >> (8 * t)) & 0xFFu;
      if (!owns<K>(e, G.q)) continue;
      const uint32_t tb = lane_bit<K>(e);
#pragma unroll
      for (int w = 0; w < NW; ++w)
        if ((tb >> 5) == (uint32_t)w) h[w] ^= 1u << (tb & 31u);
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) R.b[w] = h[w];
  }
  S.pm = alive ? (int)(kr >> 8) - (int)(kf >> 8) : 0;
  a = an;
}

// the T least reliable positions of a node of level K, as sorted keys
// (|alpha| << 12) | element
template <int K, int T>
__device__ __forceinline__ void least(RQ& R, uint32_t q, uint32_t (&s)[T]) {
  constexpr int WX = K >= 4 ? (1 << (K >= 4 ? K - 4 : 0)) : (K == 3 ? 2 : 1);
  constexpr int EW = K >= 2 ? 4 : (1 << K);
#pragma unroll
  for (int t = 0; t < T; ++t) s[t] = 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < WX; ++j) {
#pragma unroll
    for (int i = 0; i < EW; ++i) {
      const uint32_t e = K >= 4 ? 16u * j + i : 4u * j + i;
      uint32_t v = ((uint32_t)abs(sx8(X<K>(R, j), i)) << 12) | e;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const uint32_t lo = min(v, s[t]);
        v = max(v, s[t]);
        s[t] = lo;
      }
    }
    // large nodes: one word at a time, so that the byte extractions of the
    // whole node are not all held at once
    if constexpr (WX > 4) __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (K >= 4) {
    // element numbers of this lane: 16 j + 4 q + i; merge the quad's lists
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (s[t] != 0xFFFFFFFFu) s[t] |= q << 2;
    uint32_t o[T];
#pragma unroll
    for (int t = 0; t < T; ++t) o[t] = dpp<kQX1>(s[t]);
    merge_top<T>(s, o);
#pragma unroll
    for (int t = 0; t < T; ++t) o[t] = dpp<kQX2>(s[t]);
    merge_top<T>(s, o);
  }
}

template <int K, int L>
__device__ __forceinline__ void nodeL(RQ& R, PL& S, const Geo& G, uint32_t opc, uint32_t& a) {
  constexpr int NW = nwords(K);
  constexpr int WX = K >= 4 ? (1 << (K >= 4 ? K - 4 : 0)) : (K == 3 ? 2 : 1);
  constexpr int EW = K >= 2 ? 4 : (1 << K);
  const bool act = G.r < a;
  uint32_t hd[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) hd[w] = 0u;
  if (opc == OP_R0 || opc == OP_LF || opc == OP_LI || opc == OP_REP) {
    // penalties of deciding all 0 (p0) and all 1 (p1)
    int p0 = 0, p1 = 0;
#pragma unroll
    for (int j = 0; j < WX; ++j) {
#pragma unroll
      for (int i = 0; i < EW; ++i) {
        const int v = sx8(X<K>(R, j), i);
        if (v < 0)
          p0 -= v;
        else
          p1 += v;
      }
      if constexpr (WX > 4) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (K >= 4) {
      p0 = q_add(p0);
      p1 = q_add(p1);
    }
    if (opc == OP_R0 || opc == OP_LF) {
      S.pm = min(S.pm + p0, kQ8);
      S.pm -= (int)frame_min<L>(act ? (uint32_t)S.pm : 0x7FFFFFFFu, G.lane);
#pragma unroll
      for (int w = 0; w < NW; ++w) R.b[w] = 0u;
      return;
    }
    if constexpr (K <= 5) {
      const uint32_t k0 = act && G.q < 2u ? ckey(S.pm, G.q ? p1 : p0, G.r, G.q) : 0xFFFFFFFFu;
      // each quad's two candidates in order (lanes 2, 3 hold none): the
      // quad is a sorted run of four
      const uint32_t o = xchg<1>(k0, G.lane);
      fork<K, L, false, 2, 4>(R, S, G, (G.q & 1u) ? max(k0, o) : min(k0, o), 0u, 2u, a, hd, 0u, true);
    }
    return;
  }
  hard_bits<K>(R, hd);
  if (opc == OP_R1) {
    uint32_t s2[2];
    least<K, 2>(R, G.q, s2);
    const int m0 = (int)(s2[0] >> 12), m1 = (int)(s2[1] >> 12);
    const uint32_t pos = (s2[0] & 0xFFFu) | ((s2[1] & 0xFFFu) << 16);
    const int pen = ((G.q & 1u) ? m0 : 0) + ((G.q & 2u) ? m1 : 0);
    const uint32_t k0 = act ? ckey(S.pm, pen, G.r, G.q) : 0xFFFFFFFFu;
    // the quad's four keys ascend with q (penalties 0, m0, m1, m0 + m1 with
    // m0 <= m1, then the local index): a sorted run of four
    fork<K, L, false, 2, 4>(R, S, G, k0, 0u, 4u, a, hd, pos, false);
    return;
  }
  if constexpr (K <= 5 && K >= 2) {
    // SPC: masks over the 4 least reliable positions whose weight has the
    // parity of the hard decisions, in ascending order (candidate c takes
    // the mask (c << 1) | (parity of c ^ par))
    uint32_t s4[4];
    least<K, 4>(R, G.q, s4);
    uint32_t par = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) par ^= hd[w];
    par = __popc(par) & 1u;
    if constexpr (K >= 4) par = q_xor(par);
    const uint32_t pos = (s4[0] & 0xFFu) | ((s4[1] & 0xFFu) << 8) | ((s4[2] & 0xFFu) << 16) |
                         ((s4[3] & 0xFFu) << 24);
    uint32_t kk[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const uint32_t c = G.q + 4u * t;
      const uint32_t mk = (c << 1) | ((__popc(c) & 1u) ^ par);
      int pen = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((mk >> u) & 1u) pen += (int)(s4[u] >> 12);
      kk[t] = act ? ckey(S.pm, pen, G.r, mk) : 0xFFFFFFFFu;
    }
    fork<K, L, true, 4, 1>(R, S, G, kk[0], kk[1], 8u, a, hd, pos, false);
  }
}

// f / g of a split node of level K for a list: the node's LLRs are read
// from the quad its slot names (K >= 5), the child goes to the path's own
// registers
template <int K, bool G>
__device__ __forceinline__ void fg_regL(RQ& R, PL& S, uint32_t q, uint32_t Q) {
  if constexpr (K >= 5) {
    if constexpr (G) {
      keep_left<K>(R);
      if constexpr (K >= 8) S.sb = nib_set(S.sb, K - 8, Q);
    }
    const uint32_t src = 4u * nib_get(S.sl, K - 5) + q;
    constexpr int WC = 1 << (K - 5);
    // eight words at a time, which bounds the permuted words in flight
#pragma unroll
    for (int j0 = 0; j0 < WC; j0 += 8) {
#pragma unroll
      for (int j = j0; j < j0 + 8 && j < WC; ++j) {
        const uint32_t a = bperm(X<K>(R, j), src), c = bperm(X<K>(R, j + WC), src);
        X<K - 1>(R, j) = G ? g4(a, c, sgn4<K>(R, j)) : f4(a, c);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (K - 1 >= 5) S.sl = nib_set(S.sl, K - 6, Q);
  } else {
    fg_reg<K, G>(R, q);
  }
}
template <int NL, bool G>
__device__ __forceinline__ void fg_rootL(RQ& R, PL& S, const uint32_t* rw, uint32_t q, uint32_t Q) {
  if constexpr (G) S.sb = nib_set(S.sb, NL - 8, Q);
  fg_root<NL, G>(R, rw, q);
  S.sl = nib_set(S.sl, NL - 6, Q);
}
template <int K>
__device__ __forceinline__ void h_stepL(RQ& R, PL& S, uint32_t q) {
  if constexpr (K >= 8) {
    const uint32_t src = 4u * nib_get(S.sb, K - 8) + q;
    constexpr int W = nwords(K - 1);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const uint32_t l = bperm(LW<K>(R, w), src);
      R.b[W + w] = R.b[w];
      R.b[w] ^= l;
    }
  } else {
    h_step<K>(R, q);
  }
}

// ------------------------------------------------------------- dispatch
// Single-path and list versions of each kind of step
template <int NL, int L, int K, bool G>
__device__ __forceinline__ void fg_x(RQ& R, PL& S, const uint32_t* rw, uint32_t q, uint32_t Q) {
  if constexpr (K == NL) {
    if constexpr (L == 1)
      fg_root<NL, G>(R, rw, q);
    else
      fg_rootL<NL, G>(R, S, rw, q, Q);
  } else if constexpr (L == 1) {
    fg_reg<K, G>(R, q);
  } else {
    fg_regL<K, G>(R, S, q, Q);
  }
}
template <int L, int K>
__device__ __forceinline__ void h_x(RQ& R, PL& S, uint32_t q) {
  if constexpr (L == 1)
    h_step<K>(R, q);
  else
    h_stepL<K>(R, S, q);
}
template <int L, int K>
__device__ __forceinline__ void node_x(RQ& R, PL& S, const Geo& G, uint32_t opc, uint32_t& a) {
  if constexpr (L == 1)
    node1<K>(R, opc, G.q);
  else
    nodeL<K, L>(R, S, G, opc, a);
}

// Fused steps of the node program: f at level K and the left child (a node
// of level K - 1 <= 6), or g at level K, the right child and h at level K.
template <int NL, int L, int K, bool GNH>
__device__ __forceinline__ void fused_step(RQ& R, PL& S, const Geo& G, uint32_t sub,
                                           const uint32_t* rw, uint32_t& a) {
  fg_x<NL, L, K, GNH>(R, S, rw, G.q, G.Q);
  node_x<L, K - 1>(R, S, G, sub, a);
  if constexpr (GNH && K < NL) h_x<L, K>(R, S, G.q);
}

// A dedicated child of level K of a paired step: R0 or R1 (levels >= 1),
// REP (1..5), SPC (2..5) or a leaf (level 0)
template <int L, int K>
__device__ __forceinline__ void node_sub(RQ& R, PL& S, const Geo& G, uint32_t sub, uint32_t& a) {
  switch (sub) {
    case OP_R0: if constexpr (K >= 1) node_x<L, K>(R, S, G, OP_R0, a); break;
    case OP_R1: if constexpr (K >= 1) node_x<L, K>(R, S, G, OP_R1, a); break;
    case OP_REP: if constexpr (K >= 1 && K <= 5) node_x<L, K>(R, S, G, OP_REP, a); break;
    case OP_SPC: if constexpr (K >= 2 && K <= 5) node_x<L, K>(R, S, G, OP_SPC, a); break;
    case OP_LF: if constexpr (K == 0) node_x<L, K>(R, S, G, OP_LF, a); break;
    case OP_LI: if constexpr (K == 0) node_x<L, K>(R, S, G, OP_LI, a); break;
    default: break;
  }
}
// A paired step of level K: f, the left child, g, the right child, h
template <int NL, int L, int K>
__device__ __forceinline__ void pair_step(RQ& R, PL& S, const Geo& G, uint32_t w, const uint32_t* rw,
                                          uint32_t& a) {
  fg_x<NL, L, K, false>(R, S, rw, G.q, G.Q);
  node_sub<L, K - 1>(R, S, G, pair_left(w), a);
  fg_x<NL, L, K, true>(R, S, rw, G.q, G.Q);
  node_sub<L, K - 1>(R, S, G, pair_right(w), a);
  if constexpr (K < NL) h_x<L, K>(R, S, G.q);
}

// The switch key of a step: opcode, depth and fused child opcode (the node
// offset, or a paired step's child opcodes, masked out), so that one switch
// picks the step's code.
template <int NL>
constexpr uint32_t skey(uint32_t opc, int K, uint32_t sub = 0) {
  return opc | ((uint32_t)(NL - K) << 4) | (sub << 24);
}
// the key of a case that exists for some code lengths only: for a level the
// code does not have (K > KMAX) a distinct key no program word matches (bits
// 28..31 are never set under the key mask)
template <int NL, int KMAX>
constexpr uint32_t rkey(uint32_t opc, int K, uint32_t sub = 0) {
  return K <= KMAX ? skey<NL>(opc, K, sub)
                   : (0xF0000000u | opc | ((uint32_t)K << 4) | (sub << 12));
}

// One step whose level lies in [KLO, KHI], through a single switch over
// every (opcode, level, fused child) the programs use: one binary search,
// then straight code (a paired step picks its two children's code by two
// small switches).  Dedicated REP nodes have levels 1..5, SPC nodes 2..5
// (at least four positions), leaves level 0, and fused and paired steps
// levels <= 7; other keys select nothing (the root's h among them: the
// codeword is read from the root's left sums and the last right child's
// sums).
template <int NL, int L, int KLO, int KHI>
__device__ __forceinline__ void step(RQ& R, PL& S, const Geo& G, uint32_t w, const uint32_t* rw,
                                     uint32_t& a) {
  // the lane index is made opaque at every step, so that nothing derived
  // from it (element indices, addresses) is hoisted out of the walk and
  // held in registers for its whole length
  Geo Go = G;
  if constexpr (L == 1)
    asm volatile("" : "+v"(Go.q));
  else
    asm volatile("" : "+v"(Go.lane), "+v"(Go.q), "+v"(Go.Q), "+v"(Go.r), "+v"(Go.g0), "+v"(Go.fl));
  const uint32_t q = Go.q, Q = Go.Q;
#define POLAR_C_FG(K)                                                                   \
  case rkey<NL, NL - 1>(OP_F, K): if constexpr (K >= KLO && K <= KHI && K < NL) fg_x<NL, L, K, false>(R, S, rw, q, Q); break; \
  case rkey<NL, NL - 1>(OP_G, K): if constexpr (K >= KLO && K <= KHI && K < NL) fg_x<NL, L, K, true>(R, S, rw, q, Q); break;  \
  case rkey<NL, NL - 1>(OP_H, K): if constexpr (K >= KLO && K <= KHI && K < NL) h_x<L, K>(R, S, q); break;
#define POLAR_C_N(K, O) \
  case rkey<NL, NL - 1>(O, K): if constexpr (K >= KLO && K <= KHI && K < NL) node_x<L, K>(R, S, Go, O, a); break;
#define POLAR_C_NODES(K) POLAR_C_N(K, OP_R0) POLAR_C_N(K, OP_R1)
#define POLAR_C_NODES5(K) POLAR_C_NODES(K) POLAR_C_N(K, OP_REP) POLAR_C_N(K, OP_SPC)
#define POLAR_C_FU(K, O)                                                                 \
  case rkey<NL, NL>(OP_FN, K, O):                                                            \
    if constexpr (K >= KLO && K <= KHI && K <= NL) fused_step<NL, L, K, false>(R, S, Go, O, rw, a); \
    break;                                                                               \
  case rkey<NL, NL>(OP_GNH, K, O):                                                           \
    if constexpr (K >= KLO && K <= KHI && K <= NL) fused_step<NL, L, K, true>(R, S, Go, O, rw, a);  \
    break;
#define POLAR_C_PAIR(K)                                                                  \
  case rkey<NL, NL>(OP_PAIR, K):                                                             \
    if constexpr (L > 1 && K >= KLO && K <= KHI && K <= NL) pair_step<NL, L, K>(R, S, Go, w, rw, a); \
    break;
#define POLAR_C_FU4(K) POLAR_C_FU(K, OP_R0) POLAR_C_FU(K, OP_R1)
#define POLAR_C_FU6(K) POLAR_C_FU4(K) POLAR_C_FU(K, OP_REP) POLAR_C_FU(K, OP_SPC)
  switch (w & 0x0F0000FFu) {
    case skey<NL>(OP_F, NL):
      if constexpr (KHI >= NL) fg_x<NL, L, NL, false>(R, S, rw, q, Q);
      break;
    case skey<NL>(OP_G, NL):
      if constexpr (KHI >= NL) fg_x<NL, L, NL, true>(R, S, rw, q, Q);
      break;
    POLAR_C_FG(10) POLAR_C_FG(9) POLAR_C_FG(8) POLAR_C_FG(7) POLAR_C_FG(6)
    POLAR_C_FG(5) POLAR_C_FG(4) POLAR_C_FG(3) POLAR_C_FG(2) POLAR_C_FG(1)
    POLAR_C_NODES(10) POLAR_C_NODES(9) POLAR_C_NODES(8) POLAR_C_NODES(7) POLAR_C_NODES(6)
    POLAR_C_NODES5(5) POLAR_C_NODES5(4) POLAR_C_NODES5(3) POLAR_C_NODES5(2) POLAR_C_NODES(1)
    POLAR_C_N(1, OP_REP)
    POLAR_C_N(0, OP_LF) POLAR_C_N(0, OP_LI)
    // fused: f or g at level K with a child of level K - 1 (REP / SPC
    // children of level <= 5, leaves below level 1)
    POLAR_C_FU4(7) POLAR_C_FU6(6) POLAR_C_FU6(5) POLAR_C_FU6(4) POLAR_C_FU6(3)
    POLAR_C_FU(2, OP_R0) POLAR_C_FU(2, OP_R1) POLAR_C_FU(2, OP_REP)
    POLAR_C_FU(1, OP_LF) POLAR_C_FU(1, OP_LI)
    // paired: both children dedicated nodes or leaves
    POLAR_C_PAIR(7) POLAR_C_PAIR(6) POLAR_C_PAIR(5) POLAR_C_PAIR(4) POLAR_C_PAIR(3)
    POLAR_C_PAIR(2) POLAR_C_PAIR(1)
    default: break;
  }
#undef POLAR_C_FG
#undef POLAR_C_N
#undef POLAR_C_NODES
#undef POLAR_C_NODES5
#undef POLAR_C_FU
#undef POLAR_C_FU4
#undef POLAR_C_FU6
#undef POLAR_C_PAIR
}


}  // namespace

// One stage of list size L (1, 2, 4, 8 or 16) of a uniform int8 batch of a
// code of length 2^NL, 16 / L frames per wave; a persistent grid, wave g
// taking the groups g, g + G, ...  L = 1 decodes every frame of the batch
// (a frame whose CRC fails gets its next list size in state[f], the others
// are finished); L > 1 decodes the frames listed in xl (finished frames get
// state 0, the others their next stage).  Lanes past the batch or list
// decode a frame already taken and drop the result.
// Waves per SIMD the registers allow: a path's state is 157 words at N = 2048
// (two waves), about half of that less at N <= 1024 for a single path (three).
template <int NL, int L>
constexpr int rq_waves() {
  return NL <= 10 && L == 1 ? 3 : 2;
}

template <int NL, int L>
__global__ __launch_bounds__(64, (rq_waves<NL, L>())) void k_rq(KArgs A, uint32_t* state, const uint32_t* xl) {
  constexpr uint32_t FW = 16u / L;          // frames per wave
  constexpr int KB = L == 1 ? 6 : 0;        // the walk's split level (0: none)
  constexpr int CWW = 2 * nwords(NL - 1);  // codeword words per lane
  constexpr int W10 = nwords(NL - 1);
  __shared__ uint32_t cw[16][CWW][4];  // codeword estimate of each quad's path
  __shared__ uint32_t stage[16][64];   // output words of each quad's path
  extern __shared__ uint32_t prog_s[];
  Geo G;
  G.lane = threadIdx.x;
  G.q = G.lane & 3u;
  G.Q = G.lane >> 2;
  G.r = G.Q % L;
  G.g0 = G.Q - G.r;
  G.fl = G.lane & (4u * L - 1u);
  const uint32_t gi = G.Q / L;
  const DevPlan* P = uni_ptr(A.plans[0]);
  // the program with fused steps (f or g merged with an adjacent child node);
  // the lists' with paired steps as well (for a single path the paired code
  // costs more register moves than the dispatch it saves)
  const uint32_t n_ops = uni(L == 1 ? P->n_sc_ops : P->n_q_ops);
  const uint32_t iw = uni(A.info_words), L_max = uni(P->L_max), c_len = uni(P->c);
  const uint32_t* prog = uni_ptr(plan_tab(P, uni(L == 1 ? P->off_sc_prog : P->off_q_prog)));
  const uint32_t* imask = uni_ptr(plan_tab(P, uni(P->off_infomask)));
  const uint32_t* nib = uni_ptr(plan_tab(P, uni(P->off_crcnib)));
  const uint32_t* comp = uni_ptr(plan_tab(P, uni(P->off_datacomp)));
  // the node program in LDS: one step's word is read while the previous
  // step runs, at LDS rather than memory latency
  // followed by a step at the root's level that is never run: the walk
  // reads one step ahead without a bounds check, and the loop below level
  // KB ends on it
  for (uint32_t i = G.lane; i <= n_ops; i += 64u) prog_s[i] = i < n_ops ? prog[i] : op_make(OP_H, 0, 0);
  __syncthreads();
  uint32_t count = A.n_frames;
  if constexpr (L > 1) {
    // the count through a vector load at device scope; a list never holds
    // more frames than the batch, so a larger count is not trusted
    const uint32_t c0 = uni(__hip_atomic_load(&xl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    count = c0 < A.n_frames ? c0 : A.n_frames;
  }
  const uint32_t n_groups = (count + FW - 1u) / FW;
  for (uint32_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const uint32_t idx = FW * grp + gi;
    const bool valid = idx < count;
    uint32_t f;
    if constexpr (L == 1) {
      f = valid ? idx : A.n_frames - 1u;
    } else {
      const uint32_t f0 = xl[1 + (valid ? idx : FW * grp)];
      f = f0 < A.n_frames ? f0 : A.n_frames - 1u;
    }
    if (L == 1 && valid && G.q == 0u && A.times) A.times[2 * (size_t)f] = wall_clock64();
    const uint32_t* rw = reinterpret_cast<const uint32_t*>(A.llr + (size_t)f * A.llr_bytes);
    RQ R;
    {
      uint32_t* z = reinterpret_cast<uint32_t*>(&R);
#pragma unroll
      for (int i = 0; i < (int)(sizeof(RQ) / 4); ++i) z[i] = 0u;
    }
    PL S;
    S.pm = 0;
    S.sl = G.Q * 0x111111u;
    S.sb = G.Q * 0x1111u;
    uint32_t a = 1;
    uint32_t w_next = prog_s[0];
    uint32_t pc = 0;
    while (pc < n_ops) {
      uint32_t w = uni(w_next);
      w_next = prog_s[pc + 1];
      if constexpr (KB > 0) {
        if ((uint32_t)NL - op_depth(w) < (uint32_t)KB) {
          // a subtree below level KB, walked by a loop of its own: its steps
          // touch only the registers of levels < KB, so the larger levels'
          // registers pass through it untouched
          for (;;) {
            // the subtree's root LLRs, which no step of the subtree writes,
            // made opaque at every step: otherwise every computation that
            // depends on them alone (f and g at the subtree's root, the
            // statistics of a dedicated node there) is hoisted out of the
            // loop and run on every entry, used or not
            opaque_level<KB - 1>(R);
            step<NL, L, 0, KB - 1>(R, S, G, w, rw, a);
            ++pc;
            w = uni(w_next);
            if ((uint32_t)NL - op_depth(w) >= (uint32_t)KB) break;
            w_next = prog_s[pc + 1];  // pc < n_ops: w is not the end step
          }
          continue;
        }
      }
      step<NL, L, KB, NL>(R, S, G, w, rw, a);
      ++pc;
    }
    // ---- codeword estimate of each path to LDS: word v of lane q of quad
    // Q at cw[Q][v][q], so that a codeword word's four lane bytes are
    // adjacent; the root's left sums may sit in another quad
    const uint32_t s11 = L == 1 ? G.lane : 4u * nib_get(S.sb, NL - 8) + G.q;
#pragma unroll
    for (int v = 0; v < W10; ++v) {
      const uint32_t lw = L == 1 ? LW<NL>(R, v) : bperm(LW<NL>(R, v), s11);
      cw[G.Q][v][G.q] = lw ^ R.b[v];
      cw[G.Q][W10 + v][G.q] = R.b[v];
    }
    for (uint32_t t = G.q; t < 64u; t += 4u) stage[G.Q][t] = 0u;
    __syncthreads();
    // ---- per codeword word w (lane q takes w = q, q + 4, ...): the word
    // from its four lane bytes (lane q' byte w: elements 32 w + 4 q' + 0..3
    // and 32 w + 16 + 4 q' + 0..3) and its CRC syndrome terms through the
    // nibble table (information positions only)
    uint32_t syn = 0;
    if (c_len > 0) {
      // unrolled, so that every table lookup of the frame is in flight at once
#pragma unroll
      for (int i = 0; i < (1 << (NL - 7)); ++i) {
        const uint32_t wd = 4u * i + G.q;
        const uint4 lb = *reinterpret_cast<const uint4*>(&cw[G.Q][wd >> 2][0]);
        const uint32_t sh = 8u * (wd & 3u);
        const uint32_t l4[4] = {(lb.x >> sh) & 0xFFu, (lb.y >> sh) & 0xFFu, (lb.z >> sh) & 0xFFu,
                                (lb.w >> sh) & 0xFFu};
        uint32_t x = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          x |= ((l4[t] & 15u) << (4 * t)) | ((l4[t] >> 4) << (16 + 4 * t));
        // every nibble looked up (a nibble with no information position
        // masks to 0, whose table entry is 0), so the loads go out together
        const uint32_t xv = x & gld(imask + wd);
        const uint32_t* nw = nib + (wd << 7);
#pragma unroll
        for (int t = 0; t < 8; ++t) syn ^= gld(nw + ((t << 4) | ((xv >> (4 * t)) & 15u)));
      }
      syn = q_xor(syn);
    }
    // ---- the output path: the first in (metric, rank) order whose CRC
    // passes, else the first
    const bool act = G.r < a;
    const uint32_t okey = act ? (((uint32_t)S.pm << 4) | G.r) : 0xFFFFFFFFu;
    const uint32_t best_ok = frame_min<L>(act && syn == 0u ? okey : 0xFFFFFFFFu, G.lane);
    const uint32_t best = frame_min<L>(okey, G.lane);
    const bool ok = best_ok != 0xFFFFFFFFu;
    const bool win = act && okey == (ok ? best_ok : best);
    bool fin;
    if constexpr (L == 1) {
      const bool esc = valid && !ok && L_max > 1;
      if (esc && G.q == 0u) state[f] = next_stage(P, 1);
      fin = valid && !esc;
    } else {
      fin = valid && (ok || L_max <= (uint32_t)L);
      if (valid && G.r == 0u && G.q == 0u) state[f] = fin ? 0u : next_stage(P, L);
    }
    // ---- data bits of the output path, packed into its quad's output words
    if (win && fin)
#pragma unroll
      for (int i = 0; i < (1 << (NL - 7)); ++i) {
        const uint32_t wd = 4u * i + G.q;
        // {data mask, move masks 0..2}, {move masks 3..4, prefix, count}
        const uint4 c0 = gld4(comp + 8u * wd), c1 = gld4(comp + 8u * wd + 4u);
        const uint4 lb = *reinterpret_cast<const uint4*>(&cw[G.Q][wd >> 2][0]);
        const uint32_t sh = 8u * (wd & 3u);
        const uint32_t l4[4] = {(lb.x >> sh) & 0xFFu, (lb.y >> sh) & 0xFFu, (lb.z >> sh) & 0xFFu,
                                (lb.w >> sh) & 0xFFu};
        uint32_t x = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          x |= ((l4[t] & 15u) << (4 * t)) | ((l4[t] >> 4) << (16 + 4 * t));
        // the data bits gathered to the low end in five shift steps
        const uint32_t mv[5] = {c0.y, c0.z, c0.w, c1.x, c1.y};
        uint32_t v = x & c0.x;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const uint32_t m = v & mv[t];
          v = (v ^ m) | (m >> (1u << t));
        }
        const uint32_t p0 = c1.z, o = p0 & 31u, cnt = c1.w;
        if (cnt) {
          atomicOr(&stage[G.Q][p0 >> 5], v << o);
          if (o + cnt > 32u) atomicOr(&stage[G.Q][(p0 >> 5) + 1u], v >> (32u - o));
        }
      }
    __syncthreads();
    uint32_t* out = A.info + (size_t)f * iw;
    if (win && fin) {
      for (uint32_t t = G.q; t < iw; t += 4u) out[t] = stage[G.Q][t];
      if (G.q == 0u) {
        polar_status st;
        st.crc_ok = ok ? 1 : 0;
        st.L_used = (uint8_t)L;
        st.n_paths = (uint8_t)a;
        st.flags = 0;
        st.pm = (uint32_t)S.pm;
        A.status[f] = st;
        if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
      }
    }
    if (fin && A.pm_lists) {
      // the final metrics in (metric, rank) order; unused entries all ones
      uint32_t ord = 0;
#pragma unroll
      for (uint32_t t = 0; t < (uint32_t)L; ++t)
        ord += bperm(okey, 4u * (G.g0 + t)) < okey ? 1u : 0u;
      uint32_t* pl = A.pm_lists + (size_t)f * A.pm_stride;
      if (act && G.q == 0u) pl[ord] = (uint32_t)S.pm;
      if (win)
        for (uint32_t t = a + G.q; t < A.pm_stride; t += 4u) pl[t] = 0xFFFFFFFFu;
    }
    __syncthreads();
  }
}

// Launchers of the stages for codes of length 2^NL.  This file builds the
// kernels of NL = POLAR_RQ_NL (11 unless the including unit says otherwise:
// rq9.hip and rq10.hip build NL = 9 and 10 in units of their own, which
// compile in parallel), and for NL = 11 also the dispatch over NL.
template <int NL>
int launch_rq1_t(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s) {
  hipLaunchKernelGGL((k_rq<NL, 1>), dim3(grid > 0 ? grid : 1), dim3(64), (n_ops + 4u) / 4u * 16u,
                     s, A, state, (const uint32_t*)nullptr);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

template <int NL>
int launch_rqL_t(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                 uint32_t* xl, hipStream_t s) {
  int rc = launch_gather(A.n_frames, L, state, xl, s);
  if (rc) return rc;
  const dim3 gr(grid > 0 ? grid : 1), bl(64);
  const uint32_t lds = (n_ops + 4u) / 4u * 16u;
  const uint32_t* x = xl;
  switch (L) {
    case 2: hipLaunchKernelGGL((k_rq<NL, 2>), gr, bl, lds, s, A, state, x); break;
    case 4: hipLaunchKernelGGL((k_rq<NL, 4>), gr, bl, lds, s, A, state, x); break;
    case 8: hipLaunchKernelGGL((k_rq<NL, 8>), gr, bl, lds, s, A, state, x); break;
    case 16: hipLaunchKernelGGL((k_rq<NL, 16>), gr, bl, lds, s, A, state, x); break;
    default: return POLAR_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

#ifndef POLAR_RQ_NL
#define POLAR_RQ_NL 11
#endif

#if POLAR_RQ_NL == 11
int launch_rq1_n11(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s) {
  return launch_rq1_t<11>(A, n_ops, grid, state, s);
}
int launch_rqL_n11(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                   uint32_t* xl, hipStream_t s) {
  return launch_rqL_t<11>(L, A, n_ops, grid, state, xl, s);
}

int launch_decode_rq1(uint32_t nl, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                      hipStream_t s) {
  switch (nl) {
    case 9: return launch_rq1_n9(A, n_ops, grid, state, s);
    case 10: return launch_rq1_n10(A, n_ops, grid, state, s);
    case 11: return launch_rq1_n11(A, n_ops, grid, state, s);
    default: return POLAR_EINVAL;
  }
}

int launch_decode_rqL(uint32_t nl, uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid,
                      uint32_t* state, uint32_t* xl, hipStream_t s) {
  switch (nl) {
    case 9: return launch_rqL_n9(L, A, n_ops, grid, state, xl, s);
    case 10: return launch_rqL_n10(L, A, n_ops, grid, state, xl, s);
    case 11: return launch_rqL_n11(L, A, n_ops, grid, state, xl, s);
    default: return POLAR_EINVAL;
  }
}
#elif POLAR_RQ_NL == 10
int launch_rq1_n10(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s) {
  return launch_rq1_t<10>(A, n_ops, grid, state, s);
}
int launch_rqL_n10(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                   uint32_t* xl, hipStream_t s) {
  return launch_rqL_t<10>(L, A, n_ops, grid, state, xl, s);
}
#elif POLAR_RQ_NL == 9
int launch_rq1_n9(const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state, hipStream_t s) {
  return launch_rq1_t<9>(A, n_ops, grid, state, s);
}
int launch_rqL_n9(uint32_t L, const KArgs& A, uint32_t n_ops, uint32_t grid, uint32_t* state,
                  uint32_t* xl, hipStream_t s) {
  return launch_rqL_t<9>(L, A, n_ops, grid, state, xl, s);
}
#else
#error "register stages are built for NL = 9, 10 and 11"
#endif

}  // namespace polar
