// gfx950 kernels of the flexible CRC-aided SCL polar decoder.
//
// Method: Leonardon et al., "Fast and Flexible Software Polar List Decoders"
// (arXiv:1710.08314) -- Algorithm 1 (Sec. II-B2) walked as a pre-order node
// program over the pruned tree (Sec. II-B3), min-sum f/g/h (equations of
// Sec. II-B1), LLR-based path metrics, CRC-aided selection in path-metric
// order (Sec. II-B4, IV-B), adaptive list-size schedules (Sec. II-B5) and
// float32 / saturated int16 / saturated int8 arithmetic (Sec. III-B3).
//
// Execution model.  One workgroup decodes one frame at a time; all decoder
// state lives in LDS:
//   * the channel LLRs (root) are shared by every path and never written;
//   * depth-d LLRs of the path of rank r are read from slot ptr[d][r] and
//     f/g always write depth d+1 into the writer's own slot r, so a fork only
//     copies the small per-depth slot table, never LLR data (the paper keeps
//     LLRs behind pointers, Sec. IV-D);
//   * partial sums are packed bits statically owned by rank and copied on
//     fork (SSCL_cpy of Sec. IV-D, N bits per path);
//   * candidates of a fork are (metric, parent rank, local index) keys sorted
//     by a wave-level bitonic network; the first L survive, in key order.
// Bit-exactness with a scalar reading of the method: f, g and penalties are
// evaluated exactly as defined (no FMA, no reassociation: float penalty sums
// use the stride-halving order v[i] += v[i + s], s = m/2 ... 1, which the
// strided lane mapping below reproduces), ties are broken by the key.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/polar_scl.h"
#include "device_common.h"
#include "kernels.h"
#include "polar_internal.h"

namespace polar {

// ------------------------------------------------------------- frame state
// Uniform (per workgroup) view of one frame-stage.
struct Ctx {
  char* smem;
  const DevPlan* P;
  const uint32_t* prog;
  uint32_t N, n, bw, L;  // L: list size of this stage
  LdsLayout lay;
  char* gsp;  // this workgroup's depth-1 slots in global memory (spilled layouts)
};

__device__ __forceinline__ uint32_t* bits_of(const Ctx& c, uint32_t r) {
  return reinterpret_cast<uint32_t*>(c.smem + c.lay.bits) + r * c.bw;
}
__device__ __forceinline__ uint8_t* ptr_tab(const Ctx& c) {
  return reinterpret_cast<uint8_t*>(c.smem + c.lay.ptr);
}
__device__ __forceinline__ uint32_t* tabs(const Ctx& c) {
  return reinterpret_cast<uint32_t*>(c.smem + c.lay.tabs);
}
// Address of element 0 of the depth-d LLRs of the path of rank r.  With G,
// a spilled depth (1 <= d <= lay.spill) in global memory.
template <bool G = false>
__device__ __forceinline__ char* node_llr(const Ctx& c, uint32_t d, uint32_t r) {
  if constexpr (G) {
    // spilled depth, or the root (d = 0, slot stride 0) of a groot layout
    const uint32_t* t = tabs(c);
    return c.gsp + t[d] + (uint32_t)ptr_tab(c)[d * 32 + r] * t[12 + d];
  } else {
    if (d == 0) return c.smem + c.lay.root;
    const uint32_t* t = tabs(c);
    return c.smem + t[d] + (uint32_t)ptr_tab(c)[d * 32 + r] * t[12 + d];
  }
}

// ------------------------------------------------------------ F, G and H
// SG / DG: the source (depth d) / destination (depth d + 1) slots are
// spilled ones in global memory.  V elements per item; the slot bases and
// strides are read once per op.
template <typename T, int V, int NT, bool SG = false, bool DG = false>
__device__ void run_fg(const Ctx& c, uint32_t d, uint32_t o, uint32_t a, bool is_g) {
  constexpr uint32_t E = VT<T>::E;
  constexpr int NB = V * E;
  const uint32_t h = (c.N >> d) >> 1;
  const uint32_t cpp = h / V, lc = lg2(cpp);
  const uint32_t total = a << lc;
  const uint32_t* t = tabs(c);
  const uint8_t* pt = ptr_tab(c);
  const uint32_t dbase = t[d + 1], dstride = t[12 + d + 1];
  const uint32_t sbase = t[d], sstride = t[12 + d];  // the root: t[0], stride t[12] = 0
  for (uint32_t it = threadIdx.x; it < total; it += NT) {
    const uint32_t r = it >> lc, j = it & (cpp - 1);
    const uint32_t slot = d ? (uint32_t)pt[d * 32 + r] : 0u;
    const char* src;
    if constexpr (SG)
      src = c.gsp + sbase + slot * sstride + j * NB;
    else
      src = c.smem + sbase + slot * sstride + j * NB;
    uint32_t wa[4], wb[4], wo[4] = {0u, 0u, 0u, 0u};
    lds_ld<NB>(src, wa);
    lds_ld<NB>(src + h * E, wb);
    if (is_g) {
      const uint32_t bp = o + j * V;
      const uint32_t s = bits_of(c, r)[bp >> 5] >> (bp & 31);
      g_chunk<T, V>(wa, wb, s, wo);
    } else {
      f_chunk<T, V>(wa, wb, wo);
    }
    if constexpr (DG)
      lds_st<NB>(c.gsp + dbase + r * dstride + j * NB, wo);
    else
      lds_st<NB>(c.smem + dbase + r * dstride + j * NB, wo);
  }
  if (threadIdx.x < a) ptr_tab(c)[(d + 1) * 32 + threadIdx.x] = (uint8_t)threadIdx.x;
}

// Elements per item: as many as keep every thread of the workgroup busy
// (a h / NT), at most VMAX and at most h, a power of two.  Small nodes thus
// spread over many lanes instead of running their elements one after the
// other on a few.  SP: this kernel may run spilled layouts (largest list 32).
template <typename T, int NT, bool SP>
__device__ void op_fg(const Ctx& c, uint32_t d, uint32_t o, uint32_t a, bool is_g) {
  const uint32_t h = (c.N >> d) >> 1;
  constexpr uint32_t VM = VT<T>::VMAX;
  if constexpr (SP) {
    // spilled buffers belong to codes with N >= 512 and depths <= 3, so
    // h >= 32 >= VM wherever one is read or written
    const uint32_t S = c.lay.spill;
    const bool sg = d == 0 ? c.lay.groot != 0 : d <= S;
    const bool dg = d + 1 <= S;
    if (sg || dg) {
      if (sg && dg)
        run_fg<T, VM, NT, true, true>(c, d, o, a, is_g);
      else if (sg)
        run_fg<T, VM, NT, true, false>(c, d, o, a, is_g);
      else
        run_fg<T, VM, NT, false, true>(c, d, o, a, is_g);
      return;
    }
  }
  const uint32_t per = (a * h) / (uint32_t)NT;
  const uint32_t v = per < h ? per : h;
  if (v >= VM)
    run_fg<T, VM, NT>(c, d, o, a, is_g);
  else if (VM > 8 && v >= 8)
    run_fg<T, (VM > 8 ? 8 : 1), NT>(c, d, o, a, is_g);
  else if (VM > 4 && v >= 4)
    run_fg<T, (VM > 4 ? 4 : 1), NT>(c, d, o, a, is_g);
  else if (v >= 2)
    run_fg<T, 2, NT>(c, d, o, a, is_g);
  else
    run_fg<T, 1, NT>(c, d, o, a, is_g);
}

template <int NT>
__device__ void op_h(const Ctx& c, uint32_t d, uint32_t o, uint32_t a) {
  const uint32_t h = (c.N >> d) >> 1;
  if (h >= 32) {
    const uint32_t wc = h >> 5, lw = lg2(wc), total = a << lw;
    for (uint32_t it = threadIdx.x; it < total; it += NT) {
      const uint32_t r = it >> lw, k = it & (wc - 1);
      uint32_t* B = bits_of(c, r);
      B[(o >> 5) + k] ^= B[((o + h) >> 5) + k];
    }
  } else if (threadIdx.x < a) {
    uint32_t* B = bits_of(c, threadIdx.x) + (o >> 5);
    const uint32_t msk = ((1u << h) - 1u) << (o & 31);
    const uint32_t w = *B;
    *B = w ^ ((w >> h) & msk);
  }
}

// ------------------------------------------------------- wave primitives
// Bitonic sort, ascending, of 64 * KPL keys held as k[t] = element t*64+lane.
template <typename K, int KPL>
__device__ void wave_sort(K (&k)[KPL]) {
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (uint32_t size = 2; size <= 64u * KPL; size <<= 1) {
#pragma unroll
    for (uint32_t st = size >> 1; st > 0; st >>= 1) {
      if (st >= 64) {
        const uint32_t q = st >> 6;
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          if ((t & q) == 0) {
            const uint32_t e = t * 64u + lane;
            const bool asc = (e & size) == 0;
            const K x = k[t], y = k[t | q];
            const bool sw = asc ? (x > y) : (x < y);
            k[t] = sw ? y : x;
            k[t | q] = sw ? x : y;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const uint32_t e = t * 64u + lane;
          const K other = shfl_xor_k(k[t], (int)st);
          const bool lower = (lane & st) == 0;
          const bool asc = (e & size) == 0;
          const bool keep_min = (lower == asc);
          k[t] = keep_min ? (other < k[t] ? other : k[t]) : (other > k[t] ? other : k[t]);
        }
      }
    }
  }
}

// Sort `cnt` keys of src[] (wave 0 only), write the first `keep` to dst[].
template <typename K, int KPL>
__device__ void sort_keys_kpl(const K* src, uint32_t cnt, K* dst, uint32_t keep) {
  const uint32_t lane = threadIdx.x & 63u;
  K k[KPL];
#pragma unroll
  for (int t = 0; t < KPL; ++t) {
    const uint32_t e = t * 64u + lane;
    k[t] = e < cnt ? src[e] : (K)~(K)0;
  }
  wave_sort<K, KPL>(k);
#pragma unroll
  for (int t = 0; t < KPL; ++t) {
    const uint32_t e = t * 64u + lane;
    if (e < keep) dst[e] = k[t];
  }
}
// Up to 64 keys: a bitonic network over the first P = 2^ceil(log2 cnt) lanes
// only (the network on an aligned power-of-two block is self-contained);
// when a single survivor is kept, a min-reduction instead.
template <typename K>
__device__ void sort_keys_small(const K* src, uint32_t cnt, K* dst, uint32_t keep) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t P = 1;
  while (P < cnt) P <<= 1;
  K k = lane < cnt ? src[lane] : (K)~(K)0;
  if (keep == 1) {
    for (uint32_t st = 1; st < P; st <<= 1) {
      const K o = shfl_xor_k(k, (int)st);
      k = o < k ? o : k;
    }
    if (lane == 0) dst[0] = k;
    return;
  }
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t st = size >> 1; st > 0; st >>= 1) {
      const K o = shfl_xor_k(k, (int)st);
      const bool keep_min = ((lane & st) == 0) == ((lane & size) == 0);
      k = keep_min ? (o < k ? o : k) : (o > k ? o : k);
    }
  }
  if (lane < keep) dst[lane] = k;
}
template <typename K>
__device__ void sort_keys(const K* src, uint32_t cnt, K* dst, uint32_t keep) {
  if (cnt <= 64)
    sort_keys_small<K>(src, cnt, dst, keep);
  else if (cnt <= 128)
    sort_keys_kpl<K, 2>(src, cnt, dst, keep);
  else
    sort_keys_kpl<K, 4>(src, cnt, dst, keep);
}

// Selection by rank counting: every thread takes a candidate, counts the
// smaller keys (keys are unique), and a candidate of rank < keep lands at
// sel[rank].  Keys are read 16 bytes at a time (broadcast reads), the tail
// one at a time.  Unlike a sorting network this has no chain of lane
// exchanges: two dependent LDS round trips whatever the candidate count.
// `over` (nullable) receives the key of rank `keep`, the best one rejected.
template <typename K, int NT>
__device__ void rank_select(const K* cand, uint32_t total, K* sel, uint32_t keep, K* over) {
  constexpr uint32_t PER = 16 / sizeof(K);
  const uint4* c4 = reinterpret_cast<const uint4*>(cand);
  const uint32_t nv = total / PER;
  for (uint32_t i = threadIdx.x; i < total; i += NT) {
    const K k = cand[i];
    uint32_t rank = 0;
    for (uint32_t q = 0; q < nv; ++q) {
      const uint4 v = c4[q];
      if constexpr (sizeof(K) == 4) {
        rank += (v.x < k) + (v.y < k) + (v.z < k) + (v.w < k);
      } else {
        const K a = ((K)v.y << 32) | v.x, b = ((K)v.w << 32) | v.z;
        rank += (a < k) + (b < k);
      }
    }
    for (uint32_t q = nv * PER; q < total; ++q) rank += cand[q] < k;
    if (rank < keep) sel[rank] = k;
    if (over && rank == keep) *over = k;
  }
}

// Near-tie test (float32): the metric lo of the last kept candidate and hi
// of the best rejected one (lo <= hi) within 1e-4 relative, in double.
__device__ __forceinline__ bool tie_gap(float lo, float hi) {
  return (double)hi - (double)lo <= 1e-4 * fmax(1.0, fabs((double)lo));
}
// LDS words of a stage's misc area: [0] chosen rank, [1] CRC passed, [2]
// near-tie seen in this stage (float32), [4..5] the best rejected key of a
// selection
constexpr uint32_t kMiscTie = 2, kMiscOver = 4;

// ------------------------------------------------------------ keys
// Candidate key (metric, parent rank, local index), compared as one unsigned
// integer: local index in bits 0..3 (SPC masks reach 15), parent rank in bits
// 4..8, metric above (int modes: <= 32767, 15 bits; float32: the bits of a
// non-negative float, whose unsigned order is the numeric order).
constexpr uint32_t kLocalBits = 4, kParentBits = 5, kPmShift = kLocalBits + kParentBits;
template <typename T>
__device__ __forceinline__ typename VT<T>::Key make_key(typename VT<T>::Acc pm, uint32_t parent,
                                                        uint32_t local) {
  if constexpr (VT<T>::INT)
    return ((uint32_t)pm << kPmShift) | (parent << kLocalBits) | local;
  else
    return ((unsigned long long)__float_as_uint(pm) << 32) | (parent << kLocalBits) | local;
}
template <typename T>
__device__ __forceinline__ typename VT<T>::Acc key_pm(typename VT<T>::Key k) {
  if constexpr (VT<T>::INT)
    return (int)(k >> kPmShift);
  else
    return __uint_as_float((uint32_t)(k >> 32));
}
template <typename T>
__device__ __forceinline__ uint32_t key_parent(typename VT<T>::Key k) {
  return ((uint32_t)k >> kLocalBits) & ((1u << kParentBits) - 1u);
}
template <typename T>
__device__ __forceinline__ uint32_t key_local(typename VT<T>::Key k) {
  return (uint32_t)k & ((1u << kLocalBits) - 1u);
}
template <typename T>
__device__ __forceinline__ typename VT<T>::Acc pm_add(typename VT<T>::Acc pm,
                                                      typename VT<T>::Acc pen) {
  if constexpr (VT<T>::INT)
    return min(pm + pen, VT<T>::Q);  // both >= 0; pen exact in int32
  else
    return pm + pen;
}
template <typename T>
__device__ __forceinline__ typename VT<T>::Acc* pm_tab(const Ctx& c) {
  return reinterpret_cast<typename VT<T>::Acc*>(c.smem + c.lay.pm);
}

// Reliability key (|alpha|, position): ordered by magnitude, then index.
template <typename T>
__device__ __forceinline__ typename VT<T>::Key rel_key(T v, uint32_t k) {
  if constexpr (VT<T>::INT)
    return ((uint32_t)abs((int)v) << 16) | k;
  else
    return ((unsigned long long)__float_as_uint(fabsf(v)) << 16) | k;
}
template <typename T>
__device__ __forceinline__ typename VT<T>::Acc rel_mag(typename VT<T>::Key k) {
  if constexpr (VT<T>::INT)
    return (int)(k >> 16);
  else
    return __uint_as_float((uint32_t)(k >> 16));
}

// Insert key x into the sorted list s[0..NK) keeping the NK smallest.
template <typename K, int NK>
__device__ __forceinline__ void top_insert(K (&s)[NK], K x) {
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const K lo = s[i] < x ? s[i] : x;
    const K hi = s[i] < x ? x : s[i];
    s[i] = lo;
    x = hi;
  }
}

// Merge two ascending lists of NK distinct keys into the NK smallest of
// both, ascending (for NK = 4: the elementwise minimum of one list and the
// other reversed is bitonic, then two compare-exchange rounds).
template <typename K, int NK>
__device__ __forceinline__ void top_merge(K (&s)[NK], const K (&x)[NK]) {
  if constexpr (NK == 1) {
    s[0] = s[0] < x[0] ? s[0] : x[0];
  } else if constexpr (NK == 2) {
    const K lo = s[0] < x[0] ? s[0] : x[0], hi = s[0] < x[0] ? x[0] : s[0];
    const K nx = s[1] < x[1] ? s[1] : x[1];
    s[0] = lo;
    s[1] = hi < nx ? hi : nx;
  } else {
    static_assert(NK == 4, "lists of 1, 2 or 4 keys");
    K m[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = s[i] < x[3 - i] ? s[i] : x[3 - i];
    auto ce = [](K& u, K& v) {
      const K lo = u < v ? u : v, hi = u < v ? v : u;
      u = lo;
      v = hi;
    };
    ce(m[0], m[2]);
    ce(m[1], m[3]);
    ce(m[0], m[1]);
    ce(m[2], m[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = m[i];
  }
}

// ------------------------------------------------------------ node ops
constexpr uint32_t kEPL = 32;  // max elements per lane in a node (N/64)

// Candidate q of a path: the local index (R1: the Chase-2 mask q; SPC: the
// q-th mask, ascending, over the 4 least reliable positions whose weight has
// the parity of the hard decision) and its penalty.
template <typename T, int NK>
__device__ __forceinline__ void node_candidate(uint32_t opc, uint32_t q, uint32_t par,
                                               const typename VT<T>::Key (&top)[NK],
                                               uint32_t* mask_out,
                                               typename VT<T>::Acc* pen_out) {
  using Acc = typename VT<T>::Acc;
  uint32_t mask;
  if (opc == OP_R1) {
    mask = q;
  } else {
    const uint32_t ev = 0xFCA96530u, od = 0xEDB87421u;  // nibble tables
    mask = ((par ? od : ev) >> (4 * q)) & 15u;
  }
  Acc pen = (Acc)0;
#pragma unroll
  for (int i = 0; i < NK; ++i)
    if ((mask >> i) & 1u) pen = pen + rel_mag<T>(top[i]);
  *mask_out = mask;
  *pen_out = pen;
}

// Per-path statistics of a dedicated node or leaf in the integer modes.
// Integer penalty sums are exact, so any lane assignment gives the same
// result: each path gets a segment of G lanes with G as large as possible
// while every active path fits one round (lane j of a segment holds elements
// j, j + G, ...).  NK = 0: single-candidate nodes (the metric update and zero
// decisions) and REP / information leaves (two candidate keys).  NK = 2 / 4:
// R1 / SPC -- the NK least reliable positions of each path, its candidate
// keys, and its hard decisions, written into the parent's own partial-sum
// region [o, o + m) straight from the wave's sign ballots (G consecutive
// elements of a path per ballot).
template <typename T, int NT, bool GSP, int NK>
__device__ void node_stats_int_k(const Ctx& c, uint32_t opc, uint32_t d, uint32_t o, uint32_t a,
                                 uint32_t C) {
  using Key = typename VT<T>::Key;
  const uint32_t m = c.N >> d;
  uint32_t G = 64;
  while (G > 1 && G * a > (uint32_t)NT) G >>= 1;
  if (G > m) G = m;
  const uint32_t lgG = lg2(G), epl = m >> lgG, ppr = NT >> lgG;
  const uint32_t tid = threadIdx.x, j = tid & (G - 1), lane = tid & 63u;
  const uint32_t seg0 = lane & ~(G - 1);
  int* pm = pm_tab<T>(c);
  Key* cand = reinterpret_cast<Key*>(c.smem + c.lay.cand);
  uint16_t* cpos = reinterpret_cast<uint16_t*>(c.smem + c.lay.cpos);
  const bool single = (opc == OP_R0 || opc == OP_LF);
  const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << G) - 1ull);
  for (uint32_t base = 0; base < a; base += ppr) {
    const uint32_t r = base + (tid >> lgG);
    const bool valid = r < a;
    const T* al = reinterpret_cast<const T*>(node_llr<GSP>(c, d, valid ? r : 0));
    uint32_t* B = bits_of(c, valid ? r : 0) + (o >> 5);
    int p0 = 0, p1 = 0;
    uint32_t par = 0, hw = 0;
    Key top[NK > 0 ? NK : 1];
#pragma unroll
    for (int i = 0; i < (NK > 0 ? NK : 1); ++i) top[i] = ~(Key)0;
    for (uint32_t t = 0; t < epl; ++t) {
      const uint32_t k = j + (t << lgG);
      const int v = al[k];
      const int mg = abs(v);
      if constexpr (NK == 0) {
        if (v < 0)
          p0 += mg;
        else
          p1 += mg;
      } else {
        top_insert<Key, NK>(top, ((uint32_t)mg << 16) | k);
        const uint64_t bal = (uint64_t)__ballot(v < 0);
        par ^= (uint32_t)__popcll((bal >> seg0) & gmask) & 1u;
        if (G >= 32) {
          // lanes 32q .. 32q + 31 of the wave hold 32 consecutive elements
          if (valid && (j & 31u) == 0) B[((t << lgG) + j) >> 5] = (uint32_t)(bal >> (lane & 32u));
        } else {
          hw |= (uint32_t)((bal >> seg0) & gmask) << ((t << lgG) & 31u);
          if (m >= 32 && (((t + 1) << lgG) & 31u) == 0) {
            if (valid && j == 0) B[(t << lgG) >> 5] = hw;
            hw = 0;
          }
        }
      }
    }
    if constexpr (NK > 0) {
      if (m < 32 && valid && j == 0) {
        const uint32_t msk = ((1u << m) - 1u) << (o & 31);
        B[0] = (B[0] & ~msk) | (hw << (o & 31));
      }
    }
    for (uint32_t s = G >> 1; s >= 1; s >>= 1) {
      if constexpr (NK == 0) {
        p0 += __shfl_xor(p0, (int)s, 64);
        p1 += __shfl_xor(p1, (int)s, 64);
      } else {
        Key other[NK];
#pragma unroll
        for (int i = 0; i < NK; ++i) other[i] = __shfl_xor(top[i], (int)s, 64);
        top_merge<Key, NK>(top, other);
      }
    }
    if (!valid) continue;
    if constexpr (NK == 0) {
      if (single) {
        if (j == 0) pm[r] = pm_add<T>(pm[r], p0);
        if (m >= 32) {
          for (uint32_t w = j; w < (m >> 5); w += G) B[w] = 0u;
        } else if (j == 0) {
          B[0] &= ~(((1u << m) - 1u) << (o & 31));
        }
      } else if (j == 0) {
        cand[r * 2 + 0] = make_key<T>(pm_add<T>(pm[r], p0), r, 0);
        cand[r * 2 + 1] = make_key<T>(pm_add<T>(pm[r], p1), r, 1);
      }
    } else {
      for (uint32_t q = j; q < C; q += G) {
        uint32_t mask;
        int pen;
        node_candidate<T, NK>(opc, q, par, top, &mask, &pen);
        cand[r * C + q] = make_key<T>(pm_add<T>(pm[r], pen), r, mask);
        if (q < (uint32_t)NK) {
          Key tq = top[0];
#pragma unroll
          for (int i = 1; i < NK; ++i)
            if ((uint32_t)i == q) tq = top[i];
          cpos[r * 4 + q] = (uint16_t)(tq & 0xFFFFu);
        }
      }
    }
  }
}

template <typename T, int NT, bool GSP>
__device__ void node_stats_int(const Ctx& c, uint32_t opc, uint32_t d, uint32_t o, uint32_t a,
                               uint32_t C) {
  if (opc == OP_R1)
    node_stats_int_k<T, NT, GSP, 2>(c, opc, d, o, a, C);
  else if (opc == OP_SPC)
    node_stats_int_k<T, NT, GSP, 4>(c, opc, d, o, a, C);
  else
    node_stats_int_k<T, NT, GSP, 0>(c, opc, d, o, a, C);
}

// Per-path node work (float32).  Each path is handled by a segment of
// G = min(64, m) lanes; lane j holds elements j, j + G, j + 2G, ...  The
// segment sums of the penalties follow the stride-halving order exactly:
// in-lane halving of the element list, then butterflies over the lanes.
template <typename T, int NT, bool GSP>
__device__ void node_stats_float(const Ctx& c, uint32_t opc, uint32_t d, uint32_t o, uint32_t a,
                                 uint32_t C) {
  using Acc = typename VT<T>::Acc;
  using Key = typename VT<T>::Key;
  const uint32_t m = c.N >> d;
  const uint32_t G = m < 64 ? m : 64, lgG = lg2(G), epl = m >> lgG;
  const uint32_t ppr = NT >> lgG;
  const uint32_t tid = threadIdx.x, j = tid & (G - 1), lane = tid & 63u;
  Acc* pm = pm_tab<T>(c);
  Key* cand = reinterpret_cast<Key*>(c.smem + c.lay.cand);
  uint16_t* cpos = reinterpret_cast<uint16_t*>(c.smem + c.lay.cpos);
  const bool single = (opc == OP_R0 || opc == OP_LF);

  for (uint32_t base = 0; base < a; base += ppr) {
    const uint32_t r = base + (tid >> lgG);
    const bool valid = r < a;
    const T* al = reinterpret_cast<const T*>(node_llr<GSP>(c, d, valid ? r : 0));
    if (opc == OP_R0 || opc == OP_LF || opc == OP_REP || opc == OP_LI) {
      // penalties of the all-0 (v = 0) and all-1 (v = 1) decisions
      Acc x0[kEPL], x1[kEPL];
#pragma unroll
      for (uint32_t t = 0; t < kEPL; ++t) {
        if (t < epl) {
          const T v = al[j + (t << lgG)];
          const Acc mg = VT<T>::INT ? (Acc)abs((int)v) : (Acc)fabsf((float)v);
          const bool hd = v < (T)0;
          x0[t] = hd ? mg : (Acc)0;
          x1[t] = hd ? (Acc)0 : mg;
        }
      }
#pragma unroll
      for (uint32_t S = kEPL / 2; S >= 1; S >>= 1) {
        if (S < epl) {
#pragma unroll
          for (uint32_t t = 0; t < S; ++t) {
            x0[t] = x0[t] + x0[t + S];
            x1[t] = x1[t] + x1[t + S];
          }
        }
      }
      Acc p0 = x0[0], p1 = x1[0];
      for (uint32_t s = G >> 1; s >= 1; s >>= 1) {
        p0 = p0 + __shfl_xor(p0, (int)s, 64);
        p1 = p1 + __shfl_xor(p1, (int)s, 64);
      }
      if (valid && j == 0) {
        if (single) {
          pm[r] = pm_add<T>(pm[r], p0);
        } else {
          cand[r * 2 + 0] = make_key<T>(pm_add<T>(pm[r], p0), r, 0);
          cand[r * 2 + 1] = make_key<T>(pm_add<T>(pm[r], p1), r, 1);
        }
      }
      if (single && valid) {
        // the node decides all zeros
        uint32_t* B = bits_of(c, r);
        if (m >= 32) {
          for (uint32_t w = j; w < (m >> 5); w += G) B[(o >> 5) + w] = 0u;
        } else if (j == 0) {
          B[o >> 5] &= ~(((m == 32 ? 0u : (1u << m)) - 1u) << (o & 31));
        }
      }
    } else {
      // R1 (Chase-2 on the 2 least reliable positions) and SPC (even-parity
      // flips among the 4 least reliable): keys (|alpha|, position).
      constexpr int NK = 4;
      const Key kmax = (Key)~(Key)0;
      Key top[NK] = {kmax, kmax, kmax, kmax};
      uint32_t par = 0;
      // hard decisions of this lane's elements, written into the parent's own
      // partial-sum region [o, o + m): copied to every child, then flipped.
      uint32_t* B = bits_of(c, valid ? r : 0);
#pragma unroll
      for (uint32_t t = 0; t < kEPL; ++t) {
        if (t < epl) {
          const uint32_t k = j + (t << lgG);
          const T v = al[k];
          top_insert<Key, NK>(top, rel_key<T>(v, k));
          const bool hd = v < (T)0;
          par ^= hd ? 1u : 0u;
          const unsigned long long bal = __ballot(hd);
          if (G == 64) {
            if (valid && (lane & 31u) == 0) B[((o + (t << 6)) >> 5) + (lane >> 5)] =
                (uint32_t)(bal >> (lane & 32u));
          } else if (valid && j == 0) {
            const uint32_t seg = (uint32_t)(bal >> (lane & ~(G - 1u))) & ((G == 32 ? 0u : (1u << G)) - 1u);
            uint32_t w = B[o >> 5];
            const uint32_t msk = ((G == 32 ? 0u : (1u << G)) - 1u) << (o & 31);
            B[o >> 5] = (w & ~msk) | (seg << (o & 31));
          }
        }
      }
      for (uint32_t s = G >> 1; s >= 1; s >>= 1) {
        Key other[NK];
#pragma unroll
        for (int i = 0; i < NK; ++i) other[i] = shfl_xor_k(top[i], (int)s);
#pragma unroll
        for (int i = 0; i < NK; ++i) top_insert<Key, NK>(top, other[i]);
        par ^= __shfl_xor(par, (int)s, 64);
      }
      // candidate q of the path is written by lane q mod G of its segment
      // (a segment may be narrower than the candidate count: R1 with m = 2
      // has 4 candidates on 2 lanes, SPC with m = 4 has 8 on 4 lanes)
      const uint32_t npos = opc == OP_R1 ? 2u : 4u;
      for (uint32_t q = j; valid && q < C; q += G) {
        uint32_t mask;
        Acc pen;
        node_candidate<T, 4>(opc, q, par, top, &mask, &pen);
        cand[r * C + q] = make_key<T>(pm_add<T>(pm[r], pen), r, mask);
        if (q < npos) {
          Key tq = top[0];
#pragma unroll
          for (int i = 1; i < NK; ++i)
            if ((uint32_t)i == q) tq = top[i];
          cpos[r * 4 + q] = (uint16_t)(tq & 0xFFFFu);
        }
      }
    }
  }
}

// A dedicated node or leaf for every active path (update_paths(),
// Algorithm 1): candidates, selection of the min(L, a C) best keys in key
// order, path copy, metrics and the node's decisions.
template <typename T, int NT, int LMAX>
__device__ void op_node(const Ctx& c, uint32_t opc, uint32_t d, uint32_t o, uint32_t& a) {
  using Acc = typename VT<T>::Acc;
  using Key = typename VT<T>::Key;
  const uint32_t m = c.N >> d;
  const uint32_t tid = threadIdx.x;
  Acc* pm = pm_tab<T>(c);
  Key* cand = reinterpret_cast<Key*>(c.smem + c.lay.cand);
  uint16_t* cpos = reinterpret_cast<uint16_t*>(c.smem + c.lay.cpos);
  const bool single = (opc == OP_R0 || opc == OP_LF);
  const uint32_t C = single ? 1u : (opc == OP_R1 ? 4u : (opc == OP_SPC ? 8u : 2u));
  const bool gsp = d == 0 ? c.lay.groot != 0 : d <= c.lay.spill;
  if constexpr (VT<T>::INT) {
    if (gsp)
      node_stats_int<T, NT, true>(c, opc, d, o, a, C);
    else
      node_stats_int<T, NT, false>(c, opc, d, o, a, C);
  } else {
    if (gsp)
      node_stats_float<T, NT, true>(c, opc, d, o, a, C);
    else
      node_stats_float<T, NT, false>(c, opc, d, o, a, C);
  }
  __syncthreads();

  if (single) {
    if constexpr (VT<T>::INT) {
      // normalisation after every update_paths() (Sec. III-B3)
      if (tid < 64) {
        Acc v = tid < a ? pm[tid] : (Acc)VT<T>::Q;
        Acc mn = v;
        for (int s = 32; s >= 1; s >>= 1) mn = min(mn, __shfl_xor(mn, s, 64));
        if (tid < a) pm[tid] = v - mn;
      }
      __syncthreads();
    }
    return;
  }

  // ---- selection: the min(L, a*C) best keys, in key order
  Key* sel = reinterpret_cast<Key*>(c.smem + c.lay.sel);
  const uint32_t total = a * C;
  const uint32_t keep = total < c.L ? total : c.L;
  uint32_t* misc = reinterpret_cast<uint32_t*>(c.smem + c.lay.misc);
  Key* over = reinterpret_cast<Key*>(misc + kMiscOver);
  rank_select<Key, NT>(cand, total, sel, keep, VT<T>::INT ? nullptr : over);
  __syncthreads();
  // float32: the L-th kept key against the best rejected one (R-21 reading)
  if constexpr (!VT<T>::INT) {
    if (tid == 0 && total > keep && tie_gap(key_pm<T>(sel[keep - 1]), key_pm<T>(*over)))
      misc[kMiscTie] = 1u;
  }

  // ---- path copy: partial-sum words [0, nwc) and slot pointers of depths
  // 1..d from each survivor's parent (register staged: all reads, barrier,
  // all writes, so a parent can be overwritten by its own child).  A
  // survivor whose parent has its own rank already holds that state.
  uint8_t* pt = ptr_tab(c);
  if (c.L > 1) {
    uint32_t nwc = (o + m + 31u) >> 5;
    if (nwc > c.bw) nwc = c.bw;
    const uint32_t lw = nwc > 1 ? lg2(2 * nwc - 1) : 0;  // ceil log2
    const uint32_t items = keep << lw;
    constexpr int RMAX = (int)((LMAX * (kMaxN / 32) + NT - 1) / NT);
    uint32_t reg[RMAX];
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const uint32_t it = tid + q * NT;
      reg[q] = 0;
      if (it < items) {
        const uint32_t i = it >> lw, w = it & ((1u << lw) - 1u);
        const uint32_t p = key_parent<T>(sel[i]);
        if (w < nwc && p != i) reg[q] = bits_of(c, p)[w];
      }
    }
    constexpr int PMAX = (int)((kMaxLogN * LMAX + NT - 1) / NT);
    uint8_t preg[PMAX];
    const uint32_t pitems = keep * d;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      const uint32_t it = tid + q * NT;
      preg[q] = 0;
      if (it < pitems) {
        const uint32_t i = it / d, dd = 1 + it % d;
        preg[q] = pt[dd * 32 + key_parent<T>(sel[i])];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const uint32_t it = tid + q * NT;
      if (it < items) {
        const uint32_t i = it >> lw, w = it & ((1u << lw) - 1u);
        if (w < nwc && key_parent<T>(sel[i]) != i) bits_of(c, i)[w] = reg[q];
      }
    }
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      const uint32_t it = tid + q * NT;
      if (it < pitems) {
        const uint32_t i = it / d, dd = 1 + it % d;
        if (key_parent<T>(sel[i]) != i) pt[dd * 32 + i] = preg[q];
      }
    }
    __syncthreads();
  }

  // ---- metrics (normalised in the integer modes) and the node's decisions
  if (tid < keep) {
    Acc v = key_pm<T>(sel[tid]);
    if constexpr (VT<T>::INT) v -= key_pm<T>(sel[0]);
    pm[tid] = v;
  }
  if (opc == OP_LI || opc == OP_REP) {
    if (m >= 32) {
      const uint32_t wpp = m >> 5, lw = lg2(wpp), items = keep << lw;
      for (uint32_t it = tid; it < items; it += NT) {
        const uint32_t i = it >> lw, w = it & (wpp - 1u);
        bits_of(c, i)[(o >> 5) + w] = key_local<T>(sel[i]) ? ~0u : 0u;
      }
    } else if (tid < keep) {
      uint32_t* B = bits_of(c, tid) + (o >> 5);
      const uint32_t msk = ((1u << m) - 1u) << (o & 31);
      *B = key_local<T>(sel[tid]) ? (*B | msk) : (*B & ~msk);
    }
  } else if (tid < keep) {
    // R1 / SPC: flip the chosen least reliable positions of the parent's
    // hard decision (already copied into the child)
    const uint32_t mask = key_local<T>(sel[tid]), p = key_parent<T>(sel[tid]);
    uint32_t* B = bits_of(c, tid);
    for (uint32_t i = 0; i < 4; ++i) {
      if ((mask >> i) & 1u) {
        const uint32_t pos = o + cpos[p * 4 + i];
        B[pos >> 5] ^= 1u << (pos & 31);
      }
    }
  }
  __syncthreads();
  a = keep;
}

// ------------------------------------------------------------ one stage
template <typename T, int NT, int LMAX>
__device__ void run_program(const Ctx& c, uint32_t& a) {
  const uint32_t n_ops = uni(c.P->n_ops);
  // the next op word is fetched while the current op runs
  uint32_t w_next = n_ops ? c.prog[0] : 0u;
  for (uint32_t pc = 0; pc < n_ops; ++pc) {
    const uint32_t w = uni(w_next);
    if (pc + 1 < n_ops) w_next = c.prog[pc + 1];
    const uint32_t opc = op_code(w), d = op_depth(w), o = op_off(w);
    switch (opc) {
      case OP_F:
        op_fg<T, NT, true>(c, d, o, a, false);
        __syncthreads();
        break;
      case OP_G:
        op_fg<T, NT, true>(c, d, o, a, true);
        __syncthreads();
        break;
      case OP_H:
        op_h<NT>(c, d, o, a);
        __syncthreads();
        break;
      default:
        op_node<T, NT, LMAX>(c, opc, d, o, a);
        break;
    }
  }
}

// End of a stage (Sec. II-B4, IV-B): order the paths by (metric, rank),
// compute every path's CRC syndrome from its codeword estimate, and take
// the first path in that order whose syndrome is zero.  Returns the chosen
// rank; *ok = CRC passed.  ord[] keeps the order (for the metric list).
template <typename T, int NT>
__device__ uint32_t end_of_stage(const Ctx& c, uint32_t a, bool* ok) {
  using Key = typename VT<T>::Key;
  using Acc = typename VT<T>::Acc;
  const uint32_t tid = threadIdx.x;
  Key* cand = reinterpret_cast<Key*>(c.smem + c.lay.cand);
  Key* sel = reinterpret_cast<Key*>(c.smem + c.lay.sel);
  uint32_t* syn = reinterpret_cast<uint32_t*>(c.smem + c.lay.syn);
  uint32_t* ord = reinterpret_cast<uint32_t*>(c.smem + c.lay.ord);
  uint32_t* misc = reinterpret_cast<uint32_t*>(c.smem + c.lay.misc);
  const Acc* pm = pm_tab<T>(c);
  if (tid < a) {
    cand[tid] = make_key<T>(pm[tid], tid, 0);
    syn[tid] = 0;
  }
  __syncthreads();
  if (tid < 64) sort_keys<Key>(cand, a, sel, a);
  // syndromes
  const uint32_t* infomask = plan_tab(c.P, uni(c.P->off_infomask));
  const uint32_t* nib = plan_tab(c.P, uni(c.P->off_crcnib));
  const uint32_t crc_len = uni(c.P->c);
  const uint32_t lbw = lg2(c.bw), items = a << lbw;
  const uint32_t nq = c.N >= 32 ? 8u : (c.N + 3) / 4;
  if (crc_len > 0) {
    for (uint32_t it = tid; it < items; it += NT) {
      const uint32_t r = it >> lbw, w = it & (c.bw - 1u);
      const uint32_t v = bits_of(c, r)[w] & infomask[w];
      uint32_t s = 0;
      for (uint32_t q = 0; q < nq; ++q) s ^= nib[((w * 8 + q) << 4) + ((v >> (4 * q)) & 15u)];
      if (s) atomicXor(&syn[r], s);
    }
  }
  __syncthreads();
  if (tid < 64) {
    const bool in = tid < a;
    const uint32_t r = in ? key_parent<T>(sel[tid]) : 0u;
    if (in) ord[tid] = r;
    const unsigned long long good = __ballot(in && syn[r] == 0u);
    if (tid == 0) {
      misc[0] = good ? ord[__ffsll(good) - 1] : ord[0];
      misc[1] = good ? 1u : 0u;
    }
  }
  __syncthreads();
  // float32 near-tie of the final choice: another path with the chosen
  // metric within 1e-4 relative that also passes the CRC (any path when
  // none passes)
  if constexpr (!VT<T>::INT) {
    if (tid < a) {
      const uint32_t ch = misc[0], r = ord[tid];
      const bool pass = misc[1] != 0;
      if (r != ch && (!pass || syn[r] == 0u)) {
        const double d = fabs((double)pm[r] - (double)pm[ch]);
        if (d <= 1e-4 * fmax(1.0, fabs((double)pm[ch]))) atomicOr(&misc[kMiscTie], 1u);
      }
    }
    __syncthreads();
  }
  *ok = uni(misc[1]) != 0;
  return uni(misc[0]);
}

// Load the channel LLRs into the root buffer: punctured positions [0, P)
// received nothing (0), the sent ones follow, and shortened positions get the
// largest positive value (a zero received with certainty).
template <typename T, int NT>
__device__ void load_root(const Ctx& c, const char* llr) {
  constexpr uint32_t E = VT<T>::E;
  T* root = reinterpret_cast<T*>(c.lay.groot ? c.gsp : c.smem + c.lay.root);
  const uint32_t ntx = uni(c.P->n_tx), np = uni(c.P->n_punct);
  const uint32_t nbytes = ntx * E;
  if ((((uintptr_t)llr) & 15u) == 0 && (nbytes & 15u) == 0 && ((np * E) & 15u) == 0) {
    const uint4* src = reinterpret_cast<const uint4*>(llr);
    uint4* dst = reinterpret_cast<uint4*>(root + np);
    for (uint32_t i = threadIdx.x; i < (nbytes >> 4); i += NT) dst[i] = src[i];
  } else {
    const T* src = reinterpret_cast<const T*>(llr);
    for (uint32_t i = threadIdx.x; i < ntx; i += NT) root[np + i] = src[i];
  }
  for (uint32_t i = threadIdx.x; i < np; i += NT) root[i] = (T)0;
  const T known = VT<T>::INT ? (T)VT<T>::Q : (T)1048576.0f;
  for (uint32_t i = np + ntx + threadIdx.x; i < c.N; i += NT) root[i] = known;
}

// A stage's layout, its tables, and the root (its place depends on the
// layout, so it is loaded per stage).
template <typename T, int NT>
__device__ void setup_stage(Ctx& c, uint32_t L, const char* llr) {
  c.L = L;
  c.lay = lds_layout(c.N, c.n, VT<T>::E, L, (uint32_t)sizeof(typename VT<T>::Key));
  load_root<T, NT>(c, llr);
  uint32_t* t = tabs(c);
  if (threadIdx.x == 0) {
    uint32_t cur = c.lay.stages, gcur = c.lay.groot ? ru16(c.N * VT<T>::E) : 0u;
    t[0] = c.lay.groot ? 0u : c.lay.root;
    t[12] = 0;
    for (uint32_t d = 1; d <= c.n; ++d) {
      t[12 + d] = slot_bytes(c.N, d, VT<T>::E);
      if (d <= c.lay.spill) {
        t[d] = gcur;  // offset in global memory (c.gsp)
        gcur += L * t[12 + d];
        continue;
      }
      t[d] = cur;
      cur += L * t[12 + d];
    }
    pm_tab<T>(c)[0] = (typename VT<T>::Acc)0;
    reinterpret_cast<uint32_t*>(c.smem + c.lay.misc)[kMiscTie] = 0u;
  }
  __syncthreads();
}

// Decode frame f: run the plan's list-size schedule (Sec. II-B5) from
// `L_first`.  A frame whose stage at list size >= L_stop fails the CRC while
// a larger stage remains is left for the list tier: returns false and writes
// nothing but *L_last and *tie.  Otherwise writes bits, status, the metric
// list and the end stamp.  tie0: a near-tie already met by an earlier stage
// (float32; status flag bit 0 covers every stage of the frame).
template <typename T, int NT, int LMAX>
__device__ bool decode_frame(char* smem, const KArgs& A, uint32_t f, const DevPlan* P,
                             const char* llr, uint32_t out_off, uint32_t L_first,
                             uint32_t L_stop, uint32_t* L_last = nullptr, uint32_t tie0 = 0,
                             uint32_t* tie_out = nullptr) {
  using Acc = typename VT<T>::Acc;
  P = uni_ptr(P);
  llr = uni_ptr(llr);
  out_off = uni(out_off);
  L_first = uni(L_first);
  Ctx c;
  c.smem = smem;
  c.P = P;
  c.prog = uni_ptr(plan_tab(P, uni(P->off_prog)));
  c.N = uni(P->N);
  c.n = uni(P->n);
  c.bw = uni(P->bw);
  c.L = 1;
  c.gsp = A.spill ? uni_ptr(A.spill + (size_t)blockIdx.x * A.spill_stride) : nullptr;
  uint32_t L = L_first, chosen = 0, a = 1;
  const uint32_t L_max = uni(P->L_max), algo = uni(P->algo);
  bool ok = false;
  uint32_t tie = uni(tie0);
  for (;;) {
    setup_stage<T, NT>(c, L, llr);
    a = 1;
    run_program<T, NT, LMAX>(c, a);
    chosen = end_of_stage<T, NT>(c, a, &ok);
    tie |= uni(reinterpret_cast<const uint32_t*>(c.smem + c.lay.misc)[kMiscTie]);
    // every wave has read the stage's misc words before the next stage's
    // layout (whose tables may sit there) is written
    __syncthreads();
    if (ok || L >= L_max) break;
    if (L >= L_stop) {
      if (L_last) *L_last = L;
      if (tie_out) *tie_out = tie;
      return false;
    }
    L = (algo == POLAR_PA_SCL) ? L_max : 2 * L;
  }
  // ---- outputs
  const uint32_t tid = threadIdx.x;
  uint32_t* out = reinterpret_cast<uint32_t*>(c.smem + c.lay.out);
  const uint32_t iw = uni(P->info_words);
  for (uint32_t i = tid; i < iw; i += NT) out[i] = 0;
  __syncthreads();
  const uint32_t* dmask = plan_tab(P, uni(P->off_datamask));
  const uint32_t* dpre = plan_tab(P, uni(P->off_dataprefix));
  const uint32_t* xb = bits_of(c, chosen);
  for (uint32_t w = tid; w < c.bw; w += NT) {
    const uint32_t x = xb[w];
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
  __syncthreads();
  for (uint32_t i = tid; i < iw; i += NT) A.info[out_off + i] = out[i];
  const Acc* pm = pm_tab<T>(c);
  if (tid == 0) {
    polar_status st;
    st.crc_ok = ok ? 1 : 0;
    st.L_used = (uint8_t)L;
    st.n_paths = (uint8_t)a;
    st.flags = (uint8_t)tie;
    const Acc v = pm[chosen];
    if constexpr (VT<T>::INT)
      st.pm = (uint32_t)v;
    else
      st.pm = __float_as_uint(v);
    A.status[f] = st;
    if (A.times) A.times[2 * (size_t)f + 1] = wall_clock64();
  }
  if (A.pm_lists) {
    const uint32_t* ord = reinterpret_cast<const uint32_t*>(c.smem + c.lay.ord);
    const uint32_t ml = A.pm_stride;
    for (uint32_t t = tid; t < ml; t += NT) {
      uint32_t v = 0xFFFFFFFFu;
      if (t < a) {
        const Acc p = pm[ord[t]];
        if constexpr (VT<T>::INT)
          v = (uint32_t)p;
        else
          v = __float_as_uint(p);
      }
      A.pm_lists[(size_t)f * ml + t] = v;
    }
  }
  __syncthreads();
  return true;
}

__device__ __forceinline__ void frame_of(const KArgs& A, uint32_t f, const DevPlan*& P,
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

// Occupancy of the list kernels: the integer variants are held to 64 VGPRs
// (one-wave workgroups, 8 waves per SIMD) or 72 (wider workgroups, 7), so
// that registers, like the spilled LDS layouts, leave room for more
// workgroups per CU; float32 keeps its registers.
template <typename T, int NW>
constexpr int list_waves_per_eu() {
  return VT<T>::INT ? (NW == 1 ? 8 : 7) : 1;
}

// Plain schedule: each workgroup runs whole frames, every stage in place,
// with LDS sized for the largest list.
template <typename T, int NW>
__global__ __launch_bounds__(NW * 64) void k_decode_plain(KArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  for (uint32_t f = blockIdx.x; f < A.n_frames; f += gridDim.x) {
    const DevPlan* P;
    const char* llr;
    uint32_t out_off;
    frame_of(A, f, P, llr, out_off);
    if (A.times && threadIdx.x == 0) A.times[2 * (size_t)f] = wall_clock64();
    decode_frame<T, NW * 64, kMaxL>(smem, A, f, P, llr, out_off, P->first_stage, 0xFFFFFFFFu);
  }
}

// Per-frame state of the tiered schedule (device scratch): bits 0..7 of
// state[f] = the list size of frame f's next stage (a finished frame holds 0
// or 1, which no list tier takes), bit 8 = a float32 near-tie met by an
// earlier stage.  Every frame starts at its plan's first stage.
__global__ void k_state_init(KArgs A, uint32_t* state) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t f = t; f < A.n_frames; f += gridDim.x * blockDim.x) {
    const DevPlan* P = A.frames ? A.plans[A.frames[f].plan_idx] : A.plans[0];
    state[f] = P->first_stage;
  }
}

// List tier: persistent workgroups claim the frames `chunk` (1..64) at a
// time.  The frames are split into S = min(kClaimSegs, grid) contiguous
// segments, each with a claim counter of its own that the workgroups
// b = s (mod S) share, so claims stay fine-grained without every workgroup
// contending for one address.  Wave 0 reads the claimed frames' state
// words and picks the frames whose next stage lies in
// [L_lo, L_hi] (a ballot, shared through LDS with the other waves, so every
// wave of the workgroup works on the same frames).  For each picked frame the
// stages of its schedule up to L_hi run in place; its state becomes 0 when
// its outputs are written, else the list size of its next stage.  Frame
// indices come only from the claim counter, never from memory the device
// wrote.
template <typename T, int NW, int LMAX>
__global__ __launch_bounds__(NW * 64, (list_waves_per_eu<T, NW>())) void k_decode_list(
    KArgs A, uint32_t* state, uint32_t* head,
                                                         uint32_t L_lo, uint32_t L_hi,
                                                         uint32_t chunk) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ uint32_t s_base;
  __shared__ unsigned long long s_mask;
  __shared__ uint32_t s_L0[64];
  const uint32_t n_seg = gridDim.x < kClaimSegs ? gridDim.x : kClaimSegs;
  const uint32_t seg = blockIdx.x % n_seg;
  const uint32_t seg_len = (A.n_frames + n_seg - 1) / n_seg;
  const uint32_t seg_lo = seg * seg_len;
  const uint32_t seg_hi = seg_lo + seg_len < A.n_frames ? seg_lo + seg_len : A.n_frames;
  for (;;) {
    if (threadIdx.x == 0) s_base = seg_lo + atomicAdd(&head[seg], chunk);
    __syncthreads();
    const uint32_t base = uni(s_base);
    if (base >= seg_hi) break;
    if (threadIdx.x < 64) {
      const uint32_t f = base + threadIdx.x;
      const uint32_t w0 = (threadIdx.x < chunk && f < seg_hi) ? state[f] : 0u;
      s_L0[threadIdx.x] = w0;
      const uint32_t L0 = w0 & 0xFFu;
      const unsigned long long b = __ballot(L0 >= L_lo && L0 <= L_hi);
      if (threadIdx.x == 0) s_mask = b;
    }
    __syncthreads();
    uint64_t mask = uni64(s_mask);
    while (mask) {
      const uint32_t j = (uint32_t)(__ffsll((unsigned long long)mask) - 1);
      mask &= mask - 1ull;
      const uint32_t f = base + j;
      const uint32_t w0 = uni(s_L0[j]), L0 = w0 & 0xFFu;
      const DevPlan* P;
      const char* llr;
      uint32_t out_off;
      frame_of(A, f, P, llr, out_off);
      if (L0 == P->first_stage && A.times && threadIdx.x == 0)
        A.times[2 * (size_t)f] = wall_clock64();
      uint32_t L_last = L0, tie = 0;
      const bool done = decode_frame<T, NW * 64, LMAX>(smem, A, f, P, llr, out_off, L0, L_hi,
                                                       &L_last, (w0 >> 8) & 1u, &tie);
      if (threadIdx.x == 0) state[f] = done ? 0u : (next_stage(P, L_last) | (tie << 8));
    }
    __syncthreads();
  }
}

// Class schedule: persistent workgroups claim the frame descriptors 64 at a
// time; wave 0 tests the 64 frames against the class (first stage and code
// length of the frame's plan) and the workgroup decodes the matching ones,
// each in its single stage.
__device__ __forceinline__ bool in_class(const DevPlan* P, const ClassSel& sel) {
  return P->first_stage >= sel.lmin && P->first_stage <= sel.lmax && P->N >= sel.nmin &&
         P->N <= sel.nmax && P->quant == sel.quant;
}

template <typename T, int NW, int LMAX>
__global__ __launch_bounds__(NW * 64, (list_waves_per_eu<T, NW>())) void k_decode_class(
    KArgs A, uint32_t* head, ClassSel sel) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ uint32_t s_base;
  __shared__ unsigned long long s_mask;
  for (;;) {
    if (threadIdx.x == 0) s_base = atomicAdd(head, 64u);
    __syncthreads();
    const uint32_t base = uni(s_base);
    if (base >= A.n_frames) break;
    if (threadIdx.x < 64) {
      const uint32_t f = base + threadIdx.x;
      bool m = false;
      if (f < A.n_frames) m = in_class(A.plans[A.frames[f].plan_idx], sel);
      const unsigned long long b = __ballot(m);
      if (threadIdx.x == 0) s_mask = b;
    }
    __syncthreads();
    uint64_t mask = uni64(s_mask);
    __syncthreads();
    while (mask) {
      const uint32_t f = base + (uint32_t)(__ffsll((unsigned long long)mask) - 1);
      mask &= mask - 1ull;
      const DevPlan* P;
      const char* llr;
      uint32_t out_off;
      frame_of(A, f, P, llr, out_off);
      if (A.times && threadIdx.x == 0) A.times[2 * (size_t)f] = wall_clock64();
      decode_frame<T, NW * 64, LMAX>(smem, A, f, P, llr, out_off, P->first_stage, 0xFFFFFFFFu);
    }
  }
}

__global__ void k_heads_reset(uint32_t* heads, uint32_t n) {
  if (threadIdx.x < n) heads[threadIdx.x] = 0;
}

// ------------------------------------------------------------ launchers
template <typename K>
static int set_lds(K k, uint32_t lds) {
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds) == hipSuccess
             ? POLAR_OK
             : POLAR_EHIP;
}

int sc_set_attributes(int lds);

// Dynamic LDS every decoder kernel may request: the CU's LDS less room for the
// kernels' own static variables (plans never need more, see plan_lds_bytes).
constexpr uint32_t kDynLdsMax = kLdsLimit - 1024;

template <typename T>
static int set_attributes_t() {
  int rc = POLAR_OK;
  rc |= set_lds(k_decode_plain<T, 1>, kDynLdsMax);
  rc |= set_lds(k_decode_list<T, 1, (int)kTierALmax>, kDynLdsMax);
  rc |= set_lds(k_decode_list<T, kListWaves, (int)kMaxL>, kDynLdsMax);
  rc |= set_lds(k_decode_class<T, 1, 4>, kDynLdsMax);
  rc |= set_lds(k_decode_class<T, 2, 8>, kDynLdsMax);
  rc |= set_lds(k_decode_class<T, 4, (int)kMaxL>, kDynLdsMax);
  return rc ? POLAR_EHIP : POLAR_OK;
}

int init_kernel_attributes() {
  if (set_attributes_t<float>() || set_attributes_t<int16_t>() || set_attributes_t<int8_t>())
    return POLAR_EHIP;
  if (listp_set_attributes(kLdsLimit - listp_static_lds())) return POLAR_EHIP;
  return sc_set_attributes((int)kDynLdsMax);
}

template <typename T>
static int launch_class_t(const KArgs& A, const ClassLaunch& c, uint32_t* head, uint32_t* heads,
                          hipStream_t s) {
  const uint32_t quant = VT<T>::INT ? (sizeof(T) == 2 ? POLAR_I16 : POLAR_I8) : POLAR_F32;
  KArgs Ac = A;
  Ac.spill_stride = c.spill;
  switch (c.kernel) {
    case CK_SC:
      return launch_decode_sc(quant, A, c.lds, c.grid, heads, c.sel, s);
    case CK_W1_L4:
      hipLaunchKernelGGL((k_decode_class<T, 1, 4>), dim3(c.grid), dim3(64), c.lds, s, Ac, head,
                         c.sel);
      break;
    case CK_W2_L8:
      hipLaunchKernelGGL((k_decode_class<T, 2, 8>), dim3(c.grid), dim3(128), c.lds, s, Ac, head,
                         c.sel);
      break;
    default:
      hipLaunchKernelGGL((k_decode_class<T, 4, (int)kMaxL>), dim3(c.grid), dim3(256), c.lds, s, Ac,
                         head, c.sel);
      break;
  }
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_decode_classes(const KArgs& A, const ClassLaunch* cls, uint32_t n_cls, uint32_t* heads,
                          hipStream_t s, hipEvent_t ev_begin, hipEvent_t ev_end) {
  if (n_cls > kMaxClasses) return POLAR_EINVAL;
  if (ev_begin) (void)hipEventRecord(ev_begin, s);
  hipLaunchKernelGGL(k_heads_reset, dim3(1), dim3(64), 0, s, heads, n_cls);
  int rc = POLAR_OK;
  for (uint32_t i = 0; i < n_cls && rc == POLAR_OK; ++i) {
    // each class has one quantisation (its plans' LLR type)
    switch (cls[i].sel.quant) {
      case POLAR_F32: rc = launch_class_t<float>(A, cls[i], heads + i, heads, s); break;
      case POLAR_I16: rc = launch_class_t<int16_t>(A, cls[i], heads + i, heads, s); break;
      default: rc = launch_class_t<int8_t>(A, cls[i], heads + i, heads, s); break;
    }
  }
  if (ev_end) (void)hipEventRecord(ev_end, s);
  return rc;
}

template <typename T, int NW>
static int launch_plain_t(const KArgs& A, uint32_t lds, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((k_decode_plain<T, NW>), dim3(grid), dim3(NW * 64), lds, s, A);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_decode_plain(uint32_t quant, const KArgs& A, uint32_t lds, uint32_t grid,
                        hipStream_t s) {
  switch (quant) {
    case POLAR_F32: return launch_plain_t<float, 1>(A, lds, grid, s);
    case POLAR_I16: return launch_plain_t<int16_t, 1>(A, lds, grid, s);
    default: return launch_plain_t<int8_t, 1>(A, lds, grid, s);
  }
}

template <typename T>
static int launch_tiered_t(const KArgs& A, const TierPlan& tp, uint32_t* state, uint32_t* heads,
                           uint32_t* xl, hipStream_t s, hipEvent_t* ev) {
  const uint32_t blocks = (A.n_frames + 255) / 256 < 2048 ? (A.n_frames + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_heads_reset, dim3(1), dim3(64), 0, s, heads, 2 * kClaimSegs);
  hipLaunchKernelGGL(k_state_init, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, A, state);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (tp.run_sc && tp.sc_q) {
    const int rc = launch_decode_rq1(tp.sc_q, A, tp.n_ops, tp.grid_q, state, s);
    if (rc) return rc;
  } else if (tp.run_sc && tp.sc_x) {
    KArgs As = A;
    As.spill_stride = tp.spill_sc;
    const int rc = launch_decode_scx(As, tp.grid_scx, state, s);
    if (rc) return rc;
  } else if (tp.run_sc) {
    KArgs As = A;
    As.sc_groot = tp.sc_groot;
    const int rc = launch_decode_sc(VT<T>::INT ? (sizeof(T) == 2 ? POLAR_I16 : POLAR_I8) : POLAR_F32,
                                    As, tp.lds_sc, tp.grid_sc, state, ClassSel{}, s);
    if (rc) return rc;
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (tp.run_x2) {
    KArgs Ax = A;
    Ax.spill_stride = tp.spill_x2;
    const int rc = launch_decode_listx(Ax, tp.grid_x2, state, xl, s);
    if (rc) return rc;
  }
  KArgs Aa = A, Ab = A;
  Aa.spill_stride = tp.spill_a;
  Ab.spill_stride = tp.spill_b;
  // with the path-per-lane stages from L = 4 on (and the L = 2 stage one
  // frame per lane wherever the plan has one), list tier A has no frames
  if (tp.run_a && !tp.run_p)
    hipLaunchKernelGGL((k_decode_list<T, 1, (int)kTierALmax>), dim3(tp.grid_a), dim3(64), tp.lds_a,
                       s, Aa, state, heads, 2u, kTierALmax, tp.chunk_a);
  if (ev) (void)hipEventRecord(ev[2], s);
  if (tp.run_p) {
    KArgs Ap = A;
    Ap.spill_stride = tp.spill_p;
    for (uint32_t i = 0; i < tp.n_p; ++i) {
      const int rc = tp.sc_q && tp.p_stage[i] <= 16
                         ? launch_decode_rqL(tp.sc_q, tp.p_stage[i], A, tp.n_ops, tp.grid_ql[i], state, xl, s)
                         : launch_decode_listp(tp.p_stage[i], Ap, tp.grid_p[i], tp.grid_pm, tp.grid_pl,
                                               tp.lds_pl, state, xl, s);
      if (rc) return rc;
    }
  } else if (tp.run_b) {
    hipLaunchKernelGGL((k_decode_list<T, kListWaves, (int)kMaxL>), dim3(tp.grid_b),
                       dim3(kListWaves * 64), tp.lds_b, s, Ab, state, heads + kClaimSegs,
                       tp.run_a ? kTierALmax + 1 : 2u, kMaxL, tp.chunk_b);
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_decode_tiered(uint32_t quant, const KArgs& A, const TierPlan& tp, uint32_t* state,
                         uint32_t* heads, uint32_t* xl, hipStream_t s, hipEvent_t* ev) {
  switch (quant) {
    case POLAR_F32: return launch_tiered_t<float>(A, tp, state, heads, xl, s, ev);
    case POLAR_I16: return launch_tiered_t<int16_t>(A, tp, state, heads, xl, s, ev);
    default: return launch_tiered_t<int8_t>(A, tp, state, heads, xl, s, ev);
  }
}

}  // namespace polar
