// Device helpers shared by the decoder kernels: value traits of the three
// arithmetic modes, the f / g node updates, packed element access, LDS vector
// access and wave shuffles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace polar {

// ------------------------------------------------------------ value traits
template <typename T>
struct VT;
template <>
struct VT<float> {
  static constexpr uint32_t E = 4, VMAX = 4;
  using Acc = float;
  using Key = unsigned long long;
  static constexpr bool INT = false;
  static constexpr int Q = 0;
};
template <>
struct VT<int16_t> {
  static constexpr uint32_t E = 2, VMAX = 8;
  using Acc = int;
  using Key = uint32_t;
  static constexpr bool INT = true;
  static constexpr int Q = 32767;
};
template <>
struct VT<int8_t> {
  static constexpr uint32_t E = 1, VMAX = 16;
  using Acc = int;
  using Key = uint32_t;
  static constexpr bool INT = true;
  static constexpr int Q = 127;
};

// f = sign(a b) min(|a|, |b|) with the sign taken from the operand signs;
// g = (1 - 2 s) a + b, saturated in the integer modes (Sec. II-B1, III-B3).
__device__ __forceinline__ float f_op(float a, float b) {
  const float m = fminf(fabsf(a), fabsf(b));
  return ((a < 0.f) != (b < 0.f)) ? -m : m;
}
__device__ __forceinline__ float g_op(float a, float b, uint32_t s) { return s ? (b - a) : (b + a); }
// Integer f in branch-free form: max(min(a, b), -max(a, b)) equals
// sign(a) sign(b) min(|a|, |b|) for all integers (both >= 0: min(a, b);
// both <= 0: -max(a, b) = min(|a|, |b|); mixed signs: the negative operand
// or the negated positive one, whichever is closer to zero).
__device__ __forceinline__ int f_opi(int a, int b) { return max(min(a, b), -max(a, b)); }
template <int Q>
__device__ __forceinline__ int g_opi(int a, int b, uint32_t s) {
  const int v = s ? (b - a) : (b + a);
  return max(-Q, min(Q, v));
}

// ------------------------------------ packed int8 element arithmetic
// Four int8 LLRs per 32-bit word, element i in byte i.
__device__ __forceinline__ int sx8(uint32_t w, int i) { return (int)(int8_t)(w >> (8 * i)); }

// f and g of four packed elements work on pairs of 16-bit lanes: element i
// of a word goes to the high byte of a 16-bit lane (v_perm_b32), so that the
// packed 16-bit min / max / add instructions compute on 256 times the value
// and the result is the high bytes again.  For values in [-127, 127] this is
// exactly f_opi / g_opi.
typedef short s16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ s16x2 as_s16x2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ uint32_t as_u32(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
// f of four packed elements: max(min(a, b), -max(a, b))
__device__ __forceinline__ uint32_t f4(uint32_t a, uint32_t b) {
  const s16x2 z = {0, 0};
  const s16x2 al = as_s16x2(__builtin_amdgcn_perm(0u, a, 0x010C000Cu));
  const s16x2 ah = as_s16x2(__builtin_amdgcn_perm(0u, a, 0x030C020Cu));
  const s16x2 bl = as_s16x2(__builtin_amdgcn_perm(0u, b, 0x010C000Cu));
  const s16x2 bh = as_s16x2(__builtin_amdgcn_perm(0u, b, 0x030C020Cu));
  const s16x2 rl = __builtin_elementwise_max(__builtin_elementwise_min(al, bl),
                                             z - __builtin_elementwise_max(al, bl));
  const s16x2 rh = __builtin_elementwise_max(__builtin_elementwise_min(ah, bh),
                                             z - __builtin_elementwise_max(ah, bh));
  return __builtin_amdgcn_perm(as_u32(rh), as_u32(rl), 0x07050301u);
}
// g of four packed elements, saturated at [-127, 127]; bit i of s is the left
// partial sum of element i.  The sum bits become byte masks m (0xFF where
// the element is negated); a negated operand is its bitwise complement
// over a low byte of 0xFF (-256 a - 1), a kept one a over a low byte of 0,
// and b's low bytes are 0xFF, so the 16-bit sum's high byte is b + a or
// b - a exactly; the clamped add and a max at -127 * 256 saturate.
__device__ __forceinline__ uint32_t g4(uint32_t a, uint32_t b, uint32_t s) {
  // bit i of the nibble to bit 8 i (the four shifted copies do not
  // overlap), then each such bit to a whole byte: 0x80 - x per byte (no
  // borrow crosses a byte) is 0x80 or 0x7F, flipped at bit 7 to 0 or 0xFF
  const uint32_t x = ((s & 15u) * 0x00204081u) & 0x01010101u;
  const uint32_t m = (0x80808080u - x) ^ 0x80808080u;
  const uint32_t an = a ^ m;
  const s16x2 al = as_s16x2(__builtin_amdgcn_perm(m, an, 0x01050004u));
  const s16x2 ah = as_s16x2(__builtin_amdgcn_perm(m, an, 0x03070206u));
  const s16x2 bl = as_s16x2(__builtin_amdgcn_perm(0u, b, 0x010D000Du));
  const s16x2 bh = as_s16x2(__builtin_amdgcn_perm(0u, b, 0x030D020Du));
  const s16x2 lo = {-127 * 256, -127 * 256};
  const s16x2 rl = __builtin_elementwise_max(__builtin_elementwise_add_sat(bl, al), lo);
  const s16x2 rh = __builtin_elementwise_max(__builtin_elementwise_add_sat(bh, ah), lo);
  return __builtin_amdgcn_perm(as_u32(rh), as_u32(rl), 0x07050301u);
}
// hard decisions (sign bits) of four packed elements, element i at bit i:
// a dot product of the sign bits with the weights 1, 2, 4, 8
__device__ __forceinline__ uint32_t hd4(uint32_t w) {
  return __builtin_amdgcn_udot4((w >> 7) & 0x01010101u, 0x08040201u, 0u, false);
}

template <typename T>
__device__ __forceinline__ typename VT<T>::Acc as_acc(T v) {
  return (typename VT<T>::Acc)v;
}

// Element k of a small packed vector held in 32-bit words.
template <typename T>
__device__ __forceinline__ T get_el(const uint32_t* w, int k);
template <>
__device__ __forceinline__ float get_el<float>(const uint32_t* w, int k) {
  return __uint_as_float(w[k]);
}
template <>
__device__ __forceinline__ int16_t get_el<int16_t>(const uint32_t* w, int k) {
  return (int16_t)(w[k >> 1] >> ((k & 1) * 16));
}
template <>
__device__ __forceinline__ int8_t get_el<int8_t>(const uint32_t* w, int k) {
  return (int8_t)(w[k >> 2] >> ((k & 3) * 8));
}
template <typename T>
__device__ __forceinline__ void put_el(uint32_t* w, int k, T v);
template <>
__device__ __forceinline__ void put_el<float>(uint32_t* w, int k, float v) {
  w[k] = __float_as_uint(v);
}
template <>
__device__ __forceinline__ void put_el<int16_t>(uint32_t* w, int k, int16_t v) {
  w[k >> 1] |= ((uint32_t)(uint16_t)v) << ((k & 1) * 16);
}
template <>
__device__ __forceinline__ void put_el<int8_t>(uint32_t* w, int k, int8_t v) {
  w[k >> 2] |= ((uint32_t)(uint8_t)v) << ((k & 3) * 8);
}

template <int NB>
__device__ __forceinline__ void lds_ld(const char* p, uint32_t* w) {
  if constexpr (NB == 16) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  } else if constexpr (NB == 8) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    w[0] = v.x; w[1] = v.y;
  } else if constexpr (NB == 4) {
    w[0] = *reinterpret_cast<const uint32_t*>(p);
  } else if constexpr (NB == 2) {
    w[0] = *reinterpret_cast<const uint16_t*>(p);
  } else {
    w[0] = *reinterpret_cast<const uint8_t*>(p);
  }
}
template <int NB>
__device__ __forceinline__ void lds_st(char* p, const uint32_t* w) {
  if constexpr (NB == 16) {
    *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
  } else if constexpr (NB == 8) {
    *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[1]);
  } else if constexpr (NB == 4) {
    *reinterpret_cast<uint32_t*>(p) = w[0];
  } else if constexpr (NB == 2) {
    *reinterpret_cast<uint16_t*>(p) = (uint16_t)w[0];
  } else {
    *reinterpret_cast<uint8_t*>(p) = (uint8_t)w[0];
  }
}

template <typename T, int V>
__device__ __forceinline__ void f_chunk(const uint32_t* a, const uint32_t* b, uint32_t* o) {
#pragma unroll
  for (int k = 0; k < V; ++k) {
    if constexpr (VT<T>::INT)
      put_el<T>(o, k, (T)f_opi(get_el<T>(a, k), get_el<T>(b, k)));
    else
      put_el<T>(o, k, f_op(get_el<T>(a, k), get_el<T>(b, k)));
  }
}
template <typename T, int V>
__device__ __forceinline__ void g_chunk(const uint32_t* a, const uint32_t* b, uint32_t s,
                                        uint32_t* o) {
#pragma unroll
  for (int k = 0; k < V; ++k) {
    if constexpr (VT<T>::INT)
      put_el<T>(o, k, (T)g_opi<VT<T>::Q>(get_el<T>(a, k), get_el<T>(b, k), (s >> k) & 1u));
    else
      put_el<T>(o, k, g_op(get_el<T>(a, k), get_el<T>(b, k), (s >> k) & 1u));
  }
}

__device__ __forceinline__ uint32_t lg2(uint32_t x) { return 31u - __clz(x); }

// Values that are the same in every lane (a frame's plan, its node program,
// list sizes, loop bounds) are pinned to scalar registers, so that the
// control flow built on them is scalar (s_cbranch_scc) rather than
// exec-masked.  Call only where every lane of the wave is active.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
template <typename Q>
__device__ __forceinline__ Q* uni_ptr(Q* p) {
  return reinterpret_cast<Q*>(uni64(reinterpret_cast<uint64_t>(p)));
}

// ------------------------------------------------------- wave primitives
// v of lane src (0..63) of the wave, without the width arithmetic of
// __shfl (ds_bpermute takes a byte address).
template <typename V>
__device__ __forceinline__ V bperm(V v, uint32_t src) {
  static_assert(sizeof(V) == 4, "32-bit values");
  return __builtin_bit_cast(V, __builtin_amdgcn_ds_bpermute((int)(src << 2), __builtin_bit_cast(int, v)));
}

template <typename K>
__device__ __forceinline__ K shfl_xor_k(K v, int m) {
  if constexpr (sizeof(K) == 8) {
    const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((K)hi << 32) | lo;
  } else {
    return __shfl_xor(v, m, 64);
  }
}

}  // namespace polar
