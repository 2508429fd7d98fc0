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

// f of four packed elements
__device__ __forceinline__ uint32_t f4(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) r |= (uint32_t)(uint8_t)f_opi(sx8(a, i), sx8(b, i)) << (8 * i);
  return r;
}
// g of four packed elements (saturated at the int8 range); bit i of s is the
// left partial sum of element i
__device__ __forceinline__ uint32_t g4(uint32_t a, uint32_t b, uint32_t s) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    r |= (uint32_t)(uint8_t)g_opi<VT<int8_t>::Q>(sx8(a, i), sx8(b, i), (s >> i) & 1u) << (8 * i);
  return r;
}
// hard decisions (sign bits) of four packed elements, element i at bit i:
// the sign bits 7, 15, 23, 31 are gathered into bits 28..31 by one product
// whose partial terms never overlap
__device__ __forceinline__ uint32_t hd4(uint32_t w) {
  return ((w & 0x80808080u) * 0x00204081u) >> 28;
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
