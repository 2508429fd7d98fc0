// Systematic polar encoder with CRC attachment (Sec. II-A, Sec. II-B4) and
// the Monte-Carlo workload generator (BPSK over AWGN, Sec. II-C) on gfx950.
// The generator is counter-based (Philox4x32-10, Salmon et al., SC'11) so
// that any frame range regenerates independently.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace polar {

// Philox4x32 with 10 rounds: multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key
// increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

constexpr uint32_t kTagNoise = 0x4E4F4953u;  // stream tags in the 4th counter word
constexpr uint32_t kTagData = 0x44415441u;

// x = v F^{(x)n} on N packed bits, one 32-bit word per lane (lane w holds
// bits [32w, 32w + 32)); stages commute.
__device__ __forceinline__ uint32_t polar_xform(uint32_t u, uint32_t w, uint32_t N) {
  const uint32_t msk[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu, 0x0000FFFFu};
#pragma unroll
  for (uint32_t s = 1, k = 0; k < 5; s <<= 1, ++k)
    if (s < N) u ^= (u >> s) & msk[k];
  for (uint32_t S = 1; 32u * S < N; S <<= 1) {
    const uint32_t v = __shfl_xor(u, (int)S, 64);
    if (!(w & S)) u ^= v;
  }
  return u;
}

__global__ __launch_bounds__(64) void k_encode(const DevPlan* P, const uint32_t* data,
                                               uint32_t* code, uint32_t n_frames) {
  const uint32_t f = blockIdx.x;
  if (f >= n_frames) return;
  const uint32_t w = threadIdx.x, bw = P->bw, N = P->N, c = P->c;
  const uint32_t* dmask = plan_tab(P, P->off_datamask);
  const uint32_t* dpre = plan_tab(P, P->off_dataprefix);
  const uint32_t* crccol = plan_tab(P, P->off_crccol);
  const uint32_t* crcpos = plan_tab(P, P->off_crcpos);
  const uint32_t* imask = plan_tab(P, P->off_infomask);
  const uint32_t* D = data + (size_t)f * P->info_words;
  uint32_t u = 0;
  if (w < bw) {
    // deposit data bits t = pre .. pre + popcount - 1 on the data positions
    uint32_t m = dmask[w], t = dpre[w];
    while (m) {
      const uint32_t b = __ffs(m) - 1;
      u |= ((D[t >> 5] >> (t & 31)) & 1u) << b;
      ++t;
      m &= m - 1u;
    }
  }
  // CRC(data) as the XOR of the syndrome columns of the set data bits
  uint32_t s = 0;
  if (w < bw) {
    uint32_t v = u;
    while (v) {
      const uint32_t b = __ffs(v) - 1;
      s ^= crccol[(w << 5) + b];
      v &= v - 1u;
    }
  }
  for (int k = 32; k >= 1; k >>= 1) s ^= __shfl_xor(s, k, 64);
  for (uint32_t t = 0; t < c; ++t) {
    const uint32_t pos = crcpos[t];
    if ((pos >> 5) == w) u |= ((s >> (c - 1 - t)) & 1u) << (pos & 31);
  }
  u = polar_xform(u, w, N);
  if (w < bw) u &= imask[w];
  u = polar_xform(u, w, N);
  if (w < bw) code[(size_t)f * P->code_words + w] = u;
}

__global__ void k_gen_data(uint32_t iw, uint32_t kd, uint64_t seed, uint64_t frame0,
                           uint32_t n_frames, uint32_t* out) {
  const uint32_t g4 = (iw + 3) / 4;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (uint64_t)n_frames * g4) return;
  const uint32_t f = (uint32_t)(gid / g4), g = (uint32_t)(gid % g4);
  const uint64_t fr = frame0 + f;
  const uint4 r = philox4x32_10(make_uint4(g, (uint32_t)fr, (uint32_t)(fr >> 32), kTagData),
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t vals[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t wi = g * 4 + k;
    if (wi < iw) {
      uint32_t v = vals[k];
      const uint32_t lo = wi * 32;
      if (lo + 32 > kd) v &= (kd - lo >= 32) ? ~0u : ((1u << (kd - lo)) - 1u);
      out[(size_t)f * iw + wi] = v;
    }
  }
}

template <typename T>
__device__ __forceinline__ T quantise(float l, float scale, int Q) {
  if constexpr (sizeof(T) == 4) {
    return l;
  } else {
    float q = rintf(l * scale);
    q = fmaxf(-(float)Q, fminf((float)Q, q));
    return (T)(int)q;
  }
}

template <typename T>
__global__ void k_channel(const uint32_t* code, uint32_t cw, uint32_t p0, uint32_t n_tx,
                          uint32_t n_frames, float sigma, float llr_scale, float qscale, int Q,
                          uint64_t seed, uint64_t frame0, T* out) {
  const uint32_t g4 = (n_tx + 3) / 4;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (uint64_t)n_frames * g4) return;
  const uint32_t f = (uint32_t)(gid / g4), g = (uint32_t)(gid % g4);
  const uint64_t fr = frame0 + f;
  const uint4 r = philox4x32_10(make_uint4(g, (uint32_t)fr, (uint32_t)(fr >> 32), kTagNoise),
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const float inv = 2.3283064365386963e-10f;  // 2^-32
  const float u0 = ((float)r.x + 0.5f) * inv, u1 = ((float)r.y + 0.5f) * inv;
  const float u2 = ((float)r.z + 0.5f) * inv, u3 = ((float)r.w + 0.5f) * inv;
  const float ra = sqrtf(-2.f * logf(u0)), rb = sqrtf(-2.f * logf(u2));
  float sa, ca, sb, cb;
  sincospif(2.f * u1, &sa, &ca);
  sincospif(2.f * u3, &sb, &cb);
  const float z[4] = {ra * ca, ra * sa, rb * cb, rb * sb};
  const uint32_t* C = code + (size_t)f * cw;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = g * 4 + k;
    if (i < n_tx) {
      const uint32_t j = p0 + i;  // sent positions start after the punctured ones
      const float s = ((C[j >> 5] >> (j & 31)) & 1u) ? -1.f : 1.f;
      const float y = s + sigma * z[k];
      out[(size_t)f * n_tx + i] = quantise<T>(llr_scale * y, qscale, Q);
    }
  }
}

template <typename T>
__global__ void k_quantize(const float* in, uint32_t n, float qscale, int Q, T* out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = quantise<T>(in[i], qscale, Q);
}

int launch_quantize(const float* d_llr, uint32_t n, uint32_t quant, int32_t frac_bits, void* d_out,
                    hipStream_t s) {
  if (n == 0) return POLAR_OK;
  const float qscale = std::ldexp(1.0f, frac_bits);
  const uint32_t blocks = (uint32_t)(((uint64_t)n + 255) / 256);
  switch (quant) {
    case POLAR_F32:
      hipLaunchKernelGGL(k_quantize<float>, dim3(blocks), dim3(256), 0, s, d_llr, n, qscale, 0,
                         (float*)d_out);
      break;
    case POLAR_I16:
      hipLaunchKernelGGL(k_quantize<int16_t>, dim3(blocks), dim3(256), 0, s, d_llr, n, qscale, 32767,
                         (int16_t*)d_out);
      break;
    default:
      hipLaunchKernelGGL(k_quantize<int8_t>, dim3(blocks), dim3(256), 0, s, d_llr, n, qscale, 127,
                         (int8_t*)d_out);
      break;
  }
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_encode(const DevPlan* dplan, const DevPlan& h, const uint32_t* d_data,
                  uint32_t* d_code, uint32_t n_frames, hipStream_t s) {
  if (n_frames == 0) return POLAR_OK;
  hipLaunchKernelGGL(k_encode, dim3(n_frames), dim3(64), 0, s, dplan, d_data, d_code, n_frames);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_gen_data(const DevPlan& h, uint64_t seed, uint64_t frame0, uint32_t n_frames,
                    uint32_t* d_data, hipStream_t s) {
  if (n_frames == 0) return POLAR_OK;
  const uint64_t total = (uint64_t)n_frames * ((h.info_words + 3) / 4);
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  hipLaunchKernelGGL(k_gen_data, dim3(blocks), dim3(256), 0, s, h.info_words, h.k_data, seed,
                     frame0, n_frames, d_data);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

int launch_channel(const DevPlan& h, const uint32_t* d_code, uint32_t n_frames, float ebn0_db,
                   int32_t frac_bits, uint64_t seed, uint64_t frame0, void* d_llr,
                   hipStream_t s) {
  if (n_frames == 0) return POLAR_OK;
  const double rate = double(h.k_data) / double(h.n_tx);
  const double sigma = std::sqrt(1.0 / (2.0 * rate * std::pow(10.0, ebn0_db / 10.0)));
  const float llr_scale = (float)(2.0 / (sigma * sigma));
  const float qscale = std::ldexp(1.0f, frac_bits);
  const uint64_t total = (uint64_t)n_frames * ((h.n_tx + 3) / 4);
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  switch (h.quant) {
    case POLAR_F32:
      hipLaunchKernelGGL(k_channel<float>, dim3(blocks), dim3(256), 0, s, d_code, h.code_words,
                         h.n_punct, h.n_tx, n_frames, (float)sigma, llr_scale, qscale, 0, seed, frame0,
                         (float*)d_llr);
      break;
    case POLAR_I16:
      hipLaunchKernelGGL(k_channel<int16_t>, dim3(blocks), dim3(256), 0, s, d_code, h.code_words,
                         h.n_punct, h.n_tx, n_frames, (float)sigma, llr_scale, qscale, 32767, seed, frame0,
                         (int16_t*)d_llr);
      break;
    default:
      hipLaunchKernelGGL(k_channel<int8_t>, dim3(blocks), dim3(256), 0, s, d_code, h.code_words,
                         h.n_punct, h.n_tx, n_frames, (float)sigma, llr_scale, qscale, 127, seed, frame0,
                         (int8_t*)d_llr);
      break;
  }
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EHIP;
}

}  // namespace polar
