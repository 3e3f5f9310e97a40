// Shared device/host helpers of the SMC library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace smc {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

enum Act { ACT_TANH = 0, ACT_RELU = 1 };

// Round-to-nearest-even float -> bf16 conversion (the hardware convert on gfx950).
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }
__device__ __forceinline__ float from_bf16(__bf16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T cvt_out(float v);
template <> __device__ __forceinline__ float cvt_out<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 cvt_out<__bf16>(float v) { return to_bf16(v); }

template <typename T> __device__ __forceinline__ float cvt_in(T v);
template <> __device__ __forceinline__ float cvt_in<float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt_in<__bf16>(__bf16 v) { return from_bf16(v); }

__device__ __forceinline__ float act_fwd(float z, int act) {
  return act == ACT_RELU ? fmaxf(z, 0.0f) : tanhf(z);
}
// derivative expressed through the activation value a = act(z)
__device__ __forceinline__ float act_grad_from_out(float a, int act) {
  return act == ACT_RELU ? (a > 0.0f ? 1.0f : 0.0f) : 1.0f - a * a;
}

// ------------------------------------------------------------------ wave / block reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Deterministic block sum (fixed tree order); scratch needs blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += scratch[i];
  return r;
}
__device__ __forceinline__ double block_max(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double r = scratch[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, scratch[i]);
  return r;
}

// ------------------------------------------------------------------ Philox-4x32-10
// Salmon et al., "Parallel random numbers: as easy as 1, 2, 3" (SC'11).
__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    u32x4 n;
    n[0] = hi1 ^ c[1] ^ k0;
    n[1] = lo1;
    n[2] = hi0 ^ c[3] ^ k1;
    n[3] = lo0;
    c = n;
  }
  return c;
}

// uniform in (0, 1]: (x + 1) * 2^-32 with 24 significant bits kept exact
__device__ __forceinline__ float u01_open0(uint32_t x) {
  return (float)((x >> 8) + 1u) * (1.0f / 16777216.0f);
}
// uniform in [0, 1)
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// Four standard normals from one Philox block (Box-Muller on two uniform pairs).
__device__ __forceinline__ f32x4 normal4(u32x4 r) {
  f32x4 out;
  const float TWO_PI = 6.283185307179586f;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float u1 = u01_open0(r[2 * p]);
    const float u2 = u01(r[2 * p + 1]);
    const float rad = sqrtf(-2.0f * logf(u1));
    float s, c;
    sincosf(TWO_PI * u2, &s, &c);
    out[2 * p] = rad * c;
    out[2 * p + 1] = rad * s;
  }
  return out;
}

}  // namespace smc
