// Data-movement and reduction kernels of the particle-batched convolutional network
// (conv3x3 -> ReLU -> conv3x3 -> ReLU -> 2x2 average pool -> linear, NHWC images).
//
// The contractions run on the MFMA GEMM (gemm.hip) over explicit patch matrices:
//   conv1   [R x K1p] . [J*C1 x K1p]^T          one dense GEMM, the image patches are shared by
//                                                 every particle (R = images x H x W pixel rows)
//   conv2   [R x 9C1] . [C2 x 9C1]^T            batched over particles
//   linear  [n x F3]  . [ncls x F3]^T           batched over particles
//   backward: errors through the linear layer ([n x 16] . [F3 x 16]^T), the conv2 weight
//   gradient ([C2 x R] . [(9C1+1) x R]^T, the ones row yields the bias), the conv2 input error
//   ([R x C2] . [9C1 x C2]^T, then summed back onto pixels) and the conv1 weight gradient
//   ([J*C1 x R] . [(K1+1) x R]^T).
// The kernels here build those operands (im2col in both orientations, pooling and its
// adjoint with the ReLU masks, the col2im sum), the per-particle log-likelihood with its
// output error, and the linear layer's weight gradient.  Patch index k = tap * C + c with
// tap = ky * 3 + kx; output pixel (y, x) reads input pixel (y + ky - 1, x + kx - 1).
#include "kernels.h"

#include <algorithm>

namespace smc {

namespace {

// input pixel read by patch element (tap) of output pixel pix, or -1 outside the image
__device__ __forceinline__ int tap_src(const CnnDims& d, int pix, int tap) {
  const int y = pix / d.W, x = pix - y * d.W;
  const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
  return (yy >= 0 && yy < d.H && xx >= 0 && xx < d.W) ? yy * d.W + xx : -1;
}

// Index layout of the kernels below: blockIdx.z = particle, blockIdx.y = image (or tap /
// channel vector), blockIdx.x * 256 + threadIdx.x the position inside it, so every thread
// decomposes a 32-bit index with at most two divisions (the launchers check the ranges).
// Consecutive lanes take consecutive pixels: the reads, which these kernels are bound by,
// then come from neighbouring rows.

// p1[r][k] = patch of image pixel r (k < K1), zero for K1 <= k < K1p; grid (HW K1p / 256, images)
template <typename T>
__global__ void im2col_x_kernel(const T* __restrict__ X, int64_t xld, int64_t c0, int mcv, CnnDims d,
                                T* __restrict__ p1) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.HW * d.K1p) return;
  const int64_t n = blockIdx.y;
  const int pix = e / d.K1p, k = e - pix * d.K1p;
  const int64_t i = n * d.HW * d.K1p + e;
  float v = 0.0f;
  if (k < d.K1) {
    const int tap = k / d.Cin, c = k - tap * d.Cin;
    const int s = tap_src(d, pix, tap);
    if (s >= 0) v = cvt_in<T>(X[(c0 + n) * xld + (int64_t)s * d.Cin + c]);
  }
  p1[i] = cvt_out<T>(v);
}

// p1t[k][r] (row stride ld): the same patches transposed, with a ones row at k = K1;
// grid (R / 256, K1 + 1)
template <typename T>
__global__ void im2col_xt_kernel(const T* __restrict__ X, int64_t xld, int64_t c0, int mcv, CnnDims d, int64_t ld,
                                 T* __restrict__ p1t) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mcv * d.HW) return;
  const int k = blockIdx.y;
  float v = 1.0f;
  if (k < d.K1) {
    const int64_t n = r / d.HW;
    const int pix = r - (int)n * d.HW;
    const int tap = k / d.Cin, c = k - tap * d.Cin;
    const int s = tap_src(d, pix, tap);
    v = s >= 0 ? cvt_in<T>(X[(c0 + n) * xld + (int64_t)s * d.Cin + c]) : 0.0f;
  }
  p1t[(int64_t)k * ld + r] = cvt_out<T>(v);
}

// big[j][r][k] (row length K2 = 9 C1) = act1 patch, in 16-byte vectors of channels
// grid (HW K2 / (VEC 256), images, particles)
template <typename T>
__global__ void im2col_a_kernel(const T* __restrict__ act1, int64_t sA, int mcv, CnnDims d, int J,
                                T* __restrict__ big, int64_t sB) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int nv = d.K2 / VEC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.HW * nv) return;
  const int j = blockIdx.z;
  const int64_t n = blockIdx.y;
  const int pix = e / nv, kv = e - pix * nv;
  const int64_t r = n * d.HW + pix;
  const int k = kv * VEC, tap = k / d.C1, c = k - tap * d.C1;
  const int s = tap_src(d, pix, tap);
  u32x4 v = {0u, 0u, 0u, 0u};
  if (s >= 0) v = *(const u32x4*)(act1 + (int64_t)j * sA + (n * d.HW + s) * d.C1 + c);
  *(u32x4*)(big + (int64_t)j * sB + r * d.K2 + k) = v;
}

// bigT[j][k][r] (row stride ld) = act1 patch transposed, ones row at k = K2.  One thread per
// (j, tap, 8-channel vector, pixel r), pixels fastest: a 16-byte read of 8 channels of the
// source pixel, eight 2-byte writes that are contiguous across the wave's pixels.
// lanes take (pixel, channel vector) with the vector fastest, so a wave reads whole source
// pixels; grid (R C1 / (VEC 256), 10, particles): y = tap, y = 9 writes the ones row
template <typename T>
__global__ void im2col_at_kernel(const T* __restrict__ act1, int64_t sA, int mcv, CnnDims d, int J, int64_t ld,
                                 T* __restrict__ bigT, int64_t sB) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int nv = d.C1 / VEC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mcv * d.HW * nv) return;
  const int r = e / nv;
  const int c = (e - r * nv) * VEC;
  const int j = blockIdx.z;
  const int tap = blockIdx.y;
  if (tap == 9) {
    // the ones row (bias gradient)
    if (c == 0) bigT[(int64_t)j * sB + (int64_t)d.K2 * ld + r] = cvt_out<T>(1.0f);
    return;
  }
  const int64_t n = r / d.HW;
  const int pix = r - (int)n * d.HW;
  const int s = tap_src(d, pix, tap);
  u32x4 v = {0u, 0u, 0u, 0u};
  if (s >= 0) v = *(const u32x4*)(act1 + (int64_t)j * sA + (n * d.HW + s) * d.C1 + c);
  const T* vv = (const T*)&v;
  T* dst = bigT + (int64_t)j * sB + (int64_t)(tap * d.C1 + c) * ld + r;
#pragma unroll
  for (int t = 0; t < VEC; ++t) dst[(int64_t)t * ld] = vv[t];
}

// pooled[j][n][(py Wp + px) C2 + c] = mean of the 2x2 block of act2
// grid (F3 / 256, images, particles)
template <typename T>
__global__ void pool_kernel(const T* __restrict__ act2, int64_t sA, int mcv, CnnDims d, int J,
                            T* __restrict__ pooled, int64_t sP) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= d.F3) return;
  const int j = blockIdx.z;
  const int64_t n = blockIdx.y;
  const int p = f / d.C2, c = f - p * d.C2;
  const int py = p / d.Wp, px = p - py * d.Wp;
  const T* a = act2 + (int64_t)j * sA + (n * d.HW + (2 * py) * d.W + 2 * px) * d.C2 + c;
  const float s = cvt_in<T>(a[0]) + cvt_in<T>(a[d.C2]) + cvt_in<T>(a[(int64_t)d.W * d.C2]) +
                  cvt_in<T>(a[(int64_t)(d.W + 1) * d.C2]);
  pooled[(int64_t)j * sP + n * d.F3 + f] = cvt_out<T>(0.25f * s);
}

// Per particle (one workgroup): log p(y_n | x_n) from logits + bias, summed in FP64 in a
// fixed order into ll_acc[j]; TRAIN also writes d3[j][n][c] = lambda_j (1{c = y_n} - softmax)
// (zero for ncls <= c < 16); PREDICT writes log-probabilities instead.
template <typename T>
__global__ __launch_bounds__(256) void cnn_ll_kernel(const CnnLLArgs a) {
  __shared__ double red[8];
  const int j = blockIdx.x;
  const float lam = a.scale ? (float)a.scale[j] : (float)a.lambda;
  const float lam_b = a.scale ? lam : (float)a.lambda_b;
  const float* b3 = a.bias + (int64_t)j * a.ncls;
  double acc = 0.0, acc_b = 0.0;
  for (int n = threadIdx.x; n < a.mcv; n += blockDim.x) {
    const float* z = a.logits + ((int64_t)j * a.mc + n) * a.ncls;
    float zz[16];
    float mx = -INFINITY;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      zz[c] = c < a.ncls ? z[c] + b3[c] : -INFINITY;
      mx = fmaxf(mx, zz[c]);
    }
    float se = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) se += c < a.ncls ? expf(zz[c] - mx) : 0.0f;
    const float lse = mx + logf(se);
    if (a.mode == HEAD_PREDICT) {
      float* lp = a.logp + ((int64_t)j * a.ld_logp + a.c0 + n) * a.ncls;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < a.ncls) lp[c] = zz[c] - lse;
      continue;
    }
    const int y = a.ylab[a.c0 + n];
    float zy = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c == y) zy = zz[c];
    const bool segb = a.c0 + n >= a.m_split;  // second segment of a two-segment target
    acc += (double)(zy - lse);
    if (segb) acc_b += (double)(zy - lse);
    const float lm = segb ? lam_b : lam;
    if (a.mode == HEAD_TRAIN) {
      T* d = (T*)a.d3 + ((int64_t)j * a.mc + n) * 16;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        d[c] = cvt_out<T>(c < a.ncls ? lm * ((c == y ? 1.0f : 0.0f) - expf(zz[c] - lse)) : 0.0f);
    }
  }
  if (a.mode == HEAD_PREDICT) return;
  const double v = wave_sum(acc);
  const double vb = wave_sum(acc_b);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v;
    red[4 + (threadIdx.x >> 6)] = vb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, sb = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      s += red[q];
      sb += red[4 + q];
    }
    a.ll_acc[j] = a.beta ? a.ll_acc[j] + s : s;
    if (a.ll_acc_b) a.ll_acc_b[j] = a.beta ? a.ll_acc_b[j] + sb : sb;
  }
}

// linear-layer gradient g[j][off + c (F3+1) + f] (+)= sum_n d3[j][n][c] * [pooled[j][n] | 1][f]
template <typename T>
__global__ __launch_bounds__(256) void cnn_dw3_kernel(const T* __restrict__ d3, const T* __restrict__ pooled,
                                                      int64_t sP, int mc, int mcv, int F3, int ncls, float* g,
                                                      int64_t D, int64_t off, int beta) {
  extern __shared__ float dsh[];  // [mcv][16]
  const int j = blockIdx.y;
  for (int e = threadIdx.x; e < mcv * 16; e += blockDim.x) dsh[e] = cvt_in<T>(d3[((int64_t)j * mc) * 16 + e]);
  __syncthreads();
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > F3) return;
  float acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
  const T* pj = pooled + (int64_t)j * sP;
  for (int n = 0; n < mcv; ++n) {
    const float pv = f < F3 ? cvt_in<T>(pj[(int64_t)n * F3 + f]) : 1.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] += dsh[n * 16 + c] * pv;
  }
  float* gj = g + (int64_t)j * D + off;
  for (int c = 0; c < ncls; ++c) {
    float* p = gj + (int64_t)c * (F3 + 1) + f;
    *p = beta ? *p + acc[c] : acc[c];
  }
}

// error at the conv2 output: d2 = (unpooled dpool / 4) * 1{act2 > 0}, written as rows
// d2[j][r][c] and transposed d2t[j][c][r] (row stride ld).  One thread per (j, 8-channel
// vector, pixel r), pixels fastest: 16-byte reads of act2 and dpool, a 16-byte row write and
// eight 2-byte transposed writes.  Lanes take (pixel, channel vector) with the vector fastest,
// so a wave reads and writes whole pixel rows.  Grid (R C2 / (VEC 256), 1, particles).
template <typename T>
__global__ void unpool_kernel(const T* __restrict__ dpool, int64_t sP, const T* __restrict__ act2, int64_t sA,
                              int mcv, CnnDims d, int J, int64_t ld, T* __restrict__ d2, T* __restrict__ d2t) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int nv = d.C2 / VEC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mcv * d.HW * nv) return;
  const int ri = e / nv;
  const int c = (e - ri * nv) * VEC;
  const int64_t r = ri;
  const int j = blockIdx.z;
  const int64_t n = ri / d.HW;
  const int pix = ri - (int)n * d.HW;
  const int y = pix / d.W, x = pix - y * d.W;
  const int64_t ai = (int64_t)j * sA + r * d.C2 + c;
  const u32x4 av = *(const u32x4*)(act2 + ai);
  const u32x4 pv =
      *(const u32x4*)(dpool + (int64_t)j * sP + n * d.F3 + ((y >> 1) * d.Wp + (x >> 1)) * d.C2 + c);
  const T* a = (const T*)&av;
  const T* pp = (const T*)&pv;
  u32x4 ov;
  T* o = (T*)&ov;
#pragma unroll
  for (int t = 0; t < VEC; ++t) o[t] = cvt_out<T>(cvt_in<T>(a[t]) > 0.0f ? 0.25f * cvt_in<T>(pp[t]) : 0.0f);
  *(u32x4*)(d2 + ai) = ov;
  T* dt = d2t + ((int64_t)j * d.C2 + c) * ld + r;
#pragma unroll
  for (int t = 0; t < VEC; ++t) dt[(int64_t)t * ld] = o[t];
}

// error at the conv1 output: sum over taps of the patch errors that read pixel r, times
// 1{act1 > 0}; written transposed as d1t[j C1 + c][r] (row stride ld).  The patch errors are
// tap-major, dp2[j][tap][r'][c] with tap planes ld * C1 apart.  One thread per (j, pixel r,
// VEC-channel vector), channel vectors fastest: a wave reads one contiguous stretch of each
// tap plane; nine 16-byte patch-error reads, one 16-byte activation read, eight 2-byte writes.
// Grid (R C1 / (VEC 256), 1, particles).
template <typename T>
__global__ void col2im_kernel(const T* __restrict__ dp2, int64_t sB, const T* __restrict__ act1, int64_t sA,
                              int mcv, CnnDims d, int J, int64_t ld, T* __restrict__ d1t) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int nv = d.C1 / VEC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mcv * d.HW * nv) return;
  const int j = blockIdx.z;
  const int ri = e / nv;
  const int c = (e - ri * nv) * VEC;
  const int64_t r = ri;
  const int64_t n = ri / d.HW;
  const int pix = ri - (int)n * d.HW;
  const int y = pix / d.W, x = pix - y * d.W;
  float acc[VEC];
#pragma unroll
  for (int t = 0; t < VEC; ++t) acc[t] = 0.0f;
  const T* pj = dp2 + (int64_t)j * sB + n * d.HW * d.C1 + c;
  const int64_t plane = ld * d.C1;
  for (int tap = 0; tap < 9; ++tap) {
    // output pixel (y - ky + 1, x - kx + 1) reads this pixel through tap (ky, kx)
    const int yo = y - tap / 3 + 1, xo = x - tap % 3 + 1;
    if (yo < 0 || yo >= d.H || xo < 0 || xo >= d.W) continue;
    const u32x4 v = *(const u32x4*)(pj + tap * plane + (int64_t)(yo * d.W + xo) * d.C1);
    const T* vv = (const T*)&v;
#pragma unroll
    for (int t = 0; t < VEC; ++t) acc[t] += cvt_in<T>(vv[t]);
  }
  const u32x4 av = *(const u32x4*)(act1 + (int64_t)j * sA + r * d.C1 + c);
  const T* a = (const T*)&av;
  T* dt = d1t + ((int64_t)j * d.C1 + c) * ld + r;
#pragma unroll
  for (int t = 0; t < VEC; ++t) dt[(int64_t)t * ld] = cvt_out<T>(cvt_in<T>(a[t]) > 0.0f ? acc[t] : 0.0f);
}

// conv1 weight gradient from its K-slice partials: g[j][o (N) + n] (+)= sum over slices s,
// in order, of part[s][j C1 + o][n]
__global__ void slice_sum_kernel(const float* __restrict__ part, int S, int M, int N, int C1, float* g, int64_t D,
                                 int beta) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  float acc = 0.0f;
  for (int k = 0; k < S; ++k) acc += part[(int64_t)k * M * N + e];
  const int m = e / N, n = e - m * N;
  const int j = m / C1, o = m - j * C1;
  float* dst = g + (int64_t)j * D + (int64_t)o * N + n;
  *dst = beta ? *dst + acc : acc;
}

// ------------------------------------------------------------------ implicit conv2 (BF16)
// For 32-pixel-wide images with C1 = 16 and C2 = 32 channels, conv2 and its input error run as
// implicit GEMMs: one workgroup per (8-row band, image, particle) stages the band's activation
// (or error) halo in LDS and contracts it tap by tap on the matrix cores, so no patch matrix is
// written.  A halo pixel's 16-byte channel chunks are stored at slot c ^ f(col), which puts the
// 16 consecutive pixels a half-wave reads at one chunk on 16 distinct bank groups.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s16x4_t;
constexpr int IB = 8;            // output rows per workgroup
constexpr int IHR = IB + 2;      // halo rows
constexpr int IHC = 32 + 2;      // halo columns

// Eight channels (8c .. 8c+7) of the conv2 output error at pixel (y, x) of image n, from the
// pooled-feature error and the ReLU mask: 1{act2 > 0} dpool / 4 (the adjoint of the 2x2 average,
// rounded as unpool_kernel rounds it)
__device__ __forceinline__ u32x4 d2_chunk(const __bf16* __restrict__ act2n, const __bf16* __restrict__ dpooln,
                                          const CnnDims& d, int y, int x, int c) {
  const u32x4 av = *(const u32x4*)(act2n + (y * 32 + x) * 32 + c * 8);
  const u32x4 pv = *(const u32x4*)(dpooln + ((y >> 1) * d.Wp + (x >> 1)) * 32 + c * 8);
  const __bf16* a = (const __bf16*)&av;
  const __bf16* pp = (const __bf16*)&pv;
  u32x4 ov;
  __bf16* o = (__bf16*)&ov;
#pragma unroll
  for (int t = 0; t < 8; ++t) o[t] = to_bf16(from_bf16(a[t]) > 0.0f ? 0.25f * from_bf16(pp[t]) : 0.0f);
  return ov;
}

// act2 = ReLU(conv2(act1) + b2) and pooled = its 2x2 average, for one particle, image and band.
// Wave w computes rows 2w, 2w+1 of the band (one 32x32 MFMA block each: 32 pixels x 32 output
// channels); K runs over the nine taps, one v_mfma_f32_32x32x16_bf16 per tap (16 channels), in
// the same order as the explicit GEMM over the patch row.  The epilogue writes act2 (one pixel's
// 32 channels per 32 lanes) and the pool from the rounded values in pool_kernel's order.
__global__ __launch_bounds__(256) void conv2_fwd_implicit_kernel(const __bf16* __restrict__ act1, int64_t sA1,
                                                                 const __bf16* __restrict__ w2, int64_t ldw,
                                                                 const float* __restrict__ b2, __bf16* __restrict__ act2,
                                                                 int64_t sA2, __bf16* __restrict__ pooled, int64_t sP,
                                                                 CnnDims d) {
  __shared__ __attribute__((aligned(16))) char halo[IHR * IHC * 32];
  const int j = blockIdx.z, n = blockIdx.y, y0 = blockIdx.x * IB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const __bf16* a1 = act1 + (int64_t)j * sA1 + (int64_t)n * d.HW * 16;
  for (int e = tid; e < IHR * IHC * 2; e += 256) {
    const int row = e / (IHC * 2), rem = e - row * (IHC * 2), col = rem >> 1, c = rem & 1;
    const int yy = y0 - 1 + row, xx = col - 1;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (yy >= 0 && yy < d.H && xx >= 0 && xx < 32) v = *(const u32x4*)(a1 + (yy * 32 + xx) * 16 + c * 8);
    *(u32x4*)(halo + (row * IHC + col) * 32 + ((c ^ ((col >> 3) & 1)) << 4)) = v;
  }
  // B fragments of the nine taps: lane l holds W2[l % 32][tap * 16 + 8 (l / 32) .. +7]
  const __bf16* wj = w2 + ((int64_t)j * 32 + (lane & 31)) * ldw + 8 * (lane >> 5);
  u32x4 bfr[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) bfr[t] = *(const u32x4*)(wj + t * 16);
  __syncthreads();
  f32x16 acc[2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[ib][q] = 0.0f;
    const int r = 2 * w + ib;  // band row of this block
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t % 3;
      const int col = (lane & 31) + kx, c = lane >> 5;
      const u32x4 av = *(const u32x4*)(halo + ((r + ky) * IHC + col) * 32 + ((c ^ ((col >> 3) & 1)) << 4));
      acc[ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                        __builtin_bit_cast(bf16x8_t, bfr[t]), acc[ib], 0, 0, 0);
    }
  }
  // epilogue: lane l holds output channel c2 = l % 32 of pixels x = 8 (q / 4) + 4 (l / 32) + q % 4
  const int c2 = lane & 31;
  const float bias = b2[(int64_t)j * 32 + c2];
  __bf16* o2 = act2 + (int64_t)j * sA2 + (int64_t)n * d.HW * 32;
  __bf16 v[2][16];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib) {
    const int y = y0 + 2 * w + ib;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int x = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
      v[ib][q] = to_bf16(fmaxf(acc[ib][q] + bias, 0.0f));
      o2[(y * 32 + x) * 32 + c2] = v[ib][q];
    }
  }
  // 2x2 average pooling: rows y0 + 2w and +1 are this wave's two blocks, pixel pairs (x, x+1)
  // are registers q, q+1 with q % 4 in {0, 2}
  const int py = (y0 + 2 * w) >> 1;
  __bf16* po = pooled + (int64_t)j * sP + (int64_t)n * d.F3;
#pragma unroll
  for (int q = 0; q < 16; q += 2) {
    const int x = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
    const float sum = from_bf16(v[0][q]) + from_bf16(v[0][q + 1]) + from_bf16(v[1][q]) + from_bf16(v[1][q + 1]);
    po[(py * d.Wp + (x >> 1)) * 32 + c2] = to_bf16(0.25f * sum);
  }
}

// d1t[j C1 + c][r] = 1{act1[r][c] > 0} sum over taps t and channels c2 of d2[r - off(t)][c2] W2[c2][t C1 + c]
// (the error at the conv1 output; off(t) = (ky - 1, kx - 1)) for one particle, image and band;
// the conv2 output error d2 is formed in the halo from act2 and the pooled-feature error.
// Wave w computes band rows 2w, 2w+1 as four 16-pixel blocks; per block one
// v_mfma_f32_16x16x32_bf16 per tap (K = the 32 channels of d2), B from the transposed weight
// copy wT[j][t C1 + c][c2].  Lane l ends with four consecutive pixels of channel l % 16 and
// writes them as one 8-byte vector.
__global__ __launch_bounds__(256) void conv2_dgrad_implicit_kernel(const __bf16* __restrict__ act2, int64_t sA2,
                                                                   const __bf16* __restrict__ dpool, int64_t sP,
                                                                   const __bf16* __restrict__ wT, int64_t ldwT,
                                                                   const __bf16* __restrict__ act1, int64_t sA1,
                                                                   __bf16* __restrict__ d1t, int64_t ld, CnnDims d) {
  __shared__ __attribute__((aligned(16))) char halo[IHR * IHC * 64];
  __shared__ __attribute__((aligned(16))) __bf16 a1s[IB * 32 * 16];
  const int j = blockIdx.z, n = blockIdx.y, y0 = blockIdx.x * IB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const __bf16* a2n = act2 + (int64_t)j * sA2 + (int64_t)n * d.HW * 32;
  const __bf16* dpn = dpool + (int64_t)j * sP + (int64_t)n * d.F3;
  for (int e = tid; e < IHR * IHC * 4; e += 256) {
    const int row = e / (IHC * 4), rem = e - row * (IHC * 4), col = rem >> 2, c = rem & 3;
    const int yy = y0 - 1 + row, xx = col - 1;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (yy >= 0 && yy < d.H && xx >= 0 && xx < 32) v = d2_chunk(a2n, dpn, d, yy, xx, c);
    *(u32x4*)(halo + (row * IHC + col) * 64 + ((c ^ ((col >> 2) & 3)) << 4)) = v;
  }
  const __bf16* a1 = act1 + (int64_t)j * sA1 + ((int64_t)n * d.HW + y0 * 32) * 16;
  for (int e = tid; e < IB * 32 * 2; e += 256) *(u32x4*)(a1s + e * 8) = *(const u32x4*)(a1 + e * 8);
  // B fragments: lane l holds W2[c2 = 8 (l / 16) .. +7][t C1 + l % 16] from wT row t C1 + l % 16
  const __bf16* wj = wT + ((int64_t)j * d.K2 + (lane & 15)) * ldwT + 8 * (lane >> 4);
  u32x4 bfr[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) bfr[t] = *(const u32x4*)(wj + (int64_t)t * 16 * ldwT);
  __syncthreads();
  const int c = lane & 15;
  for (int mb = 0; mb < 4; ++mb) {
    const int r = 2 * w + (mb >> 1), x0 = 16 * (mb & 1);  // band row and first pixel of the block
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int ky = t / 3, kx = t % 3;
      const int hrow = r - ky + 2, col = x0 + (lane & 15) - kx + 2, ch = lane >> 4;
      const u32x4 av = *(const u32x4*)(halo + (hrow * IHC + col) * 64 + ((ch ^ ((col >> 2) & 3)) << 4));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                    __builtin_bit_cast(bf16x8_t, bfr[t]), acc, 0, 0, 0);
    }
    // rows 4 (l / 16) + i of the block: pixels x0 + 4 (l / 16) + i, channel c
    const int xb = x0 + 4 * (lane >> 4);
    s16x4_t o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float m = from_bf16(a1s[(r * 32 + xb + i) * 16 + c]);
      o[i] = __builtin_bit_cast(short, to_bf16(m > 0.0f ? acc[i] : 0.0f));
    }
    const int64_t rr = (int64_t)n * d.HW + (y0 + r) * 32 + xb;
    *(s16x4_t*)(d1t + ((int64_t)j * 16 + c) * ld + rr) = o;
  }
}

// [W2 | b2] gradient of particle j as an implicit GEMM over pixels: out[c2][t C1 + c] =
// sum_r d2[r][c2] act1[r + off(t)][c], out[c2][K2] = sum_r d2[r][c2].  M = the 32 output
// channels, N = the 145 columns in five 32-wide blocks (taps 2b, 2b+1; the last block holds tap
// 8, the ones column at 144 and zeros), K = 16 pixels per v_mfma_f32_32x32x16_bf16.  The error
// operand comes from d2t[j C2 + c2][r] (eight consecutive pixels per lane); the activation
// operand from three copies of the band's halo, channel-major and shifted by kx, so every
// eight-pixel read is aligned.  Workgroup (g, j) takes bands g, g + G, ...; wave w the 16-pixel
// steps 4w .. 4w + 3 of each band, and each wave writes its own FP32 partial
// part[j][g][w][32][145], summed in a fixed order by conv2_wgrad_sum_kernel.
constexpr int WG_COLS = 145;
constexpr int D2S = IB * 32 + 8;  // row stride of the band's channel-major error copy
__global__ __launch_bounds__(256) void conv2_wgrad_implicit_kernel(const __bf16* __restrict__ act2, int64_t sA2,
                                                                   const __bf16* __restrict__ dpool, int64_t sP,
                                                                   const __bf16* __restrict__ act1, int64_t sA1,
                                                                   int mcv, CnnDims d, int G, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) __bf16 a1T[3][16][IHR][32];
  __shared__ __attribute__((aligned(16))) __bf16 d2s[32][D2S];
  const int g = blockIdx.x, j = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int bands = mcv * (d.H / IB);
  f32x16 acc[5];
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[b][q] = 0.0f;
  // the ones column (bias) of block 4 and its zero columns beyond
  u32x4 ones;
  {
    const int col = 128 + (lane & 31);
    const uint32_t one2 = (uint32_t)__builtin_bit_cast(uint16_t, to_bf16(1.0f)) * 0x10001u;
    const uint32_t v = col == 144 ? one2 : 0u;
    ones = u32x4{v, v, v, v};
  }
  const __bf16* a1 = act1 + (int64_t)j * sA1;
  for (int band = g; band < bands; band += G) {
    const int n = band / (d.H / IB), y0 = (band - n * (d.H / IB)) * IB;
    __syncthreads();  // the previous band's reads of a1T are done
    for (int e = tid; e < IHR * IHC * 2; e += 256) {
      const int row = e / (IHC * 2), rem = e - row * (IHC * 2), hc = rem >> 1, c8 = (rem & 1) * 8;
      const int yy = y0 - 1 + row, xx = hc - 1;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (yy >= 0 && yy < d.H && xx >= 0 && xx < 32)
        v = *(const u32x4*)(a1 + ((int64_t)n * d.HW + yy * 32 + xx) * 16 + c8);
      const __bf16* vv = (const __bf16*)&v;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int p = hc - kx;  // copy kx holds halo column p + kx at position p
        if (p >= 0 && p < 32) {
#pragma unroll
          for (int i = 0; i < 8; ++i) a1T[kx][c8 + i][row][p] = vv[i];
        }
      }
    }
    {
      // the band's conv2 output error, channel-major: d2s[c2][band pixel]
      const __bf16* a2n = act2 + (int64_t)j * sA2 + (int64_t)n * d.HW * 32;
      const __bf16* dpn = dpool + (int64_t)j * sP + (int64_t)n * d.F3;
      for (int e = tid; e < IB * 32 * 4; e += 256) {
        const int p = e >> 2, c = e & 3;
        const u32x4 v = d2_chunk(a2n, dpn, d, y0 + (p >> 5), p & 31, c);
        const __bf16* vv = (const __bf16*)&v;
#pragma unroll
        for (int i = 0; i < 8; ++i) d2s[c * 8 + i][p] = vv[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int ks = 4 * w + s;                      // 16-pixel step of the band
      const int r = ks >> 1, x0 = (ks & 1) * 16 + 8 * (lane >> 5);
      const u32x4 av = *(const u32x4*)&d2s[lane & 31][r * 32 + x0];
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const int col = b * 32 + (lane & 31);
        u32x4 bv;
        if (b < 4 || col < 144) {
          const int t = col >> 4, c = col & 15, ky = t / 3, kx = t % 3;
          bv = *(const u32x4*)&a1T[kx][c][r + ky][x0];
        } else {
          bv = ones;
        }
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, av),
                                                         __builtin_bit_cast(bf16x8_t, bv), acc[b], 0, 0, 0);
      }
    }
  }
  // rows (c2) 8 (q / 4) + 4 (l / 32) + q % 4, column b * 32 + l % 32
  float* o = part + (((int64_t)j * G + g) * 4 + w) * (32 * WG_COLS);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const int col = b * 32 + (lane & 31);
    if (col >= WG_COLS) continue;
#pragma unroll
    for (int q = 0; q < 16; ++q) o[(8 * (q >> 2) + 4 * (lane >> 5) + (q & 3)) * WG_COLS + col] = acc[b][q];
  }
}

// g[j][off + e] (+)= sum over the 4 G partials of particle j in order, e < 32 * 145
__global__ void conv2_wgrad_sum_kernel(const float* __restrict__ part, int G, float* g, int64_t D, int64_t off,
                                       int beta) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= 32 * WG_COLS) return;
  const float* p = part + (int64_t)j * G * 4 * (32 * WG_COLS) + e;
  float acc = 0.0f;
  for (int k = 0; k < 4 * G; ++k) acc += p[(int64_t)k * (32 * WG_COLS)];
  float* dst = g + (int64_t)j * D + off + e;
  *dst = beta ? *dst + acc : acc;
}

inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// the kernels index pixels of a chunk (mcv * HW) and positions inside one image in 32 bits,
// images and taps / channel vectors on the y axis of the grid
bool grid_ok(int mcv, const CnnDims& d, int64_t per_image) {
  return mcv >= 1 && mcv <= 65535 && (int64_t)mcv * d.HW < ((int64_t)1 << 31) && per_image < ((int64_t)1 << 31);
}

}  // namespace

bool cnn_implicit_supported(const CnnDims& d, int bf16) {
  return bf16 && d.W == 32 && d.H % IB == 0 && d.C1 == 16 && d.C2 == 32 && d.K2 == 144 && d.Hp * 2 == d.H &&
         d.Wp * 2 == d.W;
}

hipError_t cnn_conv2_fwd_implicit_run(const void* act1, int64_t sA1, const void* w2, int64_t ldw, const float* b2,
                                      void* act2, int64_t sA2, void* pooled, int64_t sP, int mcv, const CnnDims& d,
                                      int J, hipStream_t s) {
  if (!cnn_implicit_supported(d, 1) || mcv < 1 || mcv > 65535 || J < 1 || J > 65535) return hipErrorInvalidValue;
  if (((uintptr_t)act1 | (uintptr_t)w2 | (uintptr_t)act2) & 15 || ldw % 8 || sA1 % 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(conv2_fwd_implicit_kernel, dim3(d.H / IB, mcv, J), dim3(256), 0, s, (const __bf16*)act1, sA1,
                     (const __bf16*)w2, ldw, b2, (__bf16*)act2, sA2, (__bf16*)pooled, sP, d);
  return hipGetLastError();
}

int cnn_wgrad_groups(int mcv, const CnnDims& d) { return std::min(CNN_WGRAD_GROUPS, mcv * (d.H / IB)); }

hipError_t cnn_conv2_wgrad_implicit_run(const void* act2, int64_t sA2, const void* dpool, int64_t sP,
                                        const void* act1, int64_t sA1, int mcv, const CnnDims& d, int J, float* part,
                                        float* g, int64_t D, int64_t off, int beta, hipStream_t s) {
  if (!cnn_implicit_supported(d, 1) || mcv < 1 || J < 1 || J > 65535) return hipErrorInvalidValue;
  if (((uintptr_t)act2 | (uintptr_t)dpool | (uintptr_t)act1) & 15 || sA2 % 8 || sP % 8 || sA1 % 8 || d.F3 % 8)
    return hipErrorInvalidValue;
  const int G = cnn_wgrad_groups(mcv, d);
  hipLaunchKernelGGL(conv2_wgrad_implicit_kernel, dim3(G, J), dim3(256), 0, s, (const __bf16*)act2, sA2,
                     (const __bf16*)dpool, sP, (const __bf16*)act1, sA1, mcv, d, G, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(conv2_wgrad_sum_kernel, dim3(nb(32 * WG_COLS, 256), J), dim3(256), 0, s, part, G, g, D, off,
                     beta);
  return hipGetLastError();
}

hipError_t cnn_conv2_dgrad_implicit_run(const void* act2, int64_t sA2, const void* dpool, int64_t sP, const void* wT,
                                        int64_t ldwT, const void* act1, int64_t sA1, void* d1t, int64_t ld, int mcv,
                                        const CnnDims& d, int J, hipStream_t s) {
  if (!cnn_implicit_supported(d, 1) || mcv < 1 || mcv > 65535 || J < 1 || J > 65535) return hipErrorInvalidValue;
  if (((uintptr_t)act2 | (uintptr_t)dpool | (uintptr_t)wT | (uintptr_t)act1 | (uintptr_t)d1t) & 15 || ldwT % 8 ||
      sA2 % 8 || sP % 8 || sA1 % 8 || d.F3 % 8 || ld % 4)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(conv2_dgrad_implicit_kernel, dim3(d.H / IB, mcv, J), dim3(256), 0, s, (const __bf16*)act2, sA2,
                     (const __bf16*)dpool, sP, (const __bf16*)wT, ldwT, (const __bf16*)act1, sA1, (__bf16*)d1t, ld, d);
  return hipGetLastError();
}

hipError_t cnn_im2col_x_run(const void* X, int64_t xld, int64_t c0, int mcv, const CnnDims& d, void* p1, int bf16,
                            hipStream_t s) {
  if (mcv <= 0) return hipSuccess;
  if (!grid_ok(mcv, d, (int64_t)d.HW * d.K1p)) return hipErrorInvalidValue;
  const dim3 grid(nb((int64_t)d.HW * d.K1p, 256), mcv);
  if (bf16) hipLaunchKernelGGL(im2col_x_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)X, xld, c0, mcv, d, (__bf16*)p1);
  else hipLaunchKernelGGL(im2col_x_kernel<float>, grid, dim3(256), 0, s, (const float*)X, xld, c0, mcv, d, (float*)p1);
  return hipGetLastError();
}

hipError_t cnn_im2col_xt_run(const void* X, int64_t xld, int64_t c0, int mcv, const CnnDims& d, int64_t ld, void* p1t,
                             int bf16, hipStream_t s) {
  if (mcv <= 0) return hipSuccess;
  if (!grid_ok(mcv, d, 0) || d.K1 + 1 > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb((int64_t)mcv * d.HW, 256), d.K1 + 1);
  if (bf16) hipLaunchKernelGGL(im2col_xt_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)X, xld, c0, mcv, d, ld, (__bf16*)p1t);
  else hipLaunchKernelGGL(im2col_xt_kernel<float>, grid, dim3(256), 0, s, (const float*)X, xld, c0, mcv, d, ld, (float*)p1t);
  return hipGetLastError();
}

hipError_t cnn_im2col_a_run(const void* act1, int64_t sA, int mcv, const CnnDims& d, int J, void* big, int64_t sB,
                            int bf16, hipStream_t s) {
  const int vec = bf16 ? 8 : 4;
  if (d.C1 % vec) return hipErrorInvalidValue;
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int64_t per = (int64_t)d.HW * (d.K2 / vec);
  if (!grid_ok(mcv, d, per) || J > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb(per, 256), mcv, J);
  if (bf16) hipLaunchKernelGGL(im2col_a_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)act1, sA, mcv, d, J, (__bf16*)big, sB);
  else hipLaunchKernelGGL(im2col_a_kernel<float>, grid, dim3(256), 0, s, (const float*)act1, sA, mcv, d, J, (float*)big, sB);
  return hipGetLastError();
}

hipError_t cnn_im2col_at_run(const void* act1, int64_t sA, int mcv, const CnnDims& d, int J, int64_t ld, void* bigT,
                             int64_t sB, int bf16, hipStream_t s) {
  const int vec = bf16 ? 8 : 4;
  if (d.C1 % vec) return hipErrorInvalidValue;
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int64_t work = (int64_t)mcv * d.HW * (d.C1 / vec);
  if (!grid_ok(mcv, d, 0) || work >= ((int64_t)1 << 31) || J > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb(work, 256), 10, J);  // nine taps, then the ones row
  if (bf16) hipLaunchKernelGGL(im2col_at_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)act1, sA, mcv, d, J, ld, (__bf16*)bigT, sB);
  else hipLaunchKernelGGL(im2col_at_kernel<float>, grid, dim3(256), 0, s, (const float*)act1, sA, mcv, d, J, ld, (float*)bigT, sB);
  return hipGetLastError();
}

hipError_t cnn_pool_run(const void* act2, int64_t sA, int mcv, const CnnDims& d, int J, void* pooled, int64_t sP,
                        int bf16, hipStream_t s) {
  if (mcv <= 0 || J <= 0) return hipSuccess;
  if (!grid_ok(mcv, d, d.F3) || J > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb(d.F3, 256), mcv, J);
  if (bf16) hipLaunchKernelGGL(pool_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)act2, sA, mcv, d, J, (__bf16*)pooled, sP);
  else hipLaunchKernelGGL(pool_kernel<float>, grid, dim3(256), 0, s, (const float*)act2, sA, mcv, d, J, (float*)pooled, sP);
  return hipGetLastError();
}

hipError_t cnn_ll_run(const CnnLLArgs& a, int J, int bf16, hipStream_t s) {
  if (a.ncls < 1 || a.ncls > 16) return hipErrorInvalidValue;
  if (J <= 0) return hipSuccess;
  if (bf16) hipLaunchKernelGGL(cnn_ll_kernel<__bf16>, dim3(J), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(cnn_ll_kernel<float>, dim3(J), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t cnn_dw3_run(const void* d3, const void* pooled, int64_t sP, int mc, int mcv, int F3, int ncls, int J,
                       float* g, int64_t D, int64_t off, int beta, int bf16, hipStream_t s) {
  const size_t smem = (size_t)mcv * 16 * sizeof(float);
  if (smem > 64 * 1024) return hipErrorInvalidValue;
  if (mcv <= 0 || J <= 0) return hipSuccess;
  dim3 grid(nb(F3 + 1, 256), J);
  if (bf16) hipLaunchKernelGGL(cnn_dw3_kernel<__bf16>, grid, dim3(256), smem, s, (const __bf16*)d3, (const __bf16*)pooled, sP, mc, mcv, F3, ncls, g, D, off, beta);
  else hipLaunchKernelGGL(cnn_dw3_kernel<float>, grid, dim3(256), smem, s, (const float*)d3, (const float*)pooled, sP, mc, mcv, F3, ncls, g, D, off, beta);
  return hipGetLastError();
}

hipError_t cnn_slice_sum_run(const float* part, int S, int M, int N, int C1, float* g, int64_t D, int beta,
                             hipStream_t s) {
  if (S < 1 || (int64_t)M * N >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(slice_sum_kernel, dim3(nb((int64_t)M * N, 256)), dim3(256), 0, s, part, S, M, N, C1, g, D, beta);
  return hipGetLastError();
}

hipError_t cnn_unpool_run(const void* dpool, int64_t sP, const void* act2, int64_t sA, int mcv, const CnnDims& d,
                          int J, int64_t ld, void* d2, void* d2t, int bf16, hipStream_t s) {
  const int vec = bf16 ? 8 : 4;
  if (d.C2 % vec) return hipErrorInvalidValue;
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int64_t work = (int64_t)mcv * d.HW * (d.C2 / vec);
  if (!grid_ok(mcv, d, 0) || work >= ((int64_t)1 << 31) || J > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb(work, 256), 1, J);
  if (bf16) hipLaunchKernelGGL(unpool_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)dpool, sP, (const __bf16*)act2, sA, mcv, d, J, ld, (__bf16*)d2, (__bf16*)d2t);
  else hipLaunchKernelGGL(unpool_kernel<float>, grid, dim3(256), 0, s, (const float*)dpool, sP, (const float*)act2, sA, mcv, d, J, ld, (float*)d2, (float*)d2t);
  return hipGetLastError();
}

hipError_t cnn_col2im_run(const void* dp2, int64_t sB, const void* act1, int64_t sA, int mcv, const CnnDims& d, int J,
                          int64_t ld, void* d1t, int bf16, hipStream_t s) {
  const int vec = bf16 ? 8 : 4;
  if (d.C1 % vec) return hipErrorInvalidValue;
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int64_t work = (int64_t)mcv * d.HW * (d.C1 / vec);
  if (!grid_ok(mcv, d, 0) || work >= ((int64_t)1 << 31) || J > 65535) return hipErrorInvalidValue;
  const dim3 grid(nb(work, 256), 1, J);
  if (bf16) hipLaunchKernelGGL(col2im_kernel<__bf16>, grid, dim3(256), 0, s, (const __bf16*)dp2, sB, (const __bf16*)act1, sA, mcv, d, J, ld, (__bf16*)d1t);
  else hipLaunchKernelGGL(col2im_kernel<float>, grid, dim3(256), 0, s, (const float*)dp2, sB, (const float*)act1, sA, mcv, d, J, ld, (float*)d1t);
  return hipGetLastError();
}

}  // namespace smc
