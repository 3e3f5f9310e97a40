// Convolution stack of the LeNet-5 network (the MNIST model of the paper's Table 1 study,
// Section 4):
//
//   conv kxk "same" (C1) -> act -> 2x2 average pool -> conv kxk "valid" (C2) -> act
//   -> 2x2 average pool -> F = Hq Wq C2 features
//
// followed by dense layers that run on the batched MFMA GEMM and the output-layer kernel
// like the dense networks' hidden layers.  The channel counts are tiny (1 -> 6 -> 16 for
// LeNet-5 on MNIST: contractions of length 25 and 150 into 6 and 16 outputs), so the
// convolutions run as direct FP32 arithmetic with one particle's conv weights (10 KB) and
// one image at a time in LDS:
//   lenet_fwd_kernel   per (block of images, particle): the features, row-major [mc x F]
//                      and transposed [(F+1) x mc] (the dense layer's weight-gradient operand)
//   lenet_bwd_kernel   per (block of images, particle): recomputes the stack for each image,
//                      takes the features' error from the dense layers, and accumulates the
//                      conv weight gradients in registers over the block's images; one FP32
//                      partial per block
//   lenet_reduce_kernel sums the partials in a fixed order into the gradient rows
// Work items pair two output channels with one output pixel, pixels fastest across lanes,
// so a wave's weight reads are LDS broadcasts and its image reads neighbouring pixels.
// Parameter layout: theta[j] starts with [C1 x (k k Cin + 1)] then [C2 x (k k C1 + 1)],
// weight index (ky k + kx) cin + c, bias last in each row.
#include "kernels.h"

namespace smc {

namespace {

constexpr int LT = 256;  // threads per workgroup

struct LenetSmem {
  float *wl, *xin, *a1, *p1, *a2, *dp1, *g1s;
};

// LDS carve-up (floats); the forward uses wl, xin, p1 only
__host__ __device__ inline int lenet_smem_floats(const LenetDims& d, bool bwd, int* offs) {
  const int Hpd = d.H + 2 * d.pad, Wpd = d.W + 2 * d.pad;
  int n = 0;
  auto take = [&](int q, int cnt) {
    if (offs) offs[q] = n;
    n += (cnt + 3) & ~3;
  };
  take(0, d.Dconv);
  take(1, Hpd * Wpd * d.Cin);
  take(2, bwd ? d.H * d.W * d.C1 : 0);
  take(3, d.Hp * d.Wp * d.C1);
  take(4, bwd ? d.H2 * d.W2 * d.C2 : 0);
  take(5, bwd ? d.Hp * d.Wp * d.C1 : 0);
  take(6, bwd ? d.ns1 * d.C1 * (d.K1 + 1) : 0);
  return n;
}

__device__ inline LenetSmem lenet_smem(float* base, const LenetDims& d, bool bwd) {
  int o[7];
  lenet_smem_floats(d, bwd, o);
  return LenetSmem{base + o[0], base + o[1], base + o[2], base + o[3], base + o[4], base + o[5], base + o[6]};
}

template <int ACT>
__device__ __forceinline__ float actf(float z) {
  if constexpr (ACT == ACT_RELU) return fmaxf(z, 0.0f);
  else return tanhf(z);
}
template <int ACT>
__device__ __forceinline__ float actg(float a) {
  if constexpr (ACT == ACT_RELU) return a > 0.0f ? 1.0f : 0.0f;
  else return 1.0f - a * a;
}

// Particle j's two conv blocks into LDS (contiguous at the start of its theta row).
__device__ inline void load_conv_weights(const float* theta, int64_t D, int j, const LenetDims& d, float* wl) {
  const float* src = theta + (int64_t)j * D;
  for (int e = threadIdx.x; e < d.Dconv; e += LT) wl[e] = src[e];
}

// Image n (global sample row c0 + n) into xin with a zero border of pad pixels.
__device__ inline void load_image(const float* X, int64_t xld, int64_t row, const LenetDims& d, float* xin) {
  const int Hpd = d.H + 2 * d.pad, Wpd = d.W + 2 * d.pad, tot = Hpd * Wpd * d.Cin;
  const float* src = X + row * xld;
  for (int e = threadIdx.x; e < tot; e += LT) {
    const int pix = e / d.Cin, c = e - pix * d.Cin;
    const int y = pix / Wpd - d.pad, x = pix - (pix / Wpd) * Wpd - d.pad;
    xin[e] = (y >= 0 && y < d.H && x >= 0 && x < d.W) ? src[(y * d.W + x) * d.Cin + c] : 0.0f;
  }
}

// Convolution + activation + 2x2 average pool over an LDS input of row length win pixels and
// cin channels, for output channels cout with weights w[cout][K+1] (K = k k cin, bias last).
// Item e = (channel pair, pooled pixel), pixels fastest.  The input rows of an item's
// (k+1) x (k+1) window are read once into registers.  Writes pooled[q][c] through `pool`
// (q = pooled pixel, c = channel) and, if act_out, the activations act_out[y][x][c] of the
// conv output (row length 2 Wo).
template <int KS, int ACT, typename PoolW>
__device__ __forceinline__ void conv_act_pool(const float* in, int win, int cin, const float* w, int cout, int Ho,
                                              int Wo, float* act_out, PoolW pool) {
  constexpr int K1 = KS + 1;
  const int K = KS * KS * cin, nq = Ho * Wo, ncp = (cout + 1) / 2;
  for (int e = threadIdx.x; e < ncp * nq; e += LT) {
    const int cp = e / nq, q = e - cp * nq;
    const int c0 = 2 * cp;
    const bool two = c0 + 1 < cout;
    const int py = q / Wo, px = q - py * Wo;
    const float* w0 = w + c0 * (K + 1);
    const float* w1 = two ? w0 + (K + 1) : w0;
    float acc[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b][0] = w0[K];
        acc[a][b][1] = w1[K];
      }
    for (int ci = 0; ci < cin; ++ci) {
#pragma unroll
      for (int iy = 0; iy < K1; ++iy) {
        float r[K1];
        const float* row = in + ((2 * py + iy) * win + 2 * px) * cin + ci;
#pragma unroll
        for (int ix = 0; ix < K1; ++ix) r[ix] = row[ix * cin];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int ky = iy - dy;
          if (ky < 0 || ky >= KS) continue;
#pragma unroll
          for (int kx = 0; kx < KS; ++kx) {
            const int t = (ky * KS + kx) * cin + ci;
            const float v0 = w0[t], v1 = w1[t];
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              acc[dy][dx][0] = fmaf(r[kx + dx], v0, acc[dy][dx][0]);
              acc[dy][dx][1] = fmaf(r[kx + dx], v1, acc[dy][dx][1]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      if (ch == 1 && !two) break;
      float s = 0.0f;
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const float a = actf<ACT>(acc[dy][dx][ch]);
          s += a;
          if (act_out) act_out[((2 * py + dy) * (2 * Wo) + 2 * px + dx) * cout + c0 + ch] = a;
        }
      pool(q, c0 + ch, 0.25f * s);
    }
  }
}

template <int KS, int ACT>
__global__ __launch_bounds__(LT) void lenet_fwd_kernel(const float* __restrict__ X, int64_t xld, int64_t c0, int mcv,
                                                       int rows, int ipb, LenetDims d, const float* __restrict__ theta,
                                                       int64_t D, float* __restrict__ feat, int64_t sF,
                                                       float* __restrict__ featT, int64_t ldT) {
  extern __shared__ __attribute__((aligned(16))) float lsm[];
  const LenetSmem S = lenet_smem(lsm, d, false);
  const int j = blockIdx.y;
  const int n0 = blockIdx.x * ipb, n1 = min(n0 + ipb, rows);
  float* fj = feat + (int64_t)j * sF;
  float* fTj = featT ? featT + (int64_t)j * (d.F + 1) * ldT : nullptr;
  load_conv_weights(theta, D, j, d, S.wl);
  const float* w2 = S.wl + d.C1 * (d.K1 + 1);
  for (int n = n0; n < n1; ++n) {
    if (n >= mcv) {
      // rows past the chunk's samples feed the dense GEMMs: keep them zero
      for (int f = threadIdx.x; f < d.F; f += LT) {
        fj[(int64_t)n * d.F + f] = 0.0f;
        if (fTj) fTj[(int64_t)f * ldT + n] = 0.0f;
      }
      continue;
    }
    __syncthreads();  // the previous image's readers are done with xin and p1
    load_image(X, xld, c0 + n, d, S.xin);
    __syncthreads();
    float* p1 = S.p1;
    const int C1 = d.C1;
    conv_act_pool<KS, ACT>(S.xin, d.W + 2 * d.pad, d.Cin, S.wl, d.C1, d.Hp, d.Wp, nullptr,
                           [&](int q, int c, float v) { p1[q * C1 + c] = v; });
    __syncthreads();
    const int C2 = d.C2;
    conv_act_pool<KS, ACT>(p1, d.Wp, d.C1, w2, d.C2, d.Hq, d.Wq, nullptr, [&](int q, int c, float v) {
      const int f = q * C2 + c;
      fj[(int64_t)n * d.F + f] = v;
      if (fTj) fTj[(int64_t)f * ldT + n] = v;
    });
  }
}

template <int KS, int ACT>
__global__ __launch_bounds__(LT) void lenet_bwd_kernel(const float* __restrict__ X, int64_t xld, int64_t c0, int mcv,
                                                       int ipb, LenetDims d, const float* __restrict__ theta, int64_t D,
                                                       const float* __restrict__ dfeat, int64_t sF,
                                                       float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) float lsm[];
  const LenetSmem S = lenet_smem(lsm, d, true);
  const int j = blockIdx.y, tid = threadIdx.x;
  const int n0 = blockIdx.x * ipb, n1 = min(n0 + ipb, mcv);
  load_conv_weights(theta, D, j, d, S.wl);
  const float* w2 = S.wl + d.C1 * (d.K1 + 1);
  const int Wpd = d.W + 2 * d.pad, C1 = d.C1, C2 = d.C2, Cin = d.Cin;
  constexpr int KK = KS * KS;
  // conv2 weight-gradient item: channel pair cp2 = tid / KK, tap t2 = tid % KK (all C1 inputs)
  const int cp2 = tid / KK, t2 = tid - cp2 * KK;
  const bool own2 = cp2 < (C2 + 1) / 2;
  const int o2 = 2 * cp2;
  const bool two2 = o2 + 1 < C2;
  const int ky2 = t2 / KS, kx2 = t2 - ky2 * KS;
  float g2[2][LENET_CMAX], gb2[2] = {0.0f, 0.0f};
  // conv1 weight-gradient item: (channel pair, tap, slice of the pixels)
  const int n1i = (C1 + 1) / 2 * KK;
  const int s1 = tid / n1i, r1 = tid - s1 * n1i, cp1 = r1 / KK, t1 = r1 - cp1 * KK;
  const bool own1 = s1 < d.ns1;
  const int o1 = 2 * cp1;
  const bool two1 = o1 + 1 < C1;
  const int ky1 = t1 / KS, kx1 = t1 - ky1 * KS;
  const int HW = d.H * d.W, span1 = (HW + d.ns1 - 1) / d.ns1;
  const int pa = min(HW, s1 * span1), pb = min(HW, pa + span1);
  float g1[2][LENET_CMAX], gb1[2] = {0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < LENET_CMAX; ++c) g1[0][c] = g1[1][c] = g2[0][c] = g2[1][c] = 0.0f;

  const float* dfj = dfeat + (int64_t)j * sF;
  for (int n = n0; n < n1; ++n) {
    __syncthreads();
    load_image(X, xld, c0 + n, d, S.xin);
    __syncthreads();
    // forward again, keeping the activations
    float* p1 = S.p1;
    conv_act_pool<KS, ACT>(S.xin, Wpd, Cin, S.wl, C1, d.Hp, d.Wp, S.a1,
                           [&](int q, int c, float v) { p1[q * C1 + c] = v; });
    __syncthreads();
    conv_act_pool<KS, ACT>(p1, d.Wp, C1, w2, C2, d.Hq, d.Wq, S.a2, [](int, int, float) {});
    __syncthreads();
    // dz2 = unpool(dfeat) * act'(a2), in place
    for (int e = tid; e < d.H2 * d.W2 * C2; e += LT) {
      const int pix = e / C2, c = e - pix * C2;
      const int y = pix / d.W2, x = pix - y * d.W2;
      const float g = dfj[(int64_t)n * d.F + ((y >> 1) * d.Wq + (x >> 1)) * C2 + c];
      S.a2[e] = 0.25f * g * actg<ACT>(S.a2[e]);
    }
    __syncthreads();
    const float* dz2 = S.a2;
    // conv2 weight gradient: sum over output pixels of dz2[pix][o] * p1[pix + tap][c]
    if (own2) {
      for (int pix = 0; pix < d.H2 * d.W2; ++pix) {
        const int y = pix / d.W2, x = pix - y * d.W2;
        const float e0 = dz2[pix * C2 + o2], e1 = two2 ? dz2[pix * C2 + o2 + 1] : 0.0f;
        if (t2 == 0) {
          gb2[0] += e0;
          gb2[1] += e1;
        }
        const float* src = p1 + ((y + ky2) * d.Wp + x + kx2) * C1;
#pragma unroll
        for (int c = 0; c < LENET_CMAX; ++c)
          if (c < C1) {
            g2[0][c] = fmaf(e0, src[c], g2[0][c]);
            g2[1][c] = fmaf(e1, src[c], g2[1][c]);
          }
      }
    }
    // error of the pooled conv1 map: dp1[pix][c] = sum over taps and o of dz2[pix - tap][o] w2[o][tap][c]
    for (int pix = tid; pix < d.Hp * d.Wp; pix += LT) {
      const int y = pix / d.Wp, x = pix - y * d.Wp;
      float acc[LENET_CMAX];
#pragma unroll
      for (int c = 0; c < LENET_CMAX; ++c) acc[c] = 0.0f;
      for (int ky = 0; ky < KS; ++ky) {
        const int yy = y - ky;
        if (yy < 0 || yy >= d.H2) continue;
        for (int kx = 0; kx < KS; ++kx) {
          const int xx = x - kx;
          if (xx < 0 || xx >= d.W2) continue;
          const float* e = dz2 + (yy * d.W2 + xx) * C2;
          const float* wt = w2 + (ky * KS + kx) * C1;
          for (int o = 0; o < C2; ++o) {
            const float ev = e[o];
            const float* wr = wt + o * (d.K2 + 1);
#pragma unroll
            for (int c = 0; c < LENET_CMAX; ++c)
              if (c < C1) acc[c] = fmaf(ev, wr[c], acc[c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < LENET_CMAX; ++c)
        if (c < C1) S.dp1[pix * C1 + c] = acc[c];
    }
    __syncthreads();
    // dz1 = unpool(dp1) * act'(a1), in place
    for (int e = tid; e < HW * C1; e += LT) {
      const int pix = e / C1, c = e - pix * C1;
      const int y = pix / d.W, x = pix - y * d.W;
      S.a1[e] = 0.25f * S.dp1[((y >> 1) * d.Wp + (x >> 1)) * C1 + c] * actg<ACT>(S.a1[e]);
    }
    __syncthreads();
    // conv1 weight gradient over this item's slice of pixels
    if (own1) {
      const float* dz1 = S.a1;
      for (int pix = pa; pix < pb; ++pix) {
        const int y = pix / d.W, x = pix - y * d.W;
        const float e0 = dz1[pix * C1 + o1], e1 = two1 ? dz1[pix * C1 + o1 + 1] : 0.0f;
        if (t1 == 0) {
          gb1[0] += e0;
          gb1[1] += e1;
        }
        const float* src = S.xin + ((y + ky1) * Wpd + x + kx1) * Cin;
#pragma unroll
        for (int c = 0; c < LENET_CMAX; ++c)
          if (c < Cin) {
            g1[0][c] = fmaf(e0, src[c], g1[0][c]);
            g1[1][c] = fmaf(e1, src[c], g1[1][c]);
          }
      }
    }
  }
  // the block's partial: conv2 items directly, conv1 slices summed in order through LDS
  float* pj = part + ((int64_t)j * gridDim.x + blockIdx.x) * d.Dconv;
  float* pw2 = pj + C1 * (d.K1 + 1);
  if (own2) {
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two2) break;
      float* row = pw2 + (o2 + h) * (d.K2 + 1);
#pragma unroll
      for (int c = 0; c < LENET_CMAX; ++c)
        if (c < C1) row[t2 * C1 + c] = g2[h][c];
      if (t2 == 0) row[d.K2] = gb2[h];
    }
  }
  __syncthreads();
  if (own1) {
    float* gs = S.g1s + s1 * C1 * (d.K1 + 1);
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two1) break;
      float* row = gs + (o1 + h) * (d.K1 + 1);
#pragma unroll
      for (int c = 0; c < LENET_CMAX; ++c)
        if (c < Cin) row[t1 * Cin + c] = g1[h][c];
      if (t1 == 0) row[d.K1] = gb1[h];
    }
  }
  __syncthreads();
  for (int e = tid; e < C1 * (d.K1 + 1); e += LT) {
    float s = 0.0f;
    for (int q = 0; q < d.ns1; ++q) s += S.g1s[q * C1 * (d.K1 + 1) + e];
    pj[e] = s;
  }
}

// g[j][e] (+)= sum over blocks of part[j][blk][e], e < Dconv, in block order
__global__ void lenet_reduce_kernel(const float* __restrict__ part, int nblk, int Dconv, float* __restrict__ g,
                                    int64_t D, int beta) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Dconv) return;
  const int j = blockIdx.y;
  const float* p = part + (int64_t)j * nblk * Dconv + e;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += p[(int64_t)b * Dconv];
  float* dst = g + (int64_t)j * D + e;
  *dst = beta ? *dst + s : s;
}

template <int KS, int ACT>
hipError_t launch_fwd(const float* X, int64_t xld, int64_t c0, int mcv, int rows, int ipb, const LenetDims& d,
                      const float* theta, int64_t D, int J, float* feat, int64_t sF, float* featT, int64_t ldT,
                      size_t smem, hipStream_t s) {
  const dim3 grid((unsigned)((rows + ipb - 1) / ipb), (unsigned)J);
  hipLaunchKernelGGL((lenet_fwd_kernel<KS, ACT>), grid, dim3(LT), smem, s, X, xld, c0, mcv, rows, ipb, d, theta, D,
                     feat, sF, featT, ldT);
  return hipGetLastError();
}

template <int KS, int ACT>
hipError_t launch_bwd(const float* X, int64_t xld, int64_t c0, int mcv, int ipb, int nblk, const LenetDims& d,
                      const float* theta, int64_t D, int J, const float* dfeat, int64_t sF, float* part, size_t smem,
                      hipStream_t s) {
  hipLaunchKernelGGL((lenet_bwd_kernel<KS, ACT>), dim3((unsigned)nblk, (unsigned)J), dim3(LT), smem, s, X, xld, c0,
                     mcv, ipb, d, theta, D, dfeat, sF, part);
  return hipGetLastError();
}

}  // namespace

size_t lenet_smem_bytes(const LenetDims& d, bool bwd) { return (size_t)lenet_smem_floats(d, bwd, nullptr) * 4; }

hipError_t lenet_fwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int rows, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, float* feat, int64_t sF, float* featT,
                         int64_t ldT, hipStream_t s) {
  if (rows <= 0 || J <= 0) return hipSuccess;
  if (ipb < 1 || mcv > rows || (d.k != 3 && d.k != 5)) return hipErrorInvalidValue;
  const size_t smem = lenet_smem_bytes(d, false);
  if (d.k == 3)
    return act == ACT_RELU ? launch_fwd<3, ACT_RELU>(X, xld, c0, mcv, rows, ipb, d, theta, D, J, feat, sF, featT, ldT, smem, s)
                           : launch_fwd<3, ACT_TANH>(X, xld, c0, mcv, rows, ipb, d, theta, D, J, feat, sF, featT, ldT, smem, s);
  return act == ACT_RELU ? launch_fwd<5, ACT_RELU>(X, xld, c0, mcv, rows, ipb, d, theta, D, J, feat, sF, featT, ldT, smem, s)
                         : launch_fwd<5, ACT_TANH>(X, xld, c0, mcv, rows, ipb, d, theta, D, J, feat, sF, featT, ldT, smem, s);
}

hipError_t lenet_bwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, const float* dfeat, int64_t sF, float* part,
                         int part_blocks, float* g, int beta, hipStream_t s) {
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int nblk = (mcv + ipb - 1) / ipb;
  if (ipb < 1 || nblk > part_blocks || (d.k != 3 && d.k != 5)) return hipErrorInvalidValue;
  const size_t smem = lenet_smem_bytes(d, true);
  hipError_t e;
  if (d.k == 3)
    e = act == ACT_RELU ? launch_bwd<3, ACT_RELU>(X, xld, c0, mcv, ipb, nblk, d, theta, D, J, dfeat, sF, part, smem, s)
                        : launch_bwd<3, ACT_TANH>(X, xld, c0, mcv, ipb, nblk, d, theta, D, J, dfeat, sF, part, smem, s);
  else
    e = act == ACT_RELU ? launch_bwd<5, ACT_RELU>(X, xld, c0, mcv, ipb, nblk, d, theta, D, J, dfeat, sF, part, smem, s)
                        : launch_bwd<5, ACT_TANH>(X, xld, c0, mcv, ipb, nblk, d, theta, D, J, dfeat, sF, part, smem, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lenet_reduce_kernel, dim3((unsigned)((d.Dconv + 255) / 256), (unsigned)J), dim3(256), 0, s, part,
                     nblk, d.Dconv, g, D, beta);
  return hipGetLastError();
}

}  // namespace smc
