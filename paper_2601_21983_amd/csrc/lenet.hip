// Convolution stack of the LeNet-5 network (the MNIST model of the paper's Table 1 study,
// Section 4):
//
//   conv kxk "same" (C1) -> act -> 2x2 average pool -> conv kxk "valid" (C2) -> act
//   -> 2x2 average pool -> F = Hq Wq C2 features
//
// followed by dense layers that run on the batched MFMA GEMM and the output-layer kernel
// like the dense networks' hidden layers.  The channel counts are tiny (1 -> 6 -> 16 for
// LeNet-5 on MNIST: contractions of length 25 and 150 into 6 and 16 outputs), so the
// convolutions run as direct FP32 arithmetic with one image at a time in LDS:
//   lenet_fwd_kernel   per (block of images, particle), the particle's conv weights (10 KB)
//                      in LDS: the features, row-major [mc x F] and transposed [(F+1) x mc]
//                      (the dense layer's weight-gradient operand), and in a gradient pass
//                      each image's activation maps for the backward
//   lenet_bwd_kernel   per (block of images, particle): reads the saved maps, takes the
//                      features' error from the dense layers, and accumulates the conv weight
//                      gradients in registers over the block's images; one FP32 partial per
//                      block.  Its conv2 input error reads the weights through the scalar cache.
//   lenet_reduce_kernel sums the partials in a fixed order into the gradient rows
// Forward work items pair two output channels with one output pixel, pixels fastest across
// lanes, so a wave's weight reads are LDS broadcasts and its image reads neighbouring pixels.
// Parameter layout: theta[j] starts with [C1 x (k k Cin + 1)] then [C2 x (k k C1 + 1)],
// weight index (ky k + kx) cin + c, bias last in each row.
#include "kernels.h"

namespace smc {

namespace {

constexpr int LT = 256;  // threads per workgroup

// LDS regions.  Maps are planar ([channel][row][col]); the conv weights are stored
// [out][in][ky][kx] with the biases apart, so that an item's weight reads for one
// (out, in) pair sit at compile-time offsets from one base.
struct LenetSmem {
  float *w1, *b1, *w2, *b2, *xin, *a1, *p1, *a2, *dp1, *g1s;
};

__host__ __device__ inline int lenet_smem_floats(const LenetDims& d, bool bwd, int* offs) {
  const int Hpd = d.H + 2 * d.pad, Wpd = d.W + 2 * d.pad, kk = d.k * d.k;
  const int g1s = d.ns1 * d.C1 * (d.K1 + 1);
  int n = 0;
  auto take = [&](int q, int cnt) {
    if (offs) offs[q] = n;
    n += (cnt + 3) & ~3;
  };
  // the backward recomputes conv1 from LDS weights; its conv2 input error takes the conv2
  // weights through the scalar cache
  take(0, d.C1 * d.Cin * kk);
  take(1, d.C1);
  take(2, bwd ? 0 : d.C2 * d.C1 * kk);
  take(3, bwd ? 0 : d.C2);
  take(4, Hpd * Wpd * d.Cin);
  // a1 also holds the conv1 gradient's slice partials once the last image is done
  take(5, bwd ? (d.H * d.W * d.C1 > g1s ? d.H * d.W * d.C1 : g1s) : 0);
  take(6, d.Hp * d.Wp * d.C1);
  take(7, bwd ? d.H2 * d.W2 * d.C2 : 0);
  take(8, bwd ? d.Hp * d.Wp * d.C1 : 0);
  return n;
}

__device__ inline LenetSmem lenet_smem(float* base, const LenetDims& d, bool bwd) {
  int o[9];
  lenet_smem_floats(d, bwd, o);
  return LenetSmem{base + o[0], base + o[1], base + o[2], base + o[3], base + o[4],
                   base + o[5], base + o[6], base + o[7], base + o[8], base + o[5]};
}

// tanh from the exponential: 1 - 2 / (e^{2|z|} + 1) with the sign of z, and its Taylor series
// z - z^3/3 + 2 z^5/15 - 17 z^7/315 for |z| < 1/8, where the subtraction would cancel
// (truncation error below 2e-10 there)
__device__ __forceinline__ float tanh_exp(float z) {
  const float a = fabsf(z);
  if (a < 0.125f) {
    const float z2 = z * z;
    return z * fmaf(z2, fmaf(z2, fmaf(z2, -17.0f / 315.0f, 2.0f / 15.0f), -1.0f / 3.0f), 1.0f);
  }
  const float t = 1.0f - 2.0f / (__expf(2.0f * a) + 1.0f);
  return copysignf(t, z);
}

template <int ACT>
__device__ __forceinline__ float actf(float z) {
  if constexpr (ACT == ACT_RELU) return fmaxf(z, 0.0f);
  else return tanh_exp(z);
}
template <int ACT>
__device__ __forceinline__ float actg(float a) {
  if constexpr (ACT == ACT_RELU) return a > 0.0f ? 1.0f : 0.0f;
  else return 1.0f - a * a;
}

// Particle j's conv blocks (theta layout [out][(ky k + kx) in + c | bias]) into the LDS layout
// (conv1 only when !conv2).
__device__ inline void load_conv_weights(const float* theta, int64_t D, int j, const LenetDims& d, const LenetSmem& S,
                                         bool conv2 = true) {
  const float* src = theta + (int64_t)j * D;
  const int kk = d.k * d.k, r1 = d.K1 + 1, r2 = d.K2 + 1, n1 = d.C1 * r1;
  for (int e = threadIdx.x; e < (conv2 ? d.Dconv : n1); e += LT) {
    const float v = src[e];
    const bool first = e < n1;
    const int cin = first ? d.Cin : d.C1, rl = first ? r1 : r2;
    const int ee = first ? e : e - n1;
    const int o = ee / rl, r = ee - o * rl;
    if (r == rl - 1) {
      (first ? S.b1 : S.b2)[o] = v;
    } else {
      const int tap = r / cin, c = r - tap * cin;
      (first ? S.w1 : S.w2)[(o * cin + c) * kk + tap] = v;
    }
  }
}

// Image (global sample row `row`) into the planar xin [Cin][Hpd][Wpd] with a zero border.
__device__ inline void load_image(const float* X, int64_t xld, int64_t row, const LenetDims& d, float* xin) {
  const int Hpd = d.H + 2 * d.pad, Wpd = d.W + 2 * d.pad, plane = Hpd * Wpd;
  const float* src = X + row * xld;
  for (int e = threadIdx.x; e < plane * d.Cin; e += LT) {
    const int pix = e / d.Cin, c = e - pix * d.Cin;  // read the image pixel-major (contiguous)
    const int yy = pix / Wpd, xx = pix - yy * Wpd;
    const int y = yy - d.pad, x = xx - d.pad;
    xin[c * plane + pix] = (y >= 0 && y < d.H && x >= 0 && x < d.W) ? src[(y * d.W + x) * d.Cin + c] : 0.0f;
  }
}

// Convolution + activation + 2x2 average pool over the planar LDS input `in` ([cin][.][win],
// plane stride `plane`) for cout output channels (weights w [cout][cin][KS][KS], biases b).
// Item e = (channel pair, pooled pixel), pixels fastest, so the weight reads of a wave are
// broadcasts.  Each input row of an item's (KS+1)^2 window is read once.  Writes the pooled
// value through pool(q, c, v) (q = pooled pixel) and, if act_out, the activations
// act_out[c][y][x] (planar, 2Ho x 2Wo).
template <int KS, int ACT, typename PoolW>
__device__ __forceinline__ void conv_act_pool(const float* in, int plane, int win, int cin, const float* w,
                                              const float* b, int cout, int Ho, int Wo, float* act_out, PoolW pool) {
  constexpr int K1 = KS + 1, KK = KS * KS;
  const int nq = Ho * Wo, ncp = (cout + 1) / 2;
  for (int e = threadIdx.x; e < ncp * nq; e += LT) {
    const int cp = e / nq, q = e - cp * nq;
    const int c0 = 2 * cp;
    const bool two = c0 + 1 < cout;
    const int py = q / Wo, px = q - py * Wo;
    const float* wa = w + c0 * cin * KK;
    const float* wb = two ? wa + cin * KK : wa;
    float acc[2][2][2];
    const float ba = b[c0], bb = two ? b[c0 + 1] : 0.0f;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        acc[u][v][0] = ba;
        acc[u][v][1] = bb;
      }
    const float* ib = in + 2 * py * win + 2 * px;
    for (int ci = 0; ci < cin; ++ci) {
      const float* ip = ib + ci * plane;
      const float* wca = wa + ci * KK;
      const float* wcb = wb + ci * KK;
#pragma unroll
      for (int iy = 0; iy < K1; ++iy) {
        float r[K1];
#pragma unroll
        for (int ix = 0; ix < K1; ++ix) r[ix] = ip[iy * win + ix];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int ky = iy - dy;
          if (ky < 0 || ky >= KS) continue;
#pragma unroll
          for (int kx = 0; kx < KS; ++kx) {
            const float va = wca[ky * KS + kx], vb = wcb[ky * KS + kx];
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
              acc[dy][dx][0] = fmaf(r[kx + dx], va, acc[dy][dx][0]);
              acc[dy][dx][1] = fmaf(r[kx + dx], vb, acc[dy][dx][1]);
            }
          }
        }
      }
    }
    const int oplane = 4 * nq;
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
          if (act_out) act_out[(c0 + ch) * oplane + (2 * py + dy) * (2 * Wo) + 2 * px + dx] = a;
        }
      pool(q, c0 + ch, 0.25f * s);
    }
  }
}

template <int KS, int ACT>
__global__ __launch_bounds__(LT) void lenet_fwd_kernel(const float* __restrict__ X, int64_t xld, int64_t c0, int mcv,
                                                       int rows, int ipb, LenetDims d, const float* __restrict__ theta,
                                                       int64_t D, float* __restrict__ feat, int64_t sF,
                                                       float* __restrict__ featT, int64_t ldT, float* __restrict__ maps,
                                                       int64_t sM) {
  extern __shared__ __attribute__((aligned(16))) float lsm[];
  const LenetSmem S = lenet_smem(lsm, d, false);
  const int j = blockIdx.y;
  const int n0 = blockIdx.x * ipb, n1 = min(n0 + ipb, rows);
  float* fj = feat + (int64_t)j * sF;
  float* fTj = featT ? featT + (int64_t)j * (d.F + 1) * ldT : nullptr;
  load_conv_weights(theta, D, j, d, S);
  const int Wpd = d.W + 2 * d.pad, P0 = (d.H + 2 * d.pad) * Wpd, P1 = d.Hp * d.Wp;
  for (int n = n0; n < n1; ++n) {
    if (n >= mcv) {
      // rows past the chunk's samples feed the dense GEMMs: keep them zero
      for (int f = threadIdx.x; f < d.F; f += LT) {
        fj[(int64_t)n * d.F + f] = 0.0f;
        if (fTj) fTj[(int64_t)f * ldT + n] = 0.0f;
      }
      continue;
    }
    __syncthreads();  // the weights are in; the previous image's readers are done with xin and p1
    load_image(X, xld, c0 + n, d, S.xin);
    __syncthreads();
    float* p1 = S.p1;
    float* mn = maps ? maps + (int64_t)j * sM + (int64_t)n * d.Mimg : nullptr;  // this image's conv2 activations
    conv_act_pool<KS, ACT>(S.xin, P0, Wpd, d.Cin, S.w1, S.b1, d.C1, d.Hp, d.Wp, nullptr,
                           [&](int q, int c, float v) { p1[c * P1 + q] = v; });
    __syncthreads();
    const int C2 = d.C2;
    conv_act_pool<KS, ACT>(p1, P1, d.Wp, d.C1, S.w2, S.b2, d.C2, d.Hq, d.Wq, mn,
                           [&](int q, int c, float v) {
      const int f = q * C2 + c;
      fj[(int64_t)n * d.F + f] = v;
      if (fTj) fTj[(int64_t)f * ldT + n] = v;
    });
  }
}

// Error of the pooled conv1 map: dp1[c][y][x] = sum over taps and o of dz2[o][y - ky][x - kx] w2[o][c][ky][kx],
// one pooled pixel per lane.  The tap loops run in full for every lane (out-of-range taps read
// a clamped address and contribute zero), so the weight addresses are uniform and come from the
// particle's global row (w2g, rows [o][(ky KS + kx) NC + c | bias]) through the scalar cache.
template <int KS, int NC>
__device__ __forceinline__ void conv2_input_error(const float* dz2, float* dp1,
                                                  const __attribute__((address_space(4))) float* w2g, int C2, int H2,
                                                  int W2, int Hp, int Wp) {
  constexpr int ROW = KS * KS * NC + 1;
  const int P1 = Hp * Wp, P2 = H2 * W2;
  for (int base = 0; base < P1; base += LT) {  // uniform trip count: lanes past P1 repeat the last pixel
    const int pix = min(base + (int)threadIdx.x, P1 - 1);
    const int y = pix / Wp, x = pix - y * Wp;
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0f;
    for (int o = 0; o < C2; ++o) {
      const float* eo = dz2 + o * P2;
      const __attribute__((address_space(4))) float* wo = w2g + o * ROW;
#pragma unroll
      for (int ky = 0; ky < KS; ++ky) {
        const int yy = y - ky;
        const bool vy = yy >= 0 && yy < H2;
        const int yc = vy ? yy : 0;
#pragma unroll
        for (int kx = 0; kx < KS; ++kx) {
          const int xx = x - kx;
          const bool v = vy && xx >= 0 && xx < W2;
          const float ev = eo[yc * W2 + (v ? xx : 0)];
          const float e = v ? ev : 0.0f;
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] = fmaf(e, wo[(ky * KS + kx) * NC + c], acc[c]);
        }
      }
    }
    if (base + (int)threadIdx.x < P1) {
#pragma unroll
      for (int c = 0; c < NC; ++c) dp1[c * P1 + pix] = acc[c];
    }
  }
}

template <int KS, int ACT>
__global__ __launch_bounds__(LT) void lenet_bwd_kernel(const float* __restrict__ X, int64_t xld, int64_t c0, int mcv,
                                                       int ipb, LenetDims d, const float* __restrict__ theta, int64_t D,
                                                       const float* __restrict__ dfeat, int64_t sF,
                                                       const float* __restrict__ maps, int64_t sM,
                                                       float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) float lsm[];
  const LenetSmem S = lenet_smem(lsm, d, true);
  const int j = blockIdx.y, tid = threadIdx.x;
  const int n0 = blockIdx.x * ipb, n1 = min(n0 + ipb, mcv);
  load_conv_weights(theta, D, j, d, S, false);
  const int Wpd = d.W + 2 * d.pad, P0 = (d.H + 2 * d.pad) * Wpd;
  const int HW = d.H * d.W, P1 = d.Hp * d.Wp, P2 = d.H2 * d.W2;
  const int C1 = d.C1, C2 = d.C2, Cin = d.Cin;
  // conv2 weight-gradient item (output pair o2, input channel c2i, kernel row ky2): KS
  // accumulators per output, a sweep over the rows of the conv2 output
  const int i2 = tid / KS, ky2 = tid - i2 * KS, o2 = 2 * (i2 / C1), c2i = i2 - (i2 / C1) * C1;
  const bool own2 = o2 < C2;
  const bool two2 = o2 + 1 < C2;
  // conv1 weight-gradient item (output pair o1, input channel c1i, kernel row ky1, row slice s1)
  const int n1i = (C1 + 1) / 2 * Cin * KS;
  const int s1 = tid / n1i, r1 = tid - s1 * n1i;
  const int i1 = r1 / KS, ky1 = r1 - i1 * KS, o1 = 2 * (i1 / Cin), c1i = i1 - (i1 / Cin) * Cin;
  const bool own1 = s1 < d.ns1;
  const bool two1 = o1 + 1 < C1;
  const int span1 = (d.H + d.ns1 - 1) / d.ns1;
  const int ya = min(d.H, s1 * span1), yb = min(d.H, ya + span1);
  float g2[2][KS], g1[2][KS], gb2[2] = {0.0f, 0.0f}, gb1[2] = {0.0f, 0.0f};
#pragma unroll
  for (int kx = 0; kx < KS; ++kx) g1[0][kx] = g1[1][kx] = g2[0][kx] = g2[1][kx] = 0.0f;

  const float* dfj = dfeat + (int64_t)j * sF;
  for (int n = n0; n < n1; ++n) {
    __syncthreads();
    load_image(X, xld, c0 + n, d, S.xin);
    {
      // the conv2 activations the forward saved
      const float* mn = maps + (int64_t)j * sM + (int64_t)n * d.Mimg;
      for (int e = tid; e < C2 * P2; e += LT) S.a2[e] = mn[e];
    }
    __syncthreads();
    float* p1 = S.p1;
    // conv1 again (cheaper than saving its full-resolution maps): activations a1 and the pooled p1
    conv_act_pool<KS, ACT>(S.xin, P0, Wpd, Cin, S.w1, S.b1, C1, d.Hp, d.Wp, S.a1,
                           [&](int q, int c, float v) { p1[c * P1 + q] = v; });
    __syncthreads();
    // dz2 = unpool(dfeat) * act'(a2), in place (planar)
    for (int e = tid; e < C2 * P2; e += LT) {
      const int c = e / P2, pix = e - c * P2;
      const int y = pix / d.W2, x = pix - y * d.W2;
      const float g = dfj[(int64_t)n * d.F + ((y >> 1) * d.Wq + (x >> 1)) * C2 + c];
      S.a2[e] = 0.25f * g * actg<ACT>(S.a2[e]);
    }
    __syncthreads();
    const float* dz2 = S.a2;
    // conv2 weight gradient: sum over conv2 output pixels of dz2[o][y][x] p1[c][y + ky][x + kx]
    if (own2) {
      const float* e0r = dz2 + o2 * P2;
      const float* e1r = two2 ? e0r + P2 : e0r;
      const float* pr = p1 + c2i * P1 + ky2 * d.Wp;
      const bool bias = c2i == 0 && ky2 == 0;
      for (int y = 0; y < d.H2; ++y) {
        for (int x = 0; x < d.W2; ++x) {
          const float e0 = e0r[y * d.W2 + x], e1 = e1r[y * d.W2 + x];
          if (bias) {
            gb2[0] += e0;
            gb2[1] += e1;
          }
#pragma unroll
          for (int kx = 0; kx < KS; ++kx) {
            const float v = pr[y * d.Wp + x + kx];
            g2[0][kx] = fmaf(e0, v, g2[0][kx]);
            g2[1][kx] = fmaf(e1, v, g2[1][kx]);
          }
        }
      }
    }
    // error of the pooled conv1 map (the channel count is a template parameter, so every weight
    // offset within a row is a constant)
    {
      typedef const __attribute__((address_space(4))) float* cfloat_p;  // read-only: scalar loads
      const cfloat_p w2g = (cfloat_p)(theta + (int64_t)j * D + C1 * (d.K1 + 1));  // rows [o][tap C1 + c | bias]
      switch (C1) {
#define LENET_DP1(NC) \
  case NC: conv2_input_error<KS, NC>(dz2, S.dp1, w2g, C2, d.H2, d.W2, d.Hp, d.Wp); break;
        LENET_DP1(1) LENET_DP1(2) LENET_DP1(3) LENET_DP1(4) LENET_DP1(5) LENET_DP1(6) LENET_DP1(7) LENET_DP1(8)
#undef LENET_DP1
        default: break;
      }
    }
    __syncthreads();
    // dz1 = unpool(dp1) * act'(a1), in place (planar)
    for (int e = tid; e < C1 * HW; e += LT) {
      const int c = e / HW, pix = e - c * HW;
      const int y = pix / d.W, x = pix - y * d.W;
      S.a1[e] = 0.25f * S.dp1[c * P1 + (y >> 1) * d.Wp + (x >> 1)] * actg<ACT>(S.a1[e]);
    }
    __syncthreads();
    // conv1 weight gradient over this item's slice of rows
    if (own1) {
      const float* e0r = S.a1 + o1 * HW;
      const float* e1r = two1 ? e0r + HW : e0r;
      const float* xr = S.xin + c1i * P0 + ky1 * Wpd;
      const bool bias = c1i == 0 && ky1 == 0;
      for (int y = ya; y < yb; ++y) {
        for (int x = 0; x < d.W; ++x) {
          const float e0 = e0r[y * d.W + x], e1 = e1r[y * d.W + x];
          if (bias) {
            gb1[0] += e0;
            gb1[1] += e1;
          }
#pragma unroll
          for (int kx = 0; kx < KS; ++kx) {
            const float v = xr[y * Wpd + x + kx];
            g1[0][kx] = fmaf(e0, v, g1[0][kx]);
            g1[1][kx] = fmaf(e1, v, g1[1][kx]);
          }
        }
      }
    }
  }
  // the block's partial in the theta layout: conv2 items directly, conv1 row slices summed in
  // order through LDS (the a1 region, free now)
  float* pj = part + ((int64_t)j * gridDim.x + blockIdx.x) * d.Dconv;
  float* pw2 = pj + C1 * (d.K1 + 1);
  if (own2) {
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two2) break;
      float* row = pw2 + (o2 + h) * (d.K2 + 1);
#pragma unroll
      for (int kx = 0; kx < KS; ++kx) row[(ky2 * KS + kx) * C1 + c2i] = g2[h][kx];
      if (c2i == 0 && ky2 == 0) row[d.K2] = gb2[h];
    }
  }
  __syncthreads();
  if (own1) {
    float* gs = S.g1s + s1 * C1 * (d.K1 + 1);
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two1) break;
      float* row = gs + (o1 + h) * (d.K1 + 1);
#pragma unroll
      for (int kx = 0; kx < KS; ++kx) row[(ky1 * KS + kx) * Cin + c1i] = g1[h][kx];
      if (c1i == 0 && ky1 == 0) row[d.K1] = gb1[h];
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
                      float* maps, int64_t sM, size_t smem, hipStream_t s) {
  const dim3 grid((unsigned)((rows + ipb - 1) / ipb), (unsigned)J);
  hipLaunchKernelGGL((lenet_fwd_kernel<KS, ACT>), grid, dim3(LT), smem, s, X, xld, c0, mcv, rows, ipb, d, theta, D,
                     feat, sF, featT, ldT, maps, sM);
  return hipGetLastError();
}

template <int KS, int ACT>
hipError_t launch_bwd(const float* X, int64_t xld, int64_t c0, int mcv, int ipb, int nblk, const LenetDims& d,
                      const float* theta, int64_t D, int J, const float* dfeat, int64_t sF, const float* maps,
                      int64_t sM, float* part, size_t smem, hipStream_t s) {
  hipLaunchKernelGGL((lenet_bwd_kernel<KS, ACT>), dim3((unsigned)nblk, (unsigned)J), dim3(LT), smem, s, X, xld, c0,
                     mcv, ipb, d, theta, D, dfeat, sF, maps, sM, part);
  return hipGetLastError();
}

}  // namespace

size_t lenet_smem_bytes(const LenetDims& d, bool bwd) { return (size_t)lenet_smem_floats(d, bwd, nullptr) * 4; }

int lenet_bwd_resident(const LenetDims& d, int act) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const void* f = d.k == 3 ? (act == ACT_RELU ? (const void*)lenet_bwd_kernel<3, ACT_RELU> : (const void*)lenet_bwd_kernel<3, ACT_TANH>)
                           : (act == ACT_RELU ? (const void*)lenet_bwd_kernel<5, ACT_RELU> : (const void*)lenet_bwd_kernel<5, ACT_TANH>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, LT, lenet_smem_bytes(d, true)) != hipSuccess) return 0;
  return ncu * per;
}

hipError_t lenet_fwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int rows, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, float* feat, int64_t sF, float* featT,
                         int64_t ldT, float* maps, int64_t sM, hipStream_t s) {
  if (rows <= 0 || J <= 0) return hipSuccess;
  if (ipb < 1 || mcv > rows || (d.k != 3 && d.k != 5)) return hipErrorInvalidValue;
  const size_t smem = lenet_smem_bytes(d, false);
#define LENET_FWD(KS, ACT) \
  launch_fwd<KS, ACT>(X, xld, c0, mcv, rows, ipb, d, theta, D, J, feat, sF, featT, ldT, maps, sM, smem, s)
  if (d.k == 3) return act == ACT_RELU ? LENET_FWD(3, ACT_RELU) : LENET_FWD(3, ACT_TANH);
  return act == ACT_RELU ? LENET_FWD(5, ACT_RELU) : LENET_FWD(5, ACT_TANH);
#undef LENET_FWD
}

hipError_t lenet_bwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, const float* dfeat, int64_t sF,
                         const float* maps, int64_t sM, float* part, int part_blocks, float* g, int beta,
                         hipStream_t s) {
  if (mcv <= 0 || J <= 0) return hipSuccess;
  const int nblk = (mcv + ipb - 1) / ipb;
  if (ipb < 1 || nblk > part_blocks || !maps || (d.k != 3 && d.k != 5)) return hipErrorInvalidValue;
  const size_t smem = lenet_smem_bytes(d, true);
#define LENET_BWD(KS, ACT) \
  launch_bwd<KS, ACT>(X, xld, c0, mcv, ipb, nblk, d, theta, D, J, dfeat, sF, maps, sM, part, smem, s)
  hipError_t e;
  if (d.k == 3) e = act == ACT_RELU ? LENET_BWD(3, ACT_RELU) : LENET_BWD(3, ACT_TANH);
  else e = act == ACT_RELU ? LENET_BWD(5, ACT_RELU) : LENET_BWD(5, ACT_TANH);
#undef LENET_BWD
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lenet_reduce_kernel, dim3((unsigned)((d.Dconv + 255) / 256), (unsigned)J), dim3(256), 0, s, part,
                     nblk, d.Dconv, g, D, beta);
  return hipGetLastError();
}

}  // namespace smc
