// Learned proposal-scale network: a 4 -> 64 -> 64 -> (1+G) MLP (tanh hidden
// layers) mapping per-particle features to a step size h_j and per-group masses
// m_{j,g} of a preconditioned Langevin move, and the kernels that train it.
//
// This is an extension of the method: the paper's Markov kernels use one fixed
// step size and an identity mass matrix (Section 2.1).  With state-dependent
// (h, m) the Jacobian cancellation of Eqs. q_prop / l=q_deriv does not hold, so
// the move's Gaussian forward density and a Gaussian reverse L-kernel with the
// parameters recomputed at the new state enter the general weight of
// Eq. weight_update.
//
// Parameter blob (float): mu[4], sd[4], W1[64x4], b1[64], W2[64x64], b2[64],
// W3[NO x 64], b3[NO] with NO = 1 + G; matrices [out x in] row-major.  The
// standardised inputs (f - mu) / sd are clipped to [-3, 3].
// Inference runs the 64x64 layer on BF16 MFMAs (v_mfma_f32_16x16x16_bf16);
// training runs it on FP32 MFMAs (v_mfma_f32_16x16x4_f32) and reduces per-tile
// gradient partials in a fixed order before the Adam update (Kingma and Ba).
#include "kernels.h"

#include <math.h>

namespace smc {

namespace {

constexpr int NH = 64;       // hidden width
constexpr int NF = 4;        // features
constexpr int RT = 64;       // rows per workgroup tile
constexpr int LA = NH + 4;   // padded LDS row of the activation tiles (floats)
constexpr float LN10 = 2.302585092994046f;
constexpr float LN_H = 2.0794415416798357f;  // bound of log(h / h0): the step-size grid spans h0 8^(+-1)

struct MlpOff {
  int mu, sd, W1, b1, W2, b2, W3, b3, P;
};
__host__ __device__ inline MlpOff mlp_off(int NO) {
  MlpOff o;
  o.mu = 0;
  o.sd = NF;
  o.W1 = 2 * NF;
  o.b1 = o.W1 + NH * NF;
  o.W2 = o.b1 + NH;
  o.b2 = o.W2 + NH * NH;
  o.W3 = o.b2 + NH;
  o.b3 = o.W3 + NO * NH;
  o.P = o.b3 + NO;
  return o;
}

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s16x4;

// ------------------------------------------------------------------ shared tile forward
// Forward pass of RT rows staged in LDS.  P: parameters (float, LDS);
// W2b: W2 as bf16 (LDS) when BF16; u[RT][NF]; a1, a2 [RT][LA]; o[RT][NO].
template <bool BF16>
__device__ void mlp_tile_forward(const float* P, const __bf16* W2b, const MlpOff& off, int NO, const float* u, float* a1,
                                 float* a2, float* o) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, cl = lane & 15;
  // layer 1 on the vector units
  {
    const int k = tid & 63;
    for (int r = tid >> 6; r < RT; r += 4) {
      float z = P[off.b1 + k];
#pragma unroll
      for (int f = 0; f < NF; ++f) z = fmaf(P[off.W1 + k * NF + f], u[r * NF + f], z);
      a1[r * LA + k] = tanhf(z);
    }
  }
  __syncthreads();
  // layer 2 on the matrix cores: rows 16w.., 4 blocks of 16 units
  for (int nb = 0; nb < 4; ++nb) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const float* arow = a1 + (16 * w + cl) * LA + 4 * g;
    if constexpr (BF16) {
      const __bf16* wrow = W2b + (nb * 16 + cl) * NH + 4 * g;
#pragma unroll
      for (int kb = 0; kb < NH / 16; ++kb) {
        s16x4 av, bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          av[t] = __builtin_bit_cast(short, to_bf16(arow[kb * 16 + t]));
          bv[t] = __builtin_bit_cast(short, wrow[kb * 16 + t]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
    } else {
      const float* wrow = P + off.W2 + (nb * 16 + cl) * NH + 4 * g;
#pragma unroll
      for (int kb = 0; kb < NH / 16; ++kb) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[kb * 16 + t], wrow[kb * 16 + t], acc, 0, 0, 0);
      }
    }
    // accumulator: rows 16w + 4g + i, unit nb*16 + cl
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * w + 4 * g + i, k = nb * 16 + cl;
      a2[r * LA + k] = tanhf(acc[i] + P[off.b2 + k]);
    }
  }
  __syncthreads();
  // layer 3 on the vector units
  {
    const int r = tid & 63;
    for (int c = tid >> 6; c < NO; c += 4) {
      float z = P[off.b3 + c];
      for (int k = 0; k < NH; ++k) z = fmaf(P[off.W3 + c * NH + k], a2[r * LA + k], z);
      o[r * NO + c] = z;
    }
  }
  __syncthreads();
}

// Stage parameters (and the bf16 W2) and a tile of normalised inputs into LDS.
__device__ void stage_params(const float* params, int Pn, float* P, __bf16* W2b, const MlpOff& off, bool bf16) {
  for (int e = threadIdx.x; e < Pn; e += blockDim.x) P[e] = params[e];
  if (bf16)
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x) W2b[e] = to_bf16(params[off.W2 + e]);
  __syncthreads();
}

template <typename FT>
__device__ void stage_inputs(const FT* feat, int64_t R, int64_t r0, const float* P, const MlpOff& off, float* u) {
  for (int e = threadIdx.x; e < RT * NF; e += blockDim.x) {
    const int r = e / NF, f = e - r * NF;
    const int64_t gr = r0 + r;
    const float x = gr < R ? (float)feat[gr * NF + f] : 0.0f;
    // standardised inputs are clipped to three training standard deviations (NaN passes through)
    const float z = (x - P[off.mu + f]) / P[off.sd + f];
    u[e] = z > 3.0f ? 3.0f : (z < -3.0f ? -3.0f : z);
  }
  __syncthreads();
}

struct MlpSmem {
  float* P;
  __bf16* W2b;
  float *u, *a1, *a2, *o, *d2;
};
__device__ MlpSmem mlp_smem(char* base, int NO) {
  const MlpOff off = mlp_off(NO);
  MlpSmem s;
  s.P = (float*)base;
  char* p = base + ((off.P * 4 + 15) / 16) * 16;
  s.W2b = (__bf16*)p;
  p += NH * NH * 2;
  s.u = (float*)p;
  p += RT * NF * 4;
  s.a1 = (float*)p;
  p += RT * LA * 4;
  s.a2 = (float*)p;
  p += RT * LA * 4;
  s.d2 = (float*)p;
  p += RT * LA * 4;
  s.o = (float*)p;
  return s;
}
size_t mlp_smem_bytes(int NO) {
  const MlpOff off = mlp_off(NO);
  return ((off.P * 4 + 15) / 16) * 16 + NH * NH * 2 + RT * NF * 4 + 3 * RT * LA * 4 + RT * NO * 4 + 64;
}

// ------------------------------------------------------------------ inference
// mode 0: raw outputs [R x NO]; mode 1: bounded scales (h, m_1..m_G) [R x NO]
// with the fixed-step fallback (h0, 1) for rows whose outputs are not finite.
template <bool BF16, typename FT>
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* params, const FT* feat, int64_t R, int NO,
                                                        float* out, int mode, float h0) {
  extern __shared__ __attribute__((aligned(16))) char msm[];
  const MlpOff off = mlp_off(NO);
  const MlpSmem s = mlp_smem(msm, NO);
  stage_params(params, off.P, s.P, s.W2b, off, BF16);
  const int64_t r0 = (int64_t)blockIdx.x * RT;
  stage_inputs<FT>(feat, R, r0, s.P, off, s.u);
  mlp_tile_forward<BF16>(s.P, s.W2b, off, NO, s.u, s.a1, s.a2, s.o);
  const int r = threadIdx.x;
  if (r < RT && r0 + r < R) {
    const float* o = s.o + r * NO;
    float* dst = out + (r0 + r) * NO;
    if (mode == 0) {
      for (int c = 0; c < NO; ++c) dst[c] = o[c];
    } else {
      bool ok = true;
      for (int c = 0; c < NO; ++c) ok = ok && isfinite(o[c]);
      dst[0] = ok ? h0 * expf(LN_H * tanhf(o[0])) : h0;
      for (int c = 1; c < NO; ++c) dst[c] = ok ? expf(LN10 * tanhf(o[c])) : 1.0f;
    }
  }
}

// ------------------------------------------------------------------ training
// Forward and backward of one RT-row tile of the loss (1/R) sum_r 1/2 |o_r - t_r|^2;
// writes the tile's loss and gradient partials (mu, sd get zero gradient).
__global__ __launch_bounds__(256) void mlp_train_tile_kernel(const float* params, const float* feat, const float* tgt,
                                                             int64_t R, int NO, double* loss_part, float* grad_part) {
  extern __shared__ __attribute__((aligned(16))) char msm[];
  const MlpOff off = mlp_off(NO);
  const MlpSmem s = mlp_smem(msm, NO);
  stage_params(params, off.P, s.P, s.W2b, off, false);
  const int64_t r0 = (int64_t)blockIdx.x * RT;
  stage_inputs<float>(feat, R, r0, s.P, off, s.u);
  mlp_tile_forward<false>(s.P, s.W2b, off, NO, s.u, s.a1, s.a2, s.o);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, cl = lane & 15;
  const float invR = 1.0f / (float)R;
  float* gp = grad_part + (int64_t)blockIdx.x * off.P;
  // output error (kept in s.o) and the tile loss
  double lsum = 0.0;
  if (tid < RT) {
    const int64_t gr = r0 + tid;
    for (int c = 0; c < NO; ++c) {
      float d = 0.0f;
      if (gr < R) {
        const float e = s.o[tid * NO + c] - tgt[gr * NO + c];
        lsum += 0.5 * (double)e * e;
        d = e * invR;
      }
      s.o[tid * NO + c] = d;
    }
  }
  {
    const double v = wave_sum(lsum);
    if (tid == 0) loss_part[blockIdx.x] = v * (double)invR;
  }
  __syncthreads();
  // dW3, db3 and delta2 = (delta3 W3) * (1 - a2^2)
  for (int e = tid; e < NO * NH; e += 256) {
    const int c = e / NH, k = e - c * NH;
    float acc = 0.0f;
    for (int r = 0; r < RT; ++r) acc = fmaf(s.o[r * NO + c], s.a2[r * LA + k], acc);
    gp[off.W3 + e] = acc;
  }
  if (tid < NO) {
    float acc = 0.0f;
    for (int r = 0; r < RT; ++r) acc += s.o[r * NO + tid];
    gp[off.b3 + tid] = acc;
  }
  {
    const int k = tid & 63;
    for (int r = tid >> 6; r < RT; r += 4) {
      float acc = 0.0f;
      for (int c = 0; c < NO; ++c) acc = fmaf(s.o[r * NO + c], s.P[off.W3 + c * NH + k], acc);
      const float a = s.a2[r * LA + k];
      s.d2[r * LA + k] = acc * (1.0f - a * a);
    }
  }
  __syncthreads();
  // dW2 [o][i] = sum_r d2[r][o] a1[r][i] on FP32 MFMAs: wave w owns output rows 16w.., 4 column blocks
  for (int nb = 0; nb < 4; ++nb) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < RT / 16; ++kb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = kb * 16 + 4 * g + t;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s.d2[r * LA + 16 * w + cl], s.a1[r * LA + nb * 16 + cl], acc, 0, 0,
                                                   0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) gp[off.W2 + (16 * w + 4 * g + i) * NH + nb * 16 + cl] = acc[i];
  }
  if (tid < NH) {
    float acc = 0.0f;
    for (int r = 0; r < RT; ++r) acc += s.d2[r * LA + tid];
    gp[off.b2 + tid] = acc;
  }
  // delta1 = (d2 W2) * (1 - a1^2) on FP32 MFMAs: rows 16w.., 4 column blocks; result overwrites a2
  __syncthreads();
  for (int nb = 0; nb < 4; ++nb) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < NH / 16; ++kb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int o = kb * 16 + 4 * g + t;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(s.d2[(16 * w + cl) * LA + o], s.P[off.W2 + o * NH + nb * 16 + cl],
                                                   acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * w + 4 * g + i, k = nb * 16 + cl;
      const float a = s.a1[r * LA + k];
      s.a2[r * LA + k] = acc[i] * (1.0f - a * a);
    }
  }
  __syncthreads();
  // dW1, db1
  for (int e = tid; e < NH * NF; e += 256) {
    const int k = e / NF, f = e - k * NF;
    float acc = 0.0f;
    for (int r = 0; r < RT; ++r) acc = fmaf(s.a2[r * LA + k], s.u[r * NF + f], acc);
    gp[off.W1 + e] = acc;
  }
  if (tid < NH) {
    float acc = 0.0f;
    for (int r = 0; r < RT; ++r) acc += s.a2[r * LA + tid];
    gp[off.b1 + tid] = acc;
  }
  if (tid < 2 * NF) gp[tid] = 0.0f;
}

// Fixed-order sum of the tile partials, then one Adam step (or, with lr == 0, only the gradient).
__global__ void mlp_adam_kernel(float* params, float* adam, const float* grad_part, int ntiles, int Pn, int step,
                                float lr, float b1, float b2, float eps, float* grad_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pn) return;
  double gsum = 0.0;
  for (int t = 0; t < ntiles; ++t) gsum += (double)grad_part[(int64_t)t * Pn + p];
  const float gr = (float)gsum;
  if (grad_out) grad_out[p] = gr;
  if (lr == 0.0f || p < 2 * NF) return;
  float* m = adam;
  float* v = adam + Pn;
  m[p] = b1 * m[p] + (1.0f - b1) * gr;
  v[p] = b2 * v[p] + (1.0f - b2) * gr * gr;
  const float mh = m[p] / (1.0f - powf(b1, (float)step));
  const float vh = v[p] / (1.0f - powf(b2, (float)step));
  params[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void loss_sum_kernel(const double* part, int n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
  }
}

// ------------------------------------------------------------------ sampler-side kernels
__device__ __forceinline__ void group_of(const NetShape& n, int64_t e, int& l, int& o, int& i) {
  l = 0;
#pragma unroll
  for (int q = 1; q < MAX_LAYERS; ++q)
    if (q < n.L && e >= n.off[q]) l = q;
  const int rowlen = n.nin[l] + 1;
  const int ep = (int)(e - n.off[l]);
  o = (int)((float)ep * n.rinv[l]);
  while (o * rowlen > ep) --o;
  while ((o + 1) * rowlen <= ep) ++o;
  i = ep - o * rowlen;
}


// Learned Langevin move.  FIRST: theta' = theta + (h^2/2) gf / m + h xi / sqrt(m), P <- theta' - theta,
// partial sums |xi|^2 (row 0) and |theta'|^2 (row 1).  LAST: reverse-kernel quadratic form
// sum_e (theta - theta' - (h'^2/2) gf'/m')^2 m' / (2 h'^2) (row 2).
__global__ __launch_bounds__(256) void learned_move_kernel(const LearnedMoveArgs a) {
  __shared__ double red[3][4];
  const int j = blockIdx.y;
  const int64_t D = a.net.D;
  const int64_t e0 = (int64_t)blockIdx.x * MOVE_ELEMS + 4 * threadIdx.x;
  float* th = a.theta + (int64_t)j * D;
  float* P = a.P + (int64_t)j * D;
  const float* gg = a.g + (int64_t)j * D;
  const float* sc = a.scales + (int64_t)j * a.NO;
  const float h = sc[0];
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
  f32x4 nz = {0.0f, 0.0f, 0.0f, 0.0f};
  if (a.mode == MOVE_FIRST && !a.noise && e0 < D) {
    const u32x4 c = {(uint32_t)(e0 >> 2), (uint32_t)j, a.ctr_iter, (uint32_t)TAG_MOMENTUM};
    nz = normal4(philox4x32_10(c, a.key0, a.key1));
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = e0 + q;
    if (e >= D) break;
    int l, o, i;
    group_of(a.net, e, l, o, i);
    const float m = sc[1 + 2 * l + (i == a.net.nin[l] ? 1 : 0)];
    const float t = th[e];
    const float gf = gg[e] - t * a.inv_prior_var;
    if (a.mode == MOVE_FIRST) {
      const float xi = a.noise ? a.noise[(int64_t)j * D + e] : nz[q];
      const float d = 0.5f * h * h * gf / m + h * xi * rsqrtf(m);
      const float t1 = t + d;
      P[e] = d;
      th[e] = t1;
      s0 += xi * xi;
      s1 += t1 * t1;
      weight_copy_store(a.net, j, l, o, i, t1);
    } else {
      const float r = -P[e] - 0.5f * h * h * gf / m;
      s2 += r * r * m / (2.0f * h * h);
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double v0 = wave_sum((double)s0), v1 = wave_sum((double)s1), v2 = wave_sum((double)s2);
  if (lane == 0) { red[0][wid] = v0; red[1][wid] = v1; red[2][wid] = v2; }
  __syncthreads();
  const int w = threadIdx.x;
  const bool own = (a.mode == MOVE_FIRST && w < 2) || (a.mode == MOVE_LAST && w == 2);
  if (w < 3 && own) a.part[((int64_t)w * a.net.J + j) * a.nblk + blockIdx.x] = red[w][0] + red[w][1] + red[w][2] + red[w][3];
}

// extra[j] = log L - log q + (the kinetic-free parts):
//   -D (log h' - log h) + 1/2 sum_g n_g (log m'_g - log m_g) - R_j + 1/2 |xi_j|^2
__global__ void learned_extra_kernel(const float* sc0, const float* sc1, int NO, const double* part, int J, int nblk,
                                     const int64_t* group_n, int64_t D, double* extra) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  double xi2 = 0.0, quad = 0.0;
  for (int b = 0; b < nblk; ++b) {
    xi2 += part[(int64_t)j * nblk + b];
    quad += part[((int64_t)2 * J + j) * nblk + b];
  }
  const float* a = sc0 + (int64_t)j * NO;
  const float* b = sc1 + (int64_t)j * NO;
  double v = -(double)D * (log((double)b[0]) - log((double)a[0]));
  for (int q = 1; q < NO; ++q) v += 0.5 * (double)group_n[q - 1] * (log((double)b[q]) - log((double)a[q]));
  extra[j] = v - quad + 0.5 * xi2;
}

// features (log |grad log pi|, LL / M, k / K, M / N) and per-group sums of (grad log pi)^2
__global__ __launch_bounds__(256) void features_kernel(const NetShape n, const float* theta, const float* g,
                                                       const double* ll, float inv_prior_var, double m, double k_over_K,
                                                       double m_over_N, double* feat, double* gsum, int G) {
  __shared__ double red[4];
  __shared__ double gred[2 * MAX_LAYERS][4];
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double s = 0.0;
  double gs[2 * MAX_LAYERS];
#pragma unroll
  for (int q = 0; q < 2 * MAX_LAYERS; ++q) gs[q] = 0.0;
  for (int64_t e = threadIdx.x; e < n.D; e += 256) {
    const float t = theta[(int64_t)j * n.D + e];
    const double v = (double)(g[(int64_t)j * n.D + e] - t * inv_prior_var);
    s += v * v;
    if (gsum) {
      int l, o, i;
      group_of(n, e, l, o, i);
      const int gi = 2 * l + (i == n.nin[l] ? 1 : 0);
#pragma unroll
      for (int q = 0; q < 2 * MAX_LAYERS; ++q)
        if (q == gi) gs[q] += v * v;
    }
  }
  s = block_sum(s, red);
  if (gsum) {
#pragma unroll
    for (int q = 0; q < 2 * MAX_LAYERS; ++q) {
      const double v = wave_sum(gs[q]);
      if (lane == 0) gred[q][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < G) {
      const int q = threadIdx.x;
      gsum[(int64_t)j * G + q] = gred[q][0] + gred[q][1] + gred[q][2] + gred[q][3];
    }
  }
  if (threadIdx.x == 0 && feat) {
    feat[j * 4 + 0] = 0.5 * log(s);
    feat[j * 4 + 1] = ll[j] / m;
    feat[j * 4 + 2] = k_over_K;
    feat[j * 4 + 3] = m_over_N;
  }
}

// Step-size trial scoring: D = log pi(theta') - log pi(theta) - |P_end|^2/2 + |xi|^2/2 (the
// Metropolis log-ratio of the Langevin trial under the current target) and the squared jump
// h^2 |P_half|^2; keeps the best log h per particle.
__global__ void trial_score_kernel(const double* part, int J, int nblk, const double* ll1, const double* lp0,
                                   double lambda, double inv_2pv, double h, double accept_power, const double* phalf_sq,
                                   double* best_score, double* best_logh, int first) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  double xi2 = 0.0, t2 = 0.0, pe2 = 0.0;
  for (int b = 0; b < nblk; ++b) {
    xi2 += part[(int64_t)j * nblk + b];
    t2 += part[((int64_t)J + j) * nblk + b];
    pe2 += part[((int64_t)2 * J + j) * nblk + b];
  }
  const double lp1 = lambda * ll1[j] - t2 * inv_2pv;
  const double d = lp1 - lp0[j] - 0.5 * pe2 + 0.5 * xi2;
  double score = h * h * phalf_sq[j] * exp(accept_power * fmin(d, 0.0));
  if (!isfinite(score)) score = -INFINITY;
  if (first || score > best_score[j]) {
    best_score[j] = score;
    best_logh[j] = log(h);
  }
}

// regression targets: t_0 = atanh(clip((log h* - log h0)/ln10)), t_g = atanh(clip(log m*_g / ln10)) with
// log m*_g the log RMS of group g's gradient entries centred over the groups
__global__ void targets_kernel(const double* best_logh, const double* gsum, const int64_t* group_n, int J, int G,
                               double h0, double clip, float* tgt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int NO = 1 + G;
  const double ln10 = 2.302585092994046;
  double t0 = (best_logh[j] - log(h0)) / 2.0794415416798357;  // ln 8
  t0 = fmax(-clip, fmin(clip, t0));
  tgt[(int64_t)j * NO] = (float)atanh(t0);
  double lm[2 * MAX_LAYERS];
  double mean = 0.0;
  for (int q = 0; q < G; ++q) {
    lm[q] = 0.5 * log(gsum[(int64_t)j * G + q] / (double)group_n[q]);
    mean += lm[q];
  }
  mean /= G;
  for (int q = 0; q < G; ++q) {
    double t = (lm[q] - mean) / ln10;
    t = fmax(-clip, fmin(clip, t));
    tgt[(int64_t)j * NO + 1 + q] = (float)atanh(t);
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t mlp_set_smem_limits() {
  const int big = 160 * 1024;
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)mlp_infer_kernel<true, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               big)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)mlp_infer_kernel<false, float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)mlp_infer_kernel<true, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)mlp_infer_kernel<false, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, big)) != hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)mlp_train_tile_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

int mlp_n_params(int G) { return mlp_off(1 + G).P; }

hipError_t mlp_infer_run(const float* params, const void* feat, int feat_f64, int64_t R, int G, float* out, int mode,
                         float h0, int bf16, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int NO = 1 + G;
  dim3 grid((unsigned)((R + RT - 1) / RT));
  const size_t sm = mlp_smem_bytes(NO);
  if (feat_f64) {
    if (bf16)
      hipLaunchKernelGGL((mlp_infer_kernel<true, double>), grid, dim3(256), sm, s, params, (const double*)feat, R, NO,
                         out, mode, h0);
    else
      hipLaunchKernelGGL((mlp_infer_kernel<false, double>), grid, dim3(256), sm, s, params, (const double*)feat, R, NO,
                         out, mode, h0);
  } else {
    if (bf16)
      hipLaunchKernelGGL((mlp_infer_kernel<true, float>), grid, dim3(256), sm, s, params, (const float*)feat, R, NO,
                         out, mode, h0);
    else
      hipLaunchKernelGGL((mlp_infer_kernel<false, float>), grid, dim3(256), sm, s, params, (const float*)feat, R, NO,
                         out, mode, h0);
  }
  return hipGetLastError();
}

hipError_t mlp_train_step_run(float* params, float* adam, const float* feat, const float* tgt, int64_t R, int G,
                              float* grad_part, double* loss_part, int step, float lr, float* grad_out,
                              double* loss_out, hipStream_t s) {
  const int NO = 1 + G;
  const int Pn = mlp_off(NO).P;
  const int ntiles = (int)((R + RT - 1) / RT);
  hipLaunchKernelGGL(mlp_train_tile_kernel, dim3(ntiles), dim3(256), mlp_smem_bytes(NO), s, params, feat, tgt, R, NO,
                     loss_part, grad_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (loss_out) hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, s, loss_part, ntiles, loss_out);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((Pn + 255) / 256), dim3(256), 0, s, params, adam, grad_part, ntiles, Pn,
                     step, lr, 0.9f, 0.999f, 1e-8f, grad_out);
  return hipGetLastError();
}

hipError_t learned_move_run(const LearnedMoveArgs& a, hipStream_t s) {
  dim3 grid(a.nblk, a.net.J);
  hipLaunchKernelGGL(learned_move_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t learned_extra_run(const float* sc0, const float* sc1, int NO, const double* part, int J, int nblk,
                             const int64_t* group_n, int64_t D, double* extra, hipStream_t s) {
  hipLaunchKernelGGL(learned_extra_kernel, dim3((J + 255) / 256), dim3(256), 0, s, sc0, sc1, NO, part, J, nblk, group_n,
                     D, extra);
  return hipGetLastError();
}

hipError_t features_run(const NetShape& n, const float* theta, const float* g, const double* ll, float ipv, double m,
                        double k_over_K, double m_over_N, double* feat, double* gsum, int G, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(n.J), dim3(256), 0, s, n, theta, g, ll, ipv, m, k_over_K, m_over_N, feat,
                     gsum, G);
  return hipGetLastError();
}

hipError_t trial_score_run(const double* part, int J, int nblk, const double* ll1, const double* lp0, double lambda,
                           double inv_2pv, double h, double accept_power, const double* phalf_sq, double* best_score,
                           double* best_logh,
                           int first, hipStream_t s) {
  hipLaunchKernelGGL(trial_score_kernel, dim3((J + 255) / 256), dim3(256), 0, s, part, J, nblk, ll1, lp0, lambda,
                     inv_2pv, h, accept_power, phalf_sq, best_score, best_logh, first);
  return hipGetLastError();
}

hipError_t targets_run(const double* best_logh, const double* gsum, const int64_t* group_n, int J, int G, double h0,
                       double clip, float* tgt, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3((J + 255) / 256), dim3(256), 0, s, best_logh, gsum, group_n, J, G, h0, clip,
                     tgt);
  return hipGetLastError();
}

}  // namespace smc
