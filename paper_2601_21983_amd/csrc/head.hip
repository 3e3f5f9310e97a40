// Output layer of every particle's network: logits, log-likelihood, the
// output-layer gradient and the error sent to the last hidden layer.
//
// For particle j and a tile of 64 samples the kernel
//   * stages the last hidden activations a_{L-1} (any layout, via strides) in LDS,
//   * forms z = W_L a + b_L (W_L read from the FP32 master parameters),
//   * categorical: log p = z_y - logsumexp(z), delta = lambda_j (onehot - softmax(z));
//     Gaussian:    log p = -1/2 log(2 pi s^2) - (y - z)^2 / (2 s^2), delta = lambda_j (y - z) / s^2
//     (the subset log-likelihood sum and its scaled gradient, Section 3, Eq. approx-grad),
//   * accumulates dW_L (and db_L) = sum_i delta_i [a_i, 1] in registers,
//   * writes delta_{L-1} = (W_L^T delta) * act'(a) transposed ([unit][sample]) for the
//     weight-gradient GEMM of the layer below, and optionally row-major.
// Log-likelihoods are accumulated in FP64 per thread in sample order and reduced
// in a fixed order, so results do not depend on scheduling.
#include "kernels.h"

namespace smc {

namespace {

constexpr int HT = 64;        // samples per tile
constexpr int HTHREADS = 256;
constexpr int MAXP = 40;      // register accumulators per thread for dW_L: C*(H+1) <= 40*256

template <typename T, int MODE>
__global__ __launch_bounds__(HTHREADS) void head_kernel(const HeadArgs a) {
  extern __shared__ __attribute__((aligned(16))) float hs[];
  const int H = a.H, C = a.C, HP = H + 1;  // HP: padded LDS row (odd stride for H even)
  const int HS = (H | 1);
  float* Ws = hs;                        // [C][HP]  (weights, bias in column H)
  float* As = Ws + C * HP;               // [HT][HS]
  float* Zs = As + HT * HS;              // [HT][C]  logits, then deltas
  const int j = blockIdx.y;
  const int split = blockIdx.x;
  const int tid = threadIdx.x;
  const float* wsrc = a.theta + (int64_t)j * a.D + a.offL;
  for (int e = tid; e < C * HP; e += HTHREADS) Ws[e] = wsrc[e];

  const float lam = a.scale ? (float)a.scale[j] : (float)a.lambda;
  const T* Aj = (const T*)a.A + (int64_t)j * a.sAj;
  const int ntiles = (a.m_valid + HT - 1) / HT;
  const int t0 = split * a.tiles_per_split;
  const int t1 = min(ntiles, t0 + a.tiles_per_split);
  const float rinvH = 1.0f / (float)H;

  double llacc = 0.0;
  float dacc[MAXP];
#pragma unroll
  for (int q = 0; q < MAXP; ++q) dacc[q] = 0.0f;
  const int npair = C * HP;
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int s0 = t * HT;
    // 1. stage the activation tile
    for (int e = tid; e < HT * H; e += HTHREADS) {
      int s = (int)(((float)e + 0.5f) * rinvH);
      int h = e - s * H;
      if (h < 0) { --s; h += H; } else if (h >= H) { ++s; h -= H; }
      As[s * HS + h] = cvt_in<T>(Aj[(int64_t)(s0 + s) * a.sAm + h]);
    }
    __syncthreads();
    // 2. logits
    {
      const int s = tid & 63;
      for (int c = tid >> 6; c < C; c += 4) {
        const float* w = Ws + c * HP;
        const float* x = As + s * HS;
        float z = w[H];
        for (int h = 0; h < H; ++h) z = fmaf(w[h], x[h], z);
        Zs[s * C + c] = z;
      }
    }
    __syncthreads();
    // 3. per-sample likelihood and output error
    if (tid < HT) {
      const int s = tid;
      const bool valid = s0 + s < a.m_valid;
      float* z = Zs + s * C;
      if (a.likelihood == 0) {
        float mx = z[0];
        for (int c = 1; c < C; ++c) mx = fmaxf(mx, z[c]);
        float se = 0.0f;
        for (int c = 0; c < C; ++c) se += expf(z[c] - mx);
        const float lse = mx + logf(se);
        if (MODE == HEAD_PREDICT) {
          if (valid) {
            float* lp = a.logp + ((int64_t)j * a.ld_logp + a.c0 + s0 + s) * C;
            for (int c = 0; c < C; ++c) lp[c] = z[c] - lse;
          }
        } else {
          const int y = valid ? a.ylab[a.c0 + s0 + s] : 0;
          if (valid) llacc += (double)(z[y] - lse);
          if (MODE == HEAD_TRAIN) {
            for (int c = 0; c < C; ++c) {
              const float p = expf(z[c] - lse);
              z[c] = valid ? lam * ((c == y ? 1.0f : 0.0f) - p) : 0.0f;
            }
          }
        }
      } else {
        const float y = valid ? a.yreal[a.c0 + s0 + s] : 0.0f;
        const float r = y - z[0];
        if (MODE == HEAD_PREDICT) {
          if (valid) a.logp[(int64_t)j * a.ld_logp + a.c0 + s0 + s] = z[0];
        } else {
          if (valid) llacc += (double)(a.gauss_c - 0.5f * r * r * a.inv_var);
          if (MODE == HEAD_TRAIN) z[0] = valid ? lam * r * a.inv_var : 0.0f;
        }
      }
    }
    __syncthreads();
    if (MODE == HEAD_TRAIN) {
      // 4. error of the last hidden layer, written [unit][sample]
      if (a.dT) {
        const int s = tid & 63;
        T* dT = (T*)a.dT + (int64_t)j * a.sdTj + s0 + s;
        T* dR = a.dR ? (T*)a.dR + (int64_t)j * a.sdRj + (int64_t)(s0 + s) * a.sdRm : nullptr;
        const float* dz = Zs + s * C;
        const float* x = As + s * HS;
        for (int h = tid >> 6; h < H; h += 4) {
          float v = 0.0f;
          for (int c = 0; c < C; ++c) v = fmaf(dz[c], Ws[c * HP + h], v);
          v *= act_grad_from_out(x[h], a.act);
          dT[(int64_t)h * a.sdTh] = cvt_out<T>(v);
          if (dR) dR[h] = cvt_out<T>(v);
        }
      }
      // 5. output-layer gradient partial sums
#pragma unroll
      for (int q = 0; q < MAXP; ++q) {
        const int pidx = tid + q * HTHREADS;
        if (pidx < npair) {
          const int c = pidx / HP, h = pidx - c * HP;
          float acc = 0.0f;
          if (h < H) {
            for (int s = 0; s < HT; ++s) acc = fmaf(Zs[s * C + c], As[s * HS + h], acc);
          } else {
            for (int s = 0; s < HT; ++s) acc += Zs[s * C + c];
          }
          dacc[q] += acc;
        }
      }
    }
    __syncthreads();
  }

  if (MODE != HEAD_PREDICT) {
    // fixed-order reduction of the per-sample log-likelihood sums (threads 0..63 hold them)
    if (tid < 64) {
      const double v = wave_sum(llacc);
      if (tid == 0) a.llpart[(int64_t)j * a.nsplit + split] = v;
    }
  }
  if (MODE == HEAD_TRAIN) {
    float* dst = a.dWpart + ((int64_t)j * a.nsplit + split) * npair;
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
      const int pidx = tid + q * HTHREADS;
      if (pidx < npair) dst[pidx] = dacc[q];
    }
  }
}

// Sum the per-split partials of one chunk in a fixed order and fold them into the
// running totals: ll_acc[j] (+)= sum, grad[j][offL + e] (+)= sum.
__global__ void head_reduce_kernel(const HeadArgs a, int beta, int with_grad) {
  const int j = blockIdx.x;
  const int npair = a.C * (a.H + 1);
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < a.nsplit; ++k) s += a.llpart[(int64_t)j * a.nsplit + k];
    a.ll_acc[j] = beta ? a.ll_acc[j] + s : s;
  }
  if (!with_grad) return;
  const float* src = a.dWpart + (int64_t)j * a.nsplit * npair;
  float* g = a.grad + (int64_t)j * a.D + a.offL;
  for (int e = threadIdx.x; e < npair; e += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < a.nsplit; ++k) s += (double)src[(int64_t)k * npair + e];
    g[e] = beta ? g[e] + (float)s : (float)s;
  }
}

}  // namespace

size_t head_smem_bytes(int H, int C) {
  return sizeof(float) * ((size_t)C * (H + 1) + (size_t)HT * (H | 1) + (size_t)HT * C);
}
int head_max_pairs() { return MAXP * HTHREADS; }

hipError_t head_run(const HeadArgs& a, int mode, int bf16, hipStream_t s) {
  const int ntiles = (a.m_valid + HT - 1) / HT;
  if (ntiles <= 0) return hipSuccess;
  dim3 grid(a.nsplit, a.J);
  const size_t smem = head_smem_bytes(a.H, a.C);
  if (a.C * (a.H + 1) > head_max_pairs()) return hipErrorInvalidValue;
#define HEAD_LAUNCH(T, MODE) hipLaunchKernelGGL((head_kernel<T, MODE>), grid, dim3(HTHREADS), smem, s, a)
  if (bf16) {
    if (mode == HEAD_TRAIN) HEAD_LAUNCH(__bf16, HEAD_TRAIN);
    else if (mode == HEAD_FORWARD) HEAD_LAUNCH(__bf16, HEAD_FORWARD);
    else HEAD_LAUNCH(__bf16, HEAD_PREDICT);
  } else {
    if (mode == HEAD_TRAIN) HEAD_LAUNCH(float, HEAD_TRAIN);
    else if (mode == HEAD_FORWARD) HEAD_LAUNCH(float, HEAD_FORWARD);
    else HEAD_LAUNCH(float, HEAD_PREDICT);
  }
#undef HEAD_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode == HEAD_PREDICT) return e;
  hipLaunchKernelGGL(head_reduce_kernel, dim3(a.J), dim3(256), 0, s, a, a.beta, mode == HEAD_TRAIN ? 1 : 0);
  return hipGetLastError();
}

hipError_t head_set_smem_limits() {
  const int big = 160 * 1024;
#define HEAD_ATTR(T, MODE) \
  hipFuncSetAttribute((const void*)head_kernel<T, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize, big)
  hipError_t e = hipSuccess;
  e = HEAD_ATTR(float, HEAD_TRAIN); if (e != hipSuccess) return e;
  e = HEAD_ATTR(float, HEAD_FORWARD); if (e != hipSuccess) return e;
  e = HEAD_ATTR(float, HEAD_PREDICT); if (e != hipSuccess) return e;
  e = HEAD_ATTR(__bf16, HEAD_TRAIN); if (e != hipSuccess) return e;
  e = HEAD_ATTR(__bf16, HEAD_FORWARD); if (e != hipSuccess) return e;
  e = HEAD_ATTR(__bf16, HEAD_PREDICT);
#undef HEAD_ATTR
  return e;
}

}  // namespace smc
