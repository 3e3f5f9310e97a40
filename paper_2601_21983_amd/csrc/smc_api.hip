// C ABI of the MI355X data-annealed SMC sampler: handle, buffers and the
// orchestration of one iteration on a single HIP stream.
//
// Device memory layout (all owned by the handle):
//   X   [n_pad x xld]      inputs in the GEMM operand type, rows in annealing order,
//                          features padded with zeros to ldx (a multiple of 8); split
//                          BF16 stores each row twice ([x | x], xld = 2 ldx) so that
//                          the first-layer GEMM over K = 2 ldw computes
//                          x . w_hi + x . w_lo with w rows stored as [w_hi | w_lo]
//   XT  [(n_0+1) x n_pad]  the same inputs transposed, plus a row of ones so that
//                          the weight-gradient GEMM of layer 1 also yields the bias
//                          gradient (column n_0 of the augmented block [W | b])
//   theta, g, P [J x D]    FP32 master parameters (one contiguous row per particle),
//                          the lambda-scaled log-likelihood gradient (the prior term
//                          is added where it is used) and momenta
//   w_l  [J*n_l x ldw_l]   GEMM copy of each layer's weights (operand type), b_l [J*n_l]
//   act_l [J x mc x n_l]   hidden activations of one chunk of samples, particle-major
//                          (split BF16: FP32 values, split into hi/lo by the output-layer kernel)
//                          (one contiguous [samples x units] block per particle); layer 1
//                          is still a single dense GEMM over the J*n_1 concatenated units,
//                          whose epilogue scatters each particle's columns to its block
//   dT_l [J*n_l x mc]      back-propagated errors, sample-contiguous (K-major for the
//                          weight-gradient GEMM)
// The subset [0, M_k) is processed in chunks of mc samples; activations live only
// for one chunk, so the backward pass of a chunk always works from a freshly computed
// forward pass (activation recomputation bounded by act_budget_bytes).
#include "../../include/smc.h"
#include "kernels.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace smc;

namespace {

thread_local std::string g_last_error;

struct Fail {
  smc_status st;
};

void fail(smc_status st, const std::string& msg) {
  g_last_error = msg;
  throw Fail{st};
}

#define HIPCHECK(expr)                                                                                \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      fail(e_ == hipErrorOutOfMemory ? SMC_ERR_OOM : SMC_ERR_DEVICE,                                  \
           std::string(#expr) + ": " + hipGetErrorString(e_) + " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

template <typename T>
T* dalloc(std::vector<void*>& owned, int64_t n) {
  void* p = nullptr;
  if (n <= 0) n = 1;
  hipError_t e = hipMalloc(&p, (size_t)n * sizeof(T));
  if (e != hipSuccess) fail(SMC_ERR_OOM, "hipMalloc of " + std::to_string((size_t)n * sizeof(T)) + " bytes failed");
  owned.push_back(p);
  return (T*)p;
}

// ------------------------------------------------------------------ data preparation kernels
// X[r][q*ldx + c] = x[r][c] (zero padded) for q < reps; rows of reps*ldx elements
template <typename T>
__global__ void pack_x_kernel(const float* x, int64_t n, int F, int ldx, int reps, int64_t n_pad, T* X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad * ldx) return;
  const int64_t r = i / ldx;
  const int c = (int)(i - r * ldx);
  const T v = cvt_out<T>((r < n && c < F) ? x[r * F + c] : 0.0f);
  for (int q = 0; q < reps; ++q) X[r * ldx * reps + q * ldx + c] = v;
}

template <typename T>
__global__ void pack_xt_kernel(const float* x, int64_t n, int F, int64_t n_pad, T* XT) {
  // XT[f][r] for f in [0, F], with row F all ones
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)(F + 1) * n_pad) return;
  const int f = (int)(i / n_pad);
  const int64_t r = i - (int64_t)f * n_pad;
  float v;
  if (f == F) v = 1.0f;
  else v = r < n ? x[r * F + f] : 0.0f;
  XT[i] = cvt_out<T>(v);
}

__global__ void pack_labels_kernel(const void* y, int64_t n, int64_t n_pad, int gaussian, int32_t* ylab,
                                   float* yreal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  if (gaussian) yreal[i] = i < n ? ((const float*)y)[i] : 0.0f;
  else ylab[i] = i < n ? ((const int32_t*)y)[i] : 0;
}

template <typename T>
__global__ void fill_ones_rows_kernel(T* a, int J, int H, int64_t ldm, int64_t ncols) {
  // set row H of every particle's [(H+1) x ldm] block to ones
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)J * ncols) return;
  const int j = (int)(i / ncols);
  const int64_t c = i - (int64_t)j * ncols;
  a[((int64_t)j * (H + 1) + H) * ldm + c] = cvt_out<T>(1.0f);
}

// W_l^T copy for layers >= 2: wT[j][i][o] = W_l[j][o][i], tiled through LDS
template <typename T>
__global__ void transpose_w_kernel(const float* theta, int64_t D, int64_t off, int nout, int nin, int ldwT, T* wT) {
  __shared__ float tile[32][33];
  const int j = blockIdx.z;
  const int o0 = blockIdx.y * 32, i0 = blockIdx.x * 32;
  const float* src = theta + (int64_t)j * D + off;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int o = o0 + r, i = i0 + threadIdx.x;
    tile[r][threadIdx.x] = (o < nout && i < nin) ? src[(int64_t)o * (nin + 1) + i] : 0.0f;
  }
  __syncthreads();
  T* dst = wT + (int64_t)j * nin * ldwT;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = i0 + r, o = o0 + threadIdx.x;
    if (i < nin && o < nout) dst[(int64_t)i * ldwT + o] = cvt_out<T>(tile[threadIdx.x][r]);
  }
}

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};

struct LayerBufs {
  void* act = nullptr;   // [J x mc x nout] (hidden layers)
  void* actT = nullptr;  // [J x (nout+1) x mc] (hidden layers feeding another hidden layer)
  void* dT = nullptr;    // [J*nout x mc]
  void* dR = nullptr;    // [J x mc x nout] (hidden layers >= 2)
  void* wT = nullptr;    // [J x nin x ldwT] (layers >= 2 that are not the output layer)
  int ldwT = 0;
};

// convolutional network: per-chunk operand buffers (element strides per particle)
struct CnnBufs {
  CnnDims d;
  void *p1 = nullptr, *p1t = nullptr;           // [RP x K1p], [(K1+1) x RP] image patches (shared)
  void *act1 = nullptr, *big = nullptr;         // [J][RP][C1], [J][RP*(K2+1)] conv2 patches / errors
  void *act2 = nullptr, *pooled = nullptr;      // [J][RP][C2], [J][mc][F3]
  void *d3 = nullptr, *dpool = nullptr;         // [J][mc][16], [J][mc][F3]
  void *d2 = nullptr, *d2t = nullptr;           // [J][RP][C2], [J][C2][RP]
  void* d1t = nullptr;                          // [J*C1][RP]
  float* dw1part = nullptr;                     // [kslices][J*C1][K1+1] split-K partials of the conv1 gradient
  float* dw2part = nullptr;                     // [J][groups][4][C2 x (K2+1)] partials of the implicit conv2 gradient
  int implicit = 0;                             // conv2 runs as implicit GEMMs (no patch matrices)
  int kslices = 1;                              // their capacity
  float* logits = nullptr;                      // [J][mc][ncls]
  void* wT[3] = {nullptr, nullptr, nullptr};    // transposed copies of layers 1, 2: [J][nin][ldwT]
  int ldwT[3] = {0, 0, 0};
  int64_t RP = 0, s_act1 = 0, s_big = 0, s_act2 = 0, s_pool = 0;
};

}  // namespace

struct smc_handle {
  smc_config cfg{};
  hipStream_t stream = nullptr;
  std::vector<void*> owned;
  int J = 0, L = 0, F = 0, C = 0, bf16 = 0, split = 0, cnn = 0;
  int fused = 0;  // one hidden layer, BF16 operands: layer 1 and the output layer in one kernel
  // the current pass's log-likelihood enters no weight (it only supplies a gradient): split-BF16
  // networks run its forward on the hi operands alone
  bool grad_only = false;
  CnnBufs cb;
  // LeNet-5: a convolution stack (lenet.hip) whose F features feed the dense layers in place
  // of X; per chunk lfeat [J][mc][F], lfeatT [J][(F+1)][mc] (ones row F), ldfeat [J][mc][F]
  // and the conv-gradient partials lpart [J][lpart_blocks][Dconv]
  int lenet = 0;
  LenetDims ld;
  float *lfeat = nullptr, *lfeatT = nullptr, *ldfeat = nullptr, *lpart = nullptr;
  float* lmaps = nullptr;  // [J][mc][Mimg]: each image's conv2 activations from the forward, for the backward
  int lpart_blocks = 0;  // capacity of the partials per particle
  int lbwd_blocks = 0;   // image blocks per particle of the backward: one round of resident workgroups
  int64_t D = 0;
  int64_t n_data = 0, n_pad = 0;
  int ldx = 0;  // padded feature count
  int xld = 0;  // row stride of the X operand (2 ldx with split BF16)
  size_t esz = 4;  // operand element size
  NetShape net;
  LayerBufs lb[MAX_LAYERS];
  void* X = nullptr;
  void* XT = nullptr;
  int32_t* ylab = nullptr;
  float* yreal = nullptr;
  float *theta = nullptr, *g = nullptr, *P = nullptr;
  double *ll = nullptr, *lp = nullptr, *logw = nullptr, *w = nullptr, *stats = nullptr, *part = nullptr;
  double* tsq = nullptr;
  double* extra = nullptr;
  int32_t *anc = nullptr, *place = nullptr;
  int nblk = 0;
  int64_t mc = 0;
  int nsplit_max = 0;
  double* llpart = nullptr;
  float* dWpart = nullptr;
  float* noise = nullptr;
  bool noise_pending = false;
  bool w_dirty = true;
  int64_t m = 0;
  double lam = 1.0;
  // two-segment target (smooth data annealing): samples from seg_split on weigh lam_b;
  // INT64_MAX: one segment.  ll_b holds the second segment's log-likelihood at the
  // current particles (zero with one segment).
  int64_t seg_split = INT64_MAX;
  double lam_b = 1.0;
  double* ll_b = nullptr;
  double* llpart_b = nullptr;
  uint64_t rng_iter = 0;
  int64_t grad_evals = 0;
  // learned proposal
  float* pnet = nullptr;
  int pnet_n = 0;
  double h0 = 0.0;
  int G = 0, NO = 0;
  int64_t* group_n = nullptr;   // device [G]: parameters per group
  float *sc0 = nullptr, *sc1 = nullptr;
  double* feat = nullptr;       // [J x 4]
  double* gsum = nullptr;       // [J x G]
  int64_t k_iter = 0;           // smc_step calls since init
  // trace-target scratch
  float *th_bak = nullptr, *g_bak = nullptr;
  double *ll_bak = nullptr, *ll1 = nullptr, *phalf = nullptr, *best_score = nullptr, *best_logh = nullptr,
         *lp0 = nullptr;
  // posterior-mean change criterion: the mean of the previous call
  double *pm_prev = nullptr, *pm_cur = nullptr, *pm_out = nullptr;
  bool pm_have = false;
  // posterior predictive scratch (grown on demand)
  void* tx = nullptr;
  int64_t tx_rows = 0;
  float* logp = nullptr;
  int64_t logp_n = 0;
  double* per_sample = nullptr;
  double* pred_out = nullptr;
  // kernel timing (smc_profile)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_pool;
  std::vector<ProfRec> prof_recs;
};

namespace {

void sync(smc_t h) { HIPCHECK(hipStreamSynchronize(h->stream)); }

hipEvent_t prof_event(smc_t h) {
  if (!h->prof_pool.empty()) {
    hipEvent_t e = h->prof_pool.back();
    h->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHECK(hipEventCreate(&e));
  return e;
}

// Run `launch` bracketed by events on the handle's stream when profiling is on.
template <typename F>
void timed(smc_t h, int cls, double flops, double bytes, F&& launch) {
  if (!h->prof_on) {
    launch();
    return;
  }
  ProfRec r{cls, prof_event(h), prof_event(h), flops, bytes};
  HIPCHECK(hipEventRecord(r.a, h->stream));
  launch();
  HIPCHECK(hipEventRecord(r.b, h->stream));
  h->prof_recs.push_back(r);
}

uint32_t key0(smc_t h) { return (uint32_t)(h->cfg.seed & 0xffffffffu); }
uint32_t key1(smc_t h) { return (uint32_t)(h->cfg.seed >> 32); }

int head_type(int precision) {
  return precision == SMC_PREC_BF16X3 ? HEAD_BF16_SPLIT : precision == SMC_PREC_BF16 ? HEAD_BF16 : HEAD_F32;
}

LenetDims lenet_dims(const int32_t* w) {
  LenetDims d;
  d.H = w[0], d.W = w[1], d.Cin = w[2], d.k = w[3], d.C1 = w[4], d.C2 = w[5];
  d.pad = (d.k - 1) / 2;
  d.Hp = d.H / 2, d.Wp = d.W / 2;
  d.H2 = d.Hp - d.k + 1, d.W2 = d.Wp - d.k + 1;
  d.Hq = d.H2 / 2, d.Wq = d.W2 / 2;
  d.K1 = d.k * d.k * d.Cin, d.K2 = d.k * d.k * d.C1;
  d.F = d.Hq * d.Wq * d.C2;
  d.Dconv = d.C1 * (d.K1 + 1) + d.C2 * (d.K2 + 1);
  // conv1 weight-gradient items (channel pair, input channel, kernel row) replicated over
  // slices of the image rows to fill 256 threads
  d.ns1 = std::max(1, 256 / (((d.C1 + 1) / 2) * d.Cin * d.k));
  d.Mimg = d.C2 * d.H2 * d.W2;
  return d;
}

void check_lenet(const smc_config* c) {
  const int* w = c->widths;
  if (c->n_layers != 5) fail(SMC_ERR_ARG, "LeNet has n_layers = 5 (widths H, W, Cin, k, C1, C2, F1, F2, n_cls)");
  for (int q = 0; q < 9; ++q)
    if (w[q] < 1) fail(SMC_ERR_ARG, "every LeNet dimension must be >= 1");
  if (w[3] != 3 && w[3] != 5) fail(SMC_ERR_UNSUPPORTED, "LeNet kernel size must be 3 or 5");
  if (w[0] % 2 || w[1] % 2 || w[0] > 512 || w[1] > 512) fail(SMC_ERR_UNSUPPORTED, "H and W must be even and at most 512");
  const LenetDims d = lenet_dims(w);
  if (d.H2 < 2 || d.W2 < 2 || d.H2 % 2 || d.W2 % 2)
    fail(SMC_ERR_UNSUPPORTED, "the second convolution's output (H/2 - k + 1, W/2 - k + 1) must be even and >= 2");
  if (d.Cin > LENET_CMAX || d.C1 > LENET_CMAX) fail(SMC_ERR_UNSUPPORTED, "LeNet Cin and C1 must be at most 8");
  if ((d.C2 + 1) / 2 * d.C1 * d.k > 256) fail(SMC_ERR_UNSUPPORTED, "LeNet needs ceil(C2/2) C1 k <= 256");
  if (d.F % 4 || w[6] % 4 || w[7] % 4) fail(SMC_ERR_UNSUPPORTED, "LeNet F, F1 and F2 must be multiples of 4");
  if (lenet_smem_bytes(d, true) > 65536) fail(SMC_ERR_UNSUPPORTED, "LeNet image too large for the convolution kernels");
  if (w[8] < 2 || w[8] > 16) fail(SMC_ERR_UNSUPPORTED, "categorical likelihood needs 2..16 classes");
  if (c->activation != SMC_ACT_TANH && c->activation != SMC_ACT_RELU) fail(SMC_ERR_ARG, "activation");
  if (c->likelihood != SMC_LIK_CATEGORICAL) fail(SMC_ERR_UNSUPPORTED, "LeNet is a classifier");
  if (c->precision != SMC_PREC_FP32) fail(SMC_ERR_UNSUPPORTED, "LeNet runs with FP32 operands");
  if (c->proposal != SMC_PROPOSAL_FIXED) fail(SMC_ERR_UNSUPPORTED, "LeNet uses the fixed proposal");
  if (c->leapfrog_steps < 1) fail(SMC_ERR_ARG, "leapfrog_steps must be >= 1");
  if (!(c->step_size >= 0) || !isfinite(c->step_size)) fail(SMC_ERR_ARG, "step_size must be finite and >= 0");
  if (!(c->prior_std > 0)) fail(SMC_ERR_ARG, "prior_std must be > 0");
  if (!(c->ess_frac >= 0 && c->ess_frac <= 1)) fail(SMC_ERR_ARG, "ess_frac must be in [0, 1]");
  if (c->act_budget_bytes < 0) fail(SMC_ERR_ARG, "act_budget_bytes must be >= 0");
  if (!head_supported(w[7], w[8], HEAD_F32)) fail(SMC_ERR_UNSUPPORTED, "F2 too wide for the output-layer kernel");
}

void check_config(const smc_config* c) {
  if (!c) fail(SMC_ERR_ARG, "null config");
  if (c->n_particles < 1 || c->n_particles > MAX_J)
    fail(SMC_ERR_ARG, "n_particles must be in [1, " + std::to_string(MAX_J) + "]");
  if (c->model_kind == SMC_MODEL_CNN) {
    const int* w = c->widths;
    if (c->n_layers != 3) fail(SMC_ERR_ARG, "the convolutional network has n_layers = 3 (widths H, W, Cin, C1, C2, n_cls)");
    for (int q = 0; q < 6; ++q)
      if (w[q] < 1) fail(SMC_ERR_ARG, "every CNN dimension must be >= 1");
    if (w[0] % 2 || w[1] % 2 || (w[0] * w[1]) % 8) fail(SMC_ERR_UNSUPPORTED, "H and W must be even with H*W a multiple of 8");
    if (w[3] % 8 || w[4] % 8) fail(SMC_ERR_UNSUPPORTED, "C1 and C2 must be multiples of 8");
    if ((int64_t)w[0] * w[1] * w[2] > (1 << 20) || w[3] > 256 || w[4] > 256) fail(SMC_ERR_UNSUPPORTED, "CNN too large");
    if (w[5] < 2 || w[5] > 16) fail(SMC_ERR_UNSUPPORTED, "categorical likelihood needs 2..16 classes");
    if (c->activation != SMC_ACT_RELU) fail(SMC_ERR_UNSUPPORTED, "the convolutional network uses ReLU");
    if (c->likelihood != SMC_LIK_CATEGORICAL) fail(SMC_ERR_UNSUPPORTED, "the convolutional network is a classifier");
    if (c->precision == SMC_PREC_BF16X3) fail(SMC_ERR_UNSUPPORTED, "split BF16 is not built for the convolutional network");
  } else if (c->model_kind == SMC_MODEL_LENET) {
    check_lenet(c);
    return;
  } else if (c->model_kind != SMC_MODEL_MLP) {
    fail(SMC_ERR_ARG, "model_kind");
  }
  if (c->n_layers < 1 || c->n_layers > SMC_MAX_LAYERS) fail(SMC_ERR_ARG, "n_layers must be in [1, 8]");
  if (c->model_kind == SMC_MODEL_MLP)
    for (int l = 0; l <= c->n_layers; ++l)
      if (c->widths[l] < 1) fail(SMC_ERR_ARG, "every width must be >= 1");
  if (c->activation != SMC_ACT_TANH && c->activation != SMC_ACT_RELU) fail(SMC_ERR_ARG, "activation");
  if (c->model_kind == SMC_MODEL_CNN) {
    // checked above
  } else if (c->likelihood == SMC_LIK_CATEGORICAL) {
    if (c->widths[c->n_layers] < 2 || c->widths[c->n_layers] > 16)
      fail(SMC_ERR_UNSUPPORTED, "categorical likelihood needs 2..16 classes");
  } else if (c->likelihood == SMC_LIK_GAUSSIAN) {
    if (c->widths[c->n_layers] != 1) fail(SMC_ERR_ARG, "Gaussian likelihood needs one output");
    if (!(c->noise_std > 0)) fail(SMC_ERR_ARG, "noise_std must be > 0");
  } else {
    fail(SMC_ERR_ARG, "likelihood");
  }
  if (c->precision != SMC_PREC_FP32 && c->precision != SMC_PREC_BF16 && c->precision != SMC_PREC_BF16X3)
    fail(SMC_ERR_ARG, "precision");
  if (c->precision == SMC_PREC_BF16X3 && c->n_layers > 2)
    fail(SMC_ERR_UNSUPPORTED, "split BF16 supports at most one hidden layer");
  if (c->proposal != SMC_PROPOSAL_FIXED && c->proposal != SMC_PROPOSAL_LEARNED) fail(SMC_ERR_ARG, "proposal");
  if (c->proposal == SMC_PROPOSAL_LEARNED && c->leapfrog_steps != 1)
    fail(SMC_ERR_UNSUPPORTED, "the learned proposal is a Langevin (S = 1) move");
  if (c->leapfrog_steps < 1) fail(SMC_ERR_ARG, "leapfrog_steps must be >= 1");
  if (!(c->step_size >= 0) || !isfinite(c->step_size)) fail(SMC_ERR_ARG, "step_size must be finite and >= 0");
  if (!(c->prior_std > 0)) fail(SMC_ERR_ARG, "prior_std must be > 0");
  if (!(c->ess_frac >= 0 && c->ess_frac <= 1)) fail(SMC_ERR_ARG, "ess_frac must be in [0, 1]");
  if (c->act_budget_bytes < 0) fail(SMC_ERR_ARG, "act_budget_bytes must be >= 0");
  if (c->model_kind == SMC_MODEL_CNN) return;
  // hidden layers that feed another GEMM layer use 16-byte aligned per-particle rows
  if (c->n_layers >= 3)
    for (int l = 1; l < c->n_layers; ++l)
      if (c->widths[l] % 8) fail(SMC_ERR_UNSUPPORTED, "with two or more hidden layers every hidden width must be a multiple of 8");
  const int H = c->widths[c->n_layers - 1], C = c->widths[c->n_layers];
  if (!head_supported(H, C, head_type(c->precision)))
    fail(SMC_ERR_UNSUPPORTED, "last hidden layer too wide for the output-layer kernel (at most 495 units)");
}

void setup_shapes(smc_t h) {
  const smc_config& c = h->cfg;
  h->J = c.n_particles;
  h->L = c.n_layers;
  h->F = c.widths[0];
  h->C = c.widths[c.n_layers];
  h->cnn = c.model_kind == SMC_MODEL_CNN;
  h->lenet = c.model_kind == SMC_MODEL_LENET;
  int cnn_in[3] = {0, 0, 0}, cnn_out[3] = {0, 0, 0};
  int64_t off = 0;
  if (h->lenet) {
    // the dense layers F -> F1 -> F2 -> n_cls after the convolution blocks
    h->ld = lenet_dims(c.widths);
    const LenetDims& d = h->ld;
    h->L = 3;
    h->F = d.H * d.W * d.Cin;  // the X operand holds the images
    h->C = c.widths[8];
    cnn_in[0] = d.F, cnn_in[1] = c.widths[6], cnn_in[2] = c.widths[7];
    cnn_out[0] = c.widths[6], cnn_out[1] = c.widths[7], cnn_out[2] = c.widths[8];
    off = d.Dconv;
  }
  if (h->cnn) {
    CnnDims& d = h->cb.d;
    d.H = c.widths[0];
    d.W = c.widths[1];
    d.Cin = c.widths[2];
    d.C1 = c.widths[3];
    d.C2 = c.widths[4];
    d.ncls = c.widths[5];
    d.Hp = d.H / 2;
    d.Wp = d.W / 2;
    d.HW = d.H * d.W;
    d.K1 = 9 * d.Cin;
    d.K1p = (int)round_up(d.K1, 8);
    d.K2 = 9 * d.C1;
    d.F3 = d.Hp * d.Wp * d.C2;
    h->F = d.HW * d.Cin;
    h->C = d.ncls;
    cnn_in[0] = d.K1, cnn_in[1] = d.K2, cnn_in[2] = d.F3;
    cnn_out[0] = d.C1, cnn_out[1] = d.C2, cnn_out[2] = d.ncls;
  }
  h->bf16 = c.precision != SMC_PREC_FP32;
  h->split = c.precision == SMC_PREC_BF16X3;
  h->esz = h->bf16 ? 2 : 4;
  NetShape& n = h->net;
  n.L = h->L;
  n.J = h->J;
  n.bf16 = h->bf16;
  n.split = h->split;
  for (int l = 0; l < h->L; ++l) {
    n.nin[l] = h->cnn || h->lenet ? cnn_in[l] : c.widths[l];
    n.nout[l] = h->cnn || h->lenet ? cnn_out[l] : c.widths[l + 1];
    n.off[l] = off;
    n.ldw[l] = (int)round_up(n.nin[l], 8);
    n.rowpad[l] = n.nout[l];
    n.rinv[l] = 1.0f / (float)(n.nin[l] + 1);
    off += (int64_t)n.nout[l] * (n.nin[l] + 1);
  }
  n.off[h->L] = off;
  n.D = off;
  h->D = off;
  if (h->D > (1 << 24)) fail(SMC_ERR_UNSUPPORTED, "more than 2^24 parameters per particle");
  h->ldx = (int)round_up(h->F, 8);
  h->xld = h->split ? 2 * h->ldx : h->ldx;
  h->fused = !h->cnn && h->L == 2 && h->bf16 && fwd_head_supported(n.nin[1], h->C);
  if (h->fused) n.rowpad[0] = 128;  // one 128-row tile per particle
  h->nblk = (int)((h->D + MOVE_ELEMS - 1) / MOVE_ELEMS);
}

// samples per chunk from the activation budget
int64_t choose_chunk(smc_t h) {
  int64_t budget = h->cfg.act_budget_bytes > 0 ? h->cfg.act_budget_bytes : ((int64_t)8 << 30);
  if (h->cnn) {
    // images per chunk from the bytes one image occupies across all particles
    const CnnDims& d = h->cb.d;
    const int64_t J = h->J, e = (int64_t)h->esz;
    // explicit conv2 only: the patch matrix and the conv2 output error in both layouts
    const bool impl = cnn_implicit_supported(d, h->bf16);
    const int64_t patches = impl ? 0 : d.K2 + 1, c2bufs = impl ? 1 : 3;
    const int64_t per_image = J * d.HW * (int64_t)(2 * d.C1 + patches + c2bufs * d.C2) * e +
                              J * (int64_t)(2 * d.F3 + 16) * e + J * d.ncls * 4 +
                              (int64_t)d.HW * (d.K1p + d.K1 + 1) * e;
    int64_t mc = std::max<int64_t>(1, budget / per_image);
    return std::min<int64_t>(std::min<int64_t>(mc, 1024), h->n_data);
  }
  int64_t per_sample = 0;  // bytes of activation buffers per sample
  for (int l = 0; l < h->L - 1; ++l) {
    const int64_t u = (int64_t)h->J * h->net.nout[l];
    per_sample += u * h->esz * (h->fused ? 1 : (h->split ? 3 : 2));  // dT (+ act: FP32 for split)
    if (l >= 1) per_sample += u * h->esz;                          // dR
    if (l + 1 < h->L - 1) per_sample += (int64_t)h->J * (h->net.nout[l] + 1) * h->esz;  // actT
  }
  if (h->lenet)  // features, their transpose and their error; the first dense layer's dR; the saved maps
    per_sample += (int64_t)h->J * (3 * h->ld.F + 1 + h->net.nout[0] + h->ld.Mimg) * 4;
  if (per_sample == 0) per_sample = 1;
  int64_t mc = budget / per_sample;
  mc = mc / 256 * 256;
  if (mc < 256) mc = 256;
  const int64_t cap = round_up(h->n_data, 256);
  return std::min(mc, cap);
}

void alloc_cnn(smc_t h) {
  CnnBufs& b = h->cb;
  const CnnDims& d = b.d;
  const int64_t J = h->J, mc = h->mc, e = (int64_t)h->esz;
  b.RP = mc * d.HW;
  b.s_act1 = b.RP * d.C1;
  b.s_big = b.RP * (d.K2 + 1);
  b.s_act2 = b.RP * d.C2;
  b.s_pool = mc * d.F3;
  b.p1 = dalloc<char>(h->owned, b.RP * d.K1p * e);
  b.p1t = dalloc<char>(h->owned, b.RP * (d.K1 + 1) * e);
  b.act1 = dalloc<char>(h->owned, J * b.s_act1 * e);
  b.implicit = cnn_implicit_supported(d, h->bf16) ? 1 : 0;
  if (b.implicit)
    b.dw2part = dalloc<float>(h->owned, J * CNN_WGRAD_GROUPS * 4 * d.C2 * (int64_t)(d.K2 + 1));
  else
    b.big = dalloc<char>(h->owned, J * b.s_big * e);
  b.act2 = dalloc<char>(h->owned, J * b.s_act2 * e);
  b.pooled = dalloc<char>(h->owned, J * b.s_pool * e);
  b.d3 = dalloc<char>(h->owned, J * mc * 16 * e);
  b.dpool = dalloc<char>(h->owned, J * b.s_pool * e);
  if (!b.implicit) {
    b.d2 = dalloc<char>(h->owned, J * b.s_act2 * e);
    b.d2t = dalloc<char>(h->owned, J * b.s_act2 * e);
  }
  b.d1t = dalloc<char>(h->owned, J * b.s_act1 * e);
  b.logits = dalloc<float>(h->owned, J * mc * d.ncls);
  // the conv1 weight gradient is one GEMM with J*C1 output rows over all pixels of the chunk:
  // it runs as up to 64 K-slices into FP32 partials (at most 256 MB) summed in a fixed order
  const int64_t out1 = J * d.C1 * (d.K1 + 1);
  b.kslices = (int)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)256 << 20) / (out1 * 4)));
  if (b.kslices > 1) b.dw1part = dalloc<float>(h->owned, b.kslices * out1);
  for (int l = 1; l < 3; ++l) {
    b.ldwT[l] = (int)round_up(h->net.nout[l], 8);
    const int64_t n = J * h->net.nin[l] * b.ldwT[l] * e;
    b.wT[l] = dalloc<char>(h->owned, n);
    HIPCHECK(hipMemsetAsync(b.wT[l], 0, (size_t)n, h->stream));  // padded output columns stay zero
  }
}

void alloc_all(smc_t h) {
  const int J = h->J;
  const int64_t D = h->D;
  h->n_pad = round_up(h->n_data, 256);
  h->X = dalloc<char>(h->owned, h->n_pad * h->xld * (int64_t)h->esz);
  if (!h->cnn && !h->lenet) h->XT = dalloc<char>(h->owned, (int64_t)(h->F + 1) * h->n_pad * (int64_t)h->esz);
  if (h->cfg.likelihood == SMC_LIK_GAUSSIAN) h->yreal = dalloc<float>(h->owned, h->n_pad);
  else h->ylab = dalloc<int32_t>(h->owned, h->n_pad);
  h->theta = dalloc<float>(h->owned, (int64_t)J * D);
  h->g = dalloc<float>(h->owned, (int64_t)J * D);
  h->P = dalloc<float>(h->owned, (int64_t)J * D);
  h->ll = dalloc<double>(h->owned, J);
  h->ll_b = dalloc<double>(h->owned, J);
  h->lp = dalloc<double>(h->owned, J);
  h->logw = dalloc<double>(h->owned, J);
  h->w = dalloc<double>(h->owned, J);
  h->tsq = dalloc<double>(h->owned, J);
  h->extra = dalloc<double>(h->owned, J);
  h->stats = dalloc<double>(h->owned, 16);
  h->part = dalloc<double>(h->owned, (int64_t)3 * J * h->nblk);
  h->anc = dalloc<int32_t>(h->owned, J);
  h->place = dalloc<int32_t>(h->owned, J);
  HIPCHECK(hipMemsetAsync(h->stats, 0, 16 * sizeof(double), h->stream));
  HIPCHECK(hipMemsetAsync(h->ll_b, 0, (size_t)J * sizeof(double), h->stream));
  HIPCHECK(hipMemsetAsync(h->part, 0, (size_t)3 * J * h->nblk * sizeof(double), h->stream));
  for (int l = 0; l < h->L; ++l) {
    const int64_t n = (int64_t)J * h->net.rowpad[l] * h->net.ldw[l] * (int64_t)h->esz * (h->split ? 2 : 1);
    h->net.w[l] = dalloc<char>(h->owned, n);
    HIPCHECK(hipMemsetAsync(h->net.w[l], 0, (size_t)n, h->stream));  // row padding stays zero
    h->net.bias[l] = dalloc<float>(h->owned, (int64_t)J * h->net.nout[l]);
  }
  h->mc = choose_chunk(h);
  const int64_t mc = h->mc;
  if (h->cnn) {
    alloc_cnn(h);
    return;
  }
  for (int l = 0; l < h->L - 1; ++l) {
    const int64_t u = (int64_t)J * h->net.nout[l];
    LayerBufs& b = h->lb[l];
    if (!h->fused) b.act = dalloc<char>(h->owned, mc * u * (int64_t)h->esz * (h->split ? 2 : 1));
    b.dT = dalloc<char>(h->owned, mc * u * (int64_t)h->esz);
    if (l >= 1 || h->lenet) b.dR = dalloc<char>(h->owned, mc * u * (int64_t)h->esz);
    if (l + 1 < h->L - 1) {
      const int64_t nc = (int64_t)J * (h->net.nout[l] + 1);
      b.actT = dalloc<char>(h->owned, nc * mc * (int64_t)h->esz);
      const int64_t tot = (int64_t)J * mc;
      if (h->bf16)
        hipLaunchKernelGGL(fill_ones_rows_kernel<__bf16>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                           (__bf16*)b.actT, J, h->net.nout[l], mc, mc);
      else
        hipLaunchKernelGGL(fill_ones_rows_kernel<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                           (float*)b.actT, J, h->net.nout[l], mc, mc);
      HIPCHECK(hipGetLastError());
    }
  }
  for (int l = h->lenet ? 0 : 1; l < h->L - 1; ++l) {
    LayerBufs& b = h->lb[l];
    b.ldwT = (int)round_up(h->net.nout[l], 8);
    const int64_t n = (int64_t)J * h->net.nin[l] * b.ldwT * (int64_t)h->esz;
    b.wT = dalloc<char>(h->owned, n);
    HIPCHECK(hipMemsetAsync(b.wT, 0, (size_t)n, h->stream));
  }
  if (h->lenet) {
    const int F = h->ld.F;
    h->lfeat = dalloc<float>(h->owned, (int64_t)J * mc * F);
    h->lfeatT = dalloc<float>(h->owned, (int64_t)J * (F + 1) * mc);
    h->ldfeat = dalloc<float>(h->owned, (int64_t)J * mc * F);
    h->lmaps = dalloc<float>(h->owned, (int64_t)J * mc * h->ld.Mimg);
    h->lpart_blocks = (int)std::min<int64_t>(64, mc);
    const int resident = lenet_bwd_resident(h->ld, h->cfg.activation);
    h->lbwd_blocks = std::max(1, std::min(h->lpart_blocks, resident > 0 ? resident / J : h->lpart_blocks));
    h->lpart = dalloc<float>(h->owned, (int64_t)J * h->lpart_blocks * h->ld.Dconv);
    const int64_t tot = (int64_t)J * mc;
    hipLaunchKernelGGL(fill_ones_rows_kernel<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                       h->lfeatT, J, F, mc, mc);
    HIPCHECK(hipGetLastError());
  }
  const int ntiles = (int)(mc / 64);
  h->nsplit_max = std::max(1, std::min(ntiles, (2048 + J - 1) / J));
  if (h->fused) h->nsplit_max = std::max(h->nsplit_max, (int)((mc + 255) / 256));  // one partial per 256 samples
  const int H = h->net.nin[h->L - 1];
  h->llpart = dalloc<double>(h->owned, (int64_t)J * h->nsplit_max);
  h->llpart_b = dalloc<double>(h->owned, (int64_t)J * h->nsplit_max);
  h->dWpart = dalloc<float>(h->owned, (int64_t)J * h->nsplit_max * h->C * (H + 1));
}

void upload_data(smc_t h, const float* x, const void* y) {
  const int64_t nx = h->n_pad * h->ldx;
  const int64_t nt = (int64_t)(h->F + 1) * h->n_pad;
  if (h->bf16) {
    hipLaunchKernelGGL(pack_x_kernel<__bf16>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream, x,
                       h->n_data, h->F, h->ldx, h->split ? 2 : 1, h->n_pad, (__bf16*)h->X);
    if (h->XT)
      hipLaunchKernelGGL(pack_xt_kernel<__bf16>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, h->stream, x,
                         h->n_data, h->F, h->n_pad, (__bf16*)h->XT);
  } else {
    hipLaunchKernelGGL(pack_x_kernel<float>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream, x,
                       h->n_data, h->F, h->ldx, 1, h->n_pad, (float*)h->X);
    if (h->XT)
      hipLaunchKernelGGL(pack_xt_kernel<float>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, h->stream, x,
                         h->n_data, h->F, h->n_pad, (float*)h->XT);
  }
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(pack_labels_kernel, dim3((unsigned)((h->n_pad + 255) / 256)), dim3(256), 0, h->stream, y,
                     h->n_data, h->n_pad, h->cfg.likelihood == SMC_LIK_GAUSSIAN ? 1 : 0, h->ylab, h->yreal);
  HIPCHECK(hipGetLastError());
}

void transpose_weights(smc_t h, const float* theta) {
  const int l0 = h->lenet ? 0 : 1, l1 = h->cnn ? 3 : h->L - 1;
  for (int l = l0; l < l1; ++l) {
    LayerBufs cbuf;
    if (h->cnn) {
      cbuf.wT = h->cb.wT[l];
      cbuf.ldwT = h->cb.ldwT[l];
    }
    const LayerBufs& b = h->cnn ? cbuf : h->lb[l];
    const int nout = h->net.nout[l], nin = h->net.nin[l];
    dim3 grid((nin + 31) / 32, (nout + 31) / 32, h->J);
    if (h->bf16)
      hipLaunchKernelGGL(transpose_w_kernel<__bf16>, grid, dim3(32, 8), 0, h->stream, theta, h->D, h->net.off[l], nout,
                         nin, b.ldwT, (__bf16*)b.wT);
    else
      hipLaunchKernelGGL(transpose_w_kernel<float>, grid, dim3(32, 8), 0, h->stream, theta, h->D, h->net.off[l], nout,
                         nin, b.ldwT, (float*)b.wT);
    HIPCHECK(hipGetLastError());
  }
}

void gemm(smc_t h, const GemmParams& p, int cls, double flops) {
  timed(h, cls, flops, 0.0, [&]() {
    const hipError_t e = gemm_run(p, h->bf16 ? GEMM_BF16 : GEMM_F32, h->stream);
    if (e != hipSuccess) fail(SMC_ERR_DEVICE, std::string("GEMM launch failed: ") + hipGetErrorString(e));
  });
}

// LeNet: features of images [c0, c0 + mcv) of the operand Xop (rows up to `rows` zeroed),
// and, when with_t (a gradient pass), their transpose for the first dense layer's weight
// gradient and the activation maps for the backward.
double lenet_macs_per_image(const LenetDims& d) {
  return (double)d.H * d.W * d.C1 * d.K1 + (double)d.H2 * d.W2 * d.C2 * d.K2;
}
// backward: the conv1 and conv2 weight gradients and the conv2 input error
double lenet_bwd_macs_per_image(const LenetDims& d) {
  return (double)d.H * d.W * d.C1 * d.K1 + 2.0 * d.H2 * d.W2 * d.C2 * d.K2;
}

void lenet_features(smc_t h, const float* theta, const void* Xop, int64_t c0, int mcv, int rows, bool with_t) {
  const int J = h->J;
  const int ipb = (int)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)rows * J / 4096));
  timed(h, SMC_K_OTHER, 2.0 * J * mcv * lenet_macs_per_image(h->ld), 0.0, [&]() {
    HIPCHECK(lenet_fwd_run((const float*)Xop, h->xld, c0, mcv, rows, ipb, h->ld, theta, h->D, J, h->cfg.activation,
                           h->lfeat, h->mc * h->ld.F, with_t ? h->lfeatT : nullptr, h->mc,
                           with_t ? h->lmaps : nullptr, h->mc * h->ld.Mimg, h->stream));
  });
}

// Forward through the hidden layers for samples [c0, c0 + rows) of the operand X
// (xld-strided rows).  Writes act_l (and actT_l when a hidden layer follows).
void forward_hidden(smc_t h, const void* Xop, int64_t c0, int rows, int m_valid) {
  const int J = h->J;
  for (int l = 0; l < h->L - 1; ++l) {
    const int nout = h->net.nout[l];
    const int64_t U = (int64_t)J * nout;
    GemmParams p;
    p.epi = EPI_FWD;
    p.act = h->cfg.activation;
    p.M = rows;
    p.K = h->net.ldw[l];
    if (l == 0 && h->lenet) {
      // batched over particles: particle j's features from the convolution stack
      const int F = h->ld.F;
      p.A = h->lfeat;
      p.lda = F;
      p.sAb = h->mc * F;
      p.B = h->net.w[0];
      p.ldb = h->net.ldw[0];
      p.sBb = (int64_t)h->net.rowpad[0] * h->net.ldw[0];
      p.K = F;
      p.N = nout;
      p.batch = J;
      p.bias = h->net.bias[0];
      p.sbias = nout;
      p.out0.ptr = h->lb[0].act;
      p.out0.sb = h->mc * nout;
      p.out0.rstr = nout;
      if (h->lb[0].actT) {
        p.out1.ptr = h->lb[0].actT;
        p.out1.sb = (int64_t)(nout + 1) * h->mc;
        p.out1.cstr = h->mc;
        p.out1.rstr = 1;
      }
    } else if (l == 0) {
      // one dense GEMM over the concatenation of all particles' units
      p.A = (const char*)Xop + c0 * h->xld * (int64_t)h->esz;
      p.lda = h->xld;
      p.B = h->net.w[0];
      p.ldb = h->net.ldw[0] * (h->split ? 2 : 1);
      if (h->split) {
        p.K = 2 * h->net.ldw[0];  // [x | x] . [w_hi | w_lo]
        p.out_f32 = 1;            // FP32 activations for the output layer's hi/lo split
      }
      p.N = (int)U;
      p.batch = 1;
      p.bias = h->net.bias[0];
      p.out0.ptr = h->lb[0].act;
      p.out0.rstr = nout;
      p.out0.cs = nout;
      p.out0.sC = h->mc * nout;
      if (h->lb[0].actT) {
        p.out1.ptr = h->lb[0].actT;
        p.out1.cs = nout;
        p.out1.sC = (int64_t)(nout + 1) * h->mc;
        p.out1.cstr = h->mc;
        p.out1.rstr = 1;
      }
    } else {
      // batched over particles: A_{l-1}[j] is particle j's [samples x units] block
      const int nin = h->net.nin[l];
      p.A = h->lb[l - 1].act;
      p.lda = nin;
      p.sAb = h->mc * nin;
      p.B = h->net.w[l];
      p.ldb = h->net.ldw[l];
      p.sBb = (int64_t)nout * h->net.ldw[l];
      p.K = nin;
      p.N = nout;
      p.batch = J;
      p.bias = h->net.bias[l];
      p.sbias = nout;
      p.out0.ptr = h->lb[l].act;
      p.out0.sb = h->mc * nout;
      p.out0.rstr = nout;
      if (h->lb[l].actT) {
        p.out1.ptr = h->lb[l].actT;
        p.out1.sb = (int64_t)(nout + 1) * h->mc;
        p.out1.cstr = h->mc;
        p.out1.rstr = 1;
      }
    }
    const double fl = 2.0 * m_valid * (double)U * (l == 0 && !h->lenet ? h->F : h->net.nin[l]);
    gemm(h, p, l == 0 ? SMC_K_GEMM_FWD1 : SMC_K_GEMM_OTHER, fl);
  }
}

HeadArgs head_args(smc_t h, const float* theta) {
  HeadArgs a;
  const int L = h->L;
  a.theta = theta;
  a.D = h->D;
  a.offL = h->net.off[L - 1];
  a.H = h->net.nin[L - 1];
  a.C = h->C;
  a.J = h->J;
  a.likelihood = h->cfg.likelihood == SMC_LIK_GAUSSIAN ? 1 : 0;
  const double s = h->cfg.noise_std;
  a.inv_var = (float)(1.0 / (s * s));
  a.gauss_c = (float)(-0.5 * log(2.0 * M_PI * s * s));
  a.ylab = h->ylab;
  a.yreal = h->yreal;
  a.act = h->cfg.activation;
  if (L >= 2) {
    a.A = h->lb[L - 2].act;
    a.sAj = h->mc * a.H;
    a.sAm = a.H;
    a.a_f32 = h->split;
  } else {
    a.A = h->X;
    a.sAj = 0;
    a.sAm = h->xld;
  }
  a.llpart = h->llpart;
  a.dWpart = h->dWpart;
  return a;
}

void set_splits(smc_t h, HeadArgs& a, int m_valid) {
  const int ntiles = (m_valid + 63) / 64;
  int ns = std::max(1, std::min(h->nsplit_max, ntiles));
  a.tiles_per_split = (ntiles + ns - 1) / ns;
  a.nsplit = (ntiles + a.tiles_per_split - 1) / a.tiles_per_split;
}

// ------------------------------------------------------------------ convolutional network
// Forward of images [c0, c0 + mcv) of the operand Xop (xld-strided rows) up to the
// linear layer's outputs (logits before the bias) in cb.logits.  The GEMM copies must be current.
void cnn_forward_chunk(smc_t h, const void* Xop, int64_t c0, int mcv) {
  CnnBufs& b = h->cb;
  const CnnDims& d = b.d;
  const int J = h->J, bf = h->bf16;
  const int64_t R = (int64_t)mcv * d.HW;
  timed(h, SMC_K_OTHER, 0.0, (double)R * d.K1p * h->esz,
        [&]() { HIPCHECK(cnn_im2col_x_run(Xop, h->xld, c0, mcv, d, b.p1, bf, h->stream)); });
  {
    // conv1 of every particle as one GEMM over the J*C1 concatenated filters
    GemmParams p;
    p.epi = EPI_FWD;
    p.act = ACT_RELU;
    p.A = b.p1;
    p.lda = d.K1p;
    p.M = (int)R;
    p.K = d.K1p;
    p.B = h->net.w[0];
    p.ldb = h->net.ldw[0];
    p.N = J * d.C1;
    p.bias = h->net.bias[0];
    p.out0.ptr = b.act1;
    p.out0.cs = d.C1;
    p.out0.sC = b.s_act1;
    p.out0.rstr = d.C1;
    gemm(h, p, SMC_K_GEMM_FWD1, 2.0 * R * J * d.C1 * d.K1);
  }
  if (b.implicit) {
    // conv2 as an implicit GEMM over the activation halo, with the 2x2 pooling in its epilogue
    timed(h, SMC_K_GEMM_FWD1, 2.0 * R * J * d.C2 * d.K2, 0.0, [&]() {
      HIPCHECK(cnn_conv2_fwd_implicit_run(b.act1, b.s_act1, h->net.w[1], h->net.ldw[1], h->net.bias[1], b.act2,
                                          b.s_act2, b.pooled, b.s_pool, mcv, d, J, h->stream));
    });
  } else {
  timed(h, SMC_K_OTHER, 0.0, (double)J * R * d.K2 * h->esz,
        [&]() { HIPCHECK(cnn_im2col_a_run(b.act1, b.s_act1, mcv, d, J, b.big, b.s_big, bf, h->stream)); });
  {
    // conv2, batched over particles
    GemmParams p;
    p.epi = EPI_FWD;
    p.act = ACT_RELU;
    p.A = b.big;
    p.lda = d.K2;
    p.sAb = b.s_big;
    p.M = (int)R;
    p.K = d.K2;
    p.B = h->net.w[1];
    p.ldb = h->net.ldw[1];
    p.sBb = (int64_t)d.C2 * h->net.ldw[1];
    p.N = d.C2;
    p.batch = J;
    p.bias = h->net.bias[1];
    p.sbias = d.C2;
    p.out0.ptr = b.act2;
    p.out0.sb = b.s_act2;
    p.out0.rstr = d.C2;
    gemm(h, p, SMC_K_GEMM_FWD1, 2.0 * R * J * d.C2 * d.K2);
  }
  timed(h, SMC_K_OTHER, 0.0, (double)J * R * d.C2 * h->esz * 1.25,
        [&]() { HIPCHECK(cnn_pool_run(b.act2, b.s_act2, mcv, d, J, b.pooled, b.s_pool, bf, h->stream)); });
  }
  {
    // linear layer, batched over particles; FP32 outputs (the bias is added with the softmax)
    GemmParams p;
    p.epi = EPI_GRAD;
    p.A = b.pooled;
    p.lda = d.F3;
    p.sAb = b.s_pool;
    p.M = mcv;
    p.K = d.F3;
    p.B = h->net.w[2];
    p.ldb = h->net.ldw[2];
    p.sBb = (int64_t)d.ncls * h->net.ldw[2];
    p.N = d.ncls;
    p.batch = J;
    p.out0.ptr = b.logits;
    p.out0.sb = h->mc * d.ncls;
    p.out0.rstr = d.ncls;
    gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * mcv * J * d.ncls * d.F3);
  }
}

// The second segment of a two-segment target for one pass: samples from `split` on weigh
// lam_b, and their log-likelihood goes to ll_b (when not null).
struct Seg {
  int64_t split = INT64_MAX;
  double lam_b = 1.0;
  double* ll_b = nullptr;
};

// the handle's current target (its second-segment log-likelihood into h->ll_b)
Seg target_seg(smc_t h) { return Seg{h->seg_split, h->lam_b, h->ll_b}; }

// the weight kernel's view of the current target (two segments only when split)
void set_segment(smc_t h, WeightArgs& wa) {
  if (h->seg_split != INT64_MAX) {
    wa.ll_b = h->ll_b;
    wa.lambda_b = h->lam_b;
  }
}

CnnLLArgs cnn_ll_args(smc_t h, int mode, int mcv, int64_t c0) {
  CnnLLArgs a;
  a.logits = h->cb.logits;
  a.bias = h->net.bias[2];
  a.ylab = h->ylab;
  a.c0 = c0;
  a.mc = (int)h->mc;
  a.mcv = mcv;
  a.ncls = h->cb.d.ncls;
  a.mode = mode;
  a.d3 = h->cb.d3;
  return a;
}

// the convolutional network's pass over the subset [0, m); same contract as grad_pass
void cnn_pass(smc_t h, const float* theta, int64_t m, double lambda, const double* scale, double* ll_out,
              float* g_out, const Seg& seg) {
  CnnBufs& b = h->cb;
  const CnnDims& d = b.d;
  const int J = h->J, bf = h->bf16;
  const bool train = g_out != nullptr;
  if (train) transpose_weights(h, theta);
  for (int64_t c0 = 0; c0 < m; c0 += h->mc) {
    const int mcv = (int)std::min<int64_t>(h->mc, m - c0);
    const int64_t R = (int64_t)mcv * d.HW;
    const int beta = c0 > 0 ? 1 : 0;
    cnn_forward_chunk(h, h->X, c0, mcv);
    CnnLLArgs la = cnn_ll_args(h, train ? HEAD_TRAIN : HEAD_FORWARD, mcv, c0);
    la.lambda = lambda;
    la.scale = scale;
    la.m_split = seg.split;
    la.lambda_b = seg.lam_b;
    la.ll_acc_b = seg.ll_b;
    la.ll_acc = ll_out;
    la.beta = beta;
    timed(h, SMC_K_HEAD, 0.0, 0.0, [&]() { HIPCHECK(cnn_ll_run(la, J, bf, h->stream)); });
    if (!train) continue;
    timed(h, SMC_K_OTHER, 2.0 * J * (double)mcv * d.ncls * (d.F3 + 1), 0.0, [&]() {
      HIPCHECK(cnn_dw3_run(b.d3, b.pooled, b.s_pool, (int)h->mc, mcv, d.F3, d.ncls, J, g_out, h->D, h->net.off[2],
                           beta, bf, h->stream));
    });
    {
      // error at the pooled features: d3 [n x 16] . W3^T [F3 x 16]^T
      GemmParams p;
      p.epi = EPI_FWD;
      p.act = -1;
      p.A = b.d3;
      p.lda = 16;
      p.sAb = h->mc * 16;
      p.M = mcv;
      p.K = 16;
      p.B = b.wT[2];
      p.ldb = b.ldwT[2];
      p.sBb = (int64_t)d.F3 * b.ldwT[2];
      p.N = d.F3;
      p.batch = J;
      p.out0.ptr = b.dpool;
      p.out0.sb = b.s_pool;
      p.out0.rstr = d.F3;
      gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * mcv * J * d.ncls * d.F3);
    }
    if (!b.implicit)  // the implicit kernels form the conv2 output error from act2 and dpool themselves
      timed(h, SMC_K_OTHER, 0.0, (double)J * R * d.C2 * h->esz * 3.25, [&]() {
        HIPCHECK(cnn_unpool_run(b.dpool, b.s_pool, b.act2, b.s_act2, mcv, d, J, b.RP, b.d2, b.d2t, bf, h->stream));
      });
    if (b.implicit) {
      // conv2 weight gradient [W2 | b2] as an implicit GEMM over the chunk's pixels
      timed(h, SMC_K_GEMM_DW1, 2.0 * R * J * d.C2 * (d.K2 + 1), 0.0, [&]() {
        HIPCHECK(cnn_conv2_wgrad_implicit_run(b.act2, b.s_act2, b.dpool, b.s_pool, b.act1, b.s_act1, mcv, d, J,
                                              b.dw2part, g_out, h->D, h->net.off[1], beta, h->stream));
      });
    } else {
    timed(h, SMC_K_OTHER, 0.0, (double)J * R * (d.K2 + 1) * h->esz, [&]() {
      HIPCHECK(cnn_im2col_at_run(b.act1, b.s_act1, mcv, d, J, b.RP, b.big, b.s_big, bf, h->stream));
    });
    {
      // conv2 weight gradient [W2 | b2] = d2^T [patches | 1], reduced over the chunk's pixels
      GemmParams p;
      p.epi = EPI_GRAD;
      p.beta = beta;
      p.A = b.d2t;
      p.lda = b.RP;
      p.sAb = (int64_t)d.C2 * b.RP;
      p.M = d.C2;
      p.K = (int)R;
      p.B = b.big;
      p.ldb = b.RP;
      p.sBb = b.s_big;
      p.N = d.K2 + 1;
      p.batch = J;
      p.out0.ptr = g_out + h->net.off[1];
      p.out0.sb = h->D;
      p.out0.rstr = d.K2 + 1;
      gemm(h, p, SMC_K_GEMM_DW1, 2.0 * R * J * d.C2 * (d.K2 + 1));
    }
    }
    if (b.implicit) {
      // the error at the conv1 output as an implicit GEMM over the d2 halo (transposed conv2)
      timed(h, SMC_K_GEMM_OTHER, 2.0 * R * J * d.C2 * d.K2, 0.0, [&]() {
        HIPCHECK(cnn_conv2_dgrad_implicit_run(b.act2, b.s_act2, b.dpool, b.s_pool, b.wT[1], b.ldwT[1], b.act1,
                                              b.s_act1, b.d1t, b.RP, mcv, d, J, h->stream));
      });
    } else {
    {
      // patch errors d2 [R x C2] . W2 [C2 x K2] (B operand: W2^T rows)
      GemmParams p;
      p.epi = EPI_FWD;
      p.act = -1;
      p.A = b.d2;
      p.lda = d.C2;
      p.sAb = b.s_act2;
      p.M = (int)R;
      p.K = d.C2;
      p.B = b.wT[1];
      p.ldb = b.ldwT[1];
      p.sBb = (int64_t)d.K2 * b.ldwT[1];
      p.N = d.K2;
      p.batch = J;
      // stored tap-major, [tap][r][c] with tap planes RP * C1 apart, so that col2im reads each
      // tap's errors of consecutive pixels contiguously
      p.out0.ptr = b.big;
      p.out0.sb = b.s_big;
      p.out0.rstr = d.C1;
      p.out0.cs = d.C1;
      p.out0.sC = b.RP * d.C1;
      gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * R * J * d.C2 * d.K2);
    }
    timed(h, SMC_K_OTHER, 0.0, (double)J * R * (d.K2 + 2 * d.C1) * h->esz, [&]() {
      HIPCHECK(cnn_col2im_run(b.big, b.s_big, b.act1, b.s_act1, mcv, d, J, b.RP, b.d1t, bf, h->stream));
    });
    }
    timed(h, SMC_K_OTHER, 0.0, (double)R * (d.K1 + 1) * h->esz,
          [&]() { HIPCHECK(cnn_im2col_xt_run(h->X, h->xld, c0, mcv, d, b.RP, b.p1t, bf, h->stream)); });
    {
      // conv1 weight gradient of every particle: d1^T [J*C1 x R] . [patches | 1].  Its output has
      // only J*C1/256 row tiles, so the pixels are split into S equal K-slices (S divides R/8)
      // whose FP32 partials are summed in slice order.
      const int M = J * d.C1, N = d.K1 + 1;
      const int64_t tiles = (M + 255) / 256;
      int S = (int)std::min<int64_t>(b.kslices, std::max<int64_t>(1, 1024 / tiles));
      while (S > 1 && (R / 8) % S) --S;
      GemmParams p;
      p.epi = EPI_GRAD;
      p.A = b.d1t;
      p.lda = b.RP;
      p.M = M;
      p.B = b.p1t;
      p.ldb = b.RP;
      p.N = N;
      if (S == 1) {
        p.beta = beta;
        p.K = (int)R;
        p.out0.ptr = g_out;
        p.out0.rs = d.C1;
        p.out0.sR = h->D;
        p.out0.rstr = N;
        gemm(h, p, SMC_K_GEMM_DW1, 2.0 * R * J * d.C1 * N);
      } else {
        const int Kc = (int)(R / S);
        p.beta = 0;
        p.K = Kc;
        p.sAb = Kc;
        p.sBb = Kc;
        p.batch = S;
        p.out0.ptr = b.dw1part;
        p.out0.sb = (int64_t)M * N;
        p.out0.rstr = N;
        gemm(h, p, SMC_K_GEMM_DW1, 2.0 * R * J * d.C1 * N);
        timed(h, SMC_K_OTHER, 0.0, (double)S * M * N * 4.0, [&]() {
          HIPCHECK(cnn_slice_sum_run(b.dw1part, S, M, N, d.C1, g_out, h->D, beta, h->stream));
        });
      }
    }
  }
  if (train) h->grad_evals += (int64_t)J * m;
}

// Layer 1 and the output layer of samples [c0, c0 + mcv) of the operand Xop in one fused
// kernel (networks with one hidden layer, BF16 or split-BF16 operands); a carries the
// output-layer arguments (mode, targets, dT).  Timed as the layer-1 forward class with the
// algorithmic FLOPs of both layers.
void fused_chunk(smc_t h, const void* Xop, int64_t c0, int mcv, int mode, HeadArgs& a) {
  const int rows = (int)round_up(mcv, 64);
  GemmParams p;
  p.A = (const char*)Xop + c0 * h->xld * (int64_t)h->esz;
  p.lda = h->xld;
  p.M = rows;
  p.K = h->net.ldw[0];  // split: the kernel adds the w_lo plane (second half of each weight row)
  p.B = h->net.w[0];
  p.ldb = h->net.ldw[0] * (h->split ? 2 : 1);
  p.bias = h->net.bias[0];
  a.m_valid = mcv;
  a.c0 = c0;
  a.nsplit = (rows + 255) / 256;
  const double H = h->net.nout[0], flops = 2.0 * mcv * (double)h->J * H * h->F +
                                           (mode == HEAD_TRAIN ? 6.0 : 2.0) * a.C * H * h->J * mcv;
  const int split = h->split && !h->grad_only;  // the weight copy keeps its [w_hi | w_lo] rows either way
  timed(h, SMC_K_GEMM_FWD1, flops, 0.0,
        [&]() { HIPCHECK(fwd_head_run(p, a, mode, split, h->cfg.activation, h->stream)); });
}

// Marks the passes of its scope as gradient-only (see smc_handle::grad_only).
struct GradOnlyScope {
  smc_t h;
  GradOnlyScope(smc_t h_, bool on) : h(h_) { h->grad_only = on; }
  ~GradOnlyScope() { h->grad_only = false; }
};

// One pass over the subset [0, m): log-likelihoods ll_out[j] (FP64) and, when
// g_out is given, g_out[j] = scale_j * d LL_j / d theta_j (the lambda-scaled
// likelihood gradient).  The GEMM copies of `theta` must be current.
void grad_pass(smc_t h, const float* theta, int64_t m, double lambda, const double* scale, double* ll_out,
               float* g_out, const Seg& seg = Seg{}) {
  if (h->cnn) {
    cnn_pass(h, theta, m, lambda, scale, ll_out, g_out, seg);
    return;
  }
  const int J = h->J, L = h->L;
  const bool train = g_out != nullptr;
  if (train && L >= 3) transpose_weights(h, theta);
  for (int64_t c0 = 0; c0 < m; c0 += h->mc) {
    const int mcv = (int)std::min<int64_t>(h->mc, m - c0);
    const int rows = (int)round_up(mcv, 64);
    const int beta = c0 > 0 ? 1 : 0;
    if (h->lenet) lenet_features(h, theta, h->X, c0, mcv, rows, train);
    if (!h->fused) forward_hidden(h, h->X, c0, rows, mcv);
    HeadArgs a = head_args(h, theta);
    if (L == 1) a.A = (const char*)h->X + c0 * h->xld * (int64_t)h->esz;
    a.m_valid = mcv;
    a.c0 = c0;
    a.lambda = lambda;
    a.scale = scale;
    a.m_split = seg.split;
    a.lambda_b = seg.lam_b;
    if (seg.ll_b) {
      a.ll_acc_b = seg.ll_b;
      a.llpart_b = h->llpart_b;
    }
    a.ll_acc = ll_out;
    a.grad = g_out;
    a.beta = beta;
    set_splits(h, a, mcv);
    if (train && L >= 2) {
      a.dT = h->lb[L - 2].dT;
      a.sdTj = (int64_t)a.H * h->mc;
      a.sdTh = h->mc;
      if (h->lb[L - 2].dR) {
        a.dR = h->lb[L - 2].dR;
        a.sdRj = h->mc * a.H;
        a.sdRm = a.H;
      }
    }
    if (h->fused)
      fused_chunk(h, h->X, c0, mcv, train ? HEAD_TRAIN : HEAD_FORWARD, a);
    else
      timed(h, SMC_K_HEAD, (train ? 6.0 : 2.0) * a.C * (double)a.H * J * mcv, 0.0, [&]() {
        HIPCHECK(head_run(a, train ? HEAD_TRAIN : HEAD_FORWARD, head_type(h->cfg.precision), h->stream));
      });
    if (!train) continue;
    // backward through the hidden layers, top down
    for (int l = L - 2; l >= 0; --l) {
      const int nout = h->net.nout[l], nin = h->net.nin[l];
      {
        // weight gradient [W_l | b_l] = delta_l^T [a_{l-1}, 1]
        GemmParams p;
        p.epi = EPI_GRAD;
        p.beta = beta;
        p.K = rows;
        p.A = h->lb[l].dT;
        p.lda = h->mc;
        if (l == 0 && h->lenet) {
          p.M = nout;
          p.N = nin + 1;
          p.sAb = (int64_t)nout * h->mc;
          p.B = h->lfeatT;
          p.ldb = h->mc;
          p.sBb = (int64_t)(nin + 1) * h->mc;
          p.batch = J;
          p.out0.ptr = g_out + h->net.off[0];
          p.out0.sb = h->D;
          p.out0.rstr = nin + 1;
        } else if (l == 0) {
          p.M = J * nout;
          p.N = nin + 1;
          p.B = (const char*)h->XT + c0 * (int64_t)h->esz;
          p.ldb = h->n_pad;
          p.batch = 1;
          p.out0.ptr = g_out;
          p.out0.rs = nout;
          p.out0.sR = h->D;
          p.out0.rstr = nin + 1;
        } else {
          p.M = nout;
          p.N = nin + 1;
          p.sAb = (int64_t)nout * h->mc;
          p.B = h->lb[l - 1].actT;
          p.ldb = h->mc;
          p.sBb = (int64_t)(nin + 1) * h->mc;
          p.batch = J;
          p.out0.ptr = g_out + h->net.off[l];
          p.out0.sb = h->D;
          p.out0.rstr = nin + 1;
        }
        gemm(h, p, l == 0 ? SMC_K_GEMM_DW1 : SMC_K_GEMM_OTHER, 2.0 * J * nout * (double)(nin + 1) * mcv);
      }
      if (l >= 1 && !h->lb[l - 1].dR && !h->split) {
        // error of the layer below, (delta_l W_l) * act'(a_{l-1}), as its transpose
        // W_l^T delta_l^T: rows are units and columns samples, so the error is written
        // sample-contiguous through the staged epilogue and act' reads the transposed
        // activations a_{l-1}^T row by row
        GemmParams p;
        p.epi = EPI_DELTA;
        p.act = h->cfg.activation;
        p.M = nin;
        p.N = rows;
        p.K = nout;
        p.A = h->lb[l].wT;
        p.lda = h->lb[l].ldwT;
        p.sAb = (int64_t)nin * h->lb[l].ldwT;
        p.B = h->lb[l].dR;
        p.ldb = nout;
        p.sBb = h->mc * nout;
        p.batch = J;
        p.aux.ptr = h->lb[l - 1].actT;
        p.aux.sb = (int64_t)(nin + 1) * h->mc;
        p.aux.rstr = h->mc;
        p.out0.ptr = h->lb[l - 1].dT;
        p.out0.sb = (int64_t)nin * h->mc;
        p.out0.rstr = h->mc;
        gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * J * nout * (double)nin * mcv);
      } else if (l >= 1) {
        // error of the layer below: (delta_l W_l) * act'(a_{l-1}), written sample-contiguous
        // here and sample-major to dR for the layer below it
        GemmParams p;
        p.epi = EPI_DELTA;
        p.act = h->cfg.activation;
        p.M = rows;
        p.N = nin;
        p.K = nout;
        p.A = h->lb[l].dR;
        p.lda = nout;
        p.sAb = h->mc * nout;
        p.B = h->lb[l].wT;
        p.ldb = h->lb[l].ldwT;
        p.sBb = (int64_t)nin * h->lb[l].ldwT;
        p.batch = J;
        p.aux.ptr = h->lb[l - 1].act;
        p.aux.sb = h->mc * nin;
        p.aux.rstr = nin;
        p.out0.ptr = h->lb[l - 1].dT;
        p.out0.sb = (int64_t)nin * h->mc;
        p.out0.cstr = h->mc;
        p.out0.rstr = 1;
        if (h->lb[l - 1].dR) {
          p.out1.ptr = h->lb[l - 1].dR;
          p.out1.sb = h->mc * nin;
          p.out1.rstr = nin;
        }
        gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * J * nout * (double)nin * mcv);
      }
      if (l == 0 && h->lenet) {
        // error of the features, delta_0 W_0 (the pooling and activation below it belong to
        // the convolution stack), then the convolution weight gradients
        GemmParams p;
        p.epi = EPI_FWD;
        p.M = rows;
        p.N = nin;
        p.K = nout;
        p.A = h->lb[0].dR;
        p.lda = nout;
        p.sAb = h->mc * nout;
        p.B = h->lb[0].wT;
        p.ldb = h->lb[0].ldwT;
        p.sBb = (int64_t)nin * h->lb[0].ldwT;
        p.batch = J;
        p.out0.ptr = h->ldfeat;
        p.out0.sb = h->mc * nin;
        p.out0.rstr = nin;
        gemm(h, p, SMC_K_GEMM_OTHER, 2.0 * J * nout * (double)nin * mcv);
        const int ipb = (mcv + h->lbwd_blocks - 1) / h->lbwd_blocks;
        timed(h, SMC_K_OTHER, 2.0 * J * mcv * lenet_bwd_macs_per_image(h->ld), 0.0, [&]() {
          HIPCHECK(lenet_bwd_run((const float*)h->X, h->xld, c0, mcv, ipb, h->ld, theta, h->D, J, h->cfg.activation,
                                 h->ldfeat, h->mc * h->ld.F, h->lmaps, h->mc * h->ld.Mimg, h->lpart, h->lpart_blocks,
                                 g_out, beta, h->stream));
        });
      }
    }
  }
  if (train) h->grad_evals += (int64_t)J * m;
}

void ensure_cast(smc_t h) {
  if (!h->w_dirty) return;
  timed(h, SMC_K_OTHER, 0.0, (double)h->J * h->D * (4.0 + h->esz),
        [&]() { HIPCHECK(cast_run(h->net, h->theta, nullptr, h->stream)); });
  h->w_dirty = false;
}

void read_stats(smc_t h, double* st) {
  HIPCHECK(hipMemcpyAsync(st, h->stats, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  sync(h);
}

void fill_info(smc_t h, smc_step_info* info, int64_t evals) {
  double st[8];
  read_stats(h, st);
  if (info) {
    info->ess = st[ST_ESS];
    info->log_z_increment = st[ST_LOGZ];
    info->mean_loglik = st[ST_MEANLL];
    info->max_loglik = st[ST_MAXLL];
    info->n_nonfinite = (int32_t)st[ST_NONFINITE];
    info->resample_recommended = (int32_t)st[ST_RECOMMEND];
    info->grad_evals = evals;
  }
  if (st[ST_ALLBAD] != 0.0) fail(SMC_ERR_NONFINITE, "every particle has a non-finite log-weight");
}

// initial weighting at the current subset: log w = lambda LL (Eq. init_weight)
void initial_weighting(smc_t h) {
  HIPCHECK(sq_norm_rows_run(h->theta, h->J, h->D, h->tsq, h->stream));
  WeightArgs wa;
  wa.J = h->J;
  wa.init = 1;
  wa.lambda = h->lam;
  set_segment(h, wa);
  wa.inv_2prior_var = 0.5 / (h->cfg.prior_std * h->cfg.prior_std);
  wa.ess_frac = h->cfg.ess_frac;
  wa.ll = h->ll;
  wa.tsq = h->tsq;
  wa.lp = h->lp;
  wa.logw = h->logw;
  wa.w = h->w;
  wa.stats = h->stats;
  HIPCHECK(weight_run(wa, h->stream));
}

MoveArgs move_args(smc_t h, int mode) {
  MoveArgs a;
  a.net = h->net;
  a.theta = h->theta;
  a.P = h->P;
  a.g = h->g;
  a.part = h->part;
  a.nblk = h->nblk;
  a.mode = mode;
  a.h = (float)h->cfg.step_size;
  a.inv_prior_var = (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std));
  a.key0 = key0(h);
  a.key1 = key1(h);
  a.ctr_iter = (uint32_t)h->rng_iter;
  a.cast = 1;
  return a;
}


// parameter groups of the learned proposal: W_l and b_l of every layer
void setup_groups(smc_t h) {
  h->G = 2 * h->L;
  h->NO = 1 + h->G;
  std::vector<int64_t> n(h->G);
  for (int l = 0; l < h->L; ++l) {
    n[2 * l] = (int64_t)h->net.nout[l] * h->net.nin[l];
    n[2 * l + 1] = h->net.nout[l];
  }
  h->group_n = dalloc<int64_t>(h->owned, h->G);
  HIPCHECK(hipMemcpyAsync(h->group_n, n.data(), n.size() * 8, hipMemcpyHostToDevice, h->stream));
  sync(h);
  h->sc0 = dalloc<float>(h->owned, (int64_t)h->J * h->NO);
  h->sc1 = dalloc<float>(h->owned, (int64_t)h->J * h->NO);
  h->feat = dalloc<double>(h->owned, (int64_t)h->J * 4);
  h->gsum = dalloc<double>(h->owned, (int64_t)h->J * h->G);
}

double k_over_K(smc_t h) {
  return h->cfg.n_iterations > 0 ? (double)h->k_iter / (double)h->cfg.n_iterations : 0.0;
}

// features at the handle's current (theta, g, ll) and the network's scales into `sc`
void learned_scales(smc_t h, float* sc) {
  const float ipv = (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std));
  timed(h, SMC_K_OTHER, 0.0, (double)h->J * h->D * 8.0, [&]() {
    HIPCHECK(features_run(h->net, h->theta, h->g, h->ll, ipv, (double)h->m, k_over_K(h), (double)h->m / h->n_data,
                          h->feat, nullptr, h->G, h->stream));
    HIPCHECK(mlp_infer_run(h->pnet, h->feat, 1, h->J, h->G, sc, 1, (float)h->h0, h->bf16, h->stream));
  });
}

LearnedMoveArgs learned_args(smc_t h, int mode, const float* sc) {
  LearnedMoveArgs a;
  a.net = h->net;
  a.theta = h->theta;
  a.P = h->P;
  a.g = h->g;
  a.scales = sc;
  a.NO = h->NO;
  a.part = h->part;
  a.nblk = h->nblk;
  a.mode = mode;
  a.inv_prior_var = (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std));
  a.key0 = key0(h);
  a.key1 = key1(h);
  a.ctr_iter = (uint32_t)h->rng_iter;
  return a;
}

void mlp_steps(float* params, float* adam, const float* feat, const float* tgt, int64_t R, int G, int first_step,
               int n_steps, double lr, float* grad_out, double* loss_host, hipStream_t st) {
  if (R < 1 || G < 1 || G > 2 * SMC_MAX_LAYERS) fail(SMC_ERR_ARG, "bad size");
  HIPCHECK(mlp_set_smem_limits());
  const int Pn = mlp_n_params(G);
  const int64_t ntiles = (R + 63) / 64;
  float* gp = nullptr;
  double* lp = nullptr;
  HIPCHECK(hipMalloc((void**)&gp, (size_t)ntiles * Pn * 4));
  hipError_t e = hipMalloc((void**)&lp, (size_t)(ntiles + 1) * 8);
  if (e != hipSuccess) {
    (void)hipFree(gp);
    HIPCHECK(e);
  }
  for (int i = 0; i < n_steps && e == hipSuccess; ++i)
    e = mlp_train_step_run(params, adam, feat, tgt, R, G, gp, lp, first_step + i, (float)lr, grad_out,
                           i == n_steps - 1 ? lp + ntiles : nullptr, st);
  double loss = 0.0;
  if (e == hipSuccess && loss_host) e = hipMemcpyAsync(&loss, lp + ntiles, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(gp);
  (void)hipFree(lp);
  HIPCHECK(e);
  if (loss_host) *loss_host = loss;
}

// ------------------------------------------------------------------ allocation-free training
// smc_mlp_train_noalloc keeps the per-tile gradient partials and loss partials of one Adam
// step in a fixed file-scope device array instead of hipMalloc'd buffers.  Every device the
// library runs on holds its own copy until the process ends.  In host code the array's name
// is only a stand-in for its device address, which hipGetSymbolAddress returns once per
// device (with that device current); kernels receive that address.
constexpr int64_t NOALLOC_MAX_ROWS = 32768;
constexpr int NOALLOC_MAX_GROUPS = 8;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)10 << 20;  // 10 MiB
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

inline size_t noalloc_grad_bytes(int64_t ntiles, int Pn) { return (size_t)round_up(ntiles * Pn * 4, 256); }

// device address of the current device's scratch array (looked up on the first call per device)
char* noalloc_scratch() {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) fail(SMC_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(SMC_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = (char*)p;
  }
  return g_scratch_ptr[dev];
}

void mlp_steps_noalloc(float* params, float* adam, const float* feat, const float* tgt, int64_t R, int G,
                       int first_step, int n_steps, double lr, double* loss_dev, hipStream_t st) {
  if (R < 1 || R > NOALLOC_MAX_ROWS) fail(SMC_ERR_ARG, "R must be in [1, 32768] for the allocation-free call");
  if (G < 1 || G > NOALLOC_MAX_GROUPS) fail(SMC_ERR_ARG, "n_groups must be in [1, 8] for the allocation-free call");
  const int Pn = mlp_n_params(G);
  const int64_t ntiles = (R + 63) / 64;
  const size_t gbytes = noalloc_grad_bytes(ntiles, Pn);
  if (gbytes + (size_t)ntiles * 8 > NOALLOC_SCRATCH_BYTES) fail(SMC_ERR_ARG, "scratch too small for this call");
  char* base = noalloc_scratch();
  HIPCHECK(mlp_set_smem_limits());
  float* gp = (float*)base;
  double* lp = (double*)(base + gbytes);
  for (int i = 0; i < n_steps; ++i)
    HIPCHECK(mlp_train_step_run(params, adam, feat, tgt, R, G, gp, lp, first_step + i, (float)lr, nullptr,
                                i == n_steps - 1 ? loss_dev : nullptr, st));
}

smc_status guard(void (*body)(void*), void* ctx) {
  try {
    g_last_error.clear();
    body(ctx);
    return SMC_OK;
  } catch (const Fail& f) {
    return f.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SMC_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = std::string("C++ exception: ") + e.what();
    return SMC_ERR_DEVICE;
  } catch (...) {
    g_last_error = "unexpected C++ exception";
    return SMC_ERR_DEVICE;
  }
}

template <typename F>
smc_status run(F&& f) {
  auto thunk = [](void* c) { (*(F*)c)(); };
  return guard(thunk, (void*)&f);
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char* smc_status_string(smc_status s) {
  switch (s) {
    case SMC_OK: return "ok";
    case SMC_ERR_ARG: return "invalid argument";
    case SMC_ERR_OOM: return "out of device memory";
    case SMC_ERR_DEVICE: return "HIP device error";
    case SMC_ERR_STATE: return "invalid call for the handle's state";
    case SMC_ERR_NONFINITE: return "every particle has a non-finite log-weight";
    case SMC_ERR_UNSUPPORTED: return "unsupported configuration";
    case SMC_ERR_NOLIB: return "library not loaded";
  }
  return "unknown status";
}

const char* smc_last_error(void) { return g_last_error.c_str(); }

smc_status smc_init(const smc_config* cfg, const float* x_dev, const void* y_dev, int64_t n_data,
                    const float* theta0_dev, int64_t m0, double lambda0, void* hip_stream, smc_t* out) {
  smc_t h = nullptr;
  const smc_status st = run([&]() {
    if (!out) fail(SMC_ERR_ARG, "out is null");
    *out = nullptr;
    check_config(cfg);
    if (!x_dev || !y_dev) fail(SMC_ERR_ARG, "x_dev and y_dev are required");
    if (n_data < 1 || n_data > (int64_t)1 << 30) fail(SMC_ERR_ARG, "n_data out of range");
    if (m0 < 1 || m0 > n_data) fail(SMC_ERR_ARG, "m0 must be in [1, n_data]");
    if (!(lambda0 > 0) || !isfinite(lambda0)) fail(SMC_ERR_ARG, "lambda0 must be finite and > 0");
    h = new smc_handle();
    h->cfg = *cfg;
    h->stream = (hipStream_t)hip_stream;
    h->n_data = n_data;
    setup_shapes(h);
    HIPCHECK(head_set_smem_limits());
    HIPCHECK(kernels_set_smem_limits());
    HIPCHECK(mlp_set_smem_limits());
    alloc_all(h);
    setup_groups(h);
    upload_data(h, x_dev, y_dev);
    if (theta0_dev)
      HIPCHECK(hipMemcpyAsync(h->theta, theta0_dev, (size_t)h->J * h->D * 4, hipMemcpyDeviceToDevice, h->stream));
    else
      HIPCHECK(prior_draw_run(h->theta, h->J, h->D, (float)cfg->prior_std, key0(h), key1(h), h->stream));
    h->w_dirty = true;
    ensure_cast(h);
    h->m = m0;
    h->lam = lambda0;
    grad_pass(h, h->theta, m0, lambda0, nullptr, h->ll, h->g, target_seg(h));
    initial_weighting(h);
    double st8[8];
    read_stats(h, st8);
    if (st8[ST_ALLBAD] != 0.0) fail(SMC_ERR_NONFINITE, "every particle has a non-finite initial log-weight");
    *out = h;
  });
  if (st != SMC_OK && h) {
    (void)hipStreamSynchronize(h->stream);
    for (void* p : h->owned) (void)hipFree(p);
    delete h;
  }
  return st;
}

void smc_destroy(smc_t h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (void* p : h->owned) (void)hipFree(p);
  if (h->tx) (void)hipFree(h->tx);
  if (h->logp) (void)hipFree(h->logp);
  if (h->per_sample) (void)hipFree(h->per_sample);
  for (auto& r : h->prof_recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : h->prof_pool) (void)hipEventDestroy(e);
  delete h;
}

int64_t smc_n_params(smc_t h) { return h ? h->D : -1; }
int64_t smc_chunk_samples(smc_t h) { return h ? h->mc : -1; }

namespace {

// One iteration (move + reweight) targeting lambda_k LL[0, split) + lambda_b LL[split, m_k) + log q0.
void step_impl(smc_t h, int64_t m_k, int64_t split, double lambda_k, double lambda_b, smc_step_info* info) {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    if (m_k < h->m || m_k > h->n_data) fail(SMC_ERR_ARG, "m_k must satisfy previous m <= m_k <= n_data");
    if (!(lambda_k > 0) || !isfinite(lambda_k)) fail(SMC_ERR_ARG, "lambda_k must be finite and > 0");
    if (split < 0) fail(SMC_ERR_ARG, "m_split must be >= 0");
    if (split >= m_k) {
      split = INT64_MAX;  // one segment
      lambda_b = lambda_k;
    } else if (!(lambda_b > 0) || !isfinite(lambda_b)) {
      fail(SMC_ERR_ARG, "lambda_b must be finite and > 0");
    }
    if (h->cfg.proposal == SMC_PROPOSAL_LEARNED && !h->pnet) fail(SMC_ERR_STATE, "no proposal network set");
    const int64_t ev0 = h->grad_evals;
    ensure_cast(h);
    if (m_k != h->m || lambda_k != h->lam || split != h->seg_split || lambda_b != h->lam_b) {
      // the target changed: gradient at the current particles under the new target
      h->m = m_k;
      h->lam = lambda_k;
      h->seg_split = split;
      h->lam_b = lambda_b;
      // with the fixed-step move only the gradient of this pass is used: the weight's denominator
      // is the cached log pi_{k-1}(theta_{k-1}), its numerator comes from the move's last pass
      // (the learned move's features read this pass's log-likelihood)
      GradOnlyScope go(h, h->cfg.proposal == SMC_PROPOSAL_FIXED);
      grad_pass(h, h->theta, m_k, lambda_k, nullptr, h->ll, h->g, target_seg(h));
    }
    h->rng_iter += 1;
    h->k_iter += 1;
    if (h->cfg.proposal == SMC_PROPOSAL_LEARNED) {
      // learned-scale Langevin move with its Gaussian forward / reverse densities
      learned_scales(h, h->sc0);
      LearnedMoveArgs la = learned_args(h, MOVE_FIRST, h->sc0);
      if (h->noise_pending) la.noise = h->noise;
      const double nd = (double)h->J * h->D;
      timed(h, SMC_K_MOVE, 0.0, nd * (16.0 + h->esz + (la.noise ? 4.0 : 0.0)),
            [&]() { HIPCHECK(learned_move_run(la, h->stream)); });
      h->noise_pending = false;
      grad_pass(h, h->theta, m_k, lambda_k, nullptr, h->ll, h->g, target_seg(h));
      learned_scales(h, h->sc1);
      LearnedMoveArgs lb = learned_args(h, MOVE_LAST, h->sc1);
      timed(h, SMC_K_MOVE, 0.0, nd * 12.0, [&]() { HIPCHECK(learned_move_run(lb, h->stream)); });
      HIPCHECK(learned_extra_run(h->sc0, h->sc1, h->NO, h->part, h->J, h->nblk, h->group_n, h->D, h->extra,
                                 h->stream));
      WeightArgs wa;
      wa.J = h->J;
      wa.nblk = h->nblk;
      wa.lambda = lambda_k;
      set_segment(h, wa);
      wa.inv_2prior_var = 0.5 / (h->cfg.prior_std * h->cfg.prior_std);
      wa.ess_frac = h->cfg.ess_frac;
      wa.ll = h->ll;
      wa.part = h->part;
      wa.extra = h->extra;
      wa.no_kinetic = 1;
      wa.lp = h->lp;
      wa.logw = h->logw;
      wa.w = h->w;
      wa.stats = h->stats;
      timed(h, SMC_K_WEIGHT, 0.0, 0.0, [&]() { HIPCHECK(weight_run(wa, h->stream)); });
      if (info) fill_info(h, info, h->grad_evals - ev0);
      return;
    }
    const int S = h->cfg.leapfrog_steps;
    MoveArgs ma = move_args(h, MOVE_FIRST);
    if (h->noise_pending) ma.noise = h->noise;
    const double nd = (double)h->J * h->D;
    // FIRST: read theta, g (+noise); write P, theta and the GEMM copy
    timed(h, SMC_K_MOVE, 0.0, nd * (16.0 + h->esz + (ma.noise ? 4.0 : 0.0)),
          [&]() { HIPCHECK(move_run(ma, h->stream)); });
    h->noise_pending = false;
    for (int s = 1; s <= S; ++s) {
      {
        GradOnlyScope go(h, s < S);  // intermediate leapfrog positions: gradient only
        grad_pass(h, h->theta, m_k, lambda_k, nullptr, h->ll, h->g, target_seg(h));
      }
      MoveArgs mb = move_args(h, s < S ? MOVE_MID : MOVE_LAST);
      // MID: read theta, g, P; write P, theta, copy.  LAST: read P, g, theta
      timed(h, SMC_K_MOVE, 0.0, nd * (s < S ? 20.0 + h->esz : 12.0), [&]() { HIPCHECK(move_run(mb, h->stream)); });
    }
    WeightArgs wa;
    wa.J = h->J;
    wa.nblk = h->nblk;
    wa.lambda = lambda_k;
    set_segment(h, wa);
    wa.inv_2prior_var = 0.5 / (h->cfg.prior_std * h->cfg.prior_std);
    wa.ess_frac = h->cfg.ess_frac;
    wa.ll = h->ll;
    wa.part = h->part;
    wa.lp = h->lp;
    wa.logw = h->logw;
    wa.w = h->w;
    wa.stats = h->stats;
    timed(h, SMC_K_WEIGHT, 0.0, 0.0, [&]() { HIPCHECK(weight_run(wa, h->stream)); });
    if (info) fill_info(h, info, h->grad_evals - ev0);
}

}  // namespace

smc_status smc_step(smc_t h, int64_t m_k, double lambda_k, smc_step_info* info) {
  return run([&]() { step_impl(h, m_k, INT64_MAX, lambda_k, lambda_k, info); });
}

smc_status smc_step_tempered(smc_t h, int64_t m_k, int64_t m_split, double lambda_a, double lambda_b,
                             smc_step_info* info) {
  return run([&]() { step_impl(h, m_k, m_split, lambda_a, lambda_b, info); });
}

smc_status smc_segment_moments(smc_t h, double* out4) {
  return run([&]() {
    if (!h || !out4) fail(SMC_ERR_ARG, "handle and out4 are required");
    double* d = h->stats + 12;  // device slots 12..15
    HIPCHECK(segment_moments_run(h->w, h->ll, h->ll_b, h->J, d, h->stream));
    double host[4];
    HIPCHECK(hipMemcpyAsync(host, d, sizeof(host), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    for (int i = 0; i < 4; ++i) out4[i] = host[i];
  });
}

namespace {

void resample_impl(smc_t h, int32_t mode, int scheme, const double* u, const double* u_arr_dev, int32_t* resampled,
                   int32_t* ancestors_host) {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    if (mode < 0 || mode > 2) fail(SMC_ERR_ARG, "mode");
    if (u && !(*u >= 0.0 && *u < 1.0)) fail(SMC_ERR_ARG, "u must be in [0, 1)");
    ResampleArgs ra;
    ra.J = h->J;
    ra.mode = mode;
    ra.scheme = scheme;
    ra.u_arr = u_arr_dev;
    ra.ess_frac = h->cfg.ess_frac;
    double* u_dev = nullptr;
    if (u) {
      u_dev = h->stats + 8;  // device scalar slot
      HIPCHECK(hipMemcpyAsync(u_dev, u, sizeof(double), hipMemcpyHostToDevice, h->stream));
      sync(h);  // the host value may go out of scope
    }
    ra.u_dev = u_dev;
    ra.key0 = key0(h);
    ra.key1 = key1(h);
    ra.ctr_iter = (uint32_t)h->rng_iter;
    ra.w = h->w;
    ra.logw = h->logw;
    ra.stats = h->stats;
    ra.ancestors = h->anc;
    ra.placement = h->place;
    ra.sc[0] = h->ll;
    ra.sc[1] = h->lp;
    ra.sc[2] = h->ll_b;
    timed(h, SMC_K_RESAMPLE, 0.0, 0.0, [&]() {
      HIPCHECK(resample_run(ra, h->stream));
      HIPCHECK(gather_rows_run(h->J, h->D, h->place, h->theta, h->g, h->stream));
      if (!h->w_dirty) HIPCHECK(cast_run(h->net, h->theta, h->place, h->stream));
    });
    {
      // the flags are read on every call, so that a population whose weights all became
      // non-finite in a step that returned no statistics is reported here
      double st[8];
      read_stats(h, st);
      if (st[ST_ALLBAD] != 0.0) fail(SMC_ERR_NONFINITE, "every particle has a non-finite log-weight: not resampled");
      if (resampled) *resampled = st[ST_RESAMPLED] != 0.0 ? 1 : 0;
      if (ancestors_host) {
        HIPCHECK(hipMemcpyAsync(ancestors_host, h->anc, (size_t)h->J * 4, hipMemcpyDeviceToHost, h->stream));
        sync(h);
      }
    }
}

}  // namespace

smc_status smc_resample(smc_t h, int32_t mode, const double* u, int32_t* resampled, int32_t* ancestors_host) {
  return run([&]() { resample_impl(h, mode, RESAMPLE_SYSTEMATIC, u, nullptr, resampled, ancestors_host); });
}

smc_status smc_resample_multinomial(smc_t h, int32_t mode, const double* u_dev, int32_t* resampled,
                                    int32_t* ancestors_host) {
  return run([&]() { resample_impl(h, mode, RESAMPLE_MULTINOMIAL, nullptr, u_dev, resampled, ancestors_host); });
}

smc_status smc_posterior_predict(smc_t h, const float* x_dev, const int32_t* y_dev, int64_t n, float* probs_dev,
                                 double* accuracy, double* mean_log_pred) {
  return run([&]() {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    if (!x_dev || n < 1) fail(SMC_ERR_ARG, "x_dev and n >= 1 are required");
    if ((accuracy || mean_log_pred) && !y_dev) fail(SMC_ERR_ARG, "accuracy needs labels");
    if (h->cfg.likelihood != SMC_LIK_CATEGORICAL && (accuracy || mean_log_pred))
      fail(SMC_ERR_UNSUPPORTED, "accuracy needs the categorical likelihood");
    ensure_cast(h);
    const int64_t np = round_up(n, 256);
    if (np > h->tx_rows) {
      if (h->tx) HIPCHECK(hipFree(h->tx));
      h->tx = nullptr;
      HIPCHECK(hipMalloc(&h->tx, (size_t)np * h->xld * h->esz));
      h->tx_rows = np;
    }
    if (n > h->logp_n) {
      if (h->logp) HIPCHECK(hipFree(h->logp));
      if (h->per_sample) HIPCHECK(hipFree(h->per_sample));
      h->logp = nullptr;
      h->per_sample = nullptr;
      HIPCHECK(hipMalloc((void**)&h->logp, (size_t)h->J * n * h->C * sizeof(float)));
      HIPCHECK(hipMalloc((void**)&h->per_sample, (size_t)n * 2 * sizeof(double) + 4 * sizeof(double)));
      h->logp_n = n;
    }
    const int64_t nx = np * h->ldx;
    if (h->bf16)
      hipLaunchKernelGGL(pack_x_kernel<__bf16>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream, x_dev, n,
                         h->F, h->ldx, h->split ? 2 : 1, np, (__bf16*)h->tx);
    else
      hipLaunchKernelGGL(pack_x_kernel<float>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, h->stream, x_dev, n,
                         h->F, h->ldx, 1, np, (float*)h->tx);
    HIPCHECK(hipGetLastError());
    for (int64_t c0 = 0; c0 < n; c0 += h->mc) {
      const int mcv = (int)std::min<int64_t>(h->mc, n - c0);
      if (h->cnn) {
        cnn_forward_chunk(h, h->tx, c0, mcv);
        CnnLLArgs la = cnn_ll_args(h, HEAD_PREDICT, mcv, c0);
        la.logp = h->logp;
        la.ld_logp = n;
        HIPCHECK(cnn_ll_run(la, h->J, h->bf16, h->stream));
        continue;
      }
      if (h->fused) {
        HeadArgs a = head_args(h, h->theta);
        a.logp = h->logp;
        a.ld_logp = n;
        fused_chunk(h, h->tx, c0, mcv, HEAD_PREDICT, a);
        continue;
      }
      const int rows = (int)round_up(mcv, 64);
      if (h->lenet) lenet_features(h, h->theta, h->tx, c0, mcv, rows, false);
      forward_hidden(h, h->tx, c0, rows, mcv);
      HeadArgs a = head_args(h, h->theta);
      if (h->L == 1) a.A = (const char*)h->tx + c0 * h->xld * (int64_t)h->esz;
      a.m_valid = mcv;
      a.c0 = c0;
      a.logp = h->logp;
      a.ld_logp = n;
      set_splits(h, a, mcv);
      HIPCHECK(head_run(a, HEAD_PREDICT, head_type(h->cfg.precision), h->stream));
    }
    double* pred_out = h->per_sample + 2 * n;
    HIPCHECK(predictive_run(h->logp, n, h->logw, h->J, h->C, n, y_dev, probs_dev, y_dev ? h->per_sample : nullptr,
                            h->stream));
    if (y_dev && (accuracy || mean_log_pred)) {
      HIPCHECK(predictive_finish_run(h->per_sample, n, pred_out, h->stream));
      double host[2];
      HIPCHECK(hipMemcpyAsync(host, pred_out, sizeof(host), hipMemcpyDeviceToHost, h->stream));
      sync(h);
      if (accuracy) *accuracy = host[0];
      if (mean_log_pred) *mean_log_pred = host[1];
    }
  });
}

smc_status smc_posterior_mean(smc_t h, double* mean_dev) {
  return run([&]() {
    if (!h || !mean_dev) fail(SMC_ERR_ARG, "null argument");
    HIPCHECK(posterior_mean_run(h->theta, h->w, h->J, h->D, mean_dev, h->stream));
  });
}

smc_status smc_posterior_mean_change(smc_t h, double* rel_change) {
  return run([&]() {
    if (!h || !rel_change) fail(SMC_ERR_ARG, "null argument");
    if (!h->pm_prev) {
      h->pm_prev = dalloc<double>(h->owned, h->D);
      h->pm_cur = dalloc<double>(h->owned, h->D);
      h->pm_out = dalloc<double>(h->owned, 2);
    }
    HIPCHECK(posterior_mean_run(h->theta, h->w, h->J, h->D, h->pm_cur, h->stream));
    double r = INFINITY;
    if (h->pm_have) {
      double host[2];
      HIPCHECK(mean_change_run(h->pm_cur, h->pm_prev, h->D, h->pm_out, h->stream));
      HIPCHECK(hipMemcpyAsync(host, h->pm_out, sizeof(host), hipMemcpyDeviceToHost, h->stream));
      sync(h);
      r = host[1] > 0.0 ? sqrt(host[0]) / sqrt(host[1]) : (host[0] == 0.0 ? 0.0 : INFINITY);
    }
    std::swap(h->pm_prev, h->pm_cur);
    h->pm_have = true;
    *rel_change = r;
  });
}

smc_status smc_get_state(smc_t h, float* theta_dev, double* logw_dev, double* loglik_dev, double* logpi_dev,
                         float* grad_dev) {
  return run([&]() {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    const size_t nd = (size_t)h->J * h->D;
    if (theta_dev) HIPCHECK(hipMemcpyAsync(theta_dev, h->theta, nd * 4, hipMemcpyDeviceToDevice, h->stream));
    if (logw_dev) HIPCHECK(hipMemcpyAsync(logw_dev, h->logw, h->J * 8, hipMemcpyDeviceToDevice, h->stream));
    if (loglik_dev) HIPCHECK(hipMemcpyAsync(loglik_dev, h->ll, h->J * 8, hipMemcpyDeviceToDevice, h->stream));
    if (logpi_dev) HIPCHECK(hipMemcpyAsync(logpi_dev, h->lp, h->J * 8, hipMemcpyDeviceToDevice, h->stream));
    if (grad_dev)
      HIPCHECK(grad_with_prior_run(h->theta, h->g, grad_dev, (int64_t)nd,
                                   (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std)), h->stream));
  });
}

smc_status smc_set_state(smc_t h, const float* theta_dev, const double* logw_dev, const double* logpi_dev,
                         uint64_t rng_counter) {
  return run([&]() {
    if (!h || !theta_dev) fail(SMC_ERR_ARG, "handle and theta_dev are required");
    HIPCHECK(hipMemcpyAsync(h->theta, theta_dev, (size_t)h->J * h->D * 4, hipMemcpyDeviceToDevice, h->stream));
    h->w_dirty = true;
    h->pm_have = false;
    ensure_cast(h);
    grad_pass(h, h->theta, h->m, h->lam, nullptr, h->ll, h->g, target_seg(h));
    h->rng_iter = rng_counter;
    // log pi and the initial weights at the restored particles
    initial_weighting(h);
    if (logpi_dev) HIPCHECK(hipMemcpyAsync(h->lp, logpi_dev, h->J * 8, hipMemcpyDeviceToDevice, h->stream));
    if (logw_dev) {
      double* s4 = h->stats + 8;
      HIPCHECK(normalise_run(logw_dev, h->J, h->logw, s4, h->stream, h->w));
      double host[4];
      HIPCHECK(hipMemcpyAsync(host, s4, sizeof(host), hipMemcpyDeviceToHost, h->stream));
      sync(h);
      double st[8] = {host[1], 0.0, 0.0, 0.0, host[2], host[1] < h->cfg.ess_frac * h->J ? 1.0 : 0.0,
                      host[3] == -INFINITY ? 1.0 : 0.0, 0.0};
      HIPCHECK(hipMemcpyAsync(h->stats, st, sizeof(st), hipMemcpyHostToDevice, h->stream));
      sync(h);
    }
  });
}

smc_status smc_get_rng_counter(smc_t h, uint64_t* counter) {
  if (!h || !counter) return SMC_ERR_ARG;
  *counter = h->rng_iter;
  return SMC_OK;
}

smc_status smc_set_noise(smc_t h, const float* momenta_dev) {
  return run([&]() {
    if (!h || !momenta_dev) fail(SMC_ERR_ARG, "null argument");
    if (!h->noise) h->noise = dalloc<float>(h->owned, (int64_t)h->J * h->D);
    HIPCHECK(hipMemcpyAsync(h->noise, momenta_dev, (size_t)h->J * h->D * 4, hipMemcpyDeviceToDevice, h->stream));
    h->noise_pending = true;
  });
}

smc_status smc_set_proposal_net(smc_t h, const float* params_dev, int32_t n_params, double h0) {
  return run([&]() {
    if (!h || !params_dev) fail(SMC_ERR_ARG, "null argument");
    if (n_params != mlp_n_params(h->G))
      fail(SMC_ERR_ARG, "proposal network needs " + std::to_string(mlp_n_params(h->G)) + " parameters");
    if (!(h0 > 0) || !isfinite(h0)) fail(SMC_ERR_ARG, "h0 must be finite and > 0");
    if (!h->pnet) h->pnet = dalloc<float>(h->owned, n_params);
    HIPCHECK(hipMemcpyAsync(h->pnet, params_dev, (size_t)n_params * 4, hipMemcpyDeviceToDevice, h->stream));
    h->pnet_n = n_params;
    h->h0 = h0;
  });
}

smc_status smc_set_proposal(smc_t h, int32_t proposal) {
  return run([&]() {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    if (proposal != SMC_PROPOSAL_FIXED && proposal != SMC_PROPOSAL_LEARNED) fail(SMC_ERR_ARG, "proposal");
    if (proposal == SMC_PROPOSAL_LEARNED) {
      if (h->cfg.leapfrog_steps != 1) fail(SMC_ERR_ARG, "the learned proposal is a Langevin move (leapfrog_steps 1)");
      if (!h->pnet) fail(SMC_ERR_STATE, "no proposal network set");
    }
    h->cfg.proposal = proposal;
  });
}

smc_status smc_proposal_features(smc_t h, double kk, double mm, double* feat_dev) {
  return run([&]() {
    if (!h || !feat_dev) fail(SMC_ERR_ARG, "null argument");
    const float ipv = (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std));
    HIPCHECK(features_run(h->net, h->theta, h->g, h->ll, ipv, (double)h->m, kk, mm, feat_dev, nullptr, h->G,
                          h->stream));
  });
}

smc_status smc_proposal_targets(smc_t h, int64_t m_k, double lambda_k, const double* h_grid, int32_t n_grid,
                                double k_over_K_, double accept_power, float* feat_dev, float* target_dev) {
  return run([&]() {
    if (!h || !h_grid || !feat_dev || !target_dev) fail(SMC_ERR_ARG, "null argument");
    if (!(accept_power >= 0) || !isfinite(accept_power)) fail(SMC_ERR_ARG, "accept_power must be finite and >= 0");
    if (n_grid < 1 || n_grid > 64) fail(SMC_ERR_ARG, "n_grid must be in [1, 64]");
    if (m_k < h->m || m_k > h->n_data) fail(SMC_ERR_ARG, "m_k must satisfy previous m <= m_k <= n_data");
    if (!(lambda_k > 0) || !isfinite(lambda_k)) fail(SMC_ERR_ARG, "lambda_k must be finite and > 0");
    for (int i = 0; i < n_grid; ++i)
      if (!(h_grid[i] > 0) || !isfinite(h_grid[i])) fail(SMC_ERR_ARG, "grid step sizes must be finite and > 0");
    const int J = h->J;
    const int64_t nd = (int64_t)J * h->D;
    if (!h->th_bak) {
      h->th_bak = dalloc<float>(h->owned, nd);
      h->g_bak = dalloc<float>(h->owned, nd);
      h->ll_bak = dalloc<double>(h->owned, J);
      h->ll1 = dalloc<double>(h->owned, J);
      h->phalf = dalloc<double>(h->owned, J);
      h->best_score = dalloc<double>(h->owned, J);
      h->best_logh = dalloc<double>(h->owned, J);
      h->lp0 = dalloc<double>(h->owned, J);
    }
    ensure_cast(h);
    if (m_k != h->m || lambda_k != h->lam || h->seg_split != INT64_MAX) {
      // the trace targets use the one-segment target
      h->m = m_k;
      h->lam = lambda_k;
      h->seg_split = INT64_MAX;
      h->lam_b = lambda_k;
      grad_pass(h, h->theta, m_k, lambda_k, nullptr, h->ll, h->g, target_seg(h));
    }
    const float ipv = (float)(1.0 / (h->cfg.prior_std * h->cfg.prior_std));
    const double i2pv = 0.5 / (h->cfg.prior_std * h->cfg.prior_std);
    HIPCHECK(features_run(h->net, h->theta, h->g, h->ll, ipv, (double)h->m, k_over_K_, (double)h->m / h->n_data,
                          h->feat, h->gsum, h->G, h->stream));
    HIPCHECK(f64_to_f32_run(h->feat, (int64_t)J * 4, feat_dev, h->stream));
    HIPCHECK(sq_norm_rows_run(h->theta, J, h->D, h->tsq, h->stream));
    HIPCHECK(lp_current_run(h->ll, h->tsq, J, h->lam, i2pv, h->lp0, h->stream));
    HIPCHECK(hipMemcpyAsync(h->th_bak, h->theta, nd * 4, hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipMemcpyAsync(h->g_bak, h->g, nd * 4, hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipMemcpyAsync(h->ll_bak, h->ll, J * 8, hipMemcpyDeviceToDevice, h->stream));
    const int64_t ev = h->grad_evals;
    for (int i = 0; i < n_grid; ++i) {
      if (i > 0) {
        HIPCHECK(hipMemcpyAsync(h->theta, h->th_bak, nd * 4, hipMemcpyDeviceToDevice, h->stream));
        HIPCHECK(hipMemcpyAsync(h->g, h->g_bak, nd * 4, hipMemcpyDeviceToDevice, h->stream));
      }
      // one preconditioning-free Langevin trial with step h_grid[i] and the shared noise
      MoveArgs ma = move_args(h, MOVE_FIRST);
      ma.h = (float)h_grid[i];
      ma.ctr_iter = (uint32_t)(h->rng_iter ^ 0x80000000u);
      if (h->noise_pending) ma.noise = h->noise;
      HIPCHECK(move_run(ma, h->stream));
      HIPCHECK(sq_norm_rows_run(h->P, J, h->D, h->phalf, h->stream));
      grad_pass(h, h->theta, h->m, h->lam, nullptr, h->ll1, h->g);
      MoveArgs mb = move_args(h, MOVE_LAST);
      mb.h = (float)h_grid[i];
      HIPCHECK(move_run(mb, h->stream));
      HIPCHECK(trial_score_run(h->part, J, h->nblk, h->ll1, h->lp0, h->lam, i2pv, h_grid[i], accept_power, h->phalf,
                               h->best_score, h->best_logh, i == 0 ? 1 : 0, h->stream));
    }
    h->grad_evals = ev;
    h->noise_pending = false;
    HIPCHECK(hipMemcpyAsync(h->theta, h->th_bak, nd * 4, hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipMemcpyAsync(h->g, h->g_bak, nd * 4, hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipMemcpyAsync(h->ll, h->ll_bak, J * 8, hipMemcpyDeviceToDevice, h->stream));
    h->w_dirty = true;
    ensure_cast(h);
    HIPCHECK(targets_run(h->best_logh, h->gsum, h->group_n, J, h->G, h->cfg.step_size, 0.95, target_dev, h->stream));
  });
}

int32_t smc_mlp_n_params(int32_t n_groups) { return n_groups < 1 || n_groups > 2 * SMC_MAX_LAYERS ? -1 : mlp_n_params(n_groups); }

smc_status smc_mlp_forward(const float* params_dev, const float* feat_dev, int64_t R, int32_t n_groups, float* out_dev,
                           int32_t mode, double h0, int32_t bf16, void* hip_stream) {
  return run([&]() {
    if (!params_dev || !feat_dev || !out_dev) fail(SMC_ERR_ARG, "null argument");
    if (R < 0 || n_groups < 1 || n_groups > 2 * SMC_MAX_LAYERS || (mode != 0 && mode != 1))
      fail(SMC_ERR_ARG, "bad size or mode");
    HIPCHECK(mlp_set_smem_limits());
    HIPCHECK(mlp_infer_run(params_dev, feat_dev, 0, R, n_groups, out_dev, mode, (float)h0, bf16 ? 1 : 0,
                           (hipStream_t)hip_stream));
  });
}


smc_status smc_mlp_grad(const float* params_dev, const float* feat_dev, const float* target_dev, int64_t R,
                        int32_t n_groups, float* grad_dev, double* loss, void* hip_stream) {
  return run([&]() {
    if (!params_dev || !feat_dev || !target_dev || !grad_dev) fail(SMC_ERR_ARG, "null argument");
    mlp_steps(const_cast<float*>(params_dev), nullptr, feat_dev, target_dev, R, n_groups, 1, 1, 0.0, grad_dev, loss,
              (hipStream_t)hip_stream);
  });
}

smc_status smc_mlp_train(float* params_dev, float* adam_dev, const float* feat_dev, const float* target_dev, int64_t R,
                         int32_t n_groups, int32_t first_step, int32_t n_steps, double lr, double* loss,
                         void* hip_stream) {
  return run([&]() {
    if (!params_dev || !adam_dev || !feat_dev || !target_dev) fail(SMC_ERR_ARG, "null argument");
    if (first_step < 1 || n_steps < 1 || !(lr > 0)) fail(SMC_ERR_ARG, "first_step, n_steps >= 1 and lr > 0");
    mlp_steps(params_dev, adam_dev, feat_dev, target_dev, R, n_groups, first_step, n_steps, lr, nullptr, loss,
              (hipStream_t)hip_stream);
  });
}

smc_status smc_mlp_train_noalloc(float* params_dev, float* adam_dev, const float* feat_dev, const float* target_dev,
                                 int64_t R, int32_t n_groups, int32_t first_step, int32_t n_steps, double lr,
                                 double* loss_dev, void* hip_stream) {
  return run([&]() {
    if (!params_dev || !adam_dev || !feat_dev || !target_dev) fail(SMC_ERR_ARG, "null argument");
    if (first_step < 1 || n_steps < 1 || !(lr > 0)) fail(SMC_ERR_ARG, "first_step, n_steps >= 1 and lr > 0");
    mlp_steps_noalloc(params_dev, adam_dev, feat_dev, target_dev, R, n_groups, first_step, n_steps, lr, loss_dev,
                      (hipStream_t)hip_stream);
  });
}

smc_status smc_nn_forward(smc_t h, const float* theta_dev, int64_t m, double* ll_dev) {
  return run([&]() {
    if (!h || !theta_dev || !ll_dev) fail(SMC_ERR_ARG, "null argument");
    if (m < 1 || m > h->n_data) fail(SMC_ERR_ARG, "m must be in [1, n_data]");
    HIPCHECK(cast_run(h->net, theta_dev, nullptr, h->stream));
    h->w_dirty = true;
    grad_pass(h, theta_dev, m, 1.0, nullptr, ll_dev, nullptr);
  });
}

smc_status smc_nn_backward(smc_t h, const float* theta_dev, int64_t m, const double* scale_dev, double* ll_dev,
                           float* grad_dev) {
  return run([&]() {
    if (!h || !theta_dev || !grad_dev) fail(SMC_ERR_ARG, "null argument");
    if (m < 1 || m > h->n_data) fail(SMC_ERR_ARG, "m must be in [1, n_data]");
    HIPCHECK(cast_run(h->net, theta_dev, nullptr, h->stream));
    h->w_dirty = true;
    double* ll = ll_dev ? ll_dev : h->extra;
    const int64_t ev = h->grad_evals;
    grad_pass(h, theta_dev, m, 1.0, scale_dev, ll, grad_dev);
    h->grad_evals = ev;  // not part of the sampler's own accounting
  });
}

smc_status smc_profile(smc_t h, int32_t enable) {
  if (!h) return SMC_ERR_ARG;
  h->prof_on = enable != 0;
  return SMC_OK;
}

smc_status smc_profile_read(smc_t h, double* total_ms, int64_t* launches, double* flops, double* bytes) {
  return run([&]() {
    if (!h) fail(SMC_ERR_ARG, "null handle");
    sync(h);
    double t[SMC_K_COUNT] = {0}, f[SMC_K_COUNT] = {0}, b[SMC_K_COUNT] = {0};
    int64_t n[SMC_K_COUNT] = {0};
    for (const ProfRec& r : h->prof_recs) {
      float ms = 0.0f;
      HIPCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      t[r.cls] += ms;
      n[r.cls] += 1;
      f[r.cls] += r.flops;
      b[r.cls] += r.bytes;
      h->prof_pool.push_back(r.a);
      h->prof_pool.push_back(r.b);
    }
    h->prof_recs.clear();
    for (int k = 0; k < SMC_K_COUNT; ++k) {
      if (total_ms) total_ms[k] = t[k];
      if (launches) launches[k] = n[k];
      if (flops) flops[k] = f[k];
      if (bytes) bytes[k] = b[k];
    }
  });
}

smc_status smc_normalise(const double* logw_dev, int32_t J, double* logw_out_dev, double* stats_dev,
                         void* hip_stream) {
  return run([&]() {
    if (!logw_dev || !logw_out_dev || !stats_dev) fail(SMC_ERR_ARG, "null argument");
    if (J < 1 || J > MAX_J) fail(SMC_ERR_ARG, "J out of range");
    HIPCHECK(normalise_run(logw_dev, J, logw_out_dev, stats_dev, (hipStream_t)hip_stream));
  });
}

smc_status smc_systematic_resample(const double* w_dev, int32_t J, double u, int32_t* ancestors_dev,
                                   int32_t* placement_dev, void* hip_stream) {
  return run([&]() {
    if (!w_dev || !ancestors_dev) fail(SMC_ERR_ARG, "null argument");
    if (J < 1 || J > MAX_J) fail(SMC_ERR_ARG, "J out of range");
    if (!(u >= 0.0 && u < 1.0)) fail(SMC_ERR_ARG, "u must be in [0, 1)");
    HIPCHECK(systematic_run(w_dev, J, u, ancestors_dev, placement_dev, (hipStream_t)hip_stream));
  });
}

smc_status smc_multinomial_resample(const double* w_dev, int32_t J, const double* u_dev, int32_t* ancestors_dev,
                                    int32_t* placement_dev, void* hip_stream) {
  return run([&]() {
    if (!w_dev || !u_dev || !ancestors_dev) fail(SMC_ERR_ARG, "null argument");
    if (J < 1 || J > MAX_J) fail(SMC_ERR_ARG, "J out of range");
    HIPCHECK(multinomial_run(w_dev, J, u_dev, ancestors_dev, placement_dev, (hipStream_t)hip_stream));
  });
}

smc_status smc_philox(uint32_t key0_, uint32_t key1_, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n_blocks,
                      uint32_t* out_dev, void* hip_stream) {
  return run([&]() {
    if (!out_dev || n_blocks < 0 || n_blocks > ((int64_t)1 << 32)) fail(SMC_ERR_ARG, "bad argument");
    HIPCHECK(philox_run(key0_, key1_, c1, c2, c3, n_blocks, out_dev, (hipStream_t)hip_stream));
  });
}

}  // extern "C"
