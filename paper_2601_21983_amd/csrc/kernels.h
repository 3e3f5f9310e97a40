// Launch interfaces of the SMC kernels (internal to libsmc).
#pragma once

#include "common.h"
#include "gemm.h"

namespace smc {

constexpr int MAX_LAYERS = 8;
constexpr int MAX_J = 4096;      // population size handled by the single-workgroup kernels
constexpr int MOVE_ELEMS = 1024; // parameters per move workgroup (256 threads x 4)

enum { HEAD_TRAIN = 0, HEAD_FORWARD = 1, HEAD_PREDICT = 2 };
enum { MOVE_FIRST = 0, MOVE_MID = 1, MOVE_LAST = 2 };
enum { TAG_MOMENTUM = 1, TAG_RESAMPLE_U = 2, TAG_PRIOR = 3, TAG_RESAMPLE_MULTI = 4 };
enum { RESAMPLE_SYSTEMATIC = 0, RESAMPLE_MULTINOMIAL = 1 };

struct HeadArgs {
  const void* A = nullptr;          // activation (j, m, h) at A + j*sAj + m*sAm + h
  int a_f32 = 0;                    // split BF16: A holds FP32 values, split into hi/lo when staged
  int64_t sAj = 0, sAm = 0;
  const float* theta = nullptr;     // master parameters [J x D]
  int64_t D = 0, offL = 0;          // output-layer block offset
  int H = 0, C = 0, J = 0;
  int m_valid = 0;                  // valid samples of this chunk
  int64_t c0 = 0;                   // first sample of this chunk (label index base)
  int tiles_per_split = 1, nsplit = 1;
  const int32_t* ylab = nullptr;
  const float* yreal = nullptr;
  int likelihood = 0;
  float inv_var = 1.0f, gauss_c = 0.0f;
  double lambda = 1.0;
  const double* scale = nullptr;    // per-particle gradient scale (overrides lambda and lambda_b)
  // two-segment target: samples with global index >= m_split weigh lambda_b instead of lambda,
  // and their log-likelihood is also summed on its own (ll_acc_b, through llpart_b)
  int64_t m_split = INT64_MAX;
  double lambda_b = 1.0;
  double* llpart_b = nullptr;       // [J x nsplit]
  double* ll_acc_b = nullptr;       // [J] or null
  int act = 0;
  void* dT = nullptr;               // delta_{L-1} transposed: dT + j*sdTj + h*sdTh + m
  int64_t sdTj = 0, sdTh = 0;
  void* dR = nullptr;               // optional row layout: dR + j*sdRj + m*sdRm + h
  int64_t sdRj = 0, sdRm = 0;
  double* llpart = nullptr;         // [J x nsplit]
  float* dWpart = nullptr;          // [J x nsplit x C(H+1)]
  double* ll_acc = nullptr;         // [J]
  float* grad = nullptr;            // [J x D]
  int beta = 0;                     // 0: overwrite totals, 1: accumulate (later chunks)
  float* logp = nullptr;            // predict: logp[(j*ld_logp + c0 + m)*C + c]
  int64_t ld_logp = 0;
};

// operand types of the output-layer kernel
enum HeadType { HEAD_F32 = 0, HEAD_BF16 = 1, HEAD_BF16_SPLIT = 2 };
bool head_supported(int H, int C, int type);
hipError_t head_run(const HeadArgs& a, int mode, int type, hipStream_t s);
// Fused layer-1 GEMM + output layer for networks with one hidden layer (BF16 or split-BF16
// operands): p describes z1 = X W1^T for the chunk (A = X rows, B = the weight copy with 128
// rows per particle, bias = b1); a.nsplit must equal ceil(p.M / 256).
bool fwd_head_supported(int H, int C);
hipError_t fwd_head_run(const GemmParams& p, const HeadArgs& a, int mode, int split, int act, hipStream_t s);
hipError_t head_set_smem_limits();

// Convolutional network dimensions (conv3x3 C1 -> conv3x3 C2 -> 2x2 avgpool -> linear ncls).
struct CnnDims {
  int H = 0, W = 0, Cin = 0, C1 = 0, C2 = 0, ncls = 0;
  int Hp = 0, Wp = 0, HW = 0;
  int K1 = 0, K1p = 0;  // conv1 patch length 9 Cin and its padded row length
  int K2 = 0;           // conv2 patch length 9 C1
  int F3 = 0;           // linear-layer inputs Hp Wp C2
};

struct CnnLLArgs {
  const float* logits = nullptr;  // [J x mc x ncls] (before the bias)
  const float* bias = nullptr;    // linear-layer bias [J x ncls]
  const int32_t* ylab = nullptr;
  int64_t c0 = 0;
  int mc = 0, mcv = 0, ncls = 0, mode = HEAD_TRAIN, beta = 0;
  double lambda = 1.0;
  const double* scale = nullptr;  // per-particle gradient scale (overrides lambda and lambda_b)
  int64_t m_split = INT64_MAX;    // samples from m_split on weigh lambda_b (two-segment target)
  double lambda_b = 1.0;
  double* ll_acc_b = nullptr;     // [J] log-likelihood of samples >= m_split, or null
  void* d3 = nullptr;             // [J x mc x 16] operand type
  double* ll_acc = nullptr;       // [J]
  float* logp = nullptr;          // predict: logp[(j*ld_logp + c0 + n)*ncls + c]
  int64_t ld_logp = 0;
};

hipError_t cnn_im2col_x_run(const void* X, int64_t xld, int64_t c0, int mcv, const CnnDims& d, void* p1, int bf16,
                            hipStream_t s);
hipError_t cnn_im2col_xt_run(const void* X, int64_t xld, int64_t c0, int mcv, const CnnDims& d, int64_t ld, void* p1t,
                             int bf16, hipStream_t s);
hipError_t cnn_im2col_a_run(const void* act1, int64_t sA, int mcv, const CnnDims& d, int J, void* big, int64_t sB,
                            int bf16, hipStream_t s);
hipError_t cnn_im2col_at_run(const void* act1, int64_t sA, int mcv, const CnnDims& d, int J, int64_t ld, void* bigT,
                             int64_t sB, int bf16, hipStream_t s);
hipError_t cnn_pool_run(const void* act2, int64_t sA, int mcv, const CnnDims& d, int J, void* pooled, int64_t sP,
                        int bf16, hipStream_t s);
hipError_t cnn_ll_run(const CnnLLArgs& a, int J, int bf16, hipStream_t s);
// g[j][o N + n] (+)= sum_{s < S} part[s][j C1 + o][n]: the K-slice partials of the conv1 gradient
hipError_t cnn_slice_sum_run(const float* part, int S, int M, int N, int C1, float* g, int64_t D, int beta,
                             hipStream_t s);
hipError_t cnn_dw3_run(const void* d3, const void* pooled, int64_t sP, int mc, int mcv, int F3, int ncls, int J,
                       float* g, int64_t D, int64_t off, int beta, int bf16, hipStream_t s);
hipError_t cnn_unpool_run(const void* dpool, int64_t sP, const void* act2, int64_t sA, int mcv, const CnnDims& d,
                          int J, int64_t ld, void* d2, void* d2t, int bf16, hipStream_t s);
// implicit-GEMM conv2 for BF16 networks on 32-pixel-wide images with C1 = 16, C2 = 32 (no patch
// matrices): the forward writes act2 [j][r][C2] and the 2x2-pooled features [j][n][F3]; the
// backward kernels form the conv2 output error from act2 and the pooled-feature error dpool
// [j][n][F3] themselves; the input error writes d1t [j C1 + c][ld] masked by 1{act1 > 0}, using
// the transposed weight copy
bool cnn_implicit_supported(const CnnDims& d, int bf16);
hipError_t cnn_conv2_fwd_implicit_run(const void* act1, int64_t sA1, const void* w2, int64_t ldw, const float* b2,
                                      void* act2, int64_t sA2, void* pooled, int64_t sP, int mcv, const CnnDims& d,
                                      int J, hipStream_t s);
// the [W2 | b2] gradient as an implicit GEMM over the chunk's pixels: FP32 partials part [J][G][4][32 x 145]
// (G = cnn_wgrad_groups, at most CNN_WGRAD_GROUPS) summed in a fixed order into g[j][off ..] (beta: accumulate)
constexpr int CNN_WGRAD_GROUPS = 16;
int cnn_wgrad_groups(int mcv, const CnnDims& d);
hipError_t cnn_conv2_wgrad_implicit_run(const void* act2, int64_t sA2, const void* dpool, int64_t sP,
                                        const void* act1, int64_t sA1, int mcv, const CnnDims& d, int J, float* part,
                                        float* g, int64_t D, int64_t off, int beta, hipStream_t s);
hipError_t cnn_conv2_dgrad_implicit_run(const void* act2, int64_t sA2, const void* dpool, int64_t sP, const void* wT,
                                        int64_t ldwT, const void* act1, int64_t sA1, void* d1t, int64_t ld, int mcv,
                                        const CnnDims& d, int J, hipStream_t s);
hipError_t cnn_col2im_run(const void* dp2, int64_t sB, const void* act1, int64_t sA, int mcv, const CnnDims& d, int J,
                          int64_t ld, void* d1t, int bf16, hipStream_t s);

// LeNet-5 convolution stack (lenet.hip): conv kxk "same" (C1) -> act -> 2x2 average pool ->
// conv kxk "valid" (C2) -> act -> 2x2 average pool -> F features; FP32 operands.
constexpr int LENET_CMAX = 8;  // Cin and C1 at most this
struct LenetDims {
  int H = 0, W = 0, Cin = 0, k = 0, pad = 0, C1 = 0, C2 = 0;
  int Hp = 0, Wp = 0;  // after the first pool
  int H2 = 0, W2 = 0;  // second convolution's output
  int Hq = 0, Wq = 0;  // after the second pool
  int K1 = 0, K2 = 0;  // k k Cin, k k C1
  int F = 0;           // Hq Wq C2
  int Dconv = 0;       // C1 (K1 + 1) + C2 (K2 + 1): the conv blocks at the start of each theta row
  int ns1 = 1;         // row slices of the conv1 weight-gradient items
  int Mimg = 0;        // saved per image for the backward: the conv2 activations a2 [C2][H2][W2]
};
size_t lenet_smem_bytes(const LenetDims& d, bool bwd);
// workgroups of lenet_bwd_kernel resident on the current device at once (0 if unknown)
int lenet_bwd_resident(const LenetDims& d, int act);
// feat[j][n][f] (stride sF per particle) and, if featT, featT[j][f][n] ([(F+1) x ldT] per
// particle, the ones row f = F untouched) for images n < rows of the chunk starting at global
// row c0 of X; rows mcv <= n < rows are written as zeros.  If maps, also each image's conv2
// activations at maps[j][n][Mimg] (stride sM per particle) for the backward.  ipb images per
// workgroup.
hipError_t lenet_fwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int rows, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, float* feat, int64_t sF, float* featT,
                         int64_t ldT, float* maps, int64_t sM, hipStream_t s);
// Conv weight gradients of the chunk from the features' error dfeat[j][n][f] and the conv2
// activations the forward saved (conv1 is recomputed): per-block partials part[j][blk][Dconv] (part_blocks >= ceil(mcv / ipb) per
// particle), then g[j][0, Dconv) (+)= their sum in block order (beta = 1 accumulates).
hipError_t lenet_bwd_run(const float* X, int64_t xld, int64_t c0, int mcv, int ipb, const LenetDims& d,
                         const float* theta, int64_t D, int J, int act, const float* dfeat, int64_t sF,
                         const float* maps, int64_t sM, float* part, int part_blocks, float* g, int beta,
                         hipStream_t s);

// Network shape shared by the elementwise kernels.
struct NetShape {
  int L = 0;
  int nin[MAX_LAYERS] = {0}, nout[MAX_LAYERS] = {0};
  int64_t off[MAX_LAYERS + 1] = {0};  // parameter offsets of each layer block; off[L] = D
  int ldw[MAX_LAYERS] = {0};          // padded row length of the GEMM weight copy
  int rowpad[MAX_LAYERS] = {0};       // rows per particle in the GEMM weight copy (>= nout, extra rows zero)
  float rinv[MAX_LAYERS] = {0};       // 1 / (nin + 1)
  void* w[MAX_LAYERS] = {nullptr};    // GEMM weight copy [J*rowpad x ldw] (operand type)
  float* bias[MAX_LAYERS] = {nullptr};// [J*nout]
  int64_t D = 0;
  int J = 0;
  int bf16 = 0;
  int split = 0;                      // BF16 copies hold rows [hi | lo] of 2*ldw elements
};

// Store parameter v of particle j (layer l, output unit o, input i; i == nin is the
// bias) into the GEMM copy of that layer.
__device__ __forceinline__ void weight_copy_store(const NetShape& n, int j, int l, int o, int i, float v) {
  if (i >= n.nin[l]) {
    n.bias[l][(int64_t)j * n.nout[l] + o] = v;
    return;
  }
  const int64_t r = (int64_t)j * n.rowpad[l] + o;
  if (!n.bf16) {
    ((float*)n.w[l])[r * n.ldw[l] + i] = v;
    return;
  }
  __bf16* w = (__bf16*)n.w[l];
  const __bf16 hi = to_bf16(v);
  if (n.split) {
    w[r * 2 * n.ldw[l] + i] = hi;
    w[r * 2 * n.ldw[l] + n.ldw[l] + i] = to_bf16(v - from_bf16(hi));
  } else {
    w[r * n.ldw[l] + i] = hi;
  }
}

struct MoveArgs {
  NetShape net;
  float* theta = nullptr;
  float* P = nullptr;
  const float* g = nullptr;      // gradient of the scaled log-likelihood (prior added here)
  const float* noise = nullptr;  // injected standard normals [J x D] (FIRST), or null
  double* part = nullptr;        // [3][J][nblk] per-workgroup sums: |xi|^2, |theta|^2, |P_end|^2
  int nblk = 0;
  int mode = MOVE_FIRST;
  float h = 0.0f;
  float inv_prior_var = 1.0f;
  uint32_t key0 = 0, key1 = 0, ctr_iter = 0;
  int cast = 1;                  // refresh the GEMM copy of theta
};
hipError_t move_run(const MoveArgs& a, hipStream_t s);

// Build the GEMM copy of theta (and the bias copy) for every layer; with
// `placement` only particles j with placement[j] != j are refreshed.
hipError_t cast_run(const NetShape& net, const float* theta, const int32_t* placement, hipStream_t s);

struct WeightArgs {
  int J = 0;
  int nblk = 0;
  int init = 0;                  // initial weighting (Eq. init_weight)
  double lambda = 1.0;
  double inv_2prior_var = 0.5;
  double ess_frac = 0.5;
  const double* ll = nullptr;    // [J] subset log-likelihood at the new state
  const double* ll_b = nullptr;  // [J] its second-segment part (two-segment target), or null
  double lambda_b = 1.0;         // weight of the second segment
  const double* part = nullptr;  // [3][J][nblk]
  const double* extra = nullptr; // [J] extra log-weight term (learned proposal), or null
  const double* tsq = nullptr;   // [J] |theta|^2 when part is null (initial weighting)
  int no_kinetic = 0;            // ignore the momentum terms (learned move supplies `extra`)
  double* lp = nullptr;          // [J] cached log pi (in: previous, out: new)
  double* logw = nullptr;        // [J] normalised log-weights (in/out)
  double* w = nullptr;           // [J] normalised weights (out)
  double* stats = nullptr;       // [8] out
};
// stats layout
enum { ST_ESS = 0, ST_LOGZ = 1, ST_MEANLL = 2, ST_MAXLL = 3, ST_NONFINITE = 4, ST_RECOMMEND = 5, ST_ALLBAD = 6,
       ST_RESAMPLED = 7 };
hipError_t weight_run(const WeightArgs& a, hipStream_t s);

struct ResampleArgs {
  int J = 0;
  int mode = 0;                  // 0 if needed, 1 always, 2 never
  double ess_frac = 0.5;
  const double* u_dev = nullptr; // device scalar u (or null: draw with Philox)
  int scheme = 0;                // RESAMPLE_SYSTEMATIC or RESAMPLE_MULTINOMIAL
  const double* u_arr = nullptr; // multinomial: device [J] uniforms (or null: Philox per particle)
  uint32_t key0 = 0, key1 = 0, ctr_iter = 0;
  double* w = nullptr;           // [J] normalised weights (in; reset to 1/J)
  double* logw = nullptr;        // [J] (reset to -log J)
  double* stats = nullptr;       // [8] (ESS read; ST_RESAMPLED written)
  int32_t* ancestors = nullptr;  // [J] sorted ancestors (identity if not resampled)
  int32_t* placement = nullptr;  // [J]
  double* sc[4] = {nullptr, nullptr, nullptr, nullptr};  // per-particle scalars gathered in place
};
hipError_t resample_run(const ResampleArgs& a, hipStream_t s);
hipError_t kernels_set_smem_limits();
// gather rows of the [J x D] arrays in place according to placement
hipError_t gather_rows_run(int J, int64_t D, const int32_t* placement, float* a0, float* a1, hipStream_t s);

hipError_t normalise_run(const double* logw, int J, double* out, double* stats, hipStream_t s,
                         double* wout = nullptr);
// {E[Omega^], Var(Omega^), E[Omega], Cov(Omega, Omega^)} with Omega^ = -ll_b, Omega = -(ll - ll_b)
hipError_t segment_moments_run(const double* w, const double* ll, const double* ll_b, int J, double* out,
                               hipStream_t s);
hipError_t systematic_run(const double* w, int J, double u, int32_t* anc, int32_t* placement, hipStream_t s);
hipError_t multinomial_run(const double* w, int J, const double* u_arr, int32_t* anc, int32_t* placement,
                           hipStream_t s);
hipError_t philox_run(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
                      hipStream_t s);
hipError_t prior_draw_run(float* theta, int J, int64_t D, float prior_std, uint32_t k0, uint32_t k1, hipStream_t s);

hipError_t mean_change_run(const double* cur, const double* prev, int64_t D, double* out2, hipStream_t s);
hipError_t posterior_mean_run(const float* theta, const double* w, int J, int64_t D, double* out, hipStream_t s);

// combine per-particle log-probabilities into the predictive mixture for samples [0, n)
hipError_t predictive_run(const float* logp, int64_t ld_logp, const double* logw, int J, int C, int64_t n,
                          const int32_t* y, float* probs, double* per_sample /*[n x 2]*/, hipStream_t s);
hipError_t predictive_finish_run(const double* per_sample, int64_t n, double* out2, hipStream_t s);

// fill helpers
hipError_t fill_f64_run(double* p, int64_t n, double v, hipStream_t s);
hipError_t grad_with_prior_run(const float* theta, const float* g, float* out, int64_t n, float inv_prior_var,
                               hipStream_t s);
hipError_t sq_norm_rows_run(const float* a, int J, int64_t D, double* out, hipStream_t s);
hipError_t lp_current_run(const double* ll, const double* tsq, int J, double lambda, double inv_2pv, double* out,
                          hipStream_t s);
hipError_t f64_to_f32_run(const double* in, int64_t n, float* out, hipStream_t s);

// ---------------------------------------------------------------- learned proposal
struct LearnedMoveArgs {
  NetShape net;
  float* theta = nullptr;
  float* P = nullptr;            // FIRST writes theta' - theta here; LAST reads it
  const float* g = nullptr;
  const float* noise = nullptr;
  const float* scales = nullptr; // [J x NO]: h, m_1..m_G at the state the kernel starts from
  int NO = 0;
  double* part = nullptr;        // [3][J][nblk]
  int nblk = 0;
  int mode = MOVE_FIRST;
  float inv_prior_var = 1.0f;
  uint32_t key0 = 0, key1 = 0, ctr_iter = 0;
};
hipError_t mlp_set_smem_limits();
int mlp_n_params(int G);
hipError_t mlp_infer_run(const float* params, const void* feat, int feat_f64, int64_t R, int G, float* out, int mode,
                         float h0, int bf16, hipStream_t s);
hipError_t mlp_train_step_run(float* params, float* adam, const float* feat, const float* tgt, int64_t R, int G,
                              float* grad_part, double* loss_part, int step, float lr, float* grad_out,
                              double* loss_out, hipStream_t s);
hipError_t learned_move_run(const LearnedMoveArgs& a, hipStream_t s);
hipError_t learned_extra_run(const float* sc0, const float* sc1, int NO, const double* part, int J, int nblk,
                             const int64_t* group_n, int64_t D, double* extra, hipStream_t s);
hipError_t features_run(const NetShape& n, const float* theta, const float* g, const double* ll, float ipv, double m,
                        double k_over_K, double m_over_N, double* feat, double* gsum, int G, hipStream_t s);
hipError_t trial_score_run(const double* part, int J, int nblk, const double* ll1, const double* lp0, double lambda,
                           double inv_2pv, double h, double accept_power, const double* phalf_sq, double* best_score,
                           double* best_logh,
                           int first, hipStream_t s);
hipError_t targets_run(const double* best_logh, const double* gsum, const int64_t* group_n, int J, int G, double h0,
                       double clip, float* tgt, hipStream_t s);

}  // namespace smc
