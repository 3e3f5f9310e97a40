/*
 * smc.h - C ABI of the MI355X (gfx950) data-annealed SMC sampler for
 * Bayesian neural-network posteriors.
 *
 * The method (Millard, Murphy, Green, Maskell, "Investigating Batch Inference
 * in a Sequential Monte Carlo Framework for Neural Networks"):
 *   - J weighted particles theta_j target pi(theta) ~ p(y_{1:N} | theta) q0(theta)
 *     (Section 2);
 *   - each iteration moves the particles with S leapfrog steps of a
 *     gradient-based Markov kernel (Section 2.1, Eqs. mom_first, pos_update,
 *     mom_second; Langevin dynamics is S = 1) and reweights them with the
 *     reversed-momentum L-kernel (Eq. weight_update_fp);
 *   - weights are normalised (Eq. normalise), the effective sample size is
 *     computed (Eq. jeff) and the population is resampled when it drops below
 *     a fraction of J (Section 2);
 *   - log-likelihoods and gradients are evaluated on a growing prefix
 *     y_{1:M_k} of the data and scaled by lambda_k = N / M_k
 *     (Section 3, Eq. approx-grad; data annealing, Section 3.1).
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device (HBM) pointers; all other pointers are
 *     host pointers.  Sizes are element counts.
 *   - All device work is enqueued on the HIP stream given to smc_init (or to
 *     the stateless call).  Calls that return values through host pointers
 *     synchronise that stream; calls without host outputs do not.
 *   - Buffers passed in belong to the caller.  smc_init borrows x_dev/y_dev
 *     only for the duration of the call (it makes its own padded copies); the
 *     library owns all particle state and frees it in smc_destroy.
 *   - No exception or abort crosses the ABI: every function returns an
 *     smc_status; smc_status_string gives a message, smc_last_error gives the
 *     detail of the most recent failure on the calling thread.
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Parameter layout of one particle (D floats): for each layer l = 1..L with
 * n_{l-1} inputs and n_l outputs, the block [W_l | b_l] of shape
 * [n_l x (n_{l-1} + 1)], row-major: each output unit's n_{l-1} weights
 * followed by its bias.  Populations are [J x D] row-major float32.  The
 * convolutional network and LeNet-5 (smc_config.model_kind) use the same
 * per-layer [W | b] blocks with the weight orders given with smc_config.
 */
#ifndef SMC_H_
#define SMC_H_

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SMC_API __attribute__((visibility("default")))
#else
#define SMC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum smc_status {
  SMC_OK = 0,
  SMC_ERR_ARG = 1,          /* invalid argument (size, pointer, mode, subset order) */
  SMC_ERR_OOM = 2,          /* device allocation failed */
  SMC_ERR_DEVICE = 3,       /* a HIP call failed */
  SMC_ERR_STATE = 4,        /* call not valid in the handle's current state */
  SMC_ERR_NONFINITE = 5,    /* every particle has a non-finite log-weight */
  SMC_ERR_UNSUPPORTED = 6,  /* configuration not supported by the library */
  SMC_ERR_NOLIB = 7         /* reserved for bindings: library not loaded */
} smc_status;

enum { SMC_ACT_TANH = 0, SMC_ACT_RELU = 1 };
enum { SMC_LIK_CATEGORICAL = 0, SMC_LIK_GAUSSIAN = 1 };
/*
 * GEMM operand precision (accumulation is always FP32).  SMC_PREC_BF16X3 is split
 * BF16: weights and hidden activations are carried as hi = bf16(v) and
 * lo = bf16(v - hi) and multiplied as hi*hi + hi*lo + lo*hi on the BF16 matrix
 * cores, the inputs X as one BF16 value.  Rounding X is the same at every
 * parameter value and cancels in the log-likelihood differences of the weight
 * update; the split operands keep the per-state rounding of the other factors
 * about 2^8 times smaller than plain BF16, whose log-weight increments otherwise
 * carry several nats of rounding noise at MNIST scale.  At most one hidden layer.
 */
enum { SMC_PREC_FP32 = 0, SMC_PREC_BF16 = 1, SMC_PREC_BF16X3 = 2 };
enum { SMC_PROPOSAL_FIXED = 0, SMC_PROPOSAL_LEARNED = 1 };
enum { SMC_MODEL_MLP = 0, SMC_MODEL_CNN = 1, SMC_MODEL_LENET = 2 };
enum { SMC_RESAMPLE_IF_NEEDED = 0, SMC_RESAMPLE_ALWAYS = 1, SMC_RESAMPLE_NEVER = 2 };

#define SMC_MAX_LAYERS 8

/*
 * SMC_MODEL_CNN: the image classifier conv3x3(C1) -> ReLU -> conv3x3(C2) -> ReLU ->
 * 2x2 average pool -> linear(n_cls), "same" zero padding, stride 1, on H x W images
 * with Cin channels stored channel-last (x_dev row = H*W*Cin values, NHWC).  H and W
 * even with H*W a multiple of 8, C1 and C2 multiples of 8, 2 <= n_cls <= 16,
 * categorical likelihood, FP32 or BF16 operands.  Parameter blocks, each output
 * unit's weights followed by its bias: conv1 [C1 x (9 Cin + 1)] with weight index
 * (ky*3 + kx)*Cin + c, conv2 [C2 x (9 C1 + 1)] with index (ky*3 + kx)*C1 + c, linear
 * [n_cls x ((H/2)(W/2) C2 + 1)] with input index (py*(W/2) + px)*C2 + c; output pixel
 * (y, x) reads input pixel (y + ky - 1, x + kx - 1).  act_budget_bytes bounds the
 * per-chunk operand buffers (patch matrices, activations and errors of all particles).
 *
 * SMC_MODEL_LENET: the LeNet-5 classifier of the paper's MNIST study (Section 4, Table 1)
 * conv kxk(C1) "same" -> act -> 2x2 average pool -> conv kxk(C2) "valid" -> act -> 2x2
 * average pool -> dense(F1) -> act -> dense(F2) -> act -> dense(n_cls), stride 1, zero
 * padding (k-1)/2 on the first convolution, one activation (tanh in the paper) throughout,
 * on H x W images with Cin channels stored channel-last.  n_layers = 5 and widths = {H, W,
 * Cin, k, C1, C2, F1, F2, n_cls}; {28, 28, 1, 5, 6, 16, 120, 84, 10} is LeNet-5 with
 * D = 61,706.  Limits: k = 3 or 5, H and W even, (H/2 - k + 1) and (W/2 - k + 1) even and
 * >= 2, Cin and C1 <= 8, ceil(C2/2) C1 k <= 256, F1 and F2 multiples of 4, 2 <= n_cls <= 16,
 * FP32 operands, categorical likelihood, the fixed proposal.  Parameter blocks, each
 * output unit's weights followed by its bias: conv1 [C1 x (k^2 Cin + 1)] with weight index
 * (ky*k + kx)*Cin + c, conv2 [C2 x (k^2 C1 + 1)] with index (ky*k + kx)*C1 + c, dense1
 * [F1 x (F + 1)] with input index (py*Wq + px)*C2 + c over the Hq x Wq x C2 pooled map
 * (F = Hq Wq C2), dense2 [F2 x (F1 + 1)], output [n_cls x (F2 + 1)].  Output pixel (y, x)
 * of the first convolution reads input pixel (y + ky - (k-1)/2, x + kx - (k-1)/2); of the
 * second, pooled pixel (y + ky, x + kx).
 */
typedef struct smc_config {
  int32_t n_particles;                 /* J >= 1 (at most 4096) */
  int32_t n_layers;                    /* L >= 1 weight layers (at most SMC_MAX_LAYERS); 3 for SMC_MODEL_CNN, 5 for SMC_MODEL_LENET */
  int32_t widths[SMC_MAX_LAYERS + 1];  /* MLP: n_0 = input features, ..., n_L = outputs.
                                          CNN: {H, W, Cin, C1, C2, n_cls}; LENET: {H, W, Cin, k, C1, C2, F1, F2, n_cls} */
  int32_t activation;                  /* hidden activation: SMC_ACT_TANH | SMC_ACT_RELU (CNN: ReLU) */
  int32_t model_kind;                  /* SMC_MODEL_MLP | SMC_MODEL_CNN | SMC_MODEL_LENET */
  int32_t likelihood;                  /* SMC_LIK_CATEGORICAL (n_L <= 16 classes) | SMC_LIK_GAUSSIAN (n_L = 1) */
  int32_t precision;                   /* GEMM operand precision; accumulation is always FP32 */
  int32_t proposal;                    /* SMC_PROPOSAL_FIXED | SMC_PROPOSAL_LEARNED (needs S = 1) */
  int32_t leapfrog_steps;              /* S >= 1 (Section 2.1) */
  int32_t n_iterations;                /* K (used only by the learned proposal's k/K feature; 0 = unknown) */
  double step_size;                    /* h (Section 2.1) */
  double prior_std;                    /* q0 = N(0, prior_std^2 I) */
  double noise_std;                    /* sigma of the Gaussian likelihood */
  double ess_frac;                     /* resample when ESS < ess_frac * J (Section 2: 0.5) */
  uint64_t seed;                       /* key of the device Philox-4x32-10 generator */
  int64_t act_budget_bytes;            /* activation memory of one gradient pass; 0 = 8 GiB */
} smc_config;

typedef struct smc_step_info {
  double ess;                /* J_eff after reweighting (Eq. jeff) */
  double log_z_increment;    /* log sum_j w~_{k-1,j} * exp(increment_j) */
  double mean_loglik;        /* mean over particles of the subset log-likelihood LL_k */
  double max_loglik;
  int32_t n_nonfinite;       /* particles whose weight was set to zero (log w = -inf) */
  int32_t resample_recommended; /* ESS < ess_frac * J */
  int64_t grad_evals;        /* particle-sample gradient evaluations done by this call */
} smc_step_info;

typedef struct smc_handle* smc_t;

SMC_API const char* smc_status_string(smc_status s);
/* Detail of the last error raised on the calling thread ("" if none). */
SMC_API const char* smc_last_error(void);

/*
 * Create a sampler and apply the initial weighting (Section 2, Eq. init_weight).
 *   x_dev      [n_data x n_0] float32 row-major, already in annealing order
 *              (the subset at iteration k is rows [0, M_k); Section 3).
 *   y_dev      [n_data] int32 class labels (categorical) or float32 targets (Gaussian).
 *   theta0_dev [J x D] float32 initial particles, or NULL to draw theta_0 ~ q0
 *              on the device.
 *   m0, lambda0  initial subset size M_0 (1 <= m0 <= n_data) and scale.
 *   hip_stream hipStream_t (NULL = default stream).
 * On success *out receives the handle.  Errors: SMC_ERR_ARG for invalid
 * configuration or sizes, SMC_ERR_OOM, SMC_ERR_DEVICE, SMC_ERR_NONFINITE.
 */
SMC_API smc_status smc_init(const smc_config* cfg, const float* x_dev, const void* y_dev, int64_t n_data,
                    const float* theta0_dev, int64_t m0, double lambda0, void* hip_stream, smc_t* out);
SMC_API void smc_destroy(smc_t h);

/*
 * One SMC iteration on the subset [0, m_k) with scale lambda_k: if the subset
 * or lambda changed, the gradient at the current particles is recomputed on
 * the new subset; then S leapfrog steps (Section 2.1), the L-kernel weight
 * update (Eq. weight_update_fp; the learned proposal uses the general form of
 * Eq. weight_update), normalisation (Eq. normalise) and the ESS (Eq. jeff).
 * m_k must not decrease (append-only annealing, Section 3) and must be
 * <= n_data.  info (host, nullable) receives statistics; passing it
 * synchronises the stream.  SMC_ERR_NONFINITE if every weight became zero.
 */
SMC_API smc_status smc_step(smc_t h, int64_t m_k, double lambda_k, smc_step_info* info);

/*
 * smc_step for a two-segment target (smooth data annealing, Section 3.1, Eq.
 * sda_initial_target and the annealed target after a mini-batch was appended):
 *   log pi(theta) = lambda_a LL[0, m_split) + lambda_b LL[m_split, m_k) + log q0(theta),
 * where LL[a, b) is the unscaled log-likelihood of samples a..b-1.  SDA's
 * initial phase is m_split = 0, lambda_b = beta; after an append it is
 * m_split = M_{k-1}, lambda_a = 1, lambda_b = beta.  m_split >= m_k is the
 * one-segment target of smc_step (lambda_b ignored).  The move, weight
 * update (against the cached target of the previous iteration) and ESS are
 * those of smc_step; the second segment's log-likelihood at the new particles
 * is kept for smc_segment_moments.  Errors as smc_step, plus SMC_ERR_ARG for
 * m_split < 0 or lambda_b not finite and > 0.
 */
SMC_API smc_status smc_step_tempered(smc_t h, int64_t m_k, int64_t m_split, double lambda_a, double lambda_b,
                                     smc_step_info* info);

/*
 * Weighted moments of the segment log-likelihoods of the last target at the
 * current particles (Section 3.1, the moment equations ending in Eq. E{XY}):
 * with Omega^ = -LL[m_split, m) and Omega = -LL[0, m_split), under the
 * normalised weights, out4 (host, 4 doubles) receives
 *   { E[Omega^], Var(Omega^), E[Omega], Cov(Omega, Omega^) },
 * variance and covariance as E[XY] - E[X]E[Y] in FP64; particles of zero weight
 * do not enter.  With a one-segment target Omega^ is 0.  Synchronises the stream.
 */
SMC_API smc_status smc_segment_moments(smc_t h, double* out4);

/*
 * Systematic resampling (Section 2 resamples when J_eff < J/2).
 *   mode      SMC_RESAMPLE_IF_NEEDED (decided on the device: ESS < ess_frac*J),
 *             SMC_RESAMPLE_ALWAYS or SMC_RESAMPLE_NEVER.
 *   u         host pointer to the offset u in [0, 1), or NULL to draw it on the device.
 *   resampled (host, nullable) receives 1 if the population was resampled.
 *   ancestors_host (host, nullable) [J] receives the sorted systematic ancestors
 *             (identity if not resampled).
 * Survivors keep their slot; dead slots receive the surplus copies (in-place).
 * Weights are reset to 1/J after resampling.  Synchronises the stream (the
 * device flags are read on every call).  SMC_ERR_NONFINITE if every particle's
 * log-weight is non-finite, also when the step that made them so returned no
 * statistics; the population is then left unchanged.
 */
SMC_API smc_status smc_resample(smc_t h, int32_t mode, const double* u, int32_t* resampled, int32_t* ancestors_host);

/*
 * Multinomial resampling, the paper's scheme (Section 2): J ancestors drawn
 * independently with probabilities w~_j.  Same exact integer rule as
 * smc_resample: with the weights quantised to Q_j = floor(w~_j 2^50), prefix
 * sums S_j and total T, uniform U_k goes to t_k = min(floor(U_k T), T - 1) and
 * ancestor #{j : S_j <= t_k}; the ancestors are reported sorted.
 *   u_dev  device [J] float64 uniforms in [0, 1) (clamped into [0, 1]), or NULL
 *          to draw them on the device (Philox, one counter per particle).
 * Other arguments, the decision, placement and weight reset as smc_resample.
 */
SMC_API smc_status smc_resample_multinomial(smc_t h, int32_t mode, const double* u_dev, int32_t* resampled,
                                            int32_t* ancestors_host);

/*
 * Posterior predictive p(y | x) = sum_j w~_j softmax(f_{theta_j}(x)) (Section 2,
 * posterior estimates) on n test inputs.
 *   x_dev [n x n_0] float32; y_dev [n] int32 labels or NULL;
 *   probs_dev [n x n_L] float32 or NULL;
 *   accuracy / mean_log_pred (host, nullable; need y_dev): arg-max accuracy
 *   (lowest class on ties) and mean_i log sum_j w~_j p(y_i | x_i, theta_j).
 */
SMC_API smc_status smc_posterior_predict(smc_t h, const float* x_dev, const int32_t* y_dev, int64_t n,
                                 float* probs_dev, double* accuracy, double* mean_log_pred);

/* Weighted posterior mean sum_j w~_j theta_j (Section 2), [D] float64 on the device. */
SMC_API smc_status smc_posterior_mean(smc_t h, double* mean_dev);

/*
 * Settling test for adaptive subset growth (an extension in the spirit of
 * Section 3: grow the subset once the sampler has settled on the current one).
 * Computes the weighted posterior mean theta_bar of the current population
 * (FP64), returns in *rel_change (host) |theta_bar - theta_bar_prev| /
 * |theta_bar_prev| against the mean of the previous call, and keeps the new
 * mean for the next call.  The first call after smc_init or smc_set_state
 * returns +infinity.  A caller appends kappa points when the value is below its
 * tolerance.  Synchronises the stream.
 */
SMC_API smc_status smc_posterior_mean_change(smc_t h, double* rel_change);

/*
 * Copy the population out (any pointer may be NULL):
 *   theta_dev [J x D] float32, logw_dev [J] normalised log-weights (float64),
 *   loglik_dev [J] subset log-likelihoods LL_k (float64),
 *   logpi_dev [J] cached log pi_k(theta_k) (float64),
 *   grad_dev [J x D] float32 gradient of log pi_k at theta_k (prior included).
 */
SMC_API smc_status smc_get_state(smc_t h, float* theta_dev, double* logw_dev, double* loglik_dev,
                         double* logpi_dev, float* grad_dev);

/*
 * Replace the population (checkpoint restore).  theta_dev is required; the
 * log-likelihood and gradient are recomputed on the current subset; logw_dev
 * (normalised log-weights) and logpi_dev may be NULL (then log w = lambda LL
 * as at initialisation and log pi is recomputed).  rng_counter restores the
 * device generator position (iteration counter).
 */
SMC_API smc_status smc_set_state(smc_t h, const float* theta_dev, const double* logw_dev, const double* logpi_dev,
                         uint64_t rng_counter);

/* Device generator position (advanced once per smc_step and per device-drawn u). */
SMC_API smc_status smc_get_rng_counter(smc_t h, uint64_t* counter);

/*
 * Use momenta_dev [J x D] float32 as the standard-normal draw of the next
 * smc_step instead of the device generator (the initial momentum P_{k-1} of
 * Eq. mom_first, or the noise xi of the learned move).  Consumed by that step.
 */
SMC_API smc_status smc_set_noise(smc_t h, const float* momenta_dev);

/*
 * Learned proposal-scale network (an extension: the paper's move uses a fixed
 * step).  params_dev is the flat float32 blob
 *   mu[4], sd[4], W1[64x4], b1[64], W2[64x64], b2[64], W3[(1+G)x64], b3[1+G]
 * with G = 2L parameter groups; h0 is the base step size.  The handle copies it.
 */
SMC_API smc_status smc_set_proposal_net(smc_t h, const float* params_dev, int32_t n_params, double h0);

/*
 * Switch the move of the following iterations between the fixed-step move
 * (SMC_PROPOSAL_FIXED) and the learned-scale Langevin move (SMC_PROPOSAL_LEARNED,
 * which needs leapfrog_steps == 1 and a network set with smc_set_proposal_net).
 * Both moves reweight with the L-kernel of their own step (Section 2.1, Eq.
 * weight_update), so the population stays properly weighted across a switch; this is
 * how the run-level fallback to the fixed step is applied.  Errors: SMC_ERR_ARG,
 * SMC_ERR_STATE (learned without a network).
 */
SMC_API smc_status smc_set_proposal(smc_t h, int32_t proposal);

/*
 * Per-particle features of the learned proposal at the current state,
 * [J x 4] float64: (log |grad log pi|, LL / M_k, k / K, M_k / N) with
 * k_over_K and m_over_N supplied by the caller.
 */
SMC_API smc_status smc_proposal_features(smc_t h, double k_over_K, double m_over_N, double* feat_dev);

/*
 * Stand-alone network pass for a population theta_dev [J x D] on the first m
 * samples of the handle's data (the handle's particles are not touched):
 *   smc_nn_forward:  ll_dev [J] = sum_{i<m} log p(y_i | x_i, theta_j)  (float64)
 *   smc_nn_backward: additionally grad_dev [J x D] = scale_j * d LL_j / d theta_j
 *                    (float32; scale_dev [J] float64 or NULL for 1).  The forward
 *                    activations are recomputed chunk by chunk inside the backward.
 */
SMC_API smc_status smc_nn_forward(smc_t h, const float* theta_dev, int64_t m, double* ll_dev);
SMC_API smc_status smc_nn_backward(smc_t h, const float* theta_dev, int64_t m, const double* scale_dev,
                           double* ll_dev, float* grad_dev);

/* Number of parameters D of one particle for the handle's network. */
SMC_API int64_t smc_n_params(smc_t h);
/* Samples per activation chunk chosen from act_budget_bytes (for tests). */
SMC_API int64_t smc_chunk_samples(smc_t h);

/*
 * Training targets for the learned proposal from the current population
 * (an extension; the paper's moves use a fixed step).  Moves the subset to
 * (m_k, lambda_k) first if it changed (as smc_step would), then for every step
 * size h_grid[i] runs one preconditioning-free Langevin trial from the current
 * particles with shared noise and scores it by the squared jump times
 * min(1, exp(D))^accept_power, D the Metropolis log-ratio under the current
 * target (which is also the move's log-weight increment); accept_power = 1 is
 * the expected squared jump distance, larger values favour steps whose
 * increments stay near zero and so keep the ESS.  The particles are restored
 * afterwards.  Outputs (device, float32):
 *   feat_dev   [J x 4]      features at the current state (see smc_proposal_features)
 *   target_dev [J x (1+G)]  raw-output regression targets: atanh of the clipped
 *              (log h* - log h)/ln 8 for the best grid step h* (h = step_size),
 *              and atanh of the clipped centred log RMS gradient / ln 10 per group.
 * Injected noise (smc_set_noise) is used for every trial and consumed.
 */
SMC_API smc_status smc_proposal_targets(smc_t h, int64_t m_k, double lambda_k, const double* h_grid, int32_t n_grid,
                                        double k_over_K, double accept_power, float* feat_dev, float* target_dev);

/* Parameters of the proposal network for G groups (-1 if G is out of range). */
SMC_API int32_t smc_mlp_n_params(int32_t n_groups);

/*
 * Stateless proposal-network passes on R rows of float32 features [R x 4]:
 *   smc_mlp_forward: mode 0 writes the raw outputs [R x (1+G)]; mode 1 the bounded
 *     scales (h0 exp(ln8 tanh o_0), exp(ln10 tanh o_g)) with (h0, 1) for rows whose
 *     outputs are not finite.  bf16 != 0 runs the hidden 64x64 layer on BF16 MFMAs.
 *   smc_mlp_grad: FP32 gradient of (1/R) sum_r 1/2 |o_r - t_r|^2 w.r.t. the blob
 *     (zero for the input statistics mu, sd) into grad_dev, loss to *loss (host, nullable).
 *   smc_mlp_train: n_steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) numbered from
 *     first_step, on the full batch; adam_dev [2 x n_params] holds the moment estimates
 *     (zero-initialise before the first call).  Synchronises the stream.
 */
SMC_API smc_status smc_mlp_forward(const float* params_dev, const float* feat_dev, int64_t R, int32_t n_groups,
                                   float* out_dev, int32_t mode, double h0, int32_t bf16, void* hip_stream);
SMC_API smc_status smc_mlp_grad(const float* params_dev, const float* feat_dev, const float* target_dev, int64_t R,
                                int32_t n_groups, float* grad_dev, double* loss, void* hip_stream);
SMC_API smc_status smc_mlp_train(float* params_dev, float* adam_dev, const float* feat_dev, const float* target_dev,
                                 int64_t R, int32_t n_groups, int32_t first_step, int32_t n_steps, double lr,
                                 double* loss, void* hip_stream);

/*
 * Allocation-free variant of smc_mlp_train, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels and arithmetic as smc_mlp_train (identical results); the
 * per-tile gradient and loss partials of each Adam step live in a fixed 10 MiB device
 * array that the library holds on every device it runs on until the process ends.
 *   R <= 32768 rows and 1 <= n_groups <= 8, else SMC_ERR_ARG (the scratch limit).
 *   loss_dev (device float64, nullable) receives the last step's loss.
 * Enqueues on hip_stream (the current device's stream) and returns without
 * synchronising; it calls no hipMalloc/hipFree and copies nothing to the host.
 * The scratch keeps the last call's contents; every value a call reads from it is
 * written by that call first, so nothing needs clearing.  All calls on one device
 * share that device's scratch: calls that overlap on one device (other streams or
 * threads) race and must be serialised by the caller.
 */
SMC_API smc_status smc_mlp_train_noalloc(float* params_dev, float* adam_dev, const float* feat_dev,
                                         const float* target_dev, int64_t R, int32_t n_groups, int32_t first_step,
                                         int32_t n_steps, double lr, double* loss_dev, void* hip_stream);

/* ---------------------------------------------------------------- kernel timing */
/*
 * Kernel classes timed by the profiling hook.  FLOP and byte counts are the
 * algorithmic work of each launch (unpadded sizes): GEMMs 2*M*N*K, the output
 * layer 6*C*H per particle-sample, moves the parameter bytes they must touch.
 */
enum {
  SMC_K_GEMM_FWD1 = 0,   /* layer-1 forward GEMM over all particles' units */
  SMC_K_GEMM_DW1 = 1,    /* layer-1 weight-gradient GEMM */
  SMC_K_GEMM_OTHER = 2,  /* GEMMs of layers >= 2 */
  SMC_K_HEAD = 3,        /* output layer, likelihood and its reduction */
  SMC_K_MOVE = 4,        /* leapfrog / Langevin parameter updates */
  SMC_K_WEIGHT = 5,      /* log-weight update, normalisation, ESS */
  SMC_K_RESAMPLE = 6,    /* systematic resampling + row gather + re-cast */
  SMC_K_OTHER = 7,
  SMC_K_COUNT = 8
};

/*
 * enable != 0: from now on every kernel launch of the handle is bracketed by a
 * pair of HIP events recorded on the handle's stream.  enable == 0 stops
 * recording.  Records accumulate until smc_profile_read.
 */
SMC_API smc_status smc_profile(smc_t h, int32_t enable);

/*
 * Synchronise, then for each class k < SMC_K_COUNT write total_ms[k] (summed
 * event time), launches[k], flops[k] and bytes[k] (algorithmic totals).  Any
 * pointer may be NULL.  Clears the records.
 */
SMC_API smc_status smc_profile_read(smc_t h, double* total_ms, int64_t* launches, double* flops, double* bytes);

/* ---------------------------------------------------------------- stateless kernels */

/*
 * Normalise J log-weights in FP64 (Eq. normalise, log domain) and compute the
 * ESS (Eq. jeff).  logw_out_dev [J] receives log w~; stats_dev [4] receives
 * (log sum_j w_j, ESS, number of -inf/NaN entries, max log w).  In-place
 * (logw_out_dev == logw_dev) is allowed.
 */
SMC_API smc_status smc_normalise(const double* logw_dev, int32_t J, double* logw_out_dev, double* stats_dev,
                         void* hip_stream);

/*
 * Systematic resampling of normalised weights w_dev [J] (float64) with offset
 * u in [0, 1), exact integer rule: Q_j = floor(w_j 2^50), S = inclusive prefix
 * sums, T = S_{J-1}, R = min(floor(u T), T - 1), t_k = floor((k T + R) / J),
 * ancestor_k = #{j : S_j <= t_k}.  ancestors_dev [J] int32 receives the sorted
 * ancestors; placement_dev [J] int32 (nullable) the in-place arrangement
 * (survivors keep their slot, dead slots take the surplus copies in order).
 */
SMC_API smc_status smc_systematic_resample(const double* w_dev, int32_t J, double u, int32_t* ancestors_dev,
                                   int32_t* placement_dev, void* hip_stream);

/*
 * Multinomial resampling of normalised weights w_dev [J] (float64) with the
 * device uniforms u_dev [J] (float64, clamped into [0, 1]), exact integer rule
 * of smc_resample_multinomial: t_k = min(floor(U_k T), T - 1), ancestor
 * #{j : S_j <= t_k}.  ancestors_dev [J] int32 receives the ancestors sorted;
 * placement_dev [J] int32 (nullable) the in-place arrangement.
 */
SMC_API smc_status smc_multinomial_resample(const double* w_dev, int32_t J, const double* u_dev,
                                            int32_t* ancestors_dev, int32_t* placement_dev, void* hip_stream);

/*
 * Raw Philox-4x32-10 blocks: for i in [0, n_blocks) out_dev[4i..4i+3] =
 * philox(ctr = (i, c1, c2, c3), key = (key0, key1)).
 */
SMC_API smc_status smc_philox(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n_blocks,
                      uint32_t* out_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H_ */
