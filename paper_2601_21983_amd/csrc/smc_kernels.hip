// Elementwise, reduction and population kernels of the SMC sampler.
//
//  * move_kernel     leapfrog half/full steps over the [J x D] population (Section 2.1,
//                    Eqs. mom_first, pos_update, mom_second) with Philox momenta, fused
//                    |xi|^2, |theta|^2, |P_end|^2 partial sums and the GEMM-layout re-cast;
//  * weight_kernel   the reversed-momentum L-kernel log-weight update (Eq. weight_update_fp),
//                    normalisation (Eq. normalise) and ESS (Eq. jeff) in FP64;
//  * resample_kernel exact-integer systematic resampling and the in-place placement;
//  * gather, posterior mean, predictive mixture, Philox, prior draw.
// Reductions run in a fixed order (no floating-point atomics), so results are
// reproducible run to run.
#include "kernels.h"

#include <math.h>

namespace smc {

namespace {

// ------------------------------------------------------------------ GEMM-layout cast
__device__ __forceinline__ void cast_any(const NetShape& n, int j, int64_t e, float v) {
  if (e < n.off[0]) return;  // parameters ahead of the dense layers (a convolution stack)
  int l = 0;
#pragma unroll
  for (int q = 1; q < MAX_LAYERS; ++q)
    if (q < n.L && e >= n.off[q]) l = q;
  const int rowlen = n.nin[l] + 1;
  const int ep = (int)(e - n.off[l]);
  int o = (int)((float)ep * n.rinv[l]);
  while (o * rowlen > ep) --o;
  while ((o + 1) * rowlen <= ep) ++o;
  weight_copy_store(n, j, l, o, ep - o * rowlen, v);
}

__global__ __launch_bounds__(256) void cast_kernel(const NetShape n, const float* __restrict__ theta,
                                                   const int32_t* __restrict__ placement) {
  const int j = blockIdx.y;
  if (placement && placement[j] == j) return;
  // consecutive lanes take consecutive parameters (coalesced loads and copy stores)
  const int64_t e0 = (int64_t)blockIdx.x * MOVE_ELEMS + threadIdx.x;
  const float* th = theta + (int64_t)j * n.D;
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = e0 + 256 * i < n.D ? th[e0 + 256 * i] : 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t e = e0 + 256 * i;
    if (e < n.D) cast_any(n, j, e, v[i]);
  }
}

// ------------------------------------------------------------------ move
// Lane t of workgroup b handles parameters e = 1024 b + t + 256 i (i = 0..3), so that each
// load and store instruction covers 64 consecutive parameters.  The momentum of parameter e
// is normal (e mod 4) of the Philox block e / 4 of its particle.  The four parameters of lane
// (q, s) = (t / 4, t mod 4) lie in the blocks 256 b + 64 i + q, all at position s: lane
// (q, r) draws block 256 b + 64 r + q, and a 4x4 transpose inside the lane quad hands
// every lane its four normals.
__device__ __forceinline__ float pick4(const f32x4& v, int k) {
  return k == 0 ? v[0] : (k == 1 ? v[1] : (k == 2 ? v[2] : v[3]));
}

__global__ __launch_bounds__(256) void move_kernel(const MoveArgs a) {
  __shared__ double red[3][4];
  const int j = blockIdx.y;
  const int64_t D = a.net.D;
  const int64_t e0 = (int64_t)blockIdx.x * MOVE_ELEMS + threadIdx.x;
  float* th = a.theta + (int64_t)j * D;
  float* P = a.P + (int64_t)j * D;
  const float* g = a.g + (int64_t)j * D;
  float s_xi = 0.0f, s_th = 0.0f, s_pe = 0.0f;
  float nz[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (a.mode == MOVE_FIRST && !a.noise) {
    const int q = (threadIdx.x & 63) >> 2, r = threadIdx.x & 3, w = threadIdx.x >> 6;
    // this lane's draw: block (1024 b + 256 r + 64 w + 4 q) / 4 of particle j
    const uint32_t blk = (uint32_t)(((int64_t)blockIdx.x * MOVE_ELEMS + 256 * r + 64 * w + 4 * q) >> 2);
    const u32x4 c = {blk, (uint32_t)j, a.ctr_iter, (uint32_t)TAG_MOMENTUM};
    const f32x4 mine = normal4(philox4x32_10(c, a.key0, a.key1));
    // round k: lane (q, s) receives normal s of the block drawn by lane (q, (s - k) & 3), which
    // belongs to its parameter i = (s - k) & 3; the sender offers its normal (r + k) & 3
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float offer = pick4(mine, (r + k) & 3);
      const float got = k == 0 ? offer : __shfl(offer, (r - k) & 3, 4);
      const int i = (r - k) & 3;
      nz[0] = i == 0 ? got : nz[0];
      nz[1] = i == 1 ? got : nz[1];
      nz[2] = i == 2 ? got : nz[2];
      nz[3] = i == 3 ? got : nz[3];
    }
  }
  const float h = a.h, hh = 0.5f * a.h;
  // all four parameters' loads first: the stores below could alias later loads as far as the
  // compiler knows, which would otherwise serialise the four round trips
  float tv[4], gv[4], pv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t e = e0 + 256 * i;
    const bool in = e < D;
    tv[i] = in ? th[e] : 0.0f;
    gv[i] = in ? g[e] : 0.0f;
    pv[i] = 0.0f;
    if (a.mode == MOVE_FIRST) {
      if (a.noise) pv[i] = in ? a.noise[(int64_t)j * D + e] : 0.0f;
      else pv[i] = nz[i];
    } else {
      pv[i] = in ? P[e] : 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t e = e0 + 256 * i;
    if (e >= D) break;
    float t = tv[i];
    const float gf = gv[i] - t * a.inv_prior_var;
    if (a.mode == MOVE_FIRST) {
      const float xi = pv[i];
      s_xi += xi * xi;
      const float p = xi + hh * gf;
      t = t + h * p;
      P[e] = p;
      th[e] = t;
      s_th += t * t;
      if (a.cast) cast_any(a.net, j, e, t);
    } else if (a.mode == MOVE_MID) {
      const float p = pv[i] + h * gf;
      t = t + h * p;
      P[e] = p;
      th[e] = t;
      s_th += t * t;
      if (a.cast) cast_any(a.net, j, e, t);
    } else {
      const float p = pv[i] + hh * gf;
      s_pe += p * p;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // each mode owns its rows: FIRST |xi|^2 and |theta|^2, MID |theta|^2, LAST |P_end|^2 (only
  // those are reduced)
  const double v0 = a.mode == MOVE_FIRST ? wave_sum((double)s_xi) : 0.0;
  const double v1 = a.mode != MOVE_LAST ? wave_sum((double)s_th) : 0.0;
  const double v2 = a.mode == MOVE_LAST ? wave_sum((double)s_pe) : 0.0;
  if (lane == 0) { red[0][wid] = v0; red[1][wid] = v1; red[2][wid] = v2; }
  __syncthreads();
  const int w = threadIdx.x;
  const bool own = (a.mode == MOVE_FIRST && w < 2) || (a.mode == MOVE_MID && w == 1) || (a.mode == MOVE_LAST && w == 2);
  if (w < 3 && own) {
    const double s = red[w][0] + red[w][1] + red[w][2] + red[w][3];
    a.part[((int64_t)w * a.net.J + j) * a.nblk + blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ block scans
template <typename V>
__device__ V block_exclusive_scan(V v, V* wsum, V& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  V x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const V y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  __syncthreads();
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    V run = 0;
    for (int w = 0; w < nw; ++w) {
      const V t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    wsum[nw] = run;
  }
  __syncthreads();
  const V ex = wsum[wid] + x - v;
  total = wsum[nw];
  __syncthreads();
  return ex;
}

// ------------------------------------------------------------------ weights
__global__ __launch_bounds__(1024) void weight_kernel(const WeightArgs a) {
  __shared__ double red[16];
  __shared__ double psum[3][MAX_J];  // each particle's summed move partials
  constexpr int NPT = MAX_J / 1024;
  const int J = a.J, tid = threadIdx.x;
  if (a.part) {
    // tpp neighbouring threads per particle (up to 8, as many as the block holds), each summing
    // every tpp-th partial with four accumulators, then a butterfly over the group: a fixed
    // order, so the result is reproducible, with several loads in flight per thread
    int tpp = 1;
    while (tpp < 8 && J * tpp * 2 <= 1024) tpp *= 2;
    const int sub = tid % tpp, nslot = 1024 / tpp;
    for (int base = 0; base < J; base += nslot) {
      const int j = base + tid / tpp;
      double s0[4] = {0, 0, 0, 0}, st[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0};
      if (j < J) {
        const double* p0 = a.part + (int64_t)j * a.nblk;
        const double* p1 = a.part + ((int64_t)J + j) * a.nblk;
        const double* p2 = a.part + ((int64_t)2 * J + j) * a.nblk;
        int u = 0;
        for (int b = sub; b < a.nblk; b += tpp, u = (u + 1) & 3) {
          s0[u] += p0[b];
          st[u] += p1[b];
          s1[u] += p2[b];
        }
      }
      double x0 = (s0[0] + s0[1]) + (s0[2] + s0[3]);
      double xt = (st[0] + st[1]) + (st[2] + st[3]);
      double x1 = (s1[0] + s1[1]) + (s1[2] + s1[3]);
      for (int o = 1; o < tpp; o <<= 1) {  // every lane of the block takes part
        x0 += __shfl_xor(x0, o, 64);
        xt += __shfl_xor(xt, o, 64);
        x1 += __shfl_xor(x1, o, 64);
      }
      if (j < J && sub == 0) {
        psum[0][j] = x0;
        psum[1][j] = xt;
        psum[2][j] = x1;
      }
    }
    __syncthreads();
  }
  double lwn[NPT];
  double mx = -INFINITY, llsum = 0.0, llmax = -INFINITY;
  double nbad = 0.0, nfin = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int j = tid + q * 1024;
    lwn[q] = -INFINITY;
    if (j >= J) continue;
    double k0 = 0.0, kt = a.tsq ? a.tsq[j] : 0.0, k1 = 0.0;
    if (a.part) {
      k0 += psum[0][j];
      kt += psum[1][j];
      k1 += psum[2][j];
      if (a.no_kinetic) { k0 = 0.0; k1 = 0.0; }
    }
    const double ll = a.ll[j];
    // log-likelihood term of the target: one segment (lambda LL) or two
    const double llt = a.ll_b ? a.lambda * (ll - a.ll_b[j]) + a.lambda_b * a.ll_b[j] : a.lambda * ll;
    const double lpn = llt - kt * a.inv_2prior_var;
    double incr;
    double prev;
    if (a.init) {
      incr = llt;
      prev = 0.0;
    } else {
      incr = lpn - a.lp[j] - 0.5 * k1 + 0.5 * k0 + (a.extra ? a.extra[j] : 0.0);
      prev = a.logw[j];
    }
    double v = prev + incr;
    if (!isfinite(incr) || !isfinite(ll) || isnan(v)) v = -INFINITY;
    if (v == -INFINITY) nbad += 1.0;
    a.lp[j] = lpn;
    lwn[q] = v;
    mx = fmax(mx, v);
    if (isfinite(ll)) { llsum += ll; llmax = fmax(llmax, ll); nfin += 1.0; }
  }
  const double m = block_max(mx, red);
  const double tot_bad = block_sum(nbad, red);
  const double tot_ll = block_sum(llsum, red);
  const double tot_fin = block_sum(nfin, red);
  const double max_ll = block_max(llmax, red);
  if (m == -INFINITY) {
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int j = tid + q * 1024;
      if (j < J) { a.logw[j] = -INFINITY; a.w[j] = 0.0; }
    }
    if (tid == 0) {
      a.stats[ST_ESS] = 0.0; a.stats[ST_LOGZ] = -INFINITY; a.stats[ST_MEANLL] = NAN; a.stats[ST_MAXLL] = NAN;
      a.stats[ST_NONFINITE] = tot_bad; a.stats[ST_RECOMMEND] = 0.0; a.stats[ST_ALLBAD] = 1.0;
    }
    return;
  }
  double se = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) se += (tid + q * 1024 < J) ? exp(lwn[q] - m) : 0.0;
  se = block_sum(se, red);
  const double lz = m + log(se);
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int j = tid + q * 1024;
    if (j >= J) continue;
    const double lw = lwn[q] - lz;
    const double w = exp(lw);
    a.logw[j] = lw;
    a.w[j] = w;
    s2 += w * w;
  }
  s2 = block_sum(s2, red);
  if (tid == 0) {
    const double ess = 1.0 / s2;
    a.stats[ST_ESS] = ess;
    a.stats[ST_LOGZ] = lz - (a.init ? log((double)J) : 0.0);
    a.stats[ST_MEANLL] = tot_fin > 0 ? tot_ll / tot_fin : NAN;
    a.stats[ST_MAXLL] = max_ll;
    a.stats[ST_NONFINITE] = tot_bad;
    a.stats[ST_RECOMMEND] = ess < a.ess_frac * (double)J ? 1.0 : 0.0;
    a.stats[ST_ALLBAD] = 0.0;
    a.stats[ST_RESAMPLED] = 0.0;
  }
}

__global__ __launch_bounds__(1024) void normalise_kernel(const double* logw, int J, double* out, double* stats,
                                                        double* wout) {
  __shared__ double red[16];
  constexpr int NPT = MAX_J / 1024;
  const int tid = threadIdx.x;
  double v[NPT];
  double mx = -INFINITY, nbad = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int j = tid + q * 1024;
    v[q] = j < J ? logw[j] : -INFINITY;
    if (j < J && !(v[q] > -INFINITY && v[q] < INFINITY)) { nbad += 1.0; v[q] = -INFINITY; }
    mx = fmax(mx, v[q]);
  }
  const double m = block_max(mx, red);
  const double bad = block_sum(nbad, red);
  double se = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) se += (tid + q * 1024 < J && m > -INFINITY) ? exp(v[q] - m) : 0.0;
  se = block_sum(se, red);
  const double lz = m > -INFINITY ? m + log(se) : -INFINITY;
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int j = tid + q * 1024;
    if (j >= J) continue;
    const double lw = m > -INFINITY ? v[q] - lz : -INFINITY;
    out[j] = lw;
    const double w = exp(lw);
    if (wout) wout[j] = w;
    s2 += w * w;
  }
  s2 = block_sum(s2, red);
  if (tid == 0) {
    stats[0] = lz;
    stats[1] = s2 > 0 ? 1.0 / s2 : 0.0;
    stats[2] = bad;
    stats[3] = m;
  }
}

// ------------------------------------------------------------------ systematic resampling
struct SysScratch {
  uint64_t* S;   // [J]
  int* cnt;      // [J]
  int* einc;     // [J]
  int* drank;    // [J]
  uint64_t* wsu; // [17]
  int* wsi;      // [17]
};

__device__ SysScratch sys_scratch(char* smem, int J) {
  SysScratch s;
  s.S = (uint64_t*)smem;
  s.wsu = s.S + J;
  s.cnt = (int*)(s.wsu + 17);
  s.einc = s.cnt + J;
  s.drank = s.einc + J;
  s.wsi = s.drank + J;
  return s;
}
size_t sys_smem_bytes(int J) { return (size_t)J * 8 + 17 * 8 + (size_t)J * 12 + 17 * 4; }

// a uniform double in [0, 1) (53 bits) from Philox at counter (idx, 0, iter, tag)
__device__ __forceinline__ double philox_u01_double(uint32_t k0, uint32_t k1, uint32_t iter, uint32_t tag,
                                                    uint32_t idx = 0) {
  const u32x4 c = {idx, 0u, iter, tag};
  const u32x4 r = philox4x32_10(c, k0, k1);
  const uint64_t hi = r[0] >> 5, lo = r[1] >> 6;  // 27 + 26 bits
  return (double)((hi << 26) | lo) * 0x1p-53;
}

// Uniforms of multinomial resampling: an array, or Philox at counters (k, 0, iter, TAG_RESAMPLE_MULTI)
struct Uniforms {
  const double* arr = nullptr;
  uint32_t k0 = 0, k1 = 0, iter = 0;
};

// ancestors (sorted) and in-place placement from normalised weights w: systematic with
// offset u (multi = false) or multinomial with the uniforms U (multi = true)
__device__ void systematic_core(const double* w, int J, double u, const SysScratch& s, int32_t* anc,
                                int32_t* place, bool multi = false, const Uniforms& U = Uniforms{}) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (J + nt - 1) / nt;
  const int b = min(J, tid * per), e = min(J, b + per);
  uint64_t loc = 0;
  for (int i = b; i < e; ++i) {
    loc += (uint64_t)floor(w[i] * 0x1p50);
    s.S[i] = loc;
  }
  uint64_t tot;
  const uint64_t ex = block_exclusive_scan<uint64_t>(loc, s.wsu, tot);
  for (int i = b; i < e; ++i) s.S[i] += ex;
  for (int i = tid; i < J; i += nt) s.cnt[i] = 0;
  __syncthreads();
  const uint64_t T = s.S[J - 1];
  uint64_t R = (uint64_t)floor(u * (double)T);
  if (R > T - 1) R = T - 1;
  for (int k = tid; k < J; k += nt) {
    uint64_t t;
    if (multi) {
      const double uk = U.arr ? fmin(fmax(U.arr[k], 0.0), 1.0)
                              : philox_u01_double(U.k0, U.k1, U.iter, TAG_RESAMPLE_MULTI, (uint32_t)k);
      t = (uint64_t)floor(uk * (double)T);
      if (t > T - 1) t = T - 1;
    } else {
      t = ((uint64_t)k * T + R) / (uint64_t)J;
    }
    int lo = 0, hi = J - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s.S[mid] > t) hi = mid;
      else lo = mid + 1;
    }
    if (!multi) anc[k] = lo;  // systematic positions are already in increasing order
    atomicAdd(&s.cnt[lo], 1);
  }
  __syncthreads();
  if (multi) {
    // sorted ancestor list from the counts: anc[k] = first i whose inclusive count prefix exceeds k
    int cloc = 0;
    for (int i = b; i < e; ++i) cloc += s.cnt[i];
    int ctot;
    int cr = block_exclusive_scan<int>(cloc, s.wsi, ctot);
    for (int i = b; i < e; ++i) {
      cr += s.cnt[i];
      s.einc[i] = cr;
    }
    __syncthreads();
    for (int k = tid; k < J; k += nt) {
      int lo = 0, hi = J - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s.einc[mid] > k) hi = mid;
        else lo = mid + 1;
      }
      anc[k] = lo;
    }
    __syncthreads();
  }
  if (!place) return;
  int dloc = 0, xloc = 0;
  for (int i = b; i < e; ++i) {
    const int c = s.cnt[i];
    dloc += c == 0;
    xloc += c > 1 ? c - 1 : 0;
  }
  int dtot, xtot;
  int dr = block_exclusive_scan<int>(dloc, s.wsi, dtot);
  int xr = block_exclusive_scan<int>(xloc, s.wsi, xtot);
  for (int i = b; i < e; ++i) {
    const int c = s.cnt[i];
    s.drank[i] = dr;
    dr += c == 0;
    xr += c > 1 ? c - 1 : 0;
    s.einc[i] = xr;
  }
  __syncthreads();
  for (int k = tid; k < J; k += nt) {
    if (s.cnt[k] > 0) {
      place[k] = k;
    } else {
      const int r = s.drank[k];
      int lo = 0, hi = J - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s.einc[mid] > r) hi = mid;
        else lo = mid + 1;
      }
      place[k] = lo;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void systematic_kernel(const double* w, int J, double u, int32_t* anc,
                                                          int32_t* place) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const SysScratch s = sys_scratch(smem, J);
  systematic_core(w, J, u, s, anc, place);
}

__global__ __launch_bounds__(1024) void multinomial_kernel(const double* w, int J, const double* u_arr, int32_t* anc,
                                                           int32_t* place) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const SysScratch s = sys_scratch(smem, J);
  Uniforms U;
  U.arr = u_arr;
  systematic_core(w, J, 0.0, s, anc, place, true, U);
}

__global__ __launch_bounds__(1024) void resample_kernel(const ResampleArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int J = a.J, tid = threadIdx.x;
  const double ess = a.stats[ST_ESS];
  // a population whose every log-weight is non-finite has no weights to resample from: it is
  // left as it is (and stays flagged), the host reports the error
  const bool allbad = a.stats[ST_ALLBAD] != 0.0;
  const bool doit = !allbad && (a.mode == 1 || (a.mode == 0 && ess < a.ess_frac * (double)J));
  if (!doit) {
    for (int k = tid; k < J; k += blockDim.x) {
      a.ancestors[k] = k;
      a.placement[k] = k;
    }
    if (tid == 0) a.stats[ST_RESAMPLED] = 0.0;
    return;
  }
  const SysScratch s = sys_scratch(smem, J);
  if (a.scheme == RESAMPLE_MULTINOMIAL) {
    Uniforms U;
    U.arr = a.u_arr;
    U.k0 = a.key0;
    U.k1 = a.key1;
    U.iter = a.ctr_iter;
    systematic_core(a.w, J, 0.0, s, a.ancestors, a.placement, true, U);
  } else {
    const double u = a.u_dev ? *a.u_dev : philox_u01_double(a.key0, a.key1, a.ctr_iter, TAG_RESAMPLE_U);
    systematic_core(a.w, J, u, s, a.ancestors, a.placement);
  }
  // gather the per-particle scalars (read everything before writing)
  constexpr int NPT = MAX_J / 1024;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (!a.sc[c]) continue;
    double tmp[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int k = tid + q * 1024;
      tmp[q] = k < J ? a.sc[c][a.placement[k]] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int k = tid + q * 1024;
      if (k < J) a.sc[c][k] = tmp[q];
    }
    __syncthreads();
  }
  const double lw = -log((double)J), w = 1.0 / (double)J;
  for (int k = tid; k < J; k += blockDim.x) {
    a.logw[k] = lw;
    a.w[k] = w;
  }
  if (tid == 0) {
    a.stats[ST_RESAMPLED] = 1.0;
    a.stats[ST_ESS] = (double)J;
    a.stats[ST_RECOMMEND] = 0.0;
  }
}

__global__ __launch_bounds__(256) void gather_rows_kernel(int64_t D, const int32_t* __restrict__ placement,
                                                          float* a0, float* a1) {
  const int j = blockIdx.y;
  const int p = placement[j];
  if (p == j) return;
  const int64_t e0 = (int64_t)blockIdx.x * MOVE_ELEMS + threadIdx.x;  // coalesced, as in cast_kernel
  // loads first (destination rows are never source rows, but the compiler cannot know that)
  float v0[4], v1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t e = e0 + 256 * i;
    const bool in = e < D;
    v0[i] = in ? a0[(int64_t)p * D + e] : 0.0f;
    v1[i] = in && a1 ? a1[(int64_t)p * D + e] : 0.0f;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t e = e0 + 256 * i;
    if (e >= D) break;
    a0[(int64_t)j * D + e] = v0[i];
    if (a1) a1[(int64_t)j * D + e] = v1[i];
  }
}

// ------------------------------------------------------------------ estimates
__global__ __launch_bounds__(256) void posterior_mean_kernel(const float* theta, const double* w, int J, int64_t D,
                                                             double* out) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  double s = 0.0;
  for (int j = 0; j < J; ++j) s += w[j] * (double)theta[(int64_t)j * D + d];
  out[d] = s;
}

// out[0] = |cur - prev|^2, out[1] = |prev|^2 in FP64; one workgroup, fixed summation order
__global__ __launch_bounds__(1024) void mean_change_kernel(const double* cur, const double* prev, int64_t D,
                                                          double* out) {
  __shared__ double red[2][16];
  double a = 0.0, b = 0.0;
  for (int64_t d = threadIdx.x; d < D; d += blockDim.x) {
    const double p = prev[d], e = cur[d] - p;
    a += e * e;
    b += p * p;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      sa += red[0][q];
      sb += red[1][q];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

__global__ __launch_bounds__(256) void predictive_kernel(const float* logp, int64_t ld, const double* logw, int J,
                                                         int C, int64_t n, const int32_t* y, float* probs,
                                                         double* per_sample) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pr[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) pr[c] = 0.0;
  const int yi = y ? y[i] : 0;
  double m = -INFINITY, s = 0.0;
  for (int j = 0; j < J; ++j) {
    const double lw = logw[j];
    if (lw == -INFINITY) continue;
    const float* row = logp + ((int64_t)j * ld + i) * C;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < C) pr[c] += exp(lw + (double)row[c]);
    if (y) {
      const double v = lw + (double)row[yi];
      if (v > m) { s = s * exp(m - v) + 1.0; m = v; }
      else s += exp(v - m);
    }
  }
  int best = 0;
  for (int c = 1; c < C; ++c)
    if (pr[c] > pr[best]) best = c;
  if (probs)
    for (int c = 0; c < C; ++c) probs[i * C + c] = (float)pr[c];
  if (per_sample) {
    per_sample[2 * i] = (y && best == yi) ? 1.0 : 0.0;
    per_sample[2 * i + 1] = y ? m + log(s) : 0.0;
  }
}

__global__ __launch_bounds__(1024) void predictive_finish_kernel(const double* per_sample, int64_t n, double* out2) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  // fixed per-thread contiguous ranges, then a fixed tree
  const int64_t per = (n + blockDim.x - 1) / blockDim.x;
  const int64_t lo = min(n, (int64_t)threadIdx.x * per), hi = min(n, lo + per);
  for (int64_t i = lo; i < hi; ++i) { a += per_sample[2 * i]; b += per_sample[2 * i + 1]; }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) { out2[0] = a / (double)n; out2[1] = b / (double)n; }
}

// ------------------------------------------------------------------ RNG and helpers
__global__ void philox_kernel(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                              uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const u32x4 c = {(uint32_t)i, c1, c2, c3};
  const u32x4 r = philox4x32_10(c, k0, k1);
  for (int q = 0; q < 4; ++q) out[4 * i + q] = r[q];
}

__global__ __launch_bounds__(256) void prior_draw_kernel(float* theta, int64_t D, float sd, uint32_t k0, uint32_t k1) {
  const int j = blockIdx.y;
  const int64_t e0 = (int64_t)blockIdx.x * MOVE_ELEMS + 4 * threadIdx.x;
  if (e0 >= D) return;
  const u32x4 c = {(uint32_t)(e0 >> 2), (uint32_t)j, 0u, (uint32_t)TAG_PRIOR};
  const f32x4 nz = normal4(philox4x32_10(c, k0, k1));
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (e0 + i < D) theta[(int64_t)j * D + e0 + i] = sd * nz[i];
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void grad_with_prior_kernel(const float* theta, const float* g, float* out, int64_t n, float ipv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = g[i] - theta[i] * ipv;
}

__global__ __launch_bounds__(256) void sq_norm_rows_kernel(const float* a, int64_t D, double* out) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < D; e += 256) {
    const double v = a[(int64_t)j * D + e];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ void lp_current_kernel(const double* ll, const double* tsq, int J, double lambda, double inv_2pv,
                                  double* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < J) out[j] = lambda * ll[j] - tsq[j] * inv_2pv;
}

__global__ void f64_to_f32_kernel(const double* in, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Weighted moments of the two segments' negative log-likelihoods under the normalised
// weights w (smooth data annealing, Section 3.1): with Omega^ = -ll_b and Omega = -(ll - ll_b),
// out = {E[Omega^], Var(Omega^), E[Omega], Cov(Omega, Omega^)}, variance and covariance as
// E[XY] - E[X] E[Y].  Particles of zero weight do not enter the sums.
__global__ __launch_bounds__(1024) void segment_moments_kernel(const double* __restrict__ w,
                                                               const double* __restrict__ ll,
                                                               const double* __restrict__ ll_b, int J, double* out) {
  __shared__ double red[16];
  double eb = 0.0, ebb = 0.0, ea = 0.0, eab = 0.0;
  for (int j = threadIdx.x; j < J; j += blockDim.x) {
    const double wj = w[j];
    if (!(wj > 0.0)) continue;
    const double b = -ll_b[j], a = -(ll[j] - ll_b[j]);
    eb += wj * b;
    ebb += wj * b * b;
    ea += wj * a;
    eab += wj * a * b;
  }
  eb = block_sum(eb, red);
  ebb = block_sum(ebb, red);
  ea = block_sum(ea, red);
  eab = block_sum(eab, red);
  if (threadIdx.x == 0) {
    out[0] = eb;
    out[1] = ebb - eb * eb;
    out[2] = ea;
    out[3] = eab - ea * eb;
  }
}

}  // namespace

hipError_t kernels_set_smem_limits() {
  const int big = 160 * 1024;
  hipError_t e = hipFuncSetAttribute((const void*)systematic_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)multinomial_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)resample_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

hipError_t cast_run(const NetShape& net, const float* theta, const int32_t* placement, hipStream_t s) {
  dim3 grid(nblocks(net.D, MOVE_ELEMS), net.J);
  hipLaunchKernelGGL(cast_kernel, grid, dim3(256), 0, s, net, theta, placement);
  return hipGetLastError();
}

hipError_t move_run(const MoveArgs& a, hipStream_t s) {
  dim3 grid(a.nblk, a.net.J);
  hipLaunchKernelGGL(move_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t weight_run(const WeightArgs& a, hipStream_t s) {
  if (a.J > MAX_J) return hipErrorInvalidValue;
  hipLaunchKernelGGL(weight_kernel, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t segment_moments_run(const double* w, const double* ll, const double* ll_b, int J, double* out,
                               hipStream_t s) {
  if (J > MAX_J || J < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(segment_moments_kernel, dim3(1), dim3(1024), 0, s, w, ll, ll_b, J, out);
  return hipGetLastError();
}

hipError_t normalise_run(const double* logw, int J, double* out, double* stats, hipStream_t s, double* wout) {
  if (J > MAX_J || J < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(normalise_kernel, dim3(1), dim3(1024), 0, s, logw, J, out, stats, wout);
  return hipGetLastError();
}

hipError_t resample_run(const ResampleArgs& a, hipStream_t s) {
  if (a.J > MAX_J) return hipErrorInvalidValue;
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(1024), sys_smem_bytes(a.J), s, a);
  return hipGetLastError();
}

hipError_t multinomial_run(const double* w, int J, const double* u_arr, int32_t* anc, int32_t* placement,
                           hipStream_t s) {
  if (J > MAX_J || J < 1 || !u_arr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(multinomial_kernel, dim3(1), dim3(1024), sys_smem_bytes(J), s, w, J, u_arr, anc, placement);
  return hipGetLastError();
}

hipError_t systematic_run(const double* w, int J, double u, int32_t* anc, int32_t* placement, hipStream_t s) {
  if (J > MAX_J || J < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(systematic_kernel, dim3(1), dim3(1024), sys_smem_bytes(J), s, w, J, u, anc, placement);
  return hipGetLastError();
}

hipError_t gather_rows_run(int J, int64_t D, const int32_t* placement, float* a0, float* a1, hipStream_t s) {
  dim3 grid(nblocks(D, MOVE_ELEMS), J);
  hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, s, D, placement, a0, a1);
  return hipGetLastError();
}

hipError_t philox_run(uint32_t k0, uint32_t k1, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, k0, k1, c1, c2, c3, n, out);
  return hipGetLastError();
}

hipError_t prior_draw_run(float* theta, int J, int64_t D, float prior_std, uint32_t k0, uint32_t k1, hipStream_t s) {
  dim3 grid(nblocks(D, MOVE_ELEMS), J);
  hipLaunchKernelGGL(prior_draw_kernel, grid, dim3(256), 0, s, theta, D, prior_std, k0, k1);
  return hipGetLastError();
}

hipError_t posterior_mean_run(const float* theta, const double* w, int J, int64_t D, double* out, hipStream_t s) {
  hipLaunchKernelGGL(posterior_mean_kernel, dim3(nblocks(D, 256)), dim3(256), 0, s, theta, w, J, D, out);
  return hipGetLastError();
}

hipError_t mean_change_run(const double* cur, const double* prev, int64_t D, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(mean_change_kernel, dim3(1), dim3(1024), 0, s, cur, prev, D, out2);
  return hipGetLastError();
}

hipError_t predictive_run(const float* logp, int64_t ld, const double* logw, int J, int C, int64_t n,
                          const int32_t* y, float* probs, double* per_sample, hipStream_t s) {
  if (C > 16) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(predictive_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, logp, ld, logw, J, C, n, y, probs,
                     per_sample);
  return hipGetLastError();
}

hipError_t predictive_finish_run(const double* per_sample, int64_t n, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(predictive_finish_kernel, dim3(1), dim3(1024), 0, s, per_sample, n, out2);
  return hipGetLastError();
}

hipError_t fill_f64_run(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t grad_with_prior_run(const float* theta, const float* g, float* out, int64_t n, float ipv, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(grad_with_prior_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, theta, g, out, n, ipv);
  return hipGetLastError();
}

hipError_t lp_current_run(const double* ll, const double* tsq, int J, double lambda, double inv_2pv, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(lp_current_kernel, dim3(nblocks(J, 256)), dim3(256), 0, s, ll, tsq, J, lambda, inv_2pv, out);
  return hipGetLastError();
}

hipError_t f64_to_f32_run(const double* in, int64_t n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nblocks(n, 256)), dim3(256), 0, s, in, n, out);
  return hipGetLastError();
}

hipError_t sq_norm_rows_run(const float* a, int J, int64_t D, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sq_norm_rows_kernel, dim3(J), dim3(256), 0, s, a, D, out);
  return hipGetLastError();
}

}  // namespace smc
