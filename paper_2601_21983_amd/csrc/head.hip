// Output layer of every particle's network on the matrix cores: logits,
// log-likelihood, the output-layer gradient and the error sent to the last
// hidden layer.
//
// For particle j and a tile of 64 samples (one 16-sample block per wave):
//   1. logits^T [16 classes x 16 samples] = Wc [16 x Hp] . A^T, where Wc holds
//      [W_L | b_L] zero-padded to 16 classes and Hp = roundup(H + 1, 16) columns,
//      and the staged activation tile A carries a column of ones at index H, so
//      the bias rides along in the contraction;
//   2. categorical: log p = z_y - logsumexp(z), delta = lambda (onehot - softmax(z));
//      Gaussian: log p = -1/2 log(2 pi s^2) - (y - z)^2 / (2 s^2), delta = lambda (y - z) / s^2
//      (the subset log-likelihood and its scaled gradient, Section 3, Eq. approx-grad).
//      In the 16x16 accumulator layout a lane holds classes 4g..4g+3 (g = lane/16)
//      of sample lane%16, so the softmax is a reduction over 4 registers and the
//      lanes g = 0..3;
//   3. delta_{L-1}^T [Hp x 16] = Wt [Hp x 16 classes] . delta^T: the accumulator of
//      step 2 is already the B operand of this product; the result times act'(a) is
//      staged in LDS and written sample-contiguous ([unit][sample]) for the
//      weight-gradient GEMM of the layer below;
//   4. dW_L [16 x Hp] += delta^T . [A | 1] over the tile's samples (bias column
//      included), kept in registers across tiles; each wave owns every fourth
//      16-column block.
// Split-BF16 form (SPL): every operand value v that differs between particles or
// states is carried as hi = bf16(v) and lo = bf16(v - hi); the products use
// hi*hi + hi*lo + lo*hi (lo*lo is below FP32 resolution), so logits and errors
// carry about 16 mantissa bits although every MFMA input is BF16.  The hidden
// activations arrive in FP32 and are split while they are staged in LDS; the
// weights are split when loaded.  Data X (a network without hidden layer) stays
// single BF16: its rounding is the same at every state and cancels in the
// log-likelihood differences that enter the importance weights.
// MFMA forms: bf16 v_mfma_f32_16x16x32_bf16 over two 16-wide K blocks at once (a
// lane supplies 4 consecutive K values of each block; a lone block, or a pair of
// products of one block such as w_lo a_hi + w_hi a_hi, fills the same 8 slots)
// and v_mfma_f32_16x16x16_bf16 for a block left over; fp32 v_mfma_f32_16x16x4_f32
// issued four times over a 4-wide K slice (instruction t takes component t; lane
// groups cover K offsets 4g + t), so both precisions read 4 consecutive K values
// per lane and block.  Accumulator layout: lane l holds rows 4(l/16) + i,
// column l % 16.
// Log-likelihoods are summed in FP64 in a fixed order.
#include "gemm_core.h"
#include "kernels.h"

#include <algorithm>

namespace smc {

namespace {

constexpr int HT = 64;  // samples per tile (16 per wave)
constexpr int HTHREADS = 256;
constexpr int MAXHB = 8;  // h-blocks per wave in the dW_L accumulator: Hp <= 4 * 16 * MAXHB = 512
constexpr int PF = 8;     // 8-byte chunks of the next activation tile prefetched per thread

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s16x4;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short s16x8;

template <typename T> struct V4;
template <> struct V4<__bf16> {
  typedef s16x4 type;
};
template <> struct V4<float> {
  typedef f32x4 type;
};

__device__ __forceinline__ f32x4 mma16(const s16x4& a, const s16x4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma16(const f32x4& a, const f32x4& b, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
  return c;
}
// Two 16-wide K blocks in one product: lane group g puts elements 4g..4g+3 of block 0 in K slots
// 8g..8g+3 and those of block 1 in slots 8g+4..8g+7, so the sum over the 32 slots covers both
// blocks.  BF16: one v_mfma_f32_16x16x32_bf16, which takes the matrix cores as long as one
// 16x16x16 product; FP32: the two 16-wide products.
__device__ __forceinline__ f32x4 mma16x2(const s16x4& a0, const s16x4& a1, const s16x4& b0, const s16x4& b1,
                                         f32x4 c) {
  const s16x8 a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
  const s16x8 b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}
__device__ __forceinline__ f32x4 mma16x2(const f32x4& a0, const f32x4& a1, const f32x4& b0, const f32x4& b1,
                                         f32x4 c) {
  return mma16(a1, b1, mma16(a0, b0, c));
}

template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4(const T* p) {
  return *(const typename V4<T>::type*)p;
}
template <typename T>
__device__ __forceinline__ typename V4<T>::type gather4(const T* p, int stride) {
  typename V4<T>::type v;
  if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = __builtin_bit_cast(short, p[t * stride]);
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = p[t * stride];
  }
  return v;
}
// two BF16 values as one 32-bit word, x in the low half
__device__ __forceinline__ uint32_t pack2(__bf16 x, __bf16 y) {
  return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
}
template <typename T>
__device__ __forceinline__ float v4_at(const typename V4<T>::type& v, int t) {
  if constexpr (sizeof(T) == 2) return from_bf16(__builtin_bit_cast(__bf16, (short)v[t]));
  else return v[t];
}
template <typename T>
__device__ __forceinline__ typename V4<T>::type pack4(const float* x) {
  typename V4<T>::type v;
  if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = __builtin_bit_cast(short, to_bf16(x[t]));
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = x[t];
  }
  return v;
}

struct HeadLayout {
  int Hp, AS, WT, DS, SS;  // padded widths / LDS row strides (elements)
  int offWt, offAs, offDt, offSt, offRed, total;  // byte offsets
  bool stage;
  int planes;              // 2 with split operands: Wc, Wt and As each have a lo plane after the hi plane
};

__host__ __device__ inline int rup(int x, int m) { return (x + m - 1) / m * m; }

template <typename T>
__host__ __device__ inline HeadLayout head_layout(int H, bool stage, bool spl) {
  HeadLayout L;
  const int e = (int)sizeof(T);
  L.planes = spl ? 2 : 1;
  L.Hp = rup(H + 1, 16);
  // activation / weight row stride: BF16 rows are an odd multiple of 16 elements (8 * odd
  // dwords), so the 16 rows a wave reads at once (fragment rows and activation columns) fall
  // on distinct banks; FP32 rows are padded by 32 bytes
  L.AS = e == 2 ? ((L.Hp / 16) % 2 ? L.Hp : L.Hp + 16) : L.Hp + 16 / e * 2;
  L.WT = 16 + 8 / e * 2;
  L.DS = HT + 16 / e;
  L.SS = HT + 16 / e;
  int off = L.planes * 16 * L.AS * e;  // Wc [16][AS] (per plane)
  off = rup(off, 16);
  L.offWt = off;
  off += L.planes * L.Hp * L.WT * e;
  off = rup(off, 16);
  L.offAs = off;
  off += L.planes * HT * L.AS * e;
  off = rup(off, 16);
  L.offDt = off;
  off += 16 * L.DS * e;
  off = rup(off, 16);
  L.offSt = off;
  L.stage = stage;
  if (stage) off += L.Hp * L.SS * e;
  off = rup(off, 16);
  L.offRed = off;
  off += 16 * 4 * (int)sizeof(double) + 64 * (int)sizeof(float);
  L.total = off;
  return L;
}

typedef __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t u32x2;

// LDS regions of the output-layer work (offsets from head_layout).
template <typename T>
struct HeadSmem {
  T *Wc, *Wt, *As, *WcLo, *WtLo, *AsLo, *Dt, *St;
  double* red;
};

template <typename T>
__device__ __forceinline__ HeadSmem<T> head_smem(char* base, const HeadLayout& Lo) {
  HeadSmem<T> S;
  S.Wc = (T*)base;
  S.Wt = (T*)(base + Lo.offWt);
  S.As = (T*)(base + Lo.offAs);
  S.WcLo = S.Wc + 16 * Lo.AS;  // lo planes (split operands only)
  S.WtLo = S.Wt + Lo.Hp * Lo.WT;
  S.AsLo = S.As + HT * Lo.AS;
  S.Dt = (T*)(base + Lo.offDt);
  S.St = (T*)(base + Lo.offSt);
  S.red = (double*)(base + Lo.offRed);
  return S;
}

// Output-layer weights of particle j into LDS: Wc[c][h] = [W | b], Wt[h][c] = W^T (zero
// padded), with their lo planes for split operands.
template <typename T, int MODE, bool SPL>
__device__ __forceinline__ void head_weights(const HeadArgs& a, const HeadLayout& Lo, const HeadSmem<T>& S, int j) {
  T *Wc = S.Wc, *Wt = S.Wt, *WcLo = S.WcLo, *WtLo = S.WtLo;
  const int H = a.H, C = a.C, Hp = Lo.Hp, AS = Lo.AS, WT = Lo.WT;
  const int tid = threadIdx.x;
  const float* wsrc = a.theta + (int64_t)j * a.D + a.offL;
  for (int e = tid; e < 16 * AS; e += HTHREADS) {
    const int c = e / AS, h = e - c * AS;
    const float v = (c < C && h <= H) ? wsrc[c * (H + 1) + h] : 0.0f;
    const T hi = cvt_out<T>(v);
    Wc[e] = hi;
    if (SPL) WcLo[e] = cvt_out<T>(v - cvt_in<T>(hi));
  }
  if (MODE == HEAD_TRAIN) {
    for (int e = tid; e < Hp * WT; e += HTHREADS) {
      const int h = e / WT, c = e - h * WT;
      const float v = (c < C && h < H) ? wsrc[c * (H + 1) + h] : 0.0f;
      const T hi = cvt_out<T>(v);
      Wt[e] = hi;
      if (SPL) WtLo[e] = cvt_out<T>(v - cvt_in<T>(hi));
    }
  }
}

// Steps 1-4 on the 64-sample activation tile staged in As (and AsLo): tile samples 0-31 are
// chunk samples s0.., tile samples 32-63 chunk samples s1.. (s1 = s0 + 32 for a contiguous
// tile).  Every thread of the workgroup calls it (it synchronises).
// TRN (ReLU networks, staged layout): the tile's activations also sit transposed in the St
// region ([unit][sample], written by the caller; rows H.. hold the ones column and zeros), the
// hidden error is computed sample-major (each lane ends with four consecutive samples of one
// unit) and stored straight to dT as one 4-sample vector, and the output-layer weight gradient
// reads its activation operand as vectors from the transposed copy.
template <typename T, int MODE, int NQ, bool SPL, bool TRN = false>
__device__ __forceinline__ void head_tile(const HeadArgs& a, const HeadLayout& Lo, const HeadSmem<T>& S, int j, int s0,
                                          int s1, float lam, float lam_b, bool alo, double& llacc, double& llacc_b,
                                          f32x4 (&dacc)[NQ]) {
  T *Wc = S.Wc, *Wt = S.Wt, *As = S.As, *WcLo = S.WcLo, *WtLo = S.WtLo, *AsLo = S.AsLo, *Dt = S.Dt, *St = S.St;
  const int H = a.H, C = a.C, Hp = Lo.Hp, AS = Lo.AS, WT = Lo.WT, DS = Lo.DS, SS = Lo.SS;
  const int NHB = Hp / 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  // ---- 1. logits^T for this wave's 16 samples
  const T* arow = As + (w * 16 + cl) * AS + 4 * g;
  const T* wrow = Wc + cl * AS + 4 * g;
  // two accumulators: products over pairs of K blocks, the second chain independent of the first
  f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f}, z2 = {0.0f, 0.0f, 0.0f, 0.0f};
  if (SPL) {
    // per block: w_lo a_hi + w_hi a_hi in one product; the w_hi a_lo terms over pairs of blocks
    const T* wrowlo = WcLo + cl * AS + 4 * g;
    const T* arowlo = AsLo + (w * 16 + cl) * AS + 4 * g;
    for (int kb = 0; kb < NHB; ++kb) {
      const typename V4<T>::type wv = ld4(wrow + kb * 16), av = ld4(arow + kb * 16);
      z = mma16x2(ld4(wrowlo + kb * 16), wv, av, av, z);
    }
    if (alo) {
      int kb = 0;
      for (; kb + 1 < NHB; kb += 2)
        z2 = mma16x2(ld4(wrow + kb * 16), ld4(wrow + kb * 16 + 16), ld4(arowlo + kb * 16),
                     ld4(arowlo + kb * 16 + 16), z2);
      if (kb < NHB) z2 = mma16(ld4(wrow + kb * 16), ld4(arowlo + kb * 16), z2);
    }
  } else {
    int kb = 0;
    for (; kb + 3 < NHB; kb += 4) {
      z = mma16x2(ld4(wrow + kb * 16), ld4(wrow + kb * 16 + 16), ld4(arow + kb * 16), ld4(arow + kb * 16 + 16), z);
      z2 = mma16x2(ld4(wrow + kb * 16 + 32), ld4(wrow + kb * 16 + 48), ld4(arow + kb * 16 + 32),
                   ld4(arow + kb * 16 + 48), z2);
    }
    for (; kb + 1 < NHB; kb += 2)
      z = mma16x2(ld4(wrow + kb * 16), ld4(wrow + kb * 16 + 16), ld4(arow + kb * 16), ld4(arow + kb * 16 + 16), z);
    if (kb < NHB) z2 = mma16(ld4(wrow + kb * 16), ld4(arow + kb * 16), z2);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) z[i] += z2[i];

  // ---- 2. likelihood and output error (sample cl, classes 4g + i)
  const int sl = w * 16 + cl;           // sample within the tile
  const int sg = sl < 32 ? s0 + sl : s1 + (sl - 32);  // sample within the chunk
  const bool valid = sg < a.m_valid;
  const bool segb = a.c0 + sg >= a.m_split;  // second segment of a two-segment target
  const float lm = segb ? lam_b : lam;
  float d[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (a.likelihood == 0) {
    float zz[4];
    float mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      zz[i] = (4 * g + i < C) ? z[i] : -INFINITY;
      mx = fmaxf(mx, zz[i]);
    }
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    float se = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) se += (4 * g + i < C) ? expf(zz[i] - mx) : 0.0f;
    se += __shfl_xor(se, 16, 64);
    se += __shfl_xor(se, 32, 64);
    const float lse = mx + logf(se);
    if (MODE == HEAD_PREDICT) {
      if (valid) {
        float* lp = a.logp + ((int64_t)j * a.ld_logp + a.c0 + sg) * C;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < C) lp[4 * g + i] = zz[i] - lse;
      }
    } else {
      const int y = valid ? a.ylab[a.c0 + sg] : -1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 4 * g + i;
        if (c == y) {
          llacc += (double)(zz[i] - lse);
          if (segb) llacc_b += (double)(zz[i] - lse);
        }
        if (MODE == HEAD_TRAIN && valid && c < C) d[i] = lm * ((c == y ? 1.0f : 0.0f) - expf(zz[i] - lse));
      }
    }
  } else {
    // one output: the value sits in lane group 0, register 0
    const float yv = valid ? a.yreal[a.c0 + sg] : 0.0f;
    const float r = yv - z[0];
    if (MODE == HEAD_PREDICT) {
      if (valid && g == 0) a.logp[(int64_t)j * a.ld_logp + a.c0 + sg] = z[0];
    } else if (g == 0 && valid) {
      const double l = (double)(a.gauss_c - 0.5f * r * r * a.inv_var);
      llacc += l;
      if (segb) llacc_b += l;
      if (MODE == HEAD_TRAIN) d[0] = lm * r * a.inv_var;
    }
  }

  if (MODE == HEAD_TRAIN && TRN) {
    // ---- 3. delta_{L-1} = delta W (times act'), sample-major: lane (g, cl) ends with samples
    // w*16 + 4g .. +3 of unit hb*16 + cl and stores them as one vector (ReLU: act' = [a > 0])
    const T* AsT = St;
    const int sl0 = w * 16 + 4 * g;                            // 4 samples, never across the halves
    const int sg0 = sl0 < 32 ? s0 + sl0 : s1 + (sl0 - 32);
    if (a.dT || a.dR) {
      const typename V4<T>::type bd = pack4<T>(d);
      for (int hb = 0; hb < NHB; ++hb) {
        f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
        if (SPL) v = mma16x2(bd, bd, ld4(WtLo + (hb * 16 + cl) * WT + 4 * g), ld4(Wt + (hb * 16 + cl) * WT + 4 * g), v);
        else v = mma16(bd, ld4(Wt + (hb * 16 + cl) * WT + 4 * g), v);
        const int h = hb * 16 + cl;
        if (h < H) {
          const typename V4<T>::type ah = ld4(AsT + h * SS + sl0);
          float dv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) dv[i] = v4_at<T>(ah, i) > 0.0f ? v[i] : 0.0f;
          if (a.dT)
            *(typename V4<T>::type*)((T*)a.dT + (int64_t)j * a.sdTj + (int64_t)h * a.sdTh + sg0) = pack4<T>(dv);
          if (a.dR) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              ((T*)a.dR)[(int64_t)j * a.sdRj + (int64_t)(sg0 + i) * a.sdRm + h] = cvt_out<T>(dv[i]);
          }
        }
      }
    }
    // delta^T to LDS for the dW_L product
#pragma unroll
    for (int i = 0; i < 4; ++i) Dt[(4 * g + i) * DS + sl] = cvt_out<T>(d[i]);
    __syncthreads();
    // ---- 4. dW_L += delta^T [A | 1] with the activation operand read from the transposed copy
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int hb = w + 4 * q;
      if (hb >= NHB) break;
#pragma unroll
      for (int kb = 0; kb < HT / 16; kb += 2) {
        const T* dr = Dt + cl * DS + kb * 16 + 4 * g;
        const T* ar = AsT + (hb * 16 + cl) * SS + kb * 16 + 4 * g;
        dacc[q] = mma16x2(ld4(dr), ld4(dr + 16), ld4(ar), ld4(ar + 16), dacc[q]);
      }
    }
  } else if (MODE == HEAD_TRAIN) {
    // ---- 3. delta_{L-1}^T = W^T delta^T (times act'), staged for sample-contiguous stores
    const bool dr_vec = a.dR && ((uintptr_t)a.dR % (4 * sizeof(T))) == 0 && a.sdRj % 4 == 0 && a.sdRm % 4 == 0;
    if (a.dT) {
      const typename V4<T>::type bd = pack4<T>(d);
      for (int hb = 0; hb < NHB; ++hb) {
        f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
        if (SPL) v = mma16x2(ld4(WtLo + (hb * 16 + cl) * WT + 4 * g), ld4(Wt + (hb * 16 + cl) * WT + 4 * g), bd, bd, v);
        else v = mma16(ld4(Wt + (hb * 16 + cl) * WT + 4 * g), bd, v);
        // activations of sample sl at units hb*16 + 4g .. +3, one vector read per plane; the
        // ReLU derivative needs only the hi plane (a value and its BF16 rounding share a sign)
        const typename V4<T>::type ah = ld4(As + sl * AS + hb * 16 + 4 * g);
        const bool need_lo = alo && a.act != ACT_RELU;
        typename V4<T>::type al = ah;
        if (need_lo) al = ld4(AsLo + sl * AS + hb * 16 + 4 * g);
        float dv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int h = hb * 16 + 4 * g + i;
          if (h < H) {
            const float av = v4_at<T>(ah, i) + (need_lo ? v4_at<T>(al, i) : 0.0f);
            dv[i] = v[i] * act_grad_from_out(av, a.act);
            if (Lo.stage) St[h * SS + sl] = cvt_out<T>(dv[i]);
            else ((T*)a.dT)[(int64_t)j * a.sdTj + (int64_t)h * a.sdTh + sg] = cvt_out<T>(dv[i]);
          }
        }
        if (a.dR) {
          // sample-major copy: the lane's four consecutive units as one vector when they are all real
          T* r = (T*)a.dR + (int64_t)j * a.sdRj + (int64_t)sg * a.sdRm + hb * 16 + 4 * g;
          if (dr_vec && hb * 16 + 4 * g + 3 < H) {
            *(typename V4<T>::type*)r = pack4<T>(dv);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (hb * 16 + 4 * g + i < H) r[i] = cvt_out<T>(dv[i]);
          }
        }
      }
    }
    // delta^T to LDS for the dW_L product
#pragma unroll
    for (int i = 0; i < 4; ++i) Dt[(4 * g + i) * DS + sl] = cvt_out<T>(d[i]);
    __syncthreads();
    if (a.dT && Lo.stage) {
      // rows h < H of 64 samples each (two runs of 32: s0.., s1..), 16-byte vectors
      constexpr int EPV = 16 / (int)sizeof(T);       // elements per vector
      constexpr int VPR = HT / EPV;                   // vectors per row
      for (int e = tid; e < H * VPR; e += HTHREADS) {
        const int h = e / VPR, v = e - h * VPR;
        const int t = v * EPV;                        // first tile sample of the vector
        const int dst = t < 32 ? s0 + t : s1 + (t - 32);
        const u32x4 val = *(const u32x4*)(St + h * SS + t);
        *(u32x4*)((T*)a.dT + (int64_t)j * a.sdTj + (int64_t)h * a.sdTh + dst) = val;
      }
    }
    // ---- 4. dW_L += delta^T [A | 1]: this wave owns h-blocks w, w+4, ...  Like the other weight
    // gradients, a product with the single-BF16 output error: the activations' hi plane only (the
    // rounding of the errors and of the activations changes from sample to sample and averages
    // out in the sum over samples)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int hb = w + 4 * q;
      if (hb >= NHB) break;
#pragma unroll
      for (int kb = 0; kb < HT / 16; kb += 2) {
        const T* dr = Dt + cl * DS + kb * 16 + 4 * g;
        const T* ar = As + (kb * 16 + 4 * g) * AS + hb * 16 + cl;
        dacc[q] = mma16x2(ld4(dr), ld4(dr + 16), gather4(ar, AS), gather4(ar + 16 * AS, AS), dacc[q]);
      }
    }
  }
}

// The workgroup's log-likelihood partial and output-layer gradient partial (slot `split`).
template <typename T, int MODE, int NQ>
__device__ __forceinline__ void head_finish(const HeadArgs& a, const HeadLayout& Lo, const HeadSmem<T>& S, int j,
                                            int split, double llacc, double llacc_b, const f32x4 (&dacc)[NQ]) {
  double* red = S.red;
  const int H = a.H, C = a.C;
  const int NHB = Lo.Hp / 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  if (MODE != HEAD_PREDICT) {
    const double v = wave_sum(llacc);
    const double vb = a.llpart_b ? wave_sum(llacc_b) : 0.0;
    __syncthreads();
    if (lane == 0) {
      red[w] = v;
      red[4 + w] = vb;
    }
    __syncthreads();
    if (tid == 0) {
      a.llpart[(int64_t)j * a.nsplit + split] = red[0] + red[1] + red[2] + red[3];
      if (a.llpart_b) a.llpart_b[(int64_t)j * a.nsplit + split] = red[4] + red[5] + red[6] + red[7];
    }
  }
  if (MODE == HEAD_TRAIN) {
    const int npair = C * (H + 1);
    float* dst = a.dWpart + ((int64_t)j * a.nsplit + split) * npair;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int hb = w + 4 * q;
      if (hb >= NHB) break;
      const int h = hb * 16 + cl;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 4 * g + i;
        if (c < C && h <= H) dst[c * (H + 1) + h] = dacc[q][i];
      }
    }
  }
}

// Two workgroups per CU (a register budget of 256 per lane; the wide-layer BF16 form spills a
// few dwords and still runs 20% faster at H = 256 than with one), except the split form with
// eight h-block accumulators, which would spill heavily.
template <typename T, int MODE, int NQ, bool SPL>
__global__ __launch_bounds__(HTHREADS, (SPL && NQ == 8) ? 1 : 2) void head_kernel(const HeadArgs a, const HeadLayout Lo) {
  extern __shared__ __attribute__((aligned(16))) char hsm[];
  const HeadSmem<T> S = head_smem<T>(hsm, Lo);
  T* As = S.As;
  T* AsLo = S.AsLo;
  const bool alo = SPL && a.a_f32;  // activations arrive in FP32 and get a lo plane
  const int H = a.H, AS = Lo.AS;
  const int j = blockIdx.y, split = blockIdx.x;
  const int tid = threadIdx.x;
  head_weights<T, MODE, SPL>(a, Lo, S, j);
  // activation tile: columns >= H are constant (1 at H, 0 beyond) for the whole kernel
  for (int e = tid; e < HT * (AS - H); e += HTHREADS) {
    const int s = e / (AS - H), h = H + (e - s * (AS - H));
    As[s * AS + h] = cvt_out<T>(h == H ? 1.0f : 0.0f);
    if (SPL) AsLo[s * AS + h] = cvt_out<T>(0.0f);
  }

  const float lam = a.scale ? (float)a.scale[j] : (float)a.lambda;
  const float lam_b = a.scale ? lam : (float)a.lambda_b;
  const T* Aj = (const T*)a.A + (int64_t)j * a.sAj;
  const float* Afj = (const float*)a.A + (int64_t)j * a.sAj;  // FP32 activations (alo)
  const int ntiles = (a.m_valid + HT - 1) / HT;
  const int t0 = split * a.tiles_per_split;
  const int t1 = min(ntiles, t0 + a.tiles_per_split);

  // activation tile loader: 8-byte chunks when rows allow it, else single elements
  constexpr int CE = 8 / (int)sizeof(T);  // elements per chunk
  const int ce = alo ? 4 : CE;             // FP32 activations: four per (16-byte) chunk
  const bool vec = (H % ce) == 0 && (a.sAm % ce) == 0 && (a.sAj % ce) == 0 && ((uintptr_t)a.A % (alo ? 16 : 8)) == 0;
  const int cpr = vec ? H / ce : H;       // chunks per row
  const int nch = HT * cpr;
  const float rcpr = 1.0f / (float)cpr;
  // chunk (s, c) of the activation tile.  BF16: 8 raw bytes (CE values).  FP32 (split): four
  // values read as one 16-byte vector and kept as {hi 0-1, hi 2-3, lo 0-1, lo 2-3}, pairs of
  // packed BF16 values.
  typedef typename std::conditional<SPL, u32x4, u32x2>::type PreT;
  PreT pre[PF];
  auto ld_chunk = [&](int tile, int s, int c) -> PreT {
    PreT v{};
    if constexpr (SPL) {
      if (alo) {
        const f32x4 f = *(const f32x4*)(Afj + (int64_t)(tile * HT + s) * a.sAm + c * 4);
        __bf16 hi[4], lo[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          hi[t] = to_bf16(f[t]);
          lo[t] = to_bf16(f[t] - from_bf16(hi[t]));
        }
        v[0] = pack2(hi[0], hi[1]);
        v[1] = pack2(hi[2], hi[3]);
        v[2] = pack2(lo[0], lo[1]);
        v[3] = pack2(lo[2], lo[3]);
        return v;
      }
    }
    const u32x2 r = *(const u32x2*)(Aj + (int64_t)(tile * HT + s) * a.sAm + c * CE);
    v[0] = r[0];
    v[1] = r[1];
    return v;
  };
  auto put_chunk = [&](int s, int c, PreT v) {
    if constexpr (SPL) {
      if (alo) {
        *(u32x2*)(As + s * AS + 4 * c) = u32x2{v[0], v[1]};
        *(u32x2*)(AsLo + s * AS + 4 * c) = u32x2{v[2], v[3]};
        return;
      }
    }
    *(u32x2*)(As + s * AS + c * CE) = u32x2{v[0], v[1]};
  };
  auto chunk_rc = [&](int e, int& s, int& c) {
    s = (int)(((float)e + 0.5f) * rcpr);
    c = e - s * cpr;
    if (c < 0) { --s; c += cpr; } else if (c >= cpr) { ++s; c -= cpr; }
  };
  auto prefetch = [&](int tile) {
    if (!vec) return;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * HTHREADS;
      if (e < nch) {
        int s, c;
        chunk_rc(e, s, c);
        pre[q] = ld_chunk(tile, s, c);
      }
    }
  };
  auto stage = [&](int tile) {
    if (vec) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int e = tid + q * HTHREADS;
        if (e < nch) {
          int s, c;
          chunk_rc(e, s, c);
          put_chunk(s, c, pre[q]);
        }
      }
      for (int e = tid + PF * HTHREADS; e < nch; e += HTHREADS) {
        int s, c;
        chunk_rc(e, s, c);
        put_chunk(s, c, ld_chunk(tile, s, c));
      }
    } else {
      for (int e = tid; e < nch; e += HTHREADS) {
        int s, c;
        chunk_rc(e, s, c);
        if (SPL && alo) {
          const float f = Afj[(int64_t)(tile * HT + s) * a.sAm + c];
          const T hv = cvt_out<T>(f);
          As[s * AS + c] = hv;
          AsLo[s * AS + c] = cvt_out<T>(f - cvt_in<T>(hv));
        } else {
          As[s * AS + c] = Aj[(int64_t)(tile * HT + s) * a.sAm + c];
        }
      }
    }
  };

  double llacc = 0.0, llacc_b = 0.0;
  f32x4 dacc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) dacc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  if (t0 < t1) prefetch(t0);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();  // previous tile's LDS reads are done
    stage(t);
    __syncthreads();
    if (t + 1 < t1) prefetch(t + 1);
    head_tile<T, MODE, NQ, SPL>(a, Lo, S, j, t * HT, t * HT + 32, lam, lam_b, alo, llacc, llacc_b, dacc);
  }
  head_finish<T, MODE, NQ>(a, Lo, S, j, split, llacc, llacc_b, dacc);
}

// ------------------------------------------------------------------ fused layer 1 + output layer
// For networks with one hidden layer of H <= 127 units: one workgroup computes, for 256
// samples and one particle j, z1 = X W1_j^T on the matrix cores (gemm_core.h; the weight
// copy holds 128 rows per particle, rows >= H zero), then applies bias and activation in
// registers and runs the output-layer steps (head_tile) on four 64-sample passes straight
// from the accumulators.  The hidden activations never reach HBM, and there is one launch
// per chunk instead of two.  Split operands: each staged X slice feeds one MFMA against
// the w_hi tile and one against the w_lo tile (the weight copy holds rows [w_hi | w_lo]),
// and the activations are split into hi/lo when they are written to LDS.
template <int ACT>
__device__ __forceinline__ float fused_act(float v) {
  if constexpr (ACT == ACT_RELU) return fmaxf(v, 0.0f);
  else return tanhf(v);
}

constexpr int FBM = 256, FBN = 128;  // tile: samples x (one particle's padded units)

// Pass q of the output-layer work takes row block q of both wave rows: tile samples 0-31 are
// chunk samples m0 + 32q.., tile samples 32-63 are m0 + 128 + 32q.., so all four waves stage
// activations in every pass.  TRN (ReLU): the activations' hi plane is also written transposed
// into the St region for the sample-major backward of head_tile.
template <int MODE, bool SPL, int ACT, bool TRN>
__global__ __launch_bounds__(HTHREADS, 2) void fwd_head_kernel(const GemmParams p, const HeadArgs a,
                                                                const HeadLayout Lo) {
  typedef __bf16 T;
  constexpr int WM = 128, WN = 64, FM = WM / 32, FN = WN / 32, NQ = 2;
  extern __shared__ __attribute__((aligned(16))) char fsm[];
  int tm, jp;
  gcore::tile_order((p.M + FBM - 1) / FBM, a.J, blockIdx.x, tm, jp);
  const int m0 = tm * FBM;
  f32x16 acc[FM][FN];
  // split: K = ldw over X (first half of its rows), B lo plane ldw elements after each row
  gcore::mainloop<T, FBM, FBN, WM, WN, 1, SPL>((const T*)p.A, (const T*)p.B, p.lda, p.ldb, p.M, a.J * FBN, p.K, m0,
                                               jp * FBN, fsm, acc, SPL ? (int64_t)p.K : 0);

  // the main loop ended with a barrier: its LDS stage is free for the output-layer work
  const HeadSmem<T> S = head_smem<T>(fsm, Lo);
  head_weights<T, MODE, SPL>(a, Lo, S, jp);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const int H = a.H, Hp = Lo.Hp, AS = Lo.AS, SS = Lo.SS;
  if (TRN && MODE == HEAD_TRAIN) {
    // constant rows of the transposed copy: the ones column (unit H) and zero padding
    for (int e = tid; e < (Hp - H) * HT; e += HTHREADS) {
      const int u = H + e / HT, sl = e % HT;
      S.St[u * SS + sl] = to_bf16(u == H ? 1.0f : 0.0f);
    }
  }
  const float lam = a.scale ? (float)a.scale[jp] : (float)a.lambda;
  const float lam_b = a.scale ? lam : (float)a.lambda_b;
  const float* b1 = p.bias + (int64_t)jp * H;
  double llacc = 0.0, llacc_b = 0.0;
  f32x4 dacc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) dacc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const bool odd = lane & 1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // block q of this wave: tile rows wm*32 + (0..31), units wn*64 + jj*32 + lane%32
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      const int u = wn * WN + jj * 32 + (lane & 31);
      if (u >= Hp) continue;  // Hp is a multiple of 16: pairs agree
      const float bias = u < H ? b1[u] : 0.0f;
      const f32x16& ac = acc[q][jj];
      // lane pairs (units u, u+1) trade one value per row pair (r, r+1) over DPP, so that
      // the even lane writes row r and the odd lane row r+1, each as one 4-byte store
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        const int r = wm * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const float v0 = u < H ? fused_act<ACT>(ac[e] + bias) : (u == H ? 1.0f : 0.0f);      // row r
        const float v1 = u < H ? fused_act<ACT>(ac[e + 1] + bias) : (u == H ? 1.0f : 0.0f);  // row r + 1
        const float recv = __builtin_bit_cast(
            float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, odd ? v0 : v1), 0xB1, 0xF, 0xF, false));
        const float c0 = odd ? recv : v0;  // unit u & ~1
        const float c1 = odd ? v1 : recv;  // unit u | 1
        const int off = (odd ? r + 1 : r) * AS + (u & ~1);
        const __bf16 h0 = to_bf16(c0), h1 = to_bf16(c1);
        *(uint32_t*)(S.As + off) = pack2(h0, h1);
        if (SPL) *(uint32_t*)(S.AsLo + off) = pack2(to_bf16(c0 - from_bf16(h0)), to_bf16(c1 - from_bf16(h1)));
      }
      if (TRN && MODE == HEAD_TRAIN && u < H) {
        // four consecutive tile rows of unit u per 8-byte store
#pragma unroll
        for (int ee = 0; ee < 4; ++ee) {
          float v4[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) v4[t] = fused_act<ACT>(ac[4 * ee + t] + bias);
          *(typename V4<T>::type*)(S.St + u * SS + wm * 32 + 8 * ee + 4 * (lane >> 5)) = pack4<T>(v4);
        }
      }
    }
    __syncthreads();
    head_tile<T, MODE, NQ, SPL, TRN>(a, Lo, S, jp, m0 + 32 * q, m0 + 128 + 32 * q, lam, lam_b, SPL, llacc, llacc_b,
                                     dacc);
    __syncthreads();
  }
  head_finish<T, MODE, NQ>(a, Lo, S, jp, tm, llacc, llacc_b, dacc);
}

// Sum the per-split partials of one chunk in a fixed order and fold them into the
// running totals: ll_acc[j] (+)= sum, grad[j][offL + e] (+)= sum.  Block (j, y) takes
// particle j and columns [64 y, 64 y + 64) of the output-layer gradient; its four waves
// sum the splits k = w (mod 4) with four FP64 accumulators (so each lane keeps several
// loads in flight), and wave 0 adds the four waves' sums in order.  Block (j, 0) also sums
// the log-likelihood partials (lanes over k, then a butterfly).
constexpr int HR_COLS = 64, HR_WAVES = 4;

__device__ double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(HR_COLS * HR_WAVES) void head_reduce_kernel(const HeadArgs a, int beta, int with_grad) {
  const int j = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (blockIdx.y == 0 && w == 0) {
    const double* lp = a.llpart + (int64_t)j * a.nsplit;
    double s = 0.0;
    for (int k = lane; k < a.nsplit; k += 64) s += lp[k];
    s = wave_sum_f64(s);
    if (lane == 0) a.ll_acc[j] = beta ? a.ll_acc[j] + s : s;
    if (a.ll_acc_b) {
      const double* lb = a.llpart_b + (int64_t)j * a.nsplit;
      double sb = 0.0;
      for (int k = lane; k < a.nsplit; k += 64) sb += lb[k];
      sb = wave_sum_f64(sb);
      if (lane == 0) a.ll_acc_b[j] = beta ? a.ll_acc_b[j] + sb : sb;
    }
  }
  if (!with_grad) return;
  __shared__ double part[HR_WAVES][HR_COLS];
  const int npair = a.C * (a.H + 1);
  const int e = blockIdx.y * HR_COLS + lane;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < npair) {
    const float* src = a.dWpart + (int64_t)j * a.nsplit * npair + e;
    const int64_t st = (int64_t)HR_WAVES * npair;
    int k = w;
    for (; k + 3 * HR_WAVES < a.nsplit; k += 4 * HR_WAVES) {
      const float* q = src + (int64_t)k * npair;
      s0 += (double)q[0];
      s1 += (double)q[st];
      s2 += (double)q[2 * st];
      s3 += (double)q[3 * st];
    }
    for (; k < a.nsplit; k += HR_WAVES) s0 += (double)src[(int64_t)k * npair];
  }
  part[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (w == 0 && e < npair) {
    const double t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    float* gr = a.grad + (int64_t)j * a.D + a.offL;
    gr[e] = beta ? gr[e] + (float)t : (float)t;
  }
}

hipError_t head_reduce_run(const HeadArgs& a, int mode, hipStream_t s) {
  const int with_grad = mode == HEAD_TRAIN ? 1 : 0;
  const int ncol = with_grad ? (a.C * (a.H + 1) + HR_COLS - 1) / HR_COLS : 1;
  hipLaunchKernelGGL(head_reduce_kernel, dim3(a.J, ncol), dim3(HR_COLS * HR_WAVES), 0, s, a, a.beta, with_grad);
  return hipGetLastError();
}

constexpr int LDS_LIMIT = 160 * 1024;

// The staged layout (hidden error through LDS, sample-contiguous stores) when it leaves room for
// two workgroups per CU; wide hidden layers drop the staging area instead, since one workgroup
// per CU (four waves) leaves these latency-bound passes without a second workgroup to overlap.
template <typename T>
HeadLayout pick_layout(int H, bool spl) {
  const HeadLayout st = head_layout<T>(H, true, spl), un = head_layout<T>(H, false, spl);
  if (st.total <= LDS_LIMIT / 2) return st;
  if (un.total <= LDS_LIMIT / 2) return un;
  return st.total <= LDS_LIMIT ? st : un;
}

}  // namespace

bool head_supported(int H, int C, int type) {
  if (C < 1 || C > 16 || H < 1) return false;
  const HeadLayout L = type ? pick_layout<__bf16>(H, type == HEAD_BF16_SPLIT) : pick_layout<float>(H, false);
  return L.Hp <= 4 * 16 * MAXHB && L.total <= LDS_LIMIT;
}

hipError_t head_run(const HeadArgs& a, int mode, int type, hipStream_t s) {
  const int ntiles = (a.m_valid + HT - 1) / HT;
  if (ntiles <= 0) return hipSuccess;
  if (!head_supported(a.H, a.C, type)) return hipErrorInvalidValue;
  if (a.a_f32 && type != HEAD_BF16_SPLIT) return hipErrorInvalidValue;
  dim3 grid(a.nsplit, a.J);
#define HEAD_LAUNCH(T, MODE, SPL)                                                                        \
  do {                                                                                                   \
    const HeadLayout L = pick_layout<T>(a.H, SPL);                                                       \
    const int nq = (L.Hp / 16 + 3) / 4;                                                                  \
    if (nq <= 2)                                                                                         \
      hipLaunchKernelGGL((head_kernel<T, MODE, 2, SPL>), grid, dim3(HTHREADS), (size_t)L.total, s, a, L); \
    else if (nq <= 4)                                                                                    \
      hipLaunchKernelGGL((head_kernel<T, MODE, 4, SPL>), grid, dim3(HTHREADS), (size_t)L.total, s, a, L); \
    else                                                                                                 \
      hipLaunchKernelGGL((head_kernel<T, MODE, 8, SPL>), grid, dim3(HTHREADS), (size_t)L.total, s, a, L); \
  } while (0)
  if (type == HEAD_BF16_SPLIT) {
    if (mode == HEAD_TRAIN) HEAD_LAUNCH(__bf16, HEAD_TRAIN, true);
    else if (mode == HEAD_FORWARD) HEAD_LAUNCH(__bf16, HEAD_FORWARD, true);
    else HEAD_LAUNCH(__bf16, HEAD_PREDICT, true);
  } else if (type == HEAD_BF16) {
    if (mode == HEAD_TRAIN) HEAD_LAUNCH(__bf16, HEAD_TRAIN, false);
    else if (mode == HEAD_FORWARD) HEAD_LAUNCH(__bf16, HEAD_FORWARD, false);
    else HEAD_LAUNCH(__bf16, HEAD_PREDICT, false);
  } else {
    if (mode == HEAD_TRAIN) HEAD_LAUNCH(float, HEAD_TRAIN, false);
    else if (mode == HEAD_FORWARD) HEAD_LAUNCH(float, HEAD_FORWARD, false);
    else HEAD_LAUNCH(float, HEAD_PREDICT, false);
  }
#undef HEAD_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode == HEAD_PREDICT) return e;
  return head_reduce_run(a, mode, s);
}

bool fwd_head_supported(int H, int C) {
  return H >= 1 && H < FBN && C >= 1 && C <= 16 && pick_layout<__bf16>(H, true).total <= LDS_LIMIT;
}

hipError_t fwd_head_run(const GemmParams& p, const HeadArgs& a, int mode, int split, int act, hipStream_t s) {
  if (p.M <= 0) return hipSuccess;
  if (!fwd_head_supported(a.H, a.C) || (act != ACT_RELU && act != ACT_TANH)) return hipErrorInvalidValue;
  if (p.K % 8 || p.lda % 8 || p.ldb % 8 || ((uintptr_t)p.A | (uintptr_t)p.B) & 15) return hipErrorInvalidValue;
  if (split && p.ldb < 2 * p.K) return hipErrorInvalidValue;  // rows [w_hi | w_lo]
  if (!gcore::tile_offsets_fit(p.lda, p.ldb, 2)) return hipErrorInvalidValue;
  const int nM = (p.M + FBM - 1) / FBM;
  if (a.nsplit != nM) return hipErrorInvalidValue;  // one partial per 256-sample tile
  const HeadLayout L = pick_layout<__bf16>(a.H, split != 0);
  const int stage = split ? gcore::stage_bytes<FBM, FBN, true>() : gcore::stage_bytes<FBM, FBN, false>();
  const size_t smem = (size_t)std::max(stage, L.total);
  const dim3 grid((unsigned)(nM * a.J));
#define FH_LAUNCH(MODE, SPL, ACT, TRN) \
  hipLaunchKernelGGL((fwd_head_kernel<MODE, SPL, ACT, TRN>), grid, dim3(HTHREADS), smem, s, p, a, L)
#define FH_ACT(MODE, SPL)                                          \
  do {                                                             \
    if (act == ACT_RELU && L.stage) FH_LAUNCH(MODE, SPL, ACT_RELU, true); \
    else if (act == ACT_RELU) FH_LAUNCH(MODE, SPL, ACT_RELU, false); \
    else FH_LAUNCH(MODE, SPL, ACT_TANH, false);                    \
  } while (0)
#define FH_MODE(SPL)                                           \
  do {                                                         \
    if (mode == HEAD_TRAIN) FH_ACT(HEAD_TRAIN, SPL);           \
    else if (mode == HEAD_FORWARD) FH_ACT(HEAD_FORWARD, SPL);  \
    else FH_ACT(HEAD_PREDICT, SPL);                            \
  } while (0)
  if (split) FH_MODE(true);
  else FH_MODE(false);
#undef FH_MODE
#undef FH_ACT
#undef FH_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || mode == HEAD_PREDICT) return e;
  return head_reduce_run(a, mode, s);
}

hipError_t head_set_smem_limits() {
#define HEAD_ATTR(T, MODE, NQ, SPL)                                                                       \
  hipFuncSetAttribute((const void*)head_kernel<T, MODE, NQ, SPL>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                      LDS_LIMIT)
#define HEAD_ATTR3(T, MODE, SPL)                                                                         \
  if ((e = HEAD_ATTR(T, MODE, 2, SPL)) != hipSuccess || (e = HEAD_ATTR(T, MODE, 4, SPL)) != hipSuccess || \
      (e = HEAD_ATTR(T, MODE, 8, SPL)) != hipSuccess) return e
  hipError_t e = hipSuccess;
  HEAD_ATTR3(float, HEAD_TRAIN, false);
  HEAD_ATTR3(float, HEAD_FORWARD, false);
  HEAD_ATTR3(float, HEAD_PREDICT, false);
  HEAD_ATTR3(__bf16, HEAD_TRAIN, false);
  HEAD_ATTR3(__bf16, HEAD_FORWARD, false);
  HEAD_ATTR3(__bf16, HEAD_PREDICT, false);
  HEAD_ATTR3(__bf16, HEAD_TRAIN, true);
  HEAD_ATTR3(__bf16, HEAD_FORWARD, true);
  HEAD_ATTR3(__bf16, HEAD_PREDICT, true);
#undef HEAD_ATTR3
#undef HEAD_ATTR
#define FH_ATTR(MODE, SPL, ACT, TRN)                                                                   \
  if ((e = hipFuncSetAttribute((const void*)fwd_head_kernel<MODE, SPL, ACT, TRN>,                        \
                               hipFuncAttributeMaxDynamicSharedMemorySize, LDS_LIMIT)) != hipSuccess) \
  return e
#define FH_ATTR2(MODE, SPL)            \
  FH_ATTR(MODE, SPL, ACT_RELU, true);  \
  FH_ATTR(MODE, SPL, ACT_RELU, false); \
  FH_ATTR(MODE, SPL, ACT_TANH, false)
  FH_ATTR2(HEAD_TRAIN, false);
  FH_ATTR2(HEAD_FORWARD, false);
  FH_ATTR2(HEAD_PREDICT, false);
  FH_ATTR2(HEAD_TRAIN, true);
  FH_ATTR2(HEAD_FORWARD, true);
  FH_ATTR2(HEAD_PREDICT, true);
#undef FH_ATTR2
#undef FH_ATTR
  return e;
}

}  // namespace smc
