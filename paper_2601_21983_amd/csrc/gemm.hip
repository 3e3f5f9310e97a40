// Batched MFMA GEMM kernels for gfx950 (CDNA4) with fused epilogues; the tile
// main loop (LDS staging, MFMA forms, XCD-aware tile order) is in gemm_core.h.
#include "gemm.h"
#include "gemm_core.h"

#include <type_traits>

namespace smc {

namespace {

using namespace gcore;

struct SplitIdx {
  int64_t colpart;  // (col / cs) * sC + (col % cs) * cstr + b * sb
  int rq, rr;       // row / rs, row % rs for the base row
};

__device__ __forceinline__ SplitIdx split_base(const OutDesc& d, int b, int rbase, int col) {
  SplitIdx s;
  s.colpart = (int64_t)b * d.sb + (int64_t)(col / d.cs) * d.sC + (int64_t)(col % d.cs) * d.cstr;
  s.rq = rbase / d.rs;
  s.rr = rbase - s.rq * d.rs;
  return s;
}
__device__ __forceinline__ int64_t split_at(const OutDesc& d, const SplitIdx& s, int drow) {
  int rq = s.rq, rr = s.rr + drow;
  while (rr >= d.rs) { rr -= d.rs; ++rq; }
  return s.colpart + (int64_t)rq * d.sR + (int64_t)rr * d.rstr;
}

template <int ACT>
__device__ __forceinline__ float act_apply(float v) {
  if constexpr (ACT == ACT_RELU) return fmaxf(v, 0.0f);
  else if constexpr (ACT == ACT_TANH) return tanhf(v);
  else return v;
}
template <int ACT>
__device__ __forceinline__ float act_deriv(float a) {
  if constexpr (ACT == ACT_RELU) return a > 0.0f ? 1.0f : 0.0f;
  else return 1.0f - a * a;
}

// LDS stages and workgroups per CU: the BF16 128x128 tile as four waves of 64x64 (the short-K
// products of the hidden layers) keeps one stage (37 KB) and is compiled for three workgroups per
// CU; the others follow gemm_core.h
template <typename T, int BM, int BN, int WM, int WN>
constexpr bool short_k_tile() {
  return sizeof(T) == 2 && BM == 128 && BN == 128 && WM == 64 && WN == 64;
}
template <typename T, int BM, int BN, int WM, int WN>
constexpr int gemm_nbuf() {
  return short_k_tile<T, BM, BN, WM, WN>() ? 1 : tile_nbuf(BM, BN, (int)sizeof(T));
}
template <typename T, int BM, int BN, int WM, int WN>
constexpr int gemm_minb() {
  return short_k_tile<T, BM, BN, WM, WN>() ? 3 : tile_minb(BM, BN, (int)sizeof(T));
}

// ACT: activation of the FWD epilogue / derivative of the DELTA epilogue (-1: none)
// F32O: the FWD epilogue stores FP32 values (BF16 operands only)
template <typename T, int BM, int BN, int WM, int WN, int EPI, int ACT, bool F32O>
// the second bound is waves per SIMD: gemm_minb workgroups per CU of NT / 256 waves per SIMD each
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64,
                             (gemm_minb<T, BM, BN, WM, WN>()) * (BM / WM) * (BN / WN) / 4) void gemm_nt(
    const GemmParams p) {
  constexpr int NT = (BM / WM) * (BN / WN) * 64;  // one wave per WM x WN sub-tile
  constexpr int NWN = BN / WN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int STAGE = (BM + BN) * LDS_ROW;
  constexpr int NBUF = gemm_nbuf<T, BM, BN, WM, WN>();
  // the staged epilogue's slab ([BM/WM * 32 rows][BN + pad] floats plus row and column tables) may
  // need more than the main loop's stages when the waves are stacked four deep
  constexpr int SLAB_NEED = (BM / WM) * 32 * (BN + 4) * 4 + ((BM / WM) * 32 + BN) * 8;
  constexpr int SMEM = NBUF * STAGE > SLAB_NEED ? NBUF * STAGE : SLAB_NEED;
  __shared__ __attribute__((aligned(16))) char smem[SMEM];

  const int b = blockIdx.y;
  int tm, tn;
  tile_order((p.M + BM - 1) / BM, (p.N + BN - 1) / BN, blockIdx.x, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const int M = p.M, N = p.N;
  f32x16 acc[FM][FN];
  mainloop<T, BM, BN, WM, WN, NBUF>((const T*)p.A + (int64_t)b * p.sAb, (const T*)p.B + (int64_t)b * p.sBb, p.lda,
                                    p.ldb, M, N, p.K, m0, n0, smem, acc);

  // ------------------------------------------------------------------ epilogue
  // Staged path: one output whose columns are contiguous inside each column-split
  // segment goes through LDS, so each output row piece is written by consecutive
  // lanes with the widest aligned vector stores (16, 8 or 4/2 bytes).  The error
  // epilogue keeps FP32 products in LDS and multiplies them by act'(a) while it writes
  // them out, reading a (row-major like the output, no splits) with the same vectors.
  // A forward's second output may be transposed (rows contiguous): it is written from the
  // same slab, each column's runs of 32 rows as 16-byte vectors.
  const bool aux_rows = EPI == EPI_DELTA && p.aux.cstr == 1 && p.aux.rs >= (1 << 30) && p.aux.cs >= (1 << 30);
  const bool out1_cols = EPI == EPI_FWD && p.out1.ptr && p.out1.rstr == 1 && p.out1.rs >= (1 << 30);
  if (p.out0.cstr == 1 &&
      (EPI == EPI_GRAD || (EPI == EPI_FWD && (!p.out1.ptr || out1_cols)) || (aux_rows && !p.out1.ptr))) {
    // O: element of the LDS slab
    typedef typename std::conditional<EPI == EPI_GRAD || EPI == EPI_DELTA || (EPI == EPI_FWD && F32O), float,
                                      T>::type O;
    constexpr int OS = (int)sizeof(O);
    constexpr int ES = EPI == EPI_DELTA ? (int)sizeof(T) : OS;  // element of the output
    constexpr int SROW = BN + 16 / OS;  // padded LDS row, in elements
    O* slab = (O*)smem;                 // [NWM*32][SROW]
    constexpr int NWM = BM / WM;
    constexpr int SLAB_BYTES = NWM * 32 * SROW * OS;
    static_assert(SLAB_BYTES + (NWM * 32 + BN) * 8 <= SMEM, "slab does not fit in LDS");
    int64_t* rowaddr = (int64_t*)(smem + SLAB_BYTES);
    int64_t* colpart = rowaddr + NWM * 32;
    const OutDesc& d = p.out0;
    auto aligned = [&](int ve) {
      bool ok = ((uintptr_t)d.ptr % (uintptr_t)(ve * ES)) == 0 && d.rstr % ve == 0 && d.sR % ve == 0 &&
                d.sb % ve == 0 && d.sC % ve == 0 && d.cs % ve == 0;
      if (EPI == EPI_DELTA)
        ok = ok && ((uintptr_t)p.aux.ptr % (uintptr_t)(ve * ES)) == 0 && p.aux.rstr % ve == 0 && p.aux.sb % ve == 0;
      return ok;
    };
    const int vw = aligned(16 / ES) ? 16 / ES : (aligned(8 / ES) ? 8 / ES : 1);
    for (int lc = tid; lc < BN; lc += NT) {
      const int col = n0 + lc;
      colpart[lc] = col < N ? (int64_t)(col / d.cs) * d.sC + (col % d.cs) : -1;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      // each wave drops its 32-row block i into the slab
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int lc = wn * WN + j * 32 + (lane & 31);
        const int col = n0 + lc;
        float bias = 0.0f;
        if (EPI == EPI_FWD && p.bias && col < N) bias = p.bias[(int64_t)b * p.sbias + col];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int lr = wm * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
          float v = acc[i][j][q];
          if (EPI == EPI_FWD) v = act_apply<ACT>(v + bias);
          slab[lr * SROW + lc] = cvt_out<O>(v);
        }
      }
      if (tid < NWM * 32) {
        const int row = m0 + (tid >> 5) * WM + i * 32 + (tid & 31);
        const int rq = row / d.rs, rr = row - rq * d.rs;
        rowaddr[tid] = row < M ? (int64_t)b * d.sb + (int64_t)rq * d.sR + (int64_t)rr * d.rstr : -1;
      }
      __syncthreads();
      const int vpr = BN / vw;  // vectors per slab row
      if constexpr (EPI == EPI_DELTA) {
        for (int e = tid; e < NWM * 32 * vpr; e += NT) {
          const int lr = e / vpr, lc = (e - lr * vpr) * vw;
          const int64_t ra = rowaddr[lr];
          const int col = n0 + lc;
          if (ra < 0 || col >= N) continue;
          const int row = m0 + (lr >> 5) * WM + i * 32 + (lr & 31);
          T* dst = (T*)d.ptr + ra + colpart[lc];
          const T* ax = (const T*)p.aux.ptr + (int64_t)b * p.aux.sb + (int64_t)row * p.aux.rstr + col;
          const float* src = slab + lr * SROW + lc;
          auto one = [&](float v, T a) { return cvt_out<T>(v * act_deriv<ACT>(cvt_in<T>(a))); };
          if (col + vw <= N && vw * ES == 16) {
            typedef __attribute__((__vector_size__(16))) T TV;
            const TV a = *(const TV*)ax;
            TV o;
#pragma unroll
            for (int q = 0; q < 16 / ES; ++q) o[q] = one(src[q], a[q]);
            *(TV*)dst = o;
          } else if (col + vw <= N && vw * ES == 8) {
            typedef __attribute__((__vector_size__(8))) T TV;
            const TV a = *(const TV*)ax;
            TV o;
#pragma unroll
            for (int q = 0; q < 8 / ES; ++q) o[q] = one(src[q], a[q]);
            *(TV*)dst = o;
          } else {
            const int n = min(vw, N - col);
            for (int q = 0; q < n; ++q) dst[q] = one(src[q], ax[q]);
          }
        }
        __syncthreads();
        continue;
      }
      for (int e = tid; e < NWM * 32 * vpr; e += NT) {
        const int lr = e / vpr, lc = (e - lr * vpr) * vw;
        const int64_t ra = rowaddr[lr];
        const int col = n0 + lc;
        if (ra < 0 || col >= N) continue;
        O* dst = (O*)d.ptr + ra + colpart[lc];
        const O* src = slab + lr * SROW + lc;
        if (col + vw <= N && vw * OS == 16) {
          u32x4 v = *(const u32x4*)src;
          if (EPI == EPI_GRAD && p.beta) {
            f32x4 a = __builtin_bit_cast(f32x4, v), o = *(const f32x4*)dst;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] += o[q];
            v = __builtin_bit_cast(u32x4, a);
          }
          *(u32x4*)dst = v;
        } else if (col + vw <= N && vw * OS == 8) {
          typedef __attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t u32x2;
          typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
          u32x2 v = *(const u32x2*)src;
          if (EPI == EPI_GRAD && p.beta) {
            f32x2 a = __builtin_bit_cast(f32x2, v), o = *(const f32x2*)dst;
            a[0] += o[0];
            a[1] += o[1];
            v = __builtin_bit_cast(u32x2, a);
          }
          *(u32x2*)dst = v;
        } else {
          const int n = min(vw, N - col);
          for (int q = 0; q < n; ++q) {
            if (EPI == EPI_GRAD) dst[q] = p.beta ? dst[q] + src[q] : src[q];
            else dst[q] = src[q];
          }
        }
      }
      if (EPI == EPI_FWD && p.out1.ptr) {
        // transposed second output: thread (column, run of 32 rows, vector) with the vector index
        // fastest, so neighbouring lanes fill one column's contiguous run
        const OutDesc& d1 = p.out1;
        constexpr int V1 = 16 / OS, CPR = 32 / V1;
        const bool a1 = ((uintptr_t)d1.ptr % 16) == 0 && d1.sb % V1 == 0 && d1.sC % V1 == 0 && d1.cstr % V1 == 0;
        for (int e = tid; e < BN * NWM * CPR; e += NT) {
          const int c = e % CPR, r = (e / CPR) % NWM, lc = e / (CPR * NWM);
          const int col = n0 + lc;
          const int row0 = m0 + r * WM + i * 32 + c * V1;
          if (col >= N || row0 >= M) continue;
          O* dst = (O*)d1.ptr + (int64_t)b * d1.sb + (int64_t)(col / d1.cs) * d1.sC + (int64_t)(col % d1.cs) * d1.cstr +
                   row0;
          const O* src = slab + (r * 32 + c * V1) * SROW + lc;
          if (a1 && row0 + V1 <= M) {
            typedef __attribute__((__vector_size__(16))) O OV;
            OV v;
#pragma unroll
            for (int t = 0; t < V1; ++t) v[t] = src[t * SROW];
            *(OV*)dst = v;
          } else {
            const int n = min(V1, M - row0);
            for (int t = 0; t < n; ++t) dst[t] = src[t * SROW];
          }
        }
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * WN + j * 32 + (lane & 31);
      const int rbase = m0 + wm * WM + i * 32 + 4 * (lane >> 5);
      if (col >= N) continue;
      const SplitIdx s0 = split_base(p.out0, b, rbase, col);
      SplitIdx s1 = s0, sa = s0;
      if (EPI != EPI_GRAD && p.out1.ptr) s1 = split_base(p.out1, b, rbase, col);
      if (EPI == EPI_DELTA) sa = split_base(p.aux, b, rbase, col);
      float bias = 0.0f;
      if (EPI == EPI_FWD && p.bias) bias = p.bias[(int64_t)b * p.sbias + col];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int dr = 8 * (q >> 2) + (q & 3);
        if (rbase + dr >= M) continue;
        float v = acc[i][j][q];
        if (EPI == EPI_GRAD) {
          float* g = (float*)p.out0.ptr + split_at(p.out0, s0, dr);
          *g = p.beta ? *g + v : v;
        } else {
          if (EPI == EPI_FWD) {
            v = act_apply<ACT>(v + bias);
            if (F32O) {
              *((float*)p.out0.ptr + split_at(p.out0, s0, dr)) = v;
              if (p.out1.ptr) *((float*)p.out1.ptr + split_at(p.out1, s1, dr)) = v;
              continue;
            }
          } else {
            const float a = cvt_in<T>(*((const T*)p.aux.ptr + split_at(p.aux, sa, dr)));
            v *= act_deriv<ACT>(a);
          }
          *((T*)p.out0.ptr + split_at(p.out0, s0, dr)) = cvt_out<T>(v);
          if (p.out1.ptr) *((T*)p.out1.ptr + split_at(p.out1, s1, dr)) = cvt_out<T>(v);
        }
      }
    }
  }
}

template <typename T, int BM, int BN, int WM, int WN, int EPI, int ACT>
hipError_t launch_one(const GemmParams& p, dim3 grid, hipStream_t s) {
  if constexpr (EPI == EPI_FWD && std::is_same<T, __bf16>::value) {
    if (p.out_f32) {
      hipLaunchKernelGGL((gemm_nt<T, BM, BN, WM, WN, EPI, ACT, true>), grid, dim3((BM / WM) * (BN / WN) * 64), 0, s,
                         p);
      return hipGetLastError();
    }
  } else if (EPI != EPI_FWD) {
    if (p.out_f32) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((gemm_nt<T, BM, BN, WM, WN, EPI, ACT, false>), grid, dim3((BM / WM) * (BN / WN) * 64), 0, s, p);
  return hipGetLastError();
}

// GRAD_ONLY: a tile shape that only the weight gradients use (the other epilogues are not
// instantiated for it)
template <typename T, int BM, int BN, int WM, int WN, bool GRAD_ONLY = false>
hipError_t launch_cfg(const GemmParams& p, hipStream_t s) {
  const int64_t ntiles = (int64_t)((p.N + BN - 1) / BN) * ((p.M + BM - 1) / BM);
  if (ntiles > 0x7fffffff || p.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)ntiles, p.batch);
  if constexpr (GRAD_ONLY) {
    if (p.epi != EPI_GRAD) return hipErrorInvalidValue;
    return launch_one<T, BM, BN, WM, WN, EPI_GRAD, -1>(p, grid, s);
  } else {
    switch (p.epi) {
      case EPI_FWD:
        if (p.act == ACT_RELU) return launch_one<T, BM, BN, WM, WN, EPI_FWD, ACT_RELU>(p, grid, s);
        if (p.act == ACT_TANH) return launch_one<T, BM, BN, WM, WN, EPI_FWD, ACT_TANH>(p, grid, s);
        return launch_one<T, BM, BN, WM, WN, EPI_FWD, -1>(p, grid, s);
      case EPI_GRAD: return launch_one<T, BM, BN, WM, WN, EPI_GRAD, -1>(p, grid, s);
      case EPI_DELTA:
        if (p.act == ACT_RELU) return launch_one<T, BM, BN, WM, WN, EPI_DELTA, ACT_RELU>(p, grid, s);
        if (p.act == ACT_TANH) return launch_one<T, BM, BN, WM, WN, EPI_DELTA, ACT_TANH>(p, grid, s);
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
}

}  // namespace

hipError_t gemm_run(const GemmParams& p, int type, hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return hipSuccess;
  if (p.K <= 0) return hipErrorInvalidValue;
  const int vec = type == GEMM_BF16 ? 8 : 4;
  if (p.K % vec || p.lda % vec || p.ldb % vec) return hipErrorInvalidValue;
  if (((uintptr_t)p.A | (uintptr_t)p.B) & 15) return hipErrorInvalidValue;
  if (!gcore::tile_offsets_fit(p.lda, p.ldb, vec == 8 ? 2 : 4)) return hipErrorInvalidValue;
  // the 256x128 tile keeps its 128 accumulators in registers only with the lean
  // epilogues (identity/ReLU forward, gradient); tanh and delta epilogues use 128x128
  const bool lean = p.epi == EPI_GRAD || (p.epi == EPI_FWD && p.act != ACT_TANH);
  const bool big = lean && (int64_t)p.M * p.N >= (int64_t)256 * 128 * 512;
  // narrow outputs (convolution channels, small weight-gradient blocks): 256x32 tiles for
  // N <= 32 and 32x128 tiles for M <= 32, so the matrix cores do not multiply padding
  if (type == GEMM_BF16) {
    if (p.N <= 32) return launch_cfg<__bf16, 256, 32, 64, 32>(p, stream);
    if (p.M <= 32) return launch_cfg<__bf16, 32, 128, 32, 32>(p, stream);
    // weight gradients (long K) run the large tile as sixteen waves of 64x32 (64 VGPRs, eight waves
    // per SIMD with two workgroups per CU) rather than four of 128x64 (244 VGPRs, two per SIMD):
    // more waves to cover the K-step barriers and LDS round trips (layer-1 weight gradient at
    // 30,000 samples 1.61 ms with four waves, 1.53 with eight of 64x64, 1.46 with sixteen).  The
    // forward (K = 784) lost 17% with eight waves and keeps four.
    if (big && p.epi == EPI_GRAD) return launch_cfg<__bf16, 256, 128, 64, 32, true>(p, stream);
    // smaller weight gradients: the 128x128 tile as eight waves of 64x32 (88 VGPRs, two workgroups
    // per CU): the 784-256-256-10 network's layer-2 GEMM class 1.87 -> 1.79 ms
    if (p.epi == EPI_GRAD) return launch_cfg<__bf16, 128, 128, 64, 32, true>(p, stream);
    return big ? launch_cfg<__bf16, 256, 128, 128, 64>(p, stream) : launch_cfg<__bf16, 128, 128, 64, 64>(p, stream);
  }
  if (p.N <= 32) return launch_cfg<float, 256, 32, 64, 32>(p, stream);
  if (p.M <= 32) return launch_cfg<float, 32, 128, 32, 32>(p, stream);
  // FP32 weight gradients too (one double-buffered workgroup per CU): 101 TFLOP/s with four waves,
  // 105 with eight, 109 with sixteen (69% of the FP32 matrix-core peak)
  if (big && p.epi == EPI_GRAD) return launch_cfg<float, 256, 128, 64, 32, true>(p, stream);
  return big ? launch_cfg<float, 256, 128, 128, 64>(p, stream) : launch_cfg<float, 128, 128, 64, 64>(p, stream);
}

}  // namespace smc
