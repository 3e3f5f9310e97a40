// MFMA GEMM kernels for gfx950 (CDNA4).
//
// Tiling: a 256-thread workgroup (4 wave64s) computes a BM x BN tile; each wave
// owns a WM x WN sub-tile made of 32x32 MFMA blocks.  Every K step stages a
// 128-byte-deep slice of A and B (64 bf16 or 32 fp32) in LDS with a 16-byte row
// pad (row stride 144 B, so the 16-byte fragment reads of 16 consecutive rows hit
// distinct banks) and double-buffers it, prefetching the next slice into
// registers while the current one feeds the matrix cores.
//
// MFMA forms:
//   bf16: v_mfma_f32_32x32x16_bf16 - each lane supplies 8 consecutive K values
//   fp32: v_mfma_f32_32x32x2_f32   - each lane reads 4 consecutive K values and
//         issues 4 MFMAs, instruction c taking component c (lane halves cover
//         k and k+4), so one 16-byte LDS read feeds 4 instructions.
// Both operands use the same lane->k assignment, so any such assignment yields
// the same sum; only the row/column lane mapping (row = lane % 32) and the
// accumulator layout (row = 8*(q/4) + 4*(lane/32) + q%4, col = lane % 32) matter.
#include "gemm.h"

#include <type_traits>

namespace smc {

namespace {

constexpr int THREADS = 256;
constexpr int ROW_BYTES = 128;          // K slice per stage, in bytes
constexpr int LDS_ROW = ROW_BYTES + 16; // padded LDS row stride
constexpr int ROWV = ROW_BYTES / 16;    // 16-byte vectors per row

template <typename T> struct Mf;
template <> struct Mf<__bf16> {
  static constexpr int VEC = 8;
  __device__ static __forceinline__ f32x16 mma(const u32x4& a, const u32x4& b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
  }
};
template <> struct Mf<float> {
  static constexpr int VEC = 4;
  __device__ static __forceinline__ f32x16 mma(const u32x4& a, const u32x4& b, f32x16 c) {
    const f32x4 av = __builtin_bit_cast(f32x4, a);
    const f32x4 bv = __builtin_bit_cast(f32x4, b);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[0], bv[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[1], bv[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[2], bv[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[3], bv[3], c, 0, 0, 0);
    return c;
  }
};

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

// ACT: activation of the FWD epilogue / derivative of the DELTA epilogue (-1: none)
// F32O: the FWD epilogue stores FP32 values (BF16 operands only)
// The BF16 256x128 tile keeps one LDS stage so that two workgroups share a CU (one's
// prologue and epilogue overlap the other's matrix-core loop; measured 1.3-1.6x on the
// layer-1 GEMMs).  Other tiles, and FP32 (whose weight-gradient GEMM lost 15% that way),
// double-buffer with one workgroup per CU.
constexpr int tile_nbuf(int bm, int bn, int esz) { return (bm == 256 && bn == 128 && esz == 2) ? 1 : 2; }
constexpr int tile_minb(int bm, int bn, int esz) { return tile_nbuf(bm, bn, esz) == 1 ? 2 : 1; }

template <typename T, int BM, int BN, int WM, int WN, int EPI, int ACT, bool F32O>
__global__ __launch_bounds__(THREADS, tile_minb(BM, BN, (int)sizeof(T))) void gemm_nt(const GemmParams p) {
  constexpr int VEC = Mf<T>::VEC;
  constexpr int BKE = ROW_BYTES / (int)sizeof(T);
  constexpr int NWN = BN / WN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int AV = BM * ROWV / THREADS;
  constexpr int BV = BN * ROWV / THREADS;
  constexpr int STAGE = (BM + BN) * LDS_ROW;
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  static_assert(AV >= 1 && BV >= 1, "tile too small");

  constexpr int NBUF = tile_nbuf(BM, BN, (int)sizeof(T));
  __shared__ __attribute__((aligned(16))) char smem[NBUF * STAGE];

  const int b = blockIdx.y;
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
  // renumber them so that each XCD receives a contiguous range of tiles, and walk
  // that range in groups of GROUP_M row-tiles per column-tile (the group's A panels
  // stay in the XCD's L2 while the B panel streams once per group).
  int tm, tn;
  {
    const int nM = (p.M + BM - 1) / BM, nN = (p.N + BN - 1) / BN;
    const int ntiles = nM * nN;
    const int pid = blockIdx.x;
    int t = pid;
    if (ntiles % 8 == 0) t = (pid % 8) * (ntiles / 8) + pid / 8;
    constexpr int GROUP_M = 8;
    const int group = t / (GROUP_M * nN);
    const int first_m = group * GROUP_M;
    const int gm = min(nM - first_m, GROUP_M);
    const int r = t - group * GROUP_M * nN;
    tm = first_m + r % gm;
    tn = r / gm;
  }
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const T* __restrict__ A = (const T*)p.A + (int64_t)b * p.sAb;
  const T* __restrict__ B = (const T*)p.B + (int64_t)b * p.sBb;
  const int M = p.M, N = p.N, K = p.K;

  // per-thread global source rows (clamped into range; results outside are not stored)
  const T* arow[AV];
  const T* brow[BV];
#pragma unroll
  for (int i = 0; i < AV; ++i) {
    const int r = (tid + i * THREADS) / ROWV;
    const int gr = min(m0 + r, M - 1);
    arow[i] = A + (int64_t)gr * p.lda + ((tid + i * THREADS) % ROWV) * VEC;
  }
#pragma unroll
  for (int i = 0; i < BV; ++i) {
    const int r = (tid + i * THREADS) / ROWV;
    const int gr = min(n0 + r, N - 1);
    brow[i] = B + (int64_t)gr * p.ldb + ((tid + i * THREADS) % ROWV) * VEC;
  }
  const int kvec = (tid % ROWV) * VEC;  // same for every i since THREADS % ROWV == 0

  u32x4 ra[AV], rb[BV];
  auto gload = [&](int kt) {
    const int k = kt * BKE + kvec;
    const bool ok = k < K;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      ra[i] = ok ? *(const u32x4*)(arow[i] + (int64_t)kt * BKE) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      rb[i] = ok ? *(const u32x4*)(brow[i] + (int64_t)kt * BKE) : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf) {
    char* base = smem + buf * STAGE;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + i * THREADS;
      *(u32x4*)(base + (v / ROWV) * LDS_ROW + (v % ROWV) * 16) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int v = tid + i * THREADS;
      *(u32x4*)(base + (BM + v / ROWV) * LDS_ROW + (v % ROWV) * 16) = rb[i];
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.0f;

  const int nk = (K + BKE - 1) / BKE;
  gload(0);
  sstore(0);
  __syncthreads();

  const int frow = lane & 31;
  const int fhalf = (lane >> 5) * 16;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = NBUF == 2 ? (kt & 1) : 0;
    if (kt + 1 < nk) gload(kt + 1);
    const char* base = smem + buf * STAGE;
#pragma unroll
    for (int ks = 0; ks < ROW_BYTES / 32; ++ks) {
      u32x4 fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        fa[i] = *(const u32x4*)(base + (wm * WM + i * 32 + frow) * LDS_ROW + ks * 32 + fhalf);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fb[j] = *(const u32x4*)(base + (BM + wn * WN + j * 32 + frow) * LDS_ROW + ks * 32 + fhalf);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mf<T>::mma(fa[i], fb[j], acc[i][j]);
    }
    if (NBUF == 2) {
      if (kt + 1 < nk) sstore(buf ^ 1);
    } else if (kt + 1 < nk) {
      __syncthreads();  // every wave is done reading the stage
      sstore(0);
    }
    __syncthreads();
  }

  // ------------------------------------------------------------------ epilogue
  // Staged path: one output whose columns are contiguous inside each column-split
  // segment goes through LDS, so each output row piece is written by consecutive
  // lanes with the widest aligned vector stores (16, 8 or 4/2 bytes).
  if (p.out0.cstr == 1 && (EPI == EPI_GRAD || (EPI == EPI_FWD && !p.out1.ptr))) {
    typedef typename std::conditional<EPI == EPI_GRAD || (EPI == EPI_FWD && F32O), float, T>::type O;
    constexpr int OS = (int)sizeof(O);
    constexpr int SROW = BN + 16 / OS;  // padded LDS row, in elements
    O* slab = (O*)smem;                 // [NWM*32][SROW]
    constexpr int NWM = BM / WM;
    constexpr int SLAB_BYTES = NWM * 32 * SROW * OS;
    static_assert(SLAB_BYTES + (NWM * 32 + BN) * 8 <= NBUF * STAGE, "slab does not fit in LDS");
    int64_t* rowaddr = (int64_t*)(smem + SLAB_BYTES);
    int64_t* colpart = rowaddr + NWM * 32;
    const OutDesc& d = p.out0;
    auto aligned = [&](int ve) {
      return ((uintptr_t)d.ptr % (uintptr_t)(ve * OS)) == 0 && d.rstr % ve == 0 && d.sR % ve == 0 &&
             d.sb % ve == 0 && d.sC % ve == 0 && d.cs % ve == 0;
    };
    const int vw = aligned(16 / OS) ? 16 / OS : (aligned(8 / OS) ? 8 / OS : 1);
    for (int lc = tid; lc < BN; lc += THREADS) {
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
      for (int e = tid; e < NWM * 32 * vpr; e += THREADS) {
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
      hipLaunchKernelGGL((gemm_nt<T, BM, BN, WM, WN, EPI, ACT, true>), grid, dim3(THREADS), 0, s, p);
      return hipGetLastError();
    }
  } else if (EPI != EPI_FWD) {
    if (p.out_f32) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((gemm_nt<T, BM, BN, WM, WN, EPI, ACT, false>), grid, dim3(THREADS), 0, s, p);
  return hipGetLastError();
}

template <typename T, int BM, int BN, int WM, int WN>
hipError_t launch_cfg(const GemmParams& p, hipStream_t s) {
  const int64_t ntiles = (int64_t)((p.N + BN - 1) / BN) * ((p.M + BM - 1) / BM);
  if (ntiles > 0x7fffffff || p.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)ntiles, p.batch);
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

}  // namespace

hipError_t gemm_run(const GemmParams& p, int type, hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return hipSuccess;
  if (p.K <= 0) return hipErrorInvalidValue;
  const int vec = type == GEMM_BF16 ? 8 : 4;
  if (p.K % vec || p.lda % vec || p.ldb % vec) return hipErrorInvalidValue;
  if (((uintptr_t)p.A | (uintptr_t)p.B) & 15) return hipErrorInvalidValue;
  // the 256x128 tile keeps its 128 accumulators in registers only with the lean
  // epilogues (identity/ReLU forward, gradient); tanh and delta epilogues use 128x128
  const bool lean = p.epi == EPI_GRAD || (p.epi == EPI_FWD && p.act != ACT_TANH);
  const bool big = lean && (int64_t)p.M * p.N >= (int64_t)256 * 128 * 512;
  // narrow outputs (convolution channels, small weight-gradient blocks): 256x32 tiles for
  // N <= 32 and 32x128 tiles for M <= 32, so the matrix cores do not multiply padding
  if (type == GEMM_BF16) {
    if (p.N <= 32) return launch_cfg<__bf16, 256, 32, 64, 32>(p, stream);
    if (p.M <= 32) return launch_cfg<__bf16, 32, 128, 32, 32>(p, stream);
    return big ? launch_cfg<__bf16, 256, 128, 128, 64>(p, stream) : launch_cfg<__bf16, 128, 128, 64, 64>(p, stream);
  }
  if (p.N <= 32) return launch_cfg<float, 256, 32, 64, 32>(p, stream);
  if (p.M <= 32) return launch_cfg<float, 32, 128, 32, 32>(p, stream);
  return big ? launch_cfg<float, 256, 128, 128, 64>(p, stream) : launch_cfg<float, 128, 128, 64, 64>(p, stream);
}

}  // namespace smc
