// Matrix-core main loop shared by the batched GEMM (gemm.hip) and the fused
// layer-1 + output-layer kernel (head.hip).
//
// Tiling: a workgroup of 4, 8 or 16 wave64s computes a BM x BN tile; each wave
// owns a WM x WN sub-tile made of 32x32 MFMA blocks.  Every K step stages a
// 128-byte-deep slice of A and B (64 bf16 or 32 fp32) in LDS with a 16-byte row
// pad (row stride 144 B, so the 16-byte fragment reads of 16 consecutive rows hit
// distinct banks), prefetching the next slice into registers while the current
// one feeds the matrix cores.
//
// MFMA forms:
//   bf16: v_mfma_f32_32x32x16_bf16 - each lane supplies 8 consecutive K values
//   fp32: v_mfma_f32_32x32x2_f32   - each lane reads 4 consecutive K values and
//         issues 4 MFMAs, instruction c taking component c (lane halves cover
//         k and k+4), so one 16-byte LDS read feeds 4 instructions.
// Both operands use the same lane->k assignment, so any such assignment yields
// the same sum; only the row/column lane mapping (row = lane % 32) and the
// accumulator layout (row = 8*(q/4) + 4*(lane/32) + q%4, col = lane % 32) matter.
#pragma once
#include <algorithm>

#include "common.h"

namespace smc {
namespace gcore {

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

// The BF16 256x128 tile keeps one LDS stage so that two workgroups share a CU (one's
// prologue and epilogue overlap the other's matrix-core loop; measured 1.3-1.6x on the
// layer-1 GEMMs).  Other tiles, and FP32 (whose weight-gradient GEMM lost 15% that way),
// double-buffer: two workgroups per CU for the BF16 128x128 tile (74 KB), one for FP32's
// 256x128 (110 KB).
constexpr int tile_nbuf(int bm, int bn, int esz) { return (bm == 256 && bn == 128 && esz == 2) ? 1 : 2; }
// Workgroups per CU that a tile is compiled for (its register budget follows): the single-stage
// BF16 256x128 tile and the double-buffered BF16 128x128 tile (74 KB) fit two.
constexpr int tile_minb(int bm, int bn, int esz) {
  return (tile_nbuf(bm, bn, esz) == 1 || (bm == 128 && bn == 128 && esz == 2)) ? 2 : 1;
}

// Host check: the main loop addresses a tile's rows by 32-bit byte offsets from its first
// row, so 256 rows of the larger leading dimension must span less than 4 GiB.
inline bool tile_offsets_fit(int64_t lda, int64_t ldb, int esz) {
  return 256 * std::max(lda, ldb) * esz < ((int64_t)1 << 32);
}

// XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
// renumber them so that each XCD receives a contiguous range of tiles, and walk
// that range in groups of GROUP_M row-tiles per column-tile (the group's A panels
// stay in the XCD's L2 while the B panel streams once per group).
__device__ __forceinline__ void tile_order(int nM, int nN, int pid, int& tm, int& tn) {
  const int ntiles = nM * nN;
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

// LDS bytes of one stage: A rows, B rows (and the B lo rows of the split form)
template <int BM, int BN, bool SB>
constexpr int stage_bytes() { return (BM + (SB ? 2 : 1) * BN) * LDS_ROW; }

// acc[i][j] (+)= the BM x BN tile at (m0, n0) of A[M x K] . B[N x K]^T (rows lda / ldb
// apart).  Split form (SB): B has a second plane at b_lo elements after each row (the lo
// parts of split-BF16 weights), and acc accumulates A.B_hi^T + A.B_lo^T: each A fragment
// feeds two MFMAs, so A is loaded and staged once.  Rows beyond M or N are clamped (their
// results are garbage and must not be stored).  Ends with a barrier, after which smem may
// be reused.
template <typename T, int BM, int BN, int WM, int WN, int NBUF, bool SB = false>
__device__ __forceinline__ void mainloop(const T* __restrict__ A, const T* __restrict__ B, int64_t lda, int64_t ldb,
                                         int M, int N, int K, int m0, int n0, char* smem,
                                         f32x16 (&acc)[WM / 32][WN / 32], int64_t b_lo = 0) {
  constexpr int VEC = Mf<T>::VEC;
  constexpr int BKE = ROW_BYTES / (int)sizeof(T);
  constexpr int NWN = BN / WN;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int NT = (BM / WM) * (BN / WN) * 64;  // threads: one wave per WM x WN sub-tile
  constexpr int AV = BM * ROWV / NT;
  constexpr int BV = BN * ROWV / NT;
  constexpr int STAGE = stage_bytes<BM, BN, SB>();
  constexpr int NBV = SB ? 2 * BV : BV;  // B vectors per thread per stage (both planes)
  static_assert(NT == 256 || NT == 512 || NT == 1024, "four, eight or sixteen waves per workgroup");
  static_assert(AV >= 1 && BV >= 1 && BM * ROWV % NT == 0 && BN * ROWV % NT == 0, "tile too small");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;

  // per-thread source rows (clamped into range) as 32-bit byte offsets from the tile's first
  // row, so that the loads take a uniform 64-bit base plus one VGPR each
  const char* At = (const char*)(A + (int64_t)m0 * lda);
  const char* Bt = (const char*)(B + (int64_t)n0 * ldb);
  const char* Blo = Bt + b_lo * (int64_t)sizeof(T);
  uint32_t aoff[AV], boff[BV];
#pragma unroll
  for (int i = 0; i < AV; ++i) {
    const int r = (tid + i * NT) / ROWV;
    const int gr = min(m0 + r, M - 1) - m0;
    aoff[i] = (uint32_t)((gr * (int64_t)lda + ((tid + i * NT) % ROWV) * VEC) * (int64_t)sizeof(T));
  }
#pragma unroll
  for (int i = 0; i < BV; ++i) {
    const int r = (tid + i * NT) / ROWV;
    const int gr = min(n0 + r, N - 1) - n0;
    boff[i] = (uint32_t)((gr * (int64_t)ldb + ((tid + i * NT) % ROWV) * VEC) * (int64_t)sizeof(T));
  }
  const int kvec = (tid % ROWV) * VEC;  // same for every i since NT % ROWV == 0

  u32x4 ra[AV], rb[NBV];
  auto gload = [&](int kt) {
    const int k = kt * BKE + kvec;
    const bool ok = k < K;
    const uint32_t ko = (uint32_t)kt * ROW_BYTES;  // kept 32-bit: base + zext(offset) loads
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      ra[i] = ok ? *(const u32x4*)(At + (aoff[i] + ko)) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      const char* Bp = i >= BV ? Blo : Bt;
      rb[i] = ok ? *(const u32x4*)(Bp + (boff[i % BV] + ko)) : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto sstore = [&](int buf) {
    char* base = smem + buf * STAGE;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + i * NT;
      *(u32x4*)(base + (v / ROWV) * LDS_ROW + (v % ROWV) * 16) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NBV; ++i) {
      // lo plane rows follow the BN hi rows
      const int v = tid + (i % BV) * NT;
      *(u32x4*)(base + (BM + (i / BV) * BN + v / ROWV) * LDS_ROW + (v % ROWV) * 16) = rb[i];
    }
  };

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
      if (SB) {
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fb[j] = *(const u32x4*)(base + (BM + BN + wn * WN + j * 32 + frow) * LDS_ROW + ks * 32 + fhalf);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = Mf<T>::mma(fa[i], fb[j], acc[i][j]);
      }
    }
    if (NBUF == 2) {
      if (kt + 1 < nk) sstore(buf ^ 1);
    } else if (kt + 1 < nk) {
      __syncthreads();  // every wave is done reading the stage
      sstore(0);
    }
    __syncthreads();
  }
}

}  // namespace gcore
}  // namespace smc
