// Batched MFMA GEMM with fused epilogues for the particle-batched network passes.
//
//   C[b][m][n] = sum_k A[b][m][k] * B[b][n][k]      (both operands K-contiguous)
//
// A row m lives at A + b*sAb + m*lda, B row n at B + b*sBb + n*ldb.  K must be a
// multiple of 8 (bf16) or 4 (fp32) and lda/ldb multiples of the same, with 16-byte
// aligned bases, so every 16-byte vector is either fully inside [0, K) or fully
// outside (outside vectors load as zero).  M and N are arbitrary.
#pragma once

#include "common.h"

namespace smc {

// Address of output element (b, row, col):
//   b*sb + (row / rs)*sR + (row % rs)*rstr + (col / cs)*sC + (col % cs)*cstr
// The two splits let one GEMM over the concatenation of all particles' units
// write straight into per-particle layouts.
struct OutDesc {
  void* ptr = nullptr;
  int64_t sb = 0, sR = 0, rstr = 0, sC = 0, cstr = 1;
  int rs = 1 << 30, cs = 1 << 30;
};

enum GemmEpi {
  EPI_FWD = 0,    // + bias, activation (or none), store as the operand type to out0 (and out1)
  EPI_GRAD = 1,   // fp32 store (beta = 0) or accumulate (beta = 1) into out0
  EPI_DELTA = 2,  // multiply by act'(a) with a read through `aux`, store to out0 (and out1)
};

enum GemmType { GEMM_F32 = 0, GEMM_BF16 = 1 };

struct GemmParams {
  const void* A = nullptr;
  const void* B = nullptr;
  int64_t lda = 0, ldb = 0, sAb = 0, sBb = 0;
  int M = 0, N = 0, K = 0, batch = 1;
  int epi = EPI_FWD;
  OutDesc out0, out1, aux;
  const float* bias = nullptr;  // bias[b*sbias + col]
  int64_t sbias = 0;
  int act = -1;                 // -1: identity
  int beta = 0;
  // EPI_FWD with BF16 operands: store FP32 outputs (for a consumer that splits them into
  // BF16 hi/lo pairs) instead of rounding them to BF16
  int out_f32 = 0;
};

hipError_t gemm_run(const GemmParams& p, int type, hipStream_t stream);

}  // namespace smc
