// FP64 64x64 tile engine for gfx950: one workgroup of 256 threads (four
// wave64s) owns one 64x64 output tile; each wave owns a 32x32 quadrant held
// as 2x2 accumulators of v_mfma_f64_16x16x4_f64.
//
// Accumulator layout (per lane l of wave w, accumulator (bi, bj), item v),
// as measured on gfx950 (item v of lane l holds row 4*v + l/16 of the 16x16
// block, column l%16):
//   row = 32*(w>>1) + 16*bi + 4*v + (l>>4),   col = 32*(w&1) + 16*bj + (l&15)
// MFMA operand layout for 16x16x4: lane l supplies A[l&15][l>>4] and
// B[l>>4][l&15].
//
// Operands stream from global memory (L2-resident tiles) through LDS in
// k-chunks of KC, stored k-major so that the 16 lanes of a fragment read 16
// consecutive doubles.
#pragma once
#include <hip/hip_runtime.h>
#include "devplan.hpp"

namespace mra {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;       // threads per workgroup
constexpr int KC = 16;        // k-chunk staged in LDS
constexpr int SLD = T + 4;    // LDS row pitch of a staged chunk (doubles)
constexpr int PLD = T + 1;    // LDS row pitch of a factorisation tile
constexpr int LDS_DOUBLES = T * PLD;   // >= 2 * KC * SLD

struct Acc {
  d4 c[2][2];
};

__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int acc_row(int bi, int v) {
  return 32 * (wave_id() >> 1) + 16 * bi + 4 * v + (lane_id() >> 4);
}
__device__ __forceinline__ int acc_col(int bj) { return 32 * (wave_id() & 1) + 16 * bj + (lane_id() & 15); }

__device__ __forceinline__ void acc_zero(Acc& a) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) a.c[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
}

// a (+)= C tile (row-major, leading dimension ldc)
__device__ __forceinline__ void acc_load(Acc& a, const double* C, int ldc, bool add = false) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = C[(int64_t)acc_row(bi, v) * ldc + acc_col(bj)];
        a.c[bi][bj][v] = add ? a.c[bi][bj][v] + x : x;
      }
}

__device__ __forceinline__ void acc_store(const Acc& a, double* C, int ldc) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(int64_t)acc_row(bi, v) * ldc + acc_col(bj)] = a.c[bi][bj][v];
}

// ---------------------------------------------------------------------------
// chunk loaders: fill s[k][i] (pitch SLD) for k in [0, KC), i in [0, T)
// ---------------------------------------------------------------------------

// element (i, k) = p[i * ld + k0 + k]  (row-major rows, k contiguous)
__device__ __forceinline__ void load_rows(double* s, const double* p, int ld, int k0) {
  const int t = threadIdx.x;
  const int i = t >> 2, kq = (t & 3) * 4;
  d4 v = *(const d4*)(p + (int64_t)i * ld + k0 + kq);
  s[(kq + 0) * SLD + i] = v[0];
  s[(kq + 1) * SLD + i] = v[1];
  s[(kq + 2) * SLD + i] = v[2];
  s[(kq + 3) * SLD + i] = v[3];
}

// element (i, k) = p[(k0 + k) * ld + i]  (k-major, i contiguous)
__device__ __forceinline__ void load_cols(double* s, const double* p, int ld, int k0) {
  const int t = threadIdx.x;
  const int k = t >> 4, iq = (t & 15) * 4;
  d4 v = *(const d4*)(p + (int64_t)(k0 + k) * ld + iq);
  *(d4*)(s + k * SLD + iq) = v;
}

enum class Op { N, T };

// acc += alpha * opA(A) * opB(B) over K (multiple of KC), 64x64 output.
//   opA = N: A(i,k) = A[i*lda + k]  ;  opA = T: A(i,k) = A[k*lda + i]
//   opB = T: B(k,j) = B[j*ldb + k]  ;  opB = N: B(k,j) = B[k*ldb + j]
// Ends with a barrier, so the caller may overwrite A or B afterwards.
template <Op OA, Op OB>
__device__ __forceinline__ void gemm(Acc& acc, const double* A, int lda, const double* B, int ldb, int K,
                                     double alpha, double* lds) {
  double* sA = lds;
  double* sB = lds + KC * SLD;
  const int w = wave_id(), l = lane_id();
  const int ia = 32 * (w >> 1) + (l & 15);
  const int jb = 32 * (w & 1) + (l & 15);
  const int kr = l >> 4;
  for (int k0 = 0; k0 < K; k0 += KC) {
    if (OA == Op::N) load_rows(sA, A, lda, k0); else load_cols(sA, A, lda, k0);
    if (OB == Op::T) load_rows(sB, B, ldb, k0); else load_cols(sB, B, ldb, k0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double* ra = sA + (kk + kr) * SLD;
      const double* rb = sB + (kk + kr) * SLD;
      double a0 = alpha * ra[ia], a1 = alpha * ra[ia + 16];
      double b0 = rb[jb], b1 = rb[jb + 16];
      acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
      acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
      acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
      acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// factorisation of one 64x64 tile in LDS (pitch PLD)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void acc_to_lds(const Acc& a, double* s) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) s[acc_row(bi, v) * PLD + acc_col(bj)] = a.c[bi][bj][v];
}

__device__ __forceinline__ void tile_to_lds(const double* C, int ldc, double* s) {
  for (int e = threadIdx.x; e < TT; e += NT) {
    int i = e >> 6, j = e & 63;
    s[i * PLD + j] = C[(int64_t)i * ldc + j];
  }
}

// In-place lower Cholesky of the symmetric tile in s (lower triangle read).
// Returns (uniformly) false if a pivot is not positive; the factor then
// carries NaN.  Upper triangle is zeroed.
__device__ inline bool potrf_lds(double* s) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < T; ++j) {
    if (threadIdx.x == 0) {
      double p = s[j * PLD + j];
      if (!(p > 0.0)) { bad = 1; p = __builtin_nan(""); }
      s[j * PLD + j] = sqrt(p);
    }
    __syncthreads();
    const double inv = 1.0 / s[j * PLD + j];
    for (int i = j + 1 + threadIdx.x; i < T; i += NT) s[i * PLD + j] *= inv;
    __syncthreads();
    const int m = T - 1 - j;
    for (int e = threadIdx.x; e < m * m; e += NT) {
      int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) s[i * PLD + k] -= s[i * PLD + j] * s[k * PLD + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < TT; e += NT) {
    int i = e >> 6, k = e & 63;
    if (k > i) s[i * PLD + k] = 0.0;
  }
  __syncthreads();
  return bad == 0;
}

// sum of log of the diagonal of the tile in s over rows [0, nv)
__device__ inline double logdiag_lds(const double* s, int nv, double* red) {
  double x = 0.0;
  if (threadIdx.x < T && threadIdx.x < nv) x = log(s[threadIdx.x * PLD + threadIdx.x]);
  // wave 0 reduction
  if (threadIdx.x < 64) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (threadIdx.x == 0) *red = x;
  }
  __syncthreads();
  double r = *red;
  __syncthreads();
  return r;
}

// Linv (global, ld T) = inverse of the lower-triangular tile in s.
// Column j of the inverse solves L x = e_j by forward substitution.
__device__ inline void trtri_lds_to_global(const double* s, double* Linv) {
  const int j = threadIdx.x;
  if (j < T) {
    for (int i = 0; i < j; ++i) Linv[i * T + j] = 0.0;
    double xj = 1.0 / s[j * PLD + j];
    Linv[j * T + j] = xj;
    // x kept in registers would need 64 of them; stream through global/L1
    for (int i = j + 1; i < T; ++i) {
      double acc = 0.0;
      for (int k = j; k < i; ++k) acc += s[i * PLD + k] * Linv[k * T + j];
      Linv[i * T + j] = -acc / s[i * PLD + i];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void lds_to_global(const double* s, double* C) {
  for (int e = threadIdx.x; e < TT; e += NT) {
    int i = e >> 6, j = e & 63;
    C[i * T + j] = s[i * PLD + j];
  }
}

// block-wide sum (result valid in every thread)
__device__ inline double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (lane_id() == 0) red[wave_id()] = x;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

}  // namespace mra
