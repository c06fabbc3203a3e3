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
constexpr int LDS_DOUBLES = 4 * KC * SLD;   // two stages of A and B chunks
constexpr int LDS_SWEEP = LDS_DOUBLES + 2 * KC * SLD;   // plus two B-only stages (gemm_lds_a)
static_assert(LDS_DOUBLES >= T * PLD, "the LDS buffer also holds one factorisation tile");

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

enum class Op { N, T };

// ---------------------------------------------------------------------------
// multi-segment GEMM: acc += sum_s alpha_s * opA_s(A_s) * opB_s(B_s), each
// segment a 64x64xK_s product (K_s = 16 * nch_s, nch_s in 1..4).  The
// prefetch pipeline of gemm() runs across segment boundaries, so a chain of
// short products pays the global-memory latency once.  16-row (16-column)
// blocks of the output at or beyond `mrows` (`ncols`) are not multiplied:
// their operand rows (columns) are padding, and the accumulator keeps its
// value there.
// ---------------------------------------------------------------------------
struct Seg {
  const double* A;
  const double* B;
  int lda, ldb;
  bool ak;      // A(i,k) = A[k*lda + i] (k-major) instead of A[i*lda + k]
  bool bk;      // B(k,j) = B[k*ldb + j] (k-major) instead of B[j*ldb + k]
  int nch;      // k-chunks of KC
  double alpha;
};

__device__ __forceinline__ d4 fetch_rt(const double* p, int ld, int k0, bool kmajor) {
  const int t = threadIdx.x;
  if (!kmajor) return *(const d4*)(p + (int64_t)(t >> 2) * ld + k0 + (t & 3) * 4);
  return *(const d4*)(p + (int64_t)(k0 + (t >> 4)) * ld + (t & 15) * 4);
}
__device__ __forceinline__ void stash_rt(double* s, d4 v, bool kmajor) {
  const int t = threadIdx.x;
  if (!kmajor) {
    const int i = t >> 2, kq = (t & 3) * 4;
    s[(kq + 0) * SLD + i] = v[0];
    s[(kq + 1) * SLD + i] = v[1];
    s[(kq + 2) * SLD + i] = v[2];
    s[(kq + 3) * SLD + i] = v[3];
  } else {
    *(d4*)(s + (t >> 4) * SLD + (t & 15) * 4) = v;
  }
}

template <class F>
__device__ __forceinline__ void gemm_segs(Acc& acc, int nseg, F getseg, double* lds, int mrows = T, int ncols = T) {
  if (nseg <= 0) return;
  const int w = wave_id(), l = lane_id();
  const int ia = 32 * (w >> 1) + (l & 15);
  const int jb = 32 * (w & 1) + (l & 15);
  const int kr = l >> 4;
  const bool row0 = 32 * (w >> 1) < mrows, row1 = 32 * (w >> 1) + 16 < mrows;
  const bool col0 = 32 * (w & 1) < ncols, col1 = 32 * (w & 1) + 16 < ncols;
  int s = 0, cs = 0;
  Seg cur = getseg(0);
  d4 va = fetch_rt(cur.A, cur.lda, 0, cur.ak);
  d4 vb = fetch_rt(cur.B, cur.ldb, 0, cur.bk);
  stash_rt(lds, va, cur.ak);
  stash_rt(lds + KC * SLD, vb, cur.bk);
  __syncthreads();
  double alpha_c = cur.alpha;
  int stage = 0;
  for (;;) {
    // advance the prefetch position to the next chunk
    bool more = true;
    if (cs + 1 < cur.nch) {
      ++cs;
    } else if (s + 1 < nseg) {
      ++s;
      cs = 0;
      cur = getseg(s);
    } else {
      more = false;
    }
    if (more) {
      va = fetch_rt(cur.A, cur.lda, cs * KC, cur.ak);
      vb = fetch_rt(cur.B, cur.ldb, cs * KC, cur.bk);
    }
    const double* sA = lds + stage * 2 * KC * SLD;
    const double* sB = sA + KC * SLD;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double* ra = sA + (kk + kr) * SLD;
      const double* rb = sB + (kk + kr) * SLD;
      const double b0 = rb[jb], b1 = rb[jb + 16];
      if (row0) {
        const double a0 = alpha_c * ra[ia];
        if (col0) acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
        if (col1) acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
      }
      if (row1) {
        const double a1 = alpha_c * ra[ia + 16];
        if (col0) acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
        if (col1) acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
      }
    }
    if (!more) {
      __syncthreads();
      return;
    }
    stage ^= 1;
    double* nA = lds + stage * 2 * KC * SLD;
    stash_rt(nA, va, cur.ak);
    stash_rt(nA + KC * SLD, vb, cur.bk);
    __syncthreads();
    alpha_c = cur.alpha;
  }
}

// As gemm_segs, with two chunks in flight: the loads of chunk i + 2 are
// issued while chunk i is multiplied, so each load has two chunk times to
// arrive.  Costs one more register set (16 VGPRs); meant for kernels with
// register headroom.
template <class F>
__device__ __forceinline__ void gemm_segs2(Acc& acc, int nseg, F getseg, double* lds, int mrows = T, int ncols = T) {
  if (nseg <= 0) return;
  const int w = wave_id(), l = lane_id();
  const int ia = 32 * (w >> 1) + (l & 15);
  const int jb = 32 * (w & 1) + (l & 15);
  const int kr = l >> 4;
  const bool row0 = 32 * (w >> 1) < mrows, row1 = 32 * (w >> 1) + 16 < mrows;
  const bool col0 = 32 * (w & 1) < ncols, col1 = 32 * (w & 1) + 16 < ncols;
  int s = 0, cs = 0;
  Seg cur = getseg(0);
  auto advance = [&]() -> bool {
    if (cs + 1 < cur.nch) {
      ++cs;
      return true;
    }
    if (s + 1 < nseg) {
      ++s;
      cs = 0;
      cur = getseg(s);
      return true;
    }
    return false;
  };
  auto compute = [&](const double* sA, double alpha_c) {
    const double* sB = sA + KC * SLD;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double* ra = sA + (kk + kr) * SLD;
      const double* rb = sB + (kk + kr) * SLD;
      const double b0 = rb[jb], b1 = rb[jb + 16];
      if (row0) {
        const double a0 = alpha_c * ra[ia];
        if (col0) acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
        if (col1) acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
      }
      if (row1) {
        const double a1 = alpha_c * ra[ia + 16];
        if (col0) acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
        if (col1) acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
      }
    }
  };
  // chunk 0 staged; chunks 1 and 2 in flight in register sets X and Y
  {
    const d4 va = fetch_rt(cur.A, cur.lda, 0, cur.ak);
    const d4 vb = fetch_rt(cur.B, cur.ldb, 0, cur.bk);
    stash_rt(lds, va, cur.ak);
    stash_rt(lds + KC * SLD, vb, cur.bk);
  }
  double alpha_c = cur.alpha;
  d4 xa = {0.0, 0.0, 0.0, 0.0}, xb = xa, ya = xa, yb = xa;
  bool hx = advance(), hy = false;
  bool fxa = cur.ak, fxb = cur.bk, fya = false, fyb = false;
  double ax = cur.alpha, ay = 0.0;
  if (hx) {
    xa = fetch_rt(cur.A, cur.lda, cs * KC, cur.ak);
    xb = fetch_rt(cur.B, cur.ldb, cs * KC, cur.bk);
    hy = advance();
    if (hy) {
      fya = cur.ak, fyb = cur.bk, ay = cur.alpha;
      ya = fetch_rt(cur.A, cur.lda, cs * KC, cur.ak);
      yb = fetch_rt(cur.B, cur.ldb, cs * KC, cur.bk);
    }
  }
  __syncthreads();
  int stage = 0;
  for (;;) {
    compute(lds + stage * 2 * KC * SLD, alpha_c);
    if (!hx) break;
    stage ^= 1;
    stash_rt(lds + stage * 2 * KC * SLD, xa, fxa);
    stash_rt(lds + stage * 2 * KC * SLD + KC * SLD, xb, fxb);
    alpha_c = ax;
    hx = hy && advance();
    if (hx) {
      fxa = cur.ak, fxb = cur.bk, ax = cur.alpha;
      xa = fetch_rt(cur.A, cur.lda, cs * KC, cur.ak);
      xb = fetch_rt(cur.B, cur.ldb, cs * KC, cur.bk);
    }
    __syncthreads();
    compute(lds + stage * 2 * KC * SLD, alpha_c);
    if (!hy) break;
    stage ^= 1;
    stash_rt(lds + stage * 2 * KC * SLD, ya, fya);
    stash_rt(lds + stage * 2 * KC * SLD + KC * SLD, yb, fyb);
    alpha_c = ay;
    hy = hx && advance();
    if (hy) {
      fya = cur.ak, fyb = cur.bk, ay = cur.alpha;
      ya = fetch_rt(cur.A, cur.lda, cs * KC, cur.ak);
      yb = fetch_rt(cur.B, cur.ldb, cs * KC, cur.bk);
    }
    __syncthreads();
  }
  __syncthreads();
}

// acc += alpha * A * B for one 64x64x64 product whose A operand is already
// in LDS (row-major, pitch PLD, as acc_to_lds leaves it) and whose B operand
// is in global memory, k-major (B(k, j) = B[k * ldb + j]) when bk, else
// B(k, j) = B[j * ldb + k]; only B streams, through `stage` (2 * KC * SLD
// doubles, disjoint from A).  Output row blocks at or beyond mrows are not
// multiplied.
__device__ __forceinline__ void gemm_lds_a(Acc& acc, const double* A, const double* B, int ldb, bool bk,
                                           double alpha, double* stage, int mrows = T) {
  const int w = wave_id(), l = lane_id();
  const int ia = 32 * (w >> 1) + (l & 15);
  const int jb = 32 * (w & 1) + (l & 15);
  const int kr = l >> 4;
  const bool row0 = 32 * (w >> 1) < mrows, row1 = 32 * (w >> 1) + 16 < mrows;
  d4 vb = fetch_rt(B, ldb, 0, bk);
  stash_rt(stage, vb, bk);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < T / KC; ++c) {
    const bool more = c + 1 < T / KC;
    if (more) vb = fetch_rt(B, ldb, (c + 1) * KC, bk);
    const double* sB = stage + (c & 1) * KC * SLD;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int k = c * KC + kk + kr;
      const double* rb = sB + (kk + kr) * SLD;
      const double b0 = rb[jb], b1 = rb[jb + 16];
      if (row0) {
        const double a0 = alpha * A[ia * PLD + k];
        acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
        acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
      }
      if (row1) {
        const double a1 = alpha * A[(ia + 16) * PLD + k];
        acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
        acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
      }
    }
    if (more) stash_rt(stage + ((c + 1) & 1) * KC * SLD, vb, bk);
    __syncthreads();
  }
}

// acc += alpha * A * B for one 64x64x64 product whose B operand is already
// in LDS (B(k, j) at Bs[k * PLD + j], as acc_to_lds leaves a tile) and whose
// A operand is in global memory (A(i, k) = A[k * lda + i] when ak, else
// A[i * lda + k]); only A streams, through `stage` (2 * KC * SLD doubles,
// disjoint from Bs).  Output blocks at or beyond mrows / ncols are not
// multiplied.  The products are issued in the order gemm_segs uses for a
// single segment, so the result is the same to the bit.
__device__ __forceinline__ void gemm_lds_b(Acc& acc, const double* A, int lda, bool ak, const double* Bs,
                                           double alpha, double* stage, int mrows = T, int ncols = T) {
  const int w = wave_id(), l = lane_id();
  const int ia = 32 * (w >> 1) + (l & 15);
  const int jb = 32 * (w & 1) + (l & 15);
  const int kr = l >> 4;
  const bool row0 = 32 * (w >> 1) < mrows, row1 = 32 * (w >> 1) + 16 < mrows;
  const bool col0 = 32 * (w & 1) < ncols, col1 = 32 * (w & 1) + 16 < ncols;
  d4 va = fetch_rt(A, lda, 0, ak);
  stash_rt(stage, va, ak);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < T / KC; ++c) {
    const bool more = c + 1 < T / KC;
    if (more) va = fetch_rt(A, lda, (c + 1) * KC, ak);
    const double* sA = stage + (c & 1) * KC * SLD;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int k = c * KC + kk + kr;
      const double* ra = sA + (kk + kr) * SLD;
      const double b0 = Bs[k * PLD + jb], b1 = Bs[k * PLD + jb + 16];
      if (row0) {
        const double a0 = alpha * ra[ia];
        if (col0) acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.c[0][0], 0, 0, 0);
        if (col1) acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.c[0][1], 0, 0, 0);
      }
      if (row1) {
        const double a1 = alpha * ra[ia + 16];
        if (col0) acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.c[1][0], 0, 0, 0);
        if (col1) acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.c[1][1], 0, 0, 0);
      }
    }
    if (more) stash_rt(stage + ((c + 1) & 1) * KC * SLD, va, ak);
    __syncthreads();
  }
}

// Seg for one 64x64x64 block product in the gemm<> operand conventions
template <Op OA, Op OB>
__device__ __forceinline__ Seg seg(const double* A, int lda, const double* B, int ldb, double alpha, int nch = T / KC) {
  return Seg{A, B, lda, ldb, OA == Op::T, OB == Op::N, nch, alpha};
}

// acc += alpha * opA(A) * opB(B) over K (multiple of KC), 64x64 output:
//   opA = N: A(i,k) = A[i*lda + k]  ;  opA = T: A(i,k) = A[k*lda + i]
//   opB = T: B(k,j) = B[j*ldb + k]  ;  opB = N: B(k,j) = B[k*ldb + j]
// One segment of gemm_segs2 (two k-chunks in flight).  Ends with a barrier,
// so the caller may overwrite A or B afterwards.
template <Op OA, Op OB>
__device__ __forceinline__ void gemm(Acc& acc, const double* A, int lda, const double* B, int ldb, int K,
                                     double alpha, double* lds) {
  gemm_segs2(acc, 1, [&](int) { return seg<OA, OB>(A, lda, B, ldb, alpha, K / KC); }, lds);
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

// all 16 loads of a thread are issued before the first LDS store
__device__ __forceinline__ void tile_to_lds(const double* C, int ldc, double* s) {
  double v[TT / NT];
#pragma unroll
  for (int q = 0; q < TT / NT; ++q) {
    const int e = threadIdx.x + q * NT;
    v[q] = C[(int64_t)(e >> 6) * ldc + (e & 63)];
  }
#pragma unroll
  for (int q = 0; q < TT / NT; ++q) {
    const int e = threadIdx.x + q * NT;
    s[(e >> 6) * PLD + (e & 63)] = v[q];
  }
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// In-place lower Cholesky of the symmetric tile in s (lower triangle read),
// left-looking, by wave 0: lane i owns row i of s; column j is
// a_ij - sum_{k<j} L_ik L_jk (row j read as an LDS broadcast), the pivot
// comes from lane j by readlane.  A wave's LDS accesses complete in order,
// so column j is visible to every lane in the next step.  Returns
// (uniformly) false if a pivot is not positive; the factor then carries NaN.
// The upper triangle is zeroed.
__device__ inline bool potrf_lds(double* s) {
  __shared__ int bad;
  if (threadIdx.x < T) {
    const int i = threadIdx.x;
    double* ri = s + i * PLD;
    int ok = 1;
    for (int j = 0; j < T; ++j) {
      const double* rj = s + j * PLD;
      double a0 = ri[j], a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = 0;
      for (; k + 3 < j; k += 4) {
        a0 = fma(-ri[k], rj[k], a0);
        a1 = fma(-ri[k + 1], rj[k + 1], a1);
        a2 = fma(-ri[k + 2], rj[k + 2], a2);
        a3 = fma(-ri[k + 3], rj[k + 3], a3);
      }
      for (; k < j; ++k) a0 = fma(-ri[k], rj[k], a0);
      const double a = (a0 + a1) + (a2 + a3);
      const double p = readlane_d(a, j);
      ok &= (p > 0.0) ? 1 : 0;
      const double d = (p > 0.0) ? sqrt(p) : __builtin_nan("");
      const double inv = 1.0 / d;
      ri[j] = (i > j) ? a * inv : (i == j ? d : 0.0);
      __builtin_amdgcn_wave_barrier();
    }
    if (i == 0) bad = !ok;
  }
  __syncthreads();
  return bad == 0;
}

// ---------------------------------------------------------------------------
// 16x16 block helpers for one wave (MFMA 16x16x4 layout as above)
// ---------------------------------------------------------------------------

// acc += alpha * A B^T, A and B 16 x K row-major (pitches lda, ldb)
__device__ __forceinline__ void mfma_abt(d4& acc, const double* A, int lda, const double* B, int ldb, int K,
                                         double alpha) {
  const int l = lane_id();
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double a = alpha * A[(l & 15) * lda + k0 + (l >> 4)];
    const double b = B[(l & 15) * ldb + k0 + (l >> 4)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
}
// acc += alpha * A B, A 16 x K, B K x 16, row-major
__device__ __forceinline__ void mfma_ab(d4& acc, const double* A, int lda, const double* B, int ldb, int K,
                                        double alpha) {
  const int l = lane_id();
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double a = alpha * A[(l & 15) * lda + k0 + (l >> 4)];
    const double b = B[(k0 + (l >> 4)) * ldb + (l & 15)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
}
__device__ __forceinline__ void blk_store(const d4& acc, double* C, int ldc) {
  const int l = lane_id();
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * v + (l >> 4)) * ldc + (l & 15)] = acc[v];
}
__device__ __forceinline__ void blk_load(d4& acc, const double* C, int ldc) {
  const int l = lane_id();
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = C[(4 * v + (l >> 4)) * ldc + (l & 15)];
}

// 1/sqrt(p) to full FP64 precision: the hardware estimate refined by two
// Newton steps y <- y (3 - p y^2) / 2
__device__ __forceinline__ double rsqrt_d(double p) {
  double y = __builtin_amdgcn_rsq(p);
  y = y * fma(-0.5 * p, y * y, 1.5);
  y = y * fma(-0.5 * p, y * y, 1.5);
  return y;
}

// Lower Cholesky of the 16x16 block D (pitch PLD) and the inverse of the
// factor in one right-looking sweep by one wave: lane 16 q + i keeps columns
// 4q..4q+3 of row i of the working block (a) and of the inverse (x) in
// registers.  Step j takes the pivot a_jj by readlane, forms column j of the
// factor, broadcasts it and row j of the inverse through LDS (a wave's LDS
// accesses complete in order; lanes that own nothing write to slots of their
// own), then updates the trailing columns (a_ik -= L_ij L_kj, k > j) and the
// inverse rows below j (x_i -= L_ij x_j, the forward substitution of
// L X = I).  The next pivot, a_{j+1,j+1} - L_{j+1,j}^2, is formed right after
// column j, before the broadcast.  No branches: a pivot that is not positive
// makes the reciprocal square root NaN, and the NaN spreads.  On return D
// holds L (zero above the diagonal) and X (pitch ldx) holds L^{-1}.  Returns
// 0 if a pivot was not positive.
__device__ __forceinline__ int potrf_trtri16(double* D, double* X, int ldx) {
  __shared__ double colb[16 + 64], xrow[16 + 4 * 64];
  const int l = lane_id(), i = l & 15, q = l >> 4;
  double a[4], x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    a[c] = D[i * PLD + 4 * q + c];
    x[c] = (i == 4 * q + c) ? 1.0 : 0.0;
  }
  int ok = 1;
  double p = readlane_d(a[0], 0);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int jq = j >> 2, jc = j & 3;
    ok &= (p > 0.0) ? 1 : 0;
    const double y = rsqrt_d(p);   // NaN unless p > 0
    const double lv = (i > j) ? a[jc] * y : (i == j ? p * y : 0.0);   // L_ij in the lanes of quarter jq
    double pn = 0.0;
    if (j < 15) {                  // the next pivot, with the same fma as the update below
      const int j1 = j + 1;
      if ((j1 >> 2) == jq) {
        pn = readlane_d(fma(-lv, lv, a[j1 & 3]), 16 * jq + j1);
      } else {
        const double lx = readlane_d(lv, 16 * jq + j1);
        pn = readlane_d(fma(-lx, lx, a[0]), 16 * (j1 >> 2) + j1);
      }
    }
    a[jc] = (q == jq) ? lv : a[jc];
    colb[q == jq ? i : 16 + l] = lv;
    // row j of the inverse is final once scaled by 1 / L_jj
    const double sj = (i == j) ? y : 1.0;
    double* xw = xrow + (i == j ? 4 * q : 16 + 4 * l);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[c] *= sj;
      xw[c] = x[c];
    }
    __builtin_amdgcn_wave_barrier();
    const double lb = (i > j) ? colb[i] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double lbc = (4 * q + c > j) ? lb : 0.0;
      a[c] = fma(-lbc, colb[4 * q + c], a[c]);
      x[c] = fma(-lb, xrow[4 * q + c], x[c]);
    }
    __builtin_amdgcn_wave_barrier();
    p = pn;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    D[i * PLD + 4 * q + c] = (4 * q + c <= i) ? a[c] : 0.0;
    X[i * ldx + 4 * q + c] = x[c];
  }
  return ok;
}

// Blocked lower Cholesky of the symmetric 64x64 tile in s (lower triangle
// read; 4x4 blocks of 16) and the inverse of the factor, built in the LDS
// tile sx (pitch PLD) and written to Linv (global, ld T) at the end.
// Diagonal blocks are factored and inverted by wave 0; panel and trailing
// updates and the off-diagonal blocks of the inverse
//   X_ii = L_ii^{-1},  X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj  (i > j)
// run on MFMA across the four waves.  Block row i of the inverse needs only
// the factor's columns left of i and the rows of the inverse above it, so
// rows 1 and 2 are formed by waves 1 and 2 while wave 0 factors the next
// diagonal block, and row 3 at the end.  On return s holds L (upper part
// zero).  Returns false (uniformly) if a pivot was not positive; the factor
// and the inverse then carry NaN.
__device__ inline bool potrf_trtri(double* s, double* sx, double* Linv) {
  __shared__ int ok_all;
  __shared__ double tsc[4][16 * 16];   // per-wave partial sum of an inverse block
  const int w = wave_id();
  // X_ij (i > j) for block row ib by the calling wave
  auto inv_block = [&](int ib, int jb) {
    d4 t = {0.0, 0.0, 0.0, 0.0};             // t = sum_{k=j}^{i-1} L_ik X_kj
    for (int kb = jb; kb < ib; ++kb)
      mfma_ab(t, s + 16 * ib * PLD + 16 * kb, PLD, sx + 16 * kb * PLD + 16 * jb, PLD, 16, 1.0);
    blk_store(t, tsc[w], 16);                // one wave: its LDS accesses complete in order
    __builtin_amdgcn_wave_barrier();
    d4 x = {0.0, 0.0, 0.0, 0.0};             // X_ij = -X_ii t
    mfma_ab(x, sx + 16 * ib * PLD + 16 * ib, PLD, tsc[w], 16, 16, -1.0);
    blk_store(x, sx + 16 * ib * PLD + 16 * jb, PLD);
  };
  if (threadIdx.x == 0) ok_all = 1;
  for (int kb = 0; kb < 4; ++kb) {
    double* Dk = s + 16 * kb * PLD + 16 * kb;
    double* Xk = sx + 16 * kb * PLD + 16 * kb;
    if (w == 0) {
      const int ok = potrf_trtri16(Dk, Xk, PLD);
      if (lane_id() == 0 && !ok) ok_all = 0;
    } else if (w < kb) {                       // inverse row kb - 1, block w - 1
      inv_block(kb - 1, w - 1);
    }
    __syncthreads();
    const int ib = kb + 1 + w;                 // panel: L_ik = A_ik X_kk^T
    if (ib < 4) {
      double* Aik = s + 16 * ib * PLD + 16 * kb;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      mfma_abt(acc, Aik, PLD, Xk, PLD, 16, 1.0);
      blk_store(acc, Aik, PLD);
    }
    __syncthreads();
    int idx = 0;                               // trailing: A_ij -= L_ik L_jk^T, kb < j <= i
    for (int i2 = kb + 1; i2 < 4; ++i2)
      for (int j2 = kb + 1; j2 <= i2; ++j2, ++idx)
        if ((idx & 3) == w) {
          double* Aij = s + 16 * i2 * PLD + 16 * j2;
          d4 acc;
          blk_load(acc, Aij, PLD);
          mfma_abt(acc, s + 16 * i2 * PLD + 16 * kb, PLD, s + 16 * j2 * PLD + 16 * kb, PLD, 16, -1.0);
          blk_store(acc, Aij, PLD);
        }
    if (kb < 3) __syncthreads();
  }
  if (w < 3) inv_block(3, w);                  // inverse row 3
  // zero the strictly upper blocks of L and of the inverse (callers use both
  // LDS tiles whole)
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int i = e >> 6, j = e & 63;
    if ((j >> 4) > (i >> 4)) {
      s[i * PLD + j] = 0.0;
      sx[i * PLD + j] = 0.0;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TT; e += NT) Linv[e] = sx[(e >> 6) * PLD + (e & 63)];
  __syncthreads();
  return ok_all != 0;
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

// Linv (global, ld T) = inverse of the lower-triangular tile in s, by wave 0:
// lane j solves L x = e_j by forward substitution; every lane reads the
// same L entries (LDS broadcast) and keeps its column x in the free upper
// triangle of its own row of s (x_i at s[j][i], i > j; 1/L_jj apart).
// Overwrites the upper triangle of s.
__device__ inline void trtri_lds_to_global(double* s, double* Linv) {
  __shared__ double dg[T];
  if (threadIdx.x < T) dg[threadIdx.x] = 1.0 / s[threadIdx.x * PLD + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < T) {
    const int j = threadIdx.x;
    double* xr = s + j * PLD;
    const double xj = dg[j];
    for (int i = 1; i < T; ++i) {
      const double* Li = s + i * PLD;
      double a0 = 0.0, a1 = 0.0;
      int k = 0;
      for (; k + 1 < i; k += 2) {
        const double x0 = (k > j) ? xr[k] : (k == j ? xj : 0.0);
        const double x1 = (k + 1 > j) ? xr[k + 1] : (k + 1 == j ? xj : 0.0);
        a0 = fma(Li[k], x0, a0);
        a1 = fma(Li[k + 1], x1, a1);
      }
      if (k < i) a0 = fma(Li[k], (k > j) ? xr[k] : (k == j ? xj : 0.0), a0);
      if (i > j) xr[i] = -(a0 + a1) * dg[i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TT; e += NT) {
    const int i = e >> 6, jj = e & 63;
    Linv[e] = (i > jj) ? s[jj * PLD + i] : (i == jj ? dg[i] : 0.0);
  }
  __syncthreads();
}

__device__ __forceinline__ void lds_to_global(const double* s, double* C) {
  for (int e = threadIdx.x; e < TT; e += NT) {
    int i = e >> 6, j = e & 63;
    C[i * T + j] = s[i * PLD + j];
  }
}

// sum over the 4 lanes t, t^1, t^2, t^3 (valid in each of them)
__device__ __forceinline__ double quad_sum(double x) {
  x += __shfl_xor(x, 1);
  x += __shfl_xor(x, 2);
  return x;
}

// column sums over the four waves: thread t holds a partial for column
// t & 63; returns the total in threads 0..63 (others get 0)
__device__ inline double wave_col_sum(double x, double* red4x64) {
  red4x64[threadIdx.x] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < T) s = red4x64[threadIdx.x] + red4x64[T + threadIdx.x] + red4x64[2 * T + threadIdx.x] +
                           red4x64[3 * T + threadIdx.x];
  __syncthreads();
  return s;
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
