// Throughput of the FP64 MFMA tile engine on its own (a measurement tool,
// not part of the library).  Every workgroup computes one output tile as a
// sum of nseg products with K = 64: A_s streams from HBM (row-major as the
// leaf planes, or k-major), B_s comes from a pool of 36 tiles that stays in
// L2 (as the ancestors' tiles do).  With reuse G, G consecutive workgroups
// share their A tiles (as the planes of one row tile share V).
//
//   "library 64x64": the engine the kernels use (tile.hpp, gemm_segs2: one
//                     64x64 tile per workgroup, two k-chunks in flight);
//   "A row-major/k-major BMxBN": the same LDS-staged k-chunk pipeline with one
//                     chunk in flight, for output tiles of 64x64, 64x128,
//                     128x64 and 128x128 (waves in 2x2, each owning a
//                     BM/2 x BN/2 block);
//   "B transposed t/36": the library engine with t in 36 of the products
//                     reading B transposed (row-major staging);
//   "MFMA peak":      v_mfma_f64_16x16x4f64 from registers only, four
//                     independent accumulators per wave, 8 workgroups per CU;
//   "factorisation":  one 64x64 Cholesky + inverse (potrf_trtri) in one
//                     workgroup, timed in the kernel over 100 calls.
//
// Prints one line per variant: time per launch (HIP events over 10
// launches after one warm-up) and FP64 TFLOP/s.  Buffers: 2 GiB of A,
// 256 MiB of outputs, all operands nonzero; every index stays inside them
// (checked before each launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tile.hpp"

using mra::d4;
using mra::KC;
using mra::NT;

#define CK(x)                                                                    \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

namespace {

constexpr int POOL = 36;
constexpr size_t CAP_A = (size_t)1 << 28;   // doubles
constexpr size_t CAP_C = (size_t)1 << 25;
constexpr size_t CAP_B = (size_t)64 * 64 * 64 * 2;

template <int BM, int BN>
struct Shape {
  static constexpr int SA = BM + 4, SB = BN + 4;
  static constexpr int STAGE = KC * (SA + SB);
  static constexpr int FA = BM * KC / NT / 4;   // d4 loads per thread for A
  static constexpr int FB = BN * KC / NT / 4;
  static constexpr int MB = BM / 32, NB = BN / 32;   // 16x16 blocks per wave
};

template <int BM, int BN, bool AK>
__global__ __launch_bounds__(NT, 2) void k_tiles(const double* A, const double* B, double* C, int nseg, int G) {
  using E = Shape<BM, BN>;
  __shared__ __attribute__((aligned(32))) double lds[2 * E::STAGE];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int kr = l >> 4;
  const int64_t wg = blockIdx.x;
  d4 acc[E::MB][E::NB];
#pragma unroll
  for (int i = 0; i < E::MB; ++i)
#pragma unroll
    for (int j = 0; j < E::NB; ++j) acc[i][j] = d4{0, 0, 0, 0};
  const int nch = nseg * (64 / KC);
  d4 ra[E::FA], rb[E::FB];
  auto fetch = [&](int c) {
    const int s = c / (64 / KC);
    const double* a = A + ((wg / G) * nseg + s) * (int64_t)BM * 64;
    const double* b = B + (int64_t)((wg * 7 + s) % POOL) * 64 * BN;
    const int k0 = (c % (64 / KC)) * KC;
#pragma unroll
    for (int q = 0; q < E::FA; ++q) {
      const int e = t + q * NT;
      if (AK) ra[q] = *(const d4*)(a + (int64_t)(k0 + e / (BM / 4)) * BM + 4 * (e % (BM / 4)));
      else ra[q] = *(const d4*)(a + (int64_t)(e >> 2) * 64 + k0 + (e & 3) * 4);
    }
#pragma unroll
    for (int q = 0; q < E::FB; ++q) {
      const int e = t + q * NT;
      rb[q] = *(const d4*)(b + (int64_t)(k0 + e / (BN / 4)) * BN + 4 * (e % (BN / 4)));
    }
  };
  auto stash = [&](double* s) {
    double* sa = s;
    double* sb = s + KC * E::SA;
#pragma unroll
    for (int q = 0; q < E::FA; ++q) {
      const int e = t + q * NT;
      if (AK) {
        *(d4*)(sa + (e / (BM / 4)) * E::SA + 4 * (e % (BM / 4))) = ra[q];
      } else {
        const int i = e >> 2, kq = (e & 3) * 4;
#pragma unroll
        for (int v = 0; v < 4; ++v) sa[(kq + v) * E::SA + i] = ra[q][v];
      }
    }
#pragma unroll
    for (int q = 0; q < E::FB; ++q) {
      const int e = t + q * NT;
      *(d4*)(sb + (e / (BN / 4)) * E::SB + 4 * (e % (BN / 4))) = rb[q];
    }
  };
  const int i0 = (BM / 2) * (w >> 1) + (l & 15), j0 = (BN / 2) * (w & 1) + (l & 15);
  fetch(0);
  stash(lds);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const bool more = c + 1 < nch;
    if (more) fetch(c + 1);
    const double* sa = lds + (c & 1) * E::STAGE;
    const double* sb = sa + KC * E::SA;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double av[E::MB], bv[E::NB];
#pragma unroll
      for (int i = 0; i < E::MB; ++i) av[i] = sa[(kk + kr) * E::SA + i0 + 16 * i];
#pragma unroll
      for (int j = 0; j < E::NB; ++j) bv[j] = sb[(kk + kr) * E::SB + j0 + 16 * j];
#pragma unroll
      for (int i = 0; i < E::MB; ++i)
#pragma unroll
        for (int j = 0; j < E::NB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(lds + ((c + 1) & 1) * E::STAGE);
    __syncthreads();
  }
  double* out = C + wg * (int64_t)BM * BN;
#pragma unroll
  for (int i = 0; i < E::MB; ++i)
#pragma unroll
    for (int j = 0; j < E::NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(int64_t)((BM / 2) * (w >> 1) + 16 * i + 4 * v + (l >> 4)) * BN + (BN / 2) * (w & 1) + 16 * j +
            (l & 15)] = acc[i][j][v];
}

// bt: the products with (wg + s) % 36 < bt read B transposed
__global__ __launch_bounds__(NT, 4) void k_library(const double* A, const double* B, double* C, int nseg, int G, int bt) {
  __shared__ __attribute__((aligned(32))) double lds[mra::LDS_DOUBLES];
  const int64_t wg = blockIdx.x;
  mra::Acc acc;
  mra::acc_zero(acc);
  mra::gemm_segs2(acc, nseg, [&](int s) {
    const double* a = A + ((wg / G) * nseg + s) * (int64_t)4096;
    const double* b = B + (int64_t)((wg * 7 + s) % POOL) * 4096;
    if ((wg + s) % 36 < bt) return mra::seg<mra::Op::N, mra::Op::T>(a, 64, b, 64, 1.0);
    return mra::seg<mra::Op::N, mra::Op::N>(a, 64, b, 64, 1.0);
  }, lds);
  mra::acc_store(acc, C + wg * 4096, 64);
}

// registers only: out[t] keeps the accumulators live
constexpr int PEAK_ITERS = 2000;
__global__ __launch_bounds__(NT) void k_peak(const double* seed, double* out) {
  const int t = threadIdx.x + blockIdx.x * NT;
  const double a0 = seed[t & 255], a1 = seed[(t + 1) & 255], b0 = seed[(t + 2) & 255], b1 = seed[(t + 3) & 255];
  d4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
  for (int i = 0; i < PEAK_ITERS; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c00, 0, 0, 0);
      c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c01, 0, 0, 0);
      c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c10, 0, 0, 0);
      c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c11, 0, 0, 0);
    }
  }
  const d4 s4 = c00 + c01 + c10 + c11;
  out[t] = s4[0] + s4[1] + s4[2] + s4[3];
}

// 100 factorisations of the SPD tile Asp (64x64) in one workgroup; the
// wall-clock ticks of the last 99 go to ticks[0], the factor and inverse
// of the last call to L and Li
__global__ __launch_bounds__(NT, 2) void k_factor(const double* Asp, double* L, double* Li, long long* ticks) {
  __shared__ __attribute__((aligned(32))) double lds[mra::LDS_DOUBLES];
  __shared__ double lds_x[mra::T * mra::PLD];
  long long t0 = 0;
  for (int r = 0; r < 100; ++r) {
    for (int e = threadIdx.x; e < mra::TT; e += NT) lds[(e >> 6) * mra::PLD + (e & 63)] = Asp[e];
    __syncthreads();
    if (r == 1) t0 = wall_clock64();
    mra::potrf_trtri(lds, lds_x, Li);
    __syncthreads();
  }
  const long long t1 = wall_clock64();
  for (int e = threadIdx.x; e < mra::TT; e += NT) L[e] = lds[(e >> 6) * mra::PLD + (e & 63)];
  if (threadIdx.x == 0) ticks[0] = t1 - t0;
}

template <class L>
void time_it(const char* name, int bm, int bn, int nwg, int nseg, int G, L launch) {
  const size_t need_a = (size_t)((nwg + G - 1) / G) * nseg * bm * 64, need_c = (size_t)nwg * bm * bn;
  if (need_a > CAP_A || need_c > CAP_C || (size_t)POOL * 64 * bn > CAP_B) {
    std::printf("%-24s skipped: buffers too small\n", name);
    return;
  }
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  launch();
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  constexpr int reps = 10;
  CK(hipEventRecord(e0));
  for (int r = 0; r < reps; ++r) launch();
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  const double s = ms / reps * 1e-3;
  std::printf("%-24s %4dx%-4d G %d nwg %6d nseg %3d  %8.1f us  %6.2f TF/s\n", name, bm, bn, G, nwg, nseg, s * 1e6,
              2.0 * bm * bn * 64.0 * nseg * nwg / s / 1e12);
  std::fflush(stdout);
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
}

}  // namespace

int main() {
  double *A, *B, *C;
  CK(hipMalloc(&A, CAP_A * 8));
  CK(hipMalloc(&B, CAP_B * 8));
  CK(hipMalloc(&C, CAP_C * 8));
  // nonzero operands throughout: FP64 MFMA runs measurably faster on zeros
  std::vector<double> h(CAP_B);
  for (size_t i = 0; i < CAP_B; ++i) h[i] = (double)(i % 97) * 1e-3 - 0.05;
  CK(hipMemcpy(B, h.data(), CAP_B * 8, hipMemcpyHostToDevice));
  std::vector<double> ha((size_t)1 << 22);
  for (size_t i = 0; i < ha.size(); ++i) ha[i] = (double)((i * 7919) % 1013) * 1e-3 - 0.5;
  for (size_t off = 0; off < CAP_A; off += ha.size())
    CK(hipMemcpy(A + off, ha.data(), ha.size() * 8, hipMemcpyHostToDevice));
  for (int nseg : {6, 24}) {
    const int f = nseg / 6;
    const int n64 = 8192 / f, n128 = 4096 / f, n256 = 2048 / f;
    time_it("library 64x64", 64, 64, n64, nseg, 1,
            [&] { hipLaunchKernelGGL(k_library, dim3(n64), dim3(NT), 0, 0, A, B, C, nseg, 1, 0); });
    time_it("A row-major", 64, 64, n64, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<64, 64, false>), dim3(n64), dim3(NT), 0, 0, A, B, C, nseg, 1); });
    time_it("A k-major", 64, 64, n64, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<64, 64, true>), dim3(n64), dim3(NT), 0, 0, A, B, C, nseg, 1); });
    time_it("A row-major", 64, 128, n128, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<64, 128, false>), dim3(n128), dim3(NT), 0, 0, A, B, C, nseg, 1); });
    time_it("A row-major", 128, 64, n128, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<128, 64, false>), dim3(n128), dim3(NT), 0, 0, A, B, C, nseg, 1); });
    time_it("A row-major", 128, 128, n256, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<128, 128, false>), dim3(n256), dim3(NT), 0, 0, A, B, C, nseg, 1); });
    time_it("A k-major", 128, 128, n256, nseg, 1,
            [&] { hipLaunchKernelGGL((k_tiles<128, 128, true>), dim3(n256), dim3(NT), 0, 0, A, B, C, nseg, 1); });
  }
  {
    // six output tiles of 64 columns per streamed A tile (G = 6 for 64-wide
    // tiles, 3 for 128-wide ones), six products each
    const int nseg = 6, n64 = 8192, n128 = 4096, n256 = 2048;
    time_it("library 64x64", 64, 64, n64, nseg, 6,
            [&] { hipLaunchKernelGGL(k_library, dim3(n64), dim3(NT), 0, 0, A, B, C, nseg, 6, 0); });
    time_it("A row-major", 64, 128, n128, nseg, 3,
            [&] { hipLaunchKernelGGL((k_tiles<64, 128, false>), dim3(n128), dim3(NT), 0, 0, A, B, C, nseg, 3); });
    time_it("A row-major", 128, 128, n256, nseg, 3,
            [&] { hipLaunchKernelGGL((k_tiles<128, 128, false>), dim3(n256), dim3(NT), 0, 0, A, B, C, nseg, 3); });
    for (int bt : {15, 36})
      time_it(bt == 15 ? "B transposed 15/36" : "B transposed 36/36", 64, 64, n64, nseg, 6,
              [&] { hipLaunchKernelGGL(k_library, dim3(n64), dim3(NT), 0, 0, A, B, C, nseg, 6, bt); });
  }
  {
    // registers only: 2048 workgroups of four waves, 32 products per iteration
    const int nblk = 2048;
    if ((size_t)nblk * NT > CAP_C) return 1;
    hipLaunchKernelGGL(k_peak, dim3(nblk), dim3(NT), 0, 0, B, C);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    CK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k_peak, dim3(nblk), dim3(NT), 0, 0, B, C);
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    const double fl = 5.0 * nblk * 4.0 * PEAK_ITERS * 32.0 * 2048.0;
    std::printf("MFMA peak (registers)    %8.1f us per launch  %6.2f TF/s\n", ms / 5 * 1e3, fl / (ms * 1e-3) / 1e12);
    std::fflush(stdout);
    CK(hipEventDestroy(e0));
    CK(hipEventDestroy(e1));
  }
  {
    // a well-conditioned SPD tile: 64 I + R R' with R uniform in [-0.5, 0.5]
    std::vector<double> r(mra::TT), spd(mra::TT);
    unsigned x = 12345u;
    for (auto& v : r) {
      x = x * 1664525u + 1013904223u;
      v = (double)(x >> 8) / 16777216.0 - 0.5;
    }
    for (int i = 0; i < 64; ++i)
      for (int j = 0; j < 64; ++j) {
        double acc = (i == j) ? 64.0 : 0.0;
        for (int k = 0; k < 64; ++k) acc += r[i * 64 + k] * r[j * 64 + k];
        spd[i * 64 + j] = acc;
      }
    double *dA, *dL, *dLi;
    long long* dt;
    CK(hipMalloc(&dA, mra::TT * 8));
    CK(hipMalloc(&dL, mra::TT * 8));
    CK(hipMalloc(&dLi, mra::TT * 8));
    CK(hipMalloc(&dt, 8));
    CK(hipMemcpy(dA, spd.data(), mra::TT * 8, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_factor, dim3(1), dim3(NT), 0, 0, dA, dL, dLi, dt);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    long long ticks = 0;
    int khz = 0;
    CK(hipMemcpy(&ticks, dt, 8, hipMemcpyDeviceToHost));
    CK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0));
    std::vector<double> hl(mra::TT), hi(mra::TT);
    CK(hipMemcpy(hl.data(), dL, mra::TT * 8, hipMemcpyDeviceToHost));
    CK(hipMemcpy(hi.data(), dLi, mra::TT * 8, hipMemcpyDeviceToHost));
    double e1 = 0.0, e2 = 0.0;
    for (int i = 0; i < 64; ++i)
      for (int j = 0; j < 64; ++j) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 64; ++k) {
          a += hl[i * 64 + k] * hl[j * 64 + k];
          b += hi[i * 64 + k] * hl[k * 64 + j];
        }
        e1 = std::max(e1, std::fabs(a - spd[i * 64 + j]));
        e2 = std::max(e2, std::fabs(b - (i == j ? 1.0 : 0.0)));
      }
    std::printf("factorisation 64x64      %8.2f us per call (max |LL'-A| %.1e, max |L^-1 L - I| %.1e)\n",
                (double)ticks / 99.0 / khz * 1e3, e1, e2);
    std::fflush(stdout);
    CK(hipFree(dA));
    CK(hipFree(dL));
    CK(hipFree(dLi));
    CK(hipFree(dt));
  }
  CK(hipFree(A));
  CK(hipFree(B));
  CK(hipFree(C));
  std::printf("done\n");
  return 0;
}
