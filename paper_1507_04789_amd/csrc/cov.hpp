// Covariance tiles C_0(X, Y) = sigma^2 rho(||x - y|| / kappa) evaluated
// straight into the MFMA accumulator layout.
//   Matern nu = 1.5 (eq. mat15): rho(h) = (1 + sqrt(3) h) exp(-sqrt(3) h)
//   exponential:                 rho(h) = exp(-h)
// d/dlog kappa (h = dist / kappa, dh/dlog kappa = -h):
//   Matern 1.5:  sigma^2 * 3 h^2 exp(-sqrt(3) h);  exponential: sigma^2 * h exp(-h)
// Points are stored as (x, y) pairs; one-dimensional problems use y = 0.
// Entries whose row or column index is at or beyond the valid count are
// padding: the tile is zero there, with 1 on a padded diagonal entry so a
// padded covariance stays block-diagonal with an identity block.
#pragma once
#include "tile.hpp"

namespace mra {

constexpr int COV_EXP = 0;
constexpr int COV_MATERN32 = 1;

struct CovP {
  double s2, kappa, tau2;
  double ikappa;   // 1 / kappa: h = dist * ikappa avoids a division per entry
  int kind;
};

__device__ __forceinline__ CovP load_cov(const double* theta, int kind) {
  CovP c;
  c.s2 = exp(theta[0]);
  c.kappa = exp(theta[1]);
  c.ikappa = exp(-theta[1]);
  c.tau2 = exp(theta[2]);
  c.kind = kind;
  return c;
}

__device__ __forceinline__ double dist2(const double* X, int i, const double* Y, int j) {
  double dx = X[2 * i] - Y[2 * j];
  double dy = X[2 * i + 1] - Y[2 * j + 1];
  return sqrt(dx * dx + dy * dy);
}

__device__ __forceinline__ double cov_val(double dist, const CovP& c) {
  double h = dist * c.ikappa;
  if (c.kind == COV_MATERN32) {
    double a = 1.7320508075688772 * h;
    return c.s2 * ((1.0 + a) * exp(-a));
  }
  return c.s2 * exp(-h);
}

// value and d/dlog kappa
__device__ __forceinline__ void cov_val_dk(double dist, const CovP& c, double& v, double& dk) {
  double h = dist * c.ikappa;
  if (c.kind == COV_MATERN32) {
    double a = 1.7320508075688772 * h;
    double e = exp(-a);
    v = c.s2 * ((1.0 + a) * e);
    dk = c.s2 * (a * a * e);   // 3 h^2 = a^2
  } else {
    double e = exp(-h);
    v = c.s2 * e;
    dk = c.s2 * (h * e);
  }
}

// a = C_0(X[0:64], Y[0:64]) with padding; on a diagonal tile (same point
// set) valid diagonal entries get + dadd and padded ones 1.
__device__ __forceinline__ void acc_cov(Acc& a, const double* X, int nx, const double* Y, int ny, const CovP& c,
                                        bool diag, double dadd) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = acc_row(bi, v), j = acc_col(bj);
        double x = 0.0;
        if (i < nx && j < ny) x = cov_val(dist2(X, i, Y, j), c);
        if (diag && i == j) x += (i < nx) ? dadd : 1.0;
        a.c[bi][bj][v] = x;
      }
}

// Contractions of a cotangent tile G (in the accumulator) with the
// covariance tile and its log-kappa derivative:
//   g[0] += <G, C_0(X, Y)>, g[1] += <G, dC_0/dlog kappa>  (valid entries only),
//   g[2] += sum of G over valid diagonal entries when diag.
__device__ __forceinline__ void acc_cov_contract(const Acc& G, const double* X, int nx, const double* Y, int ny,
                                                 const CovP& c, bool diag, double g[3]) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = acc_row(bi, v), j = acc_col(bj);
        if (i < nx && j < ny) {
          double cv, dk;
          cov_val_dk(dist2(X, i, Y, j), c, cv, dk);
          double gg = G.c[bi][bj][v];
          g[0] += gg * cv;
          g[1] += gg * dk;
          if (diag && i == j) g[2] += gg;
        }
      }
}

}  // namespace mra
