// Host plan builder: recursive partition and knots (Sec. 2.2, 2.5), leaf
// assignment, padded leaf-sorted storage, arena layout and task lists.
//
// Partition rules (fixed so that independent implementations agree bit for
// bit).  Every region of level m - 1 has J_m children.  A split into J is a
// g_x x g_y grid: d = 1: g_x = J; d = 2: J = 1, 2, 4, 8, 16 as 1x1, 2x1, 2x2,
// 4x2, 4x4 with the larger count along the longer side (x on ties).  The box
// is cut along y into g_y slabs, then every slab along x into g_x cells;
// child iy * g_x + ix, iy the number of y split values <= y, ix that of the
// slab's x split values <= x.  Split values of [a, b] into g parts:
// equal-area a + ((b - a) k) / g (2-D two-way splits at 0.5 (a + b)), or,
// adaptive, quantiles of the observations in the region (slab):
// 0.5 (v[i-1] + v[i]) with v sorted and i = (k len(v)) / g, equal parts when
// fewer than g observations.  Default knots: cell-centred g x g grid (d = 2,
// g = sqrt(r_m)), x_i = a + ((b-a)*(2i+1))/(2g), index iy*g + ix; d = 1:
// x_i = a + ((b-a)*(2i+1))/(2 r_m).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "plan.hpp"

namespace mra {
namespace {

struct Box {
  double a[2], b[2];
};

// split of one region into g_x x g_y children: the g_y - 1 y split values,
// then for each slab its g_x - 1 x split values (at most 15 in all: 4 x 4 in
// 2-D, 16 x 1 in 1-D)
struct Split {
  int gx = 1, gy = 1;
  double v[15] = {};
  const double* ys() const { return v; }
  double* ys() { return v; }
  const double* xs(int iy) const { return v + (gy - 1) + iy * (gx - 1); }
  double* xs(int iy) { return v + (gy - 1) + iy * (gx - 1); }
};

bool grid_shape(int d, int J, const Box& box, int& gx, int& gy) {
  if (d == 1) {
    gx = J;
    gy = 1;
    return J >= 1 && J <= 16;
  }
  const bool wide = (box.b[0] - box.a[0]) >= (box.b[1] - box.a[1]);
  switch (J) {
    case 1: gx = gy = 1; return true;
    case 4: gx = gy = 2; return true;
    case 16: gx = gy = 4; return true;
    case 2: gx = wide ? 2 : 1; gy = wide ? 1 : 2; return true;
    case 8: gx = wide ? 4 : 2; gy = wide ? 2 : 4; return true;
    default: return false;
  }
}

// split values of [a, b] into g parts: quantiles of v when it holds at least
// g values (v is sorted here), equal parts otherwise
void split_values(double a, double b, int g, int d, std::vector<double>* v, double* out) {
  if (v && (int64_t)v->size() >= g) {
    std::sort(v->begin(), v->end());
    const int64_t n = (int64_t)v->size();
    for (int k = 1; k < g; ++k) {
      const int64_t i = (k * n) / g;
      out[k - 1] = 0.5 * ((*v)[i - 1] + (*v)[i]);
    }
    return;
  }
  for (int k = 1; k < g; ++k)
    out[k - 1] = (d == 2 && g == 2) ? 0.5 * (a + b) : a + ((b - a) * (double)k) / (double)g;
}

int child_index(const Split& s, const double* x, int d) {
  int iy = 0, ix = 0;
  if (d == 2)
    for (int k = 0; k < s.gy - 1; ++k)
      if (x[1] >= s.ys()[k]) ++iy;
  for (int k = 0; k < s.gx - 1; ++k)
    if (x[0] >= s.xs(iy)[k]) ++ix;
  return iy * s.gx + ix;
}

Box child_box(const Box& p, const Split& s, int j, int d) {
  Box c = p;
  const int iy = j / s.gx, ix = j % s.gx;
  if (d == 2) {
    c.a[1] = iy == 0 ? p.a[1] : s.ys()[iy - 1];
    c.b[1] = iy == s.gy - 1 ? p.b[1] : s.ys()[iy];
  }
  c.a[0] = ix == 0 ? p.a[0] : s.xs(iy)[ix - 1];
  c.b[0] = ix == s.gx - 1 ? p.b[0] : s.xs(iy)[ix];
  return c;
}

bool inside(const double* x, int d, const double* lo, const double* hi) {
  for (int a = 0; a < d; ++a)
    if (!std::isfinite(x[a]) || x[a] < lo[a] || x[a] > hi[a]) return false;
  return true;
}

// leaf index of every point by descending the splits; false if a point is
// outside the box or not finite
bool assign_leaves(const std::vector<std::vector<Split>>& splits, const std::vector<int32_t>& Jl, const double* pts,
                   int64_t n, int d, int M, const double* lo, const double* hi, std::vector<int64_t>& leaf) {
  leaf.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) {
    const double* x = pts + p * d;
    if (!inside(x, d, lo, hi)) return false;
    int64_t i = 0;
    for (int m = 0; m < M; ++m) i = i * Jl[m + 1] + child_index(splits[m][i], x, d);
    leaf[p] = i;
  }
  return true;
}

// stable sort by leaf: perm[k] = original index, off = CSR offsets
void sort_by_leaf(const std::vector<int64_t>& leaf, int64_t n_leaves, std::vector<int64_t>& perm,
                  std::vector<int64_t>& off) {
  off.assign(n_leaves + 1, 0);
  for (int64_t v : leaf) off[v + 1]++;
  for (int64_t i = 0; i < n_leaves; ++i) off[i + 1] += off[i];
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  perm.assign(leaf.size(), 0);
  for (int64_t p = 0; p < (int64_t)leaf.size(); ++p) perm[pos[leaf[p]]++] = p;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

mra_status build_plan(const mra_config* cfg, const double* h_locs, int64_t n, const double* h_pred, int64_t n_pred,
                      const double* h_knots, mra_plan_s* P) {
  if (!cfg || (!h_locs && n > 0) || n < 1 || n_pred < 0 || (n_pred > 0 && !h_pred)) return MRA_EINVAL;
  const int d = cfg->d, M = cfg->M, J = cfg->J, r = cfg->r;
  if (d < 1 || d > 2 || M < 0 || M >= MAXL || cfg->max_theta < 1) return MRA_EINVAL;
  if (cfg->flags & ~(MRA_SYNC | MRA_PLAIN | MRA_GRAPH | MRA_NO_GRAD | MRA_CHECKPOINT | MRA_JOINT)) return MRA_EINVAL;
  if (cfg->chunks < 0 || (cfg->adaptive != 0 && cfg->adaptive != 1)) return MRA_EINVAL;
  if (cfg->cov != MRA_COV_EXPONENTIAL && cfg->cov != MRA_COV_MATERN32) return MRA_EINVAL;
  for (int a = 0; a < d; ++a)
    if (!(cfg->lo[a] < cfg->hi[a]) || !std::isfinite(cfg->lo[a]) || !std::isfinite(cfg->hi[a])) return MRA_EINVAL;
  // children and knots per level
  std::vector<int32_t> Jl(M + 1, 1), rl(std::max(M, 1), r);
  for (int m = 1; m <= M; ++m) Jl[m] = cfg->J_level[m - 1] > 0 ? cfg->J_level[m - 1] : J;
  for (int m = 0; m < M; ++m) rl[m] = cfg->r_level[m] > 0 ? cfg->r_level[m] : r;
  for (int m = 1; m <= M; ++m) {
    if (d == 2 && Jl[m] != 1 && Jl[m] != 2 && Jl[m] != 4 && Jl[m] != 8 && Jl[m] != 16) return MRA_EINVAL;
    if (d == 1 && (Jl[m] < 1 || Jl[m] > 16)) return MRA_EINVAL;
  }
  for (int m = 0; m < M; ++m) {
    if (rl[m] < 1 || rl[m] > T) return MRA_EINVAL;
    if (!h_knots && d == 2) {
      const int g = (int)std::lround(std::sqrt((double)rl[m]));
      if (g * g != rl[m]) return MRA_EINVAL;
    }
  }
  if (M == 0 && (r < 1 || r > T)) return MRA_EINVAL;
  P->cfg = *cfg;
  P->d = d; P->M = M; P->J = J; P->r = r; P->n = n; P->n_pred = n_pred;
  P->Jl = Jl;
  P->rl = rl;
  P->side_solves = M + 2;   // leaf solves forked once the forward recursion is enqueued
  // levels
  P->nreg.assign(M + 1, 1);
  for (int m = 1; m <= M; ++m) P->nreg[m] = P->nreg[m - 1] * Jl[m];
  P->reg_base.assign(M + 1, 0);
  for (int m = 1; m <= M; ++m) P->reg_base[m] = P->reg_base[m - 1] + P->nreg[m - 1];
  const int64_t n_internal = P->reg_base[M];
  const int64_t n_leaves = P->nreg[M];
  if (n_leaves > ((int64_t)1 << 31) - 1) return MRA_EINVAL;
  for (int a = 0; a < d; ++a)
    for (int64_t p = 0; p < n; ++p)
      if (!inside(h_locs + p * d, d, cfg->lo, cfg->hi)) return MRA_EINVAL;
  // boxes and splits, level by level; adaptive splits use the observations
  // of each region (grouped by a counting sort of their current region)
  std::vector<std::vector<Box>> boxes(M + 1);
  std::vector<std::vector<Split>> splits(M);
  Box root;
  for (int a = 0; a < 2; ++a) { root.a[a] = a < d ? cfg->lo[a] : 0.0; root.b[a] = a < d ? cfg->hi[a] : 0.0; }
  boxes[0].push_back(root);
  const bool adaptive = cfg->adaptive == 1;
  std::vector<int64_t> cur(n, 0), start, byreg;
  for (int m = 0; m < M; ++m) {
    const int64_t nr = P->nreg[m];
    const int J1 = Jl[m + 1];
    if (adaptive) {
      start.assign(nr + 1, 0);
      for (int64_t p = 0; p < n; ++p) start[cur[p] + 1]++;
      for (int64_t i = 0; i < nr; ++i) start[i + 1] += start[i];
      byreg.assign(n, 0);
      std::vector<int64_t> pos(start.begin(), start.end() - 1);
      for (int64_t p = 0; p < n; ++p) byreg[pos[cur[p]]++] = p;
    }
    splits[m].resize(nr);
    boxes[m + 1].resize(P->nreg[m + 1]);
    std::vector<double> vy, vx;
    for (int64_t i = 0; i < nr; ++i) {
      const Box& bx = boxes[m][i];
      Split& sp = splits[m][i];
      if (!grid_shape(d, J1, bx, sp.gx, sp.gy)) return MRA_EINVAL;
      const int64_t p0 = adaptive ? start[i] : 0, p1 = adaptive ? start[i + 1] : 0;
      if (d == 2) {
        vy.clear();
        for (int64_t q = p0; q < p1; ++q) vy.push_back(h_locs[byreg[q] * d + 1]);
        split_values(bx.a[1], bx.b[1], sp.gy, d, adaptive ? &vy : nullptr, sp.ys());
      }
      for (int iy = 0; iy < sp.gy; ++iy) {
        vx.clear();
        for (int64_t q = p0; q < p1; ++q) {
          const double* x = h_locs + byreg[q] * d;
          int cy = 0;
          if (d == 2)
            for (int k = 0; k < sp.gy - 1; ++k)
              if (x[1] >= sp.ys()[k]) ++cy;
          if (cy == iy) vx.push_back(x[0]);
        }
        split_values(bx.a[0], bx.b[0], sp.gx, d, adaptive ? &vx : nullptr, sp.xs(iy));
      }
      for (int j = 0; j < J1; ++j) boxes[m + 1][i * J1 + j] = child_box(bx, sp, j, d);
    }
    for (int64_t p = 0; p < n; ++p) cur[p] = cur[p] * J1 + child_index(splits[m][cur[p]], h_locs + p * d, d);
  }
  // knots: r_m x d per region of level m, level-major
  P->knot_off.assign(M + 1, 0);
  for (int m = 0; m < M; ++m) P->knot_off[m + 1] = P->knot_off[m] + P->nreg[m] * rl[m] * d;
  P->knots.assign((size_t)P->knot_off[M], 0.0);
  if (h_knots) {
    for (size_t q = 0; q < P->knots.size(); ++q) {
      if (!std::isfinite(h_knots[q])) return MRA_EINVAL;
      P->knots[q] = h_knots[q];
    }
  } else {
    for (int m = 0; m < M; ++m) {
      const int rm = rl[m];
      const int g = d == 2 ? (int)std::lround(std::sqrt((double)rm)) : rm;
      for (int64_t i = 0; i < P->nreg[m]; ++i) {
        const Box& b = boxes[m][i];
        double* kn = P->knots.data() + P->knot_off[m] + (size_t)i * rm * d;
        if (d == 2) {
          for (int iy = 0; iy < g; ++iy)
            for (int ix = 0; ix < g; ++ix) {
              kn[(iy * g + ix) * 2 + 0] = b.a[0] + ((b.b[0] - b.a[0]) * (double)(2 * ix + 1)) / (double)(2 * g);
              kn[(iy * g + ix) * 2 + 1] = b.a[1] + ((b.b[1] - b.a[1]) * (double)(2 * iy + 1)) / (double)(2 * g);
            }
        } else {
          for (int k = 0; k < rm; ++k)
            kn[k] = b.a[0] + ((b.b[0] - b.a[0]) * (double)(2 * k + 1)) / (double)(2 * rm);
        }
      }
    }
  }
  P->knot_xy.assign((size_t)std::max<int64_t>(n_internal, 1) * T * 2, 0.0);
  for (int m = 0; m < M; ++m)
    for (int64_t i = 0; i < P->nreg[m]; ++i) {
      const int64_t q = P->reg_base[m] + i;
      const double* kn = P->knots.data() + P->knot_off[m] + (size_t)i * rl[m] * d;
      for (int k = 0; k < rl[m]; ++k)
        for (int a = 0; a < d; ++a) P->knot_xy[(q * T + k) * 2 + a] = kn[k * d + a];
    }
  // observations
  std::vector<int64_t> leaf(cur);
  sort_by_leaf(leaf, n_leaves, P->perm, P->leaf_off);
  P->leaf_n.assign(n_leaves, 0);
  P->leaf_poff.assign(n_leaves + 1, 0);
  P->leaf_soff.assign(n_leaves, 0);
  P->leaf_doff.assign(n_leaves, 0);
  int64_t soff = 0, doff = 0;
  for (int64_t i = 0; i < n_leaves; ++i) {
    int64_t c = P->leaf_off[i + 1] - P->leaf_off[i];
    P->leaf_n[i] = (int32_t)c;
    P->max_leaf = std::max(P->max_leaf, c);
    int64_t nb = (c + T - 1) / T;
    P->leaf_poff[i + 1] = P->leaf_poff[i] + nb * T;
    P->leaf_soff[i] = soff;
    P->leaf_doff[i] = doff;
    soff += nb * nb;
    doff += nb;
  }
  P->npad = std::max<int64_t>(P->leaf_poff[n_leaves], T);
  P->n_sig_tiles = std::max<int64_t>(soff, 1);
  P->n_dinv_tiles = std::max<int64_t>(doff, 1);
  P->obs_xy.assign(P->npad * 2, 0.0);
  P->obs_gidx.assign(P->npad, -1);
  for (int64_t i = 0; i < n_leaves; ++i)
    for (int64_t k = 0; k < P->leaf_n[i]; ++k) {
      int64_t src = P->perm[P->leaf_off[i] + k];
      int64_t dst = P->leaf_poff[i] + k;
      for (int a = 0; a < d; ++a) P->obs_xy[dst * 2 + a] = h_locs[src * d + a];
      P->obs_gidx[dst] = src;
    }
  // prediction locations
  std::vector<int64_t> pleaf;
  if (n_pred > 0 && !assign_leaves(splits, Jl, h_pred, n_pred, d, M, cfg->lo, cfg->hi, pleaf)) return MRA_EINVAL;
  sort_by_leaf(pleaf, n_leaves, P->pperm, P->pleaf_off);
  P->pleaf_n.assign(n_leaves, 0);
  P->pleaf_poff.assign(n_leaves + 1, 0);
  for (int64_t i = 0; i < n_leaves; ++i) {
    int64_t c = P->pleaf_off[i + 1] - P->pleaf_off[i];
    P->pleaf_n[i] = (int32_t)c;
    P->pleaf_poff[i + 1] = P->pleaf_poff[i] + (c + T - 1) / T * T;
  }
  P->ppad = std::max<int64_t>(P->pleaf_poff[n_leaves], T);
  P->pred_xy.assign(P->ppad * 2, 0.0);
  P->pred_gidx.assign(P->ppad, -1);
  for (int64_t i = 0; i < n_leaves; ++i)
    for (int64_t k = 0; k < P->pleaf_n[i]; ++k) {
      int64_t src = P->pperm[P->pleaf_off[i] + k];
      int64_t dst = P->pleaf_poff[i] + k;
      for (int a = 0; a < d; ++a) P->pred_xy[dst * 2 + a] = h_pred[src * d + a];
      P->pred_gidx[dst] = src;
    }
  // leaf chunks (MRA_CHECKPOINT): contiguous runs of level-(M-1) regions
  // with about equal padded rows; a single chunk otherwise
  {
    const int64_t nparent = M > 0 ? P->nreg[M - 1] : 1;
    const int64_t per = M > 0 ? Jl[M] : n_leaves;   // leaves per level-(M-1) region
    int64_t K = 1;
    if ((cfg->flags & MRA_CHECKPOINT) && M > 0) K = std::min<int64_t>(cfg->chunks > 0 ? cfg->chunks : 8, nparent);
    P->chunk_leaf.assign(1, 0);
    const int64_t total = P->leaf_poff[n_leaves];
    for (int64_t c = 1; c < K; ++c) {
      const double goal = (double)total * (double)c / (double)K;
      int64_t q = P->chunk_leaf.back() / per + 1;   // at least one region per chunk
      while (q < nparent && (double)P->leaf_poff[q * per] < goal) ++q;
      if (q >= nparent) break;
      P->chunk_leaf.push_back(q * per);
    }
    P->chunk_leaf.push_back(n_leaves);
    P->nchunks = (int32_t)P->chunk_leaf.size() - 1;
    P->chunk_row.assign(P->nchunks + 1, 0);
    P->rows_cap = T;
    for (int c = 0; c <= P->nchunks; ++c) P->chunk_row[c] = P->leaf_poff[P->chunk_leaf[c]];
    for (int c = 0; c < P->nchunks; ++c) P->rows_cap = std::max(P->rows_cap, P->chunk_row[c + 1] - P->chunk_row[c]);
  }
  std::vector<int32_t> chunk_of(n_leaves, 0);
  for (int c = 0; c < P->nchunks; ++c)
    for (int64_t i = P->chunk_leaf[c]; i < P->chunk_leaf[c + 1]; ++i) chunk_of[i] = c;
  // task lists; within a chunk, leaves are visited largest first so that
  // long factorisations start early
  std::vector<int32_t> order(n_leaves);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    if (chunk_of[x] != chunk_of[y]) return chunk_of[x] < chunk_of[y];
    return P->leaf_n[x] > P->leaf_n[y];
  });
  P->row_tasks.clear(); P->sig_tasks.clear(); P->fac_tasks.clear(); P->trsm_tasks.clear(); P->linv_tasks.clear();
  P->pred_tasks.clear();
  P->ck_sig.assign(P->nchunks + 1, 0);
  P->ck_fac.assign(P->nchunks + 1, 0);
  P->ck_linv.assign(P->nchunks + 1, 0);
  for (int32_t i : order) {
    int64_t nb = (P->leaf_poff[i + 1] - P->leaf_poff[i]) / T;
    if (nb == 0) continue;
    const int c1 = chunk_of[i] + 1;
    P->fac_tasks.push_back(i);
    for (int64_t bi = 0; bi < nb; ++bi)
      for (int64_t bj = 0; bj <= bi; ++bj) {
        P->sig_tasks.push_back(i); P->sig_tasks.push_back((int32_t)bi); P->sig_tasks.push_back((int32_t)bj);
      }
    for (int c = 0; c <= M; ++c) { P->trsm_tasks.push_back(i); P->trsm_tasks.push_back(c); }
    // tile columns of L^{-1} with tiles below the diagonal
    for (int64_t j = 0; j + 1 < nb; ++j) { P->linv_tasks.push_back(i); P->linv_tasks.push_back((int32_t)j); }
    P->ck_sig[c1] = (int64_t)P->sig_tasks.size() / 3;
    P->ck_fac[c1] = (int64_t)P->fac_tasks.size();
    P->ck_linv[c1] = (int64_t)P->linv_tasks.size() / 2;
  }
  for (int c = 1; c <= P->nchunks; ++c) {   // chunks without tasks
    P->ck_sig[c] = std::max(P->ck_sig[c], P->ck_sig[c - 1]);
    P->ck_fac[c] = std::max(P->ck_fac[c], P->ck_fac[c - 1]);
    P->ck_linv[c] = std::max(P->ck_linv[c], P->ck_linv[c - 1]);
  }
  // row tiles in tree order (leaf index order is depth-first), so that
  // consecutive tasks share ancestors
  P->ck_row.assign(P->nchunks + 1, 0);
  for (int64_t i = 0; i < n_leaves; ++i) {
    const int64_t nb = (P->leaf_poff[i + 1] - P->leaf_poff[i]) / T;
    for (int64_t t = 0; t < nb; ++t) { P->row_tasks.push_back((int32_t)i); P->row_tasks.push_back((int32_t)(P->leaf_poff[i] + t * T)); }
    P->ck_row[chunk_of[i] + 1] = (int64_t)P->row_tasks.size() / 2;
  }
  for (int c = 1; c <= P->nchunks; ++c) P->ck_row[c] = std::max(P->ck_row[c], P->ck_row[c - 1]);
  {
    // a reverse row sweep costs M(M+1)/2 + M ancestor block products plus M
    // per tile of its leaf; cut the tree-ordered list into 8 runs of equal cost
    const int64_t nrow = (int64_t)P->row_tasks.size() / 2;
    std::vector<double> pre(nrow + 1, 0.0);
    for (int64_t t = 0; t < nrow; ++t) {
      const int32_t lf = P->row_tasks[2 * t];
      const double nb = (double)((P->leaf_poff[lf + 1] - P->leaf_poff[lf]) / T);
      pre[t + 1] = pre[t] + M * (M + 1) / 2 + M + M * nb;
    }
    for (int x = 0; x <= 8; ++x) {
      const double goal = pre[nrow] * x / 8.0;
      P->cut_rrows[x] = (int32_t)(std::lower_bound(pre.begin(), pre.end(), goal) - pre.begin());
    }
    P->cut_rrows[0] = 0;
    P->cut_rrows[8] = (int32_t)nrow;
  }
  // remainder blocks of each leaf's prediction points (joint distribution)
  P->pleaf_soff.assign(n_leaves, 0);
  P->pleaf_doff.assign(n_leaves, 0);
  P->pcd_tasks.clear();
  P->pfac_tasks.clear();
  {
    int64_t so = 0, dof = 0;
    for (int64_t i = 0; i < n_leaves; ++i) {
      const int64_t nbp = (P->pleaf_poff[i + 1] - P->pleaf_poff[i]) / T;
      P->pleaf_soff[i] = so;
      P->pleaf_doff[i] = dof;
      so += nbp * nbp;
      dof += nbp;
      if (nbp == 0) continue;
      P->pfac_tasks.push_back((int32_t)i);
      for (int64_t bi = 0; bi < nbp; ++bi)
        for (int64_t bj = 0; bj <= bi; ++bj) {
          P->pcd_tasks.push_back((int32_t)i); P->pcd_tasks.push_back((int32_t)bi); P->pcd_tasks.push_back((int32_t)bj);
        }
    }
    P->n_pcd_tiles = std::max<int64_t>(so, 1);
    P->n_pdinv_tiles = std::max<int64_t>(dof, 1);
  }
  P->ck_pred.assign(P->nchunks + 1, 0);
  for (int64_t i = 0; i < n_leaves; ++i) {
    int64_t nb = (P->pleaf_poff[i + 1] - P->pleaf_poff[i]) / T;
    for (int64_t t = 0; t < nb; ++t) {
      P->pred_tasks.push_back((int32_t)i); P->pred_tasks.push_back((int32_t)(P->pleaf_poff[i] + t * T));
    }
    P->ck_pred[chunk_of[i] + 1] = (int64_t)P->pred_tasks.size() / 2;
  }
  for (int c = 1; c <= P->nchunks; ++c) P->ck_pred[c] = std::max(P->ck_pred[c], P->ck_pred[c - 1]);
  if (P->npad > INT32_MAX || P->ppad > INT32_MAX) return MRA_EINVAL;

  // pruning of regions with nothing below them
  {
    std::vector<int64_t> co(P->leaf_n.begin(), P->leaf_n.end()), cp(P->pleaf_n.begin(), P->pleaf_n.end());
    std::vector<std::vector<int64_t>> obs_below(M), prd_below(M);
    for (int m = M - 1; m >= 0; --m) {
      obs_below[m].assign(P->nreg[m], 0);
      prd_below[m].assign(P->nreg[m], 0);
      for (int64_t i = 0; i < P->nreg[m]; ++i)
        for (int c = 0; c < Jl[m + 1]; ++c) {
          obs_below[m][i] += co[i * Jl[m + 1] + c];
          prd_below[m][i] += cp[i * Jl[m + 1] + c];
        }
      co = obs_below[m];
      cp = prd_below[m];
    }
    P->slot_prior.assign(n_internal, -1);
    P->slot_post.assign(n_internal, -1);
    P->act_prior.clear();
    P->act_post.clear();
    P->act_prior_off.assign(M + 1, 0);
    P->act_post_off.assign(M + 1, 0);
    for (int m = 0; m < M; ++m) {
      P->act_prior_off[m] = (int64_t)P->act_prior.size();
      P->act_post_off[m] = (int64_t)P->act_post.size();
      for (int64_t i = 0; i < P->nreg[m]; ++i) {
        if (obs_below[m][i] + prd_below[m][i] > 0) {
          P->slot_prior[P->reg_base[m] + i] = (int32_t)(P->act_prior.size() - P->act_prior_off[m]);
          P->act_prior.push_back((int32_t)i);
        }
        if (obs_below[m][i] > 0) {
          P->slot_post[P->reg_base[m] + i] = (int32_t)(P->act_post.size() - P->act_post_off[m]);
          P->act_post.push_back((int32_t)i);
        }
      }
    }
    P->act_prior_off[M] = (int64_t)P->act_prior.size();
    P->act_post_off[M] = (int64_t)P->act_post.size();
  }

  // leaf-product order of the active level-(M-1) regions
  P->reduce_order.clear();
  for (int t = 0; t < 16; ++t) P->nsmall_thr[t] = 0;
  if (M > 0) {
    const int64_t np = P->nreg[M - 1];
    std::vector<int64_t> maxnb(np, 0);
    for (int64_t q = 0; q < np; ++q)
      for (int c = 0; c < Jl[M]; ++c) {
        const int64_t lf = q * Jl[M] + c;
        maxnb[q] = std::max<int64_t>(maxnb[q], (P->leaf_poff[lf + 1] - P->leaf_poff[lf]) / T);
      }
    P->reduce_order.assign(P->act_post.begin() + P->act_post_off[M - 1], P->act_post.begin() + P->act_post_off[M]);
    std::stable_sort(P->reduce_order.begin(), P->reduce_order.end(), [&](int32_t x, int32_t y) {
      const int cx = chunk_of[(int64_t)x * Jl[M]], cy = chunk_of[(int64_t)y * Jl[M]];
      if (cx != cy) return cx < cy;
      return maxnb[x] < maxnb[y];
    });
    for (int t = 0; t < 16; ++t)
      for (int32_t q : P->reduce_order)
        if (maxnb[q] < t) ++P->nsmall_thr[t];
  }
  // per-chunk ranges of the level-(M-1) lists (both in chunk order) and of
  // the leaf-factor tiles
  P->ck_red.assign(P->nchunks + 1, 0);
  P->ck_actq.assign(P->nchunks + 1, 0);
  if (M > 0) {
    for (size_t q = 0; q < P->reduce_order.size(); ++q)
      P->ck_red[chunk_of[(int64_t)P->reduce_order[q] * Jl[M]] + 1] = (int64_t)q + 1;
    for (int64_t q = P->act_post_off[M - 1]; q < P->act_post_off[M]; ++q)
      P->ck_actq[chunk_of[(int64_t)P->act_post[q] * Jl[M]] + 1] = q - P->act_post_off[M - 1] + 1;
  }
  for (int c = 1; c <= P->nchunks; ++c) {
    P->ck_red[c] = std::max(P->ck_red[c], P->ck_red[c - 1]);
    P->ck_actq[c] = std::max(P->ck_actq[c], P->ck_actq[c - 1]);
  }
  P->ck_soff.assign(P->nchunks + 1, 0);
  P->soff_cap = 1;
  for (int c = 0; c < P->nchunks; ++c) P->ck_soff[c] = P->chunk_leaf[c] < n_leaves ? P->leaf_soff[P->chunk_leaf[c]] : soff;
  P->ck_soff[P->nchunks] = soff;
  for (int c = 0; c < P->nchunks; ++c) P->soff_cap = std::max(P->soff_cap, P->ck_soff[c + 1] - P->ck_soff[c]);

  // ---- geometry arena layout (bytes, 256-aligned) ----
  Layout& L = P->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (size_t)round_up((int64_t)(off + bytes), 256); return o; };
  L.g_knot = take(P->knot_xy.size() * 8);
  L.g_obs = take(P->obs_xy.size() * 8);
  L.g_gidx = take(P->obs_gidx.size() * 8);
  L.g_leafn = take(P->leaf_n.size() * 4);
  L.g_poff = take(P->leaf_poff.size() * 8);
  L.g_soff = take(P->leaf_soff.size() * 8);
  L.g_doff = take(P->leaf_doff.size() * 8);
  L.g_rowt = take(std::max<size_t>(P->row_tasks.size(), 1) * 4);
  L.g_sigt = take(std::max<size_t>(P->sig_tasks.size(), 1) * 4);
  L.g_fact = take(std::max<size_t>(P->fac_tasks.size(), 1) * 4);
  L.g_trst = take(std::max<size_t>(P->trsm_tasks.size(), 1) * 4);
  L.g_lint = take(std::max<size_t>(P->linv_tasks.size(), 1) * 4);
  L.g_rord = take(std::max<size_t>(P->reduce_order.size(), 1) * 4);
  L.g_slotp = take(std::max<size_t>(P->slot_prior.size(), 1) * 4);
  L.g_slotq = take(std::max<size_t>(P->slot_post.size(), 1) * 4);
  L.g_actp = take(std::max<size_t>(P->act_prior.size(), 1) * 4);
  L.g_actq = take(std::max<size_t>(P->act_post.size(), 1) * 4);
  L.g_pxy = take(P->pred_xy.size() * 8);
  L.g_pgidx = take(P->pred_gidx.size() * 8);
  L.g_pt = take(std::max<size_t>(P->pred_tasks.size(), 1) * 4);
  L.g_pleafn = take(P->pleaf_n.size() * 4);
  L.g_ppoff = take(P->pleaf_poff.size() * 8);
  L.g_psoff = take(std::max<size_t>(P->pleaf_soff.size(), 1) * 8);
  L.g_pdoff = take(std::max<size_t>(P->pleaf_doff.size(), 1) * 8);
  L.g_pcdt = take(std::max<size_t>(P->pcd_tasks.size(), 1) * 4);
  L.g_pfact = take(std::max<size_t>(P->pfac_tasks.size(), 1) * 4);
  L.geom_bytes = off;

  // ---- work arena layout (doubles per theta slice) ----
  DevPlan& D = P->dp;
  D = DevPlan{};
  D.d = d; D.M = M; D.cov = cfg->cov;
  for (int m = 0; m < MAXL; ++m) {
    D.Jl[m] = m <= M ? Jl[m] : 1;
    D.rl[m] = m < M ? rl[m] : 0;
  }
  D.n_sig_tasks = (int64_t)P->sig_tasks.size() / 3;
  D.n_sig_tiles = P->n_sig_tiles;
  D.n_row_tasks = (int64_t)P->row_tasks.size() / 2;
  D.n = n; D.npad = P->npad; D.n_leaves = n_leaves; D.ppad = P->ppad; D.n_pred = n_pred;
  int64_t w = 0;
  auto wtake = [&](int64_t doubles) { int64_t o = w; w = round_up(w + doubles, 32); return o; };
  for (int m = 0; m <= M; ++m) {
    D.nreg[m] = P->nreg[m];
    D.reg_base[m] = P->reg_base[m];
    D.act_prior_off[m] = P->act_prior_off[m];
    D.act_post_off[m] = P->act_post_off[m];
  }
  for (int m = 0; m < M; ++m) D.prior_off[m] = wtake(P->nact_prior(m) * (m + 2) * TT);
  D.plane = (P->nchunks > 1 ? P->rows_cap : P->npad) * T;
  D.off_wobs = wtake((M + 1) * D.plane);
  D.off_sig = wtake(P->n_sig_tiles * TT);
  D.off_dinv = wtake(P->n_dinv_tiles * TT);
  D.off_y = wtake((M + 1) * D.plane);
  D.off_leafd = wtake(n_leaves);
  D.off_status = wtake(4);
  D.off_scal = wtake(16);
  for (int m = 0; m < M; ++m) {
    int64_t nA = (int64_t)(m + 1) * (m + 2) / 2;
    // A tiles (the reverse pass's T-sums once the forward pass is done),
    // omega, Ltilde^{-1}, Z tiles, z_omega, d, u
    D.post_stride[m] = round_up(nA * TT + (m + 1) * T + TT + m * TT + T + 2, 32);
    D.post_off[m] = wtake(P->nact_post(m) * D.post_stride[m]);
  }
  // reverse pass: per internal region G row tiles (m+1), omega-bar (T),
  // W-bar rows (m tiles) and W-bar^m (1 tile); the T-sums take the A tiles
  if (!(cfg->flags & MRA_NO_GRAD)) {
    for (int m = 0; m < M; ++m) {
      D.grad_stride[m] = round_up((m + 1) * TT + T + m * TT + TT, 32);
      D.grad_off[m] = wtake(P->nact_post(m) * D.grad_stride[m]);
    }
    D.off_v = wtake((M + 1) * D.plane);
    D.off_linv = wtake((P->nchunks > 1 ? P->soff_cap : P->n_sig_tiles) * TT);
    // buffers that are dead by the time the reverse pass writes them: Y
    // (last read by the leaf products and by V = L^-T Y, both finished before
    // Q = V Fbar is formed) holds Q, and each W-bar row tile overwrites the Q
    // tile of the same rows and plane after reading it; Sigma-bar takes the
    // tiles of the leaf factor, whose last readers (V and L^-1) have finished
    D.off_q = D.off_y;
    D.off_wbar = D.off_y;
    D.off_sbar = D.off_sig;
    // gradient partial sums: one slot per task of every gradient-producing launch
    D.n_gpart = P->n_sig_tiles + (int64_t)P->row_tasks.size() / 2 + n_internal + 8;
    D.off_gpart = wtake(D.n_gpart * 4);
    D.off_gls0 = wtake(3 * TT + 2 * T * T);
  }
  D.off_pw = wtake(std::max(M, 1) * P->ppad * T);
  int64_t nbmax = 1;
  for (int64_t i = 0; i < n_leaves; ++i)
    if (P->pleaf_n[i] > 0) nbmax = std::max<int64_t>(nbmax, (P->leaf_poff[i + 1] - P->leaf_poff[i]) / T);
  D.pl_stride = nbmax * TT;
  D.off_pl = wtake(std::max<int64_t>((int64_t)P->pred_tasks.size() / 2, 1) * D.pl_stride);
  if ((cfg->flags & MRA_JOINT) && n_pred > 0) {
    D.off_pu = wtake(std::max(M, 1) * P->ppad * T);
    D.off_pcd = wtake(P->n_pcd_tiles * TT);
    D.off_pdinv = wtake(P->n_pdinv_tiles * TT);
    D.off_pmean = wtake(P->ppad);
    D.n_sim = n_internal * T + P->ppad;
    D.off_sim = wtake((int64_t)SIM_DRAWS * D.n_sim);
  }
  D.theta_stride = w;
  L.theta_stride = w;

  // large-leaf counts and factorisation flop prefix sums in fac_tasks order
  double rs_all = 0.0;
  for (int m = 0; m < M; ++m) rs_all += rl[m];
  {
    const int64_t nf = (int64_t)P->fac_tasks.size();
    for (int t = 0; t < 16; ++t) P->nbig_thr[t] = 0;
    P->fac_flops_pre.assign(nf + 1, 0.0);
    P->trsm_flops_pre.assign(nf + 1, 0.0);
    for (int64_t q = 0; q < nf; ++q) {
      const int32_t lf = P->fac_tasks[q];
      const int64_t nb = (P->leaf_poff[lf + 1] - P->leaf_poff[lf]) / T;
      for (int t = 0; t < 16; ++t)
        if (nb >= t) ++P->nbig_thr[t];
      const double nr = P->leaf_n[lf];
      P->fac_flops_pre[q + 1] = P->fac_flops_pre[q] + nr * nr * nr / 3.0;
      P->trsm_flops_pre[q + 1] = P->trsm_flops_pre[q] + nr * nr * (rs_all + 1);
    }
  }

  // ---- algorithmic flop model (actual r, not the padded tile) ----
  // Counts multiply-adds as 2 flops; symmetric products count one triangle;
  // triangular solves and products count r^2 per right-hand side column.
  PhaseFlops& F = P->pf;
  F = PhaseFlops{};
  // chain knots above level m: S[m] = sum_{k<m} r_k; rs = S[M]
  std::vector<double> Sk(M + 1, 0.0);
  for (int m = 0; m < M; ++m) Sk[m + 1] = Sk[m] + rl[m];
  const double rs = Sk[M];
  for (int m = 0; m < M; ++m) {
    const double Rp = (double)P->nact_prior(m), R = (double)P->nact_post(m);   // active regions
    const double rm = rl[m], Sm = Sk[m];
    double pr = rm * rm * Sm + rm * rm * rm / 3.0;                               // SYRK + POTRF
    for (int l = 0; l < m; ++l) pr += 2.0 * rm * rl[l] * Sk[l] + rm * rl[l] * rl[l];   // GEMM + TRSM
    F.prior[m] = Rp * pr;
    const double k = Sm + 1;
    F.post[m] = R * (rm * rm * rm / 3.0 + rm * rm * k);                          // POTRF + TRSM of [A^{m,<m} | w^m]
    // children of level m summed into level m-1: A~ = A - Z'Z per child
    if (m > 0) F.post_reduce[m] = R * Sm * (Sm + 1) * rm + R * 2.0 * Sm * rm;
    // reverse: V = Lt^{-T} Z, Xbar = 2 V Fbar, Pbar = -V Fbar V' - P^{-1}/2
    F.rpost[m] = R * (rm * rm * k + 2.0 * rm * Sm * Sm + 2.0 * rm * rm * Sm + rm * rm * rm);
    // Cholesky adjoint (3 triangular products), -2 Wbar^m W^^k, reverse row sweep
    double rp = 3.0 * rm * rm * rm + 2.0 * rm * rm * Sm;
    for (int l = 0; l < m; ++l) rp += 2.0 * rm * rl[l] * rl[l] + 2.0 * rm * rl[l] * Sk[l];
    F.rprior[m] = R * rp;
    // subtree sums of level m (children) into level m-1: Wbar^l' W^^k, k <= l < m
    double rt = 0.0;
    for (int l = 0; l < m; ++l) rt += 2.0 * rm * rl[l] * Sk[l + 1];
    F.rT[m] = R * rt;
  }
  double rows_sweep = 0.0, rows_rev = 0.0, rows_T = 0.0;   // per observation
  for (int l = 0; l < M; ++l) {
    rows_sweep += 2.0 * rl[l] * Sk[l] + (double)rl[l] * rl[l];
    rows_rev += 2.0 * (double)rl[l] * rl[l] + 2.0 * rl[l] * (rs - Sk[l + 1]);
    rows_T += 2.0 * rl[l] * Sk[l + 1];
  }
  for (int64_t i = 0; i < n_leaves; ++i) {
    const double nr = P->leaf_n[i];
    if (nr == 0) continue;
    F.leaf_rows += nr * rows_sweep;                            // rows of W^: GEMM + TRSM per level
    F.sigma += nr * nr * rs;                                   // Sigma_R (SYRK)
    F.potrf += nr * nr * nr / 3.0;
    F.trsm += nr * nr * (rs + 1);                              // L^{-1} [W^ | z]
    F.leaf_reduce += nr * (rs + 1) * (rs + 1);                 // [W^ | z]' Sigma^{-1} [W^ | z]
    F.rleaf_v += nr * nr * (rs + 1);                           // L^{-T} Y
    F.rleaf_linv += nr * nr * nr / 3.0;                        // L^{-1}
    F.rleaf_q += 2.0 * nr * (rs + 1) * (rs + 1);               // V Fbar
    F.rleaf_sbar += nr * nr * (rs + 1) + nr * nr * nr / 3.0;   // -Q V' - Sigma^{-1}/2 (lower half)
    F.rleaf_wbar += 2.0 * nr * nr * rs;                        // Sigma-bar W^
    F.rrows += nr * rows_rev;                                  // Wbar^l = W^bar L^{-1}, W^-bar updates
    F.rT_leaf += nr * rows_T;                                  // Wbar^l' W^^k, k <= l
  }
  double fl = F.leaf_rows + F.sigma + F.potrf + F.trsm + F.leaf_reduce;
  double rv = F.rleaf_v + F.rleaf_linv + F.rleaf_q + F.rleaf_sbar + F.rleaf_wbar + F.rrows + F.rT_leaf;
  for (int m = 0; m < M; ++m) {
    fl += F.prior[m] + F.post[m] + F.post_reduce[m];
    rv += F.rpost[m] + F.rprior[m] + F.rT[m];
  }
  P->flops_loglik = fl;
  P->flops_grad = fl + rv;
  double fp = 0.0;
  for (int64_t i = 0; i < n_leaves; ++i) {
    const double np = P->pleaf_n[i], nr = P->leaf_n[i];
    if (np == 0) continue;
    fp += np * rows_sweep;                               // U^ rows
    fp += 2.0 * np * nr * rs + np * nr * nr;             // L^M and E = L^M L^{-T}
    fp += 2.0 * np * nr * rs;                            // B~^M
    for (int l = 0; l < M; ++l) fp += np * ((double)rl[l] * rl[l] + 2.0 * rl[l] * Sk[l]);
  }
  F.predict = fp;
  P->flops_predict = fp;
  return MRA_OK;
}

}  // namespace mra
