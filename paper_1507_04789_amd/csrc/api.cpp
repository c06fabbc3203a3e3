// C ABI of the M-RA library (declared in include/mra.h).
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <new>
#include <utility>

#include "launch.hpp"
#include "plan.hpp"

namespace mra {

hipError_t launch_predict(const mra_plan_s& H, const double* y, const double* theta, double* mean, double* var,
                          hipStream_t st, bool keep = false);
hipError_t noalloc_scratch(void** out);   // noalloc.hip
hipError_t launch_predict_cov(const mra_plan_s& H, const double* theta, double* cov, hipStream_t st);
hipError_t launch_simulate(const mra_plan_s& H, const double* theta, const double* eps, int64_t n_eps, int nd,
                           double* out, hipStream_t st);

namespace {

mra_status check_hip(hipError_t e) { return e == hipSuccess ? MRA_OK : MRA_EHIP; }

// after a synchronised call: find the first parameter vector whose
// factorisations broke down
mra_status collect_failures(mra_plan_s* H, int nth, hipStream_t st) {
  if (hipStreamSynchronize(st) != hipSuccess) return MRA_EHIP;
  H->fail_theta = -1;
  H->fail_level = -1;
  H->fail_region = -1;
  for (int th = 0; th < nth; ++th) {
    int64_t code = 0;
    const double* src = H->call_work + (int64_t)th * H->dp.theta_stride + H->dp.off_status;
    if (hipMemcpy(&code, src, sizeof(code), hipMemcpyDeviceToHost) != hipSuccess) return MRA_EHIP;
    if (code != 0) {
      H->fail_theta = th;
      code -= 1;
      H->fail_level = (int32_t)(code >> 40);
      H->fail_region = code & ((1ll << 40) - 1);
      return MRA_ENOTPD;
    }
  }
  return MRA_OK;
}

// forward + reverse.  The reverse pass's leaf solves only need the forward
// leaf factors, so they run on a second stream (default priority) while the
// posterior recursion and its reverse proceed on the caller's stream.
hipError_t ensure_side(mra_plan_s* H) {
  if (H->side_stream) return hipSuccess;
  hipStream_t s2;
  constexpr int NEV = 7;
  hipEvent_t ev[NEV] = {};
  hipError_t e;
  for (int i = 0; i < NEV; ++i)
    if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return e;
    }
  if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess) {
    for (int j = 0; j < NEV; ++j) (void)hipEventDestroy(ev[j]);
    return e;
  }
  H->side_stream = s2;
  H->ev_fork = ev[0];
  H->ev_big = ev[1];
  H->ev_fork2 = ev[2];
  H->ev_join = ev[3];
  H->ev_join2 = ev[4];
  H->ev_gfork = ev[5];
  H->ev_gath = ev[6];
  return hipSuccess;
}

// the second stream is used by the batched forms without checkpointing
bool uses_side(const mra_plan_s* H) { return !(H->cfg.flags & MRA_PLAIN) && H->nchunks == 1; }

Side side_of(const mra_plan_s* H) {
  return Side{(hipStream_t)H->side_stream, (hipEvent_t)H->ev_fork,  (hipEvent_t)H->ev_big,
              (hipEvent_t)H->ev_fork2,     (hipEvent_t)H->ev_join,  (hipEvent_t)H->ev_join2,
              (hipEvent_t)H->ev_gfork,     (hipEvent_t)H->ev_gath};
}

}  // namespace

// Captured launch sequences (MRA_GRAPH).  A call's whole launch sequence,
// both streams included, is captured once on a private stream and replayed
// with one hipGraphLaunch on the caller's stream.  Kernel arguments are baked
// into the graph, so the key holds every pointer and count they depend on;
// a bind (new arenas) drops the cache.  Nothing in the sequence is a memset
// or copy node: buffers are cleared by kernels.
struct GraphKey {
  int kind;  // 0 loglik, 1 loglik + grad, 2 predict
  int nth;
  const void* p[5];
  int64_t y_stride = 0;
  bool operator<(const GraphKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (nth != o.nth) return nth < o.nth;
    if (y_stride != o.y_stride) return y_stride < o.y_stride;
    for (int i = 0; i < 5; ++i)
      if (p[i] != o.p[i]) return p[i] < o.p[i];
    return false;
  }
};
constexpr size_t kMaxGraphs = 16;
struct GraphCache {
  hipStream_t cap = nullptr;
  std::map<GraphKey, hipGraphExec_t> exec;
  void clear() {
    for (auto& kv : exec) (void)hipGraphExecDestroy(kv.second);
    exec.clear();
  }
};

namespace {

// run `enqueue(stream)` on st directly, or through the plan's graph cache
template <class F>
hipError_t run_call(mra_plan_s* H, const GraphKey& key, hipStream_t st, F enqueue) {
  const bool profiling = H->prof && H->prof->enabled;
  if (!(H->cfg.flags & MRA_GRAPH) || profiling) return enqueue(st);
  if (!H->graphs) {
    H->graphs = new (std::nothrow) GraphCache();
    if (!H->graphs) return hipErrorOutOfMemory;
  }
  GraphCache& C = *H->graphs;
  auto it = C.exec.find(key);
  if (it == C.exec.end()) {
    hipError_t e;
    if (C.exec.size() >= kMaxGraphs) C.clear();   // callers that keep changing buffers
    if (!C.cap && (e = hipStreamCreateWithFlags(&C.cap, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(C.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t el = enqueue(C.cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(C.cap, &g);
    if (el != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return el != hipSuccess ? el : e;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    it = C.exec.emplace(key, x).first;
  }
  return hipGraphLaunch(it->second, st);
}

// allow_side = false keeps every launch on st (no second stream or events)
hipError_t launch_grad_all(mra_plan_s* H, const double* y, const double* theta, int nth, double* ll, double* g,
                           double* gy, hipStream_t st, int64_t y_stride = 0, bool allow_side = true) {
  const bool overlap = allow_side && uses_side(H);
  hipError_t e;
  if (overlap && (e = ensure_side(H)) != hipSuccess) return e;
  const Side sd = side_of(H);
  const Side* side = overlap ? &sd : nullptr;
  // the partial sums are cleared up front, where the GPU is nearly idle,
  // rather than in the reverse posterior chain
  if ((e = launch_zero_gpart(*H, nth, st)) != hipSuccess) return e;
  if ((e = launch_forward_front(*H, y, theta, nth, st, side, y_stride)) != hipSuccess) return e;
  const bool on_side = side && H->side_solves > 0;
  if (!on_side) {
    if (side && H->nbig() > 0 && (e = hipStreamWaitEvent(st, sd.big, 0)) != hipSuccess) return e;   // every leaf
    if ((e = launch_grad_leafsolve(*H, nth, st)) != hipSuccess) return e;
  }
  // otherwise the leaf solves go on the side stream at stage side_solves - 1
  // of the recursion (ForkHook; event fork2): after the small leaves on the
  // main stream and, in stream order, after the large ones on the side
  // stream.  They only read the leaf factors and Y and write V and L^{-1},
  // which nothing on the main stream touches before the joins (join before
  // the first use of V, join2 before that of L^{-1}).
  struct Ctx {
    mra_plan_s* H;
    const Side* sd;
    hipStream_t st;
    int nth;
  } ctx{H, &sd, st, nth};
  ForkHook hook{H->side_solves - 1, [](void* p) -> hipError_t {
    const Ctx& c = *static_cast<const Ctx*>(p);
    hipError_t r;
    if ((r = hipEventRecord(c.sd->fork2, c.st)) != hipSuccess) return r;
    if ((r = hipStreamWaitEvent(c.sd->s, c.sd->fork2, 0)) != hipSuccess) return r;
    if ((r = launch_grad_leafsolve(*c.H, c.nth, c.sd->s, c.sd->join)) != hipSuccess) return r;
    return hipEventRecord(c.sd->join2, c.sd->s);
  }, &ctx, false};
  ForkHook* hk = on_side ? &hook : nullptr;
  if ((e = launch_forward_back(*H, nth, ll, st, side, hk)) != hipSuccess) return e;
  if ((e = launch_grad_post(*H, nth, st, hk, false)) != hipSuccess) return e;
  if (on_side && (e = hipStreamWaitEvent(st, sd.join, 0)) != hipSuccess) return e;
  return launch_grad_rest(*H, y, y_stride, theta, nth, g, gy, st, on_side ? sd.join2 : nullptr);
}

// ---- tuning table (JSON) ----
std::string tuning_json(const mra_plan_s* H, double ms) {
  std::string j = "{\"version\": 1, ";
  char buf[96];
  if (ms > 0) {
    std::snprintf(buf, sizeof buf, "\"ms_per_call\": %.6g, ", ms);
    j += buf;
  }
  std::snprintf(buf, sizeof buf, "\"big_leaf_tiles\": %d, \"side_solves\": %d, \"families\": {", H->big_tiles,
                H->side_solves);
  j += buf;
  for (int f = 0; f < F_COUNT; ++f) {
    std::snprintf(buf, sizeof buf, "%s\"%s\": \"%s\"", f ? ", " : "", fam_name(f), map_name(H->tune[f]));
    j += buf;
  }
  j += "}}";
  return j;
}

mra_status copy_out(const std::string& j, char* out, size_t cap, size_t* len) {
  if (len) *len = j.size();
  if (!out) return MRA_OK;
  if (cap < j.size() + 1) return MRA_ENOMEM;
  std::memcpy(out, j.c_str(), j.size() + 1);
  return MRA_OK;
}

// value of "key": in a flat JSON text, a quoted string or a number:
// 1 found, 0 key absent, -1 key present with a malformed value
int json_value(const char* js, const char* key, std::string& val) {
  const std::string k = std::string("\"") + key + "\"";
  const char* p = std::strstr(js, k.c_str());
  if (!p) return 0;
  p += k.size();
  while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
  if (*p != ':') return -1;
  ++p;
  while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p;
  val.clear();
  if (*p == '"') {
    ++p;
    while (*p && *p != '"') val += *p++;
    return *p == '"' ? 1 : -1;
  }
  while (*p && (*p == '-' || (*p >= '0' && *p <= '9'))) val += *p++;
  return val.empty() ? -1 : 1;
}

// a JSON number token that is a whole integer in [lo, hi]; anything else
// ("--3", "1-2", out-of-range digits) is refused rather than wrapped
bool parse_int(const std::string& v, int lo, int hi, int32_t& out) {
  if (v.empty() || v.size() > 12) return false;
  char* end = nullptr;
  errno = 0;
  const long long x = std::strtoll(v.c_str(), &end, 10);
  if (errno != 0 || end != v.c_str() + v.size() || x < lo || x > hi) return false;
  out = (int32_t)x;
  return true;
}

mra_status check_call(const mra_plan_s* H, int nth) {
  if (!H) return MRA_EINVAL;
  if (!H->bound) return MRA_ESTATE;
  if (nth < 1 || nth > H->cfg.max_theta) return MRA_EINVAL;
  return MRA_OK;
}

// every compute call records the work arena its status words live in
void set_call_work(mra_plan_s* H) { H->call_work = H->dp.work; }

}  // namespace
}  // namespace mra

using namespace mra;

extern "C" {

mra_status mra_build(const mra_config* cfg, const double* h_locs, int64_t n, const double* h_pred, int64_t n_pred,
                     const double* h_knots, mra_plan_t* out) {
  if (!out) return MRA_EINVAL;
  *out = nullptr;
  mra_plan_s* P = new (std::nothrow) mra_plan_s();
  if (!P) return MRA_ENOMEM;
  mra_status s;
  try {
    s = build_plan(cfg, h_locs, n, h_pred, n_pred, h_knots, P);
  } catch (const std::bad_alloc&) {
    s = MRA_ENOMEM;
  }
  if (s != MRA_OK) {
    delete P;
    return s;
  }
  *out = P;
  return MRA_OK;
}

mra_status mra_requirements(mra_plan_t P, size_t* geom_bytes, size_t* work_bytes) {
  if (!P) return MRA_EINVAL;
  if (geom_bytes) *geom_bytes = P->lay.geom_bytes;
  if (work_bytes) *work_bytes = (size_t)P->lay.theta_stride * 8 * (size_t)P->cfg.max_theta;
  return MRA_OK;
}

mra_status mra_get_info(mra_plan_t P, mra_info* info) {
  if (!P || !info) return MRA_EINVAL;
  info->n = P->n;
  info->n_pred = P->n_pred;
  info->n_rows_pad = P->npad;
  info->n_leaves = P->nreg[P->M];
  info->n_regions = P->reg_base[P->M] + P->nreg[P->M];
  info->max_leaf = P->max_leaf;
  info->flops_loglik = P->flops_loglik;
  info->flops_grad = P->flops_grad;
  info->flops_predict = P->flops_predict;
  info->n_sim_normals = P->reg_base[P->M] * T + P->n_pred;
  return MRA_OK;
}

mra_status mra_get_geometry(mra_plan_t P, int64_t* h_perm, int64_t* h_leaf_offsets, double* h_knots) {
  if (!P) return MRA_EINVAL;
  if (h_perm) std::memcpy(h_perm, P->perm.data(), P->perm.size() * sizeof(int64_t));
  if (h_leaf_offsets) std::memcpy(h_leaf_offsets, P->leaf_off.data(), P->leaf_off.size() * sizeof(int64_t));
  if (h_knots && !P->knots.empty()) std::memcpy(h_knots, P->knots.data(), P->knots.size() * sizeof(double));
  return MRA_OK;
}

mra_status mra_bind(mra_plan_t P, void* d_geom, size_t geom_bytes, void* d_work, size_t work_bytes, void* stream) {
  if (!P || !d_geom || (!d_work && work_bytes != 0)) return MRA_EINVAL;
  if (((uintptr_t)d_geom & 255) || ((uintptr_t)d_work & 255)) return MRA_EINVAL;
  size_t need_g, need_w;
  mra_requirements(P, &need_g, &need_w);
  if (geom_bytes < need_g || (d_work && work_bytes < need_w)) return MRA_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  char* g = (char*)d_geom;
  const Layout& L = P->lay;
  auto up = [&](size_t off, const void* src, size_t bytes) -> bool {
    if (bytes == 0) return true;
    return hipMemcpyAsync(g + off, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = up(L.g_knot, P->knot_xy.data(), P->knot_xy.size() * 8) && up(L.g_obs, P->obs_xy.data(), P->obs_xy.size() * 8) &&
            up(L.g_gidx, P->obs_gidx.data(), P->obs_gidx.size() * 8) &&
            up(L.g_leafn, P->leaf_n.data(), P->leaf_n.size() * 4) &&
            up(L.g_poff, P->leaf_poff.data(), P->leaf_poff.size() * 8) &&
            up(L.g_soff, P->leaf_soff.data(), P->leaf_soff.size() * 8) &&
            up(L.g_doff, P->leaf_doff.data(), P->leaf_doff.size() * 8) &&
            up(L.g_rowt, P->row_tasks.data(), P->row_tasks.size() * 4) &&
            up(L.g_sigt, P->sig_tasks.data(), P->sig_tasks.size() * 4) &&
            up(L.g_fact, P->fac_tasks.data(), P->fac_tasks.size() * 4) &&
            up(L.g_trst, P->trsm_tasks.data(), P->trsm_tasks.size() * 4) &&
            up(L.g_lint, P->linv_tasks.data(), P->linv_tasks.size() * 4) &&
            up(L.g_rord, P->reduce_order.data(), P->reduce_order.size() * 4) &&
            up(L.g_slotp, P->slot_prior.data(), P->slot_prior.size() * 4) &&
            up(L.g_slotq, P->slot_post.data(), P->slot_post.size() * 4) &&
            up(L.g_actp, P->act_prior.data(), P->act_prior.size() * 4) &&
            up(L.g_actq, P->act_post.data(), P->act_post.size() * 4) &&
            up(L.g_pxy, P->pred_xy.data(), P->pred_xy.size() * 8) &&
            up(L.g_pgidx, P->pred_gidx.data(), P->pred_gidx.size() * 8) &&
            up(L.g_pt, P->pred_tasks.data(), P->pred_tasks.size() * 4) &&
            up(L.g_pleafn, P->pleaf_n.data(), P->pleaf_n.size() * 4) &&
            up(L.g_ppoff, P->pleaf_poff.data(), P->pleaf_poff.size() * 8) &&
            up(L.g_psoff, P->pleaf_soff.data(), P->pleaf_soff.size() * 8) &&
            up(L.g_pdoff, P->pleaf_doff.data(), P->pleaf_doff.size() * 8) &&
            up(L.g_pcdt, P->pcd_tasks.data(), P->pcd_tasks.size() * 4) &&
            up(L.g_pfact, P->pfac_tasks.data(), P->pfac_tasks.size() * 4);
  if (!ok || hipStreamSynchronize(st) != hipSuccess) return MRA_EHIP;
  DevPlan& D = P->dp;
  D.knot_xy = (const double*)(g + L.g_knot);
  D.obs_xy = (const double*)(g + L.g_obs);
  D.obs_gidx = (const int64_t*)(g + L.g_gidx);
  D.leaf_n = (const int32_t*)(g + L.g_leafn);
  D.leaf_poff = (const int64_t*)(g + L.g_poff);
  D.leaf_soff = (const int64_t*)(g + L.g_soff);
  D.leaf_doff = (const int64_t*)(g + L.g_doff);
  D.row_tasks = (const int32_t*)(g + L.g_rowt);
  D.sig_tasks = (const int32_t*)(g + L.g_sigt);
  D.fac_tasks = (const int32_t*)(g + L.g_fact);
  D.trsm_tasks = (const int32_t*)(g + L.g_trst);
  D.linv_tasks = (const int32_t*)(g + L.g_lint);
  D.reduce_order = (const int32_t*)(g + L.g_rord);
  D.slot_prior = (const int32_t*)(g + L.g_slotp);
  D.slot_post = (const int32_t*)(g + L.g_slotq);
  D.act_prior = (const int32_t*)(g + L.g_actp);
  D.act_post = (const int32_t*)(g + L.g_actq);
  D.pred_xy = (const double*)(g + L.g_pxy);
  D.pred_gidx = (const int64_t*)(g + L.g_pgidx);
  D.pred_tasks = (const int32_t*)(g + L.g_pt);
  D.pleaf_n = (const int32_t*)(g + L.g_pleafn);
  D.pleaf_poff = (const int64_t*)(g + L.g_ppoff);
  D.pleaf_soff = (const int64_t*)(g + L.g_psoff);
  D.pleaf_doff = (const int64_t*)(g + L.g_pdoff);
  D.pcd_tasks = (const int32_t*)(g + L.g_pcdt);
  D.pfac_tasks = (const int32_t*)(g + L.g_pfact);
  D.work = (double*)d_work;
  if (P->graphs) P->graphs->clear();
  P->d_geom = d_geom;
  P->d_work = d_work;
  P->geom_bound = true;
  P->bound = d_work != nullptr;
  P->call_work = nullptr;
  return MRA_OK;
}

mra_status mra_loglik(mra_plan_t P, const double* d_y, const double* d_theta, int32_t n_theta, double* d_loglik,
                      void* stream) {
  mra_status s = check_call(P, n_theta);
  if (s != MRA_OK) return s;
  if (!d_y || !d_theta || !d_loglik) return MRA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = n_theta;
  const bool overlap = uses_side(P);
  if (overlap && (s = check_hip(ensure_side(P))) != MRA_OK) return s;
  const GraphKey key{0, n_theta, {d_y, d_theta, d_loglik, nullptr, nullptr}};
  const Side sd = side_of(P);
  s = check_hip(run_call(P, key, st, [&](hipStream_t q) {
    hipError_t e = launch_forward_front(*P, d_y, d_theta, n_theta, q, overlap ? &sd : nullptr);
    if (e != hipSuccess) return e;
    return launch_forward_back(*P, n_theta, d_loglik, q, overlap ? &sd : nullptr);
  }));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, n_theta, st);
  return MRA_OK;
}

namespace {
mra_status loglik_grad_call(mra_plan_t P, const double* d_y, int64_t y_stride, const double* d_theta,
                            int32_t n_theta, double* d_loglik, double* d_grad, double* d_grad_y, void* stream) {
  mra_status s = check_call(P, n_theta);
  if (s != MRA_OK) return s;
  if (!d_y || !d_theta || !d_loglik || !d_grad) return MRA_EINVAL;
  if (y_stride != 0 && y_stride < P->n) return MRA_EINVAL;
  if (P->cfg.flags & MRA_NO_GRAD) return MRA_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = n_theta;
  if (uses_side(P) && (s = check_hip(ensure_side(P))) != MRA_OK) return s;
  const GraphKey key{1, n_theta, {d_y, d_theta, d_loglik, d_grad, d_grad_y}, y_stride};
  s = check_hip(run_call(P, key, st, [&](hipStream_t q) {
    return launch_grad_all(P, d_y, d_theta, n_theta, d_loglik, d_grad, d_grad_y, q, y_stride);
  }));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, n_theta, st);
  return MRA_OK;
}
}  // namespace

mra_status mra_loglik_grad(mra_plan_t P, const double* d_y, const double* d_theta, int32_t n_theta, double* d_loglik,
                           double* d_grad, void* stream) {
  return loglik_grad_call(P, d_y, 0, d_theta, n_theta, d_loglik, d_grad, nullptr, stream);
}

mra_status mra_loglik_grad_data(mra_plan_t P, const double* d_y, int64_t y_stride, const double* d_theta,
                                int32_t n_theta, double* d_loglik, double* d_grad, double* d_grad_y, void* stream) {
  if (!d_grad_y) return MRA_EINVAL;
  return loglik_grad_call(P, d_y, y_stride, d_theta, n_theta, d_loglik, d_grad, d_grad_y, stream);
}

mra_status mra_loglik_grad_noalloc(mra_plan_t P, const double* d_y, const double* d_theta, int32_t n_theta,
                                   double* d_loglik, double* d_grad, void* stream) {
  if (!P) return MRA_EINVAL;
  if (!P->geom_bound) return MRA_ESTATE;
  if (n_theta < 1 || n_theta > P->cfg.max_theta) return MRA_EINVAL;
  if (!d_y || !d_theta || !d_loglik || !d_grad) return MRA_EINVAL;
  if (P->cfg.flags & MRA_NO_GRAD) return MRA_ESTATE;
  if ((size_t)P->lay.theta_stride * 8 * (size_t)n_theta > MRA_NOALLOC_MAX_BYTES) return MRA_ENOMEM;
  void* ptr = nullptr;
  mra_status s = check_hip(noalloc_scratch(&ptr));
  if (s != MRA_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  // run the ordinary launch sequence against the scratch array: one stream,
  // no captured graph, no profiling events
  double* const keep_work = P->dp.work;
  const bool prof = P->prof && P->prof->enabled;
  if (prof) P->prof->enabled = false;
  P->dp.work = (double*)ptr;
  P->call_work = (double*)ptr;
  P->last_nth = n_theta;
  s = check_hip(launch_grad_all(P, d_y, d_theta, n_theta, d_loglik, d_grad, nullptr, st, 0, false));
  P->dp.work = keep_work;
  if (prof) P->prof->enabled = true;
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, n_theta, st);
  return MRA_OK;
}

mra_status mra_gls(mra_plan_t P, const double* d_y, const double* d_X, int32_t p, const double* d_theta,
                   double* d_beta, double* d_loglik, double* d_grad, double* d_resid, double* d_XtSiX, void* stream) {
  mra_status s = check_call(P, 1);
  if (s != MRA_OK) return s;
  if (!d_y || !d_X || !d_theta || !d_beta || !d_loglik || !d_grad || !d_resid) return MRA_EINVAL;
  if (p < 1 || p > T - 1) return MRA_EINVAL;
  if (P->cfg.flags & MRA_NO_GRAD) return MRA_ESTATE;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = 1;
  s = check_hip(launch_gls(*P, d_y, d_X, p, d_theta, d_beta, d_loglik, d_XtSiX, d_grad, d_resid, st));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, 1, st);
  return MRA_OK;
}

mra_status mra_predict(mra_plan_t P, const double* d_y, const double* d_theta, double* d_mean, double* d_var,
                       void* stream) {
  mra_status s = check_call(P, 1);
  if (s != MRA_OK) return s;
  if (!d_y || !d_theta || !d_mean || !d_var) return MRA_EINVAL;
  if (P->n_pred == 0) return MRA_OK;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = 1;
  const GraphKey key{2, 1, {d_y, d_theta, d_mean, d_var, nullptr}};
  s = check_hip(run_call(P, key, st, [&](hipStream_t q) {
    hipError_t e = launch_forward(*P, d_y, d_theta, 1, nullptr, q);
    if (e != hipSuccess) return e;
    return launch_predict(*P, d_y, d_theta, d_mean, d_var, q);
  }));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, 1, st);
  return MRA_OK;
}

mra_status mra_predict_cov(mra_plan_t P, const double* d_y, const double* d_theta, double* d_mean, double* d_cov,
                           void* stream) {
  mra_status s = check_call(P, 1);
  if (s != MRA_OK) return s;
  if (!d_y || !d_theta || !d_mean || !d_cov) return MRA_EINVAL;
  if (!(P->cfg.flags & MRA_JOINT)) return MRA_ESTATE;
  if (P->n_pred == 0) return MRA_OK;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = 1;
  // the kriging pass writes its marginal variances into d_cov, which the
  // covariance tiles then overwrite entirely
  s = check_hip(launch_forward(*P, d_y, d_theta, 1, nullptr, st));
  if (s == MRA_OK) s = check_hip(launch_predict(*P, d_y, d_theta, d_mean, d_cov, st, true));
  if (s == MRA_OK) s = check_hip(launch_predict_cov(*P, d_theta, d_cov, st));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, 1, st);
  return MRA_OK;
}

mra_status mra_simulate(mra_plan_t P, const double* d_y, const double* d_theta, const double* d_eps,
                        int64_t eps_stride, int32_t n_draws, double* d_out, void* stream) {
  mra_status s = check_call(P, 1);
  if (s != MRA_OK) return s;
  if (!d_y || !d_theta || !d_eps || !d_out) return MRA_EINVAL;
  if (n_draws < 1 || n_draws > SIM_DRAWS) return MRA_EINVAL;
  if (eps_stride < P->reg_base[P->M] * T + P->n_pred) return MRA_EINVAL;
  if (!(P->cfg.flags & MRA_JOINT)) return MRA_ESTATE;
  if (P->n_pred == 0) return MRA_OK;
  hipStream_t st = (hipStream_t)stream;
  set_call_work(P);
  P->last_nth = 1;
  // the kriging pass writes its mean and variances into d_out, which the
  // draws then overwrite entirely
  s = check_hip(launch_forward(*P, d_y, d_theta, 1, nullptr, st));
  if (s == MRA_OK) s = check_hip(launch_predict(*P, d_y, d_theta, d_out, d_out, st, true));
  if (s == MRA_OK) s = check_hip(launch_simulate(*P, d_theta, d_eps, eps_stride, n_draws, d_out, st));
  if (s != MRA_OK) return s;
  if (P->cfg.flags & MRA_SYNC) return collect_failures(P, 1, st);
  return MRA_OK;
}

mra_status mra_last_failure(mra_plan_t P, int32_t* theta_idx, int32_t* level, int64_t* region, void* stream) {
  if (!P) return MRA_EINVAL;
  if (!(P->cfg.flags & MRA_SYNC) && P->call_work) {
    mra_status s = collect_failures(P, P->last_nth, (hipStream_t)stream);
    if (s == MRA_EHIP) return s;
  }
  if (theta_idx) *theta_idx = P->fail_theta;
  if (level) *level = P->fail_level;
  if (region) *region = P->fail_region;
  return MRA_OK;
}

mra_status mra_get_tuning(mra_plan_t P, char* out_json, size_t cap, size_t* len) {
  if (!P) return MRA_EINVAL;
  return copy_out(tuning_json(P, 0.0), out_json, cap, len);
}

mra_status mra_set_tuning(mra_plan_t P, const char* json) {
  if (!P || !json) return MRA_EINVAL;
  uint8_t t[32] = {};
  int32_t big = P->big_tiles;
  std::string v;
  for (int f = 0; f < F_COUNT; ++f) {
    const int got = json_value(json, fam_name(f), v);
    if (got < 0) return MRA_EINVAL;
    if (got == 0) continue;
    int m = -1;
    for (int c = 0; c < 4; ++c)
      if (v == map_name(c)) m = c;
    if (m < 0) return MRA_EINVAL;
    t[f] = (uint8_t)m;
  }
  int got = json_value(json, "big_leaf_tiles", v);
  if (got < 0 || (got > 0 && !parse_int(v, 0, 64, big))) return MRA_EINVAL;
  int32_t sides = P->side_solves;
  got = json_value(json, "side_solves", v);
  if (got < 0 || (got > 0 && !parse_int(v, 0, 64, sides))) return MRA_EINVAL;
  std::memcpy(P->tune, t, sizeof t);
  P->big_tiles = big;
  P->side_solves = sides;
  if (P->graphs) P->graphs->clear();
  return MRA_OK;
}

mra_status mra_autotune(mra_plan_t P, const double* d_y, const double* d_theta, int32_t n_theta, double* d_loglik,
                        double* d_grad, int32_t reps, char* out_json, size_t cap, size_t* len, void* stream) {
  mra_status s = check_call(P, n_theta);
  if (s != MRA_OK) return s;
  const bool grad = !(P->cfg.flags & MRA_NO_GRAD);
  if (!d_y || !d_theta || !d_loglik || (grad && !d_grad) || reps < 1) return MRA_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool overlap = uses_side(P);
  if (overlap && (s = check_hip(ensure_side(P))) != MRA_OK) return s;
  const bool prof = P->prof && P->prof->enabled;
  if (prof) P->prof->enabled = false;
  set_call_work(P);
  P->last_nth = n_theta;
  const Side sd = side_of(P);
  auto call = [&]() -> hipError_t {
    if (grad) return launch_grad_all(P, d_y, d_theta, n_theta, d_loglik, d_grad, nullptr, st);
    hipError_t e = launch_forward_front(*P, d_y, d_theta, n_theta, st, overlap ? &sd : nullptr);
    return e != hipSuccess ? e : launch_forward_back(*P, n_theta, d_loglik, st, overlap ? &sd : nullptr);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (prof) P->prof->enabled = true;
    return MRA_EHIP;
  }
  bool ok = true;
  auto measure = [&]() -> double {
    if (call() != hipSuccess) ok = false;   // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
      if (call() != hipSuccess) ok = false;
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ok = false;
    return ok ? (double)ms / reps : 1e30;
  };
  // coordinate descent: one pass over the families, then the large-leaf cut;
  // a change is kept only if it is faster by more than 0.5 %
  const bool grouped[F_COUNT] = {false, false, false, false, true, true, false, true, true, false,
                                 false, true, false, false, true, false, true, false};
  const bool reverse[F_COUNT] = {false, false, false, false, false, false, false, false, true, true,
                                 true, true, true, true, true, true, true, false};
  double best = measure();
  for (int f = 0; f < F_COUNT && ok; ++f) {
    if (f == F_PREDICT || (reverse[f] && !grad)) continue;
    const uint8_t keep = P->tune[f];
    uint8_t pick = keep;
    for (uint8_t m = MAP_IDENTITY; m <= MAP_CHUNKED && ok; ++m) {
      if (m == MAP_GROUPED && !grouped[f]) continue;
      P->tune[f] = m;
      const double t = measure();
      if (t < best * 0.995) {
        best = t;
        pick = m;
      }
    }
    P->tune[f] = pick;
  }
  if (overlap && ok) {
    const int32_t keep = P->big_tiles;
    int32_t pick = keep;
    for (int32_t b : {0, 2, 3, 4, 6}) {
      if (b == keep) continue;
      P->big_tiles = b;
      const double t = measure();
      if (t < best * 0.995) {
        best = t;
        pick = b;
      }
    }
    P->big_tiles = pick;
    if (grad) {
      const int32_t keep_s = P->side_solves;
      int32_t pick_s = keep_s;
      for (int32_t v = 0; v <= 2 * P->M + 2 && ok; ++v) {
        if (v == keep_s) continue;
        P->side_solves = v;
        const double t = measure();
        if (t < best * 0.995) {
          best = t;
          pick_s = v;
        }
      }
      P->side_solves = pick_s;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (prof) P->prof->enabled = true;
  if (P->graphs) P->graphs->clear();
  if (!ok) return MRA_EHIP;
  if (P->cfg.flags & MRA_SYNC) {
    s = collect_failures(P, n_theta, st);
    if (s != MRA_OK) return s;
  }
  return copy_out(tuning_json(P, best), out_json, cap, len);
}

mra_status mra_profile(mra_plan_t P, int32_t enable) {
  if (!P) return MRA_EINVAL;
  if (!P->prof) {
    P->prof = new (std::nothrow) Profiler();
    if (!P->prof) return MRA_ENOMEM;
  }
  P->prof->enabled = enable != 0;
  P->prof->recs.clear();
  P->prof->used = 0;
  return MRA_OK;
}

mra_status mra_profile_read(mra_plan_t P, mra_phase_stat* out, int32_t cap, int32_t* count, void* stream) {
  if (!P || !count || (cap > 0 && !out)) return MRA_EINVAL;
  *count = 0;
  if (!P->prof) return MRA_OK;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MRA_EHIP;
  std::map<std::pair<std::string, int>, mra_phase_stat> agg;
  std::vector<std::pair<std::string, int>> order;
  for (const ProfRecord& r : P->prof->recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
      return MRA_EHIP;
    auto key = std::make_pair(std::string(r.name), r.level);
    auto it = agg.find(key);
    if (it == agg.end()) {
      mra_phase_stat s{};
      std::strncpy(s.name, r.name, sizeof(s.name) - 1);
      s.level = r.level;
      it = agg.emplace(key, s).first;
      order.push_back(key);
    }
    it->second.groups += 1;
    it->second.launches += r.launches;
    it->second.total_ms += ms;
    it->second.flops += r.flops;
  }
  int32_t k = 0;
  for (const auto& key : order) {
    if (k < cap) out[k] = agg[key];
    ++k;
  }
  *count = k;
  P->prof->recs.clear();
  P->prof->used = 0;
  return MRA_OK;
}

const char* mra_status_string(mra_status s) {
  switch (s) {
    case MRA_OK: return "ok";
    case MRA_EINVAL: return "invalid argument or configuration";
    case MRA_ENOTPD: return "Cholesky factor broke down (matrix not positive definite)";
    case MRA_ENOMEM: return "out of memory or arena too small";
    case MRA_EHIP: return "HIP runtime error";
    case MRA_ESTATE: return "plan not bound";
  }
  return "unknown status";
}

void mra_destroy(mra_plan_t P) {
  if (!P) return;
  if (P->side_stream) {
    (void)hipStreamSynchronize((hipStream_t)P->side_stream);
    (void)hipStreamDestroy((hipStream_t)P->side_stream);
  }
  for (void* ev : {P->ev_fork, P->ev_big, P->ev_fork2, P->ev_join, P->ev_join2, P->ev_gfork, P->ev_gath})
    if (ev) (void)hipEventDestroy((hipEvent_t)ev);
  if (P->graphs) {
    P->graphs->clear();
    if (P->graphs->cap) (void)hipStreamDestroy(P->graphs->cap);
    delete P->graphs;
  }
  delete P->prof;
  delete P;
}

}  // extern "C"
