// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer around the library's host code (plan builder,
// argument checks, tuning-table parser).  Touches no GPU: only entry points
// documented as host only are called, plus compute entries on plans that
// were never bound (they must refuse before any HIP call).
//
//   host_checks fuzz <iterations> <seed>
//       random plans (valid and invalid configurations, boundary and
//       duplicate locations, prediction points, explicit knots), geometry
//       invariants, argument checks, and a mutation fuzz of mra_set_tuning
//   host_checks geometry <in> <out>
//       one plan from a binary request (mra_config bytes, n, locations,
//       n_pred, prediction locations, knot count, knots); writes the status,
//       mra_info, arena sizes, permutation, leaf offsets and knots so that a
//       test can compare them with an independent implementation
//
// Exit status 0 when every check holds; a sanitizer report aborts.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mra.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what, int64_t it) {
  if (!ok) {
    std::fprintf(stderr, "CHECK FAILED: %s (iteration %lld)\n", what, (long long)it);
    ++g_fail;
  }
}

// splitmix64: deterministic stream for the fuzz inputs
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  int below(int k) { return (int)(next() % (uint64_t)k); }
};

// children and knots per level as the configuration resolves them
void levels(const mra_config& c, std::vector<int64_t>& nreg, std::vector<int>& rl) {
  nreg.assign(c.M + 1, 1);
  rl.assign(c.M, c.r);
  for (int m = 1; m <= c.M; ++m) nreg[m] = nreg[m - 1] * (c.J_level[m - 1] > 0 ? c.J_level[m - 1] : c.J);
  for (int m = 0; m < c.M; ++m) rl[m] = c.r_level[m] > 0 ? c.r_level[m] : c.r;
}

int64_t knot_doubles(const mra_config& c) {
  std::vector<int64_t> nreg;
  std::vector<int> rl;
  levels(c, nreg, rl);
  int64_t k = 0;
  for (int m = 0; m < c.M; ++m) k += nreg[m] * rl[m] * c.d;
  return k;
}

// every geometry output sized exactly, so that ASan sees any overrun
void geometry_invariants(mra_plan_t P, const mra_config& c, const std::vector<double>& locs, int64_t n,
                         int64_t it) {
  mra_info info;
  check(mra_get_info(P, &info) == MRA_OK, "get_info", it);
  std::vector<int64_t> nreg;
  std::vector<int> rl;
  levels(c, nreg, rl);
  check(info.n == n && info.n_leaves == nreg[c.M], "info sizes", it);
  int64_t nr = 0;
  for (int64_t v : nreg) nr += v;
  check(info.n_regions == nr, "info region count", it);
  size_t gb = 0, wb = 0;
  check(mra_requirements(P, &gb, &wb) == MRA_OK && gb > 0 && wb > 0, "requirements", it);
  std::vector<int64_t> perm(n), off(nreg[c.M] + 1);
  std::vector<double> kn(knot_doubles(c));
  check(mra_get_geometry(P, perm.data(), off.data(), kn.empty() ? nullptr : kn.data()) == MRA_OK, "get_geometry",
        it);
  check(mra_get_geometry(P, nullptr, nullptr, nullptr) == MRA_OK, "get_geometry null outputs", it);
  std::vector<char> seen(n, 0);
  bool okp = true;
  for (int64_t k = 0; k < n; ++k) {
    if (perm[k] < 0 || perm[k] >= n || seen[perm[k]]) { okp = false; break; }
    seen[perm[k]] = 1;
  }
  check(okp, "perm is a permutation", it);
  bool oko = off[0] == 0 && off[nreg[c.M]] == n;
  int64_t mx = 0;
  for (int64_t i = 0; i < nreg[c.M]; ++i) {
    oko = oko && off[i + 1] >= off[i];
    mx = off[i + 1] - off[i] > mx ? off[i + 1] - off[i] : mx;
  }
  check(oko, "leaf offsets monotone", it);
  check(info.max_leaf == mx, "max_leaf", it);
  bool okk = true;
  for (double v : kn) okk = okk && std::isfinite(v);
  check(okk, "knots finite", it);
  // leaf order keeps each leaf's points in their original relative order
  bool stable = true;
  for (int64_t i = 0; i < nreg[c.M]; ++i)
    for (int64_t k = off[i] + 1; k < off[i + 1]; ++k) stable = stable && perm[k - 1] < perm[k];
  check(stable, "stable leaf sort", it);
  (void)locs;
}

// compute calls on a plan that was never bound refuse before touching HIP
void unbound_calls(mra_plan_t P, int64_t it) {
  double dummy[4] = {0, 0, 0, 0};
  check(mra_loglik(P, dummy, dummy, 1, dummy, nullptr) == MRA_ESTATE, "loglik unbound", it);
  check(mra_loglik_grad(P, dummy, dummy, 1, dummy, dummy, nullptr) == MRA_ESTATE, "loglik_grad unbound", it);
  check(mra_loglik_grad_data(P, dummy, 0, dummy, 1, dummy, dummy, dummy, nullptr) == MRA_ESTATE,
        "loglik_grad_data unbound", it);
  check(mra_loglik_grad_noalloc(P, dummy, dummy, 1, dummy, dummy, nullptr) == MRA_ESTATE, "noalloc unbound", it);
  check(mra_gls(P, dummy, dummy, 1, dummy, dummy, dummy, dummy, dummy, dummy, nullptr) == MRA_ESTATE,
        "gls unbound", it);
  check(mra_predict(P, dummy, dummy, dummy, dummy, nullptr) == MRA_ESTATE, "predict unbound", it);
  check(mra_predict_cov(P, dummy, dummy, dummy, dummy, nullptr) == MRA_ESTATE, "predict_cov unbound", it);
  check(mra_simulate(P, dummy, dummy, dummy, 1 << 20, 1, dummy, nullptr) == MRA_ESTATE, "simulate unbound", it);
  check(mra_autotune(P, dummy, dummy, 1, dummy, dummy, 1, nullptr, 0, nullptr, nullptr) == MRA_ESTATE,
        "autotune unbound", it);
  int32_t th = 7, lv = 7;
  int64_t rg = 7;
  check(mra_last_failure(P, &th, &lv, &rg, nullptr) == MRA_OK && th == -1, "last_failure fresh", it);
  check(mra_profile(P, 1) == MRA_OK && mra_profile(P, 0) == MRA_OK, "profile toggle", it);
}

// null handles and null required pointers are refused
void null_arguments() {
  double dummy[4] = {0, 0, 0, 0};
  size_t a, b;
  mra_info info;
  mra_plan_t P = nullptr;
  check(mra_build(nullptr, dummy, 1, nullptr, 0, nullptr, &P) == MRA_EINVAL && P == nullptr, "build null cfg", -1);
  check(mra_requirements(nullptr, &a, &b) == MRA_EINVAL, "requirements null", -1);
  check(mra_get_info(nullptr, &info) == MRA_EINVAL, "info null", -1);
  check(mra_get_geometry(nullptr, nullptr, nullptr, nullptr) == MRA_EINVAL, "geometry null", -1);
  check(mra_bind(nullptr, dummy, 8, dummy, 8, nullptr) == MRA_EINVAL, "bind null", -1);
  check(mra_loglik(nullptr, dummy, dummy, 1, dummy, nullptr) == MRA_EINVAL, "loglik null", -1);
  check(mra_loglik_grad_noalloc(nullptr, dummy, dummy, 1, dummy, dummy, nullptr) == MRA_EINVAL, "noalloc null", -1);
  check(mra_get_tuning(nullptr, nullptr, 0, nullptr) == MRA_EINVAL, "get_tuning null", -1);
  check(mra_set_tuning(nullptr, "{}") == MRA_EINVAL, "set_tuning null", -1);
  check(mra_profile(nullptr, 1) == MRA_EINVAL, "profile null", -1);
  int32_t cnt;
  check(mra_profile_read(nullptr, nullptr, 0, &cnt, nullptr) == MRA_EINVAL, "profile_read null", -1);
  check(mra_last_failure(nullptr, nullptr, nullptr, nullptr, nullptr) == MRA_EINVAL, "last_failure null", -1);
  for (int s = -6; s <= 1; ++s) check(mra_status_string((mra_status)s) != nullptr, "status string", -1);
  mra_destroy(nullptr);
}

const char* kFamilies[] = {"prior", "leaf_rows", "leaf_sigma", "leaf_potrf", "leaf_trsm", "leaf_reduce",
                           "post", "post_reduce", "rleaf_v", "rleaf_linv", "rpost", "rleaf_q",
                           "rleaf_sbar", "rrows_leaf", "rT_leaf", "rprior", "rT", "predict"};
const char* kTokens[] = {"\"", ":", ",", "{", "}", " ", "-", "0", "7", "64", "65", "-1", "2147483648",
                         "4294967297", "99999999999999999999", "--3", "1-2", "\"identity\"", "\"grouped\"",
                         "\"chunked\"", "\"default\"", "\"bogus\"", "\"big_leaf_tiles\"", "\"side_solves\"",
                         "\"families\"", "\\", "\n", "\t"};

std::string get_tuning(mra_plan_t P, int64_t it) {
  size_t len = 0;
  check(mra_get_tuning(P, nullptr, 0, &len) == MRA_OK && len > 0, "get_tuning length", it);
  std::vector<char> buf(len + 1);
  check(mra_get_tuning(P, buf.data(), len, &len) == MRA_ENOMEM, "get_tuning short buffer", it);
  check(mra_get_tuning(P, buf.data(), buf.size(), &len) == MRA_OK, "get_tuning", it);
  return std::string(buf.data(), len);
}

// value of an integer key in the library's own output
long tuning_int(const std::string& j, const char* key) {
  const std::string k = std::string("\"") + key + "\": ";
  const size_t p = j.find(k);
  return p == std::string::npos ? -999 : std::strtol(j.c_str() + p + k.size(), nullptr, 10);
}

void fuzz_tuning(mra_plan_t P, Rng& g, int rounds, int64_t it) {
  const std::string base = get_tuning(P, it);
  for (int k = 0; k < rounds; ++k) {
    std::string s = base;
    const int edits = 1 + g.below(6);
    for (int e = 0; e < edits; ++e) {
      const int op = g.below(5);
      const size_t at = s.empty() ? 0 : (size_t)g.below((int)s.size() + 1);
      if (op == 0 && !s.empty()) {
        s.resize(at);                                                   // truncate
      } else if (op == 1) {
        s.insert(at, kTokens[g.below((int)(sizeof kTokens / sizeof *kTokens))]);
      } else if (op == 2 && at < s.size()) {
        s.erase(at, 1 + (size_t)g.below(8));
      } else if (op == 3 && at < s.size()) {
        s[at] = (char)(1 + g.below(255));                               // any non-zero byte
      } else {
        s.insert(at, std::string("\"") + kFamilies[g.below(18)] + "\": ");
      }
    }
    if (g.below(10) == 0) {   // a wholly random string
      s.clear();
      const int len = g.below(200);
      for (int q = 0; q < len; ++q) s += (char)(1 + g.below(255));
    }
    const mra_status st = mra_set_tuning(P, s.c_str());
    check(st == MRA_OK || st == MRA_EINVAL, "set_tuning status", it);
    const std::string now = get_tuning(P, it);
    const long big = tuning_int(now, "big_leaf_tiles"), side = tuning_int(now, "side_solves");
    check(big >= 0 && big <= 64 && side >= 0 && side <= 64, "tuning values in range", it);
    check(mra_set_tuning(P, now.c_str()) == MRA_OK && get_tuning(P, it) == now, "tuning round trip", it);
  }
  check(mra_set_tuning(P, base.c_str()) == MRA_OK, "restore tuning", it);
  // malformed or out-of-range integers are refused, never wrapped
  for (const char* bad : {"{\"big_leaf_tiles\": 4294967297}", "{\"big_leaf_tiles\": --3}",
                          "{\"side_solves\": 1-2}", "{\"side_solves\": 99999999999999999999}",
                          "{\"big_leaf_tiles\": 65}", "{\"side_solves\": -1}", "{\"big_leaf_tiles\": }",
                          "{\"leaf_rows\": \"identity}", "{\"post\": \"bogus\"}"})
    check(mra_set_tuning(P, bad) == MRA_EINVAL, bad, it);
  check(get_tuning(P, it) == base, "refused tables leave the tuning unchanged", it);
  check(mra_set_tuning(P, "{\"big_leaf_tiles\": 64, \"side_solves\": 0}") == MRA_OK &&
            tuning_int(get_tuning(P, it), "big_leaf_tiles") == 64,
        "in-range integers accepted", it);
  check(mra_set_tuning(P, base.c_str()) == MRA_OK, "restore tuning", it);
}

mra_config random_config(Rng& g) {
  mra_config c;
  std::memset(&c, 0, sizeof c);
  c.d = 1 + g.below(2);
  c.M = g.below(6);
  static const int j2[] = {1, 2, 4, 8, 16};
  c.J = c.d == 2 ? j2[g.below(4)] : 1 + g.below(16);
  static const int sq[] = {1, 4, 9, 16, 25, 36, 49, 64};
  c.r = c.d == 2 ? sq[g.below(8)] : 1 + g.below(64);
  for (int a = 0; a < 2; ++a) {
    c.lo[a] = g.below(3) == 0 ? -1.0 - g.uniform() : 0.0;
    c.hi[a] = c.lo[a] + 0.25 + 2.0 * g.uniform();
  }
  c.cov = g.below(2);
  c.max_theta = 1 + g.below(4);
  static const uint32_t fl[] = {MRA_SYNC, 0, MRA_SYNC | MRA_PLAIN, MRA_NO_GRAD, MRA_CHECKPOINT,
                                MRA_JOINT | MRA_SYNC, MRA_CHECKPOINT | MRA_JOINT};
  c.flags = fl[g.below(7)];
  c.chunks = g.below(12);
  if (g.below(2)) {   // level-dependent children and knots
    for (int m = 0; m < c.M; ++m) {
      c.J_level[m] = c.d == 2 ? j2[g.below(5)] : 1 + g.below(16);
      c.r_level[m] = c.d == 2 ? sq[g.below(8)] : 1 + g.below(64);
    }
  }
  c.adaptive = g.below(2);
  // at most 4096 leaves, so that an iteration stays small
  for (;;) {
    std::vector<int64_t> nreg;
    std::vector<int> rl;
    levels(c, nreg, rl);
    if (nreg[c.M] <= 4096) break;
    --c.M;
  }
  return c;
}

// configurations each of which must be refused
void invalid_configs(Rng& g, int64_t it) {
  double loc[2] = {0.5, 0.5};
  for (int k = 0; k < 19; ++k) {
    mra_config c;
    std::memset(&c, 0, sizeof c);
    c.d = 2; c.M = 2; c.J = 4; c.r = 16; c.hi[0] = c.hi[1] = 1.0; c.cov = 1; c.max_theta = 1; c.flags = MRA_SYNC;
    int64_t n = 1;
    switch (k) {
      case 0: c.d = 0; break;
      case 1: c.d = 3; break;
      case 2: c.M = -1; break;
      case 3: c.M = 12; break;
      case 4: c.J = 3; break;
      case 5: c.r = 15; break;
      case 6: c.r = 65; break;
      case 7: c.hi[0] = 0.0; break;
      case 8: c.lo[1] = NAN; break;
      case 9: c.max_theta = 0; break;
      case 10: c.flags = 64; break;
      case 11: c.chunks = -1; break;
      case 12: c.adaptive = 2; break;
      case 13: c.J_level[1] = 5; break;
      case 14: c.r_level[0] = 65; break;
      case 15: c.cov = 2; break;
      case 16: n = 0; break;
      case 17: loc[0] = 1.5; break;
      case 18: loc[0] = NAN; break;
    }
    mra_plan_t P = reinterpret_cast<mra_plan_t>(&c);   // overwritten with NULL on failure
    const mra_status s = mra_build(&c, loc, n, nullptr, 0, nullptr, &P);
    char what[64];
    std::snprintf(what, sizeof what, "invalid config %d refused", k);
    check(s == MRA_EINVAL && P == nullptr, what, it);
    if (s == MRA_OK) mra_destroy(P);
    loc[0] = 0.5;
  }
  // prediction points outside the box, non-finite explicit knots
  mra_config c;
  std::memset(&c, 0, sizeof c);
  c.d = 2; c.M = 1; c.J = 4; c.r = 4; c.hi[0] = c.hi[1] = 1.0; c.max_theta = 1;
  double pred[2] = {0.5, 2.0};
  mra_plan_t P = nullptr;
  check(mra_build(&c, loc, 1, pred, 1, nullptr, &P) == MRA_EINVAL, "pred outside box", it);
  check(mra_build(&c, loc, 1, nullptr, 1, nullptr, &P) == MRA_EINVAL, "pred null", it);
  double kn[8] = {0.1, 0.1, 0.2, 0.2, 0.3, NAN, 0.4, 0.4};
  check(mra_build(&c, loc, 1, nullptr, 0, kn, &P) == MRA_EINVAL, "non-finite knot", it);
  (void)g;
}

int run_fuzz(int64_t iters, uint64_t seed) {
  Rng g{seed};
  null_arguments();
  for (int64_t it = 0; it < iters; ++it) {
    mra_config c = random_config(g);
    int64_t n = 1 + g.below(g.below(4) == 0 ? 3000 : 200);
    std::vector<double> locs((size_t)n * c.d);
    const int mode = g.below(4);
    for (int64_t p = 0; p < n; ++p)
      for (int a = 0; a < c.d; ++a) {
        double u = g.uniform();
        if (mode == 1) u = u * u * u;                                        // clustered in a corner
        if (mode == 2) u = (double)g.below(5) / 4.0;                        // on split values and edges
        locs[p * c.d + a] = c.lo[a] + (c.hi[a] - c.lo[a]) * u;
      }
    if (mode == 3 && n > 4)
      for (int64_t p = 1; p < n / 2; ++p)
        for (int a = 0; a < c.d; ++a) locs[p * c.d + a] = locs[a];          // many duplicates
    int64_t n_pred = g.below(3) == 0 ? 0 : 1 + g.below(300);
    std::vector<double> pred((size_t)n_pred * c.d + 1);
    for (int64_t p = 0; p < n_pred; ++p)
      for (int a = 0; a < c.d; ++a) pred[p * c.d + a] = c.lo[a] + (c.hi[a] - c.lo[a]) * g.uniform();
    std::vector<double> kn;
    const bool explicit_knots = g.below(4) == 0;
    if (explicit_knots) {
      kn.resize(knot_doubles(c));
      for (double& v : kn) v = g.uniform();
    }
    // the plan builder may legitimately refuse a random configuration
    // (e.g. too many leaves); it must never read or write out of bounds
    mra_plan_t P = nullptr;
    const mra_status s = mra_build(&c, locs.data(), n, n_pred ? pred.data() : nullptr, n_pred,
                                   explicit_knots && !kn.empty() ? kn.data() : nullptr, &P);
    check(s == MRA_OK || s == MRA_EINVAL, "build status", it);
    if (s != MRA_OK) {
      check(P == nullptr, "failed build leaves no plan", it);
      continue;
    }
    geometry_invariants(P, c, locs, n, it);
    if (explicit_knots && !kn.empty()) {
      std::vector<double> got(kn.size());
      check(mra_get_geometry(P, nullptr, nullptr, got.data()) == MRA_OK &&
                std::memcmp(got.data(), kn.data(), kn.size() * sizeof(double)) == 0,
            "explicit knots round trip", it);
    }
    unbound_calls(P, it);
    if (it % 4 == 0) fuzz_tuning(P, g, 60, it);
    mra_destroy(P);
    if (it % 16 == 0) invalid_configs(g, it);
  }
  std::printf("fuzz: %lld iterations, %d failed checks\n", (long long)iters, g_fail);
  return g_fail == 0 ? 0 : 1;
}

int run_geometry(const char* in_path, const char* out_path) {
  FILE* f = std::fopen(in_path, "rb");
  if (!f) return 2;
  mra_config c;
  int64_t n = 0, n_pred = 0, nk = 0;
  bool ok = std::fread(&c, sizeof c, 1, f) == 1 && std::fread(&n, 8, 1, f) == 1 && n >= 0 && n < (1ll << 32);
  std::vector<double> locs, pred, kn;
  if (ok) {
    locs.resize((size_t)n * c.d + 1);
    ok = std::fread(locs.data(), 8, (size_t)n * c.d, f) == (size_t)n * c.d && std::fread(&n_pred, 8, 1, f) == 1 &&
         n_pred >= 0 && n_pred < (1ll << 32);
  }
  if (ok) {
    pred.resize((size_t)n_pred * c.d + 1);
    ok = std::fread(pred.data(), 8, (size_t)n_pred * c.d, f) == (size_t)n_pred * c.d &&
         std::fread(&nk, 8, 1, f) == 1 && nk >= 0 && nk < (1ll << 32);
  }
  if (ok) {
    kn.resize((size_t)nk + 1);
    ok = std::fread(kn.data(), 8, (size_t)nk, f) == (size_t)nk;
  }
  std::fclose(f);
  if (!ok) return 2;
  // exact-size copies of the inputs, so that ASan sees any overrun
  std::vector<double> L(locs.begin(), locs.begin() + n * c.d), Q(pred.begin(), pred.begin() + n_pred * c.d),
      K(kn.begin(), kn.begin() + nk);
  mra_plan_t P = nullptr;
  const mra_status s = mra_build(&c, L.data(), n, n_pred ? Q.data() : nullptr, n_pred, nk ? K.data() : nullptr, &P);
  FILE* o = std::fopen(out_path, "wb");
  if (!o) return 2;
  const int32_t st = s;
  std::fwrite(&st, 4, 1, o);
  if (s == MRA_OK) {
    mra_info info;
    size_t gb = 0, wb = 0;
    mra_get_info(P, &info);
    mra_requirements(P, &gb, &wb);
    std::vector<int64_t> perm(n), off(info.n_leaves + 1);
    std::vector<double> knots(knot_doubles(c));
    mra_get_geometry(P, perm.data(), off.data(), knots.data());
    geometry_invariants(P, c, L, n, 0);
    unbound_calls(P, 0);
    std::fwrite(&info, sizeof info, 1, o);
    const uint64_t sz[2] = {gb, wb};
    std::fwrite(sz, 8, 2, o);
    std::fwrite(perm.data(), 8, perm.size(), o);
    std::fwrite(off.data(), 8, off.size(), o);
    std::fwrite(knots.data(), 8, knots.size(), o);
    std::string t = get_tuning(P, 0);
    std::fwrite(t.data(), 1, t.size(), o);
    mra_destroy(P);
  }
  std::fclose(o);
  return g_fail == 0 ? 0 : 1;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc == 4 && std::strcmp(argv[1], "fuzz") == 0)
    return run_fuzz(std::atoll(argv[2]), (uint64_t)std::strtoull(argv[3], nullptr, 10));
  if (argc == 4 && std::strcmp(argv[1], "geometry") == 0) return run_geometry(argv[2], argv[3]);
  std::fprintf(stderr, "usage: host_checks fuzz <iterations> <seed> | geometry <in> <out>\n");
  return 2;
}
