// Host-side checks of liblbkt's C ABI and planning code, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py).
// Exercises everything that runs on the CPU before a launch: validation of random
// and extreme grids, the per-grid constants, the moving-shock cell count, the
// batch work lists, the tile and partition arithmetic, and the early error returns
// of the entry points. Makes no HIP call that reaches a device.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/lbkt.h"
#include "../../paper_0706_0405_amd/csrc/lbkt_internal.hpp"

static int g_fail = 0;
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::fprintf(stderr, "CHECK failed: %s: ", #cond);  \
      std::fprintf(stderr, __VA_ARGS__);                  \
      std::fprintf(stderr, "\n");                         \
      if (++g_fail > 20) std::exit(1);                    \
    }                                                     \
  } while (0)

// xorshift64*: a small seeded generator for the fuzzed fields
struct Rng {
  uint64_t s;
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 2685821657736338717ull;
  }
  double uni() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  int pick(int n) { return (int)(next() % (uint64_t)n); }
};

static const double kNaN = std::numeric_limits<double>::quiet_NaN();
static const double kInf = std::numeric_limits<double>::infinity();

static double odd_double(Rng& r, double lo, double hi) {
  switch (r.pick(12)) {
    case 0: return kNaN;
    case 1: return kInf;
    case 2: return -kInf;
    case 3: return 0.0;
    case 4: return -1.0;
    case 5: return 1e308;
    case 6: return 4.9e-324;
    default: return lo + (hi - lo) * r.uni();
  }
}

static int32_t odd_int(Rng& r, int32_t lo, int32_t hi) {
  switch (r.pick(10)) {
    case 0: return -1;
    case 1: return 0;
    case 2: return INT32_MAX;
    case 3: return INT32_MIN;
    case 4: return 1;
    default: return lo + (int32_t)(r.next() % (uint64_t)(hi - lo + 1));
  }
}

static lb_state random_state(Rng& r, bool odd) {
  lb_state s;
  s.rho = odd ? odd_double(r, 0.1, 10.0) : 0.1 + 10.0 * r.uni();
  s.ux = odd ? odd_double(r, -5.0, 5.0) : -5.0 + 10.0 * r.uni();
  s.uy = odd ? odd_double(r, -5.0, 5.0) : -5.0 + 10.0 * r.uni();
  s.p = odd ? odd_double(r, 0.1, 10.0) : 0.1 + 10.0 * r.uni();
  return s;
}

// A grid whose fields are mostly sensible; with `odd`, any field may be extreme.
static lb_grid random_grid(Rng& r, bool odd) {
  lb_grid g;
  std::memset(&g, 0, sizeof(g));
  g.nx = odd ? odd_int(r, 1, 5000) : 1 + r.pick(5000);
  g.ny = odd ? odd_int(r, 1, 5000) : 1 + r.pick(5000);
  const int64_t up = ((int64_t)std::max(g.nx, 0) + 63) / 64 * 64;
  const int64_t pitches[6] = {up, up + 64, (int64_t)g.nx, 0, -64, ((int64_t)1 << 27) + 64};
  g.pitch = odd ? pitches[r.pick(6)] : std::max<int64_t>(up, 64);
  g.dx = odd ? odd_double(r, 1e-4, 1.0) : 1e-4 + r.uni();
  g.dt = odd ? odd_double(r, 1e-6, 1e-2) : 1e-6 + 1e-2 * r.uni();
  g.c1 = odd ? odd_double(r, 0.5, 30.0) : 0.5 + 30.0 * r.uni();
  g.c2 = r.pick(20) == 0 ? g.c1 : (odd ? odd_double(r, 1.0, 90.0) : g.c1 * (1.5 + 2.0 * r.uni()));
  g.eta0 = odd ? odd_double(r, 0.5, 60.0) : g.c1 * (1.0 + r.uni());
  g.gamma = odd ? odd_double(r, 1.0, 2.0) : 1.1 + 0.6 * r.uni();
  g.tau = odd ? odd_double(r, 0.5, 3.0) : 0.5 + 2.5 * r.uni();
  g.beta = odd ? odd_double(r, -0.1, 0.6) : 0.5 * r.uni();
  lb_default_lambda(&g);
  if (odd && r.pick(4) == 0) g.lambda[r.pick(9)] = odd_double(r, 0.0, 1.0);
  for (int e = 0; e < 4; ++e) {
    lb_edge& E = g.edge[e];
    const int kinds[8] = {0, 1, 2, 3, 4, -1, 5, 1000};
    E.kind = odd ? kinds[r.pick(8)] : (e < 2 ? r.pick(4) : r.pick(5));
    E.split = odd ? odd_int(r, 0, 10) : (r.pick(3) == 0 ? r.pick(10) : 0);
    E.a = random_state(r, odd);
    E.b = random_state(r, odd);
    E.x0 = odd ? odd_double(r, -1.0, 1.0) : r.uni();
    const double angles[6] = {60.0, 90.0, 30.0, 1e-300, 180.0, 0.0};
    E.angle_deg = odd ? (r.pick(3) ? odd_double(r, 1.0, 179.0) : angles[r.pick(6)]) : 20.0 + 140.0 * r.uni();
    E.speed = odd ? odd_double(r, -20.0, 20.0) : 20.0 * r.uni();
  }
  if (!odd) {   // periodic axes come in pairs
    if ((g.edge[0].kind == LB_BC_PERIODIC) != (g.edge[1].kind == LB_BC_PERIODIC)) g.edge[1].kind = g.edge[0].kind;
    if ((g.edge[2].kind == LB_BC_PERIODIC) != (g.edge[3].kind == LB_BC_PERIODIC)) g.edge[3].kind = g.edge[2].kind;
    for (int e = 0; e < 4; ++e)
      if (g.edge[e].kind == LB_BC_PERIODIC) g.edge[e].split = 0;
  }
  return g;
}

static bool pos(double v) { return std::isfinite(v) && v > 0.0; }

// The documented constraints of a valid grid, checked independently of lb_validate.
static bool documented_valid(const lb_grid& g) {
  if (g.nx < 1 || g.ny < 1 || g.pitch < g.nx || g.pitch % 64 != 0 || g.pitch > ((int64_t)1 << 27)) return false;
  if (!pos(g.dx) || !pos(g.dt) || !pos(g.c1) || !pos(g.c2) || !pos(g.eta0) || g.c1 == g.c2 || !pos(g.tau)) return false;
  if (!(g.beta >= 0.0 && g.beta <= 0.5) || !(std::isfinite(g.gamma) && g.gamma > 1.0)) return false;
  for (int i = 0; i < 9; ++i)
    if (!(std::isfinite(g.lambda[i]) && g.lambda[i] >= 0.0)) return false;
  for (int i = 2; i <= 4; ++i)
    if (g.lambda[i] != g.lambda[1]) return false;
  for (int i = 6; i <= 8; ++i)
    if (g.lambda[i] != g.lambda[5]) return false;
  for (int e = 0; e < 4; ++e) {
    const lb_edge& E = g.edge[e];
    if (E.kind < 0 || E.kind > 4 || E.split < 0 || (E.kind == LB_BC_SHOCK && e < 2)) return false;
    auto ok = [](const lb_state& s) { return pos(s.rho) && pos(s.p) && std::isfinite(s.ux) && std::isfinite(s.uy); };
    if ((E.kind == LB_BC_INFLOW || E.kind == LB_BC_SHOCK || E.split > 0) && !ok(E.a)) return false;
    if (E.kind == LB_BC_SHOCK) {
      const double a = E.angle_deg * (M_PI / 180.0);
      if (!ok(E.b) || !std::isfinite(a) || std::sin(a) == 0.0 || std::tan(a) == 0.0 || !std::isfinite(E.x0) ||
          !std::isfinite(E.speed))
        return false;
    }
  }
  for (int ax = 0; ax < 2; ++ax) {
    const bool p0 = g.edge[2 * ax].kind == LB_BC_PERIODIC, p1 = g.edge[2 * ax + 1].kind == LB_BC_PERIODIC;
    if (p0 != p1) return false;
    if ((p0 && g.edge[2 * ax].split) || (p1 && g.edge[2 * ax + 1].split)) return false;
  }
  return true;
}

static void check_validate(Rng& r, int n) {
  int nvalid = 0;
  for (int k = 0; k < n; ++k) {
    const bool odd = (k % 2) == 1;
    lb_grid g = random_grid(r, odd);
    const lb_status s = lb_validate(&g);
    CHECK((s == LB_OK) == documented_valid(g), "grid %d: lb_validate %d (%s)", k, (int)s, lb_last_error());
    CHECK(s == LB_OK || std::strlen(lb_last_error()) > 0, "grid %d: an error without detail text", k);
    if (s != LB_OK) continue;
    ++nvalid;
    lbkt::KTConsts K;
    lbkt_build_consts(&g, &K);
    CHECK(K.nx == g.nx && K.ny == g.ny && K.pitch == g.pitch && K.plane == g.pitch * (int64_t)g.ny, "grid %d sizes", k);
    if (!odd) {   // moderate parameters: every constant is finite
      const double v[] = {K.wc0, K.l0, K.wca, K.upa, K.dna, K.la, K.wcd, K.upd, K.dnd, K.ld, K.inv_tau, K.s,
                          K.a0T, K.k1u, K.k1T, K.r1d, K.k5u, K.k5T, K.r5d, K.rb1d, K.rb5d, K.d1, K.d5};
      for (double x : v) CHECK(std::isfinite(x), "grid %d: a constant is not finite", k);
      for (int e = 0; e < 4; ++e)
        for (int i = 0; i < 9; ++i) CHECK(std::isfinite(K.ga[e][i]) && std::isfinite(K.gb[e][i]), "grid %d ghosts", k);
    }
    int64_t elems = lb_array_elems(&g);
    CHECK(elems == 9 * g.pitch * (int64_t)g.ny, "grid %d elems", k);
    int rpb = 0, nb = 0;
    lbkt_inv_partition(&g, &rpb, &nb);
    CHECK(nb >= 1 && nb <= LBKT_INV_MAX_PARTS && rpb >= 1 && (int64_t)rpb * nb >= g.ny &&
              (int64_t)rpb * (nb - 1) < g.ny,
          "grid %d: partition %d x %d of %d rows", k, nb, rpb, g.ny);
    int bx = 0, rows = 0;
    lbkt_default_tile2(g.nx, g.ny, (k & 2) ? LB_F32 : LB_F64, &bx, &rows);
    CHECK((bx == 64 || bx == 128 || bx == 256) && rows >= 1 && rows <= g.ny, "grid %d tile %d x %d", k, bx, rows);
    // moving-shock cells against the predicate, cell by cell
    for (int e = 2; e < 4; ++e) {
      if (g.edge[e].kind != LB_BC_SHOCK) continue;
      const int64_t steps[5] = {0, 1, 977, (int64_t)1 << 31, -5};
      for (int64_t st : steps) {
        const int n = lbkt_shock_cells(&g, e, st);
        CHECK(n >= 0 && n <= g.nx, "grid %d: %d shock cells", k, n);
        if (g.nx <= 5000) {
          const lb_edge& E = g.edge[e];
          const double yg = (e == 2 ? -0.5 : g.ny + 0.5) * g.dx;
          const double ang = E.angle_deg * (M_PI / 180.0);
          const double xs = E.x0 + yg / std::tan(ang) + E.speed * ((double)st * g.dt) / std::sin(ang);
          int want = 0;
          for (int i = 0; i < g.nx; ++i) want += ((i + 0.5) * g.dx < xs) ? 1 : 0;
          CHECK(n == want, "grid %d edge %d step %lld: %d shock cells, predicate %d", k, e, (long long)st, n, want);
        }
      }
    }
  }
  std::printf("lb_validate: %d grids, %d valid\n", n, nvalid);
}

static void check_batch_plan(Rng& r, int nbatches) {
  for (int k = 0; k < nbatches; ++k) {
    const int n = 1 + r.pick(300);
    std::vector<lb_grid> grids(n);
    for (auto& g : grids) {
      g = random_grid(r, false);
      g.nx = 1 + r.pick(r.pick(4) == 0 ? 20000 : 300);
      g.ny = 1 + r.pick(8);
    }
    for (int bx : {64, 128, 256}) {
      std::vector<LbktWorkItem> a, b;
      lbkt_plan_batch(grids.data(), n, bx, &a, &b);
      std::vector<int> seen1(n, 0), seen2(n, 0);
      std::vector<std::vector<int>> hit2(n);
      for (const auto& w : a) {
        CHECK(w.prob >= 0 && w.prob < n && w.strip >= 0 && (int64_t)w.strip * bx < grids[w.prob].nx, "one-step item");
        if (w.prob >= 0 && w.prob < n) ++seen1[w.prob];
      }
      for (const auto& w : b) {
        const int wpb = bx / 64;
        CHECK(w.prob >= 0 && w.prob < n && w.strip >= 0 && (int64_t)w.strip * wpb * 60 < grids[w.prob].nx,
              "two-step item");
        if (w.prob >= 0 && w.prob < n) hit2[w.prob].push_back(w.strip);
      }
      for (int p = 0; p < n; ++p) {
        const int ns = (grids[p].nx + bx - 1) / bx;
        const int ns2 = ((grids[p].nx + 59) / 60 + bx / 64 - 1) / (bx / 64);
        CHECK(seen1[p] == ns, "problem %d: %d of %d one-step strips", p, seen1[p], ns);
        std::vector<int> h = hit2[p];
        std::vector<int> cnt(ns2, 0);
        for (int s : h)
          if (s >= 0 && s < ns2) ++cnt[s];
        bool once = (int)h.size() == ns2;
        for (int c : cnt) once = once && c == 1;
        CHECK(once, "problem %d: two-step strips not covered exactly once", p);
      }
      // neighbours of the two-step items: the adjacent strips of the same problem
      // (wrapped for a periodic x axis), symmetric, -1 at a non-periodic end
      for (auto& g : grids) g.edge[1].kind = g.edge[0].kind = (r.pick(2) ? LB_BC_PERIODIC : LB_BC_OUTFLOW);
      std::vector<int> left, right;
      lbkt_batch_neighbours(grids.data(), b, bx, &left, &right);
      CHECK(left.size() == b.size() && right.size() == b.size(), "neighbour list sizes");
      for (size_t i = 0; i < b.size() && left.size() == b.size(); ++i) {
        const auto& w = b[i];
        const int ns = ((grids[w.prob].nx + 59) / 60 + bx / 64 - 1) / (bx / 64);
        const bool per = grids[w.prob].edge[0].kind == LB_BC_PERIODIC;
        const int want_l = w.strip > 0 ? w.strip - 1 : (per && ns > 1 ? ns - 1 : -1);
        const int want_r = w.strip + 1 < ns ? w.strip + 1 : (per && ns > 1 ? 0 : -1);
        for (int side = 0; side < 2; ++side) {
          const int j = side ? right[i] : left[i];
          const int want = side ? want_r : want_l;
          if (want < 0 || want == w.strip) {
            CHECK(j == -1, "item %zu: unexpected neighbour", i);
          } else {
            CHECK(j >= 0 && j < (int)b.size() && b[j].prob == w.prob && b[j].strip == want, "item %zu neighbour", i);
            if (j >= 0 && j < (int)b.size()) CHECK((side ? left[j] : right[j]) == (int)i, "item %zu: not symmetric", i);
          }
        }
      }
      for (int depth : {4, 6, 8}) {   // deep passes: strips of 64 - 2 depth columns, each once
        std::vector<LbktWorkItem> d;
        lbkt_plan_batch_deep(grids.data(), n, bx, depth, &d);
        const int w = 64 - 2 * depth, wpb = bx / 64;
        std::vector<std::vector<int>> hit(n);
        for (const auto& it : d) {
          CHECK(it.prob >= 0 && it.prob < n && it.strip >= 0 && (int64_t)it.strip * wpb * w < grids[it.prob].nx,
                "deep item (depth %d)", depth);
          if (it.prob >= 0 && it.prob < n) hit[it.prob].push_back(it.strip);
        }
        for (int p = 0; p < n; ++p) {
          const int ns = ((grids[p].nx + w - 1) / w + wpb - 1) / wpb;
          std::vector<int> cnt(ns, 0);
          for (int s : hit[p])
            if (s >= 0 && s < ns) ++cnt[s];
          bool once = (int)hit[p].size() == ns;
          for (int c : cnt) once = once && c == 1;
          CHECK(once, "problem %d: depth-%d strips not covered exactly once", p, depth);
        }
      }
      for (size_t i = 1; i < a.size(); ++i) {   // one-step list: longest problems first
        const int64_t s0 = (int64_t)grids[a[i - 1].prob].nx * grids[a[i - 1].prob].ny;
        const int64_t s1 = (int64_t)grids[a[i].prob].nx * grids[a[i].prob].ny;
        CHECK(s0 >= s1, "one-step list not longest first");
      }
    }
  }
  std::printf("lbkt_plan_batch: %d batches\n", nbatches);
}

static void check_early_errors() {
  lb_grid g;
  std::memset(&g, 0, sizeof(g));
  g.nx = 100; g.ny = 4; g.pitch = 128; g.dx = 0.01; g.dt = 1e-4; g.c1 = 1; g.c2 = 3; g.eta0 = 2; g.gamma = 1.4;
  g.tau = 1; g.beta = 0.25;
  lb_default_lambda(&g);
  CHECK(lb_validate(&g) == LB_OK, "base grid");
  void* a = (void*)(uintptr_t)(1 << 20);
  void* b = (void*)(uintptr_t)(1 << 30);
  void* mis = (void*)(uintptr_t)((1 << 20) + 8);
  CHECK(lb_validate(nullptr) == LB_EINVAL, "NULL grid");
  CHECK(lb_default_lambda(nullptr) == LB_EINVAL, "NULL grid");
  CHECK(lb_array_elems(nullptr) == 0, "NULL grid elems");
  CHECK(lb_step(&g, LB_F64, a, a, 0, nullptr) == LB_EALIAS, "alias");
  CHECK(lb_step(&g, LB_F64, mis, b, 0, nullptr) == LB_EINVAL, "alignment");
  CHECK(lb_step(&g, (lb_prec)7, a, b, 0, nullptr) == LB_EINVAL, "precision");
  CHECK(lb_run(&g, LB_F32, a, b, 0, -1, 0, nullptr, nullptr) == LB_EINVAL, "nsteps");
  lb_tile t = {96, 4, 0, 0};
  CHECK(lb_run(&g, LB_F32, a, b, 0, 4, 0, &t, nullptr) == LB_EINVAL, "tile width");
  t = {256, 4, 0, 4};
  CHECK(lb_run(&g, LB_F32, a, b, 0, 4, 0, &t, nullptr) == LB_EINVAL, "tile steps");
  t = {256, 4, 0, 3};   // three steps per pass: FP64 arrays only
  CHECK(lb_run(&g, LB_F32, a, b, 0, 4, 0, &t, nullptr) == LB_EUNSUPPORTED, "three steps on FP32");
  CHECK(lb_init(&g, LB_F64, nullptr, nullptr, nullptr, nullptr, a, nullptr) == LB_EINVAL, "init fields");
  CHECK(lb_moments(&g, LB_F64, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LB_EINVAL, "moments f");
  CHECK(lb_invariants(&g, LB_F64, a, nullptr, nullptr) == LB_EINVAL, "invariants out");
  CHECK(lb_invariants_noalloc(&g, LB_F64, a, nullptr, nullptr) == LB_EINVAL, "noalloc out");
  CHECK(lb_step_adjoint(&g, LB_F64, a, (const double*)b, (double*)b, 0, nullptr) == LB_EALIAS, "adjoint alias");
  CHECK(lb_check_flags(nullptr, nullptr, nullptr) == LB_EINVAL, "flags NULL");
  void* outs[3] = {b, b, a};
  CHECK(lb_run_record(&g, LB_F64, a, outs, 0, 3, nullptr) == LB_EALIAS, "record alias");
  lb_batch* batch = nullptr;
  CHECK(lb_batch_create(0, &g, LB_F32, &batch) == LB_EINVAL && batch == nullptr, "empty batch");
  CHECK(lb_step_batched(nullptr, a, b, 2, nullptr) == LB_EINVAL, "NULL batch");
  lb_vn_case c;
  std::memset(&c, 0, sizeof(c));
  double kd[4] = {0, 1, 2, 3};
  double out[4];
  CHECK(lb_vn_scan(&c, 0, kd, kd, 4, 0, out, nullptr) == LB_EINVAL, "vn ncases");
  CHECK(lb_vn_scan(&c, 1, kd, kd, 4, 0, out, nullptr) == LB_EPARAM, "vn case");
  for (int s = -10; s <= 2; ++s) CHECK(lb_status_str((lb_status)s) != nullptr, "status string");
  for (int w = -3; w <= 8; ++w) CHECK((lb_struct_size(w) > 0) == (w >= 0 && w <= 4), "struct size %d", w);
  std::printf("early errors: ok\n");
}

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 20000;
  Rng r{0x9E3779B97F4A7C15ull};
  check_validate(r, n);
  check_batch_plan(r, 60);
  check_early_errors();
  if (g_fail) {
    std::printf("FAILED: %d checks\n", g_fail);
    return 1;
  }
  std::printf("all host checks passed\n");
  return 0;
}
