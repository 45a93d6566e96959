// Driver of the bounds-checked CPU build: runs the C ABI through every entry point on
// the scenarios read from stdin, with every launch checked by launch_check.cpp, under
// AddressSanitizer and UndefinedBehaviorSanitizer (host code only: there is no device
// code in this build).  Exit status 0 when every call returned what it should and no
// check failed.
//
// Input, per scenario (whitespace separated):
//   scenario <name> <precision 0|1> <s> <n>
//   a_ex (s x s) b_ex (s) a_im (s x s) b_im (s)
//   n lines: nx ny eps mach tau dt weno_order central_order
#include "apdvm.h"
#include "common.hpp"
#include "hostcheck.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iostream>
#include <string>
#include <vector>

namespace {

int g_bad = 0;

void expect(apdvm_status got, apdvm_status want, const char *call, const std::string &where) {
  if (got != want) {
    ++g_bad;
    std::fprintf(stderr, "hostcheck: %s: %s returned %d (%s), expected %d\n", where.c_str(),
                 call, (int)got, apdvm_status_string(got), (int)want);
  }
}
#define CALL(expr, want) expect((expr), (want), #expr, name)

struct Scenario {
  std::string name;
  int precision = 0, s = 0, n = 0;
  std::vector<double> at, bt, a, b;
  std::vector<apdvm_config> cfg;
};

bool read_scenario(std::istream &in, Scenario &sc) {
  std::string tag;
  if (!(in >> tag)) return false;
  if (tag != "scenario") {
    std::fprintf(stderr, "hostcheck: bad input near '%s'\n", tag.c_str());
    std::exit(2);
  }
  in >> sc.name >> sc.precision >> sc.s >> sc.n;
  const int s = sc.s;
  sc.at.resize(s * s);
  sc.bt.resize(s);
  sc.a.resize(s * s);
  sc.b.resize(s);
  for (auto *v : {&sc.at, &sc.bt, &sc.a, &sc.b})
    for (double &x : *v) in >> x;
  sc.cfg.resize(sc.n);
  for (auto &c : sc.cfg) {
    c = apdvm_config{};
    in >> c.nx >> c.ny >> c.eps >> c.mach >> c.tau >> c.dt >> c.weno_order >> c.central_order;
    c.lx = c.ly = 2.0 * M_PI;
    c.q = 6;
    c.s = s;
    c.a_ex = sc.at.data();
    c.b_ex = sc.bt.data();
    c.a_im = sc.a.data();
    c.b_im = sc.b.data();
    c.cfl = 0.25;
    c.c_visc = 0.2;
    c.precision = sc.precision;
  }
  return bool(in);
}

// Smooth fields of instance k: a divergence-free velocity of two modes, theta of one.
std::vector<std::vector<double>> fields(const apdvm_config &c, int k) {
  std::vector<std::vector<double>> f(6, std::vector<double>((size_t)c.nx * c.ny, 0.0));
  for (int y = 0; y < c.ny; ++y)
    for (int x = 0; x < c.nx; ++x) {
      const double X = (x + 0.5) * c.lx / c.nx, Y = (y + 0.5) * c.ly / c.ny;
      const size_t i = (size_t)y * c.nx + x;
      f[0][i] = 0.1 * std::sin(X + 0.3 * k) * std::cos(Y);
      f[1][i] = -0.1 * std::cos(X + 0.3 * k) * std::sin(Y);
      f[2][i] = 0.01 * std::cos(X) * std::cos(2.0 * Y);
      f[3][i] = 0.5 * (f[1][i] * f[1][i] - f[0][i] * f[0][i]);
      f[4][i] = f[0][i] * f[1][i];
    }
  return f;
}

void run(const Scenario &sc) {
  const std::string &name = sc.name;
  const int n = sc.n;
  const apdvm_config *cfg = sc.cfg.data();
  size_t bytes = 0;
  CALL(apdvm_workspace_bytes(n, cfg, &bytes), APDVM_OK);

  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) ++g_bad;
  apdvm_ctx *c = nullptr;
  CALL(apdvm_create(n, cfg, nullptr, 0, st, &c), APDVM_OK);
  if (!c) return;
  CALL(apdvm_step(c, 1), APDVM_ERR_STATE);  // no fields yet
  std::vector<std::vector<std::vector<double>>> F(n);
  for (int k = 0; k < n; ++k) {
    F[k] = fields(cfg[k], k);
    auto &f = F[k];
    CALL(apdvm_set_fields(c, k, f[0].data(), f[1].data(), f[2].data(), nullptr, nullptr, nullptr),
         APDVM_OK);
  }
  {  // a NaN is rejected and changes nothing
    auto f = F[0];
    f[2][3] = NAN;
    CALL(apdvm_set_fields(c, 0, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(),
                          f[5].data()),
         APDVM_ERR_NONFINITE);
  }
  CALL(apdvm_set_fields(c, n, F[0][0].data(), F[0][1].data(), F[0][2].data(), nullptr, nullptr,
                        nullptr),
       APDVM_ERR_ARG);
  int32_t nl = 0;
  CALL(apdvm_launches_per_step(c, &nl), APDVM_OK);
  CALL(apdvm_step(c, 2), APDVM_OK);
  CALL(apdvm_set_overlap(c, 0), APDVM_OK);
  CALL(apdvm_step(c, 1), APDVM_OK);
  CALL(apdvm_set_overlap(c, 2), APDVM_OK);  // fused schedule
  CALL(apdvm_step(c, 2), APDVM_OK);
  CALL(apdvm_set_overlap(c, 3), APDVM_ERR_ARG);
  CALL(apdvm_set_overlap(c, 1), APDVM_OK);
  int32_t ov = -1;
  CALL(apdvm_get_overlap(c, &ov), APDVM_OK);
  CALL(apdvm_set_graph(c, 1), APDVM_OK);
  CALL(apdvm_step(c, 3), APDVM_OK);  // both parities captured, then replayed
  CALL(apdvm_set_overlap(c, 0), APDVM_OK);
  CALL(apdvm_step(c, 2), APDVM_OK);  // graphs of the other stream structures
  CALL(apdvm_set_overlap(c, 2), APDVM_OK);
  CALL(apdvm_step(c, 3), APDVM_OK);
  CALL(apdvm_set_overlap(c, 1), APDVM_OK);
  for (int cls = 0; cls < APDVM_NUM_KERNEL_CLASSES; ++cls) {
    CALL(apdvm_timing_enable(c, cls), APDVM_OK);
    CALL(apdvm_timing_stride(c, cls % 2 + 1), APDVM_OK);
    CALL(apdvm_step(c, 2), APDVM_OK);
    int64_t l = 0;
    double ms = 0.0;
    CALL(apdvm_timing_read(c, &l, &ms), APDVM_OK);
    double b = 0.0;
    int32_t nlc = 0;
    CALL(apdvm_traffic(c, cls, &b, &nlc), APDVM_OK);
  }
  CALL(apdvm_timing_enable(c, -1), APDVM_OK);
  CALL(apdvm_timing_stride(c, 1), APDVM_OK);
  CALL(apdvm_set_finite_check(c, 1), APDVM_OK);
  CALL(apdvm_step(c, 2), APDVM_OK);
  CALL(apdvm_set_finite_check(c, 64), APDVM_OK);
  int32_t choice[APDVM_TUNING_LEN] = {0};
  CALL(apdvm_autotune(c, 1, choice), APDVM_OK);
  CALL(apdvm_set_tuning(c, choice), APDVM_OK);
  CALL(apdvm_step(c, 1), APDVM_OK);
  double *dev_out = nullptr;
  if (hipMalloc(&dev_out, 8 * sizeof(double)) != hipSuccess) ++g_bad;
  for (int k = 0; k < n; ++k) {
    const apdvm_config &cf = cfg[k];
    const size_t N = (size_t)cf.nx * cf.ny;
    double d[8];
    CALL(apdvm_diagnostics(c, k, d), APDVM_OK);
    CALL(apdvm_diagnostics_device(c, k, dev_out), APDVM_OK);
    std::vector<std::vector<double>> g(6, std::vector<double>(N));
    CALL(apdvm_get_fields(c, k, g[0].data(), g[1].data(), g[2].data(), g[3].data(), g[4].data(),
                          g[5].data()),
         APDVM_OK);
    std::vector<double> m(4 * N), P(6 * N);
    CALL(apdvm_get_moments(c, k, m.data(), m.data() + N, m.data() + 2 * N, m.data() + 3 * N),
         APDVM_OK);
    if (cf.eps > 0.0) {
      CALL(apdvm_get_populations(c, k, P.data()), APDVM_OK);
      CALL(apdvm_set_populations(c, k, P.data()), APDVM_OK);
    }
    double dt = 0.0, tau = 0.0;
    int64_t step = 0;
    CALL(apdvm_get_info(c, k, &dt, &tau, &step), APDVM_OK);
    // device hand-over
    double *dev[6];
    for (int i = 0; i < 6; ++i) {
      if (hipMalloc(&dev[i], N * sizeof(double)) != hipSuccess) ++g_bad;
      hipMemcpyAsync(dev[i], g[i].data(), N * sizeof(double), hipMemcpyHostToDevice, nullptr);
    }
    CALL(apdvm_set_fields_device(c, k, dev), APDVM_OK);
    CALL(apdvm_get_fields_device(c, k, dev), APDVM_OK);
    for (int i = 0; i < 6; ++i) hipFree(dev[i]);
  }
  CALL(apdvm_diagnostics(c, n, nullptr), APDVM_ERR_ARG);
  CALL(apdvm_set_step(c, 10), APDVM_OK);
  CALL(apdvm_step(c, 1), APDVM_OK);
  CALL(apdvm_set_graph(c, 0), APDVM_OK);
  CALL(apdvm_step(c, 1), APDVM_OK);
  hipFree(dev_out);
  apdvm_destroy(c);

  // caller-provided workspace, default stream; then one too small
  void *ws = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) ++g_bad;
  c = nullptr;
  CALL(apdvm_create(n, cfg, ws, bytes, nullptr, &c), APDVM_OK);
  if (c) {
    for (int k = 0; k < n; ++k)
      CALL(apdvm_set_fields(c, k, F[k][0].data(), F[k][1].data(), F[k][2].data(), nullptr,
                            nullptr, nullptr),
           APDVM_OK);
    CALL(apdvm_step(c, 2), APDVM_OK);
    CALL(apdvm_set_graph(c, 1), APDVM_ERR_ARG);  // graphs need a created stream
    apdvm_destroy(c);
  }
  c = nullptr;
  CALL(apdvm_create(n, cfg, ws, bytes - 256, nullptr, &c), APDVM_ERR_NOMEM);
  hipFree(ws);

  // the batch names
  apdvm_batch *b = nullptr;
  CALL(apdvm_batch_create(n, cfg, nullptr, 0, nullptr, &b), APDVM_OK);
  if (b) {
    for (int k = 0; k < n; ++k)
      CALL(apdvm_batch_set_fields(b, k, F[k][0].data(), F[k][1].data(), F[k][2].data(),
                                  F[k][3].data(), F[k][4].data(), F[k][5].data()),
           APDVM_OK);
    CALL(apdvm_batch_step(b, 1), APDVM_OK);
    std::vector<std::vector<double>> g(6, std::vector<double>((size_t)cfg[0].nx * cfg[0].ny));
    CALL(apdvm_batch_get_fields(b, 0, g[0].data(), g[1].data(), g[2].data(), g[3].data(),
                                g[4].data(), g[5].data()),
         APDVM_OK);
    apdvm_batch_destroy(b);
  }
  hipStreamDestroy(st);
}

}  // namespace

// ---------------------------------------------------------------- self-test
// The checks themselves must catch planted mistakes: launches with a duplicated tile, a
// tile off the grid, a slot beyond its arena, an output that is also an input, a float
// launch on a float64 arena and an FFT block beyond its LDS form each have to raise at
// least one violation, and the correct launch none.

namespace apdvm {
template <typename T>
hipError_t launch_update_uq(int, int, int, const Inst *, const Work *, int, const ArgsUQ &,
                            hipStream_t, const Ev &);
hipError_t launch_solve_part(int part, int rowv, int colv, int rowreg, int colreg,
                             const Inst *, const Work *, int, const Work *, int,
                             const ArgsSolve &, hipStream_t, const Ev &);
}  // namespace apdvm

namespace {

int self_test() {
  using namespace apdvm;
  const int nx = 64, ny = 48, TY = 8, nts = 12, nds = 4;
  const size_t plane = (size_t)nx * ny;
  void *tb = nullptr, *db = nullptr, *tw = nullptr, *lam = nullptr, *ip = nullptr, *wp = nullptr;
  hipMalloc(&tb, nts * plane * 8);
  hipMalloc(&db, nds * plane * 8);
  hipMalloc(&tw, 2 * kTwCap * sizeof(double2));
  hipMalloc(&lam, (nx / 2 + 1 + ny) * 8);
  hipMalloc(&ip, sizeof(Inst));
  hipMalloc(&wp, 64 * sizeof(Work));
  Inst &I = *static_cast<Inst *>(ip);
  std::memset(&I, 0, sizeof(I));
  I.nx = nx;
  I.ny = ny;
  I.plane = (long long)plane;
  I.tbase = tb;
  I.dbase = static_cast<double *>(db);
  I.nt_slots = nts;
  I.nd_slots = nds;
  I.tbytes = 8;
  I.row_pairs_per_block = 1;
  I.cols_per_block = 1;
  I.lam_x = static_cast<double *>(lam);
  I.lam_y = static_cast<double *>(lam) + nx / 2 + 1;
  auto plan = [&](FftPlan &P, int n, int tsc, int q) {
    P.n = n;
    P.npass = 0;
    for (int m = n; m > 1;) {
      const int r = m % 8 == 0 ? 8 : m % 4 == 0 ? 4 : m % 3 == 0 ? 3 : 2;
      P.radix[P.npass++] = r;
      m /= r;
    }
    P.tw2 = static_cast<double2 *>(tw) + q * kTwCap;
    P.lb = 0;
    while ((1LL << (2 * P.lb)) < (long long)tsc * n) ++P.lb;
    P.ntw = (1 << P.lb) + (tsc * n + (1 << P.lb) - 1) / (1 << P.lb);
    P.tsc = tsc;
  };
  plan(I.fx, nx, 1, 0);
  plan(I.fy, ny, 1, 1);
  plan(I.fyh, ny / 2, 2, 1);
  Work *w = static_cast<Work *>(wp);
  int nw = 0;
  for (int y = 0; y < ny; y += TY)
    for (int x = 0; x < nx; x += kTileX) w[nw++] = Work{0, x, y, 0};
  ArgsUQ a{};
  a.stage = 1;
  a.aii = 0.5;
  int s = 0;
  for (int m = 0; m < 2; ++m) {
    a.v[m] = s++;
    a.partner[m] = s++;
    a.un[m] = s++;
  }
  a.qn = s++;
  a.out_us[0] = s++;
  a.out_us[1] = s++;
  a.out_q = s++;
  a.out_hu[0] = a.out_hu[1] = a.out_gq = kNoSlot;
  a.th = a.ddb = a.out_lt = kNoSlot;
  a.co = 4;
  auto &k = hostcheck::counters();
  int caught = 0, cases = 0;
  auto run = [&](const char *what, bool bad, auto &&fn) {
    const long long before = k.violations;
    fn();
    const bool raised = k.violations > before;
    ++cases;
    if (raised == bad) ++caught;
    else std::fprintf(stderr, "self-test: %s: %s\n", what, bad ? "not caught" : "false alarm");
  };
  const Ev ev{};
  run("correct launch", false, [&] { launch_update_uq<double>(0, 5, 4, &I, w, nw, a, nullptr, ev); });
  run("duplicated tile", true, [&] {
    Work keep = w[nw - 1];
    w[nw - 1] = w[0];
    launch_update_uq<double>(0, 5, 4, &I, w, nw, a, nullptr, ev);
    w[nw - 1] = keep;
  });
  run("tile off the grid", true, [&] {
    Work keep = w[nw - 1];
    w[nw - 1].b = ny;
    launch_update_uq<double>(3, 5, 4, &I, w, nw, a, nullptr, ev);
    w[nw - 1] = keep;
  });
  run("slot beyond the arena", true, [&] {
    ArgsUQ b = a;
    b.out_q = nts;
    launch_update_uq<double>(0, 5, 4, &I, w, nw, b, nullptr, ev);
  });
  run("output that is an input", true, [&] {
    ArgsUQ b = a;
    b.out_q = b.qn;
    launch_update_uq<double>(0, 5, 4, &I, w, nw, b, nullptr, ev);
  });
  run("float launch on a float64 arena", true,
      [&] { launch_update_uq<float>(0, 5, 4, &I, w, nw, a, nullptr, ev); });
  run("FFT row block beyond its LDS form", true, [&] {
    I.row_pairs_per_block = ny / 2;  // 24 row pairs of 64: 1536 values in a 1024 form
    Work *r = w + 32;  // one row block in device memory
    r[0] = Work{0, 0, 0, 0};
    ArgsSolve sa{1, 0, 1, 2};
    launch_solve_part(0, 0, 0, 0, 0, &I, r, 1, r, 1, sa, nullptr, ev);
    I.row_pairs_per_block = 1;
  });
  run("FFT register form on rows shorter than the form", true, [&] {
    Work *r = w + 32;
    r[0] = Work{0, 0, 0, 0};
    ArgsSolve sa{1, 0, 1, 2};
    launch_solve_part(0, 0, 0, 1, 0, &I, r, 1, r, 1, sa, nullptr, ev);
  });
  run("FFT register form of several lines on blocks they do not fill", true, [&] {
    Work *r = w + 32;
    r[0] = Work{0, 0, 0, 0};
    ArgsSolve sa{1, 0, 1, 2};
    launch_solve_part(0, 0, 0, 2, 0, &I, r, 1, r, 1, sa, nullptr, ev);
  });
  std::printf("self-test: %d of %d planted cases judged correctly\n", caught, cases);
  for (void *p : {tb, db, tw, lam, ip, wp}) hipFree(p);
  return caught == cases ? 0 : 1;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc > 1 && std::string(argv[1]) == "--self-test") return self_test();
  Scenario sc;
  int scenarios = 0;
  while (read_scenario(std::cin, sc)) {
    run(sc);
    ++scenarios;
    sc = Scenario{};
  }
  const auto &k = hostcheck::counters();
  std::printf(
      "hostcheck: %d scenarios, %lld launches (%lld graph replays, %lld captured operations), "
      "%lld work items, %lld indices checked; %lld violations, %d unexpected statuses\n",
      scenarios, k.launches, k.graph_launches, k.captured_ops, k.items, k.indices, k.violations,
      g_bad);
  return (k.violations || g_bad || scenarios == 0) ? 1 : 0;
}
