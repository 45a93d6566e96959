// Host runtime behind the C ABI of include/apdvm.h: configuration checks, the
// per-instance parameter table, the plane layout, FFT plans, work tables and the
// launch sequence of one IMEX step (Algorithm 1 for every implicit stage).
#include "apdvm.h"
#include "common.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

namespace apdvm {

// Stencil launches: tile height, WENO order (5 or 3), central-difference order (4 or 2).
template <typename T>
hipError_t launch_helmholtz_rhs(int, int, int, const Inst *, const Work *, int, const ArgsR &,
                                hipStream_t, const Ev &);
template <typename T>
hipError_t launch_update_uq(int, int, int, const Inst *, const Work *, int, const ArgsUQ &,
                            hipStream_t, const Ev &);
template <typename T>
hipError_t launch_stage_terms(int, int, int, const Inst *, const Work *, int, const ArgsE &,
                              const ArgsV &, hipStream_t, const Ev &);
template <typename T>
hipError_t launch_grad_q(int, int, const Inst *, const Work *, int, const ArgsG &, hipStream_t,
                         const Ev &);

// Tile heights the stencil kernels are built for; the autotuner picks one per class.
constexpr int kTileRows[2] = {8, 16};
// Launch shapes of the stencil classes: tile rows and workgroup threads; the tile table
// of a shape is the one of its tile height.
constexpr int kNumShapes = 4;
constexpr int kShapeRows[kNumShapes] = {8, 16, 16, 8};
constexpr int kShapeThreads[kNumShapes] = {256, 256, 512, 512};
inline int shape_table(int si) { return kShapeRows[si] == kTileRows[0] ? 0 : 1; }
inline int shape_of(int rows, int threads) {
  for (int si = 0; si < kNumShapes; ++si)
    if (kShapeRows[si] == rows && kShapeThreads[si] == threads) return si;
  return -1;
}
hipError_t launch_solve_part(int part, int rowv, int colv, int rowreg, int colreg,
                             const Inst *, const Work *, int, const Work *, int,
                             const ArgsSolve &, hipStream_t, const Ev &);
hipError_t launch_diagnostics(const Inst *, const Work *, int, int, int, int, int, int, int, int,
                              int, int, double *, int, hipStream_t);
hipError_t launch_field_stats(int split, const void *const f[6], long long n, double *partials,
                              int nblocks, hipStream_t st);
hipError_t launch_convert(void *dst, const void *src, long long n, int to_float, hipStream_t st);
hipError_t launch_state_finite(int split, const Inst *, const Work *, int, int, const StateSet &,
                               unsigned *flag, hipStream_t);
hipError_t launch_snapshot(int split, const Inst *, const Work *, int, int, const StateSet &,
                           const StateSet &, const unsigned *flag, long long *ck_step,
                           long long step, hipStream_t);
hipError_t launch_div_u(int co, const Inst *, const Work *, int, int, int, int, hipStream_t);
hipError_t scratch_init(int device);
double *scratch_ptr(int device);
int scratch_blocks();
hipError_t launch_diag_finish(const double *partials, int nblocks, double area, double *out,
                              hipStream_t st);

namespace {

constexpr size_t kAlign = 256;
constexpr int kStatBlocks = 512;    // workgroups of the input-field statistics kernel
constexpr size_t kFlagBytes = 256;  // finite flag (unsigned) at 0, snapshot step (int64) at 8
constexpr int kDefaultFiniteEvery = 64;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Opt-in log on stderr (environment variable APDVM_LOG set and not "0"): context creation,
// derived time steps, autotuner choices and failed finite checks.
bool log_on() {
  static const bool on = [] {
    const char *e = std::getenv("APDVM_LOG");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}
__attribute__((format(printf, 1, 2))) void apdvm_log(const char *fmt, ...) {
  if (!log_on()) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[apdvm] ");
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  va_end(ap);
}

// ----------------------------------------------------------- validation helpers

bool is_2a3b(int n) {
  if (n <= 0) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

apdvm_status check_grid(const apdvm_config &c) {
  for (int n : {c.nx, c.ny})
    if (n < 8 || n > kFftCap || (n % 2) != 0 || !is_2a3b(n)) return APDVM_ERR_ARG;
  if (!(c.lx > 0.0) || !(c.ly > 0.0) || !std::isfinite(c.lx) || !std::isfinite(c.ly))
    return APDVM_ERR_ARG;
  return APDVM_OK;
}

apdvm_status check_velset(const apdvm_config &c) {
  if (c.q != 6) return APDVM_ERR_VELSET;
  if ((c.cx == nullptr) != (c.cy == nullptr)) return APDVM_ERR_VELSET;
  if (c.cx) {
    for (int i = 0; i < 6; ++i) {
      const double ang = M_PI * i / 3.0;
      if (!(std::fabs(c.cx[i] - std::cos(ang)) <= 1e-12) ||
          !(std::fabs(c.cy[i] - std::sin(ang)) <= 1e-12))
        return APDVM_ERR_VELSET;
    }
  }
  return APDVM_OK;
}

// Type A (Section 3.1): every stage implicit.  Such a tableau runs as an (s+1)-stage
// tableau of ARS form whose first stage is the state at time n with zero coefficients
// in both parts, which evaluates the same sums stage by stage.
bool is_type_a(const apdvm_config &c) { return c.a_im[0] != 0.0; }
int internal_stages(const apdvm_config &c) { return c.s + (is_type_a(c) ? 1 : 0); }

apdvm_status check_tableau(const apdvm_config &c) {
  const int s = c.s;
  if (s < 2 || s > kMaxStages) return APDVM_ERR_TABLEAU;
  if (!c.a_ex || !c.b_ex || !c.a_im || !c.b_im) return APDVM_ERR_TABLEAU;
  auto At = [&](int i, int j) { return c.a_ex[i * s + j]; };
  auto A = [&](int i, int j) { return c.a_im[i * s + j]; };
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j < s; ++j) {
      if (!std::isfinite(At(i, j)) || !std::isfinite(A(i, j))) return APDVM_ERR_TABLEAU;
      if (j >= i && At(i, j) != 0.0) return APDVM_ERR_TABLEAU;  // explicit: strictly lower
      if (j > i && A(i, j) != 0.0) return APDVM_ERR_TABLEAU;    // implicit: DIRK
    }
    if (!std::isfinite(c.b_ex[i]) || !std::isfinite(c.b_im[i])) return APDVM_ERR_TABLEAU;
  }
  if (is_type_a(c)) {
    // type A: every diagonal entry nonzero; one extra internal stage must fit
    if (s + 1 > kMaxStages) return APDVM_ERR_TABLEAU;
    for (int i = 0; i < s; ++i)
      if (A(i, i) == 0.0) return APDVM_ERR_TABLEAU;
  } else {
    // ARS type: the first stage is explicit and the first column of A vanishes
    for (int i = 0; i < s; ++i)
      if (A(i, 0) != 0.0) return APDVM_ERR_TABLEAU;
    for (int i = 1; i < s; ++i)
      if (A(i, i) == 0.0) return APDVM_ERR_TABLEAU;
  }
  // globally stiffly accurate: the last stage is the new time level
  for (int j = 0; j < s; ++j)
    if (A(s - 1, j) != c.b_im[j]) return APDVM_ERR_TABLEAU;
  for (int j = 0; j < s - 1; ++j)
    if (At(s - 1, j) != c.b_ex[j]) return APDVM_ERR_TABLEAU;
  if (c.b_ex[s - 1] != 0.0) return APDVM_ERR_TABLEAU;
  return APDVM_OK;
}

apdvm_status check_physics(const apdvm_config &c) {
  if (!(c.eps >= 0.0) || !std::isfinite(c.eps)) return APDVM_ERR_ARG;
  if (c.tau < 0.0) {
    if (!(c.mach > 0.0) || !std::isfinite(c.mach)) return APDVM_ERR_ARG;
  } else if (!std::isfinite(c.tau)) {
    return APDVM_ERR_ARG;
  }
  if (!std::isfinite(c.dt)) return APDVM_ERR_ARG;
  if (!(c.dt > 0.0)) {
    if (!(c.cfl > 0.0) || !(c.c_visc > 0.0) || !std::isfinite(c.cfl) || !std::isfinite(c.c_visc))
      return APDVM_ERR_ARG;
  }
  if (c.precision != APDVM_FP64 && c.precision != APDVM_FP32_SPLIT) return APDVM_ERR_ARG;
  if (c.weno_order != 0 && c.weno_order != 3 && c.weno_order != 5) return APDVM_ERR_ARG;
  if (c.central_order != 0 && c.central_order != 2 && c.central_order != 4) return APDVM_ERR_ARG;
  return APDVM_OK;
}

int weno_order_of(const apdvm_config &c) { return c.weno_order == 3 ? 3 : 5; }
int central_order_of(const apdvm_config &c) { return c.central_order == 2 ? 2 : 4; }

bool same_tableau(const apdvm_config &a, const apdvm_config &b) {
  if (a.s != b.s || a.precision != b.precision) return false;
  const size_t s = a.s;
  return !std::memcmp(a.a_ex, b.a_ex, s * s * sizeof(double)) &&
         !std::memcmp(a.a_im, b.a_im, s * s * sizeof(double)) &&
         !std::memcmp(a.b_ex, b.b_ex, s * sizeof(double)) &&
         !std::memcmp(a.b_im, b.b_im, s * sizeof(double));
}

apdvm_status validate(int n, const apdvm_config *cfgs) {
  if (n < 1 || !cfgs) return APDVM_ERR_ARG;
  for (int k = 0; k < n; ++k) {
    apdvm_status st;
    if ((st = check_grid(cfgs[k])) != APDVM_OK) return st;
    if ((st = check_velset(cfgs[k])) != APDVM_OK) return st;
    if ((st = check_tableau(cfgs[k])) != APDVM_OK) return st;
    if ((st = check_physics(cfgs[k])) != APDVM_OK) return st;
    if (k > 0 && !same_tableau(cfgs[0], cfgs[k])) return APDVM_ERR_ARG;
    if (weno_order_of(cfgs[k]) != weno_order_of(cfgs[0]) ||
        central_order_of(cfgs[k]) != central_order_of(cfgs[0]))
      return APDVM_ERR_ARG;
  }
  return APDVM_OK;
}

// ----------------------------------------------------------- plane layout

// Slot numbers of every plane one step touches, for an s-stage ARS tableau.  Stage 0
// is the state at time n; stages 1..s-1 are implicit; stage s-1 writes straight into
// the other state set.
struct Layout {
  int s;
  int st[2][5];  // state sets: u1, u2, v1, v2, q
  int th[2];     // float64: theta of each state set
  int ck[5], thck;  // snapshot of the last state that passed the finite check
  // FP32-split form only (float64 arena): the velocity of each state set, D0.u of each
  // state set, and the velocity of the snapshot
  int ud[2][2], du0[2], ckud[2];
  int E[kMaxStages][2], V[kMaxStages][2], Du[kMaxStages], Lt[kMaxStages];
  int Hu[kMaxStages][2], Gq[kMaxStages], U[kMaxStages][2], Q[kMaxStages];
  int ddb, G[2];
  int Us[2];                      // u*(i) of the current stage
  int Th[kMaxStages], R, spec;    // float64
  int ntrans, ndbl;
};

Layout make_layout(int s, bool split) {
  Layout L;
  std::memset(&L, 0xff, sizeof(L));  // every slot starts as kNoSlot (-1)
  L.s = s;
  int t = 0, d = 0;
  for (int p = 0; p < 2; ++p)
    for (int f = 0; f < 5; ++f) L.st[p][f] = t++;
  L.th[0] = d++;
  L.th[1] = d++;
  for (int f = 0; f < 5; ++f) L.ck[f] = t++;
  L.thck = d++;
  if (split) {
    for (int p = 0; p < 2; ++p) {
      L.ud[p][0] = d++;
      L.ud[p][1] = d++;
      L.du0[p] = d++;
    }
    L.ckud[0] = d++;
    L.ckud[1] = d++;
  }
  for (int j = 0; j <= s - 2; ++j) {
    L.E[j][0] = t++;
    L.E[j][1] = t++;
    L.Du[j] = t++;
  }
  for (int j = 1; j <= s - 2; ++j) {
    L.V[j][0] = t++;
    L.V[j][1] = t++;
    L.Lt[j] = t++;
    L.Hu[j][0] = t++;
    L.Hu[j][1] = t++;
    L.Gq[j] = t++;
    L.U[j][0] = t++;
    L.U[j][1] = t++;
    L.Q[j] = t++;
    L.Th[j] = d++;
  }
  L.ddb = t++;
  L.G[0] = t++;
  L.G[1] = t++;
  L.Us[0] = t++;
  L.Us[1] = t++;
  L.R = d++;
  L.spec = d++;
  L.ntrans = t;
  L.ndbl = d;
  return L;
}

// ----------------------------------------------------------- FFT plans

int fft_radices(int n, int *rad) {
  int np = 0;
  int m = n;
  while (m % 8 == 0) { rad[np++] = 8; m /= 8; }
  if (m % 4 == 0) { rad[np++] = 4; m /= 4; }
  if (m % 2 == 0) { rad[np++] = 2; m /= 2; }
  while (m % 3 == 0) { rad[np++] = 3; m /= 3; }
  return np;
}

// Two-level table (see FftPlan): lo[b] = w^b for b < B, hi[a] = w^(a B), w = exp(-2 pi i / n).
// Returns the number of entries; *lb receives log2 B.
int twiddles2(int n, double2 *out, int *lb) {
  int l = 0;
  while ((1 << l) * (1 << l) < n) ++l;
  const int B = 1 << l, nhi = (n + B - 1) / B;
  const long double c = -2.0L * 3.141592653589793238462643383279502884L / n;
  for (int b = 0; b < B; ++b) out[b] = make_double2((double)cosl(c * b), (double)sinl(c * b));
  for (int a = 0; a < nhi; ++a) {
    const long double t = c * ((long double)a * B);
    out[B + a] = make_double2((double)cosl(t), (double)sinl(t));
  }
  *lb = l;
  return B + nhi;
}

// Fourier symbol of the central second difference on an n-point grid with spacing h,
// th = 2 pi k / n: (-2 cos 2 th + 32 cos th - 30) / (12 h^2) for the fourth-order one.
double lap_symbol(int k, int n, double h, int order) {
  if (order == 2) {
    // (2 cos th - 2) / h^2 of the second-order central second difference
    const long double th = 2.0L * 3.141592653589793238462643383279502884L * k / n;
    return (double)((2.0L * cosl(th) - 2.0L) / ((long double)h * h));
  }
  const long double th = 2.0L * 3.141592653589793238462643383279502884L * k / n;
  return (double)((-2.0L * cosl(2.0L * th) + 32.0L * cosl(th) - 30.0L) / (12.0L * h * h));
}

double resolved_tau(const apdvm_config &c) { return c.tau >= 0.0 ? c.tau : 4.0 * c.eps / c.mach; }

// ----------------------------------------------------------- sizes

struct Sizes {
  size_t per_inst_trans, per_inst_dbl, per_inst_tab;
  size_t total;
};

int n_tiles(const apdvm_config &c, int ty) {
  return ((c.nx + kTileX - 1) / kTileX) * ((c.ny + ty - 1) / ty);
}
// FFT kernel forms by LDS capacity (0: kRowSmallCap, 1: kColMidCap, 2: kFftCap complex
// values): the smallest that holds a whole row (whole column) of every instance.
int fft_form(int longest) {
  return longest <= kRowSmallCap ? 0 : longest <= kColMidCap ? 1 : 2;
}
int form_cap(int v) { return v == 0 ? kRowSmallCap : v == 1 ? kColMidCap : kFftCap; }
int row_form(int n, const apdvm_config *cfgs) {
  int mx = 0;
  for (int k = 0; k < n; ++k) mx = cfgs[k].nx > mx ? cfgs[k].nx : mx;
  return fft_form(mx);
}
int col_form(int n, const apdvm_config *cfgs) {
  int my = 0;
  for (int k = 0; k < n; ++k) my = cfgs[k].ny > my ? cfgs[k].ny : my;
  return fft_form(my);
}
// row pairs per row workgroup
int rpb(const apdvm_config &c, int v) {
  int r = form_cap(v) / c.nx;
  if (r > c.ny / 2) r = c.ny / 2;
  return r < 1 ? 1 : r;
}
// columns per column workgroup (the spectrum has nx/2 columns: kx = nx/2 shares column 0)
int cpb(const apdvm_config &c, int v) {
  int w = form_cap(v) / c.ny;
  if (w > c.nx / 2) w = c.nx / 2;
  return w < 1 ? 1 : w;
}
int n_colblocks(const apdvm_config &c, int v) { return (c.nx / 2 + cpb(c, v) - 1) / cpb(c, v); }
int n_rowblocks(const apdvm_config &c, int v) { return (c.ny / 2 + rpb(c, v) - 1) / rpb(c, v); }

// Register form of the row (rows) or column FFT kernels of form v for these instances: 1 if
// every line is the form's capacity (one line per workgroup), 2 if every line is 8^m >= 64
// values, shorter, and the lines of every instance fill whole workgroups of cap / n lines
// (row pairs, or columns of the half spectrum), 0 otherwise.
int fft_reg_form(int n, const apdvm_config *cfgs, int v, bool rows) {
  const int cap = form_cap(v);
  bool one = true, lines = true;
  for (int k = 0; k < n; ++k) {
    const int len = rows ? cfgs[k].nx : cfgs[k].ny;
    const int cnt = rows ? cfgs[k].ny / 2 : cfgs[k].nx / 2;  // row pairs or columns
    one = one && len == cap;
    const bool pow8 = len >= 64 && (len & (len - 1)) == 0 && __builtin_ctz(len) % 3 == 0;
    lines = lines && pow8 && len < cap && cnt % (cap / len) == 0;
  }
  return one ? 1 : lines ? 2 : 0;
}

size_t inst_bytes(const apdvm_config &c, const Layout &L, size_t tsize) {
  const size_t plane = (size_t)c.nx * c.ny;
  size_t b = align_up(L.ntrans * plane * tsize);
  b += align_up(L.ndbl * plane * sizeof(double));
  b += align_up((size_t)2 * kTwCap * sizeof(double2));                 // two-level twiddles
  b += align_up((size_t)(c.nx / 2 + 1 + c.ny) * sizeof(double));        // symbols
  return b;
}

size_t workspace_bytes(int n, const apdvm_config *cfgs) {
  const bool split = cfgs[0].precision == APDVM_FP32_SPLIT;
  const Layout L = make_layout(internal_stages(cfgs[0]), split);
  const size_t tsize = split ? sizeof(float) : sizeof(double);
  size_t b = align_up(n * sizeof(Inst));
  const int rv = row_form(n, cfgs), cv = col_form(n, cfgs);
  size_t ntile8 = 0, ntile16 = 0, nrow = 0, ncol = 0;
  for (int k = 0; k < n; ++k) {
    b += inst_bytes(cfgs[k], L, tsize);
    ntile8 += n_tiles(cfgs[k], kTileRows[0]);
    ntile16 += n_tiles(cfgs[k], kTileRows[1]);
    nrow += n_rowblocks(cfgs[k], rv);
    ncol += n_colblocks(cfgs[k], cv);
  }
  b += align_up(ntile8 * sizeof(Work)) + align_up(ntile16 * sizeof(Work)) + align_up(nrow * sizeof(Work)) +
       align_up(ncol * sizeof(Work));
  b += align_up(8 * sizeof(double) * 1024);  // diagnostics partials
  b += align_up(3 * sizeof(double) * kStatBlocks);  // input-field statistics partials
  b += align_up(kFlagBytes);                          // finite flag and snapshot step
  return b;
}

}  // namespace

// One kernel launch of a step: its class, arguments and algorithmic bytes (every
// plane it must read and write, counted once).
enum LaunchClass {
  kHelmRhs = 0, kRowsFwd = 1, kCols = 2, kRowsInv = 3, kUpdateUQ = 4, kStageTerms = 5,
  kGradQ = 6, kNumClasses = 7,
  kDivU = 8  // float64 D0.u of a state set (FP32-split form, after new fields only)
};
// Stencil classes with a tuned launch shape, in the order of the tuning array.
constexpr int kNumTuned = 4;
constexpr int kTunedClasses[kNumTuned] = {kHelmRhs, kUpdateUQ, kStageTerms, kGradQ};

// Stream synchronisation entries of a plan (cls = kSync): a fork makes the solve stream
// wait for the work enqueued so far on the main stream, a join the reverse.
constexpr int kSync = -1;
enum SyncKind { kNoSync = 0, kFork = 1, kJoin = 2 };

struct Launch {
  int cls;
  int sync;   // SyncKind of a kSync entry
  int du[3];  // kDivU: float64 slots u1, u2 in, D0.u out
  bool side;  // runs on the solve stream (when the two streams overlap)
  ArgsV v;  // step 1 of the next stage, fused into a stage-terms launch
  ArgsR r;
  ArgsUQ uq;
  ArgsE e;
  ArgsSolve sv;
  ArgsG g;
  double bytes;
};

}  // namespace apdvm

using namespace apdvm;

struct apdvm_ctx {
  int n = 0;
  int s = 0;
  bool split = false;
  double At[kMaxStages][kMaxStages], A[kMaxStages][kMaxStages];
  hipStream_t stream = nullptr;
  int device = 0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  Layout L;
  std::vector<apdvm_config> cfg;
  std::vector<Inst> inst;
  Inst *d_inst = nullptr;
  Work *d_tiles[2] = {nullptr, nullptr};  // tile tables for kTileRows[0] and kTileRows[1]
  int ntiles[2] = {0, 0};
  Work *d_rows = nullptr, *d_cols = nullptr;
  int nrows = 0, ncols = 0;
  int row_v = 0, col_v = 0;  // FFT kernel forms of the rows and columns (fft_form)
  bool row_split = false;    // inverse rows split in halves (largest form, every nx % 4 == 0)
  // FFT register forms of the rows and columns (fft_reg_form): 0 none, 1 every line is its
  // form's capacity, 2 every line is 8^m values, shorter, filling the blocks of its form
  int row_reg = 0, col_reg = 0;
  int shape[apdvm::kNumClasses];     // launch shape of each stencil class (kShapeRows...)
  int wo = 5, co = 4;                // WENO and central-difference orders
  std::vector<Work> tiles;  // host copy of the 64 x 16 tiles (diagnostics use per-instance ranges)
  std::vector<int> tile_first, tile_count;
  double *d_partials = nullptr;
  int parity = 0;           // state set holding the current state
  bool terms_ready = false; // stage-0 terms computed for the current state
  std::vector<char> has_fields;
  std::vector<double> umax;
  int64_t step = 0;
  double cells = 0.0;                 // sum of nx * ny over instances
  double spec_bytes = 0.0;            // sum of ny (nx/2) * 16 over instances
  std::vector<apdvm::Launch> plan[2]; // launch list of one step from each state set
  bool use_graph = false;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  int timed_class = -1;               // kernel class bracketed by events, -1 none
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t ev_used = 0;
  int timed_stride = 1;               // bracket the timed class in every timed_stride-th step
  int64_t timed_steps = 0;            // steps enqueued since apdvm_timing_enable
  // Second stream for the Helmholtz solve, forked from and joined to the main stream
  // once per stage; with overlap off every launch goes to the main stream.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  bool fused = false;  // one stream, theta completion fused into the update launch
  // Finite check every finite_every steps (0: off): device flag, step of the snapshot.
  double *d_stats = nullptr;
  unsigned *d_flag = nullptr;
  long long *d_ck_step = nullptr;
  int finite_every = 0;
};

namespace {

apdvm_status hip_status(hipError_t e) { return e == hipSuccess ? APDVM_OK : APDVM_ERR_HIP; }

// dt rule (see apdvm.h): largest dt with ct dt max(umax, 1, tau eps / (te2 + ct dt)) <= cfl h
// and ct dt (tau/4) ct dt / (te2 + ct dt) <= c_visc h^2, found by bisection on the
// monotone left-hand sides.
double derive_dt(const apdvm_config &c, double tau, double umax, double ct) {
  const double h = std::fmin(c.lx / c.nx, c.ly / c.ny);
  const double te2 = tau * c.eps * c.eps;
  auto ok = [&](double dt) {
    const double d = ct * dt;
    const double kin = (te2 + d) > 0.0 ? tau * c.eps / (te2 + d) : 0.0;
    const bool hyp = d * std::fmax(std::fmax(umax, 1.0), kin) <= c.cfl * h;
    const bool par = d * 0.25 * tau * d / (te2 + d) <= c.c_visc * h * h;
    return hyp && par;
  };
  double lo = 0.0, hi = 100.0 * h;
  if (ok(hi)) return hi;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (ok(mid)) lo = mid; else hi = mid;
  }
  return lo;
}

void set_dt(apdvm_ctx *c, int k, double dt) {
  Inst &I = c->inst[k];
  I.dt = dt;
  for (int i = 1; i < c->s; ++i) {
    const double aii = c->A[i][i];
    I.kinv[i] = 1.0 / (I.te2 + dt * aii);
    I.sigma[i] = 2.0 * I.eps * I.eps / ((dt * aii) * (dt * aii));
    I.rdt2[i] = 1.0 / (dt * aii * aii);
    I.rdt[i] = 1.0 / (dt * aii);
  }
}

apdvm_status upload_inst(apdvm_ctx *c, int k) {
  return hip_status(hipMemcpyAsync(c->d_inst + k, &c->inst[k], sizeof(Inst), hipMemcpyHostToDevice,
                                   c->stream));
}

// Step 1 of stage k, fused into the stage-terms launch of stage k - 1 (whose E and v
// stay in registers).  Pk is the state set of the step containing stage k.
void fill_relax(const apdvm_ctx *c, int k, int Pk, ArgsV &nv, ArgsE &e, double pt,
                double &bytes) {
  const Layout &L = c->L;
  const int s = c->s;
  nv = ArgsV{};
  nv.stage = k;
  nv.vn[0] = L.st[Pk][2];
  nv.vn[1] = L.st[Pk][3];
  for (int j = 0; j + 1 < k; ++j) {
    if (c->At[k][j] != 0.0) {
      nv.E[nv.nE][0] = L.E[j][0]; nv.E[nv.nE][1] = L.E[j][1]; nv.cE[nv.nE++] = c->At[k][j];
    }
    if (j >= 1 && c->A[k][j] != 0.0) {
      nv.V[nv.nV][0] = L.V[j][0]; nv.V[nv.nV][1] = L.V[j][1]; nv.cV[nv.nV++] = c->A[k][j];
    }
  }
  e.c_e_next = c->At[k][k - 1];
  e.c_v_next = k - 1 >= 1 ? c->A[k][k - 1] : 0.0;
  const bool last = k == s - 1;
  nv.out[0] = last ? L.st[1 - Pk][2] : L.V[k][0];
  nv.out[1] = last ? L.st[1 - Pk][3] : L.V[k][1];
  bytes += (2 + 2 * nv.nE + 2 * nv.nV + 2) * pt;  // v^n, history, v(k)
}

// Stage terms of stage j that a stage other than j + 1 reads (j + 1 gets them in
// registers through the fused step 1).
bool e_stored(const apdvm_ctx *c, int j) {
  for (int k = j + 2; k < c->s; ++k)
    if (c->At[k][j] != 0.0) return true;
  return false;
}
bool implicit_stored(const apdvm_ctx *c, int j) {
  for (int k = j + 1; k < c->s; ++k)
    if (c->A[k][j] != 0.0) return true;
  return false;
}

// Launch of G = te2 D_W q[v] from q and v, into the G slots.
Launch grad_q_launch(const apdvm_ctx *c, int q, int v1, int v2) {
  const Layout &L = c->L;
  Launch l{};
  l.cls = kGradQ;
  l.g.q = q; l.g.v[0] = v1; l.g.v[1] = v2;
  l.g.out_g[0] = L.G[0]; l.g.out_g[1] = L.G[1];
  l.bytes = 5 * c->cells * (c->split ? 4.0 : 8.0);  // q, v in; G out
  return l;
}

// Stage-terms launches for the state set P itself (stage 0), used after new fields.  In
// the FP32-split form the float64 D0.u^n comes first (k_div_u); the stage-terms launch
// then forms E from the float copy of u^n.
std::vector<Launch> stage0_launches(const apdvm_ctx *c, int P) {
  const Layout &L = c->L;
  const double pt = c->cells * (c->split ? 4.0 : 8.0);
  std::vector<Launch> out;
  if (c->split) {
    Launch d{};
    d.cls = kDivU;
    d.du[0] = L.ud[P][0]; d.du[1] = L.ud[P][1]; d.du[2] = L.du0[P];
    out.push_back(d);
  }
  Launch l{};
  l.cls = kStageTerms;
  ArgsE &a = l.e;
  a.us[0] = a.us[1] = kNoSlot;
  a.u[0] = L.st[P][0]; a.u[1] = L.st[P][1]; a.v[0] = L.st[P][2]; a.v[1] = L.st[P][3];
  a.g[0] = L.G[0]; a.g[1] = L.G[1];
  a.th = kNoSlot; a.ddb = kNoSlot;
  a.out_u[0] = a.out_u[1] = a.hu[0] = a.hu[1] = kNoSlot;
  a.out_e[0] = e_stored(c, 0) ? L.E[0][0] : kNoSlot;
  a.out_e[1] = e_stored(c, 0) ? L.E[0][1] : kNoSlot;
  a.out_du = c->split ? kNoSlot : L.Du[0];
  a.out_lt = kNoSlot;
  a.ub[0] = a.ub[1] = a.out_ud[0] = a.out_ud[1] = a.du0_in = a.du0_out = kNoSlot;
  a.ui[0] = a.ui[1] = kNoSlot;
  a.q = kNoSlot;
  if (c->split) {  // E of the state from its float64 velocity
    a.ub[0] = L.ud[P][0];
    a.ub[1] = L.ud[P][1];
  }
  l.bytes = (2 + 2 + 2 + 1 + (e_stored(c, 0) ? 2 : 0)) * pt;  // u, G, v in; D0.u, E out
  if (c->split) l.bytes += 2 * (c->cells * 8.0) - 3 * pt;     // float64 u in, no D0.u out
  fill_relax(c, 1, P, l.v, a, pt, l.bytes);
  out.push_back(grad_q_launch(c, L.st[P][4], L.st[P][2], L.st[P][3]));
  out.push_back(l);
  return out;
}

// Launch list of one step starting from state set P.  Per stage: the right-hand side and
// the Helmholtz solve go to the solve stream while the theta-free part of steps 3 and 4
// and the q part of the stage terms run on the main stream; the stage-terms launch,
// which completes u(i) with theta(i), joins the two.  Fused schedule (c->fused): every
// launch on the main stream, the update launch after the solve, completing u(i), Hu(i)
// and Ltheta(i) from theta(i) itself, so u*(i) and hu make no round trip through memory
// and the stage-terms launch reads u(i) (the split form: the increment du(i)).
std::vector<Launch> build_plan(const apdvm_ctx *c, int P) {
  const Layout &L = c->L;
  const int s = c->s, Q = 1 - P;
  const double pt = c->cells * (c->split ? 4.0 : 8.0), pd = c->cells * 8.0;
  std::vector<Launch> plan;
  auto sync = [&](int kind) {
    Launch l{};
    l.cls = kSync;
    l.sync = kind;
    plan.push_back(l);
  };
  for (int i = 1; i < s; ++i) {
    const bool last = i == s - 1;
    const int v1 = last ? L.st[Q][2] : L.V[i][0], v2 = last ? L.st[Q][3] : L.V[i][1];
    const int u1 = last ? L.st[Q][0] : L.U[i][0], u2 = last ? L.st[Q][1] : L.U[i][1];
    const int qi = last ? L.st[Q][4] : L.Q[i];
    const int th = last ? L.th[Q] : L.Th[i];
    const double aii = c->A[i][i];
    const bool keep = !last && implicit_stored(c, i);
    const bool fz = c->fused;
    if (!fz) sync(kFork);
    // step 2 right-hand side (v(i) comes from the previous stage-terms launch)
    Launch l{};
    l.cls = kHelmRhs;
    l.side = !fz;
    ArgsR &ar = l.r;
    ar.stage = i; ar.aii = aii; ar.v[0] = v1; ar.v[1] = v2; ar.thn = L.th[P];
    // FP32-split: float64 D0.u^n of this state set; the D slots hold D0 of the increments
    ar.du0 = c->split ? L.du0[P] : L.Du[0];
    ar.du0_dbl = c->split ? 1 : 0;
    ar.sum_a = 0.0;
    for (int j = 1; j < i; ++j) {
      if (c->A[i][j] != 0.0) {
        ar.D[ar.nD] = L.Du[j]; ar.cD[ar.nD++] = c->A[i][j];
        ar.L[ar.nL] = L.Lt[j]; ar.cL[ar.nL++] = c->A[i][j];
        ar.sum_a += c->A[i][j];
      }
    }
    ar.out_r = L.R; ar.out_ddb = L.ddb;
    ar.c_l = 1.0 / aii;
    // v in (2), D0^2:B out (1), histories, D0.u^n (transport or float64); theta^n in, R out
    l.bytes = (2 + ar.nD + ar.nL + 1) * pt + (c->split ? pd : pt) + 2 * pd;
    plan.push_back(l);
    // step 2 solve: three kernels, each one read and one write of a float64 plane
    // (the spectrum holds nx/2 complex columns of ny values)
    ArgsSolve as{};
    as.stage = i; as.r = L.R; as.spec = L.spec; as.out = th;
    const int parts[3] = {kRowsFwd, kCols, kRowsInv};
    for (int m = 0; m < 3; ++m) {
      const int k = parts[m];
      l = Launch{};
      l.cls = k;
      l.side = !fz;
      l.sv = as;
      l.bytes = (k == kRowsFwd || k == kRowsInv) ? pd + c->spec_bytes : 2 * c->spec_bytes;
      plan.push_back(l);
    }
    // steps 3 and 4 short of theta(i), beside the solve
    l = Launch{};
    l.cls = kUpdateUQ;
    ArgsUQ &au = l.uq;
    au.stage = i; au.aii = aii; au.v[0] = v1; au.v[1] = v2;
    au.partner[0] = i == 1 ? L.st[P][0] : L.U[i - 1][0];
    au.partner[1] = i == 1 ? L.st[P][1] : L.U[i - 1][1];
    // FP32-split: the increment u*(i) - u^n, without u^n
    au.un[0] = c->split ? kNoSlot : L.st[P][0];
    au.un[1] = c->split ? kNoSlot : L.st[P][1];
    au.qn = L.st[P][4];
    for (int j = 1; j < i; ++j) {
      if (c->A[i][j] != 0.0) {
        au.H[au.nH][0] = L.Hu[j][0]; au.H[au.nH][1] = L.Hu[j][1]; au.cH[au.nH++] = c->A[i][j];
        au.G[au.nG] = L.Gq[j]; au.cG[au.nG++] = c->A[i][j];
      }
    }
    au.out_us[0] = L.Us[0]; au.out_us[1] = L.Us[1]; au.out_q = qi;
    if (keep) {
      au.out_hu[0] = L.Hu[i][0]; au.out_hu[1] = L.Hu[i][1]; au.out_gq = L.Gq[i];
    } else {
      au.out_hu[0] = au.out_hu[1] = au.out_gq = kNoSlot;
    }
    au.th = au.ddb = au.out_lt = kNoSlot;
    au.co = c->co;
    if (fz) {
      // theta(i) is solved: u(i) (the split form: du(i), in the u* slots), Hu(i), Ltheta(i)
      au.th = th;
      if (!c->split) { au.out_us[0] = u1; au.out_us[1] = u2; }
      if (keep) { au.ddb = L.ddb; au.out_lt = L.Lt[i]; }
    }
    // the partner is u^n for the first stage: read once with u^n (the split form reads
    // only the partner)
    const int reads = 2 + (i == 1 || c->split ? 0 : 2) + 3 + 2 * au.nH + au.nG;
    l.bytes = (reads + 1 + 2 + (keep ? 3 : 0)) * pt;
    if (fz) l.bytes += pd + (keep ? 2 * pt : 0);  // theta in; ddb in, Ltheta out
    plan.push_back(l);
    // the q part G of E: its own launch, or (split form, fused schedule) inside the
    // stage-terms launch
    const bool gq_here = fz && c->split;
    if (!gq_here) plan.push_back(grad_q_launch(c, qi, v1, v2));
    if (!fz) sync(kJoin);
    // u(i) from theta(i), terms of this stage for later stages, and step 1 of the next
    // stage; the last stage's terms are the next step's stage-0 terms
    l = Launch{};
    l.cls = kStageTerms;
    ArgsE &ae = l.e;
    ae.us[0] = L.Us[0]; ae.us[1] = L.Us[1]; ae.u[0] = ae.u[1] = kNoSlot;
    ae.ub[0] = ae.ub[1] = ae.out_ud[0] = ae.out_ud[1] = ae.du0_in = ae.du0_out = kNoSlot;
    ae.ui[0] = ae.ui[1] = kNoSlot;
    ae.q = kNoSlot;
    if (c->split) {
      // increment form on the float64 base u^n; the last stage writes the float64 state
      // u^{n+1} and its D0.u, the next step's D0.u^n
      ae.ub[0] = L.ud[P][0]; ae.ub[1] = L.ud[P][1];
      if (last) {
        ae.out_ud[0] = L.ud[Q][0]; ae.out_ud[1] = L.ud[Q][1];
        ae.du0_in = L.du0[P]; ae.du0_out = L.du0[Q];
      }
    }
    ae.g[0] = L.G[0]; ae.g[1] = L.G[1];
    ae.v[0] = v1; ae.v[1] = v2; ae.th = th; ae.aii = aii;
    ae.out_u[0] = u1; ae.out_u[1] = u2;
    ae.hu[0] = keep ? L.Hu[i][0] : kNoSlot;
    ae.hu[1] = keep ? L.Hu[i][1] : kNoSlot;
    ae.ddb = keep ? L.ddb : kNoSlot;
    const int ej = last ? 0 : i;  // stage index of these terms in the step that reads them
    const bool est = e_stored(c, ej);
    ae.out_e[0] = est ? L.E[ej][0] : kNoSlot;
    ae.out_e[1] = est ? L.E[ej][1] : kNoSlot;
    ae.out_du = c->split && last ? kNoSlot : L.Du[ej];
    ae.out_lt = keep ? L.Lt[i] : kNoSlot;
    // theta, u*, G, v in; u, D0.u, E out; with keep hu and ddb in, Hu and Ltheta out
    l.bytes = pd + (2 + 2 + 2 + 2 + 1 + (est ? 2 : 0) + (keep ? 6 : 0)) * pt;
    if (c->split) {
      if (last)  // base u^n and D0.u^n in, u^{n+1} and D0.u^{n+1} out, in float64
        l.bytes += 6 * pd - pt;
      else  // float64 base u^n
        l.bytes += 2 * pd;
    }
    if (fz) {
      // u(i) (or du(i)) is complete: no theta, no u* and no Hu or Ltheta here
      ae.us[0] = ae.us[1] = kNoSlot;
      ae.th = kNoSlot;
      ae.hu[0] = ae.hu[1] = kNoSlot;
      ae.ddb = kNoSlot;
      ae.out_lt = kNoSlot;
      if (c->split) {  // the increment du(i) on the float64 base; out_u the float u(i)
        ae.ui[0] = L.Us[0]; ae.ui[1] = L.Us[1];
        ae.q = qi;  // G from q(i) and v(i) here: q in, no G
        ae.g[0] = ae.g[1] = kNoSlot;
        l.bytes += pt - 2 * pt;
      } else {  // u(i) as the update launch wrote it
        ae.u[0] = u1; ae.u[1] = u2;
        ae.out_u[0] = ae.out_u[1] = kNoSlot;
      }
      l.bytes -= pd + (keep ? 6 : 0) * pt + (c->split ? 0 : 2 * pt);
    }
    if (last)
      fill_relax(c, 1, Q, l.v, ae, pt, l.bytes);  // next step, state set Q
    else
      fill_relax(c, i + 1, P, l.v, ae, pt, l.bytes);
    plan.push_back(l);
  }
  return plan;
}

hipStream_t stream_of(const apdvm_ctx *c, const Launch &l) {
  return l.side && c->overlap ? c->side : c->stream;
}

template <typename T>
hipError_t run_launch(apdvm_ctx *c, const Launch &l, const Ev &ev = Ev{}) {
  if (l.cls == kSync) {
    if (!c->overlap) return hipSuccess;
    hipStream_t from = l.sync == kFork ? c->stream : c->side;
    hipStream_t to = l.sync == kFork ? c->side : c->stream;
    hipEvent_t ev = l.sync == kFork ? c->ev_fork : c->ev_join;
    const hipError_t e = hipEventRecord(ev, from);
    return e != hipSuccess ? e : hipStreamWaitEvent(to, ev, 0);
  }
  hipStream_t st = stream_of(c, l);
  if (l.cls == kDivU)
    return launch_div_u(c->co, c->d_inst, c->d_tiles[1], c->ntiles[1], l.du[0], l.du[1], l.du[2],
                        st);
  const int si = c->shape[l.cls];
  const int ti = shape_table(si);
  Work *tiles = c->d_tiles[ti];
  const int nt = c->ntiles[ti];
  switch (l.cls) {
    case kHelmRhs:
      return launch_helmholtz_rhs<T>(si, c->wo, c->co, c->d_inst, tiles, nt, l.r, st, ev);
    case kRowsFwd:
    case kCols:
    case kRowsInv:
      return launch_solve_part(l.cls - kRowsFwd, c->row_split ? 3 : c->row_v, c->col_v,
                               c->row_reg, c->col_reg, c->d_inst, c->d_rows,
                               c->nrows, c->d_cols, c->ncols, l.sv, st, ev);
    case kUpdateUQ:
      return launch_update_uq<T>(si, c->wo, c->co, c->d_inst, tiles, nt, l.uq, st, ev);
    case kGradQ:
      return launch_grad_q<T>(si, c->wo, c->d_inst, tiles, nt, l.g, st, ev);
    default:
      return launch_stage_terms<T>(si, c->wo, c->co, c->d_inst, tiles, nt, l.e, l.v, st, ev);
  }
}

template <typename T>
apdvm_status stage0_terms(apdvm_ctx *c) {
  for (const Launch &l : stage0_launches(c, c->parity))
    if (run_launch<T>(c, l) != hipSuccess) return APDVM_ERR_HIP;
  c->terms_ready = true;
  return APDVM_OK;
}

template <typename T>
apdvm_status run_plan_direct(apdvm_ctx *c, const std::vector<Launch> &plan, bool sample) {
  for (const Launch &l : plan) {
    Ev ev;
    if (sample && c->timed_class == l.cls) {
      if (c->ev_used == c->events.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
          return APDVM_ERR_HIP;
        c->events.push_back({a, b});
      }
      ev.start = c->events[c->ev_used].first;
      ev.stop = c->events[c->ev_used].second;
      ++c->ev_used;
    }
    if (run_launch<T>(c, l, ev) != hipSuccess) return APDVM_ERR_HIP;
  }
  return APDVM_OK;
}

// Capture the plan of parity P into a graph (once).
template <typename T>
apdvm_status ensure_graph(apdvm_ctx *c, int P) {
  if (c->graph_exec[P]) return APDVM_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return APDVM_ERR_HIP;
  bool ok = true;
  for (const Launch &l : c->plan[P]) ok = ok && run_launch<T>(c, l) == hipSuccess;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (!ok || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return APDVM_ERR_HIP;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return APDVM_ERR_HIP;
  c->graph_exec[P] = ex;
  return APDVM_OK;
}

template <typename T>
apdvm_status enqueue_step(apdvm_ctx *c) {
  if (!c->terms_ready) {
    const apdvm_status st = stage0_terms<T>(c);
    if (st != APDVM_OK) return st;
  }
  const int P = c->parity;
  // a step whose launches of the timed class are bracketed by events runs launch by
  // launch on the main stream alone, so that the events see each launch by itself;
  // every other step replays the graph when graphs are on
  const bool sample = c->timed_class >= 0 && c->timed_steps % c->timed_stride == 0;
  if (c->use_graph && !sample) {
    apdvm_status st = ensure_graph<T>(c, P);
    if (st != APDVM_OK) return st;
    if (hipGraphLaunch(c->graph_exec[P], c->stream) != hipSuccess) return APDVM_ERR_HIP;
  } else {
    const bool overlap = c->overlap;
    if (sample) c->overlap = false;
    const apdvm_status st = run_plan_direct<T>(c, c->plan[P], sample);
    c->overlap = overlap;
    if (st != APDVM_OK) return st;
  }
  if (c->timed_class >= 0) ++c->timed_steps;
  c->parity = 1 - P;
  return APDVM_OK;
}

bool all_finite(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename T>
apdvm_status put_plane(apdvm_ctx *c, int k, int slot, const double *src, bool dev_src) {
  const Inst &I = c->inst[k];
  const size_t n = (size_t)I.plane;
  T *dst = reinterpret_cast<T *>(I.tbase) + (size_t)slot * n;
  if (sizeof(T) == sizeof(double)) {
    return hip_status(hipMemcpyAsync(dst, src, n * sizeof(double),
                                     dev_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                     c->stream));
  }
  if (dev_src)  // rounded to float on the device, in stream order
    return hip_status(launch_convert(dst, src, (long long)n, 1, c->stream));
  std::vector<T> t(n);
  for (size_t i = 0; i < n; ++i) t[i] = (T)src[i];
  if (hipMemcpyAsync(dst, t.data(), n * sizeof(T), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  return hip_status(hipStreamSynchronize(c->stream));
}

template <typename T>
apdvm_status get_plane(apdvm_ctx *c, int k, int slot, double *dst, bool dev_dst) {
  const Inst &I = c->inst[k];
  const size_t n = (size_t)I.plane;
  const T *src = reinterpret_cast<const T *>(I.tbase) + (size_t)slot * n;
  if (sizeof(T) == sizeof(double)) {
    return hip_status(hipMemcpyAsync(dst, src, n * sizeof(double),
                                     dev_dst ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                     c->stream));
  }
  if (dev_dst)  // widened to float64 on the device, in stream order
    return hip_status(launch_convert(dst, src, (long long)n, 0, c->stream));
  std::vector<T> t(n);
  if (hipMemcpyAsync(t.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  for (size_t i = 0; i < n; ++i) dst[i] = (double)t[i];
  return APDVM_OK;
}

apdvm_status put_state(apdvm_ctx *c, int k, const double *const f[6], bool dev) {
  const Layout &L = c->L;
  const int P = c->parity;
  const int tslots[5] = {L.st[P][0], L.st[P][1], L.st[P][2], L.st[P][3], L.st[P][4]};
  const int fidx[5] = {0, 1, 3, 4, 5};
  for (int m = 0; m < 5; ++m) {
    const apdvm_status st = c->split ? put_plane<float>(c, k, tslots[m], f[fidx[m]], dev)
                                     : put_plane<double>(c, k, tslots[m], f[fidx[m]], dev);
    if (st != APDVM_OK) return st;
  }
  const Inst &I = c->inst[k];
  const size_t nb = (size_t)I.plane * sizeof(double);
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (c->split)  // the float64 velocity beside its float copy
    for (int m = 0; m < 2; ++m)
      if (hipMemcpyAsync(I.dbase + (size_t)L.ud[P][m] * I.plane, f[m], nb, kind, c->stream) !=
          hipSuccess)
        return APDVM_ERR_HIP;
  double *th = I.dbase + (size_t)L.th[P] * I.plane;
  return hip_status(hipMemcpyAsync(th, f[2], nb, kind, c->stream));
}

apdvm_status get_state(apdvm_ctx *c, int k, double *const f[6], bool dev) {
  const Layout &L = c->L;
  const int P = c->parity;
  const int tslots[5] = {L.st[P][0], L.st[P][1], L.st[P][2], L.st[P][3], L.st[P][4]};
  const int fidx[5] = {0, 1, 3, 4, 5};
  for (int m = 0; m < 5; ++m) {
    if (!f[fidx[m]]) continue;
    if (c->split && m < 2) {  // the velocity from its float64 planes
      const Inst &I = c->inst[k];
      if (hipMemcpyAsync(f[m], I.dbase + (size_t)L.ud[P][m] * I.plane,
                         (size_t)I.plane * sizeof(double),
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         c->stream) != hipSuccess)
        return APDVM_ERR_HIP;
      continue;
    }
    const apdvm_status st = c->split ? get_plane<float>(c, k, tslots[m], f[fidx[m]], dev)
                                     : get_plane<double>(c, k, tslots[m], f[fidx[m]], dev);
    if (st != APDVM_OK) return st;
  }
  if (f[2]) {
    const Inst &I = c->inst[k];
    const double *th = I.dbase + (size_t)L.th[P] * I.plane;
    if (hipMemcpyAsync(f[2], th, (size_t)I.plane * sizeof(double),
                       dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return APDVM_ERR_HIP;
  }
  if (!dev) return hip_status(hipStreamSynchronize(c->stream));
  return APDVM_OK;
}

// The planes of state set P, or of the snapshot (P = -1).
StateSet state_set(const apdvm_ctx *c, int P) {
  const Layout &L = c->L;
  StateSet s;
  for (int f = 0; f < 5; ++f) s.t[f] = P < 0 ? L.ck[f] : L.st[P][f];
  s.d[0] = P < 0 ? L.thck : L.th[P];
  s.nd = 1;
  if (c->split) {
    for (int m = 0; m < 2; ++m) s.d[1 + m] = P < 0 ? L.ckud[m] : L.ud[P][m];
    s.nd = 3;
  }
  return s;
}

// Copy the state of instance k between state set P and the snapshot (to_snapshot: P ->
// snapshot, else snapshot -> P), enqueued on the stream.
apdvm_status copy_snapshot(apdvm_ctx *c, int k, int P, bool to_snapshot) {
  const Inst &I = c->inst[k];
  const size_t tb = (size_t)I.plane * (c->split ? sizeof(float) : sizeof(double));
  const size_t db = (size_t)I.plane * sizeof(double);
  const StateSet a = state_set(c, P), b = state_set(c, -1);
  char *tbase = static_cast<char *>(I.tbase);
  char *dbase = reinterpret_cast<char *>(I.dbase);
  for (int f = 0; f < 5 + a.nd; ++f) {
    char *base = f < 5 ? tbase : dbase;
    const size_t pb = f < 5 ? tb : db;
    const int sa = f < 5 ? a.t[f] : a.d[f - 5], sb = f < 5 ? b.t[f] : b.d[f - 5];
    char *x = base + (size_t)sa * pb, *y = base + (size_t)sb * pb;
    if (hipMemcpyAsync(to_snapshot ? y : x, to_snapshot ? x : y, pb, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return APDVM_ERR_HIP;
  }
  return APDVM_OK;
}

// Statistics of six device fields of n values (u, v, q float when split, theta float64):
// mean of theta, max |u|, all finite.
apdvm_status device_field_stats(apdvm_ctx *c, bool split, const void *const f[6], size_t n,
                                double *mean, double *umax, bool *finite) {
  std::vector<double> part(3 * (size_t)kStatBlocks);
  if (launch_field_stats(split ? 1 : 0, f, (long long)n, c->d_stats, kStatBlocks, c->stream) !=
          hipSuccess ||
      hipMemcpyAsync(part.data(), c->d_stats, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  long double s = 0.0L;
  double um = 0.0, fin = 1.0;
  for (int b = 0; b < kStatBlocks; ++b) {
    s += part[3 * b];
    um = std::fmax(um, part[3 * b + 1]);
    fin = std::fmin(fin, part[3 * b + 2]);
  }
  *mean = (double)(s / (long double)n);
  *umax = um;
  *finite = fin == 1.0 && std::isfinite((double)s);
  return APDVM_OK;
}

// After new fields for instance k (um: max |u| of the given float64 fields): the mean of
// theta from the stored state (one device reduction, whichever entry point brought the
// fields), dt derivation, parameter upload, and the snapshot of the finite check (the new
// fields are known to be finite).
apdvm_status after_fields(apdvm_ctx *c, int k, double um) {
  Inst &I = c->inst[k];
  {
    const StateSet ss = state_set(c, c->parity);
    const size_t n = (size_t)I.plane, tb = c->split ? sizeof(float) : sizeof(double);
    const void *f[5];
    for (int m = 0; m < 5; ++m)
      f[m] = static_cast<const char *>(I.tbase) + (size_t)ss.t[m] * n * tb;
    // the statistics take u1, u2, theta, v1, v2, q (u of the transport planes: only the
    // theta sum is used here)
    const void *g[6] = {f[0], f[1], I.dbase + (size_t)ss.d[0] * n, f[2], f[3], f[4]};
    double mean = 0.0, ignored = 0.0;
    bool finite = false;
    const apdvm_status st = device_field_stats(c, c->split, g, n, &mean, &ignored, &finite);
    if (st != APDVM_OK) return st;
    I.theta_mean = mean;
  }
  c->umax[k] = um;
  const apdvm_config &cf = c->cfg[k];
  if (!(cf.dt > 0.0)) {
    double ct = 0.0;
    for (int i = 0; i < c->s; ++i) {
      double r = 0.0;
      for (int j = 0; j < i; ++j) r += c->At[i][j];
      ct = std::fmax(ct, r);
    }
    if (ct <= 0.0) ct = 1.0;
    set_dt(c, k, derive_dt(cf, I.tau, um, ct));
    apdvm_log("instance %d: dt %.6g derived from max |u| %.6g", k, I.dt, um);
  }
  c->has_fields[k] = 1;
  c->terms_ready = false;
  apdvm_status st = upload_inst(c, k);
  if (st != APDVM_OK) return st;
  st = copy_snapshot(c, k, c->parity, true);
  if (st != APDVM_OK) return st;
  const long long step = c->step;
  return hip_status(hipMemcpyAsync(c->d_ck_step, &step, sizeof(step), hipMemcpyHostToDevice,
                                   c->stream)) == APDVM_OK
             ? hip_status(hipStreamSynchronize(c->stream))
             : APDVM_ERR_HIP;
}

}  // namespace

extern "C" {

const char *apdvm_status_string(apdvm_status s) {
  switch (s) {
    case APDVM_OK: return "ok";
    case APDVM_ERR_ARG: return "invalid argument";
    case APDVM_ERR_VELSET: return "velocity set is not the six-velocity hexagonal set";
    case APDVM_ERR_TABLEAU: return "tableau is not a GSA ARS-type IMEX Runge-Kutta tableau";
    case APDVM_ERR_NOMEM: return "out of device memory or workspace too small";
    case APDVM_ERR_HIP: return "HIP runtime error";
    case APDVM_ERR_NONFINITE: return "non-finite value";
    case APDVM_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

apdvm_status apdvm_workspace_bytes(int32_t n, const apdvm_config *cfgs, size_t *bytes) {
  if (!bytes) return APDVM_ERR_ARG;
  const apdvm_status st = validate(n, cfgs);
  if (st != APDVM_OK) return st;
  *bytes = workspace_bytes(n, cfgs);
  return APDVM_OK;
}

apdvm_status apdvm_create(int32_t n, const apdvm_config *cfgs, void *dev_ws, size_t ws_bytes,
                          void *hip_stream, apdvm_ctx **out) {
  if (!out) return APDVM_ERR_ARG;
  *out = nullptr;
  apdvm_status st = validate(n, cfgs);
  if (st != APDVM_OK) return st;
  const size_t need = workspace_bytes(n, cfgs);
  if (dev_ws && ws_bytes < need) return APDVM_ERR_NOMEM;

  apdvm_ctx *c = new (std::nothrow) apdvm_ctx;
  if (!c) return APDVM_ERR_NOMEM;
  c->n = n;
  c->s = internal_stages(cfgs[0]);
  c->split = cfgs[0].precision == APDVM_FP32_SPLIT;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->cfg.assign(cfgs, cfgs + n);
  for (int k = 0; k < n; ++k) {  // the caller's tableau arrays need not outlive the call
    c->cfg[k].a_ex = c->cfg[k].a_im = c->cfg[k].b_ex = c->cfg[k].b_im = nullptr;
    c->cfg[k].cx = c->cfg[k].cy = nullptr;
  }
  {
    const int s0 = cfgs[0].s, off = c->s - s0;  // off = 1: type A behind a zero stage
    for (int i = 0; i < c->s; ++i)
      for (int j = 0; j < c->s; ++j) c->At[i][j] = c->A[i][j] = 0.0;
    for (int i = 0; i < s0; ++i)
      for (int j = 0; j < s0; ++j) {
        c->At[i + off][j + off] = cfgs[0].a_ex[i * s0 + j];
        c->A[i + off][j + off] = cfgs[0].a_im[i * s0 + j];
      }
  }
  c->L = make_layout(c->s, c->split);
  c->has_fields.assign(n, 0);
  c->umax.assign(n, 0.0);
  if (hipGetDevice(&c->device) != hipSuccess || scratch_init(c->device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    apdvm_destroy(c);
    return APDVM_ERR_HIP;
  }
  if (dev_ws) {
    c->ws = static_cast<char *>(dev_ws);
    c->ws_bytes = ws_bytes;
  } else {
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      apdvm_destroy(c);
      return APDVM_ERR_NOMEM;
    }
    c->own_ws = true;
    c->ws_bytes = need;
  }

  // carve the workspace
  const size_t tsize = c->split ? sizeof(float) : sizeof(double);
  c->row_v = row_form(n, cfgs);
  c->row_split = c->row_v == 2;
  for (int k = 0; k < n; ++k) c->row_split = c->row_split && cfgs[k].nx % 4 == 0;
  c->col_v = col_form(n, cfgs);
  c->row_reg = fft_reg_form(n, cfgs, c->row_v, true);
  c->col_reg = fft_reg_form(n, cfgs, c->col_v, false);
  for (int k = 0; k < kNumClasses; ++k) c->shape[k] = 1;
  c->wo = weno_order_of(cfgs[0]);
  c->co = central_order_of(cfgs[0]);
  std::vector<Work> tiles8;
  char *p = c->ws;
  c->d_inst = reinterpret_cast<Inst *>(p);
  p += align_up(n * sizeof(Inst));
  c->inst.resize(n);
  std::vector<Work> rows, cols;
  std::vector<char> host_tables;
  struct Upload { char *dst; std::vector<char> data; };
  std::vector<Upload> uploads;
  for (int k = 0; k < n; ++k) {
    const apdvm_config &cf = cfgs[k];
    Inst &I = c->inst[k];
    std::memset(&I, 0, sizeof(I));
    I.nx = cf.nx;
    I.ny = cf.ny;
    I.plane = (long long)cf.nx * cf.ny;
    I.ihx = cf.nx / cf.lx;
    I.ihy = cf.ny / cf.ly;
    {
      const int co = central_order_of(cf);
      I.f1x = central_f1(co, I.ihx);
      I.f1y = central_f1(co, I.ihy);
      I.f2x = central_f2(co, I.ihx);
      I.f2y = central_f2(co, I.ihy);
    }
    I.eps = cf.eps;
    I.tau = resolved_tau(cf);
    I.te2 = I.tau * cf.eps * cf.eps;
    I.inv_nxny = 1.0 / ((double)cf.nx * cf.ny);
    const size_t plane = (size_t)I.plane;
    I.tbytes = (int)tsize;
    I.nt_slots = c->L.ntrans;
    I.nd_slots = c->L.ndbl;
    I.tbase = p;
    p += align_up(c->L.ntrans * plane * tsize);
    I.dbase = reinterpret_cast<double *>(p);
    p += align_up(c->L.ndbl * plane * sizeof(double));
    // two-level twiddle tables for lengths nx and ny
    I.fx.n = cf.nx;
    I.fx.npass = fft_radices(cf.nx, I.fx.radix);
    I.fy.n = cf.ny;
    I.fy.npass = fft_radices(cf.ny, I.fy.radix);
    double2 *tw2 = reinterpret_cast<double2 *>(p);
    p += align_up((size_t)2 * kTwCap * sizeof(double2));
    Upload u3{reinterpret_cast<char *>(tw2), std::vector<char>(2 * kTwCap * sizeof(double2))};
    double2 *htw2 = reinterpret_cast<double2 *>(u3.data.data());
    FftPlan *plans[2] = {&I.fx, &I.fy};
    for (int q = 0; q < 2; ++q) {
      plans[q]->ntw = twiddles2(plans[q]->n, htw2 + q * kTwCap, &plans[q]->lb);
      plans[q]->tw2 = tw2 + q * kTwCap;
      plans[q]->tsc = 1;
    }
    // half-length plans on the row and column tables (length n = 2 (n / 2))
    I.fxh = I.fx;
    I.fxh.n = cf.nx / 2;
    I.fxh.npass = fft_radices(cf.nx / 2, I.fxh.radix);
    I.fxh.tsc = 2;
    I.fyh = I.fy;
    I.fyh.n = cf.ny / 2;
    I.fyh.npass = fft_radices(cf.ny / 2, I.fyh.radix);
    I.fyh.tsc = 2;
    uploads.push_back(std::move(u3));
    // symbols
    double *lam = reinterpret_cast<double *>(p);
    p += align_up((size_t)(cf.nx / 2 + 1 + cf.ny) * sizeof(double));
    Upload u2{reinterpret_cast<char *>(lam),
              std::vector<char>((cf.nx / 2 + 1 + cf.ny) * sizeof(double))};
    double *hl = reinterpret_cast<double *>(u2.data.data());
    const int co = central_order_of(cf);
    for (int kx = 0; kx <= cf.nx / 2; ++kx) hl[kx] = lap_symbol(kx, cf.nx, cf.lx / cf.nx, co);
    for (int ky = 0; ky < cf.ny; ++ky)
      hl[cf.nx / 2 + 1 + ky] = lap_symbol(ky, cf.ny, cf.ly / cf.ny, co);
    uploads.push_back(std::move(u2));
    I.lam_x = lam;
    I.lam_y = lam + cf.nx / 2 + 1;
    I.row_pairs_per_block = rpb(cf, c->row_v);
    I.cols_per_block = cpb(cf, c->col_v);
    // work tables
    c->tile_first.push_back((int)c->tiles.size());
    for (int y0 = 0; y0 < cf.ny; y0 += kTileRows[1])
      for (int x0 = 0; x0 < cf.nx; x0 += kTileX) c->tiles.push_back(Work{k, x0, y0, 0});
    c->tile_count.push_back((int)c->tiles.size() - c->tile_first.back());
    for (int y0 = 0; y0 < cf.ny; y0 += kTileRows[0])
      for (int x0 = 0; x0 < cf.nx; x0 += kTileX) tiles8.push_back(Work{k, x0, y0, 0});
    for (int r0 = 0; r0 < cf.ny / 2; r0 += I.row_pairs_per_block) rows.push_back(Work{k, r0, 0, 0});
    for (int k0 = 0; k0 < cf.nx / 2; k0 += I.cols_per_block) cols.push_back(Work{k, k0, 0, 0});
    c->spec_bytes += (double)cf.ny * (cf.nx / 2) * 16.0;
    c->cfg[k] = cf;
    c->cfg[k].a_ex = c->cfg[k].a_im = c->cfg[k].b_ex = c->cfg[k].b_im = nullptr;
    c->cfg[k].cx = c->cfg[k].cy = nullptr;
    set_dt(c, k, cf.dt > 0.0 ? cf.dt : 0.0);
  }
  for (int k = 0; k < n; ++k) c->cells += (double)cfgs[k].nx * cfgs[k].ny;
  c->plan[0] = build_plan(c, 0);
  c->plan[1] = build_plan(c, 1);
  c->ntiles[1] = (int)c->tiles.size();
  c->ntiles[0] = (int)tiles8.size();
  c->nrows = (int)rows.size();
  c->ncols = (int)cols.size();
  c->d_tiles[1] = reinterpret_cast<Work *>(p);
  p += align_up(c->tiles.size() * sizeof(Work));
  c->d_tiles[0] = reinterpret_cast<Work *>(p);
  p += align_up(tiles8.size() * sizeof(Work));
  c->d_rows = reinterpret_cast<Work *>(p);
  p += align_up(rows.size() * sizeof(Work));
  c->d_cols = reinterpret_cast<Work *>(p);
  p += align_up(cols.size() * sizeof(Work));
  c->d_partials = reinterpret_cast<double *>(p);
  p += align_up(8 * sizeof(double) * 1024);
  c->d_stats = reinterpret_cast<double *>(p);
  p += align_up(3 * sizeof(double) * kStatBlocks);
  c->d_flag = reinterpret_cast<unsigned *>(p);
  c->d_ck_step = reinterpret_cast<long long *>(p + 8);
  p += align_up(kFlagBytes);
  c->finite_every = kDefaultFiniteEvery;
  if (const char *e = std::getenv("APDVM_FINITE_EVERY")) {
    char *end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (end != e && v >= 0 && v <= (1L << 30)) c->finite_every = (int)v;
  }

  bool ok = hipMemcpyAsync(c->d_tiles[1], c->tiles.data(), c->tiles.size() * sizeof(Work),
                           hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipMemcpyAsync(c->d_tiles[0], tiles8.data(), tiles8.size() * sizeof(Work),
                           hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipMemcpyAsync(c->d_rows, rows.data(), rows.size() * sizeof(Work),
                           hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipMemcpyAsync(c->d_cols, cols.data(), cols.size() * sizeof(Work),
                           hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipMemcpyAsync(c->d_inst, c->inst.data(), n * sizeof(Inst), hipMemcpyHostToDevice,
                           c->stream) == hipSuccess;
  for (auto &u : uploads)
    ok = ok && hipMemcpyAsync(u.dst, u.data.data(), u.data.size(), hipMemcpyHostToDevice,
                              c->stream) == hipSuccess;
  ok = ok && hipMemsetAsync(c->d_flag, 0, kFlagBytes, c->stream) == hipSuccess;
  ok = ok && hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    apdvm_destroy(c);
    return APDVM_ERR_HIP;
  }
  apdvm_log("create: %d instance(s), %s, %d internal stages, %zu workspace bytes (%s)", n,
            c->split ? "FP32-split" : "FP64", c->s, c->ws_bytes, c->own_ws ? "library" : "caller");
  *out = c;
  return APDVM_OK;
}

apdvm_status apdvm_set_fields(apdvm_ctx *c, int32_t k, const double *u1, const double *u2,
                              const double *theta, const double *v1, const double *v2,
                              const double *q) {
  if (!c || k < 0 || k >= c->n || !u1 || !u2 || !theta) return APDVM_ERR_ARG;
  if ((v1 == nullptr) != (v2 == nullptr)) return APDVM_ERR_ARG;
  const size_t n = (size_t)c->inst[k].plane;
  if (!all_finite(u1, n) || !all_finite(u2, n) || !all_finite(theta, n)) return APDVM_ERR_NONFINITE;
  if (v1 && (!all_finite(v1, n) || !all_finite(v2, n))) return APDVM_ERR_NONFINITE;
  if (q && !all_finite(q, n)) return APDVM_ERR_NONFINITE;
  std::vector<double> ev1, ev2, zq;
  if (!v1) {  // local equilibrium v = F(u)
    ev1.resize(n);
    ev2.resize(n);
    for (size_t i = 0; i < n; ++i) {
      ev1[i] = 0.5 * (u2[i] * u2[i] - u1[i] * u1[i]);
      ev2[i] = u1[i] * u2[i];
    }
    v1 = ev1.data();
    v2 = ev2.data();
  }
  if (!q) {
    zq.assign(n, 0.0);
    q = zq.data();
  }
  const double *f[6] = {u1, u2, theta, v1, v2, q};
  apdvm_status st = put_state(c, k, f, false);
  if (st != APDVM_OK) return st;
  double um = 0.0;
  for (size_t i = 0; i < n; ++i) um = std::fmax(um, std::sqrt(u1[i] * u1[i] + u2[i] * u2[i]));
  // after_fields synchronises: the copies read caller-owned and temporary host arrays
  return after_fields(c, k, um);
}

apdvm_status apdvm_set_fields_device(apdvm_ctx *c, int32_t k, const double *const dev[6]) {
  if (!c || k < 0 || k >= c->n || !dev) return APDVM_ERR_ARG;
  for (int m = 0; m < 6; ++m)
    if (!dev[m]) return APDVM_ERR_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return APDVM_ERR_HIP;
  // validate on the device before anything of the context changes: every value finite;
  // the same pass gives the mean of theta and max |u| for the dt rule
  const size_t n = (size_t)c->inst[k].plane;
  double mean = 0.0, um = 0.0;
  bool finite = false;
  const void *f[6] = {dev[0], dev[1], dev[2], dev[3], dev[4], dev[5]};
  apdvm_status st = device_field_stats(c, false, f, n, &mean, &um, &finite);
  if (st != APDVM_OK) return st;
  if (!finite) return APDVM_ERR_NONFINITE;
  st = put_state(c, k, dev, true);
  if (st != APDVM_OK) return st;
  return after_fields(c, k, um);  // synchronises
}

apdvm_status apdvm_set_populations(apdvm_ctx *c, int32_t k, const double *F) {
  if (!c || k < 0 || k >= c->n || !F) return APDVM_ERR_ARG;
  const double eps = c->inst[k].eps;
  if (!(eps > 0.0)) return APDVM_ERR_ARG;
  const size_t n = (size_t)c->inst[k].plane;
  if (!all_finite(F, 6 * n)) return APDVM_ERR_NONFINITE;
  // moment basis rows: 1, cx, cy, 1/2 - cx^2, cx cy, cx (cy^2 - 1/4)
  double m[6][6];
  for (int i = 0; i < 6; ++i) {
    const double cx = std::cos(M_PI * i / 3.0), cy = std::sin(M_PI * i / 3.0);
    m[0][i] = 1.0; m[1][i] = cx; m[2][i] = cy; m[3][i] = 0.5 - cx * cx; m[4][i] = cx * cy;
    m[5][i] = cx * (cy * cy - 0.25);
  }
  std::vector<double> f(6 * n);
  for (size_t x = 0; x < n; ++x) {
    double r[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 6; ++i)
      for (int a = 0; a < 6; ++a) r[a] += m[a][i] * F[i * n + x];
    f[0 * n + x] = r[1] / eps;                     // u1
    f[1 * n + x] = r[2] / eps;                     // u2
    f[2 * n + x] = (r[0] - 1.0) / (2 * eps * eps); // theta
    f[3 * n + x] = r[3] / (eps * eps);             // v1
    f[4 * n + x] = r[4] / (eps * eps);             // v2
    f[5 * n + x] = r[5] / (eps * eps * eps);       // q
  }
  return apdvm_set_fields(c, k, &f[0], &f[n], &f[2 * n], &f[3 * n], &f[4 * n], &f[5 * n]);
}

// Finite check of the current state of every instance, then the snapshot of it if the
// check (and every earlier one) passed.
static apdvm_status enqueue_check(apdvm_ctx *c) {
  const StateSet cur = state_set(c, c->parity), ck = state_set(c, -1);
  if (launch_state_finite(c->split ? 1 : 0, c->d_inst, c->d_tiles[1], c->ntiles[1], kTileRows[1],
                          cur, c->d_flag, c->stream) != hipSuccess ||
      launch_snapshot(c->split ? 1 : 0, c->d_inst, c->d_tiles[1], c->ntiles[1], kTileRows[1], cur,
                      ck, c->d_flag, c->d_ck_step, c->step, c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  return APDVM_OK;
}

// Read the flag of the checks enqueued so far (synchronises).  On a failed check: the
// snapshot (the last state that passed) becomes the current state, the step counter
// returns to its step, the flag is cleared, and APDVM_ERR_NONFINITE is returned.
static apdvm_status collect_checks(apdvm_ctx *c) {
  unsigned flag = 0;
  if (hipMemcpyAsync(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  if (!flag) return APDVM_OK;
  long long step = 0;
  if (hipMemcpyAsync(&step, c->d_ck_step, sizeof(step), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return APDVM_ERR_HIP;
  for (int k = 0; k < c->n; ++k)
    if (copy_snapshot(c, k, c->parity, false) != APDVM_OK) return APDVM_ERR_HIP;
  const unsigned zero = 0;
  if (hipMemcpyAsync(c->d_flag, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  apdvm_log("finite check failed: state of every instance restored to step %lld (was %lld)",
            step, (long long)c->step);
  c->step = step;
  c->terms_ready = false;
  return APDVM_ERR_NONFINITE;
}

apdvm_status apdvm_step(apdvm_ctx *c, int64_t nsteps) {
  if (!c || nsteps < 0) return APDVM_ERR_ARG;
  for (int k = 0; k < c->n; ++k)
    if (!c->has_fields[k]) return APDVM_ERR_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return APDVM_ERR_HIP;
  bool checked = false;
  for (int64_t t = 0; t < nsteps; ++t) {
    const apdvm_status st = c->split ? enqueue_step<float>(c) : enqueue_step<double>(c);
    if (st != APDVM_OK) return st;
    ++c->step;
    if (c->finite_every > 0 && c->step % c->finite_every == 0) {
      if (enqueue_check(c) != APDVM_OK) return APDVM_ERR_HIP;
      checked = true;
    }
  }
  return checked ? collect_checks(c) : APDVM_OK;
}

apdvm_status apdvm_set_finite_check(apdvm_ctx *c, int32_t every) {
  if (!c || every < 0) return APDVM_ERR_ARG;
  c->finite_every = every;
  return APDVM_OK;
}

apdvm_status apdvm_get_fields(apdvm_ctx *c, int32_t k, double *u1, double *u2, double *theta,
                              double *v1, double *v2, double *q) {
  if (!c || k < 0 || k >= c->n) return APDVM_ERR_ARG;
  if (!c->has_fields[k]) return APDVM_ERR_STATE;
  double *const f[6] = {u1, u2, theta, v1, v2, q};
  return get_state(c, k, f, false);
}

apdvm_status apdvm_get_fields_device(apdvm_ctx *c, int32_t k, double *const dev[6]) {
  if (!c || k < 0 || k >= c->n || !dev) return APDVM_ERR_ARG;
  if (!c->has_fields[k]) return APDVM_ERR_STATE;
  return get_state(c, k, dev, true);
}

apdvm_status apdvm_get_moments(apdvm_ctx *c, int32_t k, double *rho, double *u1, double *u2,
                               double *p) {
  if (!c || k < 0 || k >= c->n) return APDVM_ERR_ARG;
  const size_t n = (size_t)c->inst[k].plane;
  std::vector<double> a(n), b(n), th(n);
  apdvm_status st = apdvm_get_fields(c, k, a.data(), b.data(), th.data(), nullptr, nullptr, nullptr);
  if (st != APDVM_OK) return st;
  const double e2 = c->inst[k].eps * c->inst[k].eps;
  for (size_t i = 0; i < n; ++i) {
    if (rho) rho[i] = 1.0 + 2.0 * e2 * th[i];
    if (u1) u1[i] = a[i];
    if (u2) u2[i] = b[i];
    if (p) p[i] = th[i] - 0.5 * (a[i] * a[i] + b[i] * b[i]);
  }
  return APDVM_OK;
}

apdvm_status apdvm_get_populations(apdvm_ctx *c, int32_t k, double *F) {
  if (!c || k < 0 || k >= c->n || !F) return APDVM_ERR_ARG;
  const double eps = c->inst[k].eps;
  if (!(eps > 0.0)) return APDVM_ERR_ARG;
  const size_t n = (size_t)c->inst[k].plane;
  std::vector<double> f(6 * n);
  apdvm_status st = apdvm_get_fields(c, k, &f[0], &f[n], &f[2 * n], &f[3 * n], &f[4 * n], &f[5 * n]);
  if (st != APDVM_OK) return st;
  // F_i = sum_a m_a(i) M_a / |m_a|^2 (the basis is orthogonal with norms 6, 3, 3, 3/4,
  // 3/4, 3/8), with M = (1 + 2 eps^2 theta, eps u1, eps u2, eps^2 v1, eps^2 v2, eps^3 q).
  const double nrm[6] = {6.0, 3.0, 3.0, 0.75, 0.75, 0.375};
  for (int i = 0; i < 6; ++i) {
    const double cx = std::cos(M_PI * i / 3.0), cy = std::sin(M_PI * i / 3.0);
    const double m[6] = {1.0, cx, cy, 0.5 - cx * cx, cx * cy, cx * (cy * cy - 0.25)};
    for (size_t x = 0; x < n; ++x) {
      const double M[6] = {1.0 + 2.0 * eps * eps * f[2 * n + x], eps * f[x], eps * f[n + x],
                           eps * eps * f[3 * n + x], eps * eps * f[4 * n + x],
                           eps * eps * eps * f[5 * n + x]};
      double v = 0.0;
      for (int a = 0; a < 6; ++a) v += m[a] * M[a] / nrm[a];
      F[i * n + x] = v;
    }
  }
  return APDVM_OK;
}

apdvm_status apdvm_get_info(apdvm_ctx *c, int32_t k, double *dt, double *tau, int64_t *step) {
  if (!c || k < 0 || k >= c->n) return APDVM_ERR_ARG;
  if (dt) *dt = c->inst[k].dt;
  if (tau) *tau = c->inst[k].tau;
  if (step) *step = c->step;
  return APDVM_OK;
}

apdvm_status apdvm_set_step(apdvm_ctx *c, int64_t step) {
  if (!c || step < 0) return APDVM_ERR_ARG;
  c->step = step;
  return APDVM_OK;
}

apdvm_status apdvm_diagnostics(apdvm_ctx *c, int32_t k, double out[8]) {
  if (!c || k < 0 || k >= c->n || !out) return APDVM_ERR_ARG;
  if (!c->has_fields[k]) return APDVM_ERR_STATE;
  const Layout &L = c->L;
  const int P = c->parity;
  const int nblk = c->tile_count[k];
  const int cap = 1024;
  const int used = nblk < cap ? nblk : cap;
  // the velocity from its float64 planes (the transport planes in FP64, the float64
  // velocity of the FP32-split form)
  const int su1 = c->split ? L.ud[P][0] : L.st[P][0], su2 = c->split ? L.ud[P][1] : L.st[P][1];
  if (launch_diagnostics(c->d_inst, c->d_tiles[1] + c->tile_first[k], nblk, kTileRows[1],
                         c->split ? 1 : 0, su1, su2, L.th[P], L.st[P][2], L.st[P][3], L.st[P][4],
                         c->co, c->d_partials, used, c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  std::vector<double> part(8 * (size_t)used);
  if (hipMemcpyAsync(part.data(), c->d_partials, part.size() * sizeof(double),
                     hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  const Inst &I = c->inst[k];
  const double area = (1.0 / I.ihx) * (1.0 / I.ihy);
  double acc[8] = {0, 0, 0, 0, 1e300, -1e300, 0, 1};
  for (int b = 0; b < used; ++b) {
    const double *q = &part[8 * (size_t)b];
    acc[0] += q[0]; acc[1] += q[1]; acc[2] += q[2];
    acc[3] = std::fmax(acc[3], q[3]);
    acc[4] = std::fmin(acc[4], q[4]);
    acc[5] = std::fmax(acc[5], q[5]);
    acc[6] += q[6];
    acc[7] = std::fmin(acc[7], q[7]);
  }
  out[0] = acc[0] * area; out[1] = acc[1] * area; out[2] = acc[2] * area;
  out[3] = acc[3]; out[4] = acc[4]; out[5] = acc[5];
  out[6] = 0.5 * acc[6] * area; out[7] = acc[7];
  return APDVM_OK;
}

apdvm_status apdvm_diagnostics_device(apdvm_ctx *c, int32_t k, double *dev_out) {
  if (!c || k < 0 || k >= c->n || !dev_out) return APDVM_ERR_ARG;
  if (!c->has_fields[k]) return APDVM_ERR_STATE;
  double *part = scratch_ptr(c->device);
  if (!part) return APDVM_ERR_HIP;
  const Layout &L = c->L;
  const int P = c->parity;
  const int nblk = c->tile_count[k];
  // one partial record per workgroup, at most scratch_blocks() of them (the workgroups
  // loop over the tiles of larger instances), so no instance size exceeds the scratch
  const int used = nblk < scratch_blocks() ? nblk : scratch_blocks();
  if (used < 1 || used > scratch_blocks()) return APDVM_ERR_ARG;
  const int su1 = c->split ? L.ud[P][0] : L.st[P][0], su2 = c->split ? L.ud[P][1] : L.st[P][1];
  const Inst &I = c->inst[k];
  const double area = (1.0 / I.ihx) * (1.0 / I.ihy);
  if (launch_diagnostics(c->d_inst, c->d_tiles[1] + c->tile_first[k], nblk, kTileRows[1],
                         c->split ? 1 : 0, su1, su2, L.th[P], L.st[P][2], L.st[P][3], L.st[P][4],
                         c->co, part, used, c->stream) != hipSuccess ||
      launch_diag_finish(part, used, area, dev_out, c->stream) != hipSuccess)
    return APDVM_ERR_HIP;
  return APDVM_OK;
}

apdvm_status apdvm_launches_per_step(apdvm_ctx *c, int32_t *count) {
  if (!c || !count) return APDVM_ERR_ARG;
  int32_t n = 0;
  for (const Launch &l : c->plan[0]) n += l.cls != kSync;
  *count = n;
  return APDVM_OK;
}

apdvm_status apdvm_set_graph(apdvm_ctx *c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return APDVM_ERR_ARG;
  if (on && c->stream == nullptr) return APDVM_ERR_ARG;  // capture needs a created stream
  c->use_graph = on != 0;
  return APDVM_OK;
}

apdvm_status apdvm_set_overlap(apdvm_ctx *c, int32_t on) {
  if (!c || on < 0 || on > 2) return APDVM_ERR_ARG;
  const bool ov = on == 1, fz = on == 2;
  if (c->overlap == ov && c->fused == fz) return APDVM_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipStreamSynchronize(c->side) != hipSuccess)
    return APDVM_ERR_HIP;
  c->overlap = ov;
  if (c->fused != fz) {
    c->fused = fz;
    c->plan[0] = build_plan(c, 0);
    c->plan[1] = build_plan(c, 1);
  }
  for (int p = 0; p < 2; ++p)  // the graphs captured the other stream structure
    if (c->graph_exec[p]) {
      (void)hipGraphExecDestroy(c->graph_exec[p]);
      c->graph_exec[p] = nullptr;
    }
  return APDVM_OK;
}

apdvm_status apdvm_get_overlap(apdvm_ctx *c, int32_t *on) {
  if (!c || !on) return APDVM_ERR_ARG;
  *on = c->fused ? 2 : c->overlap ? 1 : 0;
  return APDVM_OK;
}

apdvm_status apdvm_timing_enable(apdvm_ctx *c, int32_t cls) {
  if (!c || cls < -1 || cls >= kNumClasses) return APDVM_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return APDVM_ERR_HIP;
  c->timed_class = cls;
  c->ev_used = 0;
  c->timed_steps = 0;
  return APDVM_OK;
}

apdvm_status apdvm_timing_stride(apdvm_ctx *c, int32_t stride) {
  if (!c || stride < 1) return APDVM_ERR_ARG;
  c->timed_stride = stride;
  return APDVM_OK;
}

apdvm_status apdvm_timing_read(apdvm_ctx *c, int64_t *launches, double *total_ms) {
  if (!c || !launches || !total_ms) return APDVM_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return APDVM_ERR_HIP;
  double tot = 0.0;
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->events[i].first, c->events[i].second) != hipSuccess)
      return APDVM_ERR_HIP;
    tot += ms;
  }
  *launches = (int64_t)c->ev_used;
  *total_ms = tot;
  return APDVM_OK;
}

apdvm_status apdvm_traffic(apdvm_ctx *c, int32_t cls, double *bytes_per_step,
                           int32_t *launches_per_step) {
  if (!c || !bytes_per_step || !launches_per_step || cls < -1 || cls >= kNumClasses)
    return APDVM_ERR_ARG;
  double b = 0.0;
  int n = 0;
  for (const Launch &l : c->plan[0]) {
    if (l.cls == kSync || (cls >= 0 && l.cls != cls)) continue;
    b += l.bytes;
    ++n;
  }
  *bytes_per_step = b;
  *launches_per_step = n;
  return APDVM_OK;
}

static void drop_graphs(apdvm_ctx *c) {
  for (int p = 0; p < 2; ++p)
    if (c->graph_exec[p]) {
      (void)hipGraphExecDestroy(c->graph_exec[p]);
      c->graph_exec[p] = nullptr;
    }
}

// Autotuner: for each stencil kernel class, time every launch shape on the live data
// with HIP events and keep the fastest, then the stream structure over whole steps; the
// state is restored afterwards.  With the environment variable APDVM_TUNE_CACHE naming a
// file, choices are looked up there by a key of the context's shape and appended after
// tuning.
static std::string tune_key(const apdvm_ctx *c) {
  std::ostringstream k;
  k << "gfx950 shapes4 overlap gradq colmajor fused prec=" << (c->split ? "fp32split" : "fp64") << " s=" << c->s << " n=" << c->n
    << " cells=" << (long long)c->cells << " weno=" << c->wo << " central=" << c->co;
  int mx = 0;
  for (const auto &cf : c->cfg) mx = cf.nx > mx ? cf.nx : mx;
  k << " maxnx=" << mx;
  return k.str();
}

apdvm_status apdvm_autotune(apdvm_ctx *c, int32_t steps_per_trial, int32_t *choice) {
  if (!c || steps_per_trial < 1) return APDVM_ERR_ARG;
  for (int k = 0; k < c->n; ++k)
    if (!c->has_fields[k]) return APDVM_ERR_STATE;
  const int *classes = kTunedClasses;
  const char *cache = std::getenv("APDVM_TUNE_CACHE");
  const std::string key = tune_key(c);
  bool cached = false;
  if (cache) {
    std::ifstream in(cache);
    std::string line;
    while (std::getline(in, line)) {
      if (line.compare(0, key.size(), key) == 0 && line.size() > key.size() &&
          line[key.size()] == '|') {
        std::istringstream rest(line.substr(key.size() + 1));
        int t[kNumTuned], ov = 1;
        bool good = true;
        for (int m = 0; m < kNumTuned; ++m) good = good && (rest >> t[m]) && t[m] >= 0 && t[m] < kNumShapes;
        if (good && rest >> ov) {
          for (int m = 0; m < kNumTuned; ++m) c->shape[classes[m]] = t[m];
          if (apdvm_set_overlap(c, ov >= 0 && ov <= 2 ? ov : 1) != APDVM_OK)
            return APDVM_ERR_HIP;
          cached = true;
        }
      }
    }
  }
  if (!cached) {
    // snapshot the current state of every instance
    const int P = c->parity;
    const size_t tsz = c->split ? sizeof(float) : sizeof(double);
    size_t total = 0;
    const StateSet cur = state_set(c, P);
    for (const Inst &I : c->inst) total += (size_t)I.plane * (5 * tsz + cur.nd * sizeof(double));
    char *snap = nullptr;
    if (hipMalloc(&snap, total) != hipSuccess) return APDVM_ERR_NOMEM;
    auto copy_state = [&](bool save) {
      char *q = snap;
      bool ok = true;
      for (const Inst &I : c->inst) {
        const size_t pb = (size_t)I.plane * tsz;
        for (int f = 0; f < 5; ++f) {
          char *dev = static_cast<char *>(I.tbase) + (size_t)cur.t[f] * pb;
          ok = ok && hipMemcpyAsync(save ? q : dev, save ? dev : q, pb, hipMemcpyDeviceToDevice,
                                    c->stream) == hipSuccess;
          q += pb;
        }
        const size_t db = (size_t)I.plane * sizeof(double);
        for (int m = 0; m < cur.nd; ++m) {
          char *dp = reinterpret_cast<char *>(I.dbase + (size_t)cur.d[m] * I.plane);
          ok = ok && hipMemcpyAsync(save ? q : dp, save ? dp : q, db, hipMemcpyDeviceToDevice,
                                    c->stream) == hipSuccess;
          q += db;
        }
      }
      return ok;
    };
    const int64_t step0 = c->step;
    const bool graph = c->use_graph;
    const int stride = c->timed_stride;
    const int every = c->finite_every;
    c->finite_every = 0;  // the trial steps are not part of the run
    c->use_graph = false;
    c->timed_stride = 1;
    bool ok = copy_state(true);
    // launch shapes, once with the split kernels (structures 0 and 1) and once with the
    // fused update and stage-terms kernels of structure 2, whose registers and bytes differ
    int shp[2][kNumTuned];
    for (int f = 0; f < 2; ++f) {
      ok = ok && apdvm_set_overlap(c, f ? 2 : 1) == APDVM_OK;
      for (int m = 0; ok && m < kNumTuned; ++m) {
        const int cls = classes[m];
        double best = 1e300;
        int best_si = 1;
        for (int si = 0; ok && si < kNumShapes; ++si) {
          c->shape[cls] = si;
          ok = apdvm_step(c, 1) == APDVM_OK;  // warm-up with this choice
          ok = ok && apdvm_timing_enable(c, cls) == APDVM_OK;
          ok = ok && apdvm_step(c, steps_per_trial) == APDVM_OK;
          int64_t nl = 0;
          double ms = 0.0;
          ok = ok && apdvm_timing_read(c, &nl, &ms) == APDVM_OK;
          if (ok && ms < best) {
            best = ms;
            best_si = si;
          }
        }
        c->shape[cls] = best_si;
        shp[f][m] = best_si;
      }
      ok = ok && apdvm_timing_enable(c, -1) == APDVM_OK;
    }
    auto use_shapes = [&](int structure) {
      for (int m = 0; m < kNumTuned; ++m) c->shape[classes[m]] = shp[structure == 2][m];
    };
    // the stream structure (one stream, the solve beside steps 3 and 4, or one stream with
    // the theta completion fused into the update): whole steps timed on the main stream
    ok = ok && apdvm_timing_enable(c, -1) == APDVM_OK;
    c->use_graph = graph;  // the stream structures compete in the caller's launch mode
    drop_graphs(c);        // graphs of earlier launch shapes
    if (ok) {
      // two passes over the three structures, interleaved (0, 1, 2, 0, 1, 2) so that a
      // drift of the clock or of other work on the device hits all alike; each timed run
      // has at least 2 steps_per_trial steps and, once the step time is known, enough
      // steps for about 10 ms
      double tov[3] = {0.0, 0.0, 0.0};
      int nsteps = 2 * steps_per_trial;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
      for (int t = 0; ok && t < 6; ++t) {
        const int on = t % 3;
        // two warm-up steps: in graph mode each parity's graph is captured and uploaded
        // before the timed steps
        use_shapes(on);
        drop_graphs(c);
        ok = apdvm_set_overlap(c, on) == APDVM_OK && apdvm_step(c, 2) == APDVM_OK;
        ok = ok && hipEventRecord(e0, c->stream) == hipSuccess;
        ok = ok && apdvm_step(c, nsteps) == APDVM_OK;
        ok = ok && hipEventRecord(e1, c->stream) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        tov[on] += ms / nsteps;
        if (t == 0 && ms > 0.0f && ms < 10.0f) {
          const int want = (int)(10.0f / (ms / nsteps)) + 1;
          nsteps = want > 64 ? 64 : (want > nsteps ? want : nsteps);
        }
      }
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      int best = 1;  // ties keep the solve beside the update
      for (int on = 0; on < 3; ++on)
        if (tov[on] < tov[best]) best = on;
      use_shapes(best);
      ok = ok && apdvm_set_overlap(c, best) == APDVM_OK;
    }
    c->parity = P;
    ok = ok && copy_state(false) && hipStreamSynchronize(c->stream) == hipSuccess;
    (void)hipFree(snap);
    c->terms_ready = false;
    c->step = step0;
    c->use_graph = graph;
    c->timed_stride = stride;
    c->finite_every = every;
    if (!ok) return APDVM_ERR_HIP;
    if (cache) {
      std::ofstream out(cache, std::ios::app);
      out << key << "|";
      for (int m = 0; m < kNumTuned; ++m) out << c->shape[classes[m]] << " ";
      out << (c->fused ? 2 : c->overlap ? 1 : 0) << "\n";
    }
  }
  drop_graphs(c);  // the graphs captured the old launch shapes
  apdvm_log("autotune (%s): tile rows / threads %d/%d %d/%d %d/%d %d/%d for classes 0 4 5 6, "
            "stream structure %d", cached ? "cache" : "timed",
            kShapeRows[c->shape[classes[0]]], kShapeThreads[c->shape[classes[0]]],
            kShapeRows[c->shape[classes[1]]], kShapeThreads[c->shape[classes[1]]],
            kShapeRows[c->shape[classes[2]]], kShapeThreads[c->shape[classes[2]]],
            kShapeRows[c->shape[classes[3]]], kShapeThreads[c->shape[classes[3]]],
            c->fused ? 2 : c->overlap ? 1 : 0);
  if (choice) {
    for (int k = 0; k < kNumClasses; ++k) choice[k] = 1;
    for (int m = 0; m < kNumTuned; ++m) {
      choice[classes[m]] = kShapeRows[c->shape[classes[m]]];
      choice[kNumClasses + m] = kShapeThreads[c->shape[classes[m]]];
    }
  }
  return APDVM_OK;
}

apdvm_status apdvm_set_tuning(apdvm_ctx *c, const int32_t *choice) {
  if (!c || !choice) return APDVM_ERR_ARG;
  const int *classes = kTunedClasses;
  int si[kNumTuned];
  for (int m = 0; m < kNumTuned; ++m) {
    si[m] = shape_of(choice[classes[m]], choice[kNumClasses + m]);
    if (si[m] < 0) return APDVM_ERR_ARG;
  }
  for (int m = 0; m < kNumTuned; ++m) c->shape[classes[m]] = si[m];
  drop_graphs(c);
  return APDVM_OK;
}

apdvm_status apdvm_batch_create(int32_t n, const apdvm_config *cfgs, void *dev_ws,
                                size_t ws_bytes, void *hip_stream, apdvm_batch **out) {
  return apdvm_create(n, cfgs, dev_ws, ws_bytes, hip_stream, out);
}

apdvm_status apdvm_batch_set_fields(apdvm_batch *b, int32_t k, const double *u1,
                                    const double *u2, const double *theta, const double *v1,
                                    const double *v2, const double *q) {
  return apdvm_set_fields(b, k, u1, u2, theta, v1, v2, q);
}

apdvm_status apdvm_batch_step(apdvm_batch *b, int64_t nsteps) { return apdvm_step(b, nsteps); }

apdvm_status apdvm_batch_get_fields(apdvm_batch *b, int32_t k, double *u1, double *u2,
                                    double *theta, double *v1, double *v2, double *q) {
  return apdvm_get_fields(b, k, u1, u2, theta, v1, v2, q);
}

void apdvm_batch_destroy(apdvm_batch *b) { apdvm_destroy(b); }

void apdvm_destroy(apdvm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  for (int p = 0; p < 2; ++p)
    if (c->graph_exec[p]) (void)hipGraphExecDestroy(c->graph_exec[p]);
  for (auto &e : c->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

}  // extern "C"
