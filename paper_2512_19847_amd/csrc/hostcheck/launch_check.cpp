// The kernel launches of the library, for the bounds-checked CPU build (APDVM_HOSTCHECK):
// every launch_* function the host code calls is defined here instead of in the HIP
// sources.  Instead of running a kernel, each walks the launch's whole index space with
// the index maps the kernels themselves use (xcd_remap, staged_cell, wrap_index from
// common.hpp) and checks, at the time the launch would run (at once, or at graph replay):
//  * the workgroup-to-work-item map is a bijection and every work item and Inst entry
//    lies in device memory;
//  * every stencil tile lies on its instance's grid, and the tiles cover every cell of
//    every instance exactly once;
//  * every staged halo element (halos of 1 to 5 cells) and every wrapped neighbour
//    index is the periodic image of its cell, inside the plane;
//  * every plane slot an argument names exists in its arena (transport or float64),
//    the arenas and tables lie in device memory without overlapping, and no launch
//    writes a plane it also reads, or writes one plane twice (the in-place Hu update
//    excepted);
//  * FFT row blocks and column strips fit the kernel form's LDS capacity and cover every
//    row pair and column of every instance exactly once, and every plan's radices
//    multiply to its length.
// The small kernels whose results the host reads back (input statistics, conversion,
// finite check, snapshot, diagnostics combine) are computed on the CPU, so the host
// logic around them runs as it does on the GPU; the stencil and FFT launches change
// nothing.
#include "common.hpp"
#include "hostcheck.hpp"

#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

namespace apdvm {

using hostcheck::fail;
using hostcheck::in_device;

namespace {

// Tile rows of the four stencil launch shapes (as dispatched by the stencil launches:
// 0 = 64 x 8 on 256 threads, 1 = 64 x 16 on 256, 2 = 64 x 16 on 512, 3 = 64 x 8 on 512).
constexpr int kRowsOfShape[4] = {8, 16, 16, 8};

int pmod(int a, int n) { return ((a % n) + n) % n; }

hostcheck::Counters &cnt() { return hostcheck::counters(); }

// The Inst of instance k, checked once per launch.
const Inst *inst_of(const Inst *insts, int k, size_t tsz, std::set<int> &seen) {
  if (k < 0 || !in_device(insts + k, sizeof(Inst))) {
    fail("work item names instance %d outside the instance table", k);
    return nullptr;
  }
  const Inst &I = insts[k];
  if (seen.insert(k).second) {
    if (I.tbytes != 4 && I.tbytes != 8) fail("instance %d: transport value of %d bytes", k, I.tbytes);
    if (tsz && tsz != (size_t)I.tbytes)
      fail("instance %d: launch for %zu-byte transport values on a %d-byte arena", k, tsz,
           I.tbytes);
    tsz = (size_t)I.tbytes;
    if (I.nx < 8 || I.ny < 8 || I.nx > kFftCap || I.ny > kFftCap || (I.nx & 1) || (I.ny & 1) ||
        I.plane != (long long)I.nx * I.ny)
      fail("instance %d: grid %d x %d, plane %lld", k, I.nx, I.ny, I.plane);
    const size_t pb = (size_t)I.plane;
    const size_t tbytes = (size_t)I.nt_slots * pb * tsz, dbytes = (size_t)I.nd_slots * pb * 8;
    if (I.nt_slots <= 0 || !in_device(I.tbase, tbytes))
      fail("instance %d: transport arena of %d planes outside device memory", k, I.nt_slots);
    if (I.nd_slots <= 0 || !in_device(I.dbase, dbytes))
      fail("instance %d: float64 arena of %d planes outside device memory", k, I.nd_slots);
    const char *t0 = static_cast<const char *>(I.tbase), *d0 = reinterpret_cast<const char *>(I.dbase);
    if (t0 < d0 + dbytes && d0 < t0 + tbytes) fail("instance %d: arenas overlap", k);
    const char *it = reinterpret_cast<const char *>(insts + k);
    if ((it >= t0 && it < t0 + tbytes) || (it >= d0 && it < d0 + dbytes))
      fail("instance %d: the instance table lies inside an arena", k);
    const FftPlan *plans[3] = {&I.fx, &I.fy, &I.fyh};
    const int lens[3] = {I.nx, I.ny, I.ny / 2};
    for (int q = 0; q < 3; ++q) {
      const FftPlan &P = *plans[q];
      long long prod = 1;
      bool ok = P.n == lens[q] && P.npass >= 1 && P.npass <= kMaxPasses;
      for (int s = 0; ok && s < P.npass; ++s) {
        const int r = P.radix[s];
        ok = r == 2 || r == 3 || r == 4 || r == 8;
        prod *= r;
      }
      if (!ok || prod != P.n) fail("instance %d: FFT plan %d of length %d malformed", k, q, P.n);
      const int tl = (q == 2 ? 2 : 1) * P.n;  // the table belongs to the length tsc n
      if (P.tsc != (q == 2 ? 2 : 1) || P.ntw > kTwCap || P.ntw <= 0 ||
          !in_device(P.tw2, (size_t)P.ntw * sizeof(double2)) || (1LL << (2 * P.lb)) < tl)
        fail("instance %d: twiddle table of plan %d", k, q);
    }
    if (!in_device(I.lam_x, (size_t)(I.nx / 2 + 1) * 8) || !in_device(I.lam_y, (size_t)I.ny * 8))
      fail("instance %d: symbol tables outside device memory", k);
    if (I.row_pairs_per_block < 1 || I.cols_per_block < 1)
      fail("instance %d: FFT blocking %d %d", k, I.row_pairs_per_block, I.cols_per_block);
  }
  return &I;
}

// The workgroup-to-item map over nwork workgroups is a bijection.
void check_remap(int nwork) {
  std::vector<char> hit(nwork > 0 ? nwork : 1, 0);
  for (int b = 0; b < nwork; ++b) {
    const int i = xcd_remap(b, nwork);
    if (i < 0 || i >= nwork || hit[i]) {
      fail("xcd_remap(%d, %d) = %d is not a bijection", b, nwork, i);
      return;
    }
    hit[i] = 1;
  }
}

// FNV-1a hash of a work table's contents: tables are walked once per distinct content.
unsigned long long table_hash(const Work *w, int n) {
  unsigned long long h = 1469598103934665603ull;
  if (n <= 0 || !in_device(w, (size_t)n * sizeof(Work))) return h;
  const unsigned char *p = reinterpret_cast<const unsigned char *>(w);
  for (size_t i = 0; i < (size_t)n * sizeof(Work); ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

// Plane slot sets of one launch: reads and writes per arena (0 transport, 1 float64).
struct Slots {
  const char *what;
  std::vector<std::pair<int, int>> rd, wr;  // (arena, slot)
  std::set<std::pair<int, int>> inplace;
  void r(int arena, int s, bool optional = false) { add(rd, arena, s, optional); }
  void w(int arena, int s, bool optional = false) { add(wr, arena, s, optional); }
  void add(std::vector<std::pair<int, int>> &v, int arena, int s, bool optional) {
    if (s == kNoSlot) {
      if (!optional) fail("%s: a required plane slot is unset", what);
      return;
    }
    v.push_back({arena, s});
  }
  void check(const Inst &I, int k) const {
    for (auto *v : {&rd, &wr})
      for (auto [a, s] : *v)
        if (s < 0 || s >= (a == 0 ? I.nt_slots : I.nd_slots))
          fail("%s: instance %d slot %d of arena %d out of range", what, k, s, a);
    std::set<std::pair<int, int>> w(wr.begin(), wr.end());
    if (w.size() != wr.size()) fail("%s: one plane written twice", what);
    for (auto x : rd)
      if (w.count(x) && !inplace.count(x))
        fail("%s: plane %d of arena %d both read and written", what, x.second, x.first);
  }
};

// Stencil tiles (64 x TY) of one launch: bounds, coverage, staged halo and wrapped
// neighbour indices.  A tile table is walked once per (table, instance table, tile rows);
// the slots of every launch are checked every time.
void check_tiles(const Inst *insts, const Work *work, int nwork, int TY, size_t tsz,
                 const Slots &sl) {
  ++cnt().launches;
  static std::set<std::tuple<const void *, unsigned long long, int, int>> walked;
  if (in_device(work, (size_t)nwork * sizeof(Work)) &&
      !walked.insert({insts, table_hash(work, nwork), nwork, TY}).second) {
    std::set<int> seen;
    for (int b = 0; b < nwork; ++b) seen.insert(work[b].inst);
    for (int k : seen) {
      std::set<int> once;
      if (inst_of(insts, k, tsz, once)) sl.check(insts[k], k);
    }
    return;
  }
  check_remap(nwork);
  std::set<int> seen;
  std::map<int, std::vector<char>> cover;
  for (int b = 0; b < nwork; ++b) {
    const Work *w = work + xcd_remap(b, nwork);
    if (!in_device(w, sizeof(Work))) {
      fail("work item %d outside device memory", b);
      return;
    }
    ++cnt().items;
    const Inst *Ip = inst_of(insts, w->inst, tsz, seen);
    if (!Ip) return;
    const Inst &I = *Ip;
    const int nx = I.nx, ny = I.ny, x0 = w->a, y0 = w->b;
    if (x0 < 0 || x0 >= nx || y0 < 0 || y0 >= ny || x0 % kTileX || y0 % TY) {
      fail("tile (%d, %d) of instance %d off its %d x %d grid (tile rows %d)", x0, y0, w->inst, nx,
           ny, TY);
      continue;
    }
    const int tx = (nx + kTileX - 1) / kTileX, tyn = (ny + TY - 1) / TY;
    auto &cv = cover[w->inst];
    if (cv.empty()) cv.assign((size_t)tx * tyn, 0);
    char &c = cv[(size_t)(y0 / TY) * tx + x0 / kTileX];
    if (c) fail("tile (%d, %d) of instance %d listed twice", x0, y0, w->inst);
    c = 1;
    for (int H = 1; H <= kHalo + 2; ++H) {
      const int W = kTileX + 2 * H, PL = W * (TY + 2 * H);
      const bool inner = x0 >= H && x0 + kTileX + H <= nx && y0 >= H && y0 + TY + H <= ny;
      for (int idx = 0; idx < PL; ++idx) {
        const int ly = idx / W, lx = idx % W;
        const int want = pmod(y0 + ly - H, ny) * nx + pmod(x0 + lx - H, nx);
        const int got = staged_cell(idx, W, H, nx, ny, x0, y0, inner);
        if (got != want) {
          fail("instance %d tile (%d, %d) halo %d: staged element %d reads cell %d, not %d",
               w->inst, x0, y0, H, idx, got, want);
          break;
        }
      }
      cnt().indices += PL;
    }
    for (int y = y0; y < y0 + TY && y < ny; ++y)
      for (int x = x0; x < x0 + kTileX && x < nx; ++x)
        for (int k = -2; k <= 2; ++k) {
          if (wrap_index(x + k, nx) != pmod(x + k, nx) || wrap_index(y + k, ny) != pmod(y + k, ny))
            fail("wrapped neighbour %+d of cell (%d, %d) on %d x %d", k, x, y, nx, ny);
          cnt().indices += 2;
        }
  }
  for (auto &[k, cv] : cover)
    for (char c : cv)
      if (!c) {
        fail("%s: a tile of instance %d is missing", sl.what, k);
        break;
      }
  for (int k : seen) sl.check(insts[k], k);
}

bool shape_ok(int si, int wo, int co) {
  return si >= 0 && si < 4 && (wo == 5 || wo == 3) && (co == 4 || co == 2);
}

template <typename T>
void history(Slots &s, int n, const int (*p)[2]) {
  for (int j = 0; j < n; ++j) {
    s.r(0, p[j][0]);
    s.r(0, p[j][1]);
  }
}

}  // namespace

// ---------------------------------------------------------------- stencil launches

template <typename T>
hipError_t launch_helmholtz_rhs(int si, int wo, int co, const Inst *insts, const Work *work,
                                int nwork, const ArgsR &a, hipStream_t st, const Ev &) {
  if (!shape_ok(si, wo, co)) fail("helmholtz_rhs: launch shape %d %d %d", si, wo, co);
  hostcheck::enqueue(st, [=] {
    Slots s{"helmholtz_rhs"};
    if (a.stage < 1 || a.stage >= kMaxStages || !(a.aii > 0.0) || a.nD < 0 || a.nD > kMaxStages ||
        a.nL < 0 || a.nL > kMaxStages)
      fail("helmholtz_rhs: stage %d, a_ii %g, nD %d, nL %d", a.stage, a.aii, a.nD, a.nL);
    s.r(0, a.v[0]);
    s.r(0, a.v[1]);
    s.r(1, a.thn);
    s.r(a.du0_dbl ? 1 : 0, a.du0);
    for (int j = 0; j < a.nD; ++j) s.r(0, a.D[j]);
    for (int j = 0; j < a.nL; ++j) s.r(0, a.L[j]);
    s.w(1, a.out_r);
    s.w(0, a.out_ddb);
    check_tiles(insts, work, nwork, kRowsOfShape[si & 3], sizeof(T), s);
  });
  return hipSuccess;
}

template <typename T>
hipError_t launch_update_uq(int si, int wo, int co, const Inst *insts, const Work *work,
                            int nwork, const ArgsUQ &a, hipStream_t st, const Ev &) {
  if (!shape_ok(si, wo, co)) fail("update_uq: launch shape %d %d %d", si, wo, co);
  hostcheck::enqueue(st, [=] {
    Slots s{"update_uq"};
    if (a.stage < 1 || a.stage >= kMaxStages || a.nH < 0 || a.nH > kMaxStages || a.nG < 0 ||
        a.nG > kMaxStages)
      fail("update_uq: stage %d, nH %d, nG %d", a.stage, a.nH, a.nG);
    for (int m = 0; m < 2; ++m) {
      s.r(0, a.v[m]);
      s.r(0, a.partner[m]);
      s.r(0, a.un[m], sizeof(T) == 4);  // the split form reads u^n as float64 elsewhere
      s.w(0, a.out_us[m]);
      s.w(0, a.out_hu[m], true);
    }
    s.r(0, a.qn);
    history<T>(s, a.nH, a.H);
    for (int j = 0; j < a.nG; ++j) s.r(0, a.G[j]);
    s.w(0, a.out_q);
    s.w(0, a.out_gq, true);
    // fused schedule: theta(i) in, Ltheta(i) from D0^2:B(v(i))
    s.r(1, a.th, true);
    if (a.out_lt != kNoSlot) {
      if (a.th == kNoSlot) fail("update_uq: L theta without theta");
      s.r(0, a.ddb);
      s.w(0, a.out_lt);
    }
    if (a.th != kNoSlot && a.co != 2 && a.co != 4) fail("update_uq: central order %d", a.co);
    check_tiles(insts, work, nwork, kRowsOfShape[si & 3], sizeof(T), s);
  });
  return hipSuccess;
}

template <typename T>
hipError_t launch_grad_q(int si, int wo, const Inst *insts, const Work *work, int nwork,
                         const ArgsG &a, hipStream_t st, const Ev &) {
  if (!shape_ok(si, wo, 4)) fail("grad_q: launch shape %d %d", si, wo);
  hostcheck::enqueue(st, [=] {
    Slots s{"grad_q"};
    s.r(0, a.q);
    s.r(0, a.v[0]);
    s.r(0, a.v[1]);
    s.w(0, a.out_g[0]);
    s.w(0, a.out_g[1]);
    check_tiles(insts, work, nwork, kRowsOfShape[si & 3], sizeof(T), s);
  });
  return hipSuccess;
}

template <typename T>
hipError_t launch_stage_terms(int si, int wo, int co, const Inst *insts, const Work *work,
                              int nwork, const ArgsE &a, const ArgsV &nv, hipStream_t st,
                              const Ev &) {
  if (!shape_ok(si, wo, co)) fail("stage_terms: launch shape %d %d %d", si, wo, co);
  hostcheck::enqueue(st, [=] {
    Slots s{"stage_terms"};
    const bool with_us = a.us[0] != kNoSlot;
    for (int m = 0; m < 2; ++m) {
      if (with_us) {
        s.r(0, a.us[m]);
        s.w(0, a.out_u[m]);
        if (a.hu[m] != kNoSlot) {
          s.r(0, a.hu[m]);
          s.w(0, a.hu[m]);
          s.inplace.insert({0, a.hu[m]});
        }
      } else if (a.ui[m] != kNoSlot) {  // split form, fused schedule: du(i) on u^n
        if (sizeof(T) != 4) fail("stage_terms: an increment in the float64 form");
        s.r(0, a.ui[m]);
        s.w(0, a.out_u[m]);
      } else {
        s.r(0, a.u[m]);
      }
      s.r(0, a.g[m], a.q != kNoSlot);  // no G input when it is formed here from q
      s.r(0, a.v[m]);
      s.w(0, a.out_e[m], true);
      s.r(1, a.ub[m], true);
      s.w(1, a.out_ud[m], true);
    }
    if (with_us) s.r(1, a.th);
    if (a.q != kNoSlot) {
      if (sizeof(T) != 4 || a.ui[0] == kNoSlot) fail("stage_terms: G formed outside the split fused stage");
      s.r(0, a.q);
    }
    if (a.out_lt != kNoSlot) {
      if (!with_us) fail("stage_terms: L theta without theta");
      s.r(0, a.ddb);
      s.w(0, a.out_lt);
    }
    s.w(0, a.out_du, true);
    s.r(1, a.du0_in, true);
    s.w(1, a.du0_out, true);
    if ((a.out_ud[0] != kNoSlot) != (a.du0_out != kNoSlot))
      fail("stage_terms: the last stage writes u and D0.u together");
    if (nv.stage) {
      if (nv.stage < 1 || nv.stage >= kMaxStages || nv.nE < 0 || nv.nE > kMaxStages ||
          nv.nV < 0 || nv.nV > kMaxStages)
        fail("stage_terms: relaxation of stage %d, nE %d, nV %d", nv.stage, nv.nE, nv.nV);
      for (int m = 0; m < 2; ++m) {
        s.r(0, nv.vn[m]);
        s.w(0, nv.out[m]);
      }
      history<T>(s, nv.nE, nv.E);
      history<T>(s, nv.nV, nv.V);
    }
    check_tiles(insts, work, nwork, kRowsOfShape[si & 3], sizeof(T), s);
  });
  return hipSuccess;
}

#define APDVM_INST(T)                                                                           \
  template hipError_t launch_helmholtz_rhs<T>(int, int, int, const Inst *, const Work *, int,  \
                                              const ArgsR &, hipStream_t, const Ev &);         \
  template hipError_t launch_update_uq<T>(int, int, int, const Inst *, const Work *, int,      \
                                          const ArgsUQ &, hipStream_t, const Ev &);            \
  template hipError_t launch_stage_terms<T>(int, int, int, const Inst *, const Work *, int,    \
                                            const ArgsE &, const ArgsV &, hipStream_t,         \
                                            const Ev &);                                       \
  template hipError_t launch_grad_q<T>(int, int, const Inst *, const Work *, int,              \
                                       const ArgsG &, hipStream_t, const Ev &);
APDVM_INST(double)
APDVM_INST(float)
#undef APDVM_INST

hipError_t launch_div_u(int co, const Inst *insts, const Work *tiles, int nwork, int su1, int su2,
                        int out, hipStream_t st) {
  if (co != 4 && co != 2) fail("div_u: central order %d", co);
  hostcheck::enqueue(st, [=] {
    Slots s{"div_u"};
    s.r(1, su1);
    s.r(1, su2);
    s.w(1, out);
    check_tiles(insts, tiles, nwork, 16, 0, s);
  });
  return hipSuccess;
}

// ---------------------------------------------------------------- Helmholtz solve

hipError_t launch_solve_part(int part, int rowv, int colv, int rowreg, int colreg,
                             const Inst *insts, const Work *rows, int nrows, const Work *cols,
                             int ncols, const ArgsSolve &a, hipStream_t st, const Ev &) {
  if (part < 0 || part > 2 || rowv < 0 || rowv > 3 || colv < 0 || colv > 2)
    fail("solve: part %d, forms %d %d", part, rowv, colv);
  hostcheck::enqueue(st, [=] {
    ++cnt().launches;
    const bool is_rows = part != 1;
    const Work *work = is_rows ? rows : cols;
    const int nwork = is_rows ? nrows : ncols;
    const int v = is_rows ? rowv : colv;
    const int reg = is_rows ? rowreg : colreg;
    if (reg < 0 || reg > 2) fail("solve: register form %d", reg);
    const bool full = reg == 1;
    const int cap = v == 0 ? kRowSmallCap : v == 1 ? kColMidCap : kFftCap;  // v 3: halved
    static std::set<std::tuple<const void *, unsigned long long, int, int, int, int>> walked;
    const bool walk =
        !in_device(work, (size_t)nwork * sizeof(Work)) ||
        walked.insert({insts, table_hash(work, nwork), nwork, part, v, reg}).second;
    if (walk) check_remap(nwork);
    std::set<int> seen;
    std::map<int, std::vector<char>> cover;
    for (int b = 0; b < nwork && !walk; ++b) seen.insert(work[b].inst);
    for (int b = 0; b < nwork && walk; ++b) {
      const Work *w = work + xcd_remap(b, nwork);
      if (!in_device(w, sizeof(Work))) {
        fail("solve: work item %d outside device memory", b);
        return;
      }
      ++cnt().items;
      const Inst *Ip = inst_of(insts, w->inst, 0, seen);
      if (!Ip) return;
      const Inst &I = *Ip;
      const int lines = is_rows ? I.ny / 2 : I.nx / 2;  // row pairs or spectrum columns
      const int per = is_rows ? I.row_pairs_per_block : I.cols_per_block;
      const int len = is_rows ? 2 * I.nx : I.ny;        // values of one line in LDS
      const int x0 = w->a;
      if (x0 < 0 || x0 >= lines || x0 % per) {
        fail("solve part %d: block at %d of instance %d (lines %d, %d per block)", part, x0,
             w->inst, lines, per);
        continue;
      }
      const int cnt_lines = std::min(per, lines - x0);
      const bool split_cols = !is_rows && v == 2;  // the largest column form halves
      // so do the largest inverse rows, and the forward rows that fill the form
      const bool split_rows = v == 3 && (part == 2 || (part == 0 && full));
      if (split_rows && I.nx % 4)
        fail("solve part %d: split rows of instance %d with nx = %d", part, w->inst, I.nx);
      const long long need = split_cols   ? (long long)cnt_lines * (I.ny / 2)
                             : split_rows ? (long long)cnt_lines * (I.nx / 2)
                                          : (long long)cnt_lines * len / (is_rows ? 2 : 1);
      const long long have = split_cols || split_rows ? kFftCap / 2 : cap;
      if (need > have)
        fail("solve part %d: block of instance %d needs %lld LDS values, form holds %lld", part,
             w->inst, need, have);
      if (full) {
        // register form: one line per block that fills the form's buffer, and a plan of
        // length 2^k whose first radix is 8 and whose last is 8, 2 or 4 for k mod 3 = 0, 1, 2
        const int n_line = is_rows ? I.nx : I.ny;
        const FftPlan &P = split_cols ? I.fyh : split_rows ? I.fxh : is_rows ? I.fx : I.fy;
        const int n_plan = split_cols || split_rows ? n_line / 2 : n_line;
        int k = 0;
        while ((1 << k) < P.n) ++k;
        const int last = k % 3 == 0 ? 8 : k % 3 == 1 ? 2 : 4;
        if (n_line != cap || cnt_lines != 1 || P.n != n_plan || (1 << k) != P.n ||
            P.npass < 2 || P.radix[0] != 8 || P.radix[P.npass - 1] != last)
          fail("solve part %d: register form on instance %d (line %d, form %d, %d lines, plan "
               "%d in %d passes)", part, w->inst, n_line, cap, cnt_lines, P.n, P.npass);
      }
      if (reg == 2 && !split_cols && !split_rows) {
        // several lines of 8^m values fill the block, and every pass of their plan is radix 8
        const int n_line = is_rows ? I.nx : I.ny;
        const FftPlan &P = is_rows ? I.fx : I.fy;
        int k = 0;
        while ((1 << k) < n_line) ++k;
        bool radix8 = P.npass >= 2 && P.n == n_line;
        for (int q = 0; q < P.npass && radix8; ++q) radix8 = P.radix[q] == 8;
        if ((1 << k) != n_line || k % 3 || n_line < 64 || n_line >= cap ||
            cnt_lines * n_line != cap || !radix8)
          fail("solve part %d: register form of several lines on instance %d (line %d, form "
               "%d, %d lines, plan %d in %d passes)", part, w->inst, n_line, cap, cnt_lines,
               P.n, P.npass);
      }
      auto &cv = cover[w->inst];
      if (cv.empty()) cv.assign(lines, 0);
      for (int l = x0; l < x0 + cnt_lines; ++l) {
        if (cv[l]) fail("solve part %d: line %d of instance %d covered twice", part, l, w->inst);
        cv[l] = 1;
      }
    }
    for (auto &[k, cv] : cover)
      for (char c : cv)
        if (!c) {
          fail("solve part %d: a line of instance %d is missing", part, k);
          break;
        }
    for (int k : seen) {
      Slots s{"solve"};
      if (part == 0) {
        s.r(1, a.r);
        s.w(1, a.spec);
      } else if (part == 1) {
        s.r(1, a.spec);
      } else {
        s.r(1, a.spec);
        s.w(1, a.out);
      }
      if (a.stage < 1 || a.stage >= kMaxStages) fail("solve: stage %d", a.stage);
      s.check(insts[k], k);
    }
  });
  return hipSuccess;
}

// ---------------------------------------------------------------- state kernels (CPU)

hipError_t launch_field_stats(int split, const void *const f[6], long long n, double *partials,
                              int nblocks, hipStream_t st) {
  const void *g[6] = {f[0], f[1], f[2], f[3], f[4], f[5]};
  hostcheck::enqueue(st, [=] {
    ++cnt().launches;
    const size_t ts = split ? 4 : 8;
    for (int i = 0; i < 6; ++i)
      if (!in_device(g[i], (size_t)n * (i == 2 ? 8 : ts))) fail("field_stats: field %d", i);
    if (!in_device(partials, (size_t)nblocks * 3 * 8)) {
      fail("field_stats: partials");
      return;
    }
    auto val = [&](int i, long long j) {
      if (i == 2) return static_cast<const double *>(g[2])[j];
      return split ? (double)static_cast<const float *>(g[i])[j]
                   : static_cast<const double *>(g[i])[j];
    };
    double s = 0.0, um = 0.0, fin = 1.0;
    for (long long j = 0; j < n; ++j) {
      const double a = val(0, j), b = val(1, j);
      s += val(2, j);
      um = std::fmax(um, std::sqrt(a * a + b * b));
      for (int i = 0; i < 6; ++i)
        if (!std::isfinite(val(i, j))) fin = 0.0;
    }
    for (int b = 0; b < nblocks; ++b) {
      partials[3 * b] = b == 0 ? s : 0.0;
      partials[3 * b + 1] = b == 0 ? um : 0.0;
      partials[3 * b + 2] = b == 0 ? fin : 1.0;
    }
  });
  return hipSuccess;
}

hipError_t launch_convert(void *dst, const void *src, long long n, int to_float, hipStream_t st) {
  hostcheck::enqueue(st, [=] {
    ++cnt().launches;
    if (!in_device(dst, (size_t)n * (to_float ? 4 : 8)) ||
        !in_device(src, (size_t)n * (to_float ? 8 : 4))) {
      fail("convert of %lld values outside device memory", n);
      return;
    }
    for (long long i = 0; i < n; ++i) {
      if (to_float)
        static_cast<float *>(dst)[i] = (float)static_cast<const double *>(src)[i];
      else
        static_cast<double *>(dst)[i] = (double)static_cast<const float *>(src)[i];
    }
  });
  return hipSuccess;
}

namespace {
template <typename F>
void each_cell_of_set(const Inst *insts, const Work *tiles, int ntiles, int ty, const StateSet &s,
                      const char *what, F &&fn) {
  Slots sl{what};
  for (int p = 0; p < 5; ++p) sl.r(0, s.t[p]);
  for (int p = 0; p < s.nd; ++p) sl.r(1, s.d[p]);
  check_tiles(insts, tiles, ntiles, ty, 0, sl);
  std::set<int> seen;
  for (int b = 0; b < ntiles; ++b) seen.insert(tiles[b].inst);
  for (int k : seen) fn(insts[k]);
}
}  // namespace

hipError_t launch_state_finite(int split, const Inst *insts, const Work *tiles, int ntiles, int ty,
                               const StateSet &s, unsigned *flag, hipStream_t st) {
  hostcheck::enqueue(st, [=] {
    if (!in_device(flag, 4)) fail("state_finite: flag");
    if (s.nd < 1 || s.nd > 3) fail("state_finite: %d float64 planes", s.nd);
    each_cell_of_set(insts, tiles, ntiles, ty, s, "state_finite", [&](const Inst &I) {
      bool fin = true;
      for (long long g = 0; g < I.plane; ++g) {
        for (int p = 0; p < 5; ++p) {
          const double v = split ? (double)static_cast<const float *>(I.tbase)[s.t[p] * I.plane + g]
                                 : static_cast<const double *>(I.tbase)[s.t[p] * I.plane + g];
          fin = fin && std::isfinite(v);
        }
        for (int p = 0; p < s.nd; ++p) fin = fin && std::isfinite(I.dbase[s.d[p] * I.plane + g]);
      }
      if (!fin) *flag = 1u;
    });
  });
  return hipSuccess;
}

hipError_t launch_snapshot(int split, const Inst *insts, const Work *tiles, int ntiles, int ty,
                           const StateSet &a, const StateSet &b, const unsigned *flag,
                           long long *ck_step, long long step, hipStream_t st) {
  hostcheck::enqueue(st, [=] {
    if (!in_device(flag, 4) || !in_device(ck_step, 8)) fail("snapshot: flag or step word");
    if (a.nd != b.nd) fail("snapshot: sets of %d and %d float64 planes", a.nd, b.nd);
    Slots w{"snapshot"};
    for (int p = 0; p < 5; ++p) w.w(0, b.t[p]);
    for (int p = 0; p < b.nd; ++p) w.w(1, b.d[p]);
    each_cell_of_set(insts, tiles, ntiles, ty, a, "snapshot", [&](const Inst &I) {
      w.check(I, 0);
      for (int p = 0; p < 5; ++p)
        for (int q = 0; q < 5; ++q)
          if (a.t[p] == b.t[q]) fail("snapshot: source and copy share a plane");
      if (*flag) return;
      const size_t ts = split ? 4 : 8;
      char *tb = static_cast<char *>(I.tbase);
      for (int p = 0; p < 5; ++p)
        std::memcpy(tb + (size_t)b.t[p] * I.plane * ts, tb + (size_t)a.t[p] * I.plane * ts,
                    (size_t)I.plane * ts);
      for (int p = 0; p < a.nd; ++p)
        std::memcpy(I.dbase + (size_t)b.d[p] * I.plane, I.dbase + (size_t)a.d[p] * I.plane,
                    (size_t)I.plane * 8);
    });
    if (!*flag) *ck_step = step;
  });
  return hipSuccess;
}

// ---------------------------------------------------------------- diagnostics

hipError_t launch_diagnostics(const Inst *insts, const Work *tiles, int ntiles, int ty, int split,
                              int su1, int su2, int dth, int sv1, int sv2, int sq, int co,
                              double *partials, int nblocks, hipStream_t st) {
  hostcheck::enqueue(st, [=] {
    if (co != 4 && co != 2) fail("diagnostics: central order %d", co);
    Slots s{"diagnostics"};
    s.r(split ? 1 : 0, su1);
    s.r(split ? 1 : 0, su2);
    s.r(1, dth);
    s.r(0, sv1);
    s.r(0, sv2);
    s.r(0, sq);
    check_tiles(insts, tiles, ntiles, ty, split ? 4 : 8, s);
    if (nblocks < 1 || !in_device(partials, (size_t)nblocks * 8 * 8)) {
      fail("diagnostics: %d partial records outside device memory", nblocks);
      return;
    }
    for (int b = 0; b < nblocks; ++b) {
      const double neutral[8] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 1.0};
      std::memcpy(partials + 8 * b, neutral, sizeof(neutral));
    }
  });
  return hipSuccess;
}

hipError_t launch_diag_finish(const double *partials, int nblocks, double area, double *out,
                              hipStream_t st) {
  hostcheck::enqueue(st, [=] {
    ++cnt().launches;
    if (!in_device(partials, (size_t)nblocks * 64) || !in_device(out, 64)) {
      fail("diag_finish: partials or output outside device memory");
      return;
    }
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 1.0};
    for (int b = 0; b < nblocks; ++b) {
      const double *q = partials + 8 * b;
      acc[0] += q[0];
      acc[1] += q[1];
      acc[2] += q[2];
      acc[3] = std::fmax(acc[3], q[3]);
      acc[4] = std::fmin(acc[4], q[4]);
      acc[5] = std::fmax(acc[5], q[5]);
      acc[6] += q[6];
      acc[7] = std::fmin(acc[7], q[7]);
    }
    for (int i = 0; i < 8; ++i) out[i] = acc[i] * (i < 3 ? area : i == 6 ? 0.5 * area : 1.0);
  });
  return hipSuccess;
}

// The static scratch of the allocation-free diagnostics: one host array, registered as
// device memory.
namespace {
constexpr int kScratchBlocksCheck = 1024;
double *g_scratch = nullptr;
}  // namespace
hipError_t scratch_init(int device) {
  if (device != 0) return hipErrorInvalidDevice;
  if (!g_scratch) {
    void *p = nullptr;
    if (hipMalloc(&p, 8 * kScratchBlocksCheck * sizeof(double)) != hipSuccess)
      return hipErrorOutOfMemory;
    g_scratch = static_cast<double *>(p);
  }
  return hipSuccess;
}
double *scratch_ptr(int device) { return device == 0 ? g_scratch : nullptr; }
int scratch_blocks() { return kScratchBlocksCheck; }

}  // namespace apdvm
