// Internal data structures shared by the HIP kernels and the host runtime.
//
// Every context holds one or more independent simulations ("instances").  Each
// phase of a stage is one kernel launch over a work table that lists, for every
// workgroup, the instance and the tile (or FFT row block / column strip) it owns,
// so a single launch advances every instance.  Per-instance scalars, FFT plans,
// symbols and plane base pointers live in a device array of Inst; per-stage slot
// numbers and tableau coefficients are identical for all instances and travel as
// kernel arguments.
//
// Planes: an instance owns two arenas, one of "transport" planes (T = double in the
// FP64 form, float in the FP32-split form) and one of float64 planes (theta, the
// Helmholtz right-hand side, the spectrum).  A slot number k addresses the plane at
// base + k * nx * ny.  Layout of a plane: row-major [ny][nx], x fastest.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cstdint>

namespace apdvm {

// Global-memory pointers.  Plane, table and symbol addresses are read from the device
// Inst table, where the compiler cannot see their address space; through a generic
// pointer every access would be a FLAT instruction, which also counts against the LDS
// wait counter and so makes LDS reads wait for global loads still in flight.
template <class T>
using Gp = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ Gp<T> gp(T *p) {
  return (Gp<T>)p;
}

// Optional HIP events around one launch.  With both set the launch goes through
// hipExtLaunchKernelGGL, whose events take the start and end of the kernel's own
// dispatch (not the gap in the queue before it); otherwise it is a plain launch.
struct Ev {
  hipEvent_t start = nullptr, stop = nullptr;
};
#define APDVM_LAUNCH(EV, KERNEL, GRID, BLOCK, STREAM, ...)                                   \
  do {                                                                                      \
    if ((EV).start)                                                                         \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, (EV).start, (EV).stop, 0,       \
                            __VA_ARGS__);                                                   \
    else                                                                                    \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                      \
  } while (0)

// ---------------------------------------------------------------- index maps
// Host and device: the kernels use them, and the host-side bounds check (built with
// APDVM_HOSTCHECK) walks every launch's index space through the same functions.

// Work item of workgroup b out of nwork.  The hardware hands consecutive workgroups to
// the 8 XCDs in turn; this remap gives each XCD a contiguous run of work items, so tiles
// sharing halo rows (and FFT blocks sharing spectrum lines) meet in the same L2.
// A bijection of [0, nwork).
__host__ __device__ inline int xcd_remap(int b, int nwork) {
  const int x = b & 7, i = b >> 3;
  const int q = nwork >> 3, r = nwork & 7;
  return x * q + (x < r ? x : r) + i;
}

// Periodic index in [0, n).  A staged tile reaches at most its width plus the halo past
// either end of the grid, so one add or subtract of n wraps every index of a grid of 72
// cells or more; the division remains for smaller grids, whose halos can wrap several
// times.
__host__ __device__ inline int wrap_index(int g, int n) {
  g += g < 0 ? n : (g >= n ? -n : 0);
  if ((unsigned)g >= (unsigned)n) g = ((g % n) + n) % n;
  return g;
}

// Cell (row-major index y * nx + x) of element idx of the staged (TY + 2H) x (W = 64 + 2H)
// region of the tile at (x0, y0): cell (x0 + lx - H, y0 + ly - H) taken periodically.
// inner: the region lies inside the grid, so no index wraps.
__host__ __device__ inline int staged_cell(int idx, int W, int H, int nx, int ny, int x0,
                                           int y0, bool inner) {
  const int ly = idx / W;
  const int lx = idx - ly * W;
  int gx = x0 + lx - H, gy = y0 + ly - H;
  if (!inner) {
    gx = wrap_index(gx, nx);
    gy = wrap_index(gy, ny);
  }
  return gy * nx + gx;
}

// Factors of the central differences for 1/h = ih: order 4 (the high-order extension of
// Section 3.2) D f = (f-2 - 8 f-1 + 8 f+1 - f+2) ih / 12, L f = (-f-2 + 16 f-1 - 30 f0 +
// 16 f+1 - f+2) ih^2 / 12; order 2 (as printed in Section 3.2) D f = (f+1 - f-1) ih / 2,
// L f = (f-1 - 2 f0 + f+1) ih^2.  The host evaluates them once per instance (a float64
// division on the device is a dozen vector instructions in every thread).
__host__ __device__ inline double central_f1(int co, double ih) {
  return co == 2 ? 0.5 * ih : ih / 12.0;
}
__host__ __device__ inline double central_f2(int co, double ih) {
  return co == 2 ? ih * ih : ih * ih / 12.0;
}

constexpr int kMaxStages = 8;
constexpr int kMaxPasses = 16;
constexpr int kNoSlot = -1;

// Stencil tiles: kTileX x TY interior cells, halo kHalo (WENO5 needs 3 on each side).
constexpr int kTileX = 64;
constexpr int kHalo = 3;

// FFT workgroups: capacity in complex float64 values held in LDS, and threads.  The row
// and column kernels each take the smallest form that holds a whole row (column) of
// every instance.
constexpr int kFftCap = 8192;
constexpr int kFftThreads = 1024;
constexpr int kRowSmallCap = 1024;
constexpr int kRowSmallThreads = 128;
constexpr int kColMidCap = 2048;
constexpr int kColMidThreads = 256;

// Two-level twiddle table of a length-n transform, staged into LDS by every FFT kernel:
// with B = 2^lb the smallest power of two whose square is at least n, entries
// [0, B) hold exp(-2 pi i b / n) and entries [B, B + ceil(n / B)) hold
// exp(-2 pi i a B / n), so exp(-2 pi i m / n) = hi[m >> lb] * lo[m & (B - 1)].
constexpr int kTwCap = 256;  // B + ceil(n / B) for every n <= 16384

struct FftPlan {
  int n;                  // transform length
  int npass;              // number of Stockham passes
  int radix[kMaxPasses];  // radices (2, 3, 4 or 8), first pass first
  const double2 *tw2;     // two-level table (device), ntw entries
  int lb, ntw;
  int tsc;                // table index scale: the table is of length tsc n (1, or 2 for a
                          // half-length plan that shares the table of its full length)
};

struct Inst {
  int nx, ny;
  long long plane;           // nx * ny
  double ihx, ihy;           // 1 / h
  double f1x, f1y, f2x, f2y; // central-difference factors central_f1, central_f2 of 1 / h
  double eps, tau, dt, te2;  // te2 = tau * eps^2
  double theta_mean;         // value imposed on the (0,0) Helmholtz mode
  double kinv[kMaxStages];   // 1 / (tau eps^2 + dt a_ii)
  double sigma[kMaxStages];  // 2 eps^2 / (dt a_ii)^2
  double rdt2[kMaxStages];   // 1 / (dt a_ii^2)
  double rdt[kMaxStages];    // 1 / (dt a_ii)
  double inv_nxny;           // 1 / (nx ny)
  FftPlan fx, fy;            // lengths nx and ny
  FftPlan fxh, fyh;          // lengths nx / 2, ny / 2 on the tables of fx, fy (split kernels)
  const double *lam_x;       // nx/2 + 1 values of the x symbol of D_Delta
  const double *lam_y;       // ny values of the y symbol
  void *tbase;               // transport arena
  double *dbase;             // float64 arena
  int row_pairs_per_block;   // FFT row kernels: row pairs per workgroup
  int cols_per_block;        // FFT column kernel: whole columns per workgroup
  int nt_slots, nd_slots;    // planes of the transport and float64 arenas
  int tbytes;                // bytes of a transport value (8, or 4 in the FP32-split form)
};

// Work table entry: instance and the first cell / row pair / column of the block.
struct Work {
  int inst;
  int a;  // stencil: x0;  FFT rows: first row pair;  FFT columns: first column
  int b;  // stencil: y0
  int c;  // unused
};

// ---------------------------------------------------------------- kernel arguments

// Step 1 of a stage: v(i) = [te2 v^n - dt sum_j cE_j E(j) - dt sum_j cV_j v(j)] kinv.
// stage = 0 marks "no step 1 here".
struct ArgsV {
  int stage;
  int vn[2];
  int nE, E[kMaxStages][2];
  double cE[kMaxStages];
  int nV, V[kMaxStages][2];
  double cV[kMaxStages];
  int out[2];
};

// Step 2 right-hand side:
// R = -sigma theta^n + 1/(dt a_ii^2) sum_j cD_j D0.u(j) + 1/(dt a_ii) D0.u^n
//     - D0^2:B(v(i)) - 1/a_ii sum_j cL_j Ltheta(j),
// with Ltheta(j) = D0^2:B(v(j)) + D_Delta theta(j).  Also stores D0^2:B(v(i)).
// In the FP32-split form the velocity of stage j is u^n + du(j) (u^n float64, the stage
// increment du(j) float), the D slots hold D0.du(j) and du0 is the float64 D0.u^n, so
// the u^n part enters once with the coefficient 1/(dt a_ii) + sum_a/(dt a_ii^2),
// sum_a = sum_j cD_j.
struct ArgsR {
  int stage;
  double aii;
  int v[2];       // v(i), read with a halo of 2 (corners included)
  int thn;        // theta^n (float64 slot)
  int du0;        // D0.u^n (transport slot; float64 slot when du0_dbl)
  int du0_dbl;
  double sum_a;
  int nD, D[kMaxStages];
  double cD[kMaxStages];
  int nL, L[kMaxStages];
  double cL[kMaxStages];
  int out_r;      // R (float64 slot)
  int out_ddb;    // D0^2:B(v(i))
  double c_l;     // 1 / a_ii
};

// Steps 3 and 4 short of theta(i), which the Helmholtz solve of the same stage is still
// producing when this runs:
// hu = D_W.B(v(i))[dissipation on u(i-1)]
// u*(i) = u^n - dt sum_j cH_j Hu(j) - dt a_ii hu            (formed in float64)
// (with un[0] == kNoSlot, the FP32-split form, the increment du*(i) = u*(i) - u^n)
// Hq = (tau/2) D0_W.v(i)
// q(i) = [te2 q^n - dt a_ii Hq - dt sum_j cG_j Gq(j)] kinv,   Gq(j) = Hq(j) + q(j)
// The stage-terms launch of the stage completes u(i) = u*(i) - dt a_ii D0 theta(i) and
// Hu(i) = hu + D0 theta(i).
// Fused schedule (th != kNoSlot, after the solve of the stage, one stream): this launch
// completes them itself from theta(i): out_us receives u(i) (the split form: the
// increment du(i) = du*(i) - dt a_ii D0 theta(i)), out_hu receives Hu(i), and out_lt
// Ltheta(i) = D0^2:B(v(i)) + D_Delta theta(i) from ddb; co is the central order.
struct ArgsUQ {
  int stage;
  double aii;
  int v[2];       // v(i), halo 3
  int partner[2]; // u(i-1), halo 3
  int un[2], qn;  // state at time n
  int nH, H[kMaxStages][2];
  double cH[kMaxStages];
  int nG, G[kMaxStages];
  double cG[kMaxStages];
  int out_us[2];  // u*(i)
  int out_q;
  int out_hu[2], out_gq;  // hu and Gq; kNoSlot when no later stage needs them
  int th;                 // theta(i) (float64 slot) in the fused schedule, else kNoSlot
  int ddb, out_lt;        // fused schedule: D0^2:B(v(i)) in, Ltheta(i) out, or kNoSlot
  int co;                 // central order (fused schedule)
};

// The q part of the stage terms E (it needs q(i) and v(i) only, so it runs before
// theta(i) is known): G = te2 D_W q[dissipation on v], x component from the x faces with
// the split fluxes q +- v1, y component from the y faces with q +- v2.
struct ArgsG {
  int q, v[2];  // halo 3
  int out_g[2];
};

// Completion of a stage and its terms that later stages reuse:
// u(i) = u*(i) - dt a_ii D0 theta(i), Hu(i) = hu + D0 theta(i) (in place),
// (FP32-split form: us holds the increment du*(i); du(i) = du*(i) - dt a_ii D0 theta(i)
// rounded to float, u(i) = u^n + du(i) from the base u[] (float copy of u^n) or, in the
// last stage, ub (float64 u^n) with the new float64 state written to out_ud and its
// float copy to out_u; out_du receives D0.du(i), or in the last stage du0_out receives
// the float64 D0.u^{n+1} = du0_in + D0.du(s)),
// E = (tau/4) D0_W.B(u) + G - F(u) with G from ArgsG, D0.u,
// Ltheta = D0^2:B(v) + D_Delta theta.  With us[0] == kNoSlot (the terms of a state set,
// or of a stage of the fused schedule, whose update launch completed u(i) from theta(i))
// u is read from u[] and nothing of theta is used; in the FP32-split form ui[] then holds
// the complete increment du(i) of a fused stage (kNoSlot for a state set).  The same launch performs step 1 of
// the next stage (an ArgsV passed beside it); c_e_next and c_v_next are the coefficients
// of this stage's E and v in that step (at_{k,j} and a_{k,j}), which stay in registers.
struct ArgsE {
  int us[2];          // u*(i) (halo 3) or kNoSlot
  int u[2];           // u of a state set (halo 3), when us[0] == kNoSlot
  int g[2];           // G of this stage (pointwise)
  int v[2];           // v of this stage (pointwise, for the fused step 1)
  int th;             // theta(i), float64 slot, halo 3 + reach of D0 (with us)
  double aii;         // a_ii of the stage (with us)
  int out_u[2];       // u(i) (with us)
  int hu[2];          // hu in, Hu out, or kNoSlot (with us)
  int ddb;            // D0^2:B(v) of this stage (only when out_lt != kNoSlot)
  int out_e[2];       // kNoSlot when only the fused next step reads E
  int out_du, out_lt; // out_lt only with us; out_du may be kNoSlot
  double c_e_next, c_v_next;
  int ub[2];          // split form, last stage: float64 u^n (halo 3), else kNoSlot
  int out_ud[2];      // split form, last stage: float64 u^{n+1}
  int du0_in, du0_out;  // split form, last stage: float64 D0.u^n and D0.u^{n+1}
  int ui[2];          // split form, fused schedule: the increment du(i) (halo 3), else kNoSlot
  int q;              // split form, fused schedule: q(i) (halo 3), G formed here from q and
                      // v (g[] unused); else kNoSlot
};

// The planes that hold one state set (or the snapshot of the finite check): five
// transport slots u1, u2, v1, v2, q (in the FP32-split form u1, u2 are the float copies
// of the velocity) and nd float64 slots: theta, then in the split form the float64
// velocity u1, u2.
struct StateSet {
  int t[5];
  int nd;
  int d[3];
};

// Helmholtz solve: R (float64 slot) -> theta (float64 slot), spectrum in slot spec
// (column-major [nx/2][ny] complex, kx = nx/2 in the imaginary part of column 0: the
// last float64 slot).
struct ArgsSolve {
  int stage;
  int r, spec, out;
};

}  // namespace apdvm
