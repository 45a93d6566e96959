// Stencil kernels of one IMEX stage (Algorithm 1, steps 1, 3 and 4, the right-hand
// side of step 2, and the stage terms reused by later stages), with the high-order
// space discretisation of Section 3.2: WENO5 (Jiang-Shu) reconstruction of the
// Lax-Friedrichs split fluxes and fourth-order central differences.
//
// Per stage: k_helmholtz_rhs (the right-hand side of step 2, before the solve);
// k_update_uq and k_grad_q (everything of steps 3 and 4 and of the stage terms that does
// not involve theta(i): they run while the solve produces it); k_stage_terms (u(i) with
// its theta gradient, the rest of the stage terms, and step 1 of the next stage).
//
// Tiling: a workgroup of NT threads owns a 64 x TY tile of one instance (64 x 8 or
// 64 x 16 on 256 or 512 threads, chosen per kernel class by the host autotuner).  Every
// input plane is staged once in LDS with a 3-cell periodic halo (WENO5 reads 3 cells on
// each side of a cell; the central operators 2, corners included for the mixed
// derivative).  Planes that only feed WENO fluxes are staged multiplied by 1/2, which is
// exact in binary floating point, so the split fluxes (f +- w)/2 cost one add per cell
// and round exactly like (f +- w) * 0.5.  WENO numerical fluxes are computed once per
// face into LDS; the x and y faces of one divergence share one balanced index space.
// Thread t owns column t % 64 and rows t / 64 + (NT / 64) k of the tile: every
// wavefront covers full 64-cell row segments, so all global loads and stores are
// row-contiguous.
//
// Precision: T is the transport type (double or float).  theta, the Helmholtz
// right-hand side and every history sum feeding an implicit relaxation or the
// right-hand side are float64 whatever T is.
#include "common.hpp"

#include <type_traits>

namespace apdvm {

// ------------------------------------------------------------------ helpers

// Materialises x at this point: left alone, the compiler sinks the arithmetic of x past
// the next flux round and keeps the LDS values it is made of live instead (more
// registers, fewer resident waves).
template <typename T>
__device__ __forceinline__ void keep(T &x) {
  asm volatile("" : "+v"(x));
}

// Resident waves per SIMD the WENO kernels ask the register allocator for: six (at most
// 80 VGPRs) for the 64 x 8 tiles and for 512 threads, where the LDS of a tile leaves room
// for that many (three workgroups of 512 threads or six of 256 per CU); the 64 x 16 tiles
// on 256 threads are bounded by LDS before registers.
template <int TY, int NT>
constexpr int weno_waves_per_eu() {
  return TY == 8 || NT == 512 ? 6 : 1;
}
// The float update kernel on 512 threads asks for eight (at most 64 VGPRs): it fits them
// (spilling at most 8 bytes), its LDS leaves room for four workgroups per CU, and it runs
// 3-5% faster than with six (8192^2: 1209 against 1258-1275 us per launch, same bits).
template <typename T, int TY, int NT>
constexpr int update_waves_per_eu() {
  return sizeof(T) == sizeof(float) && NT == 512 ? 8 : weno_waves_per_eu<TY, NT>();
}

__device__ __forceinline__ int xcd_item(int nwork) { return xcd_remap(blockIdx.x, nwork); }
__device__ __forceinline__ int wrap(int g, int n) { return wrap_index(g, n); }

// WENO5 of Jiang and Shu, written through 3-cell windows.  For cells g_{k-1}, g_k,
// g_{k+1} let S = g_{k-1} - 2 g_k + g_{k+1} and D = g_{k+1} - g_{k-1}.  The Jiang-Shu
// smoothness indicators of the three sub-stencils of a reconstruction are, times four,
//   4 beta0 = 13/3 S^2 + (2S + D)^2 on window i-1, 4 beta1 = 13/3 S^2 + D^2 on window i,
//   4 beta2 = 13/3 S^2 + (2S - D)^2 on window i+1
// (for window i-1, a - 4b + 3c = 2S + D; for window i+1, 3c - 4d + e = 2S - D).
// A window carries e = 4 eps_w + 13/3 S^2 (eps_w = 1e-6), S and D, so each indicator term
// (4 eps_w + 4 beta)^2 = 16 (eps_w + beta)^2 is one fused multiply-add and a square; the
// common factor 16 cancels in the normalised weights.  Candidates at face
// i+1/2: q0 = (2 g_{i-2} - 7 g_{i-1} + 11 g_i)/6, q1 = (-g_{i-1} + 5 g_i + 2 g_{i+1})/6,
// q2 = (2 g_i + 5 g_{i+1} - g_{i+2})/6, weights alpha_k = d_k / (eps_w + beta_k)^2 with
// d = (1, 6, 3)/10; the right-biased reconstruction is the mirror image.

template <typename T>
struct Win {
  T e, s, d;
};
template <typename T>
__device__ __forceinline__ Win<T> win(T l, T c, T r) {
  const T S = fma(T(-2), c, l + r);
  return Win<T>{fma(T(13.0 / 3.0) * S, S, T(4e-6)), S, r - l};
}
// 16 (eps_w + beta_k)^2 of the three indicator forms of a window
template <typename T>
__device__ __forceinline__ T ind0(const Win<T> &w) {
  const T t = fma(T(2), w.s, w.d);
  const T x = fma(t, t, w.e);
  return x * x;
}
template <typename T>
__device__ __forceinline__ T ind1(const Win<T> &w) {
  const T x = fma(w.d, w.d, w.e);
  return x * x;
}
template <typename T>
__device__ __forceinline__ T ind2(const Win<T> &w) {
  const T t = fma(T(2), w.s, -w.d);
  const T x = fma(t, t, w.e);
  return x * x;
}
// Candidates at face i+1/2: q0 = (2 a - 7 b + 11 c)/6 from cells i-2, i-1, i, and the
// other two scaled by their linear weights' ratios to the first: 6 q1 = -b + 5 c + 2 d from
// cells i-1, i, i+1, and 3 q2 = (2 c + 5 d - e)/2 from cells i, i+1, i+2.
template <typename T>
__device__ __forceinline__ T cfar(T a, T b, T c) {
  return fma(T(1.0 / 3.0), a, fma(T(-7.0 / 6.0), b, T(11.0 / 6.0) * c));
}
template <typename T>
__device__ __forceinline__ T c6(T b, T c, T d) {
  return fma(T(5), c, fma(T(2), d, -b));
}
template <typename T>
__device__ __forceinline__ T c3(T c, T d, T e) {
  return fma(T(2.5), d, fma(T(-0.5), e, c));
}

// float64 quotient through the hardware reciprocal and one Newton step (the
// reciprocal's error, about 2^-26, is squared by the step: the quotient is within a few
// ulps, far inside what the weights need).
__device__ __forceinline__ double qdiv(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return n * r;
}

// Numerator and denominator of one reconstruction from s_k = 16 (eps_w + beta_k)^2, q0,
// Q1 = 6 q1 and Q2 = 3 q2: the weights d_k / s_k with d = (1, 6, 3)/10, multiplied
// through by 10 s0 s1 s2.  s_k >= 16 eps_w^2 = 1.6e-11, so the products stay above
// 2.5e-22, normal in float too.
template <typename T>
__device__ __forceinline__ void nd(T s0, T s1, T s2, T q0, T Q1, T Q2, T &n, T &den) {
  const T w0 = s1 * s2, p02 = s0 * s2, p01 = s0 * s1;
  n = fma(w0, q0, fma(p02, Q1, p01 * Q2));
  den = fma(T(6), p02, fma(T(3), p01, w0));
}
// n+/d+ + n-/d-: float64 with one division; float with two hardware reciprocals (the
// product d+ d- can fall below the float range where every beta vanishes)
__device__ __forceinline__ double sum2(double np, double dp, double nm, double dm) {
  return qdiv(fma(np, dm, nm * dp), dp * dm);
}
__device__ __forceinline__ float sum2(float np, float dp, float nm, float dm) {
  return fma(np, __builtin_amdgcn_rcpf(dp), nm * __builtin_amdgcn_rcpf(dm));
}

// Face between cells c2 and c3 of six consecutive values c0..c5 of one function g:
// left-biased reconstruction plus right-biased reconstruction of the same g (the
// Lax-Friedrichs split without dissipation, g = f/2).  The two share windows i and i+1
// and two candidates.  Every operation commutes exactly with negation, so the flux of
// -g is the negated flux of g.
template <typename T>
__device__ __forceinline__ T flux_sym(T c0, T c1, T c2, T c3, T c4, T c5) {
  const Win<T> wa = win(c0, c1, c2), wb = win(c1, c2, c3), wc = win(c2, c3, c4),
               wd = win(c3, c4, c5);
  const T M6 = c6(c1, c2, c3);  // 6 x (window i at i+1/2)
  const T N6 = c6(c4, c3, c2);  // 6 x (window i+1 at i+1/2)
  const T P = cfar(c0, c1, c2);
  const T Pm = cfar(c5, c4, c3);
  T np, dp, nm, dm;
  nd(ind0(wa), ind1(wb), ind2(wc), P, M6, T(0.5) * N6, np, dp);
  nd(ind2(wd), ind1(wc), ind0(wb), Pm, N6, T(0.5) * M6, nm, dm);
  return sum2(np, dp, nm, dm);
}

// Same face for two functions: p (left-biased) and m (right-biased), the split fluxes
// f + w and f - w of a dissipative Lax-Friedrichs flux (inputs already halved).
template <typename T>
__device__ __forceinline__ T flux_lf(const T *p, const T *m) {
  const Win<T> pa = win(p[0], p[1], p[2]), pb = win(p[1], p[2], p[3]), pc = win(p[2], p[3], p[4]);
  const T q0 = cfar(p[0], p[1], p[2]);
  const T q1 = c6(p[1], p[2], p[3]);
  const T q2 = c3(p[2], p[3], p[4]);
  const Win<T> mb = win(m[1], m[2], m[3]), mc = win(m[2], m[3], m[4]), md = win(m[3], m[4], m[5]);
  const T r0 = cfar(m[5], m[4], m[3]);
  const T r1 = c6(m[4], m[3], m[2]);
  const T r2 = c3(m[3], m[2], m[1]);
  T np, dp, nm, dm;
  nd(ind0(pa), ind1(pb), ind2(pc), q0, q1, q2, np, dp);
  nd(ind2(md), ind1(mc), ind0(mb), r0, r1, r2, nm, dm);
  return sum2(np, dp, nm, dm);
}

// WENO3 of Jiang and Shu (r = 2) for the convergence tables of Section 4.1: at face
// i+1/2 the left-biased value combines (3 g_i - g_{i-1})/2 and (g_i + g_{i+1})/2 with
// linear weights 1/3 and 2/3 and indicators (g_i - g_{i-1})^2 and (g_{i+1} - g_i)^2;
// multiplied through by 3 (eps_w + beta_0)^2 (eps_w + beta_1)^2 the weights become
// s1 and 2 s0 with s_k = (eps_w + beta_k)^2.
template <typename T>
__device__ __forceinline__ T sq3(T d) {
  const T x = fma(d, d, T(1e-6));
  return x * x;
}
template <typename T>
__device__ __forceinline__ void nd3(T s0, T s1, T q0, T q1, T &n, T &den) {
  const T w1 = T(2) * s0;
  n = fma(s1, q0, w1 * q1);
  den = s1 + w1;
}
// Face between cells c2 and c3 of g (c1..c4 used): left- plus right-biased WENO3; the
// two share the candidate (c2 + c3)/2 and the indicator (c3 - c2)^2.
template <typename T>
__device__ __forceinline__ T flux3_sym(T c1, T c2, T c3, T c4) {
  const T mid = T(0.5) * (c2 + c3);
  const T sm = sq3(c3 - c2);
  T np, dp, nm, dm;
  nd3(sq3(c2 - c1), sm, fma(T(1.5), c2, T(-0.5) * c1), mid, np, dp);
  nd3(sq3(c3 - c4), sm, fma(T(1.5), c3, T(-0.5) * c4), mid, nm, dm);
  return sum2(np, dp, nm, dm);
}
// Same face for the split fluxes p (left-biased) and m (right-biased).
template <typename T>
__device__ __forceinline__ T flux3_lf(const T *p, const T *m) {
  T np, dp, nm, dm;
  nd3(sq3(p[2] - p[1]), sq3(p[3] - p[2]), fma(T(1.5), p[2], T(-0.5) * p[1]),
      T(0.5) * (p[2] + p[3]), np, dp);
  nd3(sq3(m[3] - m[4]), sq3(m[2] - m[3]), fma(T(1.5), m[3], T(-0.5) * m[4]),
      T(0.5) * (m[3] + m[2]), nm, dm);
  return sum2(np, dp, nm, dm);
}

// Shift of the dissipation variable inside one flux window.  A WENO reconstruction is
// exactly translation invariant (the smoothness indicators see differences only; every
// candidate is an affine combination), so adding a constant c to every value of f+ and
// -c to every value of f- changes the left-biased part by +c and the right-biased one by
// -c, and the flux not at all.  In float the split values (sf f +- w) / 2 are dominated
// by the larger dissipation variable (a velocity of order one against v of order |u|^2),
// and each reconstructed face would carry its rounding, which the flux difference
// divides by h; with w - c, c a value of w in the window, the subtraction is exact for a
// smooth w and the rounding falls to that of f and of the variation of w.  float64 keeps
// the plain form.
template <typename T>
__device__ __forceinline__ T diss_shift(T c) {
  return sizeof(T) == sizeof(float) ? c : T(0);
}

// Numerical flux at the face between cells k = 2 and k = 3 of six consecutive cells
// (stride apart in LDS).  f and w are staged halved, so f+ = sf f + w and
// f- = sf f - w are the Lax-Friedrichs split fluxes (sf f +- alpha w)/2 with alpha = 1
// (DISS) or alpha = 0: left-biased WENO of f+ plus right-biased WENO of f- (order WO,
// 5 or 3; WENO3 reads cells 1..4 only).  sf is +1 or -1.
template <typename T, bool DISS, int WO>
__device__ __forceinline__ T face_flux(const T *f, const T *w, int stride, T sf) {
  constexpr int K0 = WO == 5 ? 0 : 1, K1 = WO == 5 ? 6 : 5;
  if (DISS) {
    T p[6], m[6];
    const T c = diss_shift(w[2 * stride]);
#pragma unroll
    for (int k = K0; k < K1; ++k) {
      const T fk = f[k * stride], wk = w[k * stride] - c;
      p[k] = fma(sf, fk, wk);
      m[k] = fma(sf, fk, -wk);
    }
    if (WO == 5) return flux_lf(p, m);
    return flux3_lf(p, m);
  }
  if (WO == 5)
    return sf * flux_sym(f[0], f[stride], f[2 * stride], f[3 * stride], f[4 * stride],
                         f[5 * stride]);
  return sf * flux3_sym(f[stride], f[2 * stride], f[3 * stride], f[4 * stride]);
}

// WENO5 fluxes at the three consecutive faces k = 0, 1, 2 between cells 2 + k and 3 + k of
// eight consecutive cells (stride apart): face k takes the same operations as face_flux
// on cells k .. k + 5, but each window and split value is formed once for the up to three
// faces that use it (windows centred on cells 1..5 for f+ and 2..6 for f-, or 1..6
// without dissipation, instead of six per face).
template <typename T, bool DISS>
__device__ __forceinline__ void face_flux3(const T *f, const T *w, int stride, T sf, T *out) {
  if (DISS) {
    T p[7], m[8];  // f+ on cells 0..6, f- on cells 1..7
    const T c = diss_shift(w[3 * stride]);  // one shift for the three faces (see diss_shift)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T fk = f[k * stride], wk = w[k * stride] - c;
      if (k < 7) p[k] = fma(sf, fk, wk);
      if (k > 0) m[k] = fma(sf, fk, -wk);
    }
    Win<T> wp[6], wm[7];
#pragma unroll
    for (int c = 1; c <= 5; ++c) wp[c] = win(p[c - 1], p[c], p[c + 1]);
#pragma unroll
    for (int c = 2; c <= 6; ++c) wm[c] = win(m[c - 1], m[c], m[c + 1]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T q0 = cfar(p[j], p[j + 1], p[j + 2]);
      const T q1 = c6(p[j + 1], p[j + 2], p[j + 3]);
      const T q2 = c3(p[j + 2], p[j + 3], p[j + 4]);
      const T r0 = cfar(m[j + 5], m[j + 4], m[j + 3]);
      const T r1 = c6(m[j + 4], m[j + 3], m[j + 2]);
      const T r2 = c3(m[j + 3], m[j + 2], m[j + 1]);
      T np, dp, nm, dm;
      nd(ind0(wp[j + 1]), ind1(wp[j + 2]), ind2(wp[j + 3]), q0, q1, q2, np, dp);
      nd(ind2(wm[j + 4]), ind1(wm[j + 3]), ind0(wm[j + 2]), r0, r1, r2, nm, dm);
      out[j] = sum2(np, dp, nm, dm);
    }
  } else {
    T c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = f[k * stride];
    Win<T> wc[7];
#pragma unroll
    for (int k = 1; k <= 6; ++k) wc[k] = win(c[k - 1], c[k], c[k + 1]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T M6 = c6(c[j + 1], c[j + 2], c[j + 3]);
      const T N6 = c6(c[j + 4], c[j + 3], c[j + 2]);
      const T P = cfar(c[j], c[j + 1], c[j + 2]);
      const T Pm = cfar(c[j + 5], c[j + 4], c[j + 3]);
      T np, dp, nm, dm;
      nd(ind0(wc[j + 1]), ind1(wc[j + 2]), ind2(wc[j + 3]), P, M6, T(0.5) * N6, np, dp);
      nd(ind2(wc[j + 4]), ind1(wc[j + 3]), ind0(wc[j + 2]), Pm, N6, T(0.5) * M6, nm, dm);
      out[j] = sf * sum2(np, dp, nm, dm);
    }
  }
}

// Faces per thread in the flux rounds: three (face_flux3) for WENO5 where the registers
// allow it without fewer waves per SIMD: float, and the float64 stage-terms kernel on
// 64 x 16 tiles, whose LDS already limits it to six waves per SIMD (ST: the stage-terms
// kernel); one otherwise.
template <typename T, int WO, int TY = 8, int NT = 256, bool ST = false>
constexpr int faces_per_thread() {
  return WO == 5 && (sizeof(T) == 4 || (ST && TY == 16 && NT == 512)) ? 3 : 1;
}

// LDS tile geometry for a 64 x TY tile with a 3-cell halo, worked on by NT threads
// (NT / 64 wavefronts; thread t owns column t % 64 and rows t / 64 + (NT / 64) k).
template <int TY, int NT>
struct Geo {
  static constexpr int W = kTileX + 2 * kHalo;
  static constexpr int HT = TY + 2 * kHalo;
  static constexpr int PL = W * HT;                   // elements per staged plane
  static constexpr int FXN = TY * (kTileX + 1);       // x faces
  static constexpr int FXP = (FXN + 63) / 64 * 64;    // x faces padded to whole waves
  static constexpr int FYN = (TY + 1) * kTileX;       // y faces
  static constexpr int WV = NT / 64;                  // wavefronts
  static constexpr int ROWS = TY / WV;                // rows per thread
  static_assert(ROWS * WV == TY, "tile rows must split evenly over the wavefronts");
  __device__ static int at(int lx, int ly) { return (ly + kHalo) * W + lx + kHalo; }
};

// Value at a 32-bit byte offset from a plane base.
template <typename G>
__device__ __forceinline__ G ld_byte(Gp<const G> base, unsigned boff) {
  return *reinterpret_cast<Gp<const G>>(reinterpret_cast<Gp<const char>>(base) + boff);
}

// Staging of NP planes (with periodic halo H) into LDS in two phases: load() issues
// every global load of the thread into registers, store() converts, scales and writes
// them to LDS.  Loads of several planes (and of later phases) are thus in flight
// together instead of each waiting for the one before.  Element idx of the staged
// (TY + 2H) x (64 + 2H) region is held by thread idx % NT in slot idx / NT.
template <int TY, int NT, int NP, typename G, int H = kHalo>
struct Stage {
  static constexpr int W = kTileX + 2 * H;
  static constexpr int PL = W * (TY + 2 * H);
  static constexpr int IT = (PL + NT - 1) / NT;
  G v[NP][IT];
  __device__ __forceinline__ void load(const Gp<const G> *plane, int nx, int ny, int x0, int y0) {
    const bool inner = x0 >= H && x0 + kTileX + H <= nx && y0 >= H && y0 + TY + H <= ny;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      // byte offset in 32 bits (a plane holds at most 8192^2 float64 values, 512 MiB),
      // so each load takes the plane base as a scalar and this offset as its only
      // per-lane address
      const unsigned boff =
          idx < PL ? (unsigned)staged_cell(idx, W, H, nx, ny, x0, y0, inner) * (unsigned)sizeof(G)
                   : 0u;
#pragma unroll
      for (int p = 0; p < NP; ++p) v[p][it] = ld_byte(plane[p], boff);
    }
  }
  template <typename S>
  __device__ __forceinline__ void store(S *const *lds, S sc) const {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = threadIdx.x + it * NT;
        if (idx < PL) lds[p][idx] = sc * (S)v[p][it];
      }
  }
};

// x faces (TY rows x 65) and y faces (TY + 1 rows x 64) of two fluxes in one index
// space; the x part is padded to whole wavefronts so no wavefront mixes the two.  With
// three faces per thread an item is a run of three faces along the flux direction; the
// last run of a row (column) starts three faces before its end and stores only the faces
// no earlier run covers, so every read stays inside the staged tile.
template <int TY, int NT, int WO, typename T, bool DX, bool DY,
          int FPT = faces_per_thread<T, WO>()>
__device__ __forceinline__ void faces(T *fx, T *fy, const T *fxf, const T *fxw, T sx,
                                      const T *fyf, const T *fyw, T sy) {
  using Gm = Geo<TY, NT>;
  if constexpr (FPT == 3) {
    constexpr int NFX = kTileX + 1, NIX = (NFX + 2) / 3;  // x faces, runs per row
    constexpr int XI = TY * NIX, XIP = (XI + 63) / 64 * 64;
    constexpr int NFY = TY + 1, NIY = (NFY + 2) / 3;      // y faces, runs per column
    constexpr int YI = NIY * kTileX;
    for (int idx = threadIdx.x; idx < XIP + YI; idx += NT) {
      T o[3];
      if (idx < XIP) {
        if (idx < XI) {
          const int ly = idx / NIX, i = idx - ly * NIX;
          const int f0 = min(3 * i, NFX - 3);
          const int base = (ly + kHalo) * Gm::W + f0;  // cell f0 - 3 of row ly
          face_flux3<T, DX>(fxf + base, fxw + base, 1, sx, o);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (f0 + k >= 3 * i) fx[ly * NFX + f0 + k] = o[k];
        }
      } else {
        const int j = idx - XIP;
        const int i = j / kTileX, lx = j - i * kTileX;
        const int f0 = min(3 * i, NFY - 3);
        const int base = f0 * Gm::W + lx + kHalo;  // cell f0 - 3 of column lx
        face_flux3<T, DY>(fyf + base, fyw + base, Gm::W, sy, o);
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (f0 + k >= 3 * i) fy[(f0 + k) * kTileX + lx] = o[k];
      }
    }
    return;
  }
  for (int idx = threadIdx.x; idx < Gm::FXP + Gm::FYN; idx += NT) {
    if (idx < Gm::FXP) {
      if (idx < Gm::FXN) {
        const int ly = idx / (kTileX + 1);
        const int f = idx - ly * (kTileX + 1);
        const int base = (ly + kHalo) * Gm::W + f;  // cell f - 3 of row ly
        fx[idx] = face_flux<T, DX, WO>(fxf + base, fxw + base, 1, sx);
      }
    } else {
      const int j = idx - Gm::FXP;
      const int f = j / kTileX;
      const int lx = j - f * kTileX;
      const int base = f * Gm::W + lx + kHalo;  // cell f - 3 of column lx
      fy[j] = face_flux<T, DY, WO>(fyf + base, fyw + base, Gm::W, sy);
    }
  }
}

template <int TY, typename T>
__device__ __forceinline__ T face_dx(const T *fx, int lx, int ly, T ihx) {
  return (fx[ly * (kTileX + 1) + lx + 1] - fx[ly * (kTileX + 1) + lx]) * ihx;
}
template <int TY, typename T>
__device__ __forceinline__ T face_dy(const T *fy, int lx, int ly, T ihy) {
  return (fy[(ly + 1) * kTileX + lx] - fy[ly * kTileX + lx]) * ihy;
}

// Central differences from an LDS plane at index c (stride st: 1 for x, W for y), with
// the scale factor f passed in: order 4 (the high-order extension of Section 3.2)
//   D f = (f-2 - 8 f-1 + 8 f+1 - f+2) / (12 h),
//   L f = (-f-2 + 16 f-1 - 30 f0 + 16 f+1 - f+2) / (12 h^2),
// order 2 (as printed in Section 3.2) D f = (f+1 - f-1) / (2 h), L f = (f-1 - 2 f0 + f+1)
// / h^2; D_xy = D_x D_y in both.  The factors (central_f1, central_f2 of 1/h) come with
// the instance (Inst::f1x ... f2y), evaluated once on the host.
template <int CO>
struct Central;
template <>
struct Central<4> {
  static constexpr int R = 2;  // reach
  template <typename S>
  __device__ static S d1(const S *p, int c, int st, S f) {
    return (p[c - 2 * st] - S(8) * p[c - st] + S(8) * p[c + st] - p[c + 2 * st]) * f;
  }
  template <typename S>
  __device__ static S d2(const S *p, int c, int st, S f) {
    return (-p[c - 2 * st] + S(16) * p[c - st] - S(30) * p[c] + S(16) * p[c + st] -
            p[c + 2 * st]) *
           f;
  }
  // float64 arithmetic on values of type S
  template <typename S>
  __device__ static double d2w(const S *p, int c, int st, double f) {
    return (-(double)p[c - 2 * st] + 16.0 * (double)p[c - st] - 30.0 * (double)p[c] +
            16.0 * (double)p[c + st] - (double)p[c + 2 * st]) *
           f;
  }
  template <typename S>
  __device__ static double dxyw(const S *p, int c, int W, double fx, double fy) {
    const int o[4] = {-2, -1, 1, 2};
    const double w[4] = {1.0, -8.0, 8.0, -1.0};
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double dy = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) dy += w[b] * (double)p[c + o[a] + o[b] * W];
      acc += w[a] * (dy * fy);
    }
    return acc * fx;
  }
  template <typename S>
  __device__ static S dxy(const S *p, int c, int W, S fx, S fy) {
    const int o[4] = {-2, -1, 1, 2};
    const S w[4] = {S(1), S(-8), S(8), S(-1)};
    S acc = S(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      S dy = S(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) dy += w[b] * p[c + o[a] + o[b] * W];
      acc += w[a] * (dy * fy);
    }
    return acc * fx;
  }
};
template <>
struct Central<2> {
  static constexpr int R = 1;
  template <typename S>
  __device__ static S d1(const S *p, int c, int st, S f) {
    return (p[c + st] - p[c - st]) * f;
  }
  template <typename S>
  __device__ static S d2(const S *p, int c, int st, S f) {
    return (p[c - st] - S(2) * p[c] + p[c + st]) * f;
  }
  template <typename S>
  __device__ static S dxy(const S *p, int c, int W, S fx, S fy) {
    const S dyp = (p[c + 1 + W] - p[c + 1 - W]) * fy, dym = (p[c - 1 + W] - p[c - 1 - W]) * fy;
    return (dyp - dym) * fx;
  }
  template <typename S>
  __device__ static double d2w(const S *p, int c, int st, double f) {
    return ((double)p[c - st] - 2.0 * (double)p[c] + (double)p[c + st]) * f;
  }
  template <typename S>
  __device__ static double dxyw(const S *p, int c, int W, double fx, double fy) {
    const double dyp = ((double)p[c + 1 + W] - (double)p[c + 1 - W]) * fy,
                 dym = ((double)p[c - 1 + W] - (double)p[c - 1 - W]) * fy;
    return (dyp - dym) * fx;
  }
};

// float64 central first difference of the 2R + 1 values w[0..2R] centred on w[R], with
// its evaluation order fixed by explicit fused operations, so that every kernel forming
// D0.u of the float64 velocity (the last stage of the FP32-split form and the set-up
// kernel k_div_u) gets the same bits from the same values.
template <int CO>
__device__ __forceinline__ double d0_fixed(const double *w, double f) {
  if constexpr (CO == 2) return (w[2] - w[0]) * f;
  return fma(8.0, w[3] - w[1], w[0] - w[4]) * f;
}

template <typename T>
__device__ __forceinline__ Gp<T> tplane(const Inst &I, int slot) {
  return gp(reinterpret_cast<T *>(I.tbase) + (long long)slot * I.plane);
}
__device__ __forceinline__ Gp<double> dplane(const Inst &I, int slot) {
  return gp(I.dbase + (long long)slot * I.plane);
}

// One cell of every plane: its byte offsets in transport and float64 planes, in 32 bits
// (a plane holds at most 8192^2 float64 values, 512 MiB), so a load or store takes the
// plane base as a scalar and one shared offset as its per-lane address.
struct Cell {
  unsigned t, d;
};
template <typename T>
__device__ __forceinline__ Cell cell_at(int idx) {
  return Cell{(unsigned)idx * (unsigned)sizeof(T), (unsigned)idx * 8u};
}
template <typename T>
__device__ __forceinline__ Gp<T> tcell(const Inst &I, int slot, const Cell &c) {
  return reinterpret_cast<Gp<T>>(reinterpret_cast<Gp<char>>(tplane<T>(I, slot)) + c.t);
}
__device__ __forceinline__ Gp<double> dcell(const Inst &I, int slot, const Cell &c) {
  return reinterpret_cast<Gp<double>>(reinterpret_cast<Gp<char>>(dplane(I, slot)) + c.d);
}

// History terms of a stage update at one cell: s_k += sum_{j < n} c_j plane(slot[j][k]),
// k < NC components, accumulated in float64 in the order j = 0, 1, ...  load() issues the
// loads of the first kHistBatch terms together, ahead of any use (a plain loop waits for
// each load before issuing the next, one memory round trip per term); add() sums them
// and takes any further terms one by one.
constexpr int kHistBatch = 3;
template <typename T, int NC>
struct Hist {
  T v[kHistBatch][NC];
  __device__ __forceinline__ void load(const Inst &I, const int *slot, int n, const Cell &g) {
#pragma unroll
    for (int j = 0; j < kHistBatch; ++j)
      if (j < n)
#pragma unroll
        for (int k = 0; k < NC; ++k) v[j][k] = *tcell<T>(I, slot[j * NC + k], g);
  }
  __device__ __forceinline__ void add(const Inst &I, double *s, const int *slot, const double *c,
                                      int n, const Cell &g) const {
#pragma unroll
    for (int j = 0; j < kHistBatch; ++j)
      if (j < n)
#pragma unroll
        for (int k = 0; k < NC; ++k) s[k] += c[j] * (double)v[j][k];
    for (int j = kHistBatch; j < n; ++j)
#pragma unroll
      for (int k = 0; k < NC; ++k) s[k] += c[j] * (double)*tcell<T>(I, slot[j * NC + k], g);
  }
};

// ------------------------------------------------------------------ step 2 RHS

template <typename T, int TY, int NT, int CO>
__global__ __launch_bounds__(NT) void k_helmholtz_rhs(const Inst *__restrict__ insts,
                                                                   const Work *__restrict__ work,
                                                                   int nwork, ArgsR a) {
  using Gm = Geo<TY, NT>;
  __shared__ T sV1[Gm::PL], sV2[Gm::PL];
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  Stage<TY, NT, 2, T> st;
  {
    const Gp<const T> g[2] = {tplane<T>(I, a.v[0]), tplane<T>(I, a.v[1])};
    st.load(g, I.nx, I.ny, wk.a, wk.b);
  }
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  const bool col = gx < I.nx;
  // pointwise inputs of the right-hand side, loaded while the tile arrives
  const double sig = I.sigma[a.stage];
  const double c_d = I.rdt2[a.stage], c_0 = I.rdt[a.stage], c_l = a.c_l;
  double base[Gm::ROWS];
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int gy = wk.b + ty0 + Gm::WV * r;
    base[r] = 0.0;
    if (col && gy < I.ny) {
      const Cell g = cell_at<T>(gy * I.nx + gx);
      Hist<T, 1> HD, HL;
      HD.load(I, a.D, a.nD, g);
      HL.load(I, a.L, a.nL, g);
      const double thn = *dcell(I, a.thn, g);
      const double du0 = a.du0_dbl ? *dcell(I, a.du0, g) : (double)*tcell<T>(I, a.du0, g);
      double hd = 0.0, hl = 0.0;
      HD.add(I, &hd, a.D, a.cD, a.nD, g);
      HL.add(I, &hl, a.L, a.cL, a.nL, g);
      const double c_u0 = a.du0_dbl ? fma(c_d, a.sum_a, c_0) : c_0;
      base[r] = -sig * thn + c_d * hd + c_u0 * du0 - c_l * hl;
    }
  }
  {
    T *l[2] = {sV1, sV2};
    st.store(l, T(1));
  }
  __syncthreads();
  if (!col) return;
  using C = Central<CO>;
  const double ihx12 = I.f1x, ihy12 = I.f1y;
  const double ihx2 = I.f2x, ihy2 = I.f2y;
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + Gm::WV * r;
    const int gy = wk.b + ly;
    if (gy >= I.ny) break;
    const int c = Gm::at(tx, ly);
    // D0^2 : B(v) = -D_xx v1 + 2 D_x D_y v2 + D_yy v1, in float64 arithmetic whatever T
    // is: its rounding would enter R as white noise, which the inverse of D_Delta carries
    // into the smooth modes of theta (the rounding of v itself enters as the second
    // difference of a noise, which that inverse undoes)
    const double ddb = -C::d2w(sV1, c, 1, ihx2) + 2.0 * C::dxyw(sV2, c, Gm::W, ihx12, ihy12) +
                       C::d2w(sV1, c, Gm::W, ihy2);
    const Cell g = cell_at<T>(gy * I.nx + gx);
    *dcell(I, a.out_r, g) = base[r] - ddb;
    *tcell<T>(I, a.out_ddb, g) = (T)ddb;
  }
}

// D0 theta (both components) and D_Delta theta at staged index c of theta in LDS (row
// length w), in float64: the same stencils and factors as the stage-terms kernel's.
template <int CO>
__device__ __forceinline__ void theta_terms(const double *sT, int c, int w, const Inst &I,
                                            double &dx, double &dy, double &lap) {
  using C = Central<CO>;
  dx = C::d1(sT, c, 1, I.f1x);
  dy = C::d1(sT, c, w, I.f1y);
  lap = C::d2(sT, c, 1, I.f2x) + C::d2(sT, c, w, I.f2y);
}

// ------------------------------------------------------------------ steps 3 and 4

// Everything of steps 3 and 4 that does not involve theta(i): q(i) in full, and u(i)
// short of its theta gradient,
//   u*(i) = u^n - dt sum_j cH_j Hu(j) - dt a_ii D_W.B(v(i)),
// so this kernel can run while the Helmholtz solve of the same stage produces theta(i).
// The stage-terms kernel of the stage subtracts dt a_ii D0 theta(i) from u*(i).  In the
// FP32-split form (a.un[0] == kNoSlot) the kernel stores the increment u*(i) - u^n: it is
// of size dt |Hu|, so its float rounding is that much smaller than the rounding of u.
template <typename T, int TY, int NT, int WO, bool FUSED>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(update_waves_per_eu<T, TY, NT>()))) void k_update_uq(const Inst *__restrict__ insts,
                                                               const Work *__restrict__ work,
                                                               int nwork, ArgsUQ a) {
  using Gm = Geo<TY, NT>;
  // v1, v2 and one partner component at a time, halved for the fluxes (the second
  // component arrives in registers during the first round and replaces the first)
  // (one buffer, which the fused schedule reuses for theta(i) after the flux rounds)
  using STh = Stage<TY, NT, 1, double, 2>;  // theta(i) with the reach of D0 and D_Delta
  static_assert(STh::PL * sizeof(double) <= 3 * Gm::PL * sizeof(T), "theta staging");
  __shared__ __align__(16) T sVP[3 * Gm::PL];
  T *const sV1 = sVP, *const sV2 = sVP + Gm::PL, *const sP = sVP + 2 * Gm::PL;
  __shared__ T fx[Gm::FXN], fy[Gm::FYN];
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  Stage<TY, NT, 1, T> sp2;
  {
    Stage<TY, NT, 3, T> st;
    const Gp<const T> g[3] = {tplane<T>(I, a.v[0]), tplane<T>(I, a.v[1]), tplane<T>(I, a.partner[0])};
    st.load(g, nx, ny, wk.a, wk.b);
    const Gp<const T> g2[1] = {tplane<T>(I, a.partner[1])};
    sp2.load(g2, nx, ny, wk.a, wk.b);
    T *l[3] = {sV1, sV2, sP};
    st.store(l, T(0.5));
  }
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  const bool col = gx < nx;
  __syncthreads();
  const T ihx = T(I.ihx), ihy = T(I.ihy);
  T hu1[Gm::ROWS], hu2[Gm::ROWS], dv[Gm::ROWS];
  // first row of B(v) = (-v1, v2), dissipation on u1
  faces<TY, NT, WO, T, true, true>(fx, fy, sV1, sP, T(-1), sV2, sP, T(1));
  __syncthreads();
  {
    T *l[1] = {sP};
    sp2.store(l, T(0.5));
  }
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    hu1[r] = face_dx<TY>(fx, tx, ty0 + Gm::WV * r, ihx) + face_dy<TY>(fy, tx, ty0 + Gm::WV * r, ihy);
    keep(hu1[r]);
  }
  __syncthreads();
  // second row of B(v) = (v2, v1), dissipation on u2
  faces<TY, NT, WO, T, true, true>(fx, fy, sV2, sP, T(1), sV1, sP, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    hu2[r] = face_dx<TY>(fx, tx, ty0 + Gm::WV * r, ihx) + face_dy<TY>(fy, tx, ty0 + Gm::WV * r, ihy);
    keep(hu2[r]);
  }
  __syncthreads();
  // fused schedule: theta(i) staged with a halo of 2 into the flux planes once they are
  // free; its loads are issued before the last flux round, which hides their latency
  constexpr bool fused = FUSED;  // a.th != kNoSlot (the launch picks the instantiation)
  double *const sT = reinterpret_cast<double *>(sVP);
  STh sth;
  if constexpr (fused) {
    const Gp<const double> gt[1] = {dplane(I, a.th)};
    sth.load(gt, nx, ny, wk.a, wk.b);
  }
  // div v without dissipation
  faces<TY, NT, WO, T, false, false>(fx, fy, sV1, sV1, T(1), sV2, sV2, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r)
    dv[r] = face_dx<TY>(fx, tx, ty0 + Gm::WV * r, ihx) + face_dy<TY>(fy, tx, ty0 + Gm::WV * r, ihy);
  if constexpr (fused) {
    double *lt[1] = {sT};
    sth.store(lt, 1.0);
    __syncthreads();
  }

  if (!col) return;
  // pointwise inputs of the updates (state n and the stage history), loaded after the
  // fluxes so that they hold no registers through them; float64 history sums
  double un1[Gm::ROWS], un2[Gm::ROWS], qn[Gm::ROWS], h1[Gm::ROWS], h2[Gm::ROWS], hg[Gm::ROWS];
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int gy = wk.b + ty0 + Gm::WV * r;
    un1[r] = un2[r] = qn[r] = h1[r] = h2[r] = hg[r] = 0.0;
    if (gy < ny) {
      const Cell g = cell_at<T>(gy * nx + gx);
      Hist<T, 2> HH;
      Hist<T, 1> HG;
      HH.load(I, &a.H[0][0], a.nH, g);
      HG.load(I, a.G, a.nG, g);
      if (a.un[0] != kNoSlot) {  // else the increment du*(i) of the split form
        un1[r] = (double)*tcell<T>(I, a.un[0], g);
        un2[r] = (double)*tcell<T>(I, a.un[1], g);
      }
      qn[r] = (double)*tcell<T>(I, a.qn, g);
      double h[2] = {0.0, 0.0};
      HH.add(I, h, &a.H[0][0], a.cH, a.nH, g);
      HG.add(I, &hg[r], a.G, a.cG, a.nG, g);
      h1[r] = h[0];
      h2[r] = h[1];
    }
  }
  const double dt = I.dt, te2 = I.te2, kinv = I.kinv[a.stage], aii = a.aii;
  const double htau = 0.5 * I.tau;
  const double cth = dt * aii;
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int gy = wk.b + ty0 + Gm::WV * r;
    if (gy >= ny) break;
    const Cell g = cell_at<T>(gy * nx + gx);
    const double Hq = htau * (double)dv[r];
    const double q = (te2 * qn[r] - dt * aii * Hq - dt * hg[r]) * kinv;
    const double us1 = un1[r] - dt * (h1[r] + aii * (double)hu1[r]);
    const double us2 = un2[r] - dt * (h2[r] + aii * (double)hu2[r]);
    if constexpr (fused) {
      // the theta part of step 3, with theta(i) of this stage already solved
      double d0x, d0y, lap;
      const int ct = (ty0 + Gm::WV * r + 2) * STh::W + tx + 2;
      if (a.co == 2)
        theta_terms<2>(sT, ct, STh::W, I, d0x, d0y, lap);
      else
        theta_terms<4>(sT, ct, STh::W, I, d0x, d0y, lap);
      *tcell<T>(I, a.out_us[0], g) = (T)(us1 - cth * d0x);
      *tcell<T>(I, a.out_us[1], g) = (T)(us2 - cth * d0y);
      if (a.out_hu[0] != kNoSlot) {
        *tcell<T>(I, a.out_hu[0], g) = (T)((double)hu1[r] + d0x);
        *tcell<T>(I, a.out_hu[1], g) = (T)((double)hu2[r] + d0y);
      }
      if (a.out_lt != kNoSlot)
        *tcell<T>(I, a.out_lt, g) = (T)((double)*tcell<T>(I, a.ddb, g) + lap);
    } else {
      *tcell<T>(I, a.out_us[0], g) = (T)us1;
      *tcell<T>(I, a.out_us[1], g) = (T)us2;
      if (a.out_hu[0] != kNoSlot) {
        *tcell<T>(I, a.out_hu[0], g) = hu1[r];
        *tcell<T>(I, a.out_hu[1], g) = hu2[r];
      }
    }
    *tcell<T>(I, a.out_q, g) = (T)q;
    if (a.out_hu[0] != kNoSlot) *tcell<T>(I, a.out_gq, g) = (T)(Hq + q);
  }
}

// ------------------------------------------------------------------ grad q

// G = te2 D_W q[dissipation on v] of a stage: the part of its terms E that needs q(i)
// and v(i) only, so it runs beside the Helmholtz solve of the stage.
template <typename T, int TY, int NT, int WO>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(weno_waves_per_eu<TY, NT>()))) void k_grad_q(const Inst *__restrict__ insts,
                                                              const Work *__restrict__ work,
                                                              int nwork, ArgsG a) {
  using Gm = Geo<TY, NT>;
  __shared__ T sQ[Gm::PL], sV1[Gm::PL], sV2[Gm::PL];
  __shared__ T fx[Gm::FXN], fy[Gm::FYN];
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  {
    Stage<TY, NT, 3, T> st;
    const Gp<const T> g[3] = {tplane<T>(I, a.q), tplane<T>(I, a.v[0]), tplane<T>(I, a.v[1])};
    st.load(g, nx, ny, wk.a, wk.b);
    T *l[3] = {sQ, sV1, sV2};
    st.store(l, T(0.5));
  }
  __syncthreads();
  faces<TY, NT, WO, T, true, true>(fx, fy, sQ, sV1, T(1), sQ, sV2, T(1));
  __syncthreads();
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  if (gx >= nx) return;
  const T ihx = T(I.ihx), ihy = T(I.ihy), te2 = T(I.te2);
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + Gm::WV * r;
    const int gy = wk.b + ly;
    if (gy >= ny) break;
    const Cell g = cell_at<T>(gy * nx + gx);
    *tcell<T>(I, a.out_g[0], g) = te2 * face_dx<TY>(fx, tx, ly, ihx);
    *tcell<T>(I, a.out_g[1], g) = te2 * face_dy<TY>(fy, tx, ly, ihy);
  }
}

template <typename T, int TY, int NT, int CO, typename SU>
__device__ __forceinline__ void increment_tail(const Inst &I, const Work &wk, const ArgsE &a,
                                               double *sU1, double *sU2, double f1x,
                                               double f1y);

// FP32-split completion of a stage (the increment form of k_stage_terms, below), with
// the staged velocity in float64.  Phase 1 writes the theta terms of the interior cells
// (Hu, Ltheta) and stages the increment du(i) = du*(i) - dt a_ii D0 theta(i).  Phase 2
// forms D0.du(i) at the interior cells (the stages before the last).  Phase 3 stages
// u(i) = u^n + du(i), halved, for the flux rounds (in float64: the viscous term
// (tau/4) D0_W.B(u) of E would otherwise carry the float rounding of u divided by h), and
// writes the interior velocities: float u(i) and, in the last stage, the float64 state
// u^{n+1} = u^n + du(s) with its float copy; the last stage then forms the float64
// D0.u^{n+1} from the staged values, which are the stored state (so it equals D0 of the
// stored state bit for bit, as k_div_u forms it after a restart).  Only the float
// rounding of du*(i), of size dt |Hu|, reaches D0.u.
template <typename T, int TY, int NT, int CO, typename SU>
__device__ __forceinline__ void stage_increment(const Inst &I, const Work &wk, const ArgsE &a,
                                                const SU &su, const double *sT, double *sU1,
                                                double *sU2, const T *hv1, const T *hv2,
                                                const T *dd, bool want_hu, bool want_lt,
                                                double cth, double f1x, double f1y) {
  using Gm = Geo<TY, NT>;
  using C = Central<CO>;
  constexpr int SWW = kTileX + 2 * (kHalo + C::R);  // row length of the staged theta
  constexpr int R = C::R;
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  const bool col = gx < nx;
  // phase 1
  if (col) {
    const double f2x = I.f2x, f2y = I.f2y;
#pragma unroll
    for (int r = 0; r < Gm::ROWS; ++r) {
      const int ly = ty0 + Gm::WV * r;
      const int gy = wk.b + ly;
      if (gy >= ny) break;
      const Cell g = cell_at<T>(gy * nx + gx);
      const int cw = (ly + kHalo + R) * SWW + tx + kHalo + R;
      if (want_hu) {
        *tcell<T>(I, a.hu[0], g) = (T)((double)hv1[r] + C::d1(sT, cw, 1, f1x));
        *tcell<T>(I, a.hu[1], g) = (T)((double)hv2[r] + C::d1(sT, cw, SWW, f1y));
      }
      if (want_lt) {
        const double lap = C::d2(sT, cw, 1, f2x) + C::d2(sT, cw, SWW, f2y);
        *tcell<T>(I, a.out_lt, g) = (T)((double)dd[r] + lap);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < SU::IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= Gm::PL) break;
    const int ly = idx / Gm::W, lx = idx - ly * Gm::W;
    const int c = (ly + R) * SWW + lx + R;
    sU1[idx] = (double)su.v[0][it] - cth * C::d1(sT, c, 1, f1x);
    sU2[idx] = (double)su.v[1][it] - cth * C::d1(sT, c, SWW, f1y);
  }
  __syncthreads();
  increment_tail<T, TY, NT, CO, SU>(I, wk, a, sU1, sU2, f1x, f1y);
}

// Phases 2 and 3 of the FP32-split completion, on the staged increment du(i) in sU1, sU2
// (from phase 1, or in the fused schedule the increment the update launch completed).
template <typename T, int TY, int NT, int CO, typename SU>
__device__ __forceinline__ void increment_tail(const Inst &I, const Work &wk, const ArgsE &a,
                                               double *sU1, double *sU2, double f1x,
                                               double f1y) {
  using Gm = Geo<TY, NT>;
  using C = Central<CO>;
  constexpr int R = C::R;
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  const bool col = gx < nx;
  const bool last = a.out_ud[0] != kNoSlot;
  // u^n on the staged region (float64, or its float copy when no float64 base is given)
  double b1[SU::IT], b2[SU::IT];
  if (a.ub[0] != kNoSlot) {
    Stage<TY, NT, 2, double> sb;
    const Gp<const double> g2[2] = {dplane(I, a.ub[0]), dplane(I, a.ub[1])};
    sb.load(g2, nx, ny, wk.a, wk.b);
#pragma unroll
    for (int it = 0; it < SU::IT; ++it) {
      b1[it] = sb.v[0][it];
      b2[it] = sb.v[1][it];
    }
  } else {
    Stage<TY, NT, 2, T> sb;
    const Gp<const T> g2[2] = {tplane<T>(I, a.u[0]), tplane<T>(I, a.u[1])};
    sb.load(g2, nx, ny, wk.a, wk.b);
#pragma unroll
    for (int it = 0; it < SU::IT; ++it) {
      b1[it] = (double)sb.v[0][it];
      b2[it] = (double)sb.v[1][it];
    }
  }
  // phase 2: D0 of the increment (the stages before the last)
  if (col && !last && a.out_du != kNoSlot) {
#pragma unroll
    for (int r = 0; r < Gm::ROWS; ++r) {
      const int ly = ty0 + Gm::WV * r;
      const int gy = wk.b + ly;
      if (gy >= ny) break;
      const int c = Gm::at(tx, ly);
      double wx[2 * R + 1], wy[2 * R + 1];
#pragma unroll
      for (int k = -R; k <= R; ++k) {
        wx[k + R] = sU1[c + k];
        wy[k + R] = sU2[c + k * Gm::W];
      }
      const Cell g = cell_at<T>(gy * nx + gx);
      *tcell<T>(I, a.out_du, g) = (T)(d0_fixed<CO>(wx, f1x) + d0_fixed<CO>(wy, f1y));
    }
  }
  __syncthreads();
  // phase 3: each thread replaces the increments of its own staged elements
#pragma unroll
  for (int it = 0; it < SU::IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx >= Gm::PL) break;
    const double u1 = b1[it] + sU1[idx], u2 = b2[it] + sU2[idx];
    sU1[idx] = 0.5 * u1;
    sU2[idx] = 0.5 * u2;
    const int ly = idx / Gm::W, lx = idx - ly * Gm::W;
    const int gxs = wk.a + lx - kHalo, gys = wk.b + ly - kHalo;
    if (lx >= kHalo && lx < kHalo + kTileX && ly >= kHalo && ly < kHalo + TY && gxs < nx &&
        gys < ny) {
      const Cell g = cell_at<T>(gys * nx + gxs);
      *tcell<T>(I, a.out_u[0], g) = (T)u1;
      *tcell<T>(I, a.out_u[1], g) = (T)u2;
      if (last) {
        *dcell(I, a.out_ud[0], g) = u1;
        *dcell(I, a.out_ud[1], g) = u2;
      }
    }
  }
  if (last) {
    // the float64 D0.u of the new state from the staged u (halved exactly, so twice a
    // staged value is the u formed above)
    __syncthreads();
    if (col) {
#pragma unroll
      for (int r = 0; r < Gm::ROWS; ++r) {
        const int ly = ty0 + Gm::WV * r;
        const int gy = wk.b + ly;
        if (gy >= ny) break;
        const int c = Gm::at(tx, ly);
        double wx[2 * R + 1], wy[2 * R + 1];
#pragma unroll
        for (int k = -R; k <= R; ++k) {
          wx[k + R] = 2.0 * sU1[c + k];
          wy[k + R] = 2.0 * sU2[c + k * Gm::W];
        }
        const Cell g = cell_at<T>(gy * nx + gx);
        *dcell(I, a.du0_out, g) = d0_fixed<CO>(wx, f1x) + d0_fixed<CO>(wy, f1y);
      }
    }
  }
}

// D0.u of the float64 velocity of a state (FP32-split form): once after new fields or a
// restore; the steps then carry the float64 D0.u^n themselves.  64 x 16 tiles on 256
// threads; neighbours read straight from the planes (this runs outside the steps).
template <int CO>
__global__ __launch_bounds__(256) void k_div_u(const Inst *__restrict__ insts,
                                               const Work *__restrict__ work, int nwork,
                                               int su1, int su2, int out) {
  using C = Central<CO>;
  constexpr int R = C::R;
  const Work wk = work[blockIdx.x];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  const int gx = wk.a + (threadIdx.x & 63);
  if (gx >= nx) return;
  const Gp<const double> p1 = dplane(I, su1), p2 = dplane(I, su2);
  const double f1x = I.f1x, f1y = I.f1y;
  for (int ly = threadIdx.x >> 6; ly < 16; ly += 4) {
    const int gy = wk.b + ly;
    if (gy >= ny) break;
    double wx[2 * R + 1], wy[2 * R + 1];
#pragma unroll
    for (int k = -R; k <= R; ++k) {
      wx[k + R] = p1[(long long)gy * nx + wrap(gx + k, nx)];
      wy[k + R] = p2[(long long)wrap(gy + k, ny) * nx + gx];
    }
    const Cell g = cell_at<double>(gy * nx + gx);
    *dcell(I, out, g) = d0_fixed<CO>(wx, f1x) + d0_fixed<CO>(wy, f1y);
  }
}

// ------------------------------------------------------------------ stage terms

// Completion of a stage and the terms of it that later stages reuse:
//   u(i) = u*(i) - dt a_ii D0 theta(i)          (the theta part of step 3),
//   Hu(i) = D_W.B(v(i)) + D0 theta(i),  Ltheta = D0^2:B(v) + D_Delta theta,
//   E = (tau/4) D0_W.B(u) + G - F(u),  D0.u    (G = te2 D_W q[v] from k_grad_q),
// and, fused, step 1 of the next stage: v(next) from v^n, the history and this E and v.
// Without u* (a.us[0] == kNoSlot: the terms of a given state) u is read as it is.
//
// theta(i) is staged with a halo of 3 + reach, so that D0 theta is known on the whole
// WENO-staged region: every thread completes u on the cells it stages (the halo ones
// redundantly, in the same arithmetic as their owner), then u, Hu and Ltheta are written
// for the interior cells.  theta uses the face buffers, which the flux rounds only need
// later.
template <typename T, int TY, int NT, int WO, int CO, bool GQ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(weno_waves_per_eu<TY, NT>()))) void k_stage_terms(const Inst *__restrict__ insts,
                                                                 const Work *__restrict__ work,
                                                                 int nwork, ArgsE a, ArgsV nv) {
  // FP32-split form: u^n in float64, stage velocities as float increments on it; the
  // staged velocity and the fluxes of E in float64 (TU)
  constexpr bool INC = sizeof(T) == 4;
  using TU = std::conditional_t<INC, double, T>;
  using Gm = Geo<TY, NT>;
  using C = Central<CO>;
  using SU = Stage<TY, NT, 2, T>;                  // u*
  using SW = Stage<TY, NT, 1, double, kHalo + C::R>;  // theta(i), wide halo
  constexpr int FN = Gm::FXN + Gm::FYN;
  constexpr int FT = SW::PL * (int)(sizeof(double) / sizeof(TU));
  static_assert(!GQ || INC, "G is formed here only in the FP32-split form");
  // (one buffer for u: the split form's fused schedule stages q and v into it for G)
  __shared__ __align__(16) TU sUb[2 * Gm::PL];
  TU *const sU1 = sUb, *const sU2 = sUb + Gm::PL;
  static_assert(!GQ || 3 * Gm::PL * sizeof(T) <= 2 * Gm::PL * sizeof(TU), "q, v staging");
  __shared__ __align__(16) TU sF[FN > FT ? FN : FT];
  TU *fx = sF, *fy = sF + Gm::FXN;
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  const bool col = gx < nx;
  if (a.us[0] != kNoSlot) {
    SU su;
    const Gp<const T> g2[2] = {tplane<T>(I, a.us[0]), tplane<T>(I, a.us[1])};
    su.load(g2, nx, ny, wk.a, wk.b);
    SW sw;
    const Gp<const double> gt[1] = {dplane(I, a.th)};
    sw.load(gt, nx, ny, wk.a, wk.b);
    const bool want_hu = a.hu[0] != kNoSlot, want_lt = a.out_lt != kNoSlot;
    // pointwise inputs of this thread's interior cells
    T hv1[Gm::ROWS], hv2[Gm::ROWS], dd[Gm::ROWS];
#pragma unroll
    for (int r = 0; r < Gm::ROWS; ++r) {
      const int gy = wk.b + ty0 + Gm::WV * r;
      hv1[r] = hv2[r] = dd[r] = T(0);
      if (col && gy < ny) {
        const Cell g = cell_at<T>(gy * nx + gx);
        if (want_hu) {
          hv1[r] = *tcell<T>(I, a.hu[0], g);
          hv2[r] = *tcell<T>(I, a.hu[1], g);
        }
        if (want_lt) dd[r] = *tcell<T>(I, a.ddb, g);
      }
    }
    double *sT = reinterpret_cast<double *>(sF);
    {
      double *lt[1] = {sT};
      sw.store(lt, 1.0);
    }
    __syncthreads();
    const double cth = I.dt * a.aii;
    const double f1x = I.f1x, f1y = I.f1y;
    if constexpr (INC) {
      stage_increment<T, TY, NT, CO>(I, wk, a, su, sT, sU1, sU2, hv1, hv2, dd, want_hu, want_lt,
                                     cth, f1x, f1y);
    } else {
#pragma unroll
    for (int it = 0; it < SU::IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx >= Gm::PL) break;
      const int ly = idx / Gm::W, lx = idx - ly * Gm::W;
      const int c = (ly + C::R) * SW::W + lx + C::R;
      const double u1 = (double)su.v[0][it] - cth * C::d1(sT, c, 1, f1x);
      const double u2 = (double)su.v[1][it] - cth * C::d1(sT, c, SW::W, f1y);
      sU1[idx] = T(0.5) * (T)u1;
      sU2[idx] = T(0.5) * (T)u2;
    }
    __syncthreads();
    // u, Hu and Ltheta of this thread's interior cells (the staged u is halved exactly)
    if (col) {
      const double f2x = I.f2x, f2y = I.f2y;
#pragma unroll
      for (int r = 0; r < Gm::ROWS; ++r) {
        const int ly = ty0 + Gm::WV * r;
        const int gy = wk.b + ly;
        if (gy >= ny) break;
        const Cell g = cell_at<T>(gy * nx + gx);
        const int c = Gm::at(tx, ly);
        const int cw = (ly + kHalo + C::R) * SW::W + tx + kHalo + C::R;
        *tcell<T>(I, a.out_u[0], g) = T(2) * sU1[c];
        *tcell<T>(I, a.out_u[1], g) = T(2) * sU2[c];
        if (want_hu) {
          *tcell<T>(I, a.hu[0], g) = (T)((double)hv1[r] + C::d1(sT, cw, 1, f1x));
          *tcell<T>(I, a.hu[1], g) = (T)((double)hv2[r] + C::d1(sT, cw, SW::W, f1y));
        }
        if (want_lt) {
          const double lap = C::d2(sT, cw, 1, f2x) + C::d2(sT, cw, SW::W, f2y);
          *tcell<T>(I, a.out_lt, g) = (T)((double)dd[r] + lap);
        }
      }
    }
    }  // !INC
  } else if constexpr (INC) {
    if (a.ui[0] != kNoSlot) {
      // a stage of the fused schedule: the update launch completed the increment du(i)
      SU su;
      const Gp<const T> g2[2] = {tplane<T>(I, a.ui[0]), tplane<T>(I, a.ui[1])};
      su.load(g2, nx, ny, wk.a, wk.b);
      double *l2[2] = {sU1, sU2};
      su.store(l2, 1.0);
      __syncthreads();
      increment_tail<T, TY, NT, CO, SU>(I, wk, a, sU1, sU2, I.f1x, I.f1y);
    } else {  // the terms of a state: its float64 velocity
      Stage<TY, NT, 2, double> su;
      const Gp<const double> g2[2] = {dplane(I, a.ub[0]), dplane(I, a.ub[1])};
      su.load(g2, nx, ny, wk.a, wk.b);
      double *l2[2] = {sU1, sU2};
      su.store(l2, 0.5);
    }
  } else {
    Stage<TY, NT, 2, T> su;
    const Gp<const T> g2[2] = {tplane<T>(I, a.u[0]), tplane<T>(I, a.u[1])};
    su.load(g2, nx, ny, wk.a, wk.b);
    T *l2[2] = {sU1, sU2};
    su.store(l2, T(0.5));
  }
  __syncthreads();
  const TU ihx = TU(I.ihx), ihy = TU(I.ihy);
  // the staged u is halved: its central derivative carries a factor 2
  const T ihx6 = T(2.0 * I.f1x), ihy6 = T(2.0 * I.f1y);
  const TU qt = TU(0.25 * I.tau);
  // first component of (tau/4) D0_W.B(u); E is assembled at the end
  TU e1[Gm::ROWS];
  // first row of B(u) = (-u1, u2), no dissipation
  constexpr int FPT = faces_per_thread<TU, WO, TY, NT, true>();
  faces<TY, NT, WO, TU, false, false, FPT>(fx, fy, sU1, sU1, TU(-1), sU2, sU2, TU(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    e1[r] = qt * (face_dx<TY>(fx, tx, ty0 + Gm::WV * r, ihx) + face_dy<TY>(fy, tx, ty0 + Gm::WV * r, ihy));
    keep(e1[r]);
  }
  __syncthreads();
  // GQ (split form, fused schedule): G = te2 D_W q[v] is formed here as k_grad_q forms it,
  // from q(i) and v(i) staged after the E rounds
  // second row of B(u) = (u2, u1); D0.u and F(u) from the staged u
  faces<TY, NT, WO, TU, false, false, FPT>(fx, fy, sU2, sU2, TU(1), sU1, sU1, TU(1));
  __syncthreads();
  TU e2[Gm::ROWS], us1[Gm::ROWS], us2[Gm::ROWS];
  T gq1[Gm::ROWS], gq2[Gm::ROWS];
  if constexpr (GQ) {
    // second component of E and the staged u of this thread's cells into registers: the
    // G round reuses both buffers
#pragma unroll
    for (int r = 0; r < Gm::ROWS; ++r) {
      const int ly = ty0 + Gm::WV * r;
      const int c = Gm::at(tx, ly);
      e2[r] = qt * (face_dx<TY>(fx, tx, ly, ihx) + face_dy<TY>(fy, tx, ly, ihy));
      us1[r] = TU(2) * sU1[c];
      us2[r] = TU(2) * sU2[c];
    }
    Stage<TY, NT, 3, T> sg;
    const Gp<const T> g3[3] = {tplane<T>(I, a.q), tplane<T>(I, a.v[0]), tplane<T>(I, a.v[1])};
    sg.load(g3, nx, ny, wk.a, wk.b);
    __syncthreads();
    T *const sQ = reinterpret_cast<T *>(sUb), *const sW1 = sQ + Gm::PL,
             *const sW2 = sQ + 2 * Gm::PL;
    {
      T *l3[3] = {sQ, sW1, sW2};
      sg.store(l3, T(0.5));
    }
    __syncthreads();
    T *const gfx = reinterpret_cast<T *>(sF), *const gfy = gfx + Gm::FXN;
    faces<TY, NT, WO, T, true, true>(gfx, gfy, sQ, sW1, T(1), sQ, sW2, T(1));
    __syncthreads();
    const T ihxT = T(I.ihx), ihyT = T(I.ihy), te2 = T(I.te2);
#pragma unroll
    for (int r = 0; r < Gm::ROWS; ++r) {
      const int ly = ty0 + Gm::WV * r;
      gq1[r] = te2 * face_dx<TY>(gfx, tx, ly, ihxT);
      gq2[r] = te2 * face_dy<TY>(gfy, tx, ly, ihyT);
    }
  }
  if (!col) return;
  // pointwise inputs of E and of the fused step 1: G, v, and
  // rv = te2 v^n - dt * (its history), formed in float64
  const double dt = I.dt, te2d = I.te2;
  T g1[Gm::ROWS], g2[Gm::ROWS], w1[Gm::ROWS], w2[Gm::ROWS];
  double rv1[Gm::ROWS], rv2[Gm::ROWS];
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int gy = wk.b + ty0 + Gm::WV * r;
    g1[r] = g2[r] = w1[r] = w2[r] = T(0);
    rv1[r] = rv2[r] = 0.0;
    if (gy < ny) {
      const Cell g = cell_at<T>(gy * nx + gx);
      if constexpr (GQ) {
        g1[r] = gq1[r];
        g2[r] = gq2[r];
      } else {
        g1[r] = *tcell<T>(I, a.g[0], g);
        g2[r] = *tcell<T>(I, a.g[1], g);
      }
      if (nv.stage > 0) {
        Hist<T, 2> HE, HV;
        HE.load(I, &nv.E[0][0], nv.nE, g);
        HV.load(I, &nv.V[0][0], nv.nV, g);
        w1[r] = *tcell<T>(I, a.v[0], g);
        w2[r] = *tcell<T>(I, a.v[1], g);
        const double vn1 = (double)*tcell<T>(I, nv.vn[0], g);
        const double vn2 = (double)*tcell<T>(I, nv.vn[1], g);
        double h[2] = {0.0, 0.0};
        HE.add(I, h, &nv.E[0][0], nv.cE, nv.nE, g);
        HV.add(I, h, &nv.V[0][0], nv.cV, nv.nV, g);
        rv1[r] = te2d * vn1 - dt * h[0];
        rv2[r] = te2d * vn2 - dt * h[1];
      }
    }
  }
  const double kinv = nv.stage > 0 ? I.kinv[nv.stage] : 0.0;
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + Gm::WV * r;
    const int gy = wk.b + ly;
    if (gy >= ny) break;
    const Cell g = cell_at<T>(gy * nx + gx);
    const int c = Gm::at(tx, ly);
    TU u1, u2, ex2;
    if constexpr (GQ) {
      u1 = us1[r];
      u2 = us2[r];
      ex2 = e2[r];
    } else {
      u1 = TU(2) * sU1[c];
      u2 = TU(2) * sU2[c];
      ex2 = qt * (face_dx<TY>(fx, tx, ly, ihx) + face_dy<TY>(fy, tx, ly, ihy));
    }
    const TU E1 = (e1[r] - TU(0.5) * (u2 * u2 - u1 * u1)) + TU(g1[r]);
    const TU E2 = (ex2 - u1 * u2) + TU(g2[r]);
    if constexpr (!INC)  // the split form stores D0 of the increment, formed above
      *tcell<T>(I, a.out_du, g) = C::d1(sU1, c, 1, ihx6) + C::d1(sU2, c, Gm::W, ihy6);
    if (a.out_e[0] != kNoSlot) {
      *tcell<T>(I, a.out_e[0], g) = (T)E1;
      *tcell<T>(I, a.out_e[1], g) = (T)E2;
    }
    if (nv.stage > 0) {
      // step 1 of the next stage; its newest history terms are this E and this v
      const double v1 = (double)w1[r], v2 = (double)w2[r];
      const double s1 = a.c_e_next * (double)E1 + a.c_v_next * v1;
      const double s2 = a.c_e_next * (double)E2 + a.c_v_next * v2;
      *tcell<T>(I, nv.out[0], g) = (T)((rv1[r] - dt * s1) * kinv);
      *tcell<T>(I, nv.out[1], g) = (T)((rv2[r] - dt * s2) * kinv);
    }
  }
}

// ------------------------------------------------------------------ launchers

// Launch shapes (shape index si): 0 = 64 x 8 tiles on 256 threads, 1 = 64 x 16 on 256,
// 2 = 64 x 16 on 512, 3 = 64 x 8 on 512; then the WENO order (5 or 3) and the central
// order (4 or 2).  The right-hand side kernel has no WENO flux, the update kernel no
// central difference.
template <typename T>
hipError_t launch_helmholtz_rhs(int si, int wo, int co, const Inst *insts, const Work *work,
                                int nwork, const ArgsR &a, hipStream_t st, const Ev &ev) {
  (void)wo;
  const dim3 g(nwork);
  const int key = si * 2 + (co == 4 ? 0 : 1);
  switch (key) {
    case 0: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 8, 256, 4>), g, dim3(256), st, insts, work, nwork, a); break;
    case 1: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 8, 256, 2>), g, dim3(256), st, insts, work, nwork, a); break;
    case 2: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 16, 256, 4>), g, dim3(256), st, insts, work, nwork, a); break;
    case 3: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 16, 256, 2>), g, dim3(256), st, insts, work, nwork, a); break;
    case 4: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 16, 512, 4>), g, dim3(512), st, insts, work, nwork, a); break;
    case 5: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 16, 512, 2>), g, dim3(512), st, insts, work, nwork, a); break;
    case 6: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 8, 512, 4>), g, dim3(512), st, insts, work, nwork, a); break;
    default: APDVM_LAUNCH(ev, (k_helmholtz_rhs<T, 8, 512, 2>), g, dim3(512), st, insts, work, nwork, a); break;
  }
  return hipGetLastError();
}

#define APDVM_ONE(KERNEL, TY, NT, WO, CO, ...) \
  APDVM_LAUNCH(ev, (KERNEL<T, TY, NT, WO, CO, APDVM_GQ>), g, dim3(NT), st, __VA_ARGS__)
#define APDVM_DISPATCH(KERNEL, ...)                                                       \
  do {                                                                                    \
    const dim3 g(nwork);                                                                  \
    const int key = si * 4 + (wo == 5 ? 0 : 2) + (co == 4 ? 0 : 1);                        \
    switch (key) {                                                                        \
      case 0: APDVM_ONE(KERNEL, 8, 256, 5, 4, __VA_ARGS__); break;                         \
      case 1: APDVM_ONE(KERNEL, 8, 256, 5, 2, __VA_ARGS__); break;                         \
      case 2: APDVM_ONE(KERNEL, 8, 256, 3, 4, __VA_ARGS__); break;                         \
      case 3: APDVM_ONE(KERNEL, 8, 256, 3, 2, __VA_ARGS__); break;                         \
      case 4: APDVM_ONE(KERNEL, 16, 256, 5, 4, __VA_ARGS__); break;                        \
      case 5: APDVM_ONE(KERNEL, 16, 256, 5, 2, __VA_ARGS__); break;                        \
      case 6: APDVM_ONE(KERNEL, 16, 256, 3, 4, __VA_ARGS__); break;                        \
      case 7: APDVM_ONE(KERNEL, 16, 256, 3, 2, __VA_ARGS__); break;                        \
      case 8: APDVM_ONE(KERNEL, 16, 512, 5, 4, __VA_ARGS__); break;                        \
      case 9: APDVM_ONE(KERNEL, 16, 512, 5, 2, __VA_ARGS__); break;                        \
      case 10: APDVM_ONE(KERNEL, 16, 512, 3, 4, __VA_ARGS__); break;                       \
      case 11: APDVM_ONE(KERNEL, 16, 512, 3, 2, __VA_ARGS__); break;                       \
      case 12: APDVM_ONE(KERNEL, 8, 512, 5, 4, __VA_ARGS__); break;                        \
      case 13: APDVM_ONE(KERNEL, 8, 512, 5, 2, __VA_ARGS__); break;                        \
      case 14: APDVM_ONE(KERNEL, 8, 512, 3, 4, __VA_ARGS__); break;                        \
      default: APDVM_ONE(KERNEL, 8, 512, 3, 2, __VA_ARGS__); break;                        \
    }                                                                                     \
  } while (0)

template <typename T>
hipError_t launch_update_uq(int si, int wo, int co, const Inst *insts, const Work *work,
                            int nwork, const ArgsUQ &a, hipStream_t st, const Ev &ev) {
  (void)co;  // the central order of the fused theta part travels in a.co
  const dim3 g(nwork);
  const int key = si * 2 + (wo == 5 ? 0 : 1);
#define APDVM_UQ(TY, NT, WO)                                                                   \
  do {                                                                                         \
    if (a.th != kNoSlot)                                                                       \
      APDVM_LAUNCH(ev, (k_update_uq<T, TY, NT, WO, true>), g, dim3(NT), st, insts, work, nwork, \
                   a);                                                                         \
    else                                                                                       \
      APDVM_LAUNCH(ev, (k_update_uq<T, TY, NT, WO, false>), g, dim3(NT), st, insts, work,      \
                   nwork, a);                                                                  \
  } while (0)
  switch (key) {
    case 0: APDVM_UQ(8, 256, 5); break;
    case 1: APDVM_UQ(8, 256, 3); break;
    case 2: APDVM_UQ(16, 256, 5); break;
    case 3: APDVM_UQ(16, 256, 3); break;
    case 4: APDVM_UQ(16, 512, 5); break;
    case 5: APDVM_UQ(16, 512, 3); break;
    case 6: APDVM_UQ(8, 512, 5); break;
    default: APDVM_UQ(8, 512, 3); break;
  }
#undef APDVM_UQ
  return hipGetLastError();
}
template <typename T>
hipError_t launch_grad_q(int si, int wo, const Inst *insts, const Work *work, int nwork,
                         const ArgsG &a, hipStream_t st, const Ev &ev) {
  const dim3 g(nwork);
  const int key = si * 2 + (wo == 5 ? 0 : 1);
  switch (key) {
    case 0: APDVM_LAUNCH(ev, (k_grad_q<T, 8, 256, 5>), g, dim3(256), st, insts, work, nwork, a); break;
    case 1: APDVM_LAUNCH(ev, (k_grad_q<T, 8, 256, 3>), g, dim3(256), st, insts, work, nwork, a); break;
    case 2: APDVM_LAUNCH(ev, (k_grad_q<T, 16, 256, 5>), g, dim3(256), st, insts, work, nwork, a); break;
    case 3: APDVM_LAUNCH(ev, (k_grad_q<T, 16, 256, 3>), g, dim3(256), st, insts, work, nwork, a); break;
    case 4: APDVM_LAUNCH(ev, (k_grad_q<T, 16, 512, 5>), g, dim3(512), st, insts, work, nwork, a); break;
    case 5: APDVM_LAUNCH(ev, (k_grad_q<T, 16, 512, 3>), g, dim3(512), st, insts, work, nwork, a); break;
    case 6: APDVM_LAUNCH(ev, (k_grad_q<T, 8, 512, 5>), g, dim3(512), st, insts, work, nwork, a); break;
    default: APDVM_LAUNCH(ev, (k_grad_q<T, 8, 512, 3>), g, dim3(512), st, insts, work, nwork, a); break;
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch_stage_terms(int si, int wo, int co, const Inst *insts, const Work *work,
                              int nwork, const ArgsE &a, const ArgsV &nv, hipStream_t st,
                              const Ev &ev) {
  if constexpr (sizeof(T) == 4) {
    if (a.q != kNoSlot) {  // the split form's fused schedule forms G here
#define APDVM_GQ true
      APDVM_DISPATCH(k_stage_terms, insts, work, nwork, a, nv);
#undef APDVM_GQ
      return hipGetLastError();
    }
  }
#define APDVM_GQ false
  APDVM_DISPATCH(k_stage_terms, insts, work, nwork, a, nv);
#undef APDVM_GQ
  return hipGetLastError();
}
#undef APDVM_DISPATCH
#undef APDVM_ONE

// tiles: the 64 x 16 tile table (nwork entries, 256 threads each).
hipError_t launch_div_u(int co, const Inst *insts, const Work *tiles, int nwork, int su1, int su2,
                        int out, hipStream_t st) {
  if (co == 4)
    hipLaunchKernelGGL(k_div_u<4>, dim3(nwork), dim3(256), 0, st, insts, tiles, nwork, su1, su2, out);
  else
    hipLaunchKernelGGL(k_div_u<2>, dim3(nwork), dim3(256), 0, st, insts, tiles, nwork, su1, su2, out);
  return hipGetLastError();
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

}  // namespace apdvm
