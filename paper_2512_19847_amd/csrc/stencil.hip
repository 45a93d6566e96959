// Stencil kernels of one IMEX stage (Algorithm 1, steps 1, 3 and 4, the right-hand
// side of step 2, and the stage terms reused by later stages), with the high-order
// space discretisation of Section 3.2: WENO5 (Jiang-Shu) reconstruction of the
// Lax-Friedrichs split fluxes and fourth-order central differences.
//
// Tiling: a workgroup of 256 threads owns a 64 x TY tile of one instance (TY = 8 or 16,
// chosen per kernel class by the host autotuner).  Every input plane is staged once in
// LDS with a 3-cell periodic halo (WENO5 reads 3 cells on each side of a cell; the
// central operators 2, corners included for the mixed derivative).  Planes that only
// feed WENO fluxes are staged multiplied by 1/2, which is exact in binary floating point,
// so the split fluxes (f +- w)/2 cost one add per cell and round exactly like
// (f +- w) * 0.5.  WENO numerical fluxes are computed once per face into LDS; the x and
// y faces of one divergence share one balanced index space.  Thread t owns column
// t % 64 and rows t / 64 + 4 k of the tile: every wavefront covers full 64-cell row
// segments, so all global loads and stores are row-contiguous.
//
// Precision: T is the transport type (double or float).  theta, the Helmholtz
// right-hand side and every history sum feeding an implicit relaxation or the
// right-hand side are float64 whatever T is.
#include "common.hpp"

namespace apdvm {

// ------------------------------------------------------------------ helpers

// Work item of this workgroup.  The hardware hands consecutive workgroups to the 8
// XCDs in turn; this remap gives each XCD a contiguous run of work items so tiles
// sharing halo rows meet in the same L2.
__device__ __forceinline__ int xcd_item(int nwork) {
  const int b = blockIdx.x;
  const int x = b & 7, i = b >> 3;
  const int q = nwork >> 3, r = nwork & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int wrap(int g, int n) {
  if ((unsigned)g >= (unsigned)n) g = ((g % n) + n) % n;
  return g;
}

// Jiang-Shu WENO5 value at the right face of cell c from cells a..e (left-biased):
// candidates q_k, smoothness indicators beta_k, weights d_k / (eps_w + beta_k)^2 with
// d = (1, 6, 3)/10 and eps_w = 1e-6.  The weights are normalised with one division:
// w_k proportional to d_k times the product of the other two (eps_w + beta)^2.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
  const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
  const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
  const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
  const double t0 = a - 2.0 * b + c, t1 = a - 4.0 * b + 3.0 * c;
  const double t2 = b - 2.0 * c + d, t3 = b - d;
  const double t4 = c - 2.0 * d + e, t5 = 3.0 * c - 4.0 * d + e;
  double s0 = 1e-6 + (13.0 / 12.0) * t0 * t0 + 0.25 * t1 * t1;
  double s1 = 1e-6 + (13.0 / 12.0) * t2 * t2 + 0.25 * t3 * t3;
  double s2 = 1e-6 + (13.0 / 12.0) * t4 * t4 + 0.25 * t5 * t5;
  s0 *= s0;
  s1 *= s1;
  s2 *= s2;
  const double w0 = 0.1 * s1 * s2, w1 = 0.6 * s0 * s2, w2 = 0.3 * s0 * s1;
  return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// float form: three hardware reciprocals (a product form could overflow float).
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e) {
  const float q0 = (2.0f * a - 7.0f * b + 11.0f * c) * (1.0f / 6.0f);
  const float q1 = (-b + 5.0f * c + 2.0f * d) * (1.0f / 6.0f);
  const float q2 = (2.0f * c + 5.0f * d - e) * (1.0f / 6.0f);
  const float t0 = a - 2.0f * b + c, t1 = a - 4.0f * b + 3.0f * c;
  const float t2 = b - 2.0f * c + d, t3 = b - d;
  const float t4 = c - 2.0f * d + e, t5 = 3.0f * c - 4.0f * d + e;
  float s0 = 1e-6f + (13.0f / 12.0f) * t0 * t0 + 0.25f * t1 * t1;
  float s1 = 1e-6f + (13.0f / 12.0f) * t2 * t2 + 0.25f * t3 * t3;
  float s2 = 1e-6f + (13.0f / 12.0f) * t4 * t4 + 0.25f * t5 * t5;
  const float w0 = 0.1f * __builtin_amdgcn_rcpf(s0 * s0);
  const float w1 = 0.6f * __builtin_amdgcn_rcpf(s1 * s1);
  const float w2 = 0.3f * __builtin_amdgcn_rcpf(s2 * s2);
  return (w0 * q0 + w1 * q1 + w2 * q2) * __builtin_amdgcn_rcpf(w0 + w1 + w2);
}

// Numerical flux at the face between cells k = 2 and k = 3 of six consecutive cells
// (stride apart in LDS).  f and w are staged halved, so f+ = sf f + w and
// f- = sf f - w are the Lax-Friedrichs split fluxes (sf f +- alpha w)/2 with alpha = 1
// (DISS) or alpha = 0: left-biased WENO5 of f+ plus right-biased WENO5 of f-.
template <typename T, bool DISS>
__device__ __forceinline__ T face_flux(const T *f, const T *w, int stride, T sf) {
  T p[6], m[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T fk = sf * f[k * stride];
    if (DISS) {
      const T wk = w[k * stride];
      p[k] = fk + wk;
      m[k] = fk - wk;
    } else {
      p[k] = fk;
      m[k] = fk;
    }
  }
  return weno5(p[0], p[1], p[2], p[3], p[4]) + weno5(m[5], m[4], m[3], m[2], m[1]);
}

// LDS tile geometry for a 64 x TY tile with a 3-cell halo.
template <int TY>
struct Geo {
  static constexpr int W = kTileX + 2 * kHalo;
  static constexpr int HT = TY + 2 * kHalo;
  static constexpr int PL = W * HT;                   // elements per staged plane
  static constexpr int FXN = TY * (kTileX + 1);       // x faces
  static constexpr int FXP = (FXN + 63) / 64 * 64;    // x faces padded to whole waves
  static constexpr int FYN = (TY + 1) * kTileX;       // y faces
  static constexpr int ROWS = TY / 4;                 // rows per thread
  __device__ static int at(int lx, int ly) { return (ly + kHalo) * W + lx + kHalo; }
};

// Stage a plane (with periodic halo) into LDS, converting to S and scaling by sc.
template <int TY, typename S, typename G>
__device__ __forceinline__ void stage_plane(S *lds, const G *__restrict__ plane, int nx, int ny,
                                            int x0, int y0, S sc) {
  using Gm = Geo<TY>;
  const bool inner = x0 >= kHalo && x0 + kTileX + kHalo <= nx && y0 >= kHalo &&
                     y0 + TY + kHalo <= ny;
  for (int idx = threadIdx.x; idx < Gm::PL; idx += kStencilThreads) {
    const int ly = idx / Gm::W;
    const int lx = idx - ly * Gm::W;
    int gx = x0 + lx - kHalo, gy = y0 + ly - kHalo;
    if (!inner) {
      gx = wrap(gx, nx);
      gy = wrap(gy, ny);
    }
    lds[idx] = sc * (S)plane[(long long)gy * nx + gx];
  }
}

// x faces (TY rows x 65) and y faces (TY + 1 rows x 64) of two fluxes in one index
// space; the x part is padded to whole wavefronts so no wavefront mixes the two.
template <int TY, typename T, bool DX, bool DY>
__device__ __forceinline__ void faces(T *fx, T *fy, const T *fxf, const T *fxw, T sx,
                                      const T *fyf, const T *fyw, T sy) {
  using Gm = Geo<TY>;
  for (int idx = threadIdx.x; idx < Gm::FXP + Gm::FYN; idx += kStencilThreads) {
    if (idx < Gm::FXP) {
      if (idx < Gm::FXN) {
        const int ly = idx / (kTileX + 1);
        const int f = idx - ly * (kTileX + 1);
        const int base = (ly + kHalo) * Gm::W + f;  // cell f - 3 of row ly
        fx[idx] = face_flux<T, DX>(fxf + base, fxw + base, 1, sx);
      }
    } else {
      const int j = idx - Gm::FXP;
      const int f = j / kTileX;
      const int lx = j - f * kTileX;
      const int base = f * Gm::W + lx + kHalo;  // cell f - 3 of column lx
      fy[j] = face_flux<T, DY>(fyf + base, fyw + base, Gm::W, sy);
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

// Fourth-order central first and second derivatives from an LDS plane at index c
// (stride 1 for x, W for y): D f = (f-2 - 8 f-1 + 8 f+1 - f+2) / (12 h),
// L f = (-f-2 + 16 f-1 - 30 f0 + 16 f+1 - f+2) / (12 h^2).
template <typename S>
__device__ __forceinline__ S cd1(const S *p, int c, int st, S ih12) {
  return (p[c - 2 * st] - S(8) * p[c - st] + S(8) * p[c + st] - p[c + 2 * st]) * ih12;
}
template <typename S>
__device__ __forceinline__ S cd2(const S *p, int c, int st, S ih2_12) {
  return (-p[c - 2 * st] + S(16) * p[c - st] - S(30) * p[c] + S(16) * p[c + st] - p[c + 2 * st]) *
         ih2_12;
}
// D_x D_y f
template <typename S>
__device__ __forceinline__ S cdxy(const S *p, int c, int W, S ihx12, S ihy12) {
  const int o[4] = {-2, -1, 1, 2};
  const S w[4] = {S(1), S(-8), S(8), S(-1)};
  S acc = S(0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    S dy = S(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) dy += w[b] * p[c + o[a] + o[b] * W];
    acc += w[a] * (dy * ihy12);
  }
  return acc * ihx12;
}

template <typename T>
__device__ __forceinline__ T *tplane(const Inst &I, int slot) {
  return reinterpret_cast<T *>(I.tbase) + (long long)slot * I.plane;
}
__device__ __forceinline__ double *dplane(const Inst &I, int slot) {
  return I.dbase + (long long)slot * I.plane;
}

// Step 1 at cell g: v(i) = [te2 v^n - dt (sum_j at_ij E(j) + sum_j a_ij v(j))] kinv,
// the history sum in float64.  eh and vh are the terms of the newest stage when they are
// held in registers (nE / nV then cover the older ones only).
template <typename T>
__device__ __forceinline__ void relax_v_at(const Inst &I, const ArgsV &a, long long g, double vn1,
                                           double vn2, double h1, double h2) {
  for (int j = 0; j < a.nE; ++j) {
    h1 += a.cE[j] * (double)tplane<T>(I, a.E[j][0])[g];
    h2 += a.cE[j] * (double)tplane<T>(I, a.E[j][1])[g];
  }
  for (int j = 0; j < a.nV; ++j) {
    h1 += a.cV[j] * (double)tplane<T>(I, a.V[j][0])[g];
    h2 += a.cV[j] * (double)tplane<T>(I, a.V[j][1])[g];
  }
  const double kinv = I.kinv[a.stage], te2 = I.te2, dt = I.dt;
  tplane<T>(I, a.out[0])[g] = (T)((te2 * vn1 - dt * h1) * kinv);
  tplane<T>(I, a.out[1])[g] = (T)((te2 * vn2 - dt * h2) * kinv);
}

// ------------------------------------------------------------------ step 2 RHS

template <typename T, int TY>
__global__ __launch_bounds__(kStencilThreads) void k_helmholtz_rhs(const Inst *__restrict__ insts,
                                                                   const Work *__restrict__ work,
                                                                   int nwork, ArgsR a) {
  using Gm = Geo<TY>;
  __shared__ T sV1[Gm::PL], sV2[Gm::PL];
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  stage_plane<TY>(sV1, tplane<T>(I, a.v[0]), I.nx, I.ny, wk.a, wk.b, T(1));
  stage_plane<TY>(sV2, tplane<T>(I, a.v[1]), I.nx, I.ny, wk.a, wk.b, T(1));
  __syncthreads();
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  if (gx >= I.nx) return;
  const T ihx12 = T(I.ihx / 12.0), ihy12 = T(I.ihy / 12.0);
  const T ihx2 = T(I.ihx * I.ihx / 12.0), ihy2 = T(I.ihy * I.ihy / 12.0);
  const double sig = I.sigma[a.stage];
  const double c_d = 1.0 / (I.dt * a.aii * a.aii), c_0 = 1.0 / (I.dt * a.aii), c_l = 1.0 / a.aii;
  const double *thn = dplane(I, a.thn);
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + 4 * r;
    const int gy = wk.b + ly;
    if (gy >= I.ny) break;
    const int c = Gm::at(tx, ly);
    // D0^2 : B(v) = -D_xx v1 + 2 D_x D_y v2 + D_yy v1
    const T ddb = -cd2(sV1, c, 1, ihx2) + T(2) * cdxy(sV2, c, Gm::W, ihx12, ihy12) +
                  cd2(sV1, c, Gm::W, ihy2);
    const long long g = (long long)gy * I.nx + gx;
    double hd = 0.0, hl = 0.0;
    for (int j = 0; j < a.nD; ++j) hd += a.cD[j] * (double)tplane<T>(I, a.D[j])[g];
    for (int j = 0; j < a.nL; ++j) hl += a.cL[j] * (double)tplane<T>(I, a.L[j])[g];
    const double du0 = (double)tplane<T>(I, a.du0)[g];
    const double R = -sig * thn[g] + c_d * hd + c_0 * du0 - (double)ddb - c_l * hl;
    dplane(I, a.out_r)[g] = R;
    tplane<T>(I, a.out_ddb)[g] = ddb;
  }
}

// ------------------------------------------------------------------ steps 3 and 4

template <typename T, int TY>
__global__ __launch_bounds__(kStencilThreads) void k_update_uq(const Inst *__restrict__ insts,
                                                               const Work *__restrict__ work,
                                                               int nwork, ArgsUQ a) {
  using Gm = Geo<TY>;
  // v1, v2 and the partner velocity (halved for the fluxes); theta reuses the partner
  // planes once the fluxes that need them are done.
  __shared__ T sV1[Gm::PL], sV2[Gm::PL];
  __shared__ T sP[2 * Gm::PL];
  __shared__ T fx[Gm::FXN], fy[Gm::FYN];
  static_assert(sizeof(T) * 2 * Gm::PL >= sizeof(double) * Gm::PL, "theta reuse");
  T *sP1 = sP, *sP2 = sP + Gm::PL;
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  stage_plane<TY>(sV1, tplane<T>(I, a.v[0]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sV2, tplane<T>(I, a.v[1]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sP1, tplane<T>(I, a.partner[0]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sP2, tplane<T>(I, a.partner[1]), nx, ny, wk.a, wk.b, T(0.5));
  __syncthreads();
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const T ihx = T(I.ihx), ihy = T(I.ihy);
  T hu1[Gm::ROWS], hu2[Gm::ROWS], dv[Gm::ROWS];
  // first row of B(v) = (-v1, v2), dissipation on u1
  faces<TY, T, true, true>(fx, fy, sV1, sP1, T(-1), sV2, sP1, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r)
    hu1[r] = face_dx<TY>(fx, tx, ty0 + 4 * r, ihx) + face_dy<TY>(fy, tx, ty0 + 4 * r, ihy);
  __syncthreads();
  // second row of B(v) = (v2, v1), dissipation on u2
  faces<TY, T, true, true>(fx, fy, sV2, sP2, T(1), sV1, sP2, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r)
    hu2[r] = face_dx<TY>(fx, tx, ty0 + 4 * r, ihx) + face_dy<TY>(fy, tx, ty0 + 4 * r, ihy);
  __syncthreads();
  // div v without dissipation; theta (float64) into the partner planes meanwhile
  faces<TY, T, false, false>(fx, fy, sV1, sV1, T(1), sV2, sV2, T(1));
  double *sTh = reinterpret_cast<double *>(sP);
  stage_plane<TY>(sTh, dplane(I, a.th), nx, ny, wk.a, wk.b, 1.0);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r)
    dv[r] = face_dx<TY>(fx, tx, ty0 + 4 * r, ihx) + face_dy<TY>(fy, tx, ty0 + 4 * r, ihy);

  const int gx = wk.a + tx;
  if (gx >= nx) return;
  const double ihx12 = I.ihx / 12.0, ihy12 = I.ihy / 12.0;
  const double dt = I.dt, te2 = I.te2, kinv = I.kinv[a.stage], aii = a.aii;
  const double htau = 0.5 * I.tau;
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + 4 * r;
    const int gy = wk.b + ly;
    if (gy >= ny) break;
    const int c = Gm::at(tx, ly);
    const long long g = (long long)gy * nx + gx;
    // implicit velocity terms: D_W.B(v) + D0 theta (theta float64)
    const double Hu1 = (double)hu1[r] + cd1(sTh, c, 1, ihx12);
    const double Hu2 = (double)hu2[r] + cd1(sTh, c, Gm::W, ihy12);
    double s1 = aii * Hu1, s2 = aii * Hu2, sq = 0.0;
    for (int j = 0; j < a.nH; ++j) {
      s1 += a.cH[j] * (double)tplane<T>(I, a.H[j][0])[g];
      s2 += a.cH[j] * (double)tplane<T>(I, a.H[j][1])[g];
    }
    for (int j = 0; j < a.nG; ++j) sq += a.cG[j] * (double)tplane<T>(I, a.G[j])[g];
    const double u1 = (double)tplane<T>(I, a.un[0])[g] - dt * s1;
    const double u2 = (double)tplane<T>(I, a.un[1])[g] - dt * s2;
    const double Hq = htau * (double)dv[r];
    const double q = (te2 * (double)tplane<T>(I, a.qn)[g] - dt * aii * Hq - dt * sq) * kinv;
    tplane<T>(I, a.out_u[0])[g] = (T)u1;
    tplane<T>(I, a.out_u[1])[g] = (T)u2;
    tplane<T>(I, a.out_q)[g] = (T)q;
    if (a.out_hu[0] != kNoSlot) {
      tplane<T>(I, a.out_hu[0])[g] = (T)Hu1;
      tplane<T>(I, a.out_hu[1])[g] = (T)Hu2;
      tplane<T>(I, a.out_gq)[g] = (T)(Hq + q);
    }
  }
}

// ------------------------------------------------------------------ stage terms

// E = (tau/4) D0_W.B(u) + te2 D_W q[v] - F(u), D0.u and Ltheta of a known stage, and,
// fused, step 1 of the next stage: v(next) from v^n, the history and this E.
template <typename T, int TY>
__global__ __launch_bounds__(kStencilThreads) void k_stage_terms(const Inst *__restrict__ insts,
                                                                 const Work *__restrict__ work,
                                                                 int nwork, ArgsE a, ArgsV nv) {
  using Gm = Geo<TY>;
  // sU1 and sU2 are contiguous so that theta (float64) can reuse them at the end.
  __shared__ T sU[2 * Gm::PL];
  __shared__ T sQ[Gm::PL], sV1[Gm::PL], sV2[Gm::PL];
  __shared__ T fx[Gm::FXN], fy[Gm::FYN];
  static_assert(sizeof(T) * 2 * Gm::PL >= sizeof(double) * Gm::PL, "theta reuse");
  T *sU1 = sU, *sU2 = sU + Gm::PL;
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int nx = I.nx, ny = I.ny;
  stage_plane<TY>(sU1, tplane<T>(I, a.u[0]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sU2, tplane<T>(I, a.u[1]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sQ, tplane<T>(I, a.q), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sV1, tplane<T>(I, a.v[0]), nx, ny, wk.a, wk.b, T(0.5));
  stage_plane<TY>(sV2, tplane<T>(I, a.v[1]), nx, ny, wk.a, wk.b, T(0.5));
  __syncthreads();
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const T ihx = T(I.ihx), ihy = T(I.ihy);
  // the staged u is halved: its central derivative carries a factor 2
  const T ihx6 = T(I.ihx / 6.0), ihy6 = T(I.ihy / 6.0);
  T b1[Gm::ROWS], b2[Gm::ROWS], g1[Gm::ROWS], g2[Gm::ROWS], du[Gm::ROWS], F1[Gm::ROWS],
      F2[Gm::ROWS];
  // first row of B(u) = (-u1, u2), no dissipation
  faces<TY, T, false, false>(fx, fy, sU1, sU1, T(-1), sU2, sU2, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r)
    b1[r] = face_dx<TY>(fx, tx, ty0 + 4 * r, ihx) + face_dy<TY>(fy, tx, ty0 + 4 * r, ihy);
  __syncthreads();
  // second row of B(u) = (u2, u1)
  faces<TY, T, false, false>(fx, fy, sU2, sU2, T(1), sU1, sU1, T(1));
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + 4 * r;
    b2[r] = face_dx<TY>(fx, tx, ly, ihx) + face_dy<TY>(fy, tx, ly, ihy);
    const int c = Gm::at(tx, ly);
    du[r] = cd1(sU1, c, 1, ihx6) + cd1(sU2, c, Gm::W, ihy6);
    const T u1 = T(2) * sU1[c], u2 = T(2) * sU2[c];
    F1[r] = T(0.5) * (u2 * u2 - u1 * u1);
    F2[r] = u1 * u2;
  }
  __syncthreads();
  // grad q with dissipation on v1 (x) and v2 (y)
  faces<TY, T, true, true>(fx, fy, sQ, sV1, T(1), sQ, sV2, T(1));
  const bool want_lt = a.out_lt != kNoSlot;
  double *sTh = reinterpret_cast<double *>(sU);
  if (want_lt) stage_plane<TY>(sTh, dplane(I, a.th), nx, ny, wk.a, wk.b, 1.0);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    g1[r] = face_dx<TY>(fx, tx, ty0 + 4 * r, ihx);
    g2[r] = face_dy<TY>(fy, tx, ty0 + 4 * r, ihy);
  }
  const int gx = wk.a + tx;
  if (gx >= nx) return;
  const T qt = T(0.25 * I.tau), te2 = T(I.te2);
  const double ihx2 = I.ihx * I.ihx / 12.0, ihy2 = I.ihy * I.ihy / 12.0;
#pragma unroll
  for (int r = 0; r < Gm::ROWS; ++r) {
    const int ly = ty0 + 4 * r;
    const int gy = wk.b + ly;
    if (gy >= ny) break;
    const long long g = (long long)gy * nx + gx;
    const T e1 = qt * b1[r] + te2 * g1[r] - F1[r];
    const T e2 = qt * b2[r] + te2 * g2[r] - F2[r];
    if (a.out_e[0] != kNoSlot) {
      tplane<T>(I, a.out_e[0])[g] = e1;
      tplane<T>(I, a.out_e[1])[g] = e2;
    }
    tplane<T>(I, a.out_du)[g] = du[r];
    if (want_lt) {
      const int c = Gm::at(tx, ly);
      const double lap = cd2(sTh, c, 1, ihx2) + cd2(sTh, c, Gm::W, ihy2);
      tplane<T>(I, a.out_lt)[g] = (T)((double)tplane<T>(I, a.ddb)[g] + lap);
    }
    if (nv.stage > 0) {
      // step 1 of the next stage; its newest history terms are this E and this v
      const int c = Gm::at(tx, ly);
      const double ce = a.c_e_next, cv = a.c_v_next;
      const double v1 = 2.0 * (double)sV1[c], v2 = 2.0 * (double)sV2[c];
      relax_v_at<T>(I, nv, g, (double)tplane<T>(I, nv.vn[0])[g],
                    (double)tplane<T>(I, nv.vn[1])[g], ce * (double)e1 + cv * v1,
                    ce * (double)e2 + cv * v2);
    }
  }
}

// Step 1 on its own (the stage right after new fields, when no stage-terms launch of
// the previous stage could fuse it).
template <typename T, int TY>
__global__ __launch_bounds__(kStencilThreads) void k_relax_v(const Inst *__restrict__ insts,
                                                             const Work *__restrict__ work,
                                                             int nwork, ArgsV a) {
  const Work wk = work[xcd_item(nwork)];
  const Inst &I = insts[wk.inst];
  const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
  const int gx = wk.a + tx;
  if (gx >= I.nx) return;
  for (int r = 0; r < TY / 4; ++r) {
    const int gy = wk.b + ty0 + 4 * r;
    if (gy >= I.ny) break;
    const long long g = (long long)gy * I.nx + gx;
    relax_v_at<T>(I, a, g, (double)tplane<T>(I, a.vn[0])[g], (double)tplane<T>(I, a.vn[1])[g],
                  0.0, 0.0);
  }
}

// ------------------------------------------------------------------ launchers

template <typename T>
hipError_t launch_relax_v(int ty, const Inst *insts, const Work *work, int nwork, const ArgsV &a,
                          hipStream_t st) {
  if (ty == 8)
    hipLaunchKernelGGL((k_relax_v<T, 8>), dim3(nwork), dim3(kStencilThreads), 0, st, insts, work,
                       nwork, a);
  else
    hipLaunchKernelGGL((k_relax_v<T, 16>), dim3(nwork), dim3(kStencilThreads), 0, st, insts, work,
                       nwork, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_helmholtz_rhs(int ty, const Inst *insts, const Work *work, int nwork,
                                const ArgsR &a, hipStream_t st) {
  if (ty == 8)
    hipLaunchKernelGGL((k_helmholtz_rhs<T, 8>), dim3(nwork), dim3(kStencilThreads), 0, st, insts,
                       work, nwork, a);
  else
    hipLaunchKernelGGL((k_helmholtz_rhs<T, 16>), dim3(nwork), dim3(kStencilThreads), 0, st, insts,
                       work, nwork, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_update_uq(int ty, const Inst *insts, const Work *work, int nwork,
                            const ArgsUQ &a, hipStream_t st) {
  if (ty == 8)
    hipLaunchKernelGGL((k_update_uq<T, 8>), dim3(nwork), dim3(kStencilThreads), 0, st, insts, work,
                       nwork, a);
  else
    hipLaunchKernelGGL((k_update_uq<T, 16>), dim3(nwork), dim3(kStencilThreads), 0, st, insts,
                       work, nwork, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_stage_terms(int ty, const Inst *insts, const Work *work, int nwork,
                              const ArgsE &a, const ArgsV &nv, hipStream_t st) {
  if (ty == 8)
    hipLaunchKernelGGL((k_stage_terms<T, 8>), dim3(nwork), dim3(kStencilThreads), 0, st, insts,
                       work, nwork, a, nv);
  else
    hipLaunchKernelGGL((k_stage_terms<T, 16>), dim3(nwork), dim3(kStencilThreads), 0, st, insts,
                       work, nwork, a, nv);
  return hipGetLastError();
}

#define APDVM_INST(T)                                                                           \
  template hipError_t launch_relax_v<T>(int, const Inst *, const Work *, int, const ArgsV &,   \
                                        hipStream_t);                                          \
  template hipError_t launch_helmholtz_rhs<T>(int, const Inst *, const Work *, int,            \
                                              const ArgsR &, hipStream_t);                     \
  template hipError_t launch_update_uq<T>(int, const Inst *, const Work *, int, const ArgsUQ &, \
                                          hipStream_t);                                        \
  template hipError_t launch_stage_terms<T>(int, const Inst *, const Work *, int, const ArgsE &, \
                                            const ArgsV &, hipStream_t);
APDVM_INST(double)
APDVM_INST(float)
#undef APDVM_INST

}  // namespace apdvm
