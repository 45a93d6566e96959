// Periodic Helmholtz solve of Algorithm 1, step 2: (D_Delta - sigma) theta = R.
//
// D_Delta is the sum of two circulant operators, so the 2D DFT diagonalises it:
// theta_hat(kx, ky) = R_hat(kx, ky) / (lambda_x(kx) + lambda_y(ky) - sigma), with
// lambda the Fourier symbol of the fourth-order central second difference.  The (0,0)
// mode is set to the mean of theta^n instead of dividing by -sigma (every derivative
// term of R has zero mean, so this is the exact-arithmetic value; it also covers
// sigma = 0).  All of it runs in float64.
//
// Five kernels, each one read and one write of a float64 plane-sized array:
//  rows forward   two real rows packed as one complex length-nx FFT, split into the two
//                 half spectra kx = 0..nx/2.  Output: spectrum [ny][nx/2 + 1] complex.
//  columns A      four-step FFT along y with ny = n1 n2, y = r + n2 m: a length-n1 FFT
//                 over m for every residue r and column (strided rows, C columns of a
//                 tile side by side so each row segment is one contiguous load).
//  columns B      for each k1, the n2 contiguous rows n2 k1 + r: twiddle exp(-2 pi i r
//                 k1 / ny), length-n2 FFT over r (frequency ky = k1 + n1 k2), multiply by
//                 1 / ((lambda_x + lambda_y - sigma) nx ny) with the (0,0) rule, inverse
//                 length-n2 FFT and the conjugate twiddle.
//  columns A inv  inverse length-n1 FFTs, back to natural row order.
//  rows inverse   Hermitian extension of the half spectra, inverse FFT, two real rows.
//
// Every FFT is a mixed-radix (8, 4, 3, 2) Stockham autosort transform in LDS: each pass
// reads R strided inputs per butterfly, applies twiddles from a float64 table of
// exp(-2 pi i m / n), does a radix-R DFT in registers and writes R outputs; the pass is
// in place (every thread holds its butterflies in registers across a barrier).
#include "common.hpp"

namespace apdvm {

__device__ __forceinline__ int xcd_item_fft(int nwork) {
  const int b = blockIdx.x;
  const int x = b & 7, i = b >> 3;
  const int q = nwork >> 3, r = nwork & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ double2 rot(double2 a) {
  return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

template <int DIR>
__device__ __forceinline__ void dft4(double2 &a0, double2 &a1, double2 &a2, double2 &a3) {
  const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const double2 t2 = cadd(a1, a3), t3 = rot<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// In-register DFT of length R with kernel exp(DIR 2 pi i / R).
template <int R, int DIR>
__device__ __forceinline__ void dft(double2 *v) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const double h = 0.86602540378443864676;  // sqrt(3)/2
    const double2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
    const double2 jd = rot<DIR>(make_double2(h * d.x, h * d.y));
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, jd);
    v[2] = csub(m, jd);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    const double c = 0.70710678118654752440;
    // o_k *= exp(DIR i pi k / 4)
    o1 = make_double2(c * (o1.x - DIR * o1.y), c * (o1.y + DIR * o1.x));
    o2 = rot<DIR>(o2);
    o3 = make_double2(c * (-o3.x - DIR * o3.y), c * (-o3.y + DIR * o3.x));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  }
}

// Exact x / d by a multiply-high, for 0 <= x with x d < 2^32 (LDS indexes): m =
// ceil(2^32 / d), and the error x (m d - 2^32) / (d 2^32) stays below 1 / d.
struct Div {
  unsigned long long m;
  unsigned d;
  __device__ __forceinline__ explicit Div(unsigned dd) : m(0xFFFFFFFFull / dd + 1), d(dd) {}
  __device__ __forceinline__ int q(int x) const {
    return (int)(((unsigned long long)(unsigned)x * m) >> 32);
  }
};

// Complex values in global memory, accessed as a native two-lane vector (one 16-byte
// load or store).
using dv2 = double __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldc(Gp<const dv2> p) {
  const dv2 t = *p;
  return make_double2(t.x, t.y);
}
__device__ __forceinline__ void stc(Gp<dv2> p, double2 v) {
  dv2 t;
  t.x = v.x;
  t.y = v.y;
  *p = t;
}

// LDS layout of the FFT buffers: one padding element after every 8, so the strided
// writes of the early Stockham passes (stride R Ns elements of 16 bytes) spread over the
// banks instead of hitting the same few.
__device__ __forceinline__ int lp(int i) { return i + (i >> 3); }

// exp(-2 pi i m / n) from the two-level table staged in LDS (lo at t, hi at t + 2^lb).
__device__ __forceinline__ double2 tw_at(const double2 *t, int lb, int m) {
  return cmul(t[(1 << lb) + (m >> lb)], t[m & ((1 << lb) - 1)]);
}

// The two-level twiddle table of a plan passes through registers into LDS, so its global
// loads travel with the data loads of the kernel.
template <int NT>
struct TwStage {
  static constexpr int K = (kTwCap + NT - 1) / NT;
  double2 v[K];
  __device__ __forceinline__ void load(const FftPlan &P) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < P.ntw) v[k] = ldc(reinterpret_cast<Gp<const dv2>>(gp(P.tw2)) + i);
    }
  }
  __device__ __forceinline__ void store(double2 *t, const FftPlan &P) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < P.ntw) t[i] = make_double2(v[k].x, v[k].y);
    }
  }
};

// One Stockham pass over nb transforms of length n held in LDS, element j of
// transform b at buf[j * es + b * bs].  BMAJOR: consecutive threads take consecutive
// transforms (column tiles) instead of consecutive butterflies (rows).  The first pass
// (Ns = 1) has unit twiddles and skips them.
template <int R, int DIR, bool BMAJOR, int CAP, int NT>
__device__ __forceinline__ void pass(double2 *buf, int n, int nb, int es, int bs, int Ns,
                                     const double2 *tws, int lb) {
  constexpr int NPER = (CAP + R * NT - 1) / (R * NT);
  const int nbf = n / R;
  const int total = nbf * nb;
  const int twstep = n / (Ns * R);
  const Div dmaj(BMAJOR ? nb : nbf), dns(Ns);
  double2 v[NPER][R];
  int dst[NPER];
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int t = threadIdx.x + p * NT;
    dst[p] = -1;
    if (t < total) {
      int j, b;
      if (BMAJOR) {
        j = dmaj.q(t);
        b = t - j * nb;
      } else {
        b = dmaj.q(t);
        j = t - b * nbf;
      }
      const int jq = dns.q(j), k = j - jq * Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = buf[lp((j + r * nbf) * es + b * bs)];
      if (Ns > 1) {
        // w^r for r = 1..R-1 from one table lookup: powers by products of depth <= 3
        double2 w[R];
        w[1] = tw_at(tws, lb, k * twstep);
        if (DIR > 0) w[1].y = -w[1].y;
        if constexpr (R >= 3) w[2] = cmul(w[1], w[1]);
        if constexpr (R >= 4) w[3] = cmul(w[2], w[1]);
        if constexpr (R == 8) {
          w[4] = cmul(w[2], w[2]);
          w[5] = cmul(w[4], w[1]);
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = cmul(v[p][r], w[r]);
      }
      dft<R, DIR>(v[p]);
      dst[p] = (jq * Ns * R + k) * es + b * bs;
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    if (dst[p] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(dst[p] + r * Ns * es)] = v[p][r];
    }
  }
  __syncthreads();
}

template <int DIR, bool BMAJOR, int CAP, int NT>
__device__ __forceinline__ void fft_lds(double2 *buf, const FftPlan &P, int nb, int es, int bs,
                                        const double2 *tws) {
  int Ns = 1;
  for (int ps = 0; ps < P.npass; ++ps) {
    const int R = P.radix[ps];
    switch (R) {
      case 8: pass<8, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, tws, P.lb); break;
      case 4: pass<4, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, tws, P.lb); break;
      case 3: pass<3, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, tws, P.lb); break;
      default: pass<2, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, tws, P.lb); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ Gp<double> dslot(const Inst &I, int slot) {
  return gp(I.dbase + (long long)slot * I.plane);
}
__device__ __forceinline__ Gp<dv2> cslot(const Inst &I, int slot) {
  return reinterpret_cast<Gp<dv2>>(dslot(I, slot));
}



// Each kernel below stages its tile in two phases: every thread first issues all of its
// global loads (data, twiddle table, and the Helmholtz divisors of the elements it will
// scale), then writes them to LDS, so one memory round trip covers the whole tile.

// ------------------------------------------------------------------ rows forward

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_rows_forward(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP + CAP / 8];
  __shared__ double2 tws[kTwCap];
  constexpr int E = CAP / NT;
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, K = h + 1;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const int cnt = np * n;
  const Gp<const double> R = dslot(I, a.r) + 2LL * p0 * n;
  const Div dn(n);
  TwStage<NT> tw;
  tw.load(I.fx);
  double ra[E], rb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int o = idx + dn.q(idx) * n;  // row 2p, column x
      ra[e] = R[o];
      rb[e] = R[o + n];
    }
  }
  tw.store(tws, I.fx);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) buf[lp(idx)] = make_double2(ra[e], rb[e]);
  }
  __syncthreads();
  fft_lds<-1, false, CAP, NT>(buf, I.fx, np, 1, n, tws);
  const Gp<dv2> S = cslot(I, a.spec) + 2LL * p0 * K;
  const Div dk(K);
  for (int idx = threadIdx.x; idx < np * K; idx += NT) {
    const int p = dk.q(idx), k = idx - p * K;
    const double2 Z = buf[lp(p * n + (k == h ? h : k))];
    // Z[n-k]; its conjugate pairs with Z[k]
    const double2 W = buf[lp(p * n + (k == 0 ? 0 : n - k))];
    // A = (Z + conj W) / 2, B = (Z - conj W) / 2i: the spectra of the two real rows
    const double2 A = make_double2(0.5 * (Z.x + W.x), 0.5 * (Z.y - W.y));
    const double2 B = make_double2(0.5 * (Z.y + W.y), -0.5 * (Z.x - W.x));
    stc(S + 2 * p * K + k, A);
    stc(S + (2 * p + 1) * K + k, B);
  }
}

// ------------------------------------------------------------------ columns

// Tile of C columns of the spectrum: element j of column c at buf[j * es + c].
constexpr int kColCap = 2048;
constexpr int kColThreads = 256;
constexpr int kColPer = kColCap / kColThreads;

// A: length-n1 FFT over rows y = r + n2 m, m = 0..n1-1, for the C columns k0.. of the
// tile; work item (inst, k0, r).
template <int DIR>
__global__ __launch_bounds__(kColThreads) void k_cols_a(const Inst *__restrict__ insts,
                                                        const Work *__restrict__ work,
                                                        int nwork, ArgsSolve a) {
  __shared__ double2 buf[kColCap + kColCap / 8];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1, n1 = I.f1.n, n2 = I.f2.n;
  const int k0 = wk.a, r = wk.b;
  const int C = min(I.cols_per_block, K - k0);
  const int cnt = n1 * C;
  const Gp<dv2> S = cslot(I, a.spec) + (long long)r * K + k0;
  const long long stride = (long long)n2 * K;
  const Div dc(C);
  TwStage<kColThreads> tw;
  tw.load(I.f1);
  double2 v[kColPer];
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    if (idx < cnt) {
      const int m = dc.q(idx), c = idx - m * C;
      v[e] = ldc(S + m * stride + c);
    }
  }
  tw.store(tws, I.f1);
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    if (idx < cnt) buf[lp(idx)] = make_double2(v[e].x, v[e].y);
  }
  __syncthreads();
  fft_lds<DIR, true, kColCap, kColThreads>(buf, I.f1, C, C, 1, tws);
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    if (idx < cnt) {
      const int m = dc.q(idx), c = idx - m * C;
      stc(S + m * stride + c, buf[lp(idx)]);
    }
  }
}

// Divisor of mode (kx, ky): 1 / ((lambda_x + lambda_y - sigma) nx ny); the (0,0) mode is
// replaced by theta_mean instead (flagged by a zero divisor slot).
__device__ __forceinline__ double mode_scale(const Inst &I, double sig, int kx, int ky) {
  return (kx == 0 && ky == 0) ? 0.0 : I.inv_nxny / (gp(I.lam_x)[kx] + gp(I.lam_y)[ky] - sig);
}

// B: for G groups k1 = g0.. of n2 contiguous rows n2 k1 + r: twiddle, length-n2 FFT,
// symbol divide, inverse length-n2 FFT, conjugate twiddle.  LDS layout [r][g][c].
__global__ __launch_bounds__(kColThreads) void k_cols_b(const Inst *__restrict__ insts,
                                                        const Work *__restrict__ work, int nwork,
                                                        ArgsSolve a) {
  __shared__ double2 buf[kColCap + kColCap / 8];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1, n = I.ny, n1 = I.f1.n, n2 = I.f2.n;
  const int k0 = wk.a, g0 = wk.b;
  const int C = min(I.cols_per_block, K - k0);
  const int G = min(I.groups_per_block, n1 - g0);
  const int GC = G * C;
  const int cnt = n2 * GC;
  const Gp<dv2> S = cslot(I, a.spec) + k0;
  const Gp<const dv2> twn = reinterpret_cast<Gp<const dv2>>(gp(I.fy.tw));  // exp(-2 pi i m / ny)
  const double sig = I.sigma[a.stage];
  const Div dgc(GC), dc(C), dn(n);
  TwStage<kColThreads> tw;
  tw.load(I.f2);
  double2 v[kColPer], w[kColPer];
  double d[kColPer];
  int off[kColPer];
  // element idx = (r, g, c): row n2 (g0 + g) + r of the spectrum before the n2-point FFT,
  // mode ky = g0 + g + n1 r after it
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    off[e] = -1;
    if (idx < cnt) {
      const int r = dgc.q(idx), rem = idx - r * GC;
      const int g = dc.q(rem), c = rem - g * C;
      const int k1 = g0 + g;
      off[e] = (n2 * k1 + r) * K + c;
      v[e] = ldc(S + off[e]);
      const int m = r * k1;
      w[e] = ldc(twn + (m - dn.q(m) * n));
      d[e] = mode_scale(I, sig, k0 + c, k1 + n1 * r);
    }
  }
  tw.store(tws, I.f2);
#pragma unroll
  for (int e = 0; e < kColPer; ++e)
    if (off[e] >= 0) buf[lp(threadIdx.x + e * kColThreads)] = cmul(v[e], w[e]);
  __syncthreads();
  fft_lds<-1, true, kColCap, kColThreads>(buf, I.f2, GC, GC, 1, tws);
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    if (off[e] >= 0) {
      const double2 z = buf[lp(idx)];
      buf[lp(idx)] = d[e] == 0.0 ? make_double2(I.theta_mean, 0.0)
                             : make_double2(z.x * d[e], z.y * d[e]);
    }
  }
  __syncthreads();
  fft_lds<1, true, kColCap, kColThreads>(buf, I.f2, GC, GC, 1, tws);
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    if (off[e] >= 0) {
      const double2 c = make_double2(w[e].x, -w[e].y);
      stc(S + off[e], cmul(buf[lp(threadIdx.x + e * kColThreads)], c));
    }
  }
}

// Single pass over whole columns (ny <= kColCap / C): forward FFT along y, symbol divide
// with the (0,0) rule, inverse FFT, for the C columns k0.. of the tile; work item
// (inst, k0).  One launch instead of the three of the four-step form, for grids whose
// columns fit a tile.
__global__ __launch_bounds__(kColThreads) void k_cols_full(const Inst *__restrict__ insts,
                                                           const Work *__restrict__ work,
                                                           int nwork, ArgsSolve a) {
  __shared__ double2 buf[kColCap + kColCap / 8];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1;
  const int k0 = wk.a;
  const int C = min(I.cols_full_per_block, K - k0);
  const int cnt = I.ny * C;
  const Gp<dv2> S = cslot(I, a.spec) + k0;
  const double sig = I.sigma[a.stage];
  const Div dc(C);
  TwStage<kColThreads> tw;
  tw.load(I.fy);
  double2 v[kColPer];
  double d[kColPer];
  int off[kColPer];
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    off[e] = -1;
    if (idx < cnt) {
      const int y = dc.q(idx), c = idx - y * C;
      off[e] = y * K + c;
      v[e] = ldc(S + off[e]);
      d[e] = mode_scale(I, sig, k0 + c, y);
    }
  }
  tw.store(tws, I.fy);
#pragma unroll
  for (int e = 0; e < kColPer; ++e)
    if (off[e] >= 0) buf[lp(threadIdx.x + e * kColThreads)] = make_double2(v[e].x, v[e].y);
  __syncthreads();
  fft_lds<-1, true, kColCap, kColThreads>(buf, I.fy, C, C, 1, tws);
#pragma unroll
  for (int e = 0; e < kColPer; ++e) {
    const int idx = threadIdx.x + e * kColThreads;
    if (off[e] >= 0) {
      const double2 z = buf[lp(idx)];
      buf[lp(idx)] = d[e] == 0.0 ? make_double2(I.theta_mean, 0.0)
                             : make_double2(z.x * d[e], z.y * d[e]);
    }
  }
  __syncthreads();
  fft_lds<1, true, kColCap, kColThreads>(buf, I.fy, C, C, 1, tws);
#pragma unroll
  for (int e = 0; e < kColPer; ++e)
    if (off[e] >= 0) stc(S + off[e], buf[lp(threadIdx.x + e * kColThreads)]);
}

// ------------------------------------------------------------------ rows inverse

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_rows_inverse(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP + CAP / 8];
  __shared__ double2 tws[kTwCap];
  constexpr int E = CAP / (2 * NT);
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, K = h + 1;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const int cnt = np * h;
  const Gp<const dv2> S = cslot(I, a.spec) + 2LL * p0 * K;
  const Div dh(h);
  TwStage<NT> tw;
  tw.load(I.fx);
  double2 A[E], B[E], AN, BN;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int p = dh.q(idx), k = idx - p * h;
      A[e] = ldc(S + 2 * p * K + k);
      B[e] = ldc(S + (2 * p + 1) * K + k);
    }
  }
  // kx = nx/2 of pair p = threadIdx.x (np <= NT)
  const int pn = threadIdx.x;
  if (pn < np) {
    AN = ldc(S + 2 * pn * K + h);
    BN = ldc(S + (2 * pn + 1) * K + h);
  }
  tw.store(tws, I.fx);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int p = dh.q(idx), k = idx - p * h;
      if (k == 0) {
        // kx = 0 and kx = nx/2 are real for a real row
        buf[lp(p * n)] = make_double2(A[e].x, B[e].x);
      } else {
        buf[lp(p * n + k)] = make_double2(A[e].x - B[e].y, A[e].y + B[e].x);      // A + i B
        buf[lp(p * n + n - k)] = make_double2(A[e].x + B[e].y, B[e].x - A[e].y);  // conj A + i conj B
      }
    }
  }
  if (pn < np) buf[lp(pn * n + h)] = make_double2(AN.x, BN.x);
  __syncthreads();
  fft_lds<1, false, CAP, NT>(buf, I.fx, np, 1, n, tws);
  const Gp<double> T = dslot(I, a.out) + 2LL * p0 * n;
  const Div dn(n);
#pragma unroll
  for (int e = 0; e < 2 * E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < np * n) {
      const int o = idx + dn.q(idx) * n;
      const double2 z = buf[lp(idx)];
      T[o] = z.x;
      T[o + n] = z.y;
    }
  }
}

// part 0: rows forward, 1: columns A, 2: columns B, 3: columns A inverse, 4: rows
// inverse, 5: single-pass columns (cola then holds its strips).  big selects the row
// kernels for nx > kRowSmallCap.
hipError_t launch_solve_part(int part, bool big, const Inst *insts, const Work *rows, int nrows,
                             const Work *cola, int ncola, const Work *colb, int ncolb,
                             const ArgsSolve &a, hipStream_t st, const Ev &ev) {
  switch (part) {
    case 5:
      APDVM_LAUNCH(ev, k_cols_full, dim3(ncola), dim3(kColThreads), st, insts, cola, ncola, a);
      break;
    case 0:
      if (big)
        APDVM_LAUNCH(ev, (k_rows_forward<kFftCap, kFftThreads>), dim3(nrows), dim3(kFftThreads),
                     st, insts, rows, nrows, a);
      else
        APDVM_LAUNCH(ev, (k_rows_forward<kRowSmallCap, kRowSmallThreads>), dim3(nrows),
                     dim3(kRowSmallThreads), st, insts, rows, nrows, a);
      break;
    case 1:
      APDVM_LAUNCH(ev, k_cols_a<-1>, dim3(ncola), dim3(kColThreads), st, insts, cola, ncola, a);
      break;
    case 2:
      APDVM_LAUNCH(ev, k_cols_b, dim3(ncolb), dim3(kColThreads), st, insts, colb, ncolb, a);
      break;
    case 3:
      APDVM_LAUNCH(ev, k_cols_a<1>, dim3(ncola), dim3(kColThreads), st, insts, cola, ncola, a);
      break;
    default:
      if (big)
        APDVM_LAUNCH(ev, (k_rows_inverse<kFftCap, kFftThreads>), dim3(nrows), dim3(kFftThreads),
                     st, insts, rows, nrows, a);
      else
        APDVM_LAUNCH(ev, (k_rows_inverse<kRowSmallCap, kRowSmallThreads>), dim3(nrows),
                     dim3(kRowSmallThreads), st, insts, rows, nrows, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace apdvm
