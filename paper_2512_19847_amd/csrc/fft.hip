// Periodic Helmholtz solve of Algorithm 1, step 2: (D_Delta - sigma) theta = R.
//
// D_Delta is the sum of two circulant operators, so the 2D DFT diagonalises it:
// theta_hat(kx, ky) = R_hat(kx, ky) / (lambda_x(kx) + lambda_y(ky) - sigma), with
// lambda the Fourier symbol of the fourth-order central second difference.  The (0,0)
// mode is set to the mean of theta^n instead of dividing by -sigma (every derivative
// term of R has zero mean, so this is the exact-arithmetic value; it also covers
// sigma = 0).  All of it runs in float64.
//
// Three kernels, each one read and one write of a float64 plane-sized array:
//  rows forward   two real rows packed as one complex length-nx FFT, split into the two
//                 half spectra kx = 0..nx/2, stored column-major: spectrum [nx/2][ny]
//                 complex, so every column is ny contiguous values.  kx = 0 and
//                 kx = nx/2 are real for a real row and share column 0 as the real and
//                 imaginary part (nx/2 columns, not nx/2 + 1).
//  columns        whole columns, C of them per workgroup (C ny <= 8192 complex values in
//                 LDS): FFT along y, multiply by 1 / ((lambda_x + lambda_y - sigma) nx ny)
//                 with the (0,0) rule (column 0: separated into its two real columns'
//                 spectra by their Hermitian symmetry, each with its own divisor), inverse
//                 FFT, in place.
//  rows inverse   Hermitian extension of the half spectra, inverse FFT, two real rows.
// The largest column form, the inverse rows of the largest row form when every nx is a
// multiple of 4, and the forward rows when every nx is that form's length, run split: a
// radix-2 step in registers leaves two half-length transforms, done one after the other in
// half the LDS, so two workgroups share a CU.  Where every line of a launch fills its form,
// each transform takes its first pass from registers and, where its values stay with the
// thread, leaves its last pass there (fft_one).
//
// Every FFT is a mixed-radix (8, 4, 3, 2) Stockham autosort transform in LDS: each pass
// reads R strided inputs per butterfly, applies twiddles from a float64 table of
// exp(-2 pi i m / n), does a radix-R DFT in registers and writes R outputs; the pass is
// in place (every thread holds its butterflies in registers across a barrier).
#include "common.hpp"

namespace apdvm {

__device__ __forceinline__ int xcd_item_fft(int nwork) { return xcd_remap(blockIdx.x, nwork); }

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

// Global address at a 32-bit byte offset from a wave-uniform base (a plane or the spectrum
// is at most 512 MiB): the base stays in scalar registers and the offset is the only
// per-lane address.
template <typename P>
__device__ __forceinline__ P at_byte(P base, unsigned b) {
  using C = __attribute__((address_space(1))) const char *;
  return (P)((C)base + b);
}

// LDS layout of the FFT buffers: one padding element after every 2^SH (none for SH = 0),
// so the strided writes of the early Stockham passes (stride R Ns elements of 16 bytes)
// spread over the banks instead of hitting the same few.  SH = 3 for the whole-row and
// whole-column kernels, SH = 4 for the split kernels (their 4096-value halves, two
// workgroups per CU).
template <int SH = 3>
__device__ __forceinline__ int lp(int i) {
  return SH ? i + (i >> SH) : i;
}

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

// Twiddles w^r (r = 1..R-1, w = tws entry m, conjugated for DIR > 0) of one butterfly,
// from one table lookup: the powers by products of depth <= 3 (w^2 = w w, w^3 = w^2 w,
// w^4 = w^2 w^2, w^(4+j) = w^4 w^j), each applied as soon as it is formed, so at most w,
// w^2, w^3 and w^4 are live at once.
template <int R, int DIR>
__device__ __forceinline__ void twiddle(double2 *v, const double2 *tws, int lb, int m) {
  double2 w1 = tw_at(tws, lb, m);
  if (DIR > 0) w1.y = -w1.y;
  v[1] = cmul(v[1], w1);
  if constexpr (R >= 3) {
    const double2 w2 = cmul(w1, w1);
    v[2] = cmul(v[2], w2);
    if constexpr (R >= 4) {
      const double2 w3 = cmul(w2, w1);
      v[3] = cmul(v[3], w3);
      if constexpr (R == 8) {
        const double2 w4 = cmul(w2, w2);
        v[4] = cmul(v[4], w4);
        v[5] = cmul(v[5], cmul(w4, w1));
        v[6] = cmul(v[6], cmul(w4, w2));
        v[7] = cmul(v[7], cmul(w4, w3));
      }
    }
  }
}

// One Stockham pass over nb transforms of length n held in LDS, element j of transform b
// at buf[lp(b n + j)]; consecutive threads take consecutive butterflies of a transform.
// The first pass (Ns = 1) has unit twiddles and skips them.
template <int R, int DIR, int CAP, int NT, int SH>
__device__ __forceinline__ void pass(double2 *buf, int n, int nb, int Ns, const double2 *tws,
                                     int lb, int tsc) {
  constexpr int NPER = (CAP + R * NT - 1) / (R * NT);
  const int nbf = n / R;
  const int total = nbf * nb;
  const int twstep = n / (Ns * R);
  const Div dnbf(nbf), dns(Ns);
  double2 v[NPER][R];
  int dst[NPER];
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int t = threadIdx.x + p * NT;
    dst[p] = -1;
    if (t < total) {
      const int b = dnbf.q(t), j = t - b * nbf;
      const int jq = dns.q(j), k = j - jq * Ns;
      const int src = b * n + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = buf[lp<SH>(src + r * nbf)];
      if (Ns > 1) twiddle<R, DIR>(v[p], tws, lb, k * twstep * tsc);
      dft<R, DIR>(v[p]);
      dst[p] = b * n + jq * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    if (dst[p] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp<SH>(dst[p] + r * Ns)] = v[p][r];
    }
  }
  __syncthreads();
}

// Length-n transforms (plan P) of nb contiguous runs of n values in LDS.
template <int DIR, int CAP, int NT, int SH = 3>
__device__ __forceinline__ void fft_lds(double2 *buf, const FftPlan &P, int nb,
                                        const double2 *tws) {
  int Ns = 1;
  for (int ps = 0; ps < P.npass; ++ps) {
    const int R = P.radix[ps];
    switch (R) {
      case 8: pass<8, DIR, CAP, NT, SH>(buf, P.n, nb, Ns, tws, P.lb, P.tsc); break;
      case 4: pass<4, DIR, CAP, NT, SH>(buf, P.n, nb, Ns, tws, P.lb, P.tsc); break;
      case 3: pass<3, DIR, CAP, NT, SH>(buf, P.n, nb, Ns, tws, P.lb, P.tsc); break;
      default: pass<2, DIR, CAP, NT, SH>(buf, P.n, nb, Ns, tws, P.lb, P.tsc); break;
    }
    Ns *= R;
  }
}

// One transform that fills the buffer (n = CAP, nb = 1, CAP = 8 NT, so n is a power of two
// and every radix R of its plan is 8, 4 or 2 with R NT dividing CAP) with its values in
// registers at either end: thread t holds element t + e NT in v[e], e < 8.  A pass takes
// butterfly j = t + p NT (p < NPER = CAP / (R NT)) from elements j + r CAP / R =
// t + (p + r NPER) NT, all of them thread t's own: the first pass (Ns = 1, unit twiddles,
// outputs at j R + r) reads them from registers instead of LDS, and the last (Ns = CAP / R,
// k = j, twiddle index j) writes its outputs j + r Ns = t + (p + r NPER) NT to registers.
// The operations are those of fft_lds in the same order; the compiler may still fuse a
// multiply into an addition differently where values no longer pass through LDS (the
// whole-row forward rows and the columns give the same bits as their LDS forms, the split
// inverse rows differ in the last bits).  The first pass begins with a barrier when
// sync_first (buf still being read); the last leaves none (the caller syncs before buf is
// written).
template <int R, int DIR, int CAP, int NT, int SH>
__device__ __forceinline__ void pass_first_reg(const double2 *in, double2 *buf, bool sync_first) {
  constexpr int NPER = CAP / (R * NT);
  static_assert(NPER * R * NT == CAP, "radix and threads must tile the buffer");
  double2 v[NPER][R];
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[p][r] = in[p + r * NPER];
    dft<R, DIR>(v[p]);
  }
  if (sync_first) __syncthreads();
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int j = threadIdx.x + p * NT;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[lp<SH>(j * R + r)] = v[p][r];
  }
  __syncthreads();
}
template <int R, int DIR, int CAP, int NT, int SH>
__device__ __forceinline__ void pass_last_reg(const double2 *buf, double2 *out, const double2 *tws,
                                              int lb, int tsc) {
  constexpr int NPER = CAP / (R * NT);
  static_assert(NPER * R * NT == CAP, "radix and threads must tile the buffer");
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int j = threadIdx.x + p * NT;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = buf[lp<SH>(j + r * (CAP / R))];
    twiddle<R, DIR>(v, tws, lb, j * tsc);
    dft<R, DIR>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) out[p + r * NPER] = v[r];
  }
}
// Several transforms filling the buffer: nb = CAP / n lines of n = 8^m values (64 <= n <
// CAP), every pass radix 8, with their values in registers at either end.  With n8 = n / 8,
// thread t takes butterfly j = t mod n8 of line b = t / n8 in the first pass (elements b n +
// j + r n8, outputs at b n + 8 j + r) and in the last (Ns = n8, k = j, twiddle index j:
// elements, and outputs, b n + j + r n8), so both ends hold element (b, j + r n8) in v[r].
template <int DIR, int CAP, int NT, int SH, bool IN_REGS, bool OUT_REGS>
__device__ __forceinline__ void fft_lines(double2 *v, double2 *buf, const FftPlan &P, int n,
                                          int nb, int lg8, const double2 *tws,
                                          bool sync_first) {
  static_assert(CAP == 8 * NT, "eight values per thread");
  const int n8 = 1 << lg8, b = threadIdx.x >> lg8, j = threadIdx.x & (n8 - 1);
  int Ns = 1, ps = 0;
  if constexpr (IN_REGS) {
    double2 w[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) w[r] = v[r];
    dft<8, DIR>(w);
    if (sync_first) __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[lp<SH>(b * n + 8 * j + r)] = w[r];
    __syncthreads();
    Ns = 8;
    ps = 1;
  }
  const int last = OUT_REGS ? P.npass - 1 : P.npass;
  for (; ps < last; ++ps) {
    pass<8, DIR, CAP, NT, SH>(buf, n, nb, Ns, tws, P.lb, P.tsc);
    Ns *= 8;
  }
  if constexpr (OUT_REGS) {
    double2 w[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) w[r] = buf[lp<SH>(b * n + j + r * n8)];
    twiddle<8, DIR>(w, tws, P.lb, j * P.tsc);
    dft<8, DIR>(w);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = w[r];
  }
}

// Radix of the last pass of a length-n plan, n = 2^k: the plans take as many radix-8 passes
// as fit, first, then one of 4 (k mod 3 = 2) or 2 (k mod 3 = 1).
constexpr int last_radix_pow2(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k % 3 == 0 ? 8 : (k % 3 == 2 ? 4 : 2);
}
template <int DIR, int CAP, int NT, int SH, bool IN_REGS, bool OUT_REGS>
__device__ __forceinline__ void fft_one(double2 *v, double2 *buf, const FftPlan &P,
                                        const double2 *tws, bool sync_first) {
  static_assert(CAP == 8 * NT && (CAP & (CAP - 1)) == 0, "eight values per thread, n = 2^k");
  // the radices of the register passes are fixed by n = CAP (a switch over the plan's
  // would make the register arrays dynamically indexed)
  constexpr int RL = last_radix_pow2(CAP);
  int Ns = 1, ps = 0;
  if constexpr (IN_REGS) {
    pass_first_reg<8, DIR, CAP, NT, SH>(v, buf, sync_first);
    Ns = 8;
    ps = 1;
  }
  const int last = OUT_REGS ? P.npass - 1 : P.npass;
  for (; ps < last; ++ps) {
    const int R = P.radix[ps];
    switch (R) {
      case 8: pass<8, DIR, CAP, NT, SH>(buf, CAP, 1, Ns, tws, P.lb, P.tsc); break;
      case 4: pass<4, DIR, CAP, NT, SH>(buf, CAP, 1, Ns, tws, P.lb, P.tsc); break;
      default: pass<2, DIR, CAP, NT, SH>(buf, CAP, 1, Ns, tws, P.lb, P.tsc); break;
    }
    Ns *= R;
  }
  if constexpr (OUT_REGS) pass_last_reg<RL, DIR, CAP, NT, SH>(buf, v, tws, P.lb, P.tsc);
}

__device__ __forceinline__ Gp<double> dslot(const Inst &I, int slot) {
  return gp(I.dbase + (long long)slot * I.plane);
}
__device__ __forceinline__ Gp<dv2> cslot(const Inst &I, int slot) {
  return reinterpret_cast<Gp<dv2>>(dslot(I, slot));
}



// Each kernel below stages its tile in two phases: every thread first issues all of its
// global loads (data, twiddle table and, in the small column form, the symbol values of
// the modes it will scale), then writes them to LDS, so one memory round trip covers the
// whole tile.  The whole-line kernels come in three forms (FORM): 0 in LDS from end to
// end; 1 one line filling the buffer, its first pass taking the loaded values and its last
// leaving its outputs in registers (fft_one); 2 the same for several lines of 8^m values
// filling it (fft_lines).  The host takes 1 or 2 only when every line of the launch
// qualifies (fft_reg_form).

// ------------------------------------------------------------------ rows forward

template <int CAP, int NT, int FORM>
__global__ __launch_bounds__(NT) void k_rows_forward(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP + CAP / 8];
  __shared__ double2 tws[kTwCap];
  constexpr int E = CAP / NT;
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const int cnt = np * n;
  const Gp<const double> R = dslot(I, a.r) + 2LL * p0 * n;
  const Div dn(n);
  TwStage<NT> tw;
  tw.load(I.fx);
  // element of slot e: t + e NT, or in the form of several lines (FORM 2) element j + e n8
  // of line b, t = b n8 + j (the register layout of fft_lines)
  const int lg8 = FORM == 2 ? __builtin_ctz(n) - 3 : 0;
  auto elem = [&](int e) {
    return FORM == 2 ? (int)(threadIdx.x >> lg8) * n + (int)(threadIdx.x & ((1u << lg8) - 1)) +
                           (e << lg8)
                     : (int)threadIdx.x + e * NT;
  };
  double ra[E], rb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = elem(e);
    if (idx < cnt) {
      const int o = idx + dn.q(idx) * n;  // row 2p, column x
      ra[e] = *at_byte(R, (unsigned)o * 8u);
      rb[e] = *at_byte(R, (unsigned)(o + n) * 8u);
    }
  }
  tw.store(tws, I.fx);
  if constexpr (FORM == 1) {  // one row pair fills the buffer: the first pass takes the loads
    double2 z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = make_double2(ra[e], rb[e]);
    fft_one<-1, CAP, NT, 3, true, false>(z, buf, I.fx, tws, false);
  } else if constexpr (FORM == 2) {  // several row pairs of 8^m values fill it
    double2 z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = make_double2(ra[e], rb[e]);
    fft_lines<-1, CAP, NT, 3, true, false>(z, buf, I.fx, n, np, lg8, tws, false);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cnt) buf[lp(idx)] = make_double2(ra[e], rb[e]);
    }
    __syncthreads();
    fft_lds<-1, CAP, NT>(buf, I.fx, np, tws);
  }
  // column-major half spectra S[k][y] for the 2 np rows y = 2 p0 .. of the block:
  // consecutive threads write consecutive rows of one column
  const int ny = I.ny, m = 2 * np;
  const Gp<dv2> S = cslot(I, a.spec) + 2LL * p0;
  const Div dm(m);
  for (int idx = threadIdx.x; idx < m * h; idx += NT) {
    const int k = dm.q(idx), yl = idx - k * m, p = yl >> 1;
    const double2 Z = buf[lp(p * n + k)];
    // Z[n-k] (Z[n/2] for k = 0); its conjugate pairs with Z[k]
    const double2 W = buf[lp(p * n + (k == 0 ? h : n - k))];
    double2 o;
    if (k == 0)  // (A[0], A[n/2]) and (B[0], B[n/2]): Z[0] = A[0] + i B[0], likewise Z[n/2]
      o = (yl & 1) ? make_double2(Z.y, W.y) : make_double2(Z.x, W.x);
    else  // A = (Z + conj W) / 2, B = (Z - conj W) / 2i: the spectra of rows 2p, 2p + 1
      o = (yl & 1) ? make_double2(0.5 * (Z.y + W.y), -0.5 * (Z.x - W.x))
                   : make_double2(0.5 * (Z.x + W.x), 0.5 * (Z.y - W.y));
    stc(at_byte(S, (unsigned)(k * ny + yl) * 16u), o);
  }
}

// Forward rows of nx = kFftCap in half the LDS, as the split column kernel does for columns
// (n = nx, h = n / 2, w = exp(-2 pi i / n)): a radix-2 decimation in frequency in registers,
//   Z[2m] = FFT_h(z[t] + z[t + h])[m],  Z[2m + 1] = FFT_h((z[t] - z[t + h]) w^t)[m],
// leaves two length-h transforms, done one after the other with the odd half held in
// registers.  The Hermitian partner Z[n - k] of a mode has its parity (n is even): Z[2m]
// pairs with Z[2(h - m)] (Z[0] with Z[h] = Z[2 (h / 2)]), Z[2m + 1] with Z[2(h - 1 - m) + 1],
// so each half writes its columns of the half spectra (k = 2m, then k = 2m + 1) from LDS
// as soon as it is transformed.  One row pair per workgroup (the register form of both
// half transforms' first pass); two workgroups share a CU, so one loads or stores while the
// other transforms.
constexpr int kRowFwdSplitThreads = 512;
// LDS padding of the split forward rows (lp): one element in 16, as the other split kernels.
constexpr int kRowFwdSplitPad = 4;

template <int NT, int SH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rows_forward_split(
    const Inst *__restrict__ insts, const Work *__restrict__ work, int nwork, ArgsSolve a) {
  constexpr int CAP = kFftCap / 2;
  constexpr int E = CAP / NT;  // values of a half per thread
  __shared__ double2 buf[SH ? CAP + (CAP >> SH) : CAP];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, ny = I.ny;
  const int p0 = wk.a;
  const Gp<const double> R = dslot(I, a.r) + 2LL * p0 * n;
  TwStage<NT> tw;
  tw.load(I.fx);
  double2 v[E], x1[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {  // z[t] and z[t + h]: rows 2 p0 (real) and 2 p0 + 1 (imaginary)
    const unsigned t = threadIdx.x + e * NT;
    v[e] = make_double2(*at_byte(R, t * 8u), *at_byte(R, (t + (unsigned)n) * 8u));
    x1[e] = make_double2(*at_byte(R, (t + (unsigned)h) * 8u),
                         *at_byte(R, (t + (unsigned)(n + h)) * 8u));
  }
  tw.store(tws, I.fx);
  __syncthreads();  // the table is read below
  // radix-2 step: the even half in v, the odd half (times w^t) in x1, pinned there (left
  // alone, the compiler sinks the step past the even half's transform and keeps both loaded
  // halves live through it)
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = threadIdx.x + e * NT;
    const double2 s = cadd(v[e], x1[e]);
    x1[e] = cmul(csub(v[e], x1[e]), tw_at(tws, I.fx.lb, t));
    v[e] = s;
    asm volatile("" : "+v"(x1[e].x), "+v"(x1[e].y));
  }
  const Gp<dv2> S = cslot(I, a.spec) + 2LL * p0;
  // columns k = 2m + par of the two rows from the transformed half in LDS: A = (Z + conj W)
  // / 2 and B = (Z - conj W) / 2i, W = Z[n - k]; k = 0 packs (A[0], A[n/2]) and (B[0], B[n/2])
  auto put_columns = [&](int par) {
    for (int idx = threadIdx.x; idx < h; idx += NT) {  // h / 2 columns of two rows
      const int m = idx >> 1, yl = idx & 1, k = 2 * m + par;
      const double2 Z = buf[lp<SH>(m)];
      const double2 W = buf[lp<SH>(par ? h - 1 - m : (m == 0 ? h / 2 : h - m))];
      double2 o;
      if (k == 0)
        o = yl ? make_double2(Z.y, W.y) : make_double2(Z.x, W.x);
      else
        o = yl ? make_double2(0.5 * (Z.y + W.y), -0.5 * (Z.x - W.x))
               : make_double2(0.5 * (Z.x + W.x), 0.5 * (Z.y - W.y));
      stc(at_byte(S, (unsigned)(k * ny + yl) * 16u), o);
    }
  };
  fft_one<-1, CAP, NT, SH, true, false>(v, buf, I.fxh, tws, false);
  put_columns(0);
  fft_one<-1, CAP, NT, SH, true, false>(x1, buf, I.fxh, tws, true);
  put_columns(1);
}

// ------------------------------------------------------------------ columns

// Divisor of a mode from its symbol values: 1 / ((lambda_x + lambda_y - sigma) nx ny)
// (never the (0,0) mode, which takes theta_mean instead).
__device__ __forceinline__ double mode_div(const Inst &I, double sig, double lx, double ly) {
  return I.inv_nxny / (lx + ly - sig);
}

// The C = cols_per_block columns kx = k0.. of the column-major spectrum, one contiguous
// run of C ny complex values: forward FFT along y, symbol divide with the (0,0) rule,
// inverse FFT, stored in place.  Work item (inst, k0).
template <int CAP, int NT, int FORM>
__global__ __launch_bounds__(NT) void k_cols(const Inst *__restrict__ insts,
                                             const Work *__restrict__ work, int nwork,
                                             ArgsSolve a) {
  __shared__ double2 buf[CAP + CAP / 8];
  __shared__ double2 tws[kTwCap];
  constexpr int E = CAP / NT;
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int ny = I.ny, K = I.nx / 2, h = I.nx / 2;
  const int k0 = wk.a;
  const int C = min(I.cols_per_block, K - k0);
  const int cnt = C * ny;
  const Gp<dv2> S = cslot(I, a.spec) + (long long)k0 * ny;
  const double sig = I.sigma[a.stage];
  const Div dy(ny);
  TwStage<NT> tw;
  tw.load(I.fy);
  // element of slot e (column c = e / ny, mode y): t + e NT, or in the form of several
  // columns (FORM 2) mode j + e n8 of column b, t = b n8 + j (the register layout of fft_lines)
  const int lg8 = FORM == 2 ? __builtin_ctz(ny) - 3 : 0;
  auto elem = [&](int e) {
    return FORM == 2 ? (int)(threadIdx.x >> lg8) * ny + (int)(threadIdx.x & ((1u << lg8) - 1)) +
                           (e << lg8)
                     : (int)threadIdx.x + e * NT;
  };
  // PRE: the symbol values of the thread's modes travel with the data loads.  The larger
  // forms have no registers to spare for them (they would lower the waves per SIMD below
  // what the LDS allows) and load them after the transform; they hit the L2, every
  // workgroup reads the same ny values.
  constexpr bool PRE = NT == kRowSmallThreads;
  double2 v[E];
  double ly[PRE ? E : 1], lx[PRE ? E : 1];
  double lxh = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = elem(e);
    if (idx < cnt) {
      v[e] = ldc(at_byte(S, (unsigned)idx * 16u));
      if constexpr (PRE) {
        const int c = dy.q(idx), y = idx - c * ny;
        ly[e] = gp(I.lam_y)[y];
        lx[e] = gp(I.lam_x)[k0 + c];
      }
    }
  }
  if (PRE && k0 == 0) lxh = gp(I.lam_x)[h];
  tw.store(tws, I.fy);
  // one column fills the buffer: both transforms take and leave their values in registers
  // (the column-0 block puts the spectrum in LDS too, for the mirrored modes it pairs)
  // (several columns of 8^m values filling it: the same with the layout of fft_lines)
  constexpr bool direct = FORM != 0;
  if constexpr (direct) {
    if constexpr (FORM == 1)
      fft_one<-1, CAP, NT, 3, true, true>(v, buf, I.fy, tws, false);
    else
      fft_lines<-1, CAP, NT, 3, true, true>(v, buf, I.fy, ny, C, lg8, tws, false);
    if (k0 == 0) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) buf[lp(elem(e))] = v[e];
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cnt) buf[lp(idx)] = v[e];
    }
    __syncthreads();
    fft_lds<-1, CAP, NT>(buf, I.fy, C, tws);
  }
  double2 o[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = elem(e);
    if (idx < cnt) {
      const int c = dy.q(idx), y = idx - c * ny;
      double lyy, lxx, lxn;
      if constexpr (PRE) {
        lyy = ly[e];
        lxx = lx[e];
        lxn = lxh;
      } else {
        lyy = gp(I.lam_y)[y];
        lxx = gp(I.lam_x)[k0 + c];
        lxn = k0 + c == 0 ? gp(I.lam_x)[h] : 0.0;
      }
      const double2 z = direct ? v[e] : buf[lp(idx)];
      if (k0 + c == 0) {
        // Z = F0 + i Fh with F0, Fh the (Hermitian) y spectra of the real columns kx = 0
        // and kx = nx/2: F0 = (Z[ky] + conj Z[-ky]) / 2, Fh = (Z[ky] - conj Z[-ky]) / 2i
        const double2 zm = buf[lp(y == 0 ? 0 : ny - y)];
        double2 f0 = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
        double2 fh = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
        const double dh = mode_div(I, sig, lxn, lyy);
        if (y == 0) {
          f0 = make_double2(I.theta_mean, 0.0);  // the (0,0) rule
        } else {
          const double d0 = mode_div(I, sig, lxx, lyy);
          f0 = make_double2(f0.x * d0, f0.y * d0);
        }
        fh = make_double2(fh.x * dh, fh.y * dh);
        o[e] = make_double2(f0.x - fh.y, f0.y + fh.x);  // F0 + i Fh
      } else {
        const double d = mode_div(I, sig, lxx, lyy);
        o[e] = make_double2(z.x * d, z.y * d);
      }
    }
  }
  if constexpr (direct) {
    // (the first inverse pass syncs before it writes: column 0 reads mirrored modes)
    if constexpr (FORM == 1)
      fft_one<1, CAP, NT, 3, true, true>(o, buf, I.fy, tws, true);
    else
      fft_lines<1, CAP, NT, 3, true, true>(o, buf, I.fy, ny, C, lg8, tws, true);
#pragma unroll
    for (int e = 0; e < E; ++e) stc(at_byte(S, (unsigned)elem(e) * 16u), o[e]);
    return;
  }
  __syncthreads();  // column 0 reads mirrored elements of other threads
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) buf[lp(idx)] = o[e];
  }
  __syncthreads();
  fft_lds<1, CAP, NT>(buf, I.fy, C, tws);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) stc(at_byte(S, (unsigned)idx * 16u), buf[lp(idx)]);
  }
}

// Columns of length ny > kColMidCap (the largest form) with half the LDS: a radix-2
// decimation in frequency in registers splits each length-ny transform into two
// independent transforms of length h = ny / 2,
//   X[2k] = FFT_h(x[y] + x[y + h])[k],  X[2k + 1] = FFT_h((x[y] - x[y + h]) w^y)[k],
// w = exp(-2 pi i / ny).  The even half is transformed, divided and inverted in LDS while
// the odd half waits in registers; the two then swap places element by element; the odd
// half is transformed, divided and inverted; and the inverse recombines
//   y[t] = ya[t] + w^-t yb[t],  y[t + h] = ya[t] - w^-t yb[t]
// (ya, yb the inverse transforms of the even and odd modes; unnormalised, the divisors
// carry 1 / (nx ny)).  A workgroup of kColSplitThreads holds C h <= kFftCap / 2 values in
// LDS, so two workgroups share a CU and one loads or stores while the other transforms.
// Four waves per SIMD cap the registers at 128 (the two halves in flight spill a little in
// the LDS form; the register form spills 8 bytes); the buffer is padded one in 16.
// Work item (inst, k0) with C = cols_per_block columns.
constexpr int kColSplitThreads = 512;
// LDS padding of the split column kernel (lp): one element in 16 (register form, 8192^2:
// 365-369 us per launch against 403-406 unpadded and 410 with one in 8).
constexpr int kColSplitPad = 4;
constexpr int kColSplitCap = kFftCap / 2;

template <int NT, int SH, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_cols_split(
    const Inst *__restrict__ insts, const Work *__restrict__ work, int nwork, ArgsSolve a) {
  constexpr int CAP = kColSplitCap;
  constexpr int E = CAP / NT;  // elements of a half per thread
  __shared__ double2 buf[SH ? CAP + (CAP >> SH) : CAP];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int ny = I.ny, K = I.nx / 2, hx = I.nx / 2, h = ny / 2;
  const int k0 = wk.a;
  const int C = min(I.cols_per_block, K - k0);
  const int cnt = C * h;
  const Gp<dv2> S = cslot(I, a.spec) + (long long)k0 * ny;
  const double sig = I.sigma[a.stage];
  const Div dh(h);
  TwStage<NT> tw;
  tw.load(I.fy);
  double2 x0[E], x1[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int c = dh.q(idx), y = idx - c * h;
      const unsigned b = (unsigned)(c * ny + y) * 16u;
      x0[e] = ldc(at_byte(S, b));
      x1[e] = ldc(at_byte(S, b + (unsigned)h * 16u));
    }
  }
  tw.store(tws, I.fy);
  __syncthreads();  // the table is read below
  // one column per workgroup whose half fills the buffer: each half's two transforms take
  // and leave their values in registers (the column-0 block puts each spectrum in LDS too,
  // for the mirrored modes it pairs), and the halves swap places in registers
  constexpr bool direct = DIRECT;
  // mode ky = 2m + par of column c at position c h + m of the half; z: its value in v[e]
  // (direct) or in LDS
  auto divide_modes = [&](int par, double2 *v) {
    double2 o[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cnt) {
        const int c = dh.q(idx), m = idx - c * h;
        const int ky = 2 * m + par;
        const double lyy = gp(I.lam_y)[ky];
        const double lxx = gp(I.lam_x)[k0 + c];
        const double2 z = direct ? v[e] : buf[lp<SH>(idx)];
        if (k0 + c == 0) {
          // Z = F0 + i Fh for the real columns kx = 0 and kx = nx/2: F0 = (Z[ky] +
          // conj Z[-ky]) / 2, Fh = (Z[ky] - conj Z[-ky]) / 2i; -ky has the parity of ky,
          // at position (h - m - par) mod h of the same half
          const int mm = par ? h - 1 - m : (m == 0 ? 0 : h - m);
          const double2 zm = buf[lp<SH>(mm)];
          double2 f0 = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
          double2 fh = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));
          const double dhh = mode_div(I, sig, gp(I.lam_x)[hx], lyy);
          if (ky == 0) {
            f0 = make_double2(I.theta_mean, 0.0);  // the (0,0) rule
          } else {
            const double d0 = mode_div(I, sig, lxx, lyy);
            f0 = make_double2(f0.x * d0, f0.y * d0);
          }
          fh = make_double2(fh.x * dhh, fh.y * dhh);
          o[e] = make_double2(f0.x - fh.y, f0.y + fh.x);
        } else {
          const double d = mode_div(I, sig, lxx, lyy);
          o[e] = make_double2(z.x * d, z.y * d);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = o[e];
  };
  if constexpr (direct) {
    // radix-2 step: the even-mode half in v, the odd-mode half (times w^y) in x1 (pinned
    // there: left alone, the compiler sinks the step to the swap and keeps both loaded
    // halves live through the even half's transforms instead, which spills them)
    double2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int y = threadIdx.x + e * NT;
      v[e] = cadd(x0[e], x1[e]);
      x1[e] = cmul(csub(x0[e], x1[e]), tw_at(tws, I.fy.lb, y));
      asm volatile("" : "+v"(x1[e].x), "+v"(x1[e].y));
    }
    auto half = [&](int par) {
      fft_one<-1, CAP, NT, SH, true, true>(v, buf, I.fyh, tws, par == 1);
      if (k0 == 0) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) buf[lp<SH>(threadIdx.x + e * NT)] = v[e];
        __syncthreads();
      }
      divide_modes(par, v);
      fft_one<1, CAP, NT, SH, true, true>(v, buf, I.fyh, tws, true);
    };
    half(0);
#pragma unroll
    for (int e = 0; e < E; ++e) {  // ya to x1, the odd half to v
      const double2 t = x1[e];
      x1[e] = v[e];
      v[e] = t;
    }
    half(1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int y = threadIdx.x + e * NT;
      double2 w = tw_at(tws, I.fy.lb, y);
      w.y = -w.y;  // w^-y
      const double2 yb = cmul(v[e], w);
      const unsigned b = (unsigned)y * 16u;
      stc(at_byte(S, b), cadd(x1[e], yb));
      stc(at_byte(S, b + (unsigned)h * 16u), csub(x1[e], yb));
    }
    return;
  }
  // radix-2 step: the even-mode half to LDS, the odd-mode half (times w^y) in x1
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int c = dh.q(idx), y = idx - c * h;
      buf[lp<SH>(idx)] = cadd(x0[e], x1[e]);
      x1[e] = cmul(csub(x0[e], x1[e]), tw_at(tws, I.fy.lb, y));
    }
  }
  __syncthreads();
  auto divide = [&](int par) {
    fft_lds<-1, CAP, NT, SH>(buf, I.fyh, C, tws);
    double2 o[E];
    divide_modes(par, o);
    __syncthreads();  // column 0 reads mirrored elements of other threads
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cnt) buf[lp<SH>(idx)] = o[e];
    }
    __syncthreads();
    fft_lds<1, CAP, NT, SH>(buf, I.fyh, C, tws);
  };
  divide(0);
  // swap: each thread takes its elements of ya and puts its odd half in their place
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const double2 ya = buf[lp<SH>(idx)];
      buf[lp<SH>(idx)] = x1[e];
      x1[e] = ya;
    }
  }
  __syncthreads();
  divide(1);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int c = dh.q(idx), y = idx - c * h;
      double2 w = tw_at(tws, I.fy.lb, y);
      w.y = -w.y;  // w^-y
      const double2 yb = cmul(buf[lp<SH>(idx)], w);
      const unsigned b = (unsigned)(c * ny + y) * 16u;
      stc(at_byte(S, b), cadd(x1[e], yb));
      stc(at_byte(S, b + (unsigned)h * 16u), csub(x1[e], yb));
    }
  }
}

// ------------------------------------------------------------------ rows inverse

template <int CAP, int NT, int FORM>
__global__ __launch_bounds__(NT) void k_rows_inverse(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP + CAP / 8];
  __shared__ double2 tws[kTwCap];
  constexpr int EI = CAP / (2 * NT), EO = CAP / NT;
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, ny = I.ny;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const int cnt = np * h;
  // column-major half spectra: rows 2p and 2p + 1 of column k are adjacent
  const Gp<const dv2> S = cslot(I, a.spec) + 2LL * p0;
  const Div dp(np);
  TwStage<NT> tw;
  tw.load(I.fx);
  double2 A[EI], B[EI];
#pragma unroll
  for (int e = 0; e < EI; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int k = dp.q(idx), p = idx - k * np;
      const unsigned b = (unsigned)(k * ny + 2 * p) * 16u;
      A[e] = ldc(at_byte(S, b));
      B[e] = ldc(at_byte(S, b + 16u));
    }
  }
  tw.store(tws, I.fx);
#pragma unroll
  for (int e = 0; e < EI; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int k = dp.q(idx), p = idx - k * np;
      if (k == 0) {
        // kx = 0 and kx = nx/2 (real for a real row) share column 0
        buf[lp(p * n)] = make_double2(A[e].x, B[e].x);
        buf[lp(p * n + h)] = make_double2(A[e].y, B[e].y);
      } else {
        buf[lp(p * n + k)] = make_double2(A[e].x - B[e].y, A[e].y + B[e].x);      // A + i B
        buf[lp(p * n + n - k)] = make_double2(A[e].x + B[e].y, B[e].x - A[e].y);  // conj A + i conj B
      }
    }
  }
  __syncthreads();
  const Gp<double> T = dslot(I, a.out) + 2LL * p0 * n;
  if constexpr (FORM == 2) {  // several row pairs of 8^m values: the layout of fft_lines
    const int lg8 = __builtin_ctz(n) - 3;
    double2 z[EO];
    fft_lines<1, CAP, NT, 3, false, true>(z, buf, I.fx, n, np, lg8, tws, false);
    const int b = threadIdx.x >> lg8, j = threadIdx.x & ((1 << lg8) - 1);
#pragma unroll
    for (int e = 0; e < EO; ++e) {
      const unsigned o = (unsigned)(2 * b * n + j + (e << lg8)) * 8u;
      *at_byte(T, o) = z[e].x;
      *at_byte(T, o + (unsigned)n * 8u) = z[e].y;
    }
    return;
  }
  if constexpr (FORM == 1) {  // one row pair fills the buffer: the last pass leaves it in registers
    double2 z[EO];
    fft_one<1, CAP, NT, 3, false, true>(z, buf, I.fx, tws, false);
#pragma unroll
    for (int e = 0; e < EO; ++e) {
      const unsigned o = (unsigned)(threadIdx.x + e * NT) * 8u;
      *at_byte(T, o) = z[e].x;
      *at_byte(T, o + (unsigned)n * 8u) = z[e].y;
    }
    return;
  }
  fft_lds<1, CAP, NT>(buf, I.fx, np, tws);
  const Div dn(n);
#pragma unroll
  for (int e = 0; e < EO; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < np * n) {
      const int o = idx + dn.q(idx) * n;
      const double2 z = buf[lp(idx)];
      *at_byte(T, (unsigned)o * 8u) = z.x;
      *at_byte(T, (unsigned)(o + n) * 8u) = z.y;
    }
  }
}

// ------------------------------------------------------------------ rows inverse, split

// Inverse rows of the largest form in half the LDS, as the split column kernel does for
// columns (n = nx, h = n / 2, w = exp(-2 pi i / n)): the even modes Z[2m] and the odd modes
// Z[2m + 1] of the Hermitian extension of a row pair's half spectra go through two
// length-h inverse transforms, ya and yb, and a radix-2 step in registers gives
//   z[t] = ya[t] + w^-t yb[t],  z[t + h] = ya[t] - w^-t yb[t],
// with ya held in registers while yb is transformed.  The extension pairs Z[k] with Z[n - k],
// a mode of the same parity when h is even (the host takes this form only when every nx
// is a multiple of 4): Z[2m] with Z[2(h - m)] (Z[h] = the even mode h / 2 shares column 0
// with Z[0]), Z[2m + 1] with Z[2(h - 1 - m) + 1].  A workgroup holds C h <= kFftCap / 2
// values (C the row pairs of a block, as in the whole-row form), so two workgroups share a
// CU and one loads or stores while the other transforms.  (The forward rows split the same
// way only where every nx is kFftCap, k_rows_forward_split: with the first pass of each half
// taken from registers and the odd half pinned there, it spills nothing.)
constexpr int kRowSplitThreads = 512;
// LDS padding of the split row kernel (lp): one element in 16 (register form, 8192^2:
// 342 us per launch against 354 unpadded; one in 8 as fast).
constexpr int kRowSplitPad = 4;

// Even (par 0) or odd (par 1) modes of the Hermitian extensions of C row pairs' half
// spectra into buf (pair p at p h), from the loaded column-major values A, B of rows 2p and
// 2p + 1 at k = 2m + par, item idx = m C + p of the h / 2 C items.
template <int SH>
__device__ __forceinline__ void put_modes(double2 *buf, int h, int par, int m, int p,
                                          double2 A, double2 B) {
  if (par == 0 && m == 0) {
    // kx = 0 and kx = nx/2 (real for a real row) share column 0; Z[h] = even mode h / 2
    buf[lp<SH>(p * h)] = make_double2(A.x, B.x);
    buf[lp<SH>(p * h + h / 2)] = make_double2(A.y, B.y);
  } else {
    buf[lp<SH>(p * h + m)] = make_double2(A.x - B.y, A.y + B.x);  // A + i B
    // conj A + i conj B at n - k: even mode h - m, odd mode h - 1 - m
    buf[lp<SH>(p * h + (par ? h - 1 - m : h - m))] = make_double2(A.x + B.y, B.x - A.y);
  }
}

template <int NT, int SH, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_rows_inverse_split(
    const Inst *__restrict__ insts, const Work *__restrict__ work, int nwork, ArgsSolve a) {
  constexpr int CAP = kFftCap / 2;
  constexpr int E = CAP / NT;       // output elements of a half per thread
  constexpr int EI = CAP / (2 * NT);  // loaded modes of a half per thread
  __shared__ double2 buf[SH ? CAP + (CAP >> SH) : CAP];
  __shared__ double2 tws[kTwCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, ny = I.ny;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const int cnt = np * h, cin = np * (h / 2);
  const Gp<const dv2> S = cslot(I, a.spec) + 2LL * p0;
  const Div dp(np), dh(h);
  TwStage<NT> tw;
  tw.load(I.fx);
  // modes k = 2m + par of rows 2p and 2p + 1 into LDS as the half par of the extension
  auto load_half = [&](int par, bool with_table) {
    double2 A[EI], B[EI];
#pragma unroll
    for (int e = 0; e < EI; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cin) {
        const int m = dp.q(idx), p = idx - m * np;
        const unsigned b = (unsigned)((2 * m + par) * ny + 2 * p) * 16u;
        A[e] = ldc(at_byte(S, b));
        B[e] = ldc(at_byte(S, b + 16u));
      }
    }
    if (with_table) tw.store(tws, I.fx);
#pragma unroll
    for (int e = 0; e < EI; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cin) {
        const int m = dp.q(idx), p = idx - m * np;
        put_modes<SH>(buf, h, par, m, p, A[e], B[e]);
      }
    }
    __syncthreads();
  };
  // one row pair whose half fills the buffer: the last pass of each half transform leaves
  // it in registers
  constexpr bool direct = DIRECT;
  load_half(0, true);
  double2 ya[E], yb[E];
  if constexpr (direct) {
    fft_one<1, CAP, NT, SH, false, true>(ya, buf, I.fxh, tws, false);
  } else {
    fft_lds<1, CAP, NT, SH>(buf, I.fxh, np, tws);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = threadIdx.x + e * NT;
      if (idx < cnt) ya[e] = buf[lp<SH>(idx)];
    }
  }
  __syncthreads();
  load_half(1, false);
  if constexpr (direct)
    fft_one<1, CAP, NT, SH, false, true>(yb, buf, I.fxh, tws, false);
  else
    fft_lds<1, CAP, NT, SH>(buf, I.fxh, np, tws);
  const Gp<double> T = dslot(I, a.out) + 2LL * p0 * n;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = threadIdx.x + e * NT;
    if (idx < cnt) {
      const int p = dh.q(idx), t = idx - p * h;
      double2 w = tw_at(tws, I.fx.lb, t);
      w.y = -w.y;  // w^-t
      const double2 yb_t = cmul(direct ? yb[e] : buf[lp<SH>(idx)], w);
      const double2 lo = cadd(ya[e], yb_t), hi = csub(ya[e], yb_t);
      const unsigned o = (unsigned)(2 * p * n + t) * 8u;
      *at_byte(T, o) = lo.x;
      *at_byte(T, o + (unsigned)n * 8u) = lo.y;
      *at_byte(T, o + (unsigned)h * 8u) = hi.x;
      *at_byte(T, o + (unsigned)(n + h) * 8u) = hi.y;
    }
  }
}

// Kernel forms by LDS capacity: 0 kRowSmallCap, 1 kColMidCap, 2 kFftCap complex values;
// D: 0 the LDS form, 1 the register form of one line filling the buffer, 2 that of several
// lines of 8^m values filling it (the launch
// takes ev, st, insts and a of the calling function).
#define APDVM_FFT_FORM_D(V, D, KERNEL, WORK, NWORK)                                           \
  do {                                                                                       \
    if ((V) == 2)                                                                            \
      APDVM_LAUNCH(ev, (KERNEL<kFftCap, kFftThreads, D>), dim3(NWORK), dim3(kFftThreads), st, \
                   insts, WORK, NWORK, a);                                                   \
    else if ((V) == 1)                                                                       \
      APDVM_LAUNCH(ev, (KERNEL<kColMidCap, kColMidThreads, D>), dim3(NWORK),                 \
                   dim3(kColMidThreads), st, insts, WORK, NWORK, a);                         \
    else                                                                                     \
      APDVM_LAUNCH(ev, (KERNEL<kRowSmallCap, kRowSmallThreads, D>), dim3(NWORK),             \
                   dim3(kRowSmallThreads), st, insts, WORK, NWORK, a);                       \
  } while (0)
#define APDVM_FFT_FORM(V, REG, KERNEL, WORK, NWORK)                  \
  do {                                                              \
    if ((REG) == 1)                                                 \
      APDVM_FFT_FORM_D(V, 1, KERNEL, WORK, NWORK);                  \
    else if ((REG) == 2)                                            \
      APDVM_FFT_FORM_D(V, 2, KERNEL, WORK, NWORK);                  \
    else                                                            \
      APDVM_FFT_FORM_D(V, 0, KERNEL, WORK, NWORK);                  \
  } while (0)

// part 0: rows forward, 1: columns, 2: rows inverse; rowv and colv the kernel forms
// (the smallest that holds a whole row, a whole column; rowv 3: the largest row form,
// with the inverse rows split in halves); rowreg (colreg): 1 every row (column) of every
// instance is as long as its form holds (the largest form: kFftCap), so each workgroup
// transforms one line with its values in registers at the ends of the transforms; 2 every
// row (column) is 8^m values, shorter, and fills the blocks of its form (the whole-line
// kernels transform those lines the same way; the split kernels take their LDS form).
hipError_t launch_solve_part(int part, int rowv, int colv, int rowreg, int colreg,
                             const Inst *insts, const Work *rows, int nrows, const Work *cols,
                             int ncols, const ArgsSolve &a, hipStream_t st, const Ev &ev) {
  switch (part) {
    case 0:
      if (rowv == 3 && rowreg == 1)  // rows of kFftCap: half the LDS, two workgroups per CU
        APDVM_LAUNCH(ev, (k_rows_forward_split<kRowFwdSplitThreads, kRowFwdSplitPad>), dim3(nrows),
                     dim3(kRowFwdSplitThreads), st, insts, rows, nrows, a);
      else
        APDVM_FFT_FORM(rowv == 3 ? 2 : rowv, rowreg, k_rows_forward, rows, nrows);
      break;
    case 1:
      if (colv == 2) {  // the largest columns: half the LDS, two workgroups per CU
        if (colreg == 1)
          APDVM_LAUNCH(ev, (k_cols_split<kColSplitThreads, kColSplitPad, true>), dim3(ncols),
                       dim3(kColSplitThreads), st, insts, cols, ncols, a);
        else
          APDVM_LAUNCH(ev, (k_cols_split<kColSplitThreads, kColSplitPad, false>), dim3(ncols),
                       dim3(kColSplitThreads), st, insts, cols, ncols, a);
      } else {
        APDVM_FFT_FORM(colv, colreg, k_cols, cols, ncols);
      }
      break;
    default:
      if (rowv == 3) {  // the largest rows, nx a multiple of 4: half the LDS, two per CU
        if (rowreg == 1)
          APDVM_LAUNCH(ev, (k_rows_inverse_split<kRowSplitThreads, kRowSplitPad, true>),
                       dim3(nrows), dim3(kRowSplitThreads), st, insts, rows, nrows, a);
        else
          APDVM_LAUNCH(ev, (k_rows_inverse_split<kRowSplitThreads, kRowSplitPad, false>),
                       dim3(nrows), dim3(kRowSplitThreads), st, insts, rows, nrows, a);
      } else {
        APDVM_FFT_FORM(rowv, rowreg, k_rows_inverse, rows, nrows);
      }
      break;
  }
  return hipGetLastError();
}

}  // namespace apdvm
