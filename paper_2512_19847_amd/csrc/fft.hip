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

// One Stockham pass over nb transforms of length n held in LDS, element j of
// transform b at buf[j * es + b * bs].  BMAJOR: consecutive threads take consecutive
// transforms (column tiles) instead of consecutive butterflies (rows).
template <int R, int DIR, bool BMAJOR, int CAP, int NT>
__device__ __forceinline__ void pass(double2 *buf, int n, int nb, int es, int bs, int Ns,
                                     const double2 *__restrict__ tw) {
  constexpr int NPER = (CAP + R * NT - 1) / (R * NT);
  const int nbf = n / R;
  const int total = nbf * nb;
  const int twstep = n / (Ns * R);
  double2 v[NPER][R];
  int dst[NPER];
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int t = threadIdx.x + p * NT;
    dst[p] = -1;
    if (t < total) {
      int j, b;
      if (BMAJOR) {
        j = t / nb;
        b = t - j * nb;
      } else {
        b = t / nbf;
        j = t - b * nbf;
      }
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = buf[(j + r * nbf) * es + b * bs];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[k * r * twstep];
        if (DIR > 0) w.y = -w.y;
        v[p][r] = cmul(v[p][r], w);
      }
      dft<R, DIR>(v[p]);
      dst[p] = ((j / Ns) * Ns * R + k) * es + b * bs;
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    if (dst[p] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[p] + r * Ns * es] = v[p][r];
    }
  }
  __syncthreads();
}

template <int DIR, bool BMAJOR, int CAP, int NT>
__device__ void fft_lds(double2 *buf, const FftPlan &P, int nb, int es, int bs) {
  int Ns = 1;
  for (int ps = 0; ps < P.npass; ++ps) {
    const int R = P.radix[ps];
    switch (R) {
      case 8: pass<8, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      case 4: pass<4, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      case 3: pass<3, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      default: pass<2, DIR, BMAJOR, CAP, NT>(buf, P.n, nb, es, bs, Ns, P.tw); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ double *dslot(const Inst &I, int slot) {
  return I.dbase + (long long)slot * I.plane;
}

// ------------------------------------------------------------------ rows forward

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_rows_forward(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, K = h + 1;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const double *R = dslot(I, a.r);
  for (int idx = threadIdx.x; idx < np * n; idx += NT) {
    const int p = idx / n, x = idx - p * n;
    const long long ya = 2LL * (p0 + p);
    buf[idx] = make_double2(R[ya * n + x], R[(ya + 1) * n + x]);
  }
  __syncthreads();
  fft_lds<-1, false, CAP, NT>(buf, I.fx, np, 1, n);
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < np * K; idx += NT) {
    const int p = idx / K, k = idx - p * K;
    const double2 Z = buf[p * n + (k == h ? h : k)];
    const double2 W = buf[p * n + ((n - k) % n)];  // Z[n-k]; its conjugate pairs with Z[k]
    // A = (Z + conj W) / 2, B = (Z - conj W) / 2i: the spectra of the two real rows
    const double2 A = make_double2(0.5 * (Z.x + W.x), 0.5 * (Z.y - W.y));
    const double2 B = make_double2(0.5 * (Z.y + W.y), -0.5 * (Z.x - W.x));
    const long long ya = 2LL * (p0 + p);
    S[ya * K + k] = A;
    S[(ya + 1) * K + k] = B;
  }
}

// ------------------------------------------------------------------ columns

// Tile of C columns of the spectrum: element j of column c at buf[j * es + c].
constexpr int kColCap = 2048;
constexpr int kColThreads = 256;

// A: length-n1 FFT over rows y = r + n2 m, m = 0..n1-1, for the C columns k0.. of the
// tile; work item (inst, k0, r).
template <int DIR>
__global__ __launch_bounds__(kColThreads) void k_cols_a(const Inst *__restrict__ insts,
                                                        const Work *__restrict__ work,
                                                        int nwork, ArgsSolve a) {
  __shared__ double2 buf[kColCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1, n1 = I.f1.n, n2 = I.f2.n;
  const int k0 = wk.a, r = wk.b;
  const int C = min(I.cols_per_block, K - k0);
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < n1 * C; idx += kColThreads) {
    const int m = idx / C, c = idx - m * C;
    buf[idx] = S[(long long)(r + n2 * m) * K + k0 + c];
  }
  __syncthreads();
  fft_lds<DIR, true, kColCap, kColThreads>(buf, I.f1, C, C, 1);
  for (int idx = threadIdx.x; idx < n1 * C; idx += kColThreads) {
    const int m = idx / C, c = idx - m * C;
    S[(long long)(r + n2 * m) * K + k0 + c] = buf[idx];
  }
}

// B: for G groups k1 = g0.. of n2 contiguous rows n2 k1 + r: twiddle, length-n2 FFT,
// symbol divide, inverse length-n2 FFT, conjugate twiddle.  LDS layout [r][g][c].
__global__ __launch_bounds__(kColThreads) void k_cols_b(const Inst *__restrict__ insts,
                                                        const Work *__restrict__ work, int nwork,
                                                        ArgsSolve a) {
  __shared__ double2 buf[kColCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1, n = I.ny, n1 = I.f1.n, n2 = I.f2.n;
  const int k0 = wk.a, g0 = wk.b;
  const int C = min(I.cols_per_block, K - k0);
  const int G = min(I.groups_per_block, n1 - g0);
  const int GC = G * C;
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  const double2 *twn = I.fy.tw;  // exp(-2 pi i m / ny)
  for (int idx = threadIdx.x; idx < n2 * GC; idx += kColThreads) {
    const int r = idx / GC, rem = idx - r * GC;
    const int g = rem / C, c = rem - g * C;
    const int k1 = g0 + g;
    const double2 v = S[(long long)(n2 * k1 + r) * K + k0 + c];
    buf[idx] = cmul(v, twn[(r * k1) % n]);
  }
  __syncthreads();
  fft_lds<-1, true, kColCap, kColThreads>(buf, I.f2, GC, GC, 1);
  const double sig = I.sigma[a.stage], s = I.inv_nxny;
  for (int idx = threadIdx.x; idx < n2 * GC; idx += kColThreads) {
    const int k2 = idx / GC, rem = idx - k2 * GC;
    const int g = rem / C, c = rem - g * C;
    const int ky = g0 + g + n1 * k2, kx = k0 + c;
    if (kx == 0 && ky == 0) {
      buf[idx] = make_double2(I.theta_mean, 0.0);
    } else {
      const double d = s / (I.lam_x[kx] + I.lam_y[ky] - sig);
      buf[idx] = make_double2(buf[idx].x * d, buf[idx].y * d);
    }
  }
  __syncthreads();
  fft_lds<1, true, kColCap, kColThreads>(buf, I.f2, GC, GC, 1);
  for (int idx = threadIdx.x; idx < n2 * GC; idx += kColThreads) {
    const int r = idx / GC, rem = idx - r * GC;
    const int g = rem / C, c = rem - g * C;
    const int k1 = g0 + g;
    double2 w = twn[(r * k1) % n];
    w.y = -w.y;
    S[(long long)(n2 * k1 + r) * K + k0 + c] = cmul(buf[idx], w);
  }
}

// Single pass over whole columns (ny <= kColCap / C): forward FFT along y, symbol divide
// with the (0,0) rule, inverse FFT, for the C columns k0.. of the tile; work item
// (inst, k0).  One launch instead of the three of the four-step form, for grids whose
// columns fit a tile.
__global__ __launch_bounds__(kColThreads) void k_cols_full(const Inst *__restrict__ insts,
                                                           const Work *__restrict__ work,
                                                           int nwork, ArgsSolve a) {
  __shared__ double2 buf[kColCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int K = I.nx / 2 + 1, n = I.ny;
  const int k0 = wk.a;
  const int C = min(I.cols_full_per_block, K - k0);
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < n * C; idx += kColThreads) {
    const int y = idx / C, c = idx - y * C;
    buf[idx] = S[(long long)y * K + k0 + c];
  }
  __syncthreads();
  fft_lds<-1, true, kColCap, kColThreads>(buf, I.fy, C, C, 1);
  const double sig = I.sigma[a.stage], s = I.inv_nxny;
  for (int idx = threadIdx.x; idx < n * C; idx += kColThreads) {
    const int ky = idx / C, c = idx - ky * C;
    const int kx = k0 + c;
    if (kx == 0 && ky == 0) {
      buf[idx] = make_double2(I.theta_mean, 0.0);
    } else {
      const double d = s / (I.lam_x[kx] + I.lam_y[ky] - sig);
      buf[idx] = make_double2(buf[idx].x * d, buf[idx].y * d);
    }
  }
  __syncthreads();
  fft_lds<1, true, kColCap, kColThreads>(buf, I.fy, C, C, 1);
  for (int idx = threadIdx.x; idx < n * C; idx += kColThreads) {
    const int y = idx / C, c = idx - y * C;
    S[(long long)y * K + k0 + c] = buf[idx];
  }
}

// ------------------------------------------------------------------ rows inverse

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_rows_inverse(const Inst *__restrict__ insts,
                                                     const Work *__restrict__ work, int nwork,
                                                     ArgsSolve a) {
  __shared__ double2 buf[CAP];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2, K = h + 1;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const double2 *S = reinterpret_cast<const double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < np * h; idx += NT) {
    const int p = idx / h, k = idx - p * h;
    const long long ya = 2LL * (p0 + p);
    const double2 A = S[ya * K + k], B = S[(ya + 1) * K + k];
    if (k == 0) {
      // kx = 0 and kx = nx/2 are real for a real row
      const double2 AN = S[ya * K + h], BN = S[(ya + 1) * K + h];
      buf[p * n] = make_double2(A.x, B.x);
      buf[p * n + h] = make_double2(AN.x, BN.x);
    } else {
      buf[p * n + k] = make_double2(A.x - B.y, A.y + B.x);          // A + i B
      buf[p * n + n - k] = make_double2(A.x + B.y, B.x - A.y);      // conj A + i conj B
    }
  }
  __syncthreads();
  fft_lds<1, false, CAP, NT>(buf, I.fx, np, 1, n);
  double *T = dslot(I, a.out);
  for (int idx = threadIdx.x; idx < np * n; idx += NT) {
    const int p = idx / n, x = idx - p * n;
    const long long ya = 2LL * (p0 + p);
    const double2 z = buf[idx];
    T[ya * n + x] = z.x;
    T[(ya + 1) * n + x] = z.y;
  }
}

// part 0: rows forward, 1: columns A, 2: columns B, 3: columns A inverse, 4: rows
// inverse, 5: single-pass columns (cola then holds its strips).  big selects the row
// kernels for nx > kRowSmallCap.
hipError_t launch_solve_part(int part, bool big, const Inst *insts, const Work *rows, int nrows,
                             const Work *cola, int ncola, const Work *colb, int ncolb,
                             const ArgsSolve &a, hipStream_t st) {
  switch (part) {
    case 5:
      hipLaunchKernelGGL(k_cols_full, dim3(ncola), dim3(kColThreads), 0, st, insts, cola, ncola,
                         a);
      break;
    case 0:
      if (big)
        hipLaunchKernelGGL((k_rows_forward<kFftCap, kFftThreads>), dim3(nrows), dim3(kFftThreads),
                           0, st, insts, rows, nrows, a);
      else
        hipLaunchKernelGGL((k_rows_forward<kRowSmallCap, kRowSmallThreads>), dim3(nrows),
                           dim3(kRowSmallThreads), 0, st, insts, rows, nrows, a);
      break;
    case 1:
      hipLaunchKernelGGL(k_cols_a<-1>, dim3(ncola), dim3(kColThreads), 0, st, insts, cola, ncola,
                         a);
      break;
    case 2:
      hipLaunchKernelGGL(k_cols_b, dim3(ncolb), dim3(kColThreads), 0, st, insts, colb, ncolb, a);
      break;
    case 3:
      hipLaunchKernelGGL(k_cols_a<1>, dim3(ncola), dim3(kColThreads), 0, st, insts, cola, ncola,
                         a);
      break;
    default:
      if (big)
        hipLaunchKernelGGL((k_rows_inverse<kFftCap, kFftThreads>), dim3(nrows), dim3(kFftThreads),
                           0, st, insts, rows, nrows, a);
      else
        hipLaunchKernelGGL((k_rows_inverse<kRowSmallCap, kRowSmallThreads>), dim3(nrows),
                           dim3(kRowSmallThreads), 0, st, insts, rows, nrows, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace apdvm
