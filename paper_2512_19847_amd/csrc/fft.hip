// Periodic Helmholtz solve of Algorithm 1, step 2: (D_Delta - sigma) theta = R.
//
// D_Delta is the sum of two circulant operators, so the 2D DFT diagonalises it:
// theta_hat(kx, ky) = R_hat(kx, ky) / (lambda_x(kx) + lambda_y(ky) - sigma), with
// lambda the Fourier symbol of the fourth-order central second difference.  The (0,0)
// mode is set to the mean of theta^n instead of dividing by -sigma (every derivative
// term of R has zero mean, so this is the exact-arithmetic value; it also covers
// sigma = 0).  All of it runs in float64.
//
// Three kernels, each one read and one write of a float64 plane:
//  rows forward  two real rows packed as one complex length-nx FFT, split into the
//                two half spectra; slot 0 of a half spectrum packs the real kx = 0
//                and kx = nx/2 values.  Output: spectrum [ny][nx/2] complex.
//  columns       a strip of C complex columns staged in LDS: FFT along y, multiply by
//                1 / ((lambda_x + lambda_y - sigma) nx ny), inverse FFT along y.  The
//                packed column 0 holds the real kx = 0 and kx = nx/2 columns; its
//                modes ky and -ky are combined to apply their two different symbols.
//  rows inverse  the reverse of rows forward (Hermitian extension, inverse FFT).
//
// The FFT is a mixed-radix (8, 4, 3, 2) Stockham autosort transform in LDS: each pass
// reads R strided inputs per butterfly, applies twiddles from a float64 table of
// exp(-2 pi i m / n), does a radix-R DFT in registers and writes R outputs; the pass
// is in place (every thread holds its butterflies in registers across a barrier).
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

// In-register DFT of length R with kernel exp(DIR 2 pi i / R).
template <int R, int DIR>
__device__ __forceinline__ void dft(double2 *v);

template <>
__device__ __forceinline__ void dft<2, -1>(double2 *v) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <>
__device__ __forceinline__ void dft<2, 1>(double2 *v) {
  dft<2, -1>(v);
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
template <>
__device__ __forceinline__ void dft<4, -1>(double2 *v) {
  dft4<-1>(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ void dft<4, 1>(double2 *v) {
  dft4<1>(v[0], v[1], v[2], v[3]);
}

template <int DIR>
__device__ __forceinline__ void dft8(double2 *v) {
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
template <>
__device__ __forceinline__ void dft<8, -1>(double2 *v) {
  dft8<-1>(v);
}
template <>
__device__ __forceinline__ void dft<8, 1>(double2 *v) {
  dft8<1>(v);
}

template <int DIR>
__device__ __forceinline__ void dft3(double2 *v) {
  const double h = 0.86602540378443864676;  // sqrt(3)/2
  const double2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
  const double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
  const double2 jd = rot<DIR>(make_double2(h * d.x, h * d.y));
  v[0] = cadd(v[0], s);
  v[1] = cadd(m, jd);
  v[2] = csub(m, jd);
}
template <>
__device__ __forceinline__ void dft<3, -1>(double2 *v) {
  dft3<-1>(v);
}
template <>
__device__ __forceinline__ void dft<3, 1>(double2 *v) {
  dft3<1>(v);
}

// One Stockham pass over nb transforms of length n held in LDS, element j of
// transform b at buf[j * es + b * bs].  BMAJOR: consecutive threads take consecutive
// transforms (column layout) instead of consecutive butterflies (row layout).
template <int R, int DIR, bool BMAJOR>
__device__ __forceinline__ void pass(double2 *buf, int n, int nb, int es, int bs, int Ns,
                                     const double2 *__restrict__ tw) {
  constexpr int NPER = (kFftCap + R * kFftThreads - 1) / (R * kFftThreads);
  const int nbf = n / R;
  const int total = nbf * nb;
  const int twstep = n / (Ns * R);
  double2 v[NPER][R];
  int dst[NPER];
#pragma unroll
  for (int p = 0; p < NPER; ++p) {
    const int t = threadIdx.x + p * kFftThreads;
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

template <int DIR, bool BMAJOR>
__device__ void fft_lds(double2 *buf, const FftPlan &P, int nb, int es, int bs) {
  int Ns = 1;
  for (int ps = 0; ps < P.npass; ++ps) {
    const int R = P.radix[ps];
    switch (R) {
      case 8: pass<8, DIR, BMAJOR>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      case 4: pass<4, DIR, BMAJOR>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      case 3: pass<3, DIR, BMAJOR>(buf, P.n, nb, es, bs, Ns, P.tw); break;
      default: pass<2, DIR, BMAJOR>(buf, P.n, nb, es, bs, Ns, P.tw); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ double *dslot(const Inst &I, int slot) {
  return I.dbase + (long long)slot * I.plane;
}

// ------------------------------------------------------------------ rows forward

__global__ __launch_bounds__(kFftThreads) void k_rows_forward(const Inst *__restrict__ insts,
                                                              const Work *__restrict__ work,
                                                              int nwork, ArgsSolve a) {
  __shared__ double2 buf[kFftCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const double *R = dslot(I, a.r);
  for (int idx = threadIdx.x; idx < np * n; idx += kFftThreads) {
    const int p = idx / n, x = idx - p * n;
    const long long ya = 2LL * (p0 + p);
    buf[idx] = make_double2(R[ya * n + x], R[(ya + 1) * n + x]);
  }
  __syncthreads();
  fft_lds<-1, false>(buf, I.fx, np, 1, n);
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < np * h; idx += kFftThreads) {
    const int p = idx / h, k = idx - p * h;
    const double2 Z = buf[p * n + k];
    double2 A, B;
    if (k == 0) {
      const double2 Zh = buf[p * n + h];
      A = make_double2(Z.x, Zh.x);
      B = make_double2(Z.y, Zh.y);
    } else {
      const double2 W = buf[p * n + n - k];  // Z[n-k]; its conjugate pairs with Z[k]
      A = make_double2(0.5 * (Z.x + W.x), 0.5 * (Z.y - W.y));
      B = make_double2(0.5 * (Z.y + W.y), -0.5 * (Z.x - W.x));
    }
    const long long ya = 2LL * (p0 + p);
    S[ya * h + k] = A;
    S[(ya + 1) * h + k] = B;
  }
}

// ------------------------------------------------------------------ columns

__global__ __launch_bounds__(kFftThreads) void k_columns(const Inst *__restrict__ insts,
                                                         const Work *__restrict__ work, int nwork,
                                                         ArgsSolve a) {
  __shared__ double2 buf[kFftCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.ny, K = I.nx / 2;
  const int k0 = wk.a;
  const int C = min(I.cols_per_block, K - k0);
  double2 *S = reinterpret_cast<double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < n * C; idx += kFftThreads) {
    const int y = idx / C, c = idx - y * C;
    buf[idx] = S[(long long)y * K + k0 + c];
  }
  __syncthreads();
  fft_lds<-1, true>(buf, I.fy, C, C, 1);
  const double sig = I.sigma[a.stage], s = I.inv_nxny;
  const double *lx = I.lam_x, *ly = I.lam_y;
  for (int idx = threadIdx.x; idx < n * C; idx += kFftThreads) {
    const int ky = idx / C, c = idx - ky * C;
    const int k = k0 + c;
    if (k > 0) {
      const double d = s / (lx[k] + ly[ky] - sig);
      buf[idx] = make_double2(buf[idx].x * d, buf[idx].y * d);
    }
  }
  if (k0 == 0) {
    // packed column: Z = S0 + i SN with S0, SN the spectra of the real kx = 0 and
    // kx = nx/2 columns; S0(ky) = (Z(ky) + conj Z(-ky))/2, SN(ky) = (Z(ky) - conj Z(-ky))/2i.
    // Applying d0 to S0 and dN to SN and recombining gives
    // Z'(ky) = (d0 + dN)/2 Z(ky) + (d0 - dN)/2 conj Z(-ky).
    const double lxN = lx[K];
    for (int ky = threadIdx.x; ky <= n / 2; ky += kFftThreads) {
      const int km = (n - ky) % n;
      const double2 Z1 = buf[ky * C], Z2 = buf[km * C];
      if (ky == 0) {
        const double dN = s / (lxN + ly[0] - sig);
        buf[0] = make_double2(I.theta_mean, Z1.y * dN);
      } else {
        const double d0a = s / (lx[0] + ly[ky] - sig), dNa = s / (lxN + ly[ky] - sig);
        const double pa = 0.5 * (d0a + dNa), ma = 0.5 * (d0a - dNa);
        const double2 o1 = make_double2(pa * Z1.x + ma * Z2.x, pa * Z1.y - ma * Z2.y);
        if (km == ky) {
          buf[ky * C] = o1;
        } else {
          const double d0b = s / (lx[0] + ly[km] - sig), dNb = s / (lxN + ly[km] - sig);
          const double pb = 0.5 * (d0b + dNb), mb = 0.5 * (d0b - dNb);
          const double2 o2 = make_double2(pb * Z2.x + mb * Z1.x, pb * Z2.y - mb * Z1.y);
          buf[ky * C] = o1;
          buf[km * C] = o2;
        }
      }
    }
  }
  __syncthreads();
  fft_lds<1, true>(buf, I.fy, C, C, 1);
  for (int idx = threadIdx.x; idx < n * C; idx += kFftThreads) {
    const int y = idx / C, c = idx - y * C;
    S[(long long)y * K + k0 + c] = buf[idx];
  }
}

// ------------------------------------------------------------------ rows inverse

__global__ __launch_bounds__(kFftThreads) void k_rows_inverse(const Inst *__restrict__ insts,
                                                              const Work *__restrict__ work,
                                                              int nwork, ArgsSolve a) {
  __shared__ double2 buf[kFftCap];
  const Work wk = work[xcd_item_fft(nwork)];
  const Inst &I = insts[wk.inst];
  const int n = I.nx, h = n / 2;
  const int p0 = wk.a;
  const int np = min(I.row_pairs_per_block, I.ny / 2 - p0);
  const double2 *S = reinterpret_cast<const double2 *>(dslot(I, a.spec));
  for (int idx = threadIdx.x; idx < np * h; idx += kFftThreads) {
    const int p = idx / h, k = idx - p * h;
    const long long ya = 2LL * (p0 + p);
    const double2 A = S[ya * h + k], B = S[(ya + 1) * h + k];
    if (k == 0) {
      buf[p * n] = make_double2(A.x, B.x);
      buf[p * n + h] = make_double2(A.y, B.y);
    } else {
      buf[p * n + k] = make_double2(A.x - B.y, A.y + B.x);
      buf[p * n + n - k] = make_double2(A.x + B.y, B.x - A.y);
    }
  }
  __syncthreads();
  fft_lds<1, false>(buf, I.fx, np, 1, n);
  double *T = dslot(I, a.out);
  for (int idx = threadIdx.x; idx < np * n; idx += kFftThreads) {
    const int p = idx / n, x = idx - p * n;
    const long long ya = 2LL * (p0 + p);
    const double2 z = buf[idx];
    T[ya * n + x] = z.x;
    T[(ya + 1) * n + x] = z.y;
  }
}

// part 0: rows forward, 1: columns, 2: rows inverse.
hipError_t launch_solve_part(int part, const Inst *insts, const Work *rows, int nrows,
                             const Work *cols, int ncols, const ArgsSolve &a, hipStream_t st) {
  if (part == 0)
    hipLaunchKernelGGL(k_rows_forward, dim3(nrows), dim3(kFftThreads), 0, st, insts, rows, nrows,
                       a);
  else if (part == 1)
    hipLaunchKernelGGL(k_columns, dim3(ncols), dim3(kFftThreads), 0, st, insts, cols, ncols, a);
  else
    hipLaunchKernelGGL(k_rows_inverse, dim3(nrows), dim3(kFftThreads), 0, st, insts, rows, nrows,
                       a);
  return hipGetLastError();
}

}  // namespace apdvm
