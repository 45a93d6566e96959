// State handling on the device: statistics of initial fields given in device memory,
// precision conversion between the float64 boundary and the transport planes, and the
// finite check of the state with a snapshot of the last state that passed it.
//
// Finite check (every K steps, inside apdvm_step): k_state_finite reads the six state
// planes of every instance and marks a flag word when any value is NaN or Inf;
// k_snapshot then copies the state into the snapshot set only while the flag is clear,
// and records the step number of the copy.  The flag is sticky, so after a failure the
// snapshot keeps the last state that passed; the host restores it from there.
#include "common.hpp"

namespace apdvm {

// ------------------------------------------------------------ statistics of input fields

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Per workgroup (fixed grid, grid-stride): sum of theta, max |u|, and 0 if any of the six
// fields holds a non-finite value (else 1).  Three doubles per workgroup; the host adds
// them in workgroup order, so the result does not depend on scheduling.  u, v and q are
// of type T (float64 input fields, or the transport planes of the state), theta float64.
constexpr int kStatThreads = 256;
template <typename T>
__global__ __launch_bounds__(kStatThreads) void k_field_stats(
    const T *__restrict__ u1, const T *__restrict__ u2, const double *__restrict__ th,
    const T *__restrict__ v1, const T *__restrict__ v2, const T *__restrict__ q,
    long long n, double *__restrict__ partials) {
  double s = 0.0, um = 0.0, fin = 1.0;
  for (long long i = (long long)blockIdx.x * kStatThreads + threadIdx.x; i < n;
       i += (long long)gridDim.x * kStatThreads) {
    const double a = (double)u1[i], b = (double)u2[i], t = th[i];
    s += t;
    const double m = sqrt(a * a + b * b);
    // a NaN in u would be dropped by fmax; the finite flag catches it
    um = fmax(um, m);
    if (!(isfinite(a) && isfinite(b) && isfinite(t) && isfinite((double)v1[i]) &&
          isfinite((double)v2[i]) && isfinite((double)q[i])))
      fin = 0.0;
  }
  __shared__ double red[kStatThreads / 64][3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  s = wsum(s);
  um = wmax(um);
  fin = -wmax(-fin);  // minimum
  if (lane == 0) {
    red[w][0] = s;
    red[w][1] = um;
    red[w][2] = fin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o0 = red[0][0], o1 = red[0][1], o2 = red[0][2];
    for (int k = 1; k < kStatThreads / 64; ++k) {
      o0 += red[k][0];
      o1 = fmax(o1, red[k][1]);
      o2 = fmin(o2, red[k][2]);
    }
    partials[3 * blockIdx.x + 0] = o0;
    partials[3 * blockIdx.x + 1] = o1;
    partials[3 * blockIdx.x + 2] = o2;
  }
}

// f: u1, u2, theta, v1, v2, q; u, v, q float (split = 1) or float64, theta float64.
hipError_t launch_field_stats(int split, const void *const f[6], long long n, double *partials,
                              int nblocks, hipStream_t st) {
  const double *th = static_cast<const double *>(f[2]);
  if (split)
    hipLaunchKernelGGL(k_field_stats<float>, dim3(nblocks), dim3(kStatThreads), 0, st,
                       static_cast<const float *>(f[0]), static_cast<const float *>(f[1]), th,
                       static_cast<const float *>(f[3]), static_cast<const float *>(f[4]),
                       static_cast<const float *>(f[5]), n, partials);
  else
    hipLaunchKernelGGL(k_field_stats<double>, dim3(nblocks), dim3(kStatThreads), 0, st,
                       static_cast<const double *>(f[0]), static_cast<const double *>(f[1]), th,
                       static_cast<const double *>(f[3]), static_cast<const double *>(f[4]),
                       static_cast<const double *>(f[5]), n, partials);
  return hipGetLastError();
}

// ------------------------------------------------------------ precision conversion

template <typename D, typename S>
__global__ __launch_bounds__(256) void k_convert(D *__restrict__ dst, const S *__restrict__ src,
                                                 long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    dst[i] = (D)src[i];
}

// float64 -> float (to_float = 1) or float -> float64 (to_float = 0), n values.
hipError_t launch_convert(void *dst, const void *src, long long n, int to_float, hipStream_t st) {
  long long b = (n + 255) / 256;
  const int nb = (int)(b < 16384 ? (b < 1 ? 1 : b) : 16384);
  if (to_float)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(256), 0, st,
                       static_cast<float *>(dst), static_cast<const double *>(src), n);
  else
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(256), 0, st,
                       static_cast<double *>(dst), static_cast<const float *>(src), n);
  return hipGetLastError();
}

// ------------------------------------------------------------ finite check and snapshot

// Marks *flag when any value of the state is not finite.  One 64 x ty tile per workgroup
// of 256 threads (the 16-row tile table), every instance of the context.
template <typename T>
__global__ __launch_bounds__(256) void k_state_finite(const Inst *__restrict__ insts,
                                                      const Work *__restrict__ tiles, int ntiles,
                                                      int ty, StateSet s,
                                                      unsigned *__restrict__ flag) {
  const Work wk = tiles[blockIdx.x];
  const Inst &I = insts[wk.inst];
  const int x = wk.a + (threadIdx.x & 63);
  if (x >= I.nx) return;
  const T *tb = reinterpret_cast<const T *>(I.tbase);
  bool fin = true;
  for (int ly = threadIdx.x >> 6; ly < ty; ly += 4) {
    const int y = wk.b + ly;
    if (y >= I.ny) break;
    const long long g = (long long)y * I.nx + x;
#pragma unroll
    for (int p = 0; p < 5; ++p) fin = fin && isfinite((double)tb[(long long)s.t[p] * I.plane + g]);
    for (int p = 0; p < s.nd; ++p) fin = fin && isfinite(I.dbase[(long long)s.d[p] * I.plane + g]);
  }
  if (!fin) *flag = 1u;  // every writer stores the same value
}

// Copies the state slots src to dst while *flag is clear; the first workgroup records
// step in *ck_step.
template <typename T>
__global__ __launch_bounds__(256) void k_snapshot(const Inst *__restrict__ insts,
                                                  const Work *__restrict__ tiles, int ntiles,
                                                  int ty, StateSet src, StateSet dst,
                                                  const unsigned *__restrict__ flag,
                                                  long long *__restrict__ ck_step,
                                                  long long step) {
  if (*flag) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ck_step = step;
  const Work wk = tiles[blockIdx.x];
  const Inst &I = insts[wk.inst];
  const int x = wk.a + (threadIdx.x & 63);
  if (x >= I.nx) return;
  T *tb = reinterpret_cast<T *>(I.tbase);
  for (int ly = threadIdx.x >> 6; ly < ty; ly += 4) {
    const int y = wk.b + ly;
    if (y >= I.ny) break;
    const long long g = (long long)y * I.nx + x;
#pragma unroll
    for (int p = 0; p < 5; ++p)
      tb[(long long)dst.t[p] * I.plane + g] = tb[(long long)src.t[p] * I.plane + g];
    for (int p = 0; p < src.nd; ++p)
      I.dbase[(long long)dst.d[p] * I.plane + g] = I.dbase[(long long)src.d[p] * I.plane + g];
  }
}

hipError_t launch_state_finite(int split, const Inst *insts, const Work *tiles, int ntiles,
                               int ty, const StateSet &s, unsigned *flag, hipStream_t st) {
  if (split)
    hipLaunchKernelGGL(k_state_finite<float>, dim3(ntiles), dim3(256), 0, st, insts, tiles,
                       ntiles, ty, s, flag);
  else
    hipLaunchKernelGGL(k_state_finite<double>, dim3(ntiles), dim3(256), 0, st, insts, tiles,
                       ntiles, ty, s, flag);
  return hipGetLastError();
}

hipError_t launch_snapshot(int split, const Inst *insts, const Work *tiles, int ntiles, int ty,
                           const StateSet &a, const StateSet &b, const unsigned *flag,
                           long long *ck_step, long long step, hipStream_t st) {
  if (split)
    hipLaunchKernelGGL(k_snapshot<float>, dim3(ntiles), dim3(256), 0, st, insts, tiles, ntiles,
                       ty, a, b, flag, ck_step, step);
  else
    hipLaunchKernelGGL(k_snapshot<double>, dim3(ntiles), dim3(256), 0, st, insts, tiles, ntiles,
                       ty, a, b, flag, ck_step, step);
  return hipGetLastError();
}

}  // namespace apdvm
