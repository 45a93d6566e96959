// Diagnostics of one instance: sum theta, sum u1, sum u2, max |D0.u| (the divergence
// diagnostic of Section 4, with the central differences of the scheme: fourth or second
// order), min and max of the vorticity D_x u2 - D_y u1, sum |u|^2
// and a finite flag over all six fields.  Two levels: each workgroup reduces its tiles
// with wavefront shuffles and LDS into one record of partials; the host combines the
// records (deterministic: no atomics).
#include "common.hpp"

#include <mutex>

namespace apdvm {

template <typename T>
__device__ __forceinline__ double at(const T *p, int nx, int ny, int x, int y) {
  return (double)p[(long long)wrap_index(y, ny) * nx + wrap_index(x, nx)];
}

// Central first derivative along (ox, oy); f = 1/(12h) for order 4, 1/(2h) for order 2.
template <typename T>
__device__ __forceinline__ double dcen(const T *p, int nx, int ny, int x, int y, int ox, int oy,
                                       double f, int co) {
  if (co == 2) return (at(p, nx, ny, x + ox, y + oy) - at(p, nx, ny, x - ox, y - oy)) * f;
  return (at(p, nx, ny, x - 2 * ox, y - 2 * oy) - 8.0 * at(p, nx, ny, x - ox, y - oy) +
          8.0 * at(p, nx, ny, x + ox, y + oy) - at(p, nx, ny, x + 2 * ox, y + 2 * oy)) *
         f;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag(const Inst *__restrict__ insts,
                                              const Work *__restrict__ tiles, int ntiles, int ty,
                                              int su1, int su2, int dth, int sv1, int sv2, int sq,
                                              int co, double *__restrict__ partials) {
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 1.0};
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Work wk = tiles[t];
    const Inst &I = insts[wk.inst];
    const int nx = I.nx, ny = I.ny;
    const T *tb = reinterpret_cast<const T *>(I.tbase);
    // the velocity is float64 in both forms: transport planes of the FP64 form, the
    // float64 velocity planes of the FP32-split form
    const double *ub = sizeof(T) == sizeof(double) ? reinterpret_cast<const double *>(I.tbase)
                                                   : I.dbase;
    const double *u1 = ub + (long long)su1 * I.plane, *u2 = ub + (long long)su2 * I.plane;
    const T *v1 = tb + (long long)sv1 * I.plane, *v2 = tb + (long long)sv2 * I.plane;
    const T *q = tb + (long long)sq * I.plane;
    const double *th = I.dbase + (long long)dth * I.plane;
    const double ihx12 = co == 2 ? 0.5 * I.ihx : I.ihx / 12.0;
    const double ihy12 = co == 2 ? 0.5 * I.ihy : I.ihy / 12.0;
    const int tx = threadIdx.x & 63, ty0 = threadIdx.x >> 6;
    const int x = wk.a + tx;
    if (x >= nx) continue;
    for (int ly = ty0; ly < ty; ly += 4) {
      const int y = wk.b + ly;
      if (y >= ny) break;
      const long long g = (long long)y * nx + x;
      const double a = (double)u1[g], b = (double)u2[g], c = th[g];
      acc[0] += c;
      acc[1] += a;
      acc[2] += b;
      const double div =
          dcen(u1, nx, ny, x, y, 1, 0, ihx12, co) + dcen(u2, nx, ny, x, y, 0, 1, ihy12, co);
      const double vor =
          dcen(u2, nx, ny, x, y, 1, 0, ihx12, co) - dcen(u1, nx, ny, x, y, 0, 1, ihy12, co);
      acc[3] = fmax(acc[3], fabs(div));
      acc[4] = fmin(acc[4], vor);
      acc[5] = fmax(acc[5], vor);
      acc[6] += a * a + b * b;
      const bool fin = isfinite(a) && isfinite(b) && isfinite(c) && isfinite((double)v1[g]) &&
                       isfinite((double)v2[g]) && isfinite((double)q[g]);
      if (!fin) acc[7] = 0.0;
    }
  }
  __shared__ double red[4][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double r[8];
  r[0] = wave_sum(acc[0]);
  r[1] = wave_sum(acc[1]);
  r[2] = wave_sum(acc[2]);
  r[3] = wave_max(acc[3]);
  r[4] = wave_min(acc[4]);
  r[5] = wave_max(acc[5]);
  r[6] = wave_sum(acc[6]);
  r[7] = wave_min(acc[7]);
  if (lane == 0)
    for (int k = 0; k < 8; ++k) red[w][k] = r[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double o[8];
    for (int k = 0; k < 8; ++k) o[k] = red[0][k];
    for (int ww = 1; ww < 4; ++ww) {
      o[0] += red[ww][0];
      o[1] += red[ww][1];
      o[2] += red[ww][2];
      o[3] = fmax(o[3], red[ww][3]);
      o[4] = fmin(o[4], red[ww][4]);
      o[5] = fmax(o[5], red[ww][5]);
      o[6] += red[ww][6];
      o[7] = fmin(o[7], red[ww][7]);
    }
    for (int k = 0; k < 8; ++k) partials[8 * blockIdx.x + k] = o[k];
  }
}

// tiles: the stencil work items (64 x ty cells) of one instance.
hipError_t launch_diagnostics(const Inst *insts, const Work *tiles, int ntiles, int ty, int split,
                              int su1, int su2, int dth, int sv1, int sv2, int sq, int co,
                              double *partials, int nblocks, hipStream_t st) {
  if (split)
    hipLaunchKernelGGL(k_diag<float>, dim3(nblocks), dim3(256), 0, st, insts, tiles, ntiles, ty,
                       su1, su2, dth, sv1, sv2, sq, co, partials);
  else
    hipLaunchKernelGGL(k_diag<double>, dim3(nblocks), dim3(256), 0, st, insts, tiles, ntiles, ty,
                       su1, su2, dth, sv1, sv2, sq, co, partials);
  return hipGetLastError();
}

// ------------------------------------------------------------------ static scratch

// Scratch of apdvm_diagnostics_device: up to kScratchBlocks records of eight partials
// (64 KiB), one set per GPU, held until the process ends.  In host code the name
// `scratch` is a host-side stand-in: kernels receive the device address that
// hipGetSymbolAddress returned for the current device (scratch_init).
constexpr int kScratchBlocks = 1024;
static __device__ __align__(256) double scratch[8 * kScratchBlocks];

constexpr int kMaxDevices = 64;
static double *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Once per device, with that device current: resolve the device address of `scratch`.
hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<double *>(p);
  return hipSuccess;
}

// Device address of the scratch of `device` (nullptr before scratch_init succeeded).
double *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

int scratch_blocks() { return kScratchBlocks; }

// Combines the nblocks partial records in block order, as the host does in
// apdvm_diagnostics, and writes the eight diagnostics (area = hx hy).  One thread: the
// records are few and the fixed order keeps the result identical to the host's.
__global__ __launch_bounds__(64) void k_diag_finish(const double *__restrict__ partials,
                                                    int nblocks, double area,
                                                    double *__restrict__ out) {
  if (threadIdx.x != 0) return;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 1e300, -1e300, 0.0, 1.0};
  for (int b = 0; b < nblocks; ++b) {
    const double *q = partials + 8 * b;
    acc[0] += q[0];
    acc[1] += q[1];
    acc[2] += q[2];
    acc[3] = fmax(acc[3], q[3]);
    acc[4] = fmin(acc[4], q[4]);
    acc[5] = fmax(acc[5], q[5]);
    acc[6] += q[6];
    acc[7] = fmin(acc[7], q[7]);
  }
  out[0] = acc[0] * area;
  out[1] = acc[1] * area;
  out[2] = acc[2] * area;
  out[3] = acc[3];
  out[4] = acc[4];
  out[5] = acc[5];
  out[6] = 0.5 * acc[6] * area;
  out[7] = acc[7];
}

hipError_t launch_diag_finish(const double *partials, int nblocks, double area, double *out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(64), 0, st, partials, nblocks, area, out);
  return hipGetLastError();
}

}  // namespace apdvm
