// Host-only stand-in for the part of the HIP runtime API that the library's host code
// uses, for the bounds-checked CPU build (APDVM_HOSTCHECK).  "Device" memory is host
// memory from a registry of live allocations, so every range the host code hands to a
// copy, a fill or a launch can be checked against it; streams run their work at once,
// except while they are being captured, when the work is recorded into a graph and runs
// when the graph is launched.  Events carry no time (elapsed time reads a fixed 1 us).
// Not a HIP implementation: kernels do not exist here (see launch_check.cpp).
#pragma once

#include <cstddef>
#include <cstdint>

#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline
#define __launch_bounds__(...)

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorInvalidResourceHandle = 400,
  hipErrorIllegalState = 401,
  hipErrorStreamCaptureUnsupported = 900
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

struct ihipStream_t;
typedef ihipStream_t *hipStream_t;
struct ihipEvent_t;
typedef ihipEvent_t *hipEvent_t;
struct ihipGraph;
typedef ihipGraph *hipGraph_t;
struct hipGraphExec;
typedef hipGraphExec *hipGraphExec_t;
struct hipGraphNode;
typedef hipGraphNode *hipGraphNode_t;

struct double2 {
  double x, y;
};
inline double2 make_double2(double x, double y) { return double2{x, y}; }

hipError_t hipMalloc(void **p, size_t bytes);
template <typename T>
inline hipError_t hipMalloc(T **p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void **>(p), bytes);
}
hipError_t hipFree(void *p);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s);
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int *d);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *err_node,
                               char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphDestroy(hipGraph_t g);
