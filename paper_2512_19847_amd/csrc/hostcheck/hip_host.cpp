// Host-only runtime stand-in of the bounds-checked CPU build (see hip/hip_runtime.h).
#include "hostcheck.hpp"

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

struct Capture {
  hipStream_t origin = nullptr;
  std::vector<std::function<void()>> ops;
};
struct ihipStream_t {
  Capture *cap = nullptr;
};
struct ihipEvent_t {
  Capture *cap = nullptr;
  bool recorded = false;
};
struct ihipGraph {
  std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
  std::vector<std::function<void()>> ops;
};

namespace {

std::mutex g_mu;
std::map<uintptr_t, size_t> g_alloc;  // base -> bytes
std::set<hipStream_t> g_streams;
ihipStream_t g_null_stream;
hostcheck::Counters g_count;

hipStream_t real(hipStream_t s) { return s ? s : &g_null_stream; }

bool known_stream(hipStream_t s) { return !s || g_streams.count(s) != 0; }

}  // namespace

namespace hostcheck {

bool in_device(const void *p, size_t bytes) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_alloc.upper_bound(a);
  if (it == g_alloc.begin()) return false;
  --it;
  return a >= it->first && a + bytes <= it->first + it->second && a + bytes >= a;
}

void fail(const char *fmt, ...) {
  const long long n = ++g_count.violations;
  if (n <= 20) {
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hostcheck violation: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
  }
}

void enqueue(hipStream_t s, std::function<void()> fn) {
  hipStream_t r = real(s);
  if (r->cap) {
    r->cap->ops.push_back(std::move(fn));
    ++g_count.captured_ops;
  } else {
    fn();
  }
}

Counters &counters() { return g_count; }

}  // namespace hostcheck

using hostcheck::fail;
using hostcheck::in_device;

hipError_t hipMalloc(void **p, size_t bytes) {
  if (!p) return hipErrorInvalidValue;
  const size_t n = (bytes + 255) / 256 * 256;
  void *q = std::aligned_alloc(256, n ? n : 256);
  if (!q) return hipErrorOutOfMemory;
  std::memset(q, 0xA5, n ? n : 256);  // device memory starts as garbage
  std::lock_guard<std::mutex> lock(g_mu);
  g_alloc[reinterpret_cast<uintptr_t>(q)] = bytes;
  *p = q;
  return hipSuccess;
}

hipError_t hipFree(void *p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_alloc.find(reinterpret_cast<uintptr_t>(p));
    if (it == g_alloc.end()) {
      fail("hipFree of %p, which is not the base of a live allocation", p);
      return hipErrorInvalidValue;
    }
    g_alloc.erase(it);
  }
  std::free(p);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s) {
  if (!known_stream(s)) return hipErrorInvalidResourceHandle;
  const bool dd = kind == hipMemcpyHostToDevice || kind == hipMemcpyDeviceToDevice;
  const bool sd = kind == hipMemcpyDeviceToHost || kind == hipMemcpyDeviceToDevice;
  if (kind == hipMemcpyDefault) {
    if (!in_device(dst, bytes) && !in_device(src, bytes)) fail("default copy between host ranges");
  } else {
    if (dd && !in_device(dst, bytes)) fail("copy of %zu bytes to %p outside device memory", bytes, dst);
    if (sd && !in_device(src, bytes)) fail("copy of %zu bytes from %p outside device memory", bytes, src);
  }
  if (bytes == 0) return hipSuccess;
  hostcheck::enqueue(s, [=] { std::memmove(dst, src, bytes); });
  return hipSuccess;
}

hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s) {
  if (!known_stream(s)) return hipErrorInvalidResourceHandle;
  if (real(s)->cap) fail("hipMemsetAsync recorded into a captured graph");
  if (!in_device(dst, bytes)) fail("fill of %zu bytes at %p outside device memory", bytes, dst);
  hostcheck::enqueue(s, [=] { std::memset(dst, value, bytes); });
  return hipSuccess;
}

hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int *d) {
  if (!d) return hipErrorInvalidValue;
  *d = 0;
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  if (!s) return hipErrorInvalidValue;
  *s = new ihipStream_t;
  std::lock_guard<std::mutex> lock(g_mu);
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!s || !g_streams.erase(s)) return hipErrorInvalidResourceHandle;
  }
  if (s->cap) fail("stream destroyed during capture");
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (!known_stream(s)) return hipErrorInvalidResourceHandle;
  if (real(s)->cap) {
    fail("stream synchronised during capture");
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  if (!known_stream(s) || !e) return hipErrorInvalidResourceHandle;
  hipStream_t r = real(s);
  if (e->cap && !r->cap) r->cap = e->cap;  // the stream joins the capture (a fork)
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || !known_stream(s)) return hipErrorInvalidResourceHandle;
  if (s->cap) return hipErrorIllegalState;
  s->cap = new Capture;
  s->cap->origin = s;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
  if (!s || !g || !s->cap || s->cap->origin != s) return hipErrorIllegalState;
  Capture *c = s->cap;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    for (hipStream_t t : g_streams)
      if (t->cap == c) t->cap = nullptr;
  }
  *g = new ihipGraph{std::move(c->ops)};
  delete c;
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) {
  if (!e) return hipErrorInvalidValue;
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e || !known_stream(s)) return hipErrorInvalidResourceHandle;
  e->cap = real(s)->cap;
  e->recorded = true;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  if (!ms || !a || !b) return hipErrorInvalidValue;
  *ms = 1e-3f;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *,
                               size_t) {
  if (!x || !g) return hipErrorInvalidValue;
  *x = new hipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (!x || !known_stream(s)) return hipErrorInvalidValue;
  ++hostcheck::counters().graph_launches;
  hostcheck::enqueue(s, [x] {
    for (auto &op : x->ops) op();
  });
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
