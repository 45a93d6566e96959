// Shared by the host-only runtime stand-in (hip_host.cpp), the launch checks
// (launch_check.cpp) and the driver (driver.cpp) of the bounds-checked CPU build.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

namespace hostcheck {

// True when [p, p + bytes) lies inside one live device allocation.
bool in_device(const void *p, size_t bytes);
// Records a violation (counted, the first ones printed to stderr).
void fail(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
// Runs fn in the order of stream s: at once, or at graph launch while s is captured.
void enqueue(hipStream_t s, std::function<void()> fn);

struct Counters {
  long long launches = 0;    // kernel launches checked
  long long items = 0;       // work items (workgroups) checked
  long long indices = 0;     // staged or wrapped indices checked
  long long violations = 0;  // failed checks
  long long graph_launches = 0;
  long long captured_ops = 0;
};
Counters &counters();

}  // namespace hostcheck
