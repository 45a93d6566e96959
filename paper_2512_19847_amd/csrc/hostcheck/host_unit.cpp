// The library's host runtime, compiled as plain C++ against the host-only runtime
// stand-in for the bounds-checked CPU build.
#include "../host.hip"
