// Stand-in for drsf_kernels.h when the serving scheduler is built on the
// host with tests/server_host/stubs.cpp (test infrastructure only).
#pragma once
#include <hip/hip_runtime.h>
namespace drsf {
void launch_digest(int32_t n, const int32_t *parent, const int32_t *label, unsigned long long *out, hipStream_t s);
}
