// Host-only stand-in for the few HIP declarations the serving scheduler
// (paper_2607_20211_amd/csrc/drsf_server.hip) uses, so that the scheduler
// can be compiled with g++ and run under the address, undefined-behaviour
// and thread sanitizers without a GPU (tests/test_server_host.py installs
// it as <hip/hip_runtime.h>).  Test infrastructure only.
#pragma once
#include <cstddef>
#include <cstdint>
typedef struct StubStream *hipStream_t;
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1 };
enum { hipStreamNonBlocking = 1, hipStreamDefault = 0 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipGetLastError();
hipError_t hipMalloc(void **p, size_t n);
template <class T> hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags = 0);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int *d);
