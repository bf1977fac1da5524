// CPU stand-in for the part of the HIP runtime API that the library's host
// sources call (runtime.cpp, mesh_step.cpp), so that they can be built with
// g++ and run under AddressSanitizer / UndefinedBehaviorSanitizer /
// ThreadSanitizer on a machine without a GPU.  TEST INFRASTRUCTURE ONLY:
// "device" memory is host memory, copies are memcpy, streams and events are
// synchronous, and device allocations can be made to fail on purpose
// (fakehip::fail_after) to drive the library's E_NOMEM paths.
#pragma once

#include <atomic>
#include <chrono>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

// HIP's function-space attributes (host and device inline helpers in the
// library's shared headers): no meaning on the CPU
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidDevice = 101,
    hipErrorNotReady = 600,
} hipError_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

struct fake_stream {
    int id;
};
struct fake_event {
    std::chrono::steady_clock::time_point t;
};
typedef fake_stream *hipStream_t;
typedef fake_event *hipEvent_t;

struct hipDeviceProp_t {
    char name[256];
    int multiProcessorCount;
    size_t sharedMemPerBlock;
};

struct float2 {
    float x, y;
};
struct float4 {
    float x, y, z, w;
};

namespace fakehip {
// Device allocations made so far, and the number after which they fail
// (negative: never).
inline std::atomic<long> malloc_calls{0};
inline std::atomic<long> fail_after{-1};
inline std::atomic<long> live_blocks{0};
}  // namespace fakehip

inline const char *hipGetErrorString(hipError_t e)
{
    switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorInvalidDevice: return "hipErrorInvalidDevice";
    default: return "hipErrorInvalidValue";
    }
}
inline hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
inline hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int d)
{
    if (d != 0) return hipErrorInvalidDevice;
    std::memset(p, 0, sizeof *p);
    std::strcpy(p->name, "host stand-in");
    p->multiProcessorCount = 8;
    p->sharedMemPerBlock = 160 * 1024;
    return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t *free_b, size_t *total_b)
{
    *free_b = (size_t)4 << 30;
    *total_b = (size_t)8 << 30;
    return hipSuccess;
}
inline hipError_t hipMalloc(void **p, size_t n)
{
    const long k = ++fakehip::malloc_calls;
    const long limit = fakehip::fail_after.load();
    if (limit >= 0 && k > limit) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    *p = std::calloc(n ? n : 1, 1);
    if (!*p) return hipErrorOutOfMemory;
    ++fakehip::live_blocks;
    return hipSuccess;
}
inline hipError_t hipFree(void *p)
{
    if (p) {
        --fakehip::live_blocks;
        std::free(p);
    }
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind)
{
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t)
{
    return hipMemcpy(dst, src, n, k);
}
inline hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t)
{
    if (n) std::memset(dst, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamCreate(hipStream_t *s)
{
    *s = new fake_stream{1};
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new fake_event{std::chrono::steady_clock::now()};
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    e->t = std::chrono::steady_clock::now();
    return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
