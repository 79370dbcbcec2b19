// A CPU stand-in for the part of the HIP runtime API that the library's host
// runtime (knnf_api.cpp, knnf_server.cpp) calls -- TEST INFRASTRUCTURE ONLY.
//
// The serving tests build those two product files against this header and
// against fake_device.cpp (the filtering launches, executed by the CPU
// oracle) so that admission, batching, ordering and failure handling can run
// under AddressSanitizer and ThreadSanitizer on a machine without a GPU.
// "Device" memory is host memory; a stream is a worker thread that runs its
// operations in order; an event completes when its stream reaches it.
#pragma once

#include <stddef.h>
#include <stdint.h>

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidDevice = 101,
    hipErrorNotReady = 600,
    hipErrorLaunchFailure = 719,
};

struct FakeStream;
struct FakeEvent;
typedef FakeStream* hipStream_t;
typedef FakeEvent* hipEvent_t;

typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum { hipMemoryTypeHost = 0, hipMemoryTypeDevice = 1 } hipMemoryType;

struct hipDeviceProp_t {
    char name[256];
    int multiProcessorCount;
};

struct hipPointerAttribute_t {
    hipMemoryType type;
    int device;
    void* devicePointer;
    void* hostPointer;
};

#define hipEventDefault 0u
#define hipEventDisableTiming 2u
#define hipStreamDefault 0u
#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u
#define hipHostMallocMapped 2u
#define hipHostMallocCoherent 0x40000000u

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetLastError(void);
hipError_t hipDeviceSynchronize(void);

hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned flags);
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemset(void* p, int v, size_t n);

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamQuery(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);

// ---- controls of the fake, for the tests ----------------------------------
#include <functional>
namespace fakehip {
// Run `op` on stream s in order (null stream: at once, on the calling thread).
hipError_t enqueue(hipStream_t s, std::function<void()> op);
// From now on, the n-th next hipMemcpyAsync (0 = the next one) fails.
void fail_copy_after(int n);
// Number of operations each stream has run (all streams together).
long ops_run();
}  // namespace fakehip
