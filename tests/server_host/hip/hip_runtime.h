// Host-only stand-in for the few HIP runtime calls the request server makes, so that its
// admission and lane threads can be tested on a CPU (tests/test_server_host.py).  Device
// memory is host memory, copies are immediate, and an event is "done" once recorded.  The
// stub can make the query of a chosen request's copy event report an error.
#pragma once
#include <stddef.h>
#include <stdint.h>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorUnknown = 999 };
typedef struct stub_event* hipEvent_t;
typedef struct stub_stream* hipStream_t;
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2

extern "C" {
hipError_t hipSetDevice(int);
hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipGetLastError(void);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, int kind, hipStream_t s);
}
