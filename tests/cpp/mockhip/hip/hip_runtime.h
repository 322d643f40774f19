// A host-only stand-in for the HIP runtime header, used to build the
// library's scheduler (pd_host.cpp) with g++ and the sanitizers, without a
// GPU.  "Device memory" is host memory; every stream operation runs at once
// on the calling thread, unless a graph capture is open, in which case it is
// recorded and replayed by hipGraphLaunch.  Only what pd_host.cpp uses is
// declared; the definitions live in sched_mock.cpp.
#pragma once

#include <cstddef>
#include <cstdint>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorLaunchTimeOut = 702,
  hipErrorNotSupported = 801
} hipError_t;

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct hipGraphExec;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef ihipGraph* hipGraph_t;
typedef hipGraphExec* hipGraphExec_t;
struct hipGraphNode;
typedef hipGraphNode* hipGraphNode_t;

enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1 };
#define hipHostMallocDefault 0u
#define hipStreamNonBlocking 1u

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
};
extern thread_local dim3 blockIdx, threadIdx, gridDim, blockDim;

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
const char* hipGetErrorName(hipError_t e);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t* err, char* log, size_t n);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
