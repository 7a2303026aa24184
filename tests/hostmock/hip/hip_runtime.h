// A host-only stand-in for the HIP runtime header, so that the library's host sources (api.cpp,
// autotune.cpp, ligand_prep.cpp, schedule.cpp, server.cpp) compile with g++ and run under the
// host sanitizers without a GPU.  Test infrastructure: "device" memory is host memory, streams
// run their work in the calling thread, capture records launches into a replayable list, and
// the kernel launchers are replaced by the host emulation in mock_runtime.cpp.  Only the calls
// the host sources make are declared.
#pragma once

#include <cstddef>
#include <cstdint>

#define __host__
#define __device__

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorStreamCaptureUnjoined = 904,
  hipErrorUnknown = 999
} hipError_t;

typedef struct MockStream* hipStream_t;
typedef struct MockEvent* hipEvent_t;
typedef struct MockGraph* hipGraph_t;
typedef struct MockGraphExec* hipGraphExec_t;

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

#define hipStreamDefault 0u
#define hipStreamNonBlocking 1u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u

struct alignas(8) int2 {
  int x, y;
};
struct alignas(16) float4 {
  float x, y, z, w;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipDeviceSynchronize();
const char* hipGetErrorString(hipError_t e);

hipError_t hipMalloc(void** p, size_t bytes);
template <class T>
hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
hipError_t hipFree(void* p);
hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t s);
hipError_t hipFreeAsync(void* p, hipStream_t s);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags = 0);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, void* error_node, char* log, size_t log_size);
hipError_t hipGraphDestroy(hipGraph_t graph);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
