// CPU stand-in for the part of the HIP runtime API that the library's host
// code uses.  TEST INFRASTRUCTURE ONLY: it lets the host side of the library
// (lb_api.hip and the launch sequences of lb_kernels.hip, compiled host-only)
// run under AddressSanitizer and UndefinedBehaviorSanitizer on a machine
// without a GPU.  Kernels are not executed; device memory is host memory;
// streams, events and graphs are tracked objects whose misuse (use after
// destroy, unjoined forks in a capture, copies outside an allocation) aborts
// with a message.  Nothing in the solver includes this header.
#pragma once
#include <stddef.h>
#include <stdint.h>
// clang's own HIP wrapper: __host__/__device__ attributes and device math
#include <__clang_hip_runtime_wrapper.h>

#define __forceinline__ inline __attribute__((always_inline))
#define __launch_bounds__(...) __attribute__((amdgpu_flat_work_group_size(1, 1024)))
#define HIP_SYMBOL(x) (&(x))
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidResourceHandle = 400,
    hipErrorStreamCaptureUnsupported = 900,
    hipErrorStreamCaptureUnjoined = 904,
    hipErrorIllegalState = 401
} hipError_t;

typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
               hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;
typedef enum { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1,
               hipStreamCaptureStatusInvalidated = 2 } hipStreamCaptureStatus;

#define hipStreamDefault 0u
#define hipStreamNonBlocking 1u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u

typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct hipGraphExec *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;

extern "C" {
hipError_t hipMalloc(void **p, size_t n);
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t s);
hipError_t hipDeviceSynchronize(void);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus *st);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *en, char *log,
                               size_t n);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGetLastError(void);
hipError_t hipGetSymbolAddress(void **p, const void *sym);
hipError_t hipGetDevice(int *d);
const char *hipGetErrorString(hipError_t e);
// kernel launch interface that clang's HIP mode emits for <<<...>>>
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t shm, hipStream_t s);
unsigned __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm = 0, hipStream_t s = 0);
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *shm, hipStream_t *s);
}

#if __HIP__
// device-side names the kernels use (declarations only: kernels are not
// compiled in the host-only build)
struct __hc_idx {
    __device__ unsigned get_x() const;
    __device__ unsigned get_y() const;
    __device__ unsigned get_z() const;
    __declspec(property(get = get_x)) unsigned x;
    __declspec(property(get = get_y)) unsigned y;
    __declspec(property(get = get_z)) unsigned z;
};
extern const __device__ __hc_idx threadIdx, blockIdx, blockDim, gridDim;
__device__ void __syncthreads();
__device__ int __syncthreads_or(int);
__device__ int __shfl(int, int, int = 64);
__device__ unsigned __shfl(unsigned, int, int = 64);
__device__ float __shfl(float, int, int = 64);
__device__ double __shfl(double, int, int = 64);
__device__ int __shfl_up(int, unsigned, int = 64);
__device__ int __shfl_xor(int, int, int = 64);
__device__ double __shfl_xor(double, int, int = 64);
__device__ float __shfl_xor(float, int, int = 64);
__device__ int atomicAdd(int *, int);
__device__ int atomicOr(int *, int);
__device__ unsigned atomicOr(unsigned *, unsigned);
__device__ int __popc(unsigned);
#endif
