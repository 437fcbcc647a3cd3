// CPU stand-in for the half-precision type (declarations only); see
// hip_runtime.h in this folder.  TEST INFRASTRUCTURE ONLY.
#pragma once
#include <stdint.h>
struct __half { uint16_t bits; };
__device__ float __half2float(__half);
__device__ __half __float2half_rn(float);
__device__ __half __ushort_as_half(unsigned short);
__device__ unsigned short __half_as_ushort(__half);
