// Host-only stand-in for the HIP runtime calls made by the library's host
// code, so that its table builder can be compiled with g++ and checked on a
// machine without a GPU.  "Device" memory is host memory; copies are memcpy.
#pragma once
#include <cstdint>
#include <cstdlib>
#include <cstring>

typedef int hipError_t;
typedef void *hipStream_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipHostMallocDefault = 0, hipHostMallocMapped = 2, hipHostMallocCoherent = 4 };
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)

inline const char *hipGetErrorString(hipError_t) { return "host stand-in"; }
template <typename T>
inline hipError_t hipMalloc(T **p, size_t n) {
    *p = static_cast<T *>(calloc(n ? n : 1, 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) {
    free(p);
    return hipSuccess;
}
template <typename T>
inline hipError_t hipHostMalloc(T **p, size_t n, unsigned = 0) {
    return hipMalloc(p, n);
}
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
template <typename T>
inline hipError_t hipHostGetDevicePointer(T **d, void *h, unsigned) {
    *d = static_cast<T *>(h);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, int, hipStream_t = nullptr) {
    memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemset(void *d, int v, size_t n) {
    memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *o, const void *, int, size_t) {
    *o = 2;
    return hipSuccess;
}
inline hipError_t hipLaunchKernel(const void *, dim3, dim3, void **, size_t, hipStream_t) { return hipSuccess; }
template <typename T>
inline T atomicAdd(T *p, T v) {
    T o = *p;
    *p += v;
    return o;
}
