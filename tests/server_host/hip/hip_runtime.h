// CPU stand-in for the few HIP runtime calls the serving loop's host code
// makes, so that code can be built with the host compiler and run under
// ThreadSanitizer / AddressSanitizer with a fake engine (no GPU, no kernels).
// Streams are plain tokens; pool allocations are malloc/free.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdlib>

#define __host__
#define __device__
#define __global__
#define __shared__

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipMemPool_t* hipMemPool_t;
enum { hipStreamNonBlocking = 1 };
enum hipMemAllocationType { hipMemAllocationTypePinned = 1 };
enum hipMemAllocationHandleType { hipMemHandleTypeNone = 0 };
enum hipMemLocationType { hipMemLocationTypeDevice = 1 };
enum hipMemPoolAttr { hipMemPoolAttrReleaseThreshold = 4 };
struct hipMemLocation {
  hipMemLocationType type;
  int id;
};
struct hipMemPoolProps {
  hipMemAllocationType allocType;
  hipMemAllocationHandleType handleTypes;
  hipMemLocation location;
};

inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char[1]);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete[] reinterpret_cast<char*>(s);
  return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  *free_b = size_t(1) << 30;
  *total_b = size_t(1) << 31;
  return hipSuccess;
}
inline hipError_t hipMemPoolCreate(hipMemPool_t* p, const hipMemPoolProps*) {
  *p = reinterpret_cast<hipMemPool_t>(new char[1]);
  return hipSuccess;
}
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return hipSuccess; }
inline hipError_t hipMemPoolDestroy(hipMemPool_t p) {
  delete[] reinterpret_cast<char*>(p);
  return hipSuccess;
}
inline hipError_t hipMallocFromPoolAsync(void** ptr, size_t bytes, hipMemPool_t, hipStream_t) {
  *ptr = std::malloc(bytes ? bytes : 1);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFreeAsync(void* ptr, hipStream_t) {
  std::free(ptr);
  return hipSuccess;
}
