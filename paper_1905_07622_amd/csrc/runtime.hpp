// Host helpers shared by the set-up code and the time-stepping engine.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "gather.hpp"
#include "solver.hpp"

namespace femheat {

constexpr int kT = 256;  // threads of the 1-D kernels

inline int fail(fem_heat* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      (void)hipGetLastError();                                                            \
      return fail(h, FEM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    }                                                                                     \
  } while (0)

#define RC_TRY(expr)               \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != FEM_OK) return rc_; \
  } while (0)

// Device memory: through a caller's allocator (stream-ordered on `s`) when
// one is given, else hipMalloc / hipFree (hipFree synchronises the device).
inline bool dev_alloc(const fem_allocator* a, hipStream_t s, void** p, size_t bytes) {
  *p = nullptr;
  if (a && a->alloc) return a->alloc(a->ctx, p, bytes, s) == 0 && *p != nullptr;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}
inline void dev_free(const fem_allocator* a, hipStream_t s, void* p) {
  if (!p) return;
  if (a && a->release)
    a->release(a->ctx, p, s);
  else
    (void)hipFree(p);
}

// Buffers of a handle, on its stream and through its allocator.
template <typename T>
int dalloc(fem_heat* h, T** p, size_t n) {
  const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  void* v = nullptr;
  if (!dev_alloc(h->opts.allocator, h->stream, &v, bytes)) {
    *p = nullptr;
    return fail(h, FEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  *p = static_cast<T*>(v);
  return FEM_OK;
}

template <typename T>
void dfree(fem_heat* h, T*& p) {
  dev_free(h->opts.allocator, h->stream, p);
  p = nullptr;
}

inline uint32_t nblk(uint32_t n) { return (n + kT - 1) / kT; }

inline hipMemcpyKind in_kind(const fem_heat* h) {
  return h->devptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
inline hipMemcpyKind out_kind(const fem_heat* h) {
  return h->devptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

inline int copy_in(fem_heat* h, double* dst, const double* src, size_t n) {
  HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double), in_kind(h), h->stream));
  return FEM_OK;
}
inline int copy_out(fem_heat* h, void* dst, const void* src, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, out_kind(h), h->stream));
  return FEM_OK;
}

// Gather arguments of the operator cm*M + ck*K of a handle (FP64 or FP32
// coefficients; they must exist).
template <typename V>
GatherArgs<V> gather_args(const fem_heat* h, double cm, double ck);

// Jacobi preconditioner and Dirichlet lifting for stiffness scale
// ck = theta*dt (and the FP32 copies when need32); cached per ck.
int prepare_operator(fem_heat* h, double ck, bool need32);

}  // namespace femheat
