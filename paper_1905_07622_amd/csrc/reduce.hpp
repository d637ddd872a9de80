// Deterministic FP64 reductions for wave64 blocks and the device-side scalar
// updates of Algorithm 1 (VVM_A/VVM_reduce/VVM_C, Beta_update of App. A.2,
// done here in one pass: block partials, then the last block to arrive sums
// them in block order and updates the solve's scalars on the device).
#pragma once

#include "common.hpp"

namespace femheat {

// Sum over the block; the result is valid in thread 0.  blockDim.x must be a
// multiple of 64 and at most 1024.  Deterministic: fixed shuffle tree, then
// waves summed in order.
__device__ inline double block_sum(double v, double* wsum) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wsum[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) s += wsum[w];
  }
  __syncthreads();
  return s;
}

__device__ inline void finalize_scalars(int32_t fin, Scalars* S, double s, const Ctl& c) {
  switch (fin) {
    case FIN_RHS:
      S->delta_b = s;
      S->zero_rhs = (c.stop_rule == 0 && s == 0.0) ? 1 : 0;
      break;
    case FIN_INIT: {
      S->delta = s;
      S->delta0 = s;
      S->delta_old = s;
      S->beta = 0.0;
      S->iter = 0;
      S->status = 0;
      const double tol = c.stop_rule == 1 ? c.rtol2 * s : c.rtol2 * S->delta_b;
      S->tol = tol;
      if (!isfinite(s)) {
        S->status = kStatusBreakdown;
        S->done = 1;
      } else {
        S->done = (c.max_iter <= 0 || !(s > tol)) ? 1 : 0;
      }
    } break;
    case FIN_ALPHA: {
      S->dq = s;
      const double a = S->delta / s;
      if (!(s > 0.0) || !isfinite(s) || !isfinite(a)) {
        S->status = kStatusBreakdown;
        S->done = 1;
      } else {
        S->alpha = a;
      }
    } break;
    case FIN_DELTA: {
      const double old = S->delta;  // delta_old <- delta_new before the new value
      S->delta_old = old;
      S->delta = s;
      S->beta = s / old;
      S->iter += 1;
      if (!isfinite(s)) {
        S->status = kStatusBreakdown;
        S->done = 1;
      } else {
        S->done = (!(s > S->tol) || S->iter >= c.max_iter) ? 1 : 0;
      }
    } break;
    case FIN_CHECK:
      S->delta = s;
      if (!isfinite(s)) {
        S->status = kStatusBreakdown;
        S->done = 1;
      } else {
        S->done = !(s > S->tol) ? 1 : 0;
      }
      break;
    case FIN_STORE:
      S->aux = s;
      break;
    default:
      break;
  }
}

// Publish this block's partial; the last block to arrive sums all partials in
// block order and runs the finalisation.  Every thread of every block must
// call it (uniform control flow).
__device__ inline void reduce_and_finalize(double v, double* partials, Scalars* S, uint32_t nblocks,
                                           uint32_t block, int32_t fin, const Ctl& c) {
  __shared__ double wsum[16];
  __shared__ int am_last;
  const double bs = block_sum(v, wsum);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&partials[block], bs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t t = __hip_atomic_fetch_add(&S->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!am_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double s = 0.0;
  for (uint32_t k = threadIdx.x; k < nblocks; k += blockDim.x)
    s += __hip_atomic_load(&partials[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s = block_sum(s, wsum);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&S->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    finalize_scalars(fin, S, s, c);
  }
}

}  // namespace femheat
