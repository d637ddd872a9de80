// Device-side control of Algorithm 1 without atomics or cross-block fences.
//
// The VVM_A / VVM_reduce / VVM_C / Beta_update kernels of App. A.2 become:
//  * every kernel that produces a dot product writes one FP64 partial per
//    block (plain stores);
//  * the NEXT kernel in stream order reads those partials at its start,
//    together with the relayed state (one memory round trip), sums them in
//    one fixed order (so every block obtains the bit-identical value),
//    evaluates the pending scalar update of Algorithm 1 (alpha, or
//    delta/beta and the stop test) and broadcasts it to the block;
//  * the solve state is relayed through a ping-pong pair of Scalars: a kernel
//    reads Sin and one block of the solve (its tile 0) writes the updated
//    state to Sout, so no block ever reads a value another block of the same
//    kernel writes.
// A kernel may serve many independent solves at once (batched launches):
// each block belongs to one solve and sees only that solve's Relay, and the
// partial of a block is stored at its index within its solve, so a solve's
// reductions do not depend on what else shares the launch.
// Kernel boundaries order everything (stream order makes a kernel's writes
// visible to the next one on every XCD), which is why no atomics are needed.
// Once a solve is done, every further iteration kernel copies the state and
// returns immediately.
#pragma once

#include "common.hpp"
#include "gmem.hpp"

namespace femheat {

struct Relay {
  const Scalars* sin;
  Scalars* sout;
  const double* pin;   // partials of the previous kernel of this solve
  uint32_t npin;
  double* pout;        // this kernel's partials (one per block), or nullptr
  int32_t mode;
  Ctl ctl;
  uint32_t ld;         // distance between the components of multi-valued partials
  int32_t next_xc;     // M_RHS_NEXT: iterate buffer the launch assumed (replacements mod 2)
  int32_t next_R;      //             replacement period (< 0: refinement sweep, no buffer test)
};

// Sum of n partials in one canonical order that does not depend on the block
// size: 256 slots (slot j adds partials j, j+256, j+512, ... in sequence),
// grouped in 4 virtual waves of 64 reduced by an xor-shuffle tree, then the 4
// wave sums added in order.  Real wave w handles virtual waves w, w+nw, ...
// All threads of the block must call it; every thread gets the same value.
__device__ inline double canonical_sum(const double* p, uint32_t n, double* red4) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (uint32_t vw = wid; vw < 4; vw += nw) {
    const uint32_t slot = vw * 64 + lane;
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t k = slot + 256u * u;
      v[u] = k < n ? gld(p, k) : 0.0;
    }
    double s = v[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) s += v[u];
    for (uint32_t k = slot + 2048u; k < n; k += 256u) s += gld(p, k);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red4[vw] = s;
  }
  __syncthreads();
  return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// canonical_sum with each thread's first 8 partials already loaded (v, by
// waves 0..3: blocks of at least 4 waves): the same order, so the same value.
__device__ inline double canonical_sum_pre(const double* p, uint32_t n, const double* v, double* red4) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
  if (wid < 4) {
    const uint32_t slot = wid * 64 + lane;
    double s = v[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) s += v[u];
    for (uint32_t k = slot + 2048u; k < n; k += 256u) s += gld(p, k);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red4[wid] = s;
  }
  __syncthreads();
  return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// Four canonical sums at once (components c at p + c*ld), in the order of
// canonical_sum, with every load issued before the first reduction.
__device__ inline void canonical_sum4(const double* p, uint32_t ld, uint32_t n, double* out, double* red16) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (uint32_t vw = wid; vw < 4; vw += nw) {
    const uint32_t slot = vw * 64 + lane;
    double v[4][8];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t k = slot + 256u * u;
        v[c][u] = k < n ? femheat::gld(p, c * ld + k) : 0.0;
      }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double s = v[c][0];
#pragma unroll
      for (int u = 1; u < 8; ++u) s += v[c][u];
      for (uint32_t k = slot + 2048u; k < n; k += 256u) s += femheat::gld(p, c * ld + k);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) red16[c * 4 + vw] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = ((red16[c * 4 + 0] + red16[c * 4 + 1]) + red16[c * 4 + 2]) + red16[c * 4 + 3];
}

// Sum over the block (blockDim.x a multiple of 64, at most 1024); valid in thread 0.
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

// The scalar update that the previous kernel's partial sums x complete
// (x[0] only, except after a one-reduction direction kernel: x[0..3]).
__device__ inline void evaluate_pending(Scalars& s, const double* xs, const Ctl& c) {
  const double x = xs[0];
  switch (s.phase) {
    case PH_AFTER_INIT: {  // r0^T P^-1 r0: tolerance and the test before the first iteration
      // (rtol2 < 0: the squared tolerance came with the state, in tol, from
      // the kernel that started the solve)
      const double rt2 = c.rtol2 < 0.0 ? s.tol : c.rtol2;
      s.delta = x;
      s.delta0 = x;
      s.delta_old = x;
      s.beta = 0.0;
      s.iter = 0;
      s.tol = c.stop_rule == 1 ? rt2 * x : rt2 * s.delta_b;
      if (!isfinite(x)) {
        s.status = kStatusBreakdown;
        s.done = 1;
      } else {
        s.done = (c.max_iter <= 0 || !(x > s.tol)) ? 1 : 0;
      }
    } break;
    case PH_AFTER_UPD: {  // delta_new = r^T P^-1 r: beta and the stop test
      const double old = s.delta;  // delta_old <- delta_new before the new value
      s.delta_old = old;
      s.delta = x;
      s.beta = x / old;
      if (!isfinite(x)) {
        s.status = kStatusBreakdown;
        s.done = 1;
      } else {
        s.done = (!(x > s.tol) || s.iter >= c.max_iter) ? 1 : 0;
      }
    } break;
    case PH_AFTER_CHECK:  // FP64 residual of a refinement sweep
      s.delta = x;
      if (!isfinite(x)) {
        s.status = kStatusBreakdown;
        s.done = 1;
      } else {
        s.done = !(x > s.tol) ? 1 : 0;
      }
      break;
    case PH_AFTER_FUSED: {
      // One-reduction form.  The direction kernel that produced these sums
      // also advanced r (when `fresh`): its r^T P^-1 r is Algorithm 1's
      // delta_new, and the stop test is taken on it exactly as there.  If the
      // solve goes on, alpha = delta / d^T q is Algorithm 1's, the next update
      // is counted, and the next beta comes from the delta that update will
      // produce, r'^T P^-1 r' = delta - 2 alpha q^T P^-1 r + alpha^2 q^T P^-1 q
      // (restarted from the directly summed delta every iteration).
      const double gq = xs[0], mu = xs[1], nu = xs[2];
      if (s.fresh) {
        s.delta_old = s.delta;
        s.delta = xs[3];
      }
      s.dq = gq;
      s.mu = mu;
      s.nu = nu;
      if (!isfinite(s.delta)) {
        s.status = kStatusBreakdown;
        s.done = 1;
      } else if (!(s.delta > s.tol) || s.iter >= c.max_iter) {
        s.done = 1;
      } else {
        const double a = s.delta / gq;
        if (!(gq > 0.0) || !isfinite(gq) || !isfinite(a)) {
          s.status = kStatusBreakdown;
          s.done = 1;
        } else {
          s.alpha = a;
          s.iter += 1;
          const double next = (s.delta - 2.0 * a * mu) + (a * a) * nu;
          s.beta = next / s.delta;
        }
      }
    } break;
    default:
      break;
  }
  s.phase = PH_DECIDED;
}

__device__ inline bool is_fused_mode(int32_t m) { return m == M_FDIR || m == M_FUPD || m == M_FREPL; }

// The scalar step of the x/r update (Algorithm 1's alpha = delta / d^T q),
// given x = d^T q; returns whether the update has work.
__device__ inline bool settle_update(Scalars& t, double x) {
  if (t.done) return false;
  const double a = t.delta / x;
  t.dq = x;
  if (!(x > 0.0) || !isfinite(x) || !isfinite(a)) {
    t.status = kStatusBreakdown;
    t.done = 1;
    return false;
  }
  t.alpha = a;
  t.iter += 1;
  t.phase = PH_AFTER_UPD;
  return true;
}

// The relayed state as a kernel finds it, before the pending update.
struct StageIn {
  Scalars t;
  bool pending;  // the previous kernel's partials complete a scalar update
  bool need;     // this kernel sums those partials
  bool pre;      // pv holds this thread's first partials (blocks of >= 4 waves)
  double pv[8];
};

// First half of a relayed kernel's entry: reads the state (one uniform load).
// Kernels can issue their first global loads after it and before
// stage_finish, whose partial sum then overlaps them.
template <bool kPre = false>
__device__ inline StageIn stage_load(const Relay& R) {
  StageIn in;
  // kPre: the partials are read together with the state (before it is known
  // whether they are needed: a wasted read costs less than a second memory
  // round trip), in canonical_sum's slot order: wave w < 4 holds virtual
  // wave w.  It costs registers, so only the FP64 kernels do it (the FP32
  // inner solves run in batches, where occupancy matters more).
  in.pre = kPre && (blockDim.x >> 6) >= 4 && R.pin != nullptr;  // uniform
  if (in.pre) {
    const uint32_t slot = threadIdx.x;  // only waves 0..3 use theirs
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t k = slot + 256u * u;
      in.pv[u] = (slot < 256u && k < R.npin) ? gld(R.pin, k) : 0.0;
    }
  }
  in.t = Scalars{};
  if (R.sin) in.t = gld_at(R.sin);
  in.pending = !in.t.done && in.t.phase != PH_DECIDED && in.t.phase != PH_NONE;
  in.need = R.mode == M_INIT || R.mode == M_INIT_NEXT || (R.mode == M_UPD && !in.t.done) ||
            ((R.mode == M_DIR || R.mode == M_DECIDE || is_fused_mode(R.mode)) && in.pending);
  return in;
}

// A search-direction or update kernel of a finished solve has no work and
// leaves the state unchanged: only the writer relays it.  Uniform.
__device__ inline bool stage_idle(const Relay& R, const StageIn& in, bool writer) {
  if ((R.mode == M_DIR || R.mode == M_UPD || R.mode == M_PASS || is_fused_mode(R.mode)) && in.t.done) {
    if (writer && threadIdx.x == 0 && R.sout) gst_at(R.sout, in.t);
    return true;
  }
  return false;
}

// Second half: sums the partials if needed, evaluates the state this kernel
// works with, has the writer block publish it to Sout, and returns whether
// the kernel has work.  Called by all threads of the block.  kFour: the
// kernel may follow a one-reduction direction kernel and sum its four
// partials (only those kernels carry that code: it needs many registers).
template <bool kFour = false>
__device__ inline bool stage_finish(const Relay& R, const StageIn& in, Scalars& out, bool writer) {
  __shared__ Scalars sh;
  __shared__ int go;
  __shared__ double red16[16];
  Scalars t = in.t;
  const bool pending = in.pending;
  double xs[4] = {0.0, 0.0, 0.0, 0.0};
  if (in.need) {  // uniform
    bool four = false;
    if constexpr (kFour) {
      four = pending && in.t.phase == PH_AFTER_FUSED;
      if (four) canonical_sum4(R.pin, R.ld, R.npin, xs, red16);
    }
    if (four) {
    } else if (in.pre)
      xs[0] = canonical_sum_pre(R.pin, R.npin, in.pv, red16);
    else
      xs[0] = canonical_sum(R.pin, R.npin, red16);
  }
  const double x = xs[0];
  if (threadIdx.x == 0) {
    int g = 1;
    int mode = R.mode;
    if (mode == M_RHS_NEXT) {
      // the solve must have ended without breakdown, with its iterate in the
      // buffer the launch assumed; otherwise the state passes unchanged
      // (next_R < 0: a refinement sweep's correction, whose buffer is known)
      const int xc = (R.next_R <= 0 || t.iter <= 0) ? 0 : ((t.iter - 1) / R.next_R + 1) & 1;
      mode = (t.done && t.status == 0 && (R.next_R < 0 || xc == R.next_xc)) ? M_RHS : M_SKIP;
    } else if (mode == M_INIT_NEXT) {
      mode = (t.phase == PH_NONE && !t.done) ? M_INIT : M_SKIP;  // the M_RHS_NEXT before it ran
    }
    switch (mode) {
      case M_RHS:  // a new step: b and b^T P^-1 b
        t.done = 0;
        t.status = 0;
        t.phase = PH_NONE;
        break;
      case M_INIT:  // b^T P^-1 b known: the guess prologue needs the zero-RHS flag
        t.delta_b = x;
        t.zero_rhs = (R.ctl.stop_rule == 0 && x == 0.0) ? 1 : 0;
        t.done = 0;
        t.status = 0;
        t.phase = PH_AFTER_INIT;
        break;
      case M_START:  // a solve whose initial residual this kernel produces
        t.done = 0;
        t.status = 0;
        t.delta_b = 0.0;
        t.zero_rhs = 0;
        t.tol = R.ctl.rtol2;  // its squared tolerance, for a Ctl that defers it (rtol2 < 0)
        t.phase = PH_AFTER_INIT;
        break;
      case M_DIR:
      case M_DECIDE:
        if (pending) evaluate_pending(t, xs, R.ctl);
        g = (R.mode == M_DIR && !t.done) ? 1 : 0;
        break;
      case M_FDIR:
      case M_FUPD:  // one-reduction direction kernel: publishes the four sums
        if (pending) evaluate_pending(t, xs, R.ctl);
        g = t.done ? 0 : 1;
        if (g) {
          t.phase = PH_AFTER_FUSED;
          t.fresh = R.mode == M_FUPD ? 1 : 0;
        }
        break;
      case M_FREPL:  // one-reduction residual replacement: publishes r^T P^-1 r
        if (pending) evaluate_pending(t, xs, R.ctl);
        g = t.done ? 0 : 1;
        if (g) t.phase = PH_AFTER_UPD;
        break;
      case M_UPD:
        g = settle_update(t, x) ? 1 : 0;
        break;
      case M_CORR:
        t.phase = PH_AFTER_CHECK;
        g = t.done ? 0 : 1;
        break;
      case M_SKIP:
        g = 0;
        break;
      case M_PASS:  // state unchanged (done solves returned in stage_idle)
        g = 1;
        break;
      case M_IDLE:  // settled: done with zero iterations, nothing pending
        t.done = 1;
        t.status = 0;
        t.iter = 0;
        t.phase = PH_DECIDED;
        g = 0;
        break;
      default:  // M_NONE
        break;
    }
    sh = t;
    go = g;
    if (writer && R.sout) gst_at(R.sout, t);
  }
  __syncthreads();
  out = sh;
  return go != 0;
}

// Entry of a relayed kernel in one piece.
__device__ inline bool stage_entry(const Relay& R, Scalars& out, bool writer) {
  const StageIn in = stage_load(R);
  return stage_finish(R, in, out, writer);
}

// One partial per block for the next kernel, at the block's index `slot`
// within its solve.
__device__ inline void publish_partial(const Relay& R, double v, uint32_t slot) {
  __shared__ double wsum[16];
  const double bs = block_sum(v, wsum);
  if (threadIdx.x == 0 && R.pout) gst(R.pout, slot, bs);
}

// Four partials per block (component c at pout[c*ld + slot]), each summed in
// the order of block_sum.
__device__ inline void publish_partial4(const Relay& R, const double* v, uint32_t slot) {
  __shared__ double wsum4[4][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double x = v[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) wsum4[c][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < 4 && R.pout) {
    const int c = threadIdx.x, nw = blockDim.x >> 6;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += wsum4[c][w];
    gst(R.pout, c * R.ld + slot, s);
  }
}

}  // namespace femheat
