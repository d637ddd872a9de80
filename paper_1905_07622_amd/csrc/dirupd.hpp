// One PCG iteration of one simulation in one kernel (gfx950): the
// search-direction gather with q = A d and d^T q, a grid-wide
// barrier, then alpha and the x/r update with r^T P^-1 r (Algorithm 1).
//
// Algorithm 1 needs the whole d^T q before any r can be updated, so the two
// halves normally run as two kernels (gather_batch_kernel with RoleDir, then
// update_batch_kernel).  Here every block of the gather stays resident (the
// launch checks that they all fit at once), publishes its d^T q partial to a
// place every XCD reads coherently, and waits at a barrier for all the
// others; each block then sums the partials in the canonical order (every
// block gets the same alpha, bit for bit) and updates r (and, for FP32 inner
// solves, x) at its own nodes.  During the march each block keeps, at its
// own nodes, q, r and P^-1 (and d and x in FP32) in LDS: r, P^-1 and x come
// from the epilogue's early fetch, which finds them in L2 (the march loaded
// the same planes a few layers before), so after the barrier the update only
// writes.  What this saves is one launch per iteration, the update kernel's
// start-up and tail, and its HBM traffic except the writes.  The arithmetic
// of every step is the one of the two kernels (only the r^T P^-1 r partials
// are summed per gather block instead of per update block).
#pragma once

#include "batch.hpp"

namespace femheat {

// The grid-wide barrier.  Every block adds its arrival to `count`; the block
// whose arrival completes the launch (count reaches `target`) writes
// `target` into every block's flag, and the other blocks each poll their own
// flag.  (All blocks polling the counter itself would put every poll on one
// memory channel: measured, that slowed the march of the blocks still
// gathering by half and the barrier by microseconds.)  `count` and the flags
// only grow (target = the arrivals of every earlier launch plus this grid),
// so nothing is reset between launches.  A wait that runs out after
// `spin_limit` polls (all blocks of the launch are resident, so it should
// not) sets `fail`, and the blocks leave without the update: the host stops
// the run at the end of the chunk and reports it as failed.
struct GridBar {
  unsigned long long* count;
  unsigned long long* flags;  // one per block, kBarFlagStride apart
  int32_t* fail;
  unsigned long long target;
  uint32_t spin_limit;
};

constexpr uint32_t kBarSpinLimit = 1u << 20;  // about a second of polls
constexpr uint32_t kBarFlagStride = 16;  // 128 bytes: one flag per cache line

// Keeps, at the block's own nodes, q (and r, P^-1, and in FP32 also d and x)
// in LDS: arrays [plane within the z-chunk][thread], `nk` planes each.
template <typename V>
struct EpiQKeep {
  static constexpr bool kKeeps = true;
  const V* r;
  const V* pinv;
  const V* x;  // FP32 inner solves; nullptr in FP64
  V* lds;
  int plane;   // elements per array (TZ * blockDim.x)
  struct Raw {
    V r, p, x;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(r, i), gld(pinv, i), x ? gld(x, i) : V(0)}; }
  __device__ double keep(int zl, V acc, V v, bool live, const Raw& w) const {
    const int li = zl * (int)blockDim.x + (int)threadIdx.x;
    lds[li] = acc;
    lds[plane + li] = w.r;
    lds[2 * plane + li] = w.p;
    if (x) {
      lds[3 * plane + li] = v;
      lds[4 * plane + li] = w.x;
    }
    return live ? (double)v * (double)acc : 0.0;
  }
};

// canonical_sum of partials that other XCDs wrote in this kernel: the same
// order, with loads at device scope (past the per-XCD caches).
__device__ inline double canonical_sum_device(const double* p, uint32_t n, double* red4) {
  const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (uint32_t vw = wid; vw < 4; vw += nw) {
    const uint32_t slot = vw * 64 + lane;
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t k = slot + 256u * u;
      v[u] = k < n ? __hip_atomic_load(p + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
    }
    double s = v[0];
#pragma unroll
    for (int u = 1; u < 8; ++u) s += v[u];
    for (uint32_t k = slot + 2048u; k < n; k += 256u) s += __hip_atomic_load(p + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red4[vw] = s;
  }
  __syncthreads();
  return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// Every block arrives once per launch; returns false in every thread if the
// wait ran out.  The only data that crosses blocks (and XCDs) here is the
// d^T q partials, written and read as device-scope atomics (past the
// per-XCD caches).  Thread 0 waits for its partial's store to complete
// before it adds its arrival (a release at device scope would also write
// back its XCD's whole L2, measured at 14 us per launch); the last arrival
// sees every other one, so every partial is complete before any flag is
// set, and the waiting side reads its flag and then the partials with
// device-scope loads, issued after the flag has been seen.  (The waiting
// side takes no acquire fence: that would drop the whole L2 of its XCD,
// which other blocks there are still marching through.)
__device__ inline bool grid_barrier(const GridBar& gb) {
  __shared__ int ok, last;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned long long before = __hip_atomic_fetch_add(gb.count, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = before + 1ull == gb.target;
  }
  __syncthreads();
  if (last) {
    for (uint32_t k = threadIdx.x; k < gridDim.x; k += blockDim.x)
      __hip_atomic_store(gb.flags + kBarFlagStride * k, gb.target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) ok = 1;
  } else if (threadIdx.x == 0) {
    int good = 1;
    uint32_t spins = 0;
    while (__hip_atomic_load(gb.flags + kBarFlagStride * blockIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gb.target) {
      if (++spins > gb.spin_limit) {
        __hip_atomic_store(gb.fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);  // host memory
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// The update half's outputs (the relay of the update: it writes the state
// and partials the next kernel reads).
template <typename V>
struct UpdHalf {
  V* r;
  V* x;               // FP32 inner solves: x += alpha d here; nullptr in FP64 (deferred to the next gather)
  Scalars* sout;      // state after the update (the next kernel's Sin)
  double* pout;       // r^T P^-1 r partials, one per gather block
};

template <int KIND, typename V>
__global__ void __launch_bounds__(kMaxBlockThreads)
    dirupd_kernel(GatherArgs<V> ga, ProDirection<V> pro, Relay R, UpdHalf<V> u, const V* pinv, GridBar gb,
                  uint32_t lds_base) {
  const uint32_t logical = xcd_work_item(blockIdx.x, gridDim.x);
  extern __shared__ unsigned char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw + lds_base);
  const int plane = ga.s.tz * (int)blockDim.x;
  TileOut to;
  Relay Rg = R;
  Rg.pout = nullptr;  // the d^T q partial goes out below, at device scope
  gather_tile<V, KIND>(ga, pro, EpiQKeep<V>{u.r, pinv, u.x, lds, plane}, Rg, logical, &to);
  __shared__ double wsum[16];
  const double bs = block_sum(to.dot, wsum);
  if (threadIdx.x == 0) __hip_atomic_store(R.pout + logical, bs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!grid_barrier(gb)) return;
  Scalars t = to.st;
  if (!to.settled || t.done) {  // uniform: a solve that is finished (or finished in this evaluation)
    // the kernels after this one read the state where this one read it: the
    // finished state goes there too (else the next kernel would evaluate the
    // same pending update again, and apply its deferred x += alpha d twice)
    if (logical == 0 && threadIdx.x == 0) gst_at(u.sout, t);
    return;
  }
  __shared__ double red4[4];
  const double dq = canonical_sum_device(R.pout, gridDim.x, red4);
  const bool go = settle_update(t, dq);
  double acc = 0.0;
  if (go && logical < ga.s.ntiles) {
    // the block's own nodes: column (gx, gy), planes z0 .. z1-1
    uint32_t b = logical;
    const int tz = (int)(b % (uint32_t)ga.s.ntz);
    b /= (uint32_t)ga.s.ntz;
    const int txi = (int)(b % (uint32_t)ga.s.ntx);
    const int tyi = (int)(b / (uint32_t)ga.s.ntx);
    const int th = threadIdx.x;
    const int gx = txi * ga.s.tx + th % ga.s.tx, gy = tyi * ga.s.ty + th / ga.s.tx;
    const int z0 = tz * ga.s.tz, z1 = min(z0 + ga.s.tz, ga.g.pz);
    if (th < ga.s.tx * ga.s.ty && gx < ga.g.px && gy < ga.g.py) {
      const uint32_t pstride = (uint32_t)ga.g.px * (uint32_t)ga.g.py;
      const uint32_t col_xy = (uint32_t)gx + (uint32_t)ga.g.px * (uint32_t)gy;
      const V alpha = (V)t.alpha;
      for (int z = z0; z < z1; ++z) {
        const uint32_t i = col_xy + pstride * (uint32_t)z;
        const int li = (z - z0) * (int)blockDim.x + th;
        V rr = lds[plane + li];
        upd1(rr, lds[li], lds[2 * plane + li], alpha, acc);
        gst(u.r, i, rr);
        if (u.x) gst(u.x, i, fma(alpha, lds[3 * plane + li], lds[4 * plane + li]));
      }
    }
  }
  const double ub = block_sum(acc, wsum);
  if (threadIdx.x == 0) {
    if (go) gst(u.pout, logical, ub);
    if (logical == 0) gst_at(u.sout, t);
  }
}

}  // namespace femheat
