// Host runtime of the assembly-free theta-scheme heat solver on gfx950.
//
// One handle keeps the whole problem resident in HBM: coefficients, load
// vector, Jacobi preconditioner, the two previous fields and the PCG vectors.
// A run enqueues, per time step (Sec. 3.1): the right-hand side b = L T + dt*s*F
// (gather with the RHS epilogue), the initial guess and residual (gather with
// the guess prologue and residual epilogue), then the iterations of
// Algorithm 1, two kernels each: the search-direction update fused into the
// operator apply (q = A d, d^T q -> alpha on the device) and the fused x/r
// update with the preconditioned residual norm (delta, beta and the
// convergence test on the device).  Every 50th iteration (i mod 50 == 0, as
// printed) the update is replaced by a gather computing r = b - A x.
//
// The paper's host read the residual back every iteration (App. A.3).  Here
// the scalars of Algorithm 1 and the convergence decision live on the device
// and are relayed from kernel to kernel (reduce.hpp): once a solve is done
// every further iteration kernel returns immediately, so the host enqueues
// iterations in chunks, ends a chunk with a one-block decide kernel and reads
// a small pinned scalar block once per chunk, sizing the first chunk of a
// step from the previous step's iteration count.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gather.hpp"
#include "solver.hpp"
#include "vector_kernels.hpp"

namespace femheat {
namespace {

constexpr int kT = 256;  // threads of the 1-D kernels

int fail(fem_heat* h, int code, const std::string& msg) {
  h->err = msg;
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

#define RC_TRY(expr)           \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != FEM_OK) return rc_; \
  } while (0)

template <typename T>
int dalloc(fem_heat* h, T** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(h, FEM_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return FEM_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

uint32_t nblk(uint32_t n) { return (n + kT - 1) / kT; }

hipMemcpyKind in_kind(const fem_heat* h) { return h->devptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind out_kind(const fem_heat* h) { return h->devptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

int copy_in(fem_heat* h, double* dst, const double* src, size_t n) {
  HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double), in_kind(h), h->stream));
  return FEM_OK;
}
int copy_out(fem_heat* h, void* dst, const void* src, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, out_kind(h), h->stream));
  return FEM_OK;
}

// LDS row pitch (in values) of a tile of width `width`: the smallest pitch
// for which the 64 lanes of every wave, split into half-waves of 32 lanes,
// read 8-byte words in distinct banks (64 banks of 4 bytes) for each of the
// neighbourhood offsets the gather uses (3x3 for the plane, 2x2 for the
// coefficients).  Falls back to the width when no pitch within 64 is free.
int lds_pitch(int tx, int ty, int nthreads, int width, bool plane) {
  const int span = plane ? 3 : 2;
  for (int p = width; p < width + 64; ++p) {
    bool ok = true;
    for (int w = 0; w < nthreads / 64 && ok; ++w)
      for (int half = 0; half < 2 && ok; ++half)
        for (int dy = 0; dy < span && ok; ++dy)
          for (int dx = 0; dx < span && ok; ++dx) {
            bool used[32] = {false};
            for (int l = 0; l < 32; ++l) {
              const int t = w * 64 + half * 32 + l;
              const int lx = t < tx * ty ? t % tx : 0, ly = t < tx * ty ? t / tx : 0;
              if (t >= tx * ty) continue;
              const int slot = (((ly + dy) * p + lx + dx) % 32 + 32) % 32;
              if (used[slot]) {
                ok = false;
                break;
              }
              used[slot] = true;
            }
          }
    if (ok) return p;
  }
  return width;
}

// Blocks of the hot gather (search direction fused with the apply) that one
// CU holds at once for a block of `nthreads` threads: occupancy is bounded by
// the kernel's registers and LDS, so it is asked of the runtime.
int resident_blocks(bool cubic, bool fp32, int nthreads, size_t smem) {
  int n = 0;
  hipError_t e;
  if (fp32)
    e = cubic ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, reinterpret_cast<const void*>(&gather_kernel<float, true, ProDirection<float>, EpiQDot<float>>),
                    nthreads, smem)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, reinterpret_cast<const void*>(&gather_kernel<float, false, ProDirection<float>, EpiQDot<float>>),
                    nthreads, smem);
  else
    e = cubic ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, reinterpret_cast<const void*>(&gather_kernel<double, true, ProDirection<double>, EpiQDot<double>>),
                    nthreads, smem)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, reinterpret_cast<const void*>(&gather_kernel<double, false, ProDirection<double>, EpiQDot<double>>),
                    nthreads, smem);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 2;
  }
  return std::max(n, 1);
}

// Launch shape of the gather: TX spans the x-row of nodes in as few equal
// pieces of at most 64 as possible, TY fills the block to <= 256 threads.
// Unless given, TZ splits the columns into as many z-chunks as the chip holds
// blocks at once (`capacity`): the gather is latency-bound, so the launch
// should fill every CU to its occupancy limit in a single round -- a second,
// partial round of blocks costs a whole extra block time -- and longer
// z-marches pay the start-up of the plane pipeline less often.
GatherShape choose_shape(const Geom& g, const fem_opts& o, int capacity) {
  GatherShape s{};
  const int px = g.px, py = g.py, pz = g.pz;
  int tx = o.tile_x > 0 ? o.tile_x : (px + (px + 63) / 64 - 1) / ((px + 63) / 64);
  tx = std::max(1, std::min(tx, 256));
  int ty;
  if (o.tile_y > 0) {
    ty = o.tile_y;
  } else {
    const int tymax = std::max(1, 256 / tx);
    const int nty = (py + tymax - 1) / tymax;
    ty = (py + nty - 1) / nty;
  }
  ty = std::max(1, std::min(ty, 256 / tx));
  // every thread stages at most kSlots entries of the plane and coefficient tiles
  auto fits = [](int a, int b) {
    const int nt = ((a * b + 63) / 64) * 64;
    return (a + 2) * (b + 2) <= kSlots * nt && (a + 1) * (b + 1) <= kSlots * nt;
  };
  if (o.tile_y <= 0)
    while (ty > 1 && !fits(tx, ty)) --ty;
  s.tx = tx;
  s.ty = ty;
  s.ntx = (px + tx - 1) / tx;
  s.nty = (py + ty - 1) / ty;
  int tz;
  if (o.tile_z > 0) {
    tz = o.tile_z;
  } else {
    const int cols = s.ntx * s.nty;
    const int ntz_target = std::max(1, capacity / cols);
    tz = std::max(4, (pz + ntz_target - 1) / ntz_target);
  }
  tz = std::max(1, std::min(tz, pz));
  s.tz = tz;
  s.ntz = (pz + tz - 1) / tz;
  s.nthreads = ((tx * ty + 63) / 64) * 64;
  s.pw = lds_pitch(tx, ty, s.nthreads, tx + 2, true);
  s.cw = lds_pitch(tx, ty, s.nthreads, tx + 1, false);
  s.ntiles = (uint32_t)s.ntx * s.nty * s.ntz;
  s.nblocks = ((s.ntiles + 7) / 8) * 8;
  return s;
}

template <typename V>
void fill_classes(const Geom& g, GatherArgs<V>& ga, double cm, double ck, bool cubic) {
  if (cubic) {
    const double h = g.hx;
    ga.sa = (V)(cm * h * h * h / 216.0);
    ga.sb = (V)(ck * h / 12.0);
    for (int c = 0; c < 8; ++c) ga.Mc[c] = ga.Kc[c] = V(0);
    return;
  }
  // entry class c = a xor b (bit d set when the corners differ along axis d):
  // M[c] = prod_d m_d(c_d), K[c] = sum_d s_d(c_d) prod_{d' != d} m_d'(c_d'),
  // with 1-D entries m = h/3 (same), h/6 (differ) and s = 1/h, -1/h.
  const double h[3] = {g.hx, g.hy, g.hz};
  for (int c = 0; c < 8; ++c) {
    double m[3], st[3];
    for (int d = 0; d < 3; ++d) {
      const bool diff = (c >> d) & 1;
      m[d] = diff ? h[d] / 6.0 : h[d] / 3.0;
      st[d] = diff ? -1.0 / h[d] : 1.0 / h[d];
    }
    ga.Mc[c] = (V)(m[0] * m[1] * m[2]);
    ga.Kc[c] = (V)(st[0] * m[1] * m[2] + m[0] * st[1] * m[2] + m[0] * m[1] * st[2]);
  }
  ga.sa = (V)cm;
  ga.sb = (V)ck;
}

// Relay arguments of the next kernel of a solve: it reads the state and
// partials the previous kernel left and writes the other buffer of each pair.
Relay next_relay(RelayCtx& c, int32_t mode, bool partials, uint32_t grid) {
  Relay R{c.S[c.cur], c.S[c.cur ^ 1], c.P[c.cur], c.npin, partials ? c.P[c.cur ^ 1] : nullptr, mode, c.ctl};
  c.cur ^= 1;
  if (partials) c.npin = grid;
  return R;
}

Relay no_relay() { return Relay{nullptr, nullptr, nullptr, 0, nullptr, M_NONE, Ctl{0.0, 0, 0}}; }

template <typename V, class Pro, class Epi>
int launch_gather(fem_heat* h, const V* rhoc, const V* kc, double cm, double ck, Pro pro, Epi epi, const Relay& R) {
  GatherArgs<V> ga{};
  ga.g = h->g;
  ga.s = h->shape;
  ga.rhoc = rhoc;
  ga.kc = kc;
  ga.sink = reinterpret_cast<V*>(h->sink);
  fill_classes(h->g, ga, cm, ck, h->cubic);
  const size_t smem = h->shape.smem_bytes(sizeof(V));
  if (h->cubic)
    hipLaunchKernelGGL((gather_kernel<V, true, Pro, Epi>), dim3(h->shape.nblocks), dim3(h->shape.nthreads), smem,
                       h->stream, ga, pro, epi, R);
  else
    hipLaunchKernelGGL((gather_kernel<V, false, Pro, Epi>), dim3(h->shape.nblocks), dim3(h->shape.nthreads), smem,
                       h->stream, ga, pro, epi, R);
  HIP_TRY(hipGetLastError());
  return FEM_OK;
}

template <typename V, class Pro, class Epi>
int gather_step(fem_heat* h, RelayCtx& c, int32_t mode, const V* rhoc, const V* kc, double cm, double ck, Pro pro,
                Epi epi) {
  return launch_gather<V>(h, rhoc, kc, cm, ck, pro, epi, next_relay(c, mode, true, h->shape.nblocks));
}

// Settles the pending decision of a solve and copies its state to the host.
int decide_and_read(fem_heat* h, RelayCtx& c, Scalars* host) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(64), 0, h->stream, next_relay(c, M_DECIDE, false, 1));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host, c.S[c.cur], sizeof(Scalars), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FEM_OK;
}

int ensure_fp32(fem_heat* h) {
  if (h->pinv32) return FEM_OK;
  const uint32_t N = h->g.N, E = h->g.E;
  RC_TRY(dalloc(h, &h->rhoc32, E));
  RC_TRY(dalloc(h, &h->k32, E));
  RC_TRY(dalloc(h, &h->pinv32, N));
  RC_TRY(dalloc(h, &h->e32[0], N));
  RC_TRY(dalloc(h, &h->e32[1], N));
  RC_TRY(dalloc(h, &h->r32, N));
  RC_TRY(dalloc(h, &h->q32, N));
  RC_TRY(dalloc(h, &h->d32[0], N));
  RC_TRY(dalloc(h, &h->d32[1], N));
  RC_TRY(dalloc(h, &h->rhs32, N));
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(E)), dim3(kT), 0, h->stream, h->rhoc64, h->rhoc32, E);
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(E)), dim3(kT), 0, h->stream, h->k64, h->k32, E);
  HIP_TRY(hipGetLastError());
  h->ck_cached = -1.0;  // pinv32 must be (re)built
  return FEM_OK;
}

// Jacobi preconditioner (a0) and, for non-zero Dirichlet values, the lifting
// A_fD g, for the system matrix with stiffness scale ck = theta*dt.
int prepare_operator(fem_heat* h, double ck, bool need32) {
  if (need32) RC_TRY(ensure_fp32(h));
  if (h->ck_cached == ck && (!need32 || h->pinv32)) return FEM_OK;
  const uint32_t N = h->g.N;
  hipLaunchKernelGGL((jacobi_kernel<double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->g, h->rhoc64, h->k64, ck,
                     h->pinv64);
  if (h->pinv32)
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->pinv64, h->pinv32, N);
  HIP_TRY(hipGetLastError());
  if (h->nonzero_dirichlet) {
    double* gext = h->q64;  // scratch
    hipLaunchKernelGGL(dirichlet_field_kernel, dim3(nblk(N)), dim3(kT), 0, h->stream, h->g, gext);
    RC_TRY(launch_gather<double>(h, h->rhoc64, h->k64, 1.0, ck, ProPlain<double>{gext},
                                 EpiStore<double>{h->lift64}, no_relay()));
    hipLaunchKernelGGL(mask_free_kernel, dim3(nblk(N)), dim3(kT), 0, h->stream, h->pinv64, h->lift64, N);
    HIP_TRY(hipGetLastError());
  }
  h->ck_cached = ck;
  return FEM_OK;
}

int ensure_events(fem_heat* h, size_t n) {
  while (h->events.size() < n) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    h->events.push_back(e);
  }
  return FEM_OK;
}

template <typename V>
struct PcgBufs {
  V* x[2];
  int xc;
  V* r;
  V* q;
  V* d[2];
  int dp;
  const V* pinv;
  const V* b;
  const V* rhoc;
  const V* kc;
  RelayCtx* ctx;
  Scalars* S_host;
  double ck;
  uint32_t upd_blocks;
};

// Iterations of Algorithm 1 until the device marks the solve done.  Returns
// FEM_OK with *iters set, FEM_EBREAKDOWN or a device error.
template <typename V>
int pcg_loop(fem_heat* h, PcgBufs<V>& B, int first_chunk, int* iters) {
  const int R = h->opts.replace_every;
  RelayCtx& c = *B.ctx;
  int done_iters = 0;
  int k = std::max(1, first_chunk);
  for (;;) {
    if (h->timing) RC_TRY(ensure_events(h, 3 * (size_t)k));
    int dp = B.dp, xc = B.xc;
    for (int j = 0; j < k; ++j) {
      const int it = done_iters + j;
      if (h->timing) HIP_TRY(hipEventRecord(h->events[3 * j], h->stream));
      RC_TRY(gather_step<V>(h, c, M_DIR, B.rhoc, B.kc, 1.0, B.ck,
                            ProDirection<V>{B.r, B.pinv, B.d[dp], B.d[dp ^ 1], V(0)}, EpiQDot<V>{B.q}));
      dp ^= 1;
      if (h->timing) HIP_TRY(hipEventRecord(h->events[3 * j + 1], h->stream));
      if (R > 0 && it % R == 0) {
        RC_TRY(gather_step<V>(h, c, M_UPD, B.rhoc, B.kc, 1.0, B.ck,
                              ProAxpy<V, V>{B.x[xc], B.d[dp], B.x[xc ^ 1], 0, V(0)},
                              EpiResidual<V>{B.b, B.pinv, B.r}));
        xc ^= 1;
      } else {
        hipLaunchKernelGGL((update_kernel<V>), dim3(B.upd_blocks), dim3(kT), 0, h->stream, B.x[xc], B.d[dp], B.r, B.q,
                           B.pinv, h->g.N, next_relay(c, M_UPD, true, B.upd_blocks));
        HIP_TRY(hipGetLastError());
      }
      if (h->timing) HIP_TRY(hipEventRecord(h->events[3 * j + 2], h->stream));
    }
    RC_TRY(decide_and_read(h, c, B.S_host));
    const int real = B.S_host->iter;
    const int ran = std::max(0, std::min(real - done_iters, k));
    for (int j = 0; j < ran; ++j) {
      const int it = done_iters + j;
      B.dp ^= 1;
      const bool rep = R > 0 && it % R == 0;
      if (rep) B.xc ^= 1;
      if (h->timing) {
        float g_ms = 0.f, u_ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&g_ms, h->events[3 * j], h->events[3 * j + 1]));
        HIP_TRY(hipEventElapsedTime(&u_ms, h->events[3 * j + 1], h->events[3 * j + 2]));
        h->stats.gather_launches += 1;
        h->stats.gather_ms += g_ms;
        if (rep) {
          h->stats.replace_launches += 1;
          h->stats.replace_ms += u_ms;
        } else {
          h->stats.update_launches += 1;
          h->stats.update_ms += u_ms;
        }
      }
    }
    done_iters = real;
    if (B.S_host->status != 0) return fail(h, FEM_EBREAKDOWN, "PCG breakdown (d^T A d <= 0 or non-finite scalar)");
    if (B.S_host->done) break;
    k = 4;
  }
  *iters = done_iters;
  return FEM_OK;
}

struct RunState {
  double* T1;
  double* T2;
  double* X[2];
  int dp64 = 0, dp32 = 0;
  int est = 8;
};

double schedule_value(const fem_heat* h, int64_t m) {
  if (h->sched.empty()) return 1.0;
  if (m < 1 || m > (int64_t)h->sched.size()) return 0.0;
  return h->sched[(size_t)(m - 1)];
}

// One theta-scheme step in FP64.  Leaves the new field in X[*xc].
int step_fp64(fem_heat* h, RunState& st, double dt, double theta, double s_n, int* iters, int* xc_out) {
  const double ckA = theta * dt, ckL = -(1.0 - theta) * dt;
  RelayCtx& c = h->outer;
  RC_TRY(gather_step<double>(h, c, M_RHS, h->rhoc64, h->k64, 1.0, ckL, ProPlain<double>{st.T1},
                             EpiRhs<double>{h->b64, h->F64, h->pinv64, h->lift64, dt * s_n}));
  RC_TRY(gather_step<double>(
      h, c, M_INIT, h->rhoc64, h->k64, 1.0, ckA,
      ProGuess<double>{st.T1, st.T2, h->pinv64, st.X[0], h->opts.guess == FEM_GUESS_PREV ? 1 : 0, 0},
      EpiResidual<double>{h->b64, h->pinv64, h->r64}));
  PcgBufs<double> B{{st.X[0], st.X[1]}, 0,      h->r64,   h->q64, {h->d64[0], h->d64[1]}, st.dp64, h->pinv64,
                    h->b64,             h->rhoc64, h->k64, &c,     h->S_host,              ckA,     h->upd_blocks64};
  RC_TRY(pcg_loop<double>(h, B, st.est, iters));
  st.dp64 = B.dp;
  *xc_out = B.xc;
  return FEM_OK;
}

// One step of the mixed form: FP64 right-hand side, guess and residual; FP32
// inner PCG on A e = r (FP64 dot products and scalars); FP64 correction
// x += e and residual r = b - A x, repeated until the FP64 stop rule holds.
int step_mixed(fem_heat* h, RunState& st, double dt, double theta, double s_n, int* iters, int* sweeps,
               int* xc_out) {
  const double ckA = theta * dt, ckL = -(1.0 - theta) * dt;
  const uint32_t N = h->g.N;
  RelayCtx& c = h->outer;
  RC_TRY(gather_step<double>(h, c, M_RHS, h->rhoc64, h->k64, 1.0, ckL, ProPlain<double>{st.T1},
                             EpiRhs<double>{h->b64, h->F64, h->pinv64, h->lift64, dt * s_n}));
  RC_TRY(gather_step<double>(
      h, c, M_INIT, h->rhoc64, h->k64, 1.0, ckA,
      ProGuess<double>{st.T1, st.T2, h->pinv64, st.X[0], h->opts.guess == FEM_GUESS_PREV ? 1 : 0, 0},
      EpiResidual<double>{h->b64, h->pinv64, h->r64}));
  int xc = 0;
  Scalars* so = h->S_host;
  RC_TRY(decide_and_read(h, c, so));
  if (so->status != 0) return fail(h, FEM_EBREAKDOWN, "non-finite initial residual");
  int total = 0, nsw = 0;
  const uint32_t sblocks = std::min<uint32_t>(nblk(N), 1024);
  while (!so->done && nsw < h->opts.max_refine) {
    // Inner tolerance: half the reduction the FP64 stop rule still needs,
    // never tighter than inner_rtol (FP32 arithmetic bounds what the inner
    // solve can reach); one sweep then usually suffices.
    const double ref = h->opts.stop_rule == FEM_STOP_INITIAL ? so->delta0 : so->delta_b;
    const double need = so->delta > 0 ? 0.5 * std::sqrt(c.ctl.rtol2 * ref / so->delta) : 1.0;
    const double irt = std::min(0.5, std::max(h->opts.inner_rtol, need));
    h->inner.ctl.rtol2 = irt * irt;
    hipLaunchKernelGGL(inner_start_kernel, dim3(sblocks), dim3(kT), 0, h->stream, h->r64, h->rhs32, h->r32, h->e32[0],
                       h->pinv32, N, next_relay(h->inner, M_START, true, sblocks));
    HIP_TRY(hipGetLastError());
    PcgBufs<float> B{{h->e32[0], h->e32[1]}, 0,         h->r32, h->q32,    {h->d32[0], h->d32[1]}, st.dp32, h->pinv32,
                     h->rhs32,               h->rhoc32, h->k32, &h->inner, h->S_host + 1,          ckA,     h->upd_blocks32};
    int it = 0;
    RC_TRY(pcg_loop<float>(h, B, nsw == 0 ? st.est : std::max(1, st.est / 4), &it));
    st.dp32 = B.dp;
    total += it;
    RC_TRY(gather_step<double>(h, c, M_CORR, h->rhoc64, h->k64, 1.0, ckA,
                               ProAxpy<double, float>{st.X[xc], h->e32[B.xc], st.X[xc ^ 1], 1, 0.0},
                               EpiResidual<double>{h->b64, h->pinv64, h->r64}));
    xc ^= 1;
    ++nsw;
    RC_TRY(decide_and_read(h, c, so));
    if (so->status != 0) return fail(h, FEM_EBREAKDOWN, "non-finite residual in the refinement");
  }
  *iters = total;
  *sweeps = nsw;
  *xc_out = xc;
  return FEM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

int solver_init(fem_heat* h, const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc) {
  Geom& g = h->g;
  g.nx = grid->nx;
  g.ny = grid->ny;
  g.nz = grid->nz;
  g.px = grid->nx + 1;
  g.py = grid->ny + 1;
  g.pz = grid->nz + 1;
  g.N = (uint32_t)g.px * g.py * g.pz;
  g.E = (uint32_t)g.nx * g.ny * g.nz;
  g.hx = grid->hx;
  g.hy = grid->hy;
  g.hz = grid->hz;
  g.dir_mask = bc ? bc->dirichlet_mask : 0u;
  g.flux_mask = bc ? bc->flux_mask : 0u;
  h->nonzero_dirichlet = false;
  for (int f = 0; f < 6; ++f) {
    g.dir_val[f] = bc ? bc->dirichlet_value[f] : 0.0;
    g.flux[f] = bc ? bc->flux[f] : 0.0;
    if (((g.dir_mask >> f) & 1u) && g.dir_val[f] != 0.0) h->nonzero_dirichlet = true;
  }
  if (bc && bc->flux_schedule && bc->n_schedule > 0)
    h->sched.assign(bc->flux_schedule, bc->flux_schedule + bc->n_schedule);
  h->cubic = (g.hx == g.hy && g.hy == g.hz);
  HIP_TRY(hipSetDevice(h->opts.device));
  {
    // the x-y tiling does not depend on the capacity: size the block first
    const GatherShape probe = choose_shape(g, h->opts, 1);
    const bool fp32 = h->opts.precision == FEM_FP32_FP64DOT;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->opts.device));
    const int per_cu = resident_blocks(h->cubic, fp32, probe.nthreads, probe.smem_bytes(fp32 ? 4 : 8));
    h->shape = choose_shape(g, h->opts, std::max(1, cus) * per_cu);
  }
  {
    const GatherShape& s = h->shape;
    if ((s.tx + 2) * (s.ty + 2) > kSlots * s.nthreads || (s.tx + 1) * (s.ty + 1) > kSlots * s.nthreads)
      return fail(h, FEM_EINVAL, "tile shape too thin for the staging scheme");
  }
  h->upd_blocks64 = std::max<uint32_t>(1, std::min<uint32_t>(nblk((g.N + 1) / 2), 512));
  h->upd_blocks32 = std::max<uint32_t>(1, std::min<uint32_t>(nblk((g.N + 3) / 4), 512));
  h->stats.tile_x = h->shape.tx;
  h->stats.tile_y = h->shape.ty;
  h->stats.tile_z = h->shape.tz;
  h->stats.grid_blocks = (int32_t)h->shape.nblocks;

  if (h->opts.hip_stream) {
    h->stream = reinterpret_cast<hipStream_t>(h->opts.hip_stream);
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  const uint32_t N = g.N, E = g.E;
  RC_TRY(dalloc(h, &h->rhoc64, E));
  RC_TRY(dalloc(h, &h->k64, E));
  RC_TRY(dalloc(h, &h->F64, N));
  RC_TRY(dalloc(h, &h->pinv64, N));
  RC_TRY(dalloc(h, &h->b64, N));
  RC_TRY(dalloc(h, &h->r64, N));
  RC_TRY(dalloc(h, &h->q64, N));
  RC_TRY(dalloc(h, &h->d64[0], N));
  RC_TRY(dalloc(h, &h->d64[1], N));
  for (auto& p : h->pool) RC_TRY(dalloc(h, &p, N));
  if (h->nonzero_dirichlet) RC_TRY(dalloc(h, &h->lift64, N));
  RC_TRY(dalloc(h, &h->sink, 256));
  h->n_partials = std::max({h->shape.nblocks, h->upd_blocks64, h->upd_blocks32, 1024u});
  for (RelayCtx* c : {&h->outer, &h->inner})
    for (int k = 0; k < 2; ++k) {
      RC_TRY(dalloc(h, &c->S[k], 1));
      RC_TRY(dalloc(h, &c->P[k], h->n_partials));
      HIP_TRY(hipMemsetAsync(c->S[k], 0, sizeof(Scalars), h->stream));
      HIP_TRY(hipMemsetAsync(c->P[k], 0, h->n_partials * sizeof(double), h->stream));
    }
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&h->S_host), 2 * sizeof(Scalars), hipHostMallocDefault));
  RC_TRY(copy_in(h, h->rhoc64, rhoc_e, E));
  RC_TRY(copy_in(h, h->k64, k_e, E));
  hipLaunchKernelGGL(load_vector_kernel, dim3(nblk(N)), dim3(kT), 0, h->stream, g, h->F64);
  HIP_TRY(hipGetLastError());
  if (h->opts.precision == FEM_FP32_FP64DOT) RC_TRY(ensure_fp32(h));
  HIP_TRY(hipEventCreate(&h->ev_run[0]));
  HIP_TRY(hipEventCreate(&h->ev_run[1]));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FEM_OK;
}

int solver_run(fem_heat* h, const double* T0, const double* T_prev, double dt, double theta, int32_t nsteps,
               double rtol, fem_out* o) {
  HIP_TRY(hipSetDevice(h->opts.device));
  const bool mixed = h->opts.precision == FEM_FP32_FP64DOT;
  const uint32_t N = h->g.N;
  RC_TRY(prepare_operator(h, theta * dt, mixed));
  RunState st;
  st.T1 = h->pool[0];
  st.T2 = h->pool[1];
  st.X[0] = h->pool[2];
  st.X[1] = h->pool[3];
  RC_TRY(copy_in(h, st.T1, T0, N));
  RC_TRY(copy_in(h, st.T2, T_prev ? T_prev : T0, N));
  hipLaunchKernelGGL((apply_dirichlet_kernel<double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->g, st.T1);
  hipLaunchKernelGGL((apply_dirichlet_kernel<double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->g, st.T2);
  for (int k = 0; k < 2; ++k)
    hipLaunchKernelGGL((fill_kernel<double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->d64[k], 0.0, N);
  if (mixed)
    for (int k = 0; k < 2; ++k)
      hipLaunchKernelGGL((fill_kernel<float>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->d32[k], 0.0f, N);
  HIP_TRY(hipGetLastError());

  const int S = (o && o->sensor_xyz && o->n_sensors > 0) ? o->n_sensors : 0;
  if (S > 0) {
    if (h->xyz_cap < (size_t)S) {
      dfree(h->xyz_dev);
      RC_TRY(dalloc(h, &h->xyz_dev, 3 * (size_t)S));
      h->xyz_cap = S;
    }
    RC_TRY(copy_in(h, h->xyz_dev, o->sensor_xyz, 3 * (size_t)S));
    const size_t need = (size_t)std::max(nsteps, 1) * S;
    if (h->traces_cap < need) {
      dfree(h->traces_dev);
      RC_TRY(dalloc(h, &h->traces_dev, need));
      h->traces_cap = need;
    }
  }
  std::vector<int32_t> iters((size_t)std::max(nsteps, 0), 0), sweeps(iters.size(), 0);
  std::vector<double> relres(iters.size(), 0.0);
  h->stats.gather_launches = h->stats.update_launches = h->stats.replace_launches = 0;
  h->stats.gather_ms = h->stats.update_ms = h->stats.replace_ms = 0.0;

  h->outer.ctl = Ctl{rtol * rtol, h->opts.max_iter, h->opts.stop_rule};
  h->inner.ctl = Ctl{h->opts.inner_rtol * h->opts.inner_rtol, h->opts.max_iter, 1};
  const int first = o ? o->first_step : 0;
  int status = FEM_OK;
  int64_t total = 0;
  HIP_TRY(hipEventRecord(h->ev_run[0], h->stream));
  for (int32_t n = 1; n <= nsteps; ++n) {
    const double s_n = schedule_value(h, (int64_t)first + n);
    int it = 0, nsw = 0, xc = 0;
    int rc = mixed ? step_mixed(h, st, dt, theta, s_n, &it, &nsw, &xc) : step_fp64(h, st, dt, theta, s_n, &it, &xc);
    if (rc == FEM_EBREAKDOWN) {
      status = rc;
      break;
    }
    if (rc != FEM_OK) return rc;
    const Scalars& so = h->S_host[0];
    iters[n - 1] = it;
    sweeps[n - 1] = nsw;
    relres[n - 1] = so.delta_b > 0 ? std::sqrt(std::max(so.delta, 0.0) / so.delta_b) : 0.0;
    const bool unconverged = mixed ? (so.delta > so.tol) : (it >= h->opts.max_iter && so.delta > so.tol);
    if (unconverged && status == FEM_OK) status = FEM_ENOCONV;
    total += it;
    st.est = std::max(1, it);
    double* xnew = st.X[xc];
    if (S > 0) {
      hipLaunchKernelGGL(sensor_kernel, dim3((S + 63) / 64), dim3(64), 0, h->stream, h->g, xnew, h->xyz_dev, S,
                         h->traces_dev + (size_t)(n - 1) * S);
      HIP_TRY(hipGetLastError());
    }
    if (o && o->T_saved && o->save_every > 0 && n % o->save_every == 0)
      RC_TRY(copy_out(h, o->T_saved + (size_t)(n / o->save_every - 1) * N, xnew, (size_t)N * sizeof(double)));
    double* freed = st.T2;
    double* spare = st.X[xc ^ 1];
    st.T2 = st.T1;
    st.T1 = xnew;
    st.X[0] = freed;
    st.X[1] = spare;
  }
  HIP_TRY(hipEventRecord(h->ev_run[1], h->stream));
  HIP_TRY(hipEventSynchronize(h->ev_run[1]));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev_run[0], h->ev_run[1]));
  if (o) {
    o->device_ms = ms;
    o->total_iters = total;
    if (o->T_final) RC_TRY(copy_out(h, o->T_final, st.T1, (size_t)N * sizeof(double)));
    if (S > 0 && o->traces)
      RC_TRY(copy_out(h, o->traces, h->traces_dev, (size_t)std::max(nsteps, 0) * S * sizeof(double)));
    if (o->iters) {
      if (h->devptrs)
        HIP_TRY(hipMemcpyAsync(o->iters, iters.data(), iters.size() * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
      else
        std::memcpy(o->iters, iters.data(), iters.size() * sizeof(int32_t));
    }
    if (o->relres) {
      if (h->devptrs)
        HIP_TRY(hipMemcpyAsync(o->relres, relres.data(), relres.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
      else
        std::memcpy(o->relres, relres.data(), relres.size() * sizeof(double));
    }
    if (o->refine_sweeps) {
      if (h->devptrs)
        HIP_TRY(hipMemcpyAsync(o->refine_sweeps, sweeps.data(), sweeps.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               h->stream));
      else
        std::memcpy(o->refine_sweeps, sweeps.data(), sweeps.size() * sizeof(int32_t));
    }
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return status;
}

int solver_apply(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  HIP_TRY(hipSetDevice(h->opts.device));
  const uint32_t N = h->g.N;
  const bool fp32 = (which & FEM_OP_FP32) != 0;
  const int op = which & 0xff;
  double* xd = h->pool[0];
  double* yd = h->pool[1];
  if (op != FEM_OP_LOAD) RC_TRY(copy_in(h, xd, x, N));
  if (op == FEM_OP_A || op == FEM_OP_L) {
    const double ck = op == FEM_OP_A ? theta * dt : -(1.0 - theta) * dt;
    if (fp32) {
      RC_TRY(ensure_fp32(h));
      hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(N)), dim3(kT), 0, h->stream, xd, h->e32[0], N);
      RC_TRY(launch_gather<float>(h, h->rhoc32, h->k32, 1.0, ck, ProPlain<float>{h->e32[0]}, EpiStore<float>{h->q32},
                                  no_relay()));
      hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->q32, yd, N);
    } else {
      RC_TRY(launch_gather<double>(h, h->rhoc64, h->k64, 1.0, ck, ProPlain<double>{xd}, EpiStore<double>{yd},
                                   no_relay()));
    }
  } else if (op == FEM_OP_JACOBI) {
    RC_TRY(prepare_operator(h, theta * dt, fp32));
    if (fp32) {
      hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(N)), dim3(kT), 0, h->stream, xd, h->e32[0], N);
      hipLaunchKernelGGL((scale_kernel<float>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->pinv32, h->e32[0], yd, N);
    } else {
      hipLaunchKernelGGL((scale_kernel<double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->pinv64, xd, yd, N);
    }
  } else if (op == FEM_OP_LOAD) {
    HIP_TRY(hipMemcpyAsync(yd, h->F64, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else {
    return fail(h, FEM_EINVAL, "unknown operator");
  }
  HIP_TRY(hipGetLastError());
  RC_TRY(copy_out(h, y, yd, (size_t)N * sizeof(double)));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FEM_OK;
}

void solver_free(fem_heat* h) {
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  dfree(h->rhoc64);
  dfree(h->k64);
  dfree(h->rhoc32);
  dfree(h->k32);
  dfree(h->F64);
  dfree(h->pinv64);
  dfree(h->b64);
  dfree(h->r64);
  dfree(h->q64);
  for (auto& p : h->d64) dfree(p);
  for (auto& p : h->pool) dfree(p);
  dfree(h->lift64);
  dfree(h->sink);
  dfree(h->pinv32);
  for (auto& p : h->e32) dfree(p);
  dfree(h->r32);
  dfree(h->q32);
  for (auto& p : h->d32) dfree(p);
  dfree(h->rhs32);
  for (RelayCtx* c : {&h->outer, &h->inner})
    for (int k = 0; k < 2; ++k) {
      dfree(c->S[k]);
      dfree(c->P[k]);
    }
  dfree(h->xyz_dev);
  dfree(h->traces_dev);
  if (h->S_host) (void)hipHostFree(h->S_host);
  h->S_host = nullptr;
  for (auto e : h->events) (void)hipEventDestroy(e);
  h->events.clear();
  for (auto& e : h->ev_run)
    if (e) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  h->stream = nullptr;
}

}  // namespace femheat
