// Batched launches of the time-stepping path (gfx950).
//
// One launch of each kernel below serves every simulation of a batch: the
// repeated forward solves of a coefficient study (Sec. 5.4) share the GPU
// instead of taking it in turn.  Every block belongs to one simulation: a
// work table maps the block's work item to (simulation, block index within
// it), and the block then runs exactly the code, on exactly the data, that a
// launch for that simulation alone would run -- same tiles, same block
// counts, partials stored at the same index, same relay state -- so a
// simulation's results do not depend on its co-runners, bit for bit.
//
// What differs between the launches of one time step is uniform across the
// batch: all simulations advance one step per epoch in lockstep, and inside
// a solve the buffer parities follow from the iteration index alone (the
// search direction ping-pongs every iteration, x every residual
// replacement).  Per-simulation data -- buffers, operator constants, relay
// state, tolerances -- sit in a SimDev array in device memory that the host
// rewrites only at step and refinement-sweep boundaries.  A simulation whose
// solve has converged stays in the launches: its blocks read the relayed
// state, see that it is done and return.
#pragma once

#include "gather.hpp"
#include "vector_kernels.hpp"

namespace femheat {

// Kernel kinds whose block partials a relay reads (their block counts differ).
enum PartKind : int32_t { PK_GATHER = 0, PK_UPD64 = 1, PK_UPD32 = 2, PK_START = 3 };

// Everything the batched kernels need of one simulation.
struct SimDev {
  GatherArgs<double> A64;  // A = M + theta*dt*K
  GatherArgs<double> L64;  // L = M - (1-theta)*dt*K
  GatherArgs<float> A32;   // A in FP32 (mixed form)
  const double* F64;
  const double* pinv64;
  const double* lift64;
  double* b64;
  double* r64;
  double* q64;
  double* r64b;  // one-reduction form: second residual and apply buffers (ping-pong with r64, q64)
  double* q64b;
  double* d64[2];
  const double* T1;  // T^{n-1}
  const double* T2;  // T^{n-2}
  double* X[2];      // iterate ping-pong; the guess is written to X[0]
  const float* pinv32;
  float* r32;
  float* q32;
  float* r32b;  // one-reduction form of the inner solves: second residual and apply buffers
  float* q32b;
  float* d32[2];
  float* e32[2];
  float* rhs32;
  Scalars* oS[2];  // outer (FP64) relay state and partials
  double* oP[2];
  Scalars* iS[2];  // inner (FP32) relay state and partials
  double* iP[2];
  Ctl octl, ictl;
  uint32_t N;
  uint32_t nblk[4];    // blocks of each PartKind
  uint32_t ldp;        // capacity of each partial component (one-reduction form: four per block)
  double fs;           // dt * s_n of the current step
  int32_t guess_prev;  // 1: x0 = T^{n-1}
  int32_t xc;          // mixed form: X buffer of the current FP64 iterate
  int32_t exc;         // mixed form: e buffer of the last inner solution
  int32_t sweep;       // mixed form: this sweep runs an inner solve and a correction
  double inner_rtol;   // mixed form: floor of the inner relative tolerance
  // Chebyshev preconditioner (FP64 solves): the preconditioned residual s,
  // the chain's residual and direction ping-pong, 1/c and the coefficients
  // a_k = rho_k rho_{k-1}, b_k = 2 rho_k / w of its steps k = 1 .. m-1
  double* s64;
  double* cr64;
  double* cd64[2];
  double ch_inv_c;
  double ch_a[kChebMaxDegree], ch_b[kChebMaxDegree];
};

// What the update kernel of a launch with a single simulation needs, passed
// with the launch itself: it then starts without first reading the
// simulation's SimDev (one dependent memory read less on its critical path).
struct UpdView {
  uint32_t N, nblk;
  void* r;
  const void* q;
  const void* pinv;
  void* x;          // FP32 inner solves: x += alpha d here (nullptr in FP64)
  const void* d;
  Relay R;
};

// Uniform arguments of one batched launch.
struct BatchArgs {
  const SimDev* sims;
  const uint2* table;  // work item -> (simulation, block within it); nullptr: one simulation
  Scalars* snap;       // decide: per-simulation copy of the settled state
  int32_t cur;         // relay parity: state/partials buffer this launch reads
  int32_t prev;        // PartKind of the partials it reads
  int32_t j;           // iteration index within the current solve
  int32_t xpar;        // replacements so far in this solve, mod 2 (x or e buffer)
  int32_t corr;        // the previous kernel was a plain update: x += alpha d is still due
  UpdView uv;          // update launches of a single simulation
  int32_t ocur;        // inner start: parity of the settled outer state
  int32_t next_xc;     // next-step launches: iterate buffer the current solve is assumed to end in
  int32_t next_R;      //                     replacement period (< 0: mixed form, buffer known)
  double next_fs;      //                     dt * s of the next step
  int32_t cheb_k;      // Chebyshev chain: step k (1 .. m-1) of this launch
  int32_t cheb_last;   //                  the chain's last step (it publishes r_in^T s)
  int32_t cheb_rhs;    //                  the chain preconditions the lifted right-hand side (else r)
  uint32_t* seq;       // decide of one simulation whose host polls: sequence word per simulation (else nullptr)
  uint32_t seq_val;    //                                         the value this decide writes there
};

__host__ __device__ inline Relay outer_relay(const SimDev& s, const BatchArgs& a, int32_t mode, bool partials) {
  return Relay{s.oS[a.cur], s.oS[a.cur ^ 1], s.oP[a.cur], s.nblk[a.prev], partials ? s.oP[a.cur ^ 1] : nullptr,
               mode, s.octl, s.ldp};
}
__host__ __device__ inline Relay inner_relay(const SimDev& s, const BatchArgs& a, int32_t mode, bool partials) {
  return Relay{s.iS[a.cur], s.iS[a.cur ^ 1], s.iP[a.cur], s.nblk[a.prev], partials ? s.iP[a.cur ^ 1] : nullptr,
               mode, s.ictl, s.ldp};
}

// The direction ping-pongs every iteration: iteration j reads d[j&1] and
// writes d[(j+1)&1], which the update of iteration j then uses.
__host__ __device__ inline int dir_in(const BatchArgs& a) { return a.j & 1; }
__host__ __device__ inline int dir_out(const BatchArgs& a) { return (a.j + 1) & 1; }

// ---- gather roles: operator, prologue, epilogue and relay of each gather ----

struct RoleRhs {  // b = L T^{n-1} + dt*s_n*F, with b^T P^-1 b
  using V = double;
  using Pro = ProPlain<double>;
  using Epi = EpiRhs<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.L64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs&) { return Pro{s.T1}; }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.b64, s.F64, s.pinv64, s.lift64, s.fs}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_RHS, true); }
};

struct RoleInit {  // x0 by the guess rule, r = b - A x0, r^T P^-1 r
  using V = double;
  using Pro = ProGuess<double>;
  using Epi = EpiResidual<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs&) {
    return Pro{s.T1, s.T2, s.pinv64, s.X[0], s.guess_prev, 0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.b64, s.pinv64, s.r64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_INIT, true); }
};

// The next step's RHS and initial residual, launched right after a decide
// and before the host has read it (the host would otherwise leave the GPU
// idle for its round trip).  They see the fields as the step's end will
// rotate them -- T^n = X[next_xc], T^{n-1} = T1, the guess into T2's buffer --
// and run only if the solve has ended well in X[next_xc]; otherwise they
// pass the state through and the host carries on (see M_RHS_NEXT).
__host__ __device__ inline Relay next_relay(const SimDev& s, const BatchArgs& a, int32_t mode) {
  Relay R = outer_relay(s, a, mode, true);
  R.next_xc = a.next_xc;
  R.next_R = a.next_R;
  return R;
}

struct RoleRhsNext {
  using V = double;
  using Pro = ProPlain<double>;
  using Epi = EpiRhs<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.L64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) { return Pro{s.X[a.next_xc]}; }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) {
    return Epi{s.b64, s.F64, s.pinv64, s.lift64, a.next_fs};
  }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return next_relay(s, a, M_RHS_NEXT); }
};

struct RoleInitNext {
  using V = double;
  using Pro = ProGuess<double>;
  using Epi = EpiResidual<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.X[a.next_xc], s.T1, s.pinv64, const_cast<double*>(s.T2), s.guess_prev, 0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.b64, s.pinv64, s.r64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return next_relay(s, a, M_INIT_NEXT); }
};

template <typename V>
struct RoleDir;  // d = P^-1 r + beta d, q = A d, d^T q; deferred x += alpha d_old

template <>
struct RoleDir<double> {
  using V = double;
  using Pro = ProDirection<double>;
  using Epi = EpiQDot<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.r64, s.pinv64, s.d64[dir_in(a)], s.d64[dir_out(a)], s.X[a.xpar], a.corr, 0.0, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.q64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_DIR, true); }
};

template <>
struct RoleDir<float> {
  using V = float;
  using Pro = ProDirection<float>;
  using Epi = EpiQDot<float>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A32; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.r32, s.pinv32, s.d32[dir_in(a)], s.d32[dir_out(a)], s.e32[a.xpar], a.corr, 0.0f, 0.0f};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.q32}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return inner_relay(s, a, M_DIR, true); }
};

template <typename V>
struct RoleRepl;  // residual replacement: x += alpha d, r = b - A x (i mod 50 == 0)

template <>
struct RoleRepl<double> {
  using V = double;
  using Pro = ProAxpy<double, double>;
  using Epi = EpiResidual<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.X[a.xpar], s.d64[dir_out(a)], s.X[a.xpar ^ 1], 0, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.b64, s.pinv64, s.r64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_UPD, true); }
};

template <>
struct RoleRepl<float> {
  using V = float;
  using Pro = ProAxpy<float, float>;
  using Epi = EpiResidual<float>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A32; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.e32[a.xpar], s.d32[dir_out(a)], s.e32[a.xpar ^ 1], 0, 0.0f};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.rhs32, s.pinv32, s.r32}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return inner_relay(s, a, M_UPD, true); }
};

// One-reduction form (FP64): iteration j's residual lives in buffer j&1 of
// (r64, r64b) and its q = A d in buffer j&1 of (q64, q64b); the initial
// residual is in r64 (buffer 0).
__host__ __device__ inline double* rbuf(const SimDev& s, int k) { return (k & 1) ? s.r64b : s.r64; }
__host__ __device__ inline double* qbuf(const SimDev& s, int k) { return (k & 1) ? s.q64b : s.q64; }

struct RoleFused {  // (r -= alpha q, x += alpha d_old,) d = P^-1 r + beta d, q = A d, four sums
  using V = double;
  using Pro = ProFused<double>;
  using Epi = EpiQ<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{rbuf(s, a.corr ? a.j + 1 : a.j), qbuf(s, a.j + 1), s.pinv64, s.d64[dir_in(a)], s.d64[dir_out(a)],
               s.X[a.xpar], rbuf(s, a.j), a.corr, 0.0, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) { return Epi{qbuf(s, a.j)}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) {
    return outer_relay(s, a, a.corr ? M_FUPD : M_FDIR, true);
  }
};

struct RoleReplFused {  // one-reduction form: x += alpha d, r = b - A x into the next residual buffer
  using V = double;
  static constexpr bool kFour = true;  // follows a one-reduction direction kernel
  using Pro = ProAxpy<double, double>;
  using Epi = EpiResidual<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.X[a.xpar], s.d64[dir_out(a)], s.X[a.xpar ^ 1], 0, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) { return Epi{s.b64, s.pinv64, rbuf(s, a.j + 1)}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_FREPL, true); }
};

// The one-reduction form of the FP32 inner solves of the mixed form: the
// same kernels on the FP32 set (r32, r32b; q32, q32b; the inner iterate e)
// with the inner relay (FP64 sums and scalars).
__host__ __device__ inline float* rbuf32(const SimDev& s, int k) { return (k & 1) ? s.r32b : s.r32; }
__host__ __device__ inline float* qbuf32(const SimDev& s, int k) { return (k & 1) ? s.q32b : s.q32; }

struct RoleFused32 {
  using V = float;
  using Pro = ProFused<float>;
  using Epi = EpiQ<float>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A32; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{rbuf32(s, a.corr ? a.j + 1 : a.j), qbuf32(s, a.j + 1), s.pinv32, s.d32[dir_in(a)], s.d32[dir_out(a)],
               s.e32[a.xpar], rbuf32(s, a.j), a.corr, 0.0f, 0.0f};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) { return Epi{qbuf32(s, a.j)}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) {
    return inner_relay(s, a, a.corr ? M_FUPD : M_FDIR, true);
  }
};

struct RoleReplFused32 {  // e += alpha d, r = rhs - A e into the next residual buffer
  using V = float;
  static constexpr bool kFour = true;
  using Pro = ProAxpy<float, float>;
  using Epi = EpiResidual<float>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A32; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.e32[a.xpar], s.d32[dir_out(a)], s.e32[a.xpar ^ 1], 0, 0.0f};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) {
    return Epi{s.rhs32, s.pinv32, rbuf32(s, a.j + 1)};
  }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return inner_relay(s, a, M_FREPL, true); }
};

struct RoleCorr {  // mixed form: x64 += e, r64 = b - A x64, FP64 residual norm
  using V = double;
  using Pro = ProAxpy<double, float>;
  using Epi = EpiResidual<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs&) {
    return Pro{s.X[s.xc], s.e32[s.exc], s.X[s.xc ^ 1], 1, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.b64, s.pinv64, s.r64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) {
    return outer_relay(s, a, s.sweep ? M_CORR : M_SKIP, true);
  }
};

// Search direction from the Chebyshev-preconditioned residual s.
struct RoleDirS {
  using V = double;
  using Pro = ProDirectionS<double>;
  using Epi = EpiQDot<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{s.s64, s.d64[dir_in(a)], s.d64[dir_out(a)], s.X[a.xpar], a.corr, 0.0, 0.0};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs&) { return Epi{s.q64}; }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) { return outer_relay(s, a, M_DIR, true); }
};

// The Chebyshev preconditioner s = q(D^-1 A) D^-1 r_in as a chain of gathers
// relayed with M_PASS; the last one publishes r_in^T s, which completes the
// scalar update pending before the chain (delta_b of a right-hand side, or
// the delta of an initial residual, an update or a replacement).
__host__ __device__ inline const double* cheb_rin(const SimDev& s, const BatchArgs& a) { return a.cheb_rhs ? s.b64 : s.r64; }
__host__ __device__ inline const double* cheb_lift(const SimDev& s, const BatchArgs& a) {
  return a.cheb_rhs ? s.lift64 : nullptr;
}

struct RoleChebFirst {  // step 1: gathers d_0 = P^-1 (r_in - lift) / c
  using V = double;
  using Pro = ProChebStart<double>;
  using Epi = EpiCheb<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) {
    return Pro{cheb_rin(s, a), cheb_lift(s, a), s.pinv64, s.ch_inv_c};
  }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) {
    return Epi{cheb_rin(s, a), cheb_lift(s, a), s.pinv64, nullptr, cheb_rin(s, a), cheb_lift(s, a), s.cr64,
               s.cd64[1], s.s64, s.ch_a[0], s.ch_b[0], a.cheb_last};
  }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) {
    return outer_relay(s, a, M_PASS, a.cheb_last != 0);
  }
};

struct RoleChebNext {  // step k >= 2: gathers d_{k-1}
  using V = double;
  using Pro = ProPlain<double>;
  using Epi = EpiCheb<double>;
  static __host__ __device__ const GatherArgs<V>& ga(const SimDev& s) { return s.A64; }
  static __host__ __device__ Pro pro(const SimDev& s, const BatchArgs& a) { return Pro{s.cd64[(a.cheb_k - 1) & 1]}; }
  static __host__ __device__ Epi epi(const SimDev& s, const BatchArgs& a) {
    return Epi{s.cr64, nullptr, s.pinv64, s.s64, cheb_rin(s, a), cheb_lift(s, a), s.cr64, s.cd64[a.cheb_k & 1],
               s.s64, s.ch_a[a.cheb_k - 1], s.ch_b[a.cheb_k - 1], a.cheb_last};
  }
  static __host__ __device__ Relay relay(const SimDev& s, const BatchArgs& a) {
    return outer_relay(s, a, M_PASS, a.cheb_last != 0);
  }
};

// ---- kernels -----------------------------------------------------------------

// Whether a role's kernel may follow a one-reduction direction kernel (and so
// sum four partials): roles that say so with kFour.
template <class Role>
constexpr auto reads_four(int) -> decltype(Role::kFour, bool()) { return Role::kFour; }
template <class Role>
constexpr bool reads_four(long) { return false; }

__device__ inline void work_item(const BatchArgs& a, uint32_t w, uint32_t& sim, uint32_t& local) {
  sim = 0;
  local = w;
  if (a.table) {
    const uint2 e = a.table[w];
    sim = e.x;
    local = e.y;
  }
}

// One gather role over every simulation of a launch group (grid = the sum
// of the group's per-simulation block counts, each a multiple of 8).
template <int KIND, class Role>
__global__ void __launch_bounds__(256, 2) gather_batch_kernel(BatchArgs a) {
  uint32_t sim, local;
  work_item(a, xcd_work_item(blockIdx.x, gridDim.x), sim, local);
  const SimDev& s = a.sims[sim];
  const GatherArgs<typename Role::V> ga = Role::ga(s);
  using Pro = typename Role::Pro;
  gather_tile<typename Role::V, KIND, Pro, typename Role::Epi, reads_four<Role>(0) || AdvancesResidual<Pro>::value>(
      ga, Role::pro(s, a), Role::epi(s, a), Role::relay(s, a), local);
}

// One gather role of a single simulation, its operator, functors and relay
// passed by value in the launch: the first plane loads need no dependent
// read of the simulation's record (the same code as gather_batch_kernel on
// the same data, so the same bits).
template <int KIND, class Role>
__global__ void __launch_bounds__(kMaxBlockThreads)
    gather_one_kernel(GatherArgs<typename Role::V> ga, typename Role::Pro pro, typename Role::Epi epi, Relay R) {
  using Pro = typename Role::Pro;
  gather_tile<typename Role::V, KIND, Pro, typename Role::Epi, reads_four<Role>(0) || AdvancesResidual<Pro>::value>(
      ga, pro, epi, R, xcd_work_item(blockIdx.x, gridDim.x));
}

// Residual update and preconditioned residual norm, FP64 outer solve
// or FP32 inner solve; kOne: the launch serves one simulation (UpdView).
template <typename V, bool kOne>
__global__ void __launch_bounds__(256) update_batch_kernel(BatchArgs a) {
  if constexpr (kOne) {  // one simulation, its vectors and relay in the launch arguments
    V* x = nullptr;  // (a literal null in FP64, so that kernel has no x path)
    const V* d = nullptr;
    if constexpr (sizeof(V) == 4) {
      x = static_cast<V*>(a.uv.x);
      d = static_cast<const V*>(a.uv.d);
    }
    update_body<V, true, sizeof(V) == 8 ? 4 : 2>(static_cast<V*>(a.uv.r), static_cast<const V*>(a.uv.q),
                                                 static_cast<const V*>(a.uv.pinv), a.uv.N, a.uv.R, blockIdx.x,
                                                 a.uv.nblk, x, d);
    return;
  }
  uint32_t sim, local;
  work_item(a, blockIdx.x, sim, local);
  const SimDev& s = a.sims[sim];
  if constexpr (sizeof(V) == 8) {
    update_body<double>(s.r64, s.q64, s.pinv64, s.N, outer_relay(s, a, M_UPD, true), local, s.nblk[PK_UPD64]);
  } else {
    update_body<float>(s.r32, s.q32, s.pinv32, s.N, inner_relay(s, a, M_UPD, true), local, s.nblk[PK_UPD32],
                       s.e32[a.xpar], s.d32[dir_out(a)]);
  }
}

// Start of the inner solves of a refinement sweep.  A simulation sweeps
// if the host asked for it and its settled outer state (read here, so the
// host need not have seen it) is neither done nor broken down; the others get
// an idle, already finished inner solve.  The inner tolerance is half the
// reduction the FP64 stop rule still needs, never tighter than inner_rtol
// (FP32 arithmetic bounds what the inner solve can reach) nor looser than
// 0.5; it goes to the first evaluation with the relayed state.
__device__ inline void inner_start_sim(const SimDev& s, const BatchArgs& a, uint32_t local) {
  Relay R = inner_relay(s, a, M_IDLE, true);
  if (s.sweep) {
    const Scalars o = gld_at(s.oS[a.ocur]);
    if (!o.done && o.status == 0) {
      const double ref = s.octl.stop_rule == 1 ? o.delta0 : o.delta_b;
      const double need = o.delta > 0.0 ? 0.5 * sqrt(s.octl.rtol2 * ref / o.delta) : 1.0;
      const double irt = fmin(0.5, fmax(s.inner_rtol, need));
      R.mode = M_START;
      R.ctl.rtol2 = irt * irt;
    }
  }
  inner_start_body(s.r64, s.rhs32, s.r32, s.e32[0], s.pinv32, s.N, R, local, s.nblk[PK_START]);
}

static __global__ void __launch_bounds__(256) inner_start_batch_kernel(BatchArgs a) {
  uint32_t sim, local;
  work_item(a, blockIdx.x, sim, local);
  inner_start_sim(a.sims[sim], a, local);
}

// The same for a launch with one simulation, whose record comes with the
// launch (so it is never copied to device memory; the bits are the same).
static __global__ void __launch_bounds__(256) inner_start_one_kernel(BatchArgs a, SimDev s) {
  inner_start_sim(s, a, blockIdx.x);
}

// Settles the pending decision of every simulation and copies the settled
// state to snap[sim] for the host.  Blocks follow the update kernel's layout
// (every block settles the same state; block 0 of a simulation writes it):
// a solve that finishes here after a plain update still owes the deferred
// x += alpha d, which the simulation's blocks apply.  V selects the relay
// and vectors: double the outer (FP64) solve, float the inner one.
template <typename V, bool kFour>
__device__ inline void decide_sim(const SimDev& s, const BatchArgs& a, uint32_t sim, uint32_t local) {
  constexpr bool inner = sizeof(V) == 4;
  const Relay R = inner ? inner_relay(s, a, M_DECIDE, false) : outer_relay(s, a, M_DECIDE, false);
  const StageIn in = stage_load(R);
  Scalars st;
  (void)stage_finish<kFour>(R, in, st, local == 0);
  if (local == 0 && threadIdx.x == 0) {
    if (a.seq) {
      // the host polls a.seq instead of waiting for the end of the kernel:
      // the state goes to host memory at system scope first, and once those
      // stores have completed, the sequence word that tells the host so
      static_assert(sizeof(Scalars) % 8 == 0, "the state moves as 8-byte words");
      uint64_t w[sizeof(Scalars) / 8];
      __builtin_memcpy(w, &st, sizeof(Scalars));
      uint64_t* p = reinterpret_cast<uint64_t*>(a.snap + sim);
#pragma unroll
      for (int k = 0; k < (int)(sizeof(Scalars) / 8); ++k)
        __hip_atomic_store(p + k, w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_store(a.seq + sim, a.seq_val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
      gst_at(a.snap + sim, st);
    }
  }
  if (a.corr && in.pending && st.done && st.status == 0) {
    if constexpr (inner)
      axpy_body<float>(s.e32[a.xpar], s.d32[dir_out(a)], (float)st.alpha, s.N, local, s.nblk[PK_UPD32]);
    else
      axpy_body<double>(s.X[a.xpar], s.d64[dir_out(a)], st.alpha, s.N, local, s.nblk[PK_UPD64]);
  }
}

template <typename V, bool kFour>
__global__ void __launch_bounds__(256) decide_batch_kernel(BatchArgs a) {
  uint32_t sim, local;
  work_item(a, blockIdx.x, sim, local);
  decide_sim<V, kFour>(a.sims[sim], a, sim, local);
}

// One simulation, its record in the launch arguments.
template <typename V, bool kFour>
__global__ void __launch_bounds__(256) decide_one_kernel(BatchArgs a, SimDev s) {
  decide_sim<V, kFour>(s, a, 0, blockIdx.x);
}

}  // namespace femheat
