// Time stepping of one simulation or of a batch of simulations (gfx950).
//
// Every implicit theta-scheme step (Sec. 3.1) is, per simulation: the
// right-hand side b = L T^{n-1} + dt*s_n*F (one gather, RHS epilogue), the
// initial guess and residual (one gather), then the iterations of
// Algorithm 1, two kernels each: the search-direction update fused into the
// operator apply (q = A d, d^T q -> alpha on the device; it also applies the
// previous iteration's x += alpha d at its own nodes) and the residual update
// with the preconditioned residual norm (delta, beta and the stop test on
// the device).  When i mod replace_every == 0 (50 in Algorithm 1) the update
// is a gather computing x += alpha d, r = b - A x instead.  The mixed form
// runs that loop in FP32 on A e = r64 inside FP64 refinement sweeps; the
// option FEM_ONE_REDUCTION runs the FP64 loop with one kernel per iteration.
//
// The paper's host read the residual back every iteration (App. A.3).  Here
// the scalars of Algorithm 1 and the convergence decision live on the device
// and are relayed from kernel to kernel (reduce.hpp): once a solve is done,
// every further iteration kernel returns immediately.  The host enqueues
// iterations in chunks (the previous step's count, then 2, then 4), ends a
// chunk with a decide kernel that writes one pinned, mapped state block per
// simulation, and waits for that kernel alone: with one simulation, the next
// step's RHS and initial residual are already queued behind it and run on
// the device if the solve has ended, so the GPU works through the host's
// round trip.
//
// The engine advances every simulation it holds in lockstep, one step per
// epoch, with batched launches (batch.hpp): one launch of each kernel serves
// all simulations, each block working for one of them.  A single run is the
// batch of one.  Between epochs, finished simulations leave the batch.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <type_traits>
#include <vector>

#include <hip/hip_ext.h>

#include "batch.hpp"
#include "dirupd.hpp"
#include "engine.hpp"
#include "runtime.hpp"
#include "tune.hpp"

namespace femheat {
namespace {

double schedule_value(const fem_heat* h, int64_t m) {
  if (h->sched.empty()) return 1.0;
  if (m < 1 || m > (int64_t)h->sched.size()) return 0.0;
  return h->sched[(size_t)(m - 1)];
}

// Residual replacements among iterations 0..j-1 of a solve (i mod R == 0).
int replacements_before(int j, int R) { return (R <= 0 || j <= 0) ? 0 : (j - 1) / R + 1; }

}  // namespace

// Host state of one simulation of the engine.
struct Sim {
  RunRequest rq{};
  int status = FEM_OK;
  bool finished = false;
  int32_t step = 0;   // steps completed
  int32_t first = 0;  // global index of the step before the run's first step
  double* T1 = nullptr;
  double* T2 = nullptr;
  double* X[2] = {nullptr, nullptr};
  int32_t nsens = 0;
  std::vector<int32_t> iters, sweeps;
  std::vector<double> relres;
  int64_t total = 0;
  int est = 8;  // FP64 solve: first chunk of the next step (this step's count)
  // mixed form: first chunk of refinement sweep k of the next step (sweep k's
  // count in the latest step that ran it; the last entry serves later sweeps)
  int est_sw[4] = {8, 2, 2, 2};
  // within the current step
  int32_t it = 0, nsw = 0, xc = 0, exc = 0;
  bool sweeping = false, broke = false;
  Scalars so{}, si{};  // latest settled outer and inner state
};

namespace {

// A set of simulations launched together: one kernel per gather for the
// cubic and one for the general-element members.
struct Group {
  int kind = kElemCubic;  // element kind of the group's simulations (the gather's template argument)
  uint32_t off = 0, nwork = 0, nthreads = 64;
  size_t smem64 = 0, smem32 = 0, smem64f = 0, smem32f = 0;  // *f: one-reduction direction kernels (three planes)
};

// Work-table layout of a batched launch: where each kernel kind's entries
// start in the table and how many there are.
struct Layout {
  Group groups[3];
  int ngroups = 0;
  uint32_t off_upd64 = 0, n_upd64 = 0, off_upd32 = 0, n_upd32 = 0, off_start = 0, n_start = 0, off_one = 0,
           n_one = 0;
};

}  // namespace

class Engine {
 public:
  Engine(hipStream_t stream, const fem_opts& o, fem_heat* err) : stream_(stream), opts_(o), h_(err) {
    mixed_ = o.precision == FEM_FP32_FP64DOT;
    timing_ = (o.flags & FEM_TIMING) != 0;
    fused_ = !mixed_ && (o.flags & FEM_ONE_REDUCTION) != 0;
    ifused_ = mixed_ && (o.flags & FEM_ONE_REDUCTION) != 0;
    cheb_ = !mixed_ && !fused_ && o.precond == FEM_PRECOND_CHEBYSHEV;
    R_ = o.replace_every;
    dirupd_ = false;
  }
  void allow_one_kernel(bool on) {
    dirupd_ = on && (opts_.flags & FEM_ONE_KERNEL) != 0;
    if (const char* v = std::getenv("FEMHEAT_BARRIER_SPIN_LIMIT")) bar_spin_ = (uint32_t)std::strtoul(v, nullptr, 10);
  }
  ~Engine() {
    (void)hipStreamSynchronize(stream_);
    efree(bar_count_);
    if (bar_fail_host_) (void)hipHostFree(bar_fail_host_);
    efree(sd_dev_);
    efree(tab_dev_);
    for (auto& p : sd_host_)
      if (p) (void)hipHostFree(p);
    if (snap_host_) (void)hipHostFree(snap_host_);
    if (tab_host_) (void)hipHostFree(tab_host_);
    for (auto e : ev_) (void)hipEventDestroy(e);
    if (ev_decide_) (void)hipEventDestroy(ev_decide_);
    for (const Timed& t : pending_)
      for (hipEvent_t e : t.e)
        if (e) (void)hipEventDestroy(e);
    for (auto e : ev_run_)
      if (e) (void)hipEventDestroy(e);
  }

  int add(const RunRequest& r, Sim** out = nullptr);
  int tune(fem_heat* h, double dt, double theta, bool batch, fem_tune_result* out);
  // The engine's own device buffers, on its stream and through its allocator.
  template <typename T>
  int ealloc(T** p, size_t n) {
    void* v = nullptr;
    if (!dev_alloc(opts_.allocator, stream_, &v, std::max<size_t>(n, 1) * sizeof(T))) {
      *p = nullptr;
      return fail(h_, FEM_ENOMEM, "device allocation of the engine's tables failed");
    }
    *p = static_cast<T*>(v);
    return FEM_OK;
  }
  template <typename T>
  void efree(T*& p) {
    dev_free(opts_.allocator, stream_, p);
    p = nullptr;
  }
  int run();
  int step(int* active);
  int write_outputs(Sim& s, float ms);
  void remove(Sim* s);
  std::vector<std::unique_ptr<Sim>>& sims() { return sims_; }
  fem_stats stats{};

 private:
  int compose();
  int upload_simdev();
  void fill_simdev(const Sim& s, SimDev& d) const;
  BatchArgs args(int cur, int prev, int j, int xpar, int corr = 0) const {
    BatchArgs a{sd_dev_, nullptr, snap_map_, cur, prev, j, xpar, corr, UpdView{}, ocur_, 0, R_, 0.0};
    return a;
  }
  // Whether the update of iteration jj - 1 was a plain one, whose x += alpha d
  // the direction kernel of iteration jj (or the decide after it) applies.
  bool deferred(int jj) const { return jj > 0 && !(R_ > 0 && (jj - 1) % R_ == 0); }
  // Launches; e0/e1 (optional) are recorded at the start of the first and the
  // end of the last kernel of the launch by the dispatch itself.
  template <class Role>
  int gather(BatchArgs a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
  template <typename V>
  int update(BatchArgs a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
  // One iteration in one kernel with a grid-wide barrier (dirupd.hpp): a
  // single simulation whose gather fits the device at once.  *done = false:
  // not possible here (the caller launches the two kernels).
  template <typename V>
  int dirupd(BatchArgs a, hipEvent_t e0, hipEvent_t e1, bool* done);
  int check_barrier();
  int decide(bool inner, int j_end = 0, bool launch_next = false, bool wait = true, int slot = 0);
  // The next step's RHS and initial residual launched behind a decide (one
  // simulation): set when they ran, so the next epoch does not launch them.
  bool next_ran_ = false;
  const Sim* next_sim_ = nullptr;
  hipEvent_t ev_decide_ = nullptr;  // the host waits for the decide only, not what follows it
  template <typename V>
  int pcg(int first_chunk);
  int epoch();
  int mixed_sweeps();
  int finish_step(Sim& s);
  // Timing of sampled iterations: events come from a pool; a chunk's records
  // are read while the GPU runs a later chunk, not at the chunk boundary,
  // where the GPU waits for the host.
  struct Timed {
    hipEvent_t e[4];  // direction kernel start/end, update or replacement start/end
    bool gather;      // the direction kernel is in the sample
    int kind;         // 0: no second kernel timed, 1: update, 2: replacement
    bool one;         // the direction kernel also did the update (one-kernel iteration)
  };
  hipEvent_t take_event();
  int flush_timing();
  std::vector<Timed> pending_;

  hipStream_t stream_;
  fem_opts opts_;
  fem_heat* h_;  // receives error messages
  bool mixed_ = false, timing_ = false;
  bool fused_ = false;   // FP64 PCG in the one-reduction form
  bool ifused_ = false;  // the FP32 inner solves of the mixed form in the one-reduction form
  bool cheb_ = false;   // FP64 PCG with the Chebyshev preconditioner
  // The preconditioner chain behind the kernel that made a residual (or the
  // right-hand side): m - 1 gathers computing s = M^-1 r_in, the last one
  // publishing r_in^T s for the scalar update that kernel left pending.
  int cheb_chain(bool rhs) {
    if (!cheb_) return FEM_OK;
    const int m = opts_.cheb_degree;
    for (int k = 1; k <= m - 1; ++k) {
      BatchArgs a = args(ocur_, oprev_, 0, 0);
      a.cheb_k = k;
      a.cheb_last = k == m - 1 ? 1 : 0;
      a.cheb_rhs = rhs ? 1 : 0;
      if (k == 1)
        RC_TRY(gather<RoleChebFirst>(a));
      else
        RC_TRY(gather<RoleChebNext>(a));
      ocur_ ^= 1;
      oprev_ = PK_GATHER;
    }
    return FEM_OK;
  }
  int R_ = 50;
  uint64_t sample_ctr_ = 0;         // iterations launched with timing, across solves
  uint64_t replace_ctr_ = 0;        // residual replacements launched with timing

  std::vector<std::unique_ptr<Sim>> sims_;
  std::vector<Sim*> act_;  // simulations of the current epoch, in SimDev order
  bool dirty_ = true;      // membership changed since the last composition
  bool multi_ = false;     // more than one simulation: launches go through work tables

  SimDev* sd_dev_ = nullptr;
  SimDev sd_one_{};  // host copy of the uploaded SimDev when the batch holds one simulation
  // one-kernel iterations (FEM_ONE_KERNEL, runs of one handle); the grid-wide
  // barrier's arrival counter followed by one flag per block (bar_blocks_ of
  // them), its failure flag, and the arrivals so far
  bool dirupd_ = false;
  unsigned long long* bar_count_ = nullptr;
  uint32_t bar_blocks_ = 0;
  // the failure flag in mapped pinned host memory: the host reads it after
  // every chunk's decide without a copy (bar_fail_: its device address)
  int32_t* bar_fail_host_ = nullptr;
  int32_t* bar_fail_ = nullptr;
  unsigned long long bar_total_ = 0;
  // polls before a barrier wait gives up: kBarSpinLimit, or
  // FEMHEAT_BARRIER_SPIN_LIMIT from the environment (tests of the failure path)
  uint32_t bar_spin_ = kBarSpinLimit;
  int dirupd_cap_[2] = {-1, -1};  // blocks the device holds at once (FP64, FP32), -1: not yet asked
  size_t dirupd_cap_smem_[2] = {0, 0};
  SimDev* sd_host_[2] = {nullptr, nullptr};  // pinned staging, used alternately
  int sd_flip_ = 0;
  size_t sd_cap_ = 0;
  Scalars* snap_host_ = nullptr;  // pinned, coherent: the decide kernel writes it directly
  Scalars* snap_map_ = nullptr;   // its device address
  size_t snap_cap_ = 0;
  // after the snapshots, in the same allocation: one sequence word per
  // snapshot, which a decide of one simulation writes once its snapshot is in
  // host memory (the host polls it: see wait_decide)
  uint32_t* seq_host_ = nullptr;
  uint32_t* seq_map_ = nullptr;
  uint32_t dseq_ = 0;  // the last sequence number given to a decide
  int wait_decide(const volatile uint32_t* seq, uint32_t want);
  uint2* tab_dev_ = nullptr;
  uint2* tab_host_ = nullptr;
  size_t tab_cap_ = 0;

  // The table of the epoch (region 0 of tab_dev_) and, within a PCG solve of
  // a batch, compactions of it that leave out the simulations whose solve is
  // done (regions 1 and 2, used alternately): a lockstep batch then stops
  // launching blocks for members that only wait for the slowest one.
  Layout full_, lay_;
  const uint2* tab_cur_ = nullptr;
  int ctab_flip_ = 0;
  size_t live_count_ = 0;
  void build_layout(const std::vector<char>& live, std::vector<uint2>& tab, Layout& L) const;
  int compact(const std::vector<char>& live);
  void uncompact() {
    lay_ = full_;
    tab_cur_ = tab_dev_;
    live_count_ = act_.size();
  }

  // relay parity and the kind of partials the next kernel reads, per relay
  int ocur_ = 0, oprev_ = PK_GATHER, icur_ = 0, iprev_ = PK_GATHER;

  std::vector<hipEvent_t> ev_;
  hipEvent_t ev_run_[2] = {nullptr, nullptr};
};

hipEvent_t Engine::take_event() {
  hipEvent_t e = nullptr;
  if (!ev_.empty()) {
    e = ev_.back();
    ev_.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Reads every pending record (their events have completed: each was followed
// by a decide the host has waited for) and returns the events to the pool.
int Engine::flush_timing() {
  fem_heat* h = h_;
  for (const Timed& t : pending_) {
    float ms = 0.f;
    if (t.gather) {
      HIP_TRY(hipEventElapsedTime(&ms, t.e[0], t.e[1]));
      stats.gather_launches += 1;
      stats.gather_ms += ms;
      if (t.one) stats.one_kernel_launches += 1;
    }
    if (t.kind != 0) {
      HIP_TRY(hipEventElapsedTime(&ms, t.e[2], t.e[3]));
      if (t.kind == 2) {
        stats.replace_launches += 1;
        stats.replace_ms += ms;
      } else {
        stats.update_launches += 1;
        stats.update_ms += ms;
      }
    }
    for (hipEvent_t e : t.e)
      if (e) ev_.push_back(e);
  }
  pending_.clear();
  return FEM_OK;
}

// Set-up of one simulation: operator for its theta*dt, fields, sensors.
int Engine::add(const RunRequest& r, Sim** out) {
  fem_heat* h = r.h;
  auto sp = std::make_unique<Sim>();
  Sim& s = *sp;
  s.rq = r;
  const uint32_t N = h->g.N;
  RC_TRY(prepare_operator(h, r.theta * r.dt, mixed_));
  s.T1 = h->pool[0];
  s.T2 = h->pool[1];
  s.X[0] = h->pool[2];
  s.X[1] = h->pool[3];
  RC_TRY(copy_in(h, s.T1, r.T0, N));
  RC_TRY(copy_in(h, s.T2, r.T_prev ? r.T_prev : r.T0, N));
  hipLaunchKernelGGL((apply_dirichlet_kernel<double>), dim3(nblk(N)), dim3(kT), 0, stream_, h->g, s.T1);
  hipLaunchKernelGGL((apply_dirichlet_kernel<double>), dim3(nblk(N)), dim3(kT), 0, stream_, h->g, s.T2);
  // the first direction of every solve has beta = 0, but 0 * d must be 0
  for (int k = 0; k < 2; ++k)
    hipLaunchKernelGGL((fill_kernel<double>), dim3(nblk(N)), dim3(kT), 0, stream_, h->d64[k], 0.0, N);
  if (mixed_)
    for (int k = 0; k < 2; ++k)
      hipLaunchKernelGGL((fill_kernel<float>), dim3(nblk(N)), dim3(kT), 0, stream_, h->d32[k], 0.0f, N);
  HIP_TRY(hipGetLastError());
  const fem_out* o = r.out;
  s.first = o ? o->first_step : 0;
  s.nsens = (o && o->sensor_xyz && o->n_sensors > 0) ? o->n_sensors : 0;
  if (s.nsens > 0) {
    if (h->xyz_cap < (size_t)s.nsens) {
      dfree(h, h->xyz_dev);
      RC_TRY(dalloc(h, &h->xyz_dev, 3 * (size_t)s.nsens));
      h->xyz_cap = s.nsens;
    }
    RC_TRY(copy_in(h, h->xyz_dev, o->sensor_xyz, 3 * (size_t)s.nsens));
    const size_t need = (size_t)std::max(r.nsteps, 1) * s.nsens;
    if (h->traces_cap < need) {
      dfree(h, h->traces_dev);
      RC_TRY(dalloc(h, &h->traces_dev, need));
      h->traces_cap = need;
    }
  }
  const size_t ns = (size_t)std::max(r.nsteps, 0);
  s.iters.assign(ns, 0);
  s.sweeps.assign(ns, 0);
  s.relres.assign(ns, 0.0);
  s.finished = r.nsteps <= 0;
  if (out) *out = sp.get();
  sims_.push_back(std::move(sp));
  dirty_ = true;
  return FEM_OK;
}

void Engine::remove(Sim* s) {
  next_ran_ = false;  // a later simulation may be allocated where this one was
  next_sim_ = nullptr;
  for (size_t i = 0; i < sims_.size(); ++i)
    if (sims_[i].get() == s) {
      sims_.erase(sims_.begin() + (long)i);
      dirty_ = true;
      return;
    }
}

void Engine::fill_simdev(const Sim& s, SimDev& d) const {
  const fem_heat* h = s.rq.h;
  const double dt = s.rq.dt, theta = s.rq.theta;
  std::memset(&d, 0, sizeof(d));
  d.A64 = gather_args<double>(h, 1.0, theta * dt);
  d.L64 = gather_args<double>(h, 1.0, -(1.0 - theta) * dt);
  if (mixed_) d.A32 = gather_args<float>(h, 1.0, theta * dt);
  d.F64 = h->F64;
  d.pinv64 = h->pinv64;
  d.lift64 = h->lift64;
  d.b64 = h->b64;
  d.r64 = h->r64;
  d.q64 = h->q64;
  d.r64b = h->r64b ? h->r64b : h->r64;
  d.q64b = h->q64b ? h->q64b : h->q64;
  d.ldp = h->n_partials;
  d.d64[0] = h->d64[0];
  d.d64[1] = h->d64[1];
  d.T1 = s.T1;
  d.T2 = s.T2;
  d.X[0] = s.X[0];
  d.X[1] = s.X[1];
  d.pinv32 = h->pinv32;
  d.r32 = h->r32;
  d.q32 = h->q32;
  d.r32b = h->r32b ? h->r32b : h->r32;
  d.q32b = h->q32b ? h->q32b : h->q32;
  d.d32[0] = h->d32[0];
  d.d32[1] = h->d32[1];
  d.e32[0] = h->e32[0];
  d.e32[1] = h->e32[1];
  d.rhs32 = h->rhs32;
  for (int k = 0; k < 2; ++k) {
    d.oS[k] = h->outer.S[k];
    d.oP[k] = h->outer.P[k];
    d.iS[k] = h->inner.S[k];
    d.iP[k] = h->inner.P[k];
  }
  d.octl = Ctl{s.rq.rtol * s.rq.rtol, opts_.max_iter, opts_.stop_rule};
  // the inner tolerance comes from the settled outer state, in the inner
  // start kernel (see inner_start_batch_kernel): one sweep then usually suffices
  d.ictl = Ctl{-1.0, opts_.max_iter, FEM_STOP_INITIAL};
  d.inner_rtol = opts_.inner_rtol;
  d.s64 = h->s64;
  d.cr64 = h->cr64;
  d.cd64[0] = h->cd64[0];
  d.cd64[1] = h->cd64[1];
  d.ch_inv_c = h->ch_inv_c;
  for (int k = 0; k < kChebMaxDegree; ++k) {
    d.ch_a[k] = h->ch_a[k];
    d.ch_b[k] = h->ch_b[k];
  }
  d.N = h->g.N;
  d.nblk[PK_GATHER] = h->shape.nblocks;
  d.nblk[PK_UPD64] = h->upd_blocks64;
  d.nblk[PK_UPD32] = h->upd_blocks32;
  d.nblk[PK_START] = h->start_blocks;
  d.fs = dt * schedule_value(h, (int64_t)s.first + s.step + 1);
  d.guess_prev = opts_.guess == FEM_GUESS_PREV ? 1 : 0;
  d.xc = s.xc;
  d.exc = s.exc;
  d.sweep = s.sweeping ? 1 : 0;
}

// Copies the SimDev array of the current epoch to the device.  Callers only
// do so after waiting for a decide launched after the previous copy, so the
// staging buffer being written is never still in use.  A batch of one
// simulation needs no copy: every kernel launched for it takes its record
// (sd_one_, as filled here) with the launch arguments.
int Engine::upload_simdev() {
  fem_heat* h = h_;
  if (!multi_ && act_.size() == 1) {
    fill_simdev(*act_[0], sd_one_);
    return FEM_OK;
  }
  SimDev* stage = sd_host_[sd_flip_];
  sd_flip_ ^= 1;
  for (size_t k = 0; k < act_.size(); ++k) fill_simdev(*act_[k], stage[k]);
  if (act_.size() == 1) sd_one_ = stage[0];
  HIP_TRY(hipMemcpyAsync(sd_dev_, stage, act_.size() * sizeof(SimDev), hipMemcpyHostToDevice, stream_));
  return FEM_OK;
}

// The simulations that still have steps to run form the next epoch's batch;
// rebuilds the launch groups and work tables when that set changed.
int Engine::compose() {
  fem_heat* h = h_;
  std::vector<Sim*> next;
  for (auto& sp : sims_)
    if (!sp->finished) next.push_back(sp.get());
  if (!dirty_ && next == act_ && full_.ngroups > 0) return FEM_OK;
  dirty_ = false;
  HIP_TRY(hipStreamSynchronize(stream_));  // buffers below may be freed or rewritten
  act_ = next;
  const size_t n = act_.size();
  if (n == 0) return FEM_OK;
  multi_ = n > 1;
  // capacities grow geometrically: freeing pinned host memory synchronises
  // the whole device (every stream, other servers' lanes included)
  auto grow = [](size_t cap, size_t need) { return std::max<size_t>({need, 2 * cap, 16}); };
  if (sd_cap_ < n) {
    const size_t cap = grow(sd_cap_, n);
    efree(sd_dev_);
    for (auto& p : sd_host_)
      if (p) (void)hipHostFree(p);
    sd_host_[0] = sd_host_[1] = nullptr;
    sd_cap_ = 0;
    RC_TRY(ealloc(&sd_dev_, cap));
    for (auto& p : sd_host_) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&p), cap * sizeof(SimDev), hipHostMallocDefault));
    sd_cap_ = cap;
  }
  if (snap_cap_ < n) {  // two slots per simulation (see decide)
    const size_t cap = grow(snap_cap_, n);
    if (snap_host_) (void)hipHostFree(snap_host_);
    snap_host_ = snap_map_ = nullptr;
    seq_host_ = seq_map_ = nullptr;
    snap_cap_ = 0;
    const size_t bytes = 2 * cap * (sizeof(Scalars) + sizeof(uint32_t));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&snap_host_), bytes, hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&snap_map_), snap_host_, 0));
    std::memset(static_cast<void*>(snap_host_), 0, bytes);  // sequence numbers start above 0
    seq_host_ = reinterpret_cast<uint32_t*>(snap_host_ + 2 * cap);
    seq_map_ = reinterpret_cast<uint32_t*>(snap_map_ + 2 * cap);
    snap_cap_ = cap;
  }
  std::vector<uint2> tab;
  build_layout(std::vector<char>(n, 1), tab, full_);
  // the batched kernels are built for blocks of at most 256 threads (the
  // wider blocks of a simulation alone run only in the one-simulation kernels)
  if (multi_)
    for (int gi = 0; gi < full_.ngroups; ++gi)
      if (full_.groups[gi].nthreads > (uint32_t)kMaxBatchThreads)
        return fail(h_, FEM_EINVAL, "a batched launch with blocks of more than 256 threads");
  lay_ = full_;
  live_count_ = n;
  if (multi_) {
    // region 0: this table; regions 1 and 2: compactions (at most as long)
    if (tab_cap_ < tab.size()) {
      const size_t cap = grow(tab_cap_, tab.size());
      efree(tab_dev_);
      if (tab_host_) (void)hipHostFree(tab_host_);
      tab_host_ = nullptr;
      tab_cap_ = 0;
      RC_TRY(ealloc(&tab_dev_, 3 * cap));
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&tab_host_), 3 * cap * sizeof(uint2), hipHostMallocDefault));
      tab_cap_ = cap;
    }
    std::memcpy(tab_host_, tab.data(), tab.size() * sizeof(uint2));
    HIP_TRY(hipMemcpyAsync(tab_dev_, tab_host_, tab.size() * sizeof(uint2), hipMemcpyHostToDevice, stream_));
  }
  tab_cur_ = tab_dev_;
  return FEM_OK;
}

// Launch groups by element class and the entries of every kernel kind, for
// the simulations of the epoch marked live (table entries name a simulation
// by its index in the epoch, so a compaction keeps the SimDev array).
void Engine::build_layout(const std::vector<char>& live, std::vector<uint2>& tab, Layout& L) const {
  const size_t n = act_.size();
  L = Layout{};
  for (int cls : {kElemCubic, kElemBox, kElemTet6}) {
    Group g;
    g.kind = cls;
    g.off = (uint32_t)tab.size();
    for (size_t k = 0; k < n; ++k) {
      const fem_heat* sh = act_[k]->rq.h;
      if (sh->kind != g.kind) continue;
      // launch parameters from every member of the class, live or not, so a
      // compaction launches the same block shape and LDS size
      g.nthreads = std::max<uint32_t>(g.nthreads, (uint32_t)sh->shape.nthreads);
      g.smem64 = std::max(g.smem64, sh->shape.smem_bytes(8));
      g.smem32 = std::max(g.smem32, sh->shape.smem_bytes(4));
      g.smem64f = std::max(g.smem64f, sh->shape.smem_bytes(8, 3));
      g.smem32f = std::max(g.smem32f, sh->shape.smem_bytes(4, 3));
      if (!live[k]) continue;
      for (uint32_t b = 0; b < sh->shape.nblocks; ++b) tab.push_back(make_uint2((uint32_t)k, b));
    }
    g.nwork = (uint32_t)tab.size() - g.off;
    if (g.nwork > 0) L.groups[L.ngroups++] = g;
  }
  auto add_kind = [&](uint32_t fem_heat::*count, uint32_t& off, uint32_t& total) {
    off = (uint32_t)tab.size();
    for (size_t k = 0; k < n; ++k) {
      if (!live[k]) continue;
      const fem_heat* sh = act_[k]->rq.h;
      for (uint32_t b = 0; b < sh->*count; ++b) tab.push_back(make_uint2((uint32_t)k, b));
    }
    total = (uint32_t)tab.size() - off;
  };
  add_kind(&fem_heat::upd_blocks64, L.off_upd64, L.n_upd64);
  add_kind(&fem_heat::upd_blocks32, L.off_upd32, L.n_upd32);
  add_kind(&fem_heat::start_blocks, L.off_start, L.n_start);
  L.off_one = (uint32_t)tab.size();  // one block per simulation (decides that owe no x += alpha d)
  for (size_t k = 0; k < n; ++k)
    if (live[k]) tab.push_back(make_uint2((uint32_t)k, 0u));
  L.n_one = (uint32_t)tab.size() - L.off_one;
}

// Launches from here on serve only the live simulations.  The others' relay
// state is left as their last kernel wrote it: they take no part until the
// layout is restored, and the next kernel that does serve them starts a new
// solve (the right-hand side of a step, the start of an inner solve, a
// refinement correction), which resets what it reads.  Their settled state
// stays in the host snapshot, which later decides do not rewrite.
int Engine::compact(const std::vector<char>& live) {
  fem_heat* h = h_;
  std::vector<uint2> tab;
  Layout L;
  build_layout(live, tab, L);
  ctab_flip_ ^= 1;
  const size_t region = (size_t)(1 + ctab_flip_) * tab_cap_;
  // the staging region was last copied two compactions ago, before a decide
  // the host has waited for since
  std::memcpy(tab_host_ + region, tab.data(), tab.size() * sizeof(uint2));
  HIP_TRY(hipMemcpyAsync(tab_dev_ + region, tab_host_ + region, tab.size() * sizeof(uint2), hipMemcpyHostToDevice,
                         stream_));
  lay_ = L;
  tab_cur_ = tab_dev_ + region;
  live_count_ = 0;
  for (char c : live) live_count_ += c ? 1 : 0;
  return FEM_OK;
}

template <class Role>
int Engine::gather(BatchArgs a, hipEvent_t e0, hipEvent_t e1) {
  fem_heat* h = h_;
  for (int gi = 0; gi < lay_.ngroups; ++gi) {
    const Group& g = lay_.groups[gi];
    a.table = multi_ ? tab_cur_ + g.off : nullptr;
    const size_t smem = std::is_same<Role, RoleFused>::value     ? g.smem64f
                        : std::is_same<Role, RoleFused32>::value ? g.smem32f
                        : sizeof(typename Role::V) == 8          ? g.smem64
                                                                 : g.smem32;
    hipEvent_t s0 = gi == 0 ? e0 : nullptr, s1 = gi == lay_.ngroups - 1 ? e1 : nullptr;
    if (!multi_) {  // one simulation: its record (sd_one_, as uploaded) goes into the launch
      const auto ga = Role::ga(sd_one_);
      const auto pro = Role::pro(sd_one_, a);
      const auto epi = Role::epi(sd_one_, a);
      const Relay R = Role::relay(sd_one_, a);
      if (g.kind == kElemCubic)
        hipExtLaunchKernelGGL((gather_one_kernel<kElemCubic, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                              s0, s1, 0, ga, pro, epi, R);
      else if (g.kind == kElemTet6)
        hipExtLaunchKernelGGL((gather_one_kernel<kElemTet6, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                              s0, s1, 0, ga, pro, epi, R);
      else
        hipExtLaunchKernelGGL((gather_one_kernel<kElemBox, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                              s0, s1, 0, ga, pro, epi, R);
      continue;
    }
    if (g.kind == kElemCubic)
      hipExtLaunchKernelGGL((gather_batch_kernel<kElemCubic, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                            s0, s1, 0, a);
    else if (g.kind == kElemTet6)
      hipExtLaunchKernelGGL((gather_batch_kernel<kElemTet6, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                            s0, s1, 0, a);
    else
      hipExtLaunchKernelGGL((gather_batch_kernel<kElemBox, Role>), dim3(g.nwork), dim3(g.nthreads), smem, stream_,
                            s0, s1, 0, a);
  }
  HIP_TRY(hipGetLastError());
  return FEM_OK;
}

template <typename V>
int Engine::dirupd(BatchArgs a, hipEvent_t e0, hipEvent_t e1, bool* done) {
  fem_heat* h = h_;
  *done = false;
  if (lay_.ngroups != 1) return FEM_OK;
  const Group& g = lay_.groups[0];
  constexpr bool f64 = sizeof(V) == 8;
  const int kind = g.kind;
  const void* fn = kind == kElemCubic  ? reinterpret_cast<const void*>(&dirupd_kernel<kElemCubic, V>)
                   : kind == kElemTet6 ? reinterpret_cast<const void*>(&dirupd_kernel<kElemTet6, V>)
                                       : reinterpret_cast<const void*>(&dirupd_kernel<kElemBox, V>);
  const SimDev& s = sd_one_;
  using Role = RoleDir<V>;
  GatherArgs<V> ga = Role::ga(s);
  // LDS: the gather's planes and coefficient tiles, then q, r and P^-1 (and,
  // in FP32, d and x) at the block's own nodes
  const uint32_t lds_base = (uint32_t)((f64 ? g.smem64 : g.smem32) + 255) / 256 * 256;
  const size_t smem = lds_base + (size_t)ga.s.tz * g.nthreads * sizeof(V) * (f64 ? 3 : 5);
  int& cap = dirupd_cap_[f64 ? 0 : 1];
  if (cap < 0 || dirupd_cap_smem_[f64 ? 0 : 1] != smem) {
    int per_cu = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)g.nthreads, smem));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->opts.device));
    cap = per_cu * cus;
    dirupd_cap_smem_[f64 ? 0 : 1] = smem;
  }
  if ((int)g.nwork > cap || smem > 160 * 1024) return FEM_OK;  // not every block at once: two kernels
  if (bar_blocks_ < g.nwork) {  // (re)start the barrier: counter and flags at 0
    efree(bar_count_);
    bar_count_ = nullptr;
    bar_blocks_ = 0;
    const size_t words = (size_t)kBarFlagStride * (1 + g.nwork);
    RC_TRY(ealloc(&bar_count_, words));
    if (!bar_fail_host_) {
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&bar_fail_host_), sizeof(int32_t),
                            hipHostMallocMapped | hipHostMallocCoherent));
      *bar_fail_host_ = 0;
      HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&bar_fail_), bar_fail_host_, 0));
    }
    HIP_TRY(hipMemsetAsync(bar_count_, 0, words * sizeof(unsigned long long), stream_));
    bar_blocks_ = g.nwork;
    bar_total_ = 0;
  }
  ProDirection<V> pro = Role::pro(s, a);
  Relay R = Role::relay(s, a);
  UpdHalf<V> u{};
  const V* pinv = nullptr;
  if constexpr (f64) {
    u = UpdHalf<V>{s.r64, nullptr, s.oS[a.cur], s.oP[a.cur]};
    pinv = s.pinv64;
  } else {
    u = UpdHalf<V>{s.r32, s.e32[a.xpar], s.iS[a.cur], s.iP[a.cur]};
    pinv = s.pinv32;
  }
  bar_total_ += g.nwork;
  GridBar gb{bar_count_, bar_count_ + kBarFlagStride, bar_fail_, bar_total_, bar_spin_};
  uint32_t lb = lds_base;
  void* kargs[] = {&ga, &pro, &R, &u, &pinv, &gb, &lb};
  if (e0) HIP_TRY(hipEventRecord(e0, stream_));
  // A plain launch: a cooperative one would guarantee that every block is
  // resident, but costs about 14 us more per launch here (measured).  The
  // grid was checked against the device's occupancy above; work that other
  // streams or processes run at the same time can still hold CUs, and then
  // the barrier's bounded wait runs out and the run fails (FEM_ONE_KERNEL
  // is an option for that reason).
  HIP_TRY(hipLaunchKernel(fn, dim3(g.nwork), dim3(g.nthreads), kargs, (unsigned int)smem, stream_));
  if (e1) HIP_TRY(hipEventRecord(e1, stream_));
  *done = true;
  return FEM_OK;
}

// A grid-wide barrier that ran out of time leaves its launch's results void:
// the run fails (checked after every chunk's decide, when the stream has
// drained up to it), and the counter starts over.
int Engine::check_barrier() {
  fem_heat* h = h_;
  if (!bar_fail_host_ || *reinterpret_cast<volatile int32_t*>(bar_fail_host_) == 0) return FEM_OK;
  HIP_TRY(hipStreamSynchronize(stream_));
  HIP_TRY(hipMemsetAsync(bar_count_, 0, (size_t)kBarFlagStride * (1 + bar_blocks_) * sizeof(unsigned long long), stream_));
  HIP_TRY(hipStreamSynchronize(stream_));
  *bar_fail_host_ = 0;
  bar_total_ = 0;
  return fail(h, FEM_EDEVICE,
              "a grid-wide barrier of the one-kernel iteration timed out (other work on the device held "
              "some of its blocks back)");
}

template <typename V>
int Engine::update(BatchArgs a, hipEvent_t e0, hipEvent_t e1) {
  fem_heat* h = h_;
  const bool f64 = sizeof(V) == 8;
  a.table = multi_ ? tab_cur_ + (f64 ? lay_.off_upd64 : lay_.off_upd32) : nullptr;
  const dim3 grid(f64 ? lay_.n_upd64 : lay_.n_upd32);
  if (multi_) {
    hipExtLaunchKernelGGL((update_batch_kernel<V, false>), grid, dim3(kT), 0, stream_, e0, e1, 0, a);
  } else {  // the same vectors and relay as the SimDev would give (outer_relay, inner_relay)
    const SimDev& s = sd_one_;
    UpdView& u = a.uv;
    u.N = s.N;
    if (f64) {
      u.nblk = s.nblk[PK_UPD64];
      u.r = s.r64;
      u.q = s.q64;
      u.pinv = s.pinv64;
      u.R = Relay{s.oS[a.cur], s.oS[a.cur ^ 1], s.oP[a.cur], s.nblk[a.prev], s.oP[a.cur ^ 1], M_UPD, s.octl, s.ldp};
    } else {
      u.nblk = s.nblk[PK_UPD32];
      u.r = s.r32;
      u.q = s.q32;
      u.pinv = s.pinv32;
      u.x = s.e32[a.xpar];
      u.d = s.d32[(a.j + 1) & 1];  // the direction this iteration's gather wrote
      u.R = Relay{s.iS[a.cur], s.iS[a.cur ^ 1], s.iP[a.cur], s.nblk[a.prev], s.iP[a.cur ^ 1], M_UPD, s.ictl, s.ldp};
    }
    hipExtLaunchKernelGGL((update_batch_kernel<V, true>), grid, dim3(kT), 0, stream_, e0, e1, 0, a);
  }
  HIP_TRY(hipGetLastError());
  return FEM_OK;
}

// Settles the pending decision of every simulation of a relay and reads the
// settled states into snap_host_ (synchronises the stream).  j_end > 0: the
// relay's last kernel was the update of iteration j_end - 1 of a PCG chunk,
// and a solve that finishes here gets that update's deferred x += alpha d.
// launch_next: see below.  wait = false: the host does not wait (it reads
// the snapshot after a later decide); slot 1 writes the states to the second
// snapshot slot (snap_host_[n + q]), which later decides leave alone.
int Engine::decide(bool inner, int j_end, bool launch_next, bool wait, int slot) {
  fem_heat* h = h_;
  int& cur = inner ? icur_ : ocur_;
  int& prev = inner ? iprev_ : oprev_;
  const int jl = std::max(0, j_end - 1);
  // (nothing is owed by the one-reduction form, whose direction kernel
  // completes each update before the stop test, nor by the FP32 inner
  // solves of the two-kernel form, whose update kernel applies x += alpha d
  // itself)
  BatchArgs a = args(cur, prev, jl, replacements_before(jl, R_) & 1,
                     !inner && !fused_ && j_end > 0 && deferred(j_end) ? 1 : 0);
  if (slot) a.snap += act_.size();
  // one simulation: the host polls the decide's sequence word (wait_decide)
  const bool poll = wait && !multi_;
  a.seq = poll ? seq_map_ + (slot ? act_.size() : 0) : nullptr;
  a.seq_val = ++dseq_;
  // a decide that may owe x += alpha d runs over the update kernel's blocks,
  // which then share that work; otherwise one block per simulation settles it
  uint32_t grid;
  if (a.corr) {
    a.table = multi_ ? tab_cur_ + (inner ? lay_.off_upd32 : lay_.off_upd64) : nullptr;
    grid = inner ? lay_.n_upd32 : lay_.n_upd64;
  } else {
    a.table = multi_ ? tab_cur_ + lay_.off_one : nullptr;
    grid = lay_.n_one;
  }
  if (!multi_) {  // one simulation: its record goes into the launch
    if (inner && ifused_)
      hipLaunchKernelGGL((decide_one_kernel<float, true>), dim3(grid), dim3(kT), 0, stream_, a, sd_one_);
    else if (inner)
      hipLaunchKernelGGL((decide_one_kernel<float, false>), dim3(grid), dim3(kT), 0, stream_, a, sd_one_);
    else if (fused_)
      hipLaunchKernelGGL((decide_one_kernel<double, true>), dim3(grid), dim3(kT), 0, stream_, a, sd_one_);
    else
      hipLaunchKernelGGL((decide_one_kernel<double, false>), dim3(grid), dim3(kT), 0, stream_, a, sd_one_);
  } else if (inner && ifused_) {
    hipLaunchKernelGGL((decide_batch_kernel<float, true>), dim3(grid), dim3(kT), 0, stream_, a);
  } else if (inner) {
    hipLaunchKernelGGL((decide_batch_kernel<float, false>), dim3(grid), dim3(kT), 0, stream_, a);
  } else if (fused_) {
    hipLaunchKernelGGL((decide_batch_kernel<double, true>), dim3(grid), dim3(kT), 0, stream_, a);
  } else {
    hipLaunchKernelGGL((decide_batch_kernel<double, false>), dim3(grid), dim3(kT), 0, stream_, a);
  }
  HIP_TRY(hipGetLastError());
  cur ^= 1;
  if (!ev_decide_) HIP_TRY(hipEventCreateWithFlags(&ev_decide_, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev_decide_, stream_));
  // The next step's RHS and initial residual go in behind the decide, so the
  // GPU has work while the host waits for it and prepares the next launches;
  // on the device they run only if the solve ended well in the iterate
  // buffer assumed here (the one its iteration count so far gives).
  int next_xc = -1;
  if (launch_next) {
    const Sim& s = *act_[0];
    // FP64 solve: the buffer its iteration count gives (replacements mod 2);
    // mixed form: the one the sweep's correction just wrote
    next_xc = mixed_ ? s.xc : replacements_before(j_end, R_) & 1;
    BatchArgs b = args(ocur_, oprev_, 0, 0);
    b.next_xc = next_xc;
    if (mixed_) b.next_R = -1;
    b.next_fs = s.rq.dt * schedule_value(s.rq.h, (int64_t)s.first + s.step + 2);
    RC_TRY(gather<RoleRhsNext>(b));
    ocur_ ^= 1;
    oprev_ = PK_GATHER;
    b.cur = ocur_;
    b.prev = oprev_;
    RC_TRY(gather<RoleInitNext>(b));
    ocur_ ^= 1;
  }
  if (poll)
    RC_TRY(wait_decide(seq_host_ + (slot ? act_.size() : 0), a.seq_val));
  else if (wait)
    HIP_TRY(hipEventSynchronize(ev_decide_));
  if (launch_next) {
    const Scalars& t = snap_host_[0];
    next_ran_ = t.done && t.status == 0 && (mixed_ || (replacements_before(t.iter, R_) & 1) == next_xc);
    next_sim_ = act_[0];
  }
  return FEM_OK;
}

// The host's wait for the decide of one simulation.  It polls the sequence
// word that the decide kernel writes once the snapshot is in host memory
// (the kernel and everything queued behind it may still be running: the host
// only reads the snapshot, and every later launch is ordered behind the
// decide on the stream).  Waiting for the kernel's completion signal instead
// takes the GPU's end-of-kernel work and the runtime's wake-up on top, while
// the GPU idles until the host's next launch.  The event is queried now and
// then, so a device error, or a kernel that ended without writing the word,
// also ends the wait.
int Engine::wait_decide(const volatile uint32_t* seq, uint32_t want) {
  fem_heat* h = h_;
  for (uint32_t spins = 1; *seq != want; ++spins) {
    if ((spins & 1023u) == 0) {
      const hipError_t q = hipEventQuery(ev_decide_);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) return fail(h, FEM_EDEVICE, std::string("decide kernel failed: ") + hipGetErrorString(q));
      (void)hipGetLastError();  // "not ready" is no error of a later call
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return FEM_OK;
}

// Iterations of Algorithm 1 for every simulation of the batch until all are
// done (FP64 outer solve, or FP32 inner solves of the mixed form).
template <typename V>
int Engine::pcg(int first_chunk) {
  fem_heat* h = h_;
  constexpr bool inner = sizeof(V) == 4;
  int& cur = inner ? icur_ : ocur_;
  int& prev = inner ? iprev_ : oprev_;
  const int upd_kind = inner ? PK_UPD32 : PK_UPD64;
  const bool one_red = inner ? ifused_ : fused_;  // one kernel per iteration (plus replacements)
  // Timing samples one iteration in kSampleEvery and one residual replacement
  // in kReplaceEvery, counted across solves so that the sample holds the
  // forms of the direction kernel (with or without the deferred update) in
  // their overall proportion, with events the dispatch itself records at the
  // start and end of each kernel.  Each timed launch still costs ~5 us of
  // GPU time between kernels (sampling every 8th iteration slowed the 1M-DOF
  // run by 4%), hence the sparse sample; marker events between every launch
  // would lengthen the run they time far more.
  constexpr int kSampleEvery = 64, kReplaceEvery = 8;
  auto replacing = [&](int jj) { return R_ > 0 && jj % R_ == 0; };
  int j = 0;
  int k = std::max(1, first_chunk);
  int chunks = 0;
  std::vector<Timed> recs;  // this chunk's sampled iterations (index c)
  std::vector<int> rec_c;
  for (;;) {
    recs.clear();
    rec_c.clear();
    for (int c = 0; c < k; ++c) {
      const int jj = j + c;
      const bool pick = timing_ && (sample_ctr_++ % kSampleEvery) == 0;
      const bool rep = replacing(jj);
      const bool pick_rep = rep && timing_ && (replace_ctr_++ % kReplaceEvery) == 0;
      Timed t{{nullptr, nullptr, nullptr, nullptr}, pick, pick_rep ? 2 : (pick && !rep && !one_red ? 1 : 0), false};
      if (timing_ && (t.gather || t.kind != 0)) {
        for (int q = 0; q < 4; ++q)
          if ((q < 2 && t.gather) || (q >= 2 && t.kind != 0)) {
            t.e[q] = take_event();
            if (!t.e[q]) return fail(h, FEM_EDEVICE, "hipEventCreate failed");
          }
        recs.push_back(t);
        rec_c.push_back(c);
      }
      const Timed* tr = recs.empty() || rec_c.back() != c ? nullptr : &recs.back();
      hipEvent_t e0 = tr ? tr->e[0] : nullptr, e1 = tr ? tr->e[1] : nullptr;
      hipEvent_t e2 = tr ? tr->e[2] : nullptr, e3 = tr ? tr->e[3] : nullptr;
      const int xpar = replacements_before(jj, R_) & 1;
      if (one_red) {
        if constexpr (inner)
          RC_TRY(gather<RoleFused32>(args(cur, prev, jj, xpar, deferred(jj) ? 1 : 0), e0, e1));
        else
          RC_TRY(gather<RoleFused>(args(cur, prev, jj, xpar, deferred(jj) ? 1 : 0), e0, e1));
      } else if (cheb_ && !inner) {
        RC_TRY(gather<RoleDirS>(args(cur, prev, jj, xpar, deferred(jj) ? 1 : 0), e0, e1));
      } else if (!rep && dirupd_ && !multi_) {
        // direction, apply and update in one kernel; the state and partials
        // it leaves are in the buffers the gather read (cur)
        bool one = false;
        RC_TRY(dirupd<V>(args(cur, prev, jj, xpar, !inner && deferred(jj) ? 1 : 0), e0, e1, &one));
        if (one) {
          prev = PK_GATHER;
          if (tr) {  // the sample has no separate update kernel
            Timed& rt = recs.back();
            for (int q = 2; q < 4; ++q)
              if (rt.e[q]) {
                ev_.push_back(rt.e[q]);
                rt.e[q] = nullptr;
              }
            rt.kind = 0;
            rt.one = true;
          }
          continue;
        }
        RC_TRY(gather<RoleDir<V>>(args(cur, prev, jj, xpar, !inner && deferred(jj) ? 1 : 0), e0, e1));
      } else {
        RC_TRY(gather<RoleDir<V>>(args(cur, prev, jj, xpar, !inner && deferred(jj) ? 1 : 0), e0, e1));
      }
      cur ^= 1;
      prev = PK_GATHER;
      if (rep) {
        if (one_red && inner)
          RC_TRY(gather<RoleReplFused32>(args(cur, prev, jj, xpar), e2, e3));
        else if (one_red)
          RC_TRY(gather<RoleReplFused>(args(cur, prev, jj, xpar), e2, e3));
        else
          RC_TRY(gather<RoleRepl<V>>(args(cur, prev, jj, xpar), e2, e3));
        prev = PK_GATHER;
        cur ^= 1;
      } else if (!one_red) {
        RC_TRY(update<V>(args(cur, prev, jj, xpar), e2, e3));
        prev = upd_kind;
        cur ^= 1;
      }
      if (cheb_ && !inner) RC_TRY(cheb_chain(false));  // s = M^-1 r and its delta for the next direction
    }
    // the GPU is busy with this chunk: read the earlier chunks' samples now
    if (timing_) RC_TRY(flush_timing());
    const bool launch_next =
        !inner && !mixed_ && !cheb_ && act_.size() == 1 && act_[0]->step + 1 < act_[0]->rq.nsteps;
    RC_TRY(decide(inner, j + k, launch_next));
    if (dirupd_) RC_TRY(check_barrier());  // a failed barrier left this chunk's results void
    bool all_done = true;
    int most = j;
    for (size_t q = 0; q < act_.size(); ++q) {
      Sim& s = *act_[q];
      const Scalars& t = snap_host_[q];
      (inner ? s.si : s.so) = t;
      if (!t.done) all_done = false;
      most = std::max(most, (int)t.iter);
    }
    if (timing_) {
      // iterations past the end of every solve ran idle: not in the sample
      const int ran = std::max(0, std::min(most - j, k));
      for (size_t q = 0; q < recs.size(); ++q) {
        if (rec_c[q] < ran) {
          pending_.push_back(recs[q]);
        } else {
          for (hipEvent_t e : recs[q].e)
            if (e) ev_.push_back(e);
        }
      }
    }
    j += k;
    if (all_done) break;
    if (multi_) {  // later chunks serve only the simulations still iterating
      std::vector<char> live(act_.size(), 0);
      size_t nlive = 0;
      for (size_t q = 0; q < act_.size(); ++q) {
        const Scalars& t = inner ? act_[q]->si : act_[q]->so;
        live[q] = t.done ? 0 : 1;
        nlive += live[q];
      }
      if (nlive < live_count_) RC_TRY(compact(live));
    }
    // the first chunk runs the estimate (the last step's count); a solve
    // that needs more mostly needs one or two more iterations
    k = ++chunks == 1 ? 2 : 4;
  }
  if (live_count_ != act_.size()) uncompact();
  return FEM_OK;
}

// Refinement sweeps of the mixed form: FP32 inner PCG on A e = r64 (FP64 dot
// products and scalars), then x64 += e and the FP64 residual, repeated until
// the FP64 stop rule holds or max_refine sweeps are spent.
int Engine::mixed_sweeps() {
  fem_heat* h = h_;
  const size_t n = act_.size();
  // The first sweep does not wait for the decide after the initial residual:
  // the inner start kernel reads the settled outer state itself (it starts
  // the inner solve only where that solve is neither done nor broken down,
  // with the inner tolerance taken from it), and the host reads the state
  // from the second snapshot slot once the inner solve's first decide is back.
  const bool early = opts_.max_refine > 0;
  RC_TRY(decide(false, 0, false, !early, early ? 1 : 0));
  if (!early)
    for (size_t q = 0; q < n; ++q) {
      Sim& s = *act_[q];
      s.so = snap_host_[q];
      if (s.so.status != 0) s.broke = true;
    }
  bool first = early;
  for (;;) {
    bool any = false;
    int est = 1;
    for (Sim* sp : act_) {
      Sim& s = *sp;
      s.sweeping = !s.broke && (first || !s.so.done) && s.nsw < opts_.max_refine;
      if (s.sweeping) {
        any = true;
        est = std::max(est, s.est_sw[std::min(s.nsw, 3)]);
      }
    }
    if (!any) break;
    RC_TRY(upload_simdev());
    BatchArgs a = args(icur_, iprev_, 0, 0);
    a.table = multi_ ? tab_cur_ + lay_.off_start : nullptr;
    if (multi_)
      hipLaunchKernelGGL(inner_start_batch_kernel, dim3(lay_.n_start), dim3(kT), 0, stream_, a);
    else
      hipLaunchKernelGGL(inner_start_one_kernel, dim3(lay_.n_start), dim3(kT), 0, stream_, a, sd_one_);
    HIP_TRY(hipGetLastError());
    icur_ ^= 1;
    iprev_ = PK_START;
    RC_TRY(pcg<float>(est));
    if (first) {  // the outer state the inner start kernel went by
      first = false;
      bool swept = false;
      for (size_t q = 0; q < n; ++q) {
        Sim& s = *act_[q];
        s.so = snap_host_[n + q];
        if (s.so.status != 0) s.broke = true;
        if (s.so.done || s.broke) s.sweeping = false;  // its inner solve ran idle
        swept = swept || s.sweeping;
      }
      if (!swept) break;
    }
    for (Sim* sp : act_) {
      Sim& s = *sp;
      if (!s.sweeping) continue;
      if (s.si.status != 0) {
        s.broke = true;
        s.sweeping = false;  // no correction from a broken inner solve
        continue;
      }
      s.it += s.si.iter;
      s.est_sw[std::min(s.nsw, 3)] = std::max(1, (int)s.si.iter);
      s.exc = replacements_before(s.si.iter, R_) & 1;
    }
    RC_TRY(upload_simdev());
    RC_TRY(gather<RoleCorr>(args(ocur_, oprev_, 0, 0)));
    ocur_ ^= 1;
    oprev_ = PK_GATHER;
    for (Sim* sp : act_) {
      Sim& s = *sp;
      if (!s.sweeping) continue;
      s.xc ^= 1;
      s.nsw += 1;
    }
    // One simulation whose previous step ran more sweeps than this one has so
    // far: the next sweep goes in behind this decide before the host has read
    // it, as the first sweep does (the inner start kernel finds on the device
    // whether the step has ended and then starts an idle solve; the host
    // reads the state from the second snapshot slot after the inner solve's
    // first decide).
    if (early && act_.size() == 1 && !multi_) {
      const Sim& s = *act_[0];
      if (s.sweeping && s.nsw < opts_.max_refine && s.step > 0 && s.sweeps[s.step - 1] > s.nsw) {
        RC_TRY(decide(false, 0, false, false, 1));
        first = true;
        continue;
      }
    }
    // otherwise the host waits for the decide; with one simulation, the next
    // step's RHS and initial residual go in behind it (they run if this sweep
    // ended the step)
    const bool launch_next = act_.size() == 1 && act_[0]->step + 1 < act_[0]->rq.nsteps;
    RC_TRY(decide(false, 0, launch_next));
    for (size_t q = 0; q < act_.size(); ++q) {
      Sim& s = *act_[q];
      s.so = snap_host_[q];
      if (s.so.status != 0) s.broke = true;
    }
  }
  for (Sim* sp : act_) sp->sweeping = false;
  return FEM_OK;
}

// One theta-scheme step of every simulation of the batch.
int Engine::epoch() {
  for (Sim* sp : act_) {
    Sim& s = *sp;
    s.it = s.nsw = s.xc = s.exc = 0;
    s.sweeping = s.broke = false;
  }
  RC_TRY(upload_simdev());
  // the RHS and initial residual of this step already ran behind the last
  // decide of the previous one (one simulation, same batch); running them
  // again would give the same values
  const bool prepared = next_ran_ && act_.size() == 1 && next_sim_ == act_[0];
  next_ran_ = false;
  next_sim_ = nullptr;
  if (!prepared) {
    RC_TRY(gather<RoleRhs>(args(ocur_, oprev_, 0, 0)));
    ocur_ ^= 1;
    oprev_ = PK_GATHER;
    RC_TRY(cheb_chain(true));  // delta_b in the preconditioner's norm
    RC_TRY(gather<RoleInit>(args(ocur_, oprev_, 0, 0)));
    ocur_ ^= 1;
    oprev_ = PK_GATHER;
    RC_TRY(cheb_chain(false));  // s_0 = M^-1 r_0 and delta_0
  }
  if (mixed_) {
    RC_TRY(mixed_sweeps());
  } else {
    int est = 1;
    for (Sim* sp : act_) est = std::max(est, sp->est);
    RC_TRY(pcg<double>(est));
    for (Sim* sp : act_) {
      Sim& s = *sp;
      s.it = s.so.iter;
      if (s.so.status != 0) s.broke = true;
      s.xc = replacements_before(s.it, R_) & 1;
    }
  }
  for (Sim* sp : act_) RC_TRY(finish_step(*sp));
  return FEM_OK;
}

// Records a finished step of one simulation and rotates its fields.
int Engine::finish_step(Sim& s) {
  fem_heat* h = s.rq.h;
  if (s.broke) {  // outputs stop at the last good step
    if (s.status == FEM_OK || s.status == FEM_ENOCONV) s.status = FEM_EBREAKDOWN;
    h->err = "PCG breakdown (d^T A d <= 0 or non-finite scalar)";
    s.finished = true;
    return FEM_OK;
  }
  const uint32_t N = h->g.N;
  const int n = s.step + 1;
  const Scalars& so = s.so;
  s.iters[n - 1] = s.it;
  s.sweeps[n - 1] = s.nsw;
  s.relres[n - 1] = so.delta_b > 0 ? std::sqrt(std::max(so.delta, 0.0) / so.delta_b) : 0.0;
  const bool unconverged = mixed_ ? (so.delta > so.tol) : (s.it >= opts_.max_iter && so.delta > so.tol);
  if (unconverged && s.status == FEM_OK) s.status = FEM_ENOCONV;
  s.total += s.it;
  s.est = std::max(1, s.it);
  double* xnew = s.X[s.xc];
  if (s.nsens > 0) {
    hipLaunchKernelGGL(sensor_kernel, dim3((s.nsens + 63) / 64), dim3(64), 0, stream_, h->g, xnew, h->xyz_dev,
                       s.nsens, h->traces_dev + (size_t)(n - 1) * s.nsens);
    HIP_TRY(hipGetLastError());
  }
  const fem_out* o = s.rq.out;
  if (o && o->T_saved && o->save_every > 0 && n % o->save_every == 0)
    RC_TRY(copy_out(h, o->T_saved + (size_t)(n / o->save_every - 1) * N, xnew, (size_t)N * sizeof(double)));
  double* freed = s.T2;
  double* spare = s.X[s.xc ^ 1];
  s.T2 = s.T1;
  s.T1 = xnew;
  s.X[0] = freed;
  s.X[1] = spare;
  s.step = n;
  if (s.step >= s.rq.nsteps) s.finished = true;
  return FEM_OK;
}

int Engine::write_outputs(Sim& s, float ms) {
  fem_heat* h = s.rq.h;
  fem_out* o = s.rq.out;
  if (!o) return FEM_OK;
  const uint32_t N = h->g.N;
  o->device_ms = ms;
  o->total_iters = s.total;
  if (o->T_final) RC_TRY(copy_out(h, o->T_final, s.T1, (size_t)N * sizeof(double)));
  if (s.nsens > 0 && o->traces)
    RC_TRY(copy_out(h, o->traces, h->traces_dev, (size_t)std::max(s.rq.nsteps, 0) * s.nsens * sizeof(double)));
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (!dst || bytes == 0) return FEM_OK;
    if (h->devptrs) {
      HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream_));
      HIP_TRY(hipStreamSynchronize(stream_));  // src is host memory that goes away
    } else {
      std::memcpy(dst, src, bytes);
    }
    return FEM_OK;
  };
  RC_TRY(put(o->iters, s.iters.data(), s.iters.size() * sizeof(int32_t)));
  RC_TRY(put(o->relres, s.relres.data(), s.relres.size() * sizeof(double)));
  RC_TRY(put(o->refine_sweeps, s.sweeps.data(), s.sweeps.size() * sizeof(int32_t)));
  return FEM_OK;
}

// One epoch: every simulation that still has steps advances by one step.
// *active receives how many took part (0: nothing left to do).
int Engine::step(int* active) {
  RC_TRY(compose());
  *active = (int)act_.size();
  if (act_.empty()) return FEM_OK;
  return epoch();
}

int Engine::run() {
  fem_heat* h = h_;
  for (auto& e : ev_run_) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipEventRecord(ev_run_[0], stream_));
  for (;;) {
    int active = 0;
    RC_TRY(step(&active));
    if (active == 0) break;
  }
  HIP_TRY(hipEventRecord(ev_run_[1], stream_));
  HIP_TRY(hipEventSynchronize(ev_run_[1]));
  RC_TRY(check_barrier());
  RC_TRY(flush_timing());
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ev_run_[0], ev_run_[1]));
  for (auto& s : sims_) RC_TRY(write_outputs(*s, ms));
  HIP_TRY(hipStreamSynchronize(stream_));
  return FEM_OK;
}

// Autotuner (fem_heat_tune): times the hot gather of the PCG iteration of
// `h` -- the search direction fused with q = A d, d^T q and the deferred
// x += alpha d, in the handle's precision -- through the batched launch the
// engine uses, for every candidate shape.  The timed launches work on zeroed
// vectors of the handle with a relayed state that is never done (so every
// block does its full work) and never read back.  A batch member is timed
// with enough copies of the simulation in one launch to fill the device
// (the copies share the handle's buffers; their identical stores race
// harmlessly), per copy.
int Engine::tune(fem_heat* h, double dt, double theta, bool batch, fem_tune_result* out) {
  fem_heat* eh = h_;
  const uint32_t N = h->g.N;
  RC_TRY(prepare_operator(h, theta * dt, mixed_));
  for (double* p : {h->r64, h->q64, h->d64[0], h->d64[1], h->pool[0], h->pool[1], h->pool[2], h->pool[3]})
    hipLaunchKernelGGL((fill_kernel<double>), dim3(nblk(N)), dim3(kT), 0, stream_, p, 0.0, N);
  if (mixed_)
    for (float* p : {h->r32, h->q32, h->d32[0], h->d32[1], h->e32[0], h->e32[1]})
      hipLaunchKernelGGL((fill_kernel<float>), dim3(nblk(N)), dim3(kT), 0, stream_, p, 0.0f, N);
  for (RelayCtx* c : {&h->outer, &h->inner})
    for (int k = 0; k < 2; ++k) HIP_TRY(hipMemsetAsync(c->S[k], 0, sizeof(Scalars), stream_));
  HIP_TRY(hipGetLastError());
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->opts.device));
  const GatherShape before = h->shape;
  const bool was_batched = h->batched;
  h->batched = batch;
  const std::vector<GatherShape> cands = tune_candidates(h, std::max(cus, 1));
  h->batched = was_batched;
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& x : ev) HIP_TRY(hipEventCreate(&x));
  constexpr int kReps = 6;
  double best = 0.0, rule = 0.0;
  size_t bi = 0;
  int rc = FEM_OK;
  // Time per launch and copy of the candidate installed on h, with `copies`
  // copies of the simulation in each launch.
  auto time_copies = [&](int copies, double* us) -> int {
    sims_.clear();
    for (int q = 0; q < copies; ++q) {
      auto sp = std::make_unique<Sim>();
      sp->rq = RunRequest{h, nullptr, nullptr, dt, theta, 1.0, 1, nullptr};
      sp->T1 = h->pool[0];
      sp->T2 = h->pool[1];
      sp->X[0] = h->pool[2];
      sp->X[1] = h->pool[3];
      sims_.push_back(std::move(sp));
    }
    dirty_ = true;
    int r = compose();
    if (r == FEM_OK) r = upload_simdev();
    auto launch = [&]() {
      return mixed_ ? gather<RoleDir<float>>(args(0, PK_GATHER, 1, 0, 0))
                    : gather<RoleDir<double>>(args(0, PK_GATHER, 1, 0, 1));
    };
    for (int w = 0; w < 2 && r == FEM_OK; ++w) r = launch();
    if (r == FEM_OK && hipEventRecord(ev[0], stream_) != hipSuccess) r = fail(eh, FEM_EDEVICE, "hipEventRecord");
    for (int k = 0; k < kReps && r == FEM_OK; ++k) r = launch();
    if (r == FEM_OK && (hipEventRecord(ev[1], stream_) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess))
      r = fail(eh, FEM_EDEVICE, "timing events failed");
    float ms = 0.f;
    if (r == FEM_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) r = fail(eh, FEM_EDEVICE, "hipEventElapsedTime");
    *us = (double)ms * 1e3 / kReps / copies;
    return r;
  };
  for (size_t i = 0; i < cands.size() && rc == FEM_OK; ++i) {
    const GatherShape& c = cands[i];
    rc = set_shape(h, c);
    if (rc != FEM_OK) break;
    double us = 0.0;
    if (!batch) {
      rc = time_copies(1, &us);
    } else {
      // A batch member's score: its share of a launch that fills the device,
      // plus a sixteenth of a launch holding it alone.  In a lockstep batch
      // the last iterations of a step serve only its slowest members, and
      // then a tile's latency (the length of its z-march) is what counts:
      // measured on 64 x 48^3, whole 49-plane columns per block were the
      // fastest full launches and the slowest batch (95 against 108 solves/s
      // with two-chunk columns).
      const int copies = std::min<int>(64, std::max<int>(1, (4 * cus + (int)c.nblocks - 1) / (int)c.nblocks));
      double full = 0.0, alone = 0.0;
      rc = time_copies(copies, &full);
      if (rc == FEM_OK) rc = time_copies(1, &alone);
      us = full + alone / 16.0;
    }
    if (rc != FEM_OK) break;
    if (i == 0) rule = us;
    if (i == 0 || us < best) {
      best = us;
      bi = i;
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  (void)hipStreamSynchronize(stream_);
  sims_.clear();
  act_.clear();
  dirty_ = true;
  RC_TRY(rc);
  // a simulation alone runs with the tile found; a batch member's tile is
  // only recorded (this handle itself runs alone)
  RC_TRY(set_shape(h, batch ? before : cands[bi]));
  if (!batch) h->tuned = true;
  const GatherShape& b = cands[bi];
  int rec = 0;
  if (h->opts.tune_cache) {
    const int t[3] = {b.tx, b.ty, b.tz};
    rec = tune_store(h->opts.tune_cache, tune_key(h->opts.device, mixed_, h->kind, batch, h->g.px, h->g.py, h->g.pz),
                     t, best, rule, (int)cands.size())
              ? 1
              : 0;
  }
  if (out) {
    out->tile_x = b.tx;
    out->tile_y = b.ty;
    out->tile_z = b.tz;
    out->candidates = (int32_t)cands.size();
    out->best_us = best;
    out->rule_us = rule;
    out->recorded = rec;
  }
  return FEM_OK;
}

int engine_tune(fem_heat* h, double dt, double theta, uint32_t flags, fem_tune_result* out) {
  HIP_TRY(hipSetDevice(h->opts.device));
  fem_opts o = h->opts;
  o.flags &= ~(uint32_t)FEM_TIMING;
  Engine e(h->stream, o, h);
  return e.tune(h, dt, theta, (flags & FEM_TUNE_BATCH) != 0, out);
}

// ---- opaque interface for the server ------------------------------------------

Engine* engine_new(hipStream_t stream, const fem_opts& opts, fem_heat* err) { return new Engine(stream, opts, err); }
void engine_delete(Engine* e) { delete e; }
int engine_add(Engine* e, const RunRequest& r, Sim** out) { return e->add(r, out); }
int engine_step(Engine* e, int* active) { return e->step(active); }
bool engine_sim_finished(const Sim* s) { return s->finished; }
int engine_sim_status(const Sim* s) { return s->status; }
int32_t engine_sim_steps(const Sim* s) { return s->step; }
int engine_finish(Engine* e, Sim* s, double ms) {
  const int rc = e->write_outputs(*s, (float)ms);
  e->remove(s);
  return rc;
}
void engine_drop(Engine* e, Sim* s) { e->remove(s); }

int solver_run(fem_heat* h, const double* T0, const double* T_prev, double dt, double theta, int32_t nsteps,
               double rtol, fem_out* out) {
  HIP_TRY(hipSetDevice(h->opts.device));
  RunRequest r{h, T0, T_prev, dt, theta, rtol, nsteps, out};
  int32_t st = FEM_OK;
  std::string err;
  RC_TRY(engine_run(&r, 1, h->stream, h->opts, &st, &err, true));
  return st;
}

int engine_run(const RunRequest* reqs, int32_t n, hipStream_t stream, const fem_opts& opts, int32_t* status,
               std::string* err, bool one_kernel) {
  fem_heat* h = n == 1 ? reqs[0].h : nullptr;
  fem_heat scratch;
  if (!h) h = &scratch;
  Engine e(stream, opts, h);
  // a run of one handle may iterate in one kernel; batches (and servers)
  // keep two, so a simulation's bits do not depend on what it runs with
  e.allow_one_kernel(one_kernel && n == 1);
  for (int32_t i = 0; i < n; ++i) {
    const int rc = e.add(reqs[i]);
    if (rc != FEM_OK) {
      if (err) *err = reqs[i].h->err;
      return rc;
    }
  }
  const int rc = e.run();
  if (rc != FEM_OK) {
    if (err) *err = h->err;
    return rc;
  }
  for (int32_t i = 0; i < n; ++i) status[i] = e.sims()[(size_t)i]->status;
  if (n == 1 && (opts.flags & FEM_TIMING)) {
    fem_heat* one = reqs[0].h;
    const fem_stats keep = one->stats;
    one->stats = e.stats;
    one->stats.grid_blocks = keep.grid_blocks;
    one->stats.tile_x = keep.tile_x;
    one->stats.tile_y = keep.tile_y;
    one->stats.tile_z = keep.tile_z;
  }
  return FEM_OK;
}

}  // namespace femheat
