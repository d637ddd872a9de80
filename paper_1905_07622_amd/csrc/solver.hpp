// Host-side state of one solver handle (device-resident problem and PCG state).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "fem_heat.h"
#include "common.hpp"

namespace femheat {
// Device buffers of one relayed solve: the ping-pong state blocks and the
// block-partial buffers.
struct RelayCtx {
  Scalars* S[2] = {nullptr, nullptr};
  double* P[2] = {nullptr, nullptr};
};
}  // namespace femheat

struct fem_heat {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  fem_opts opts{};
  bool devptrs = false;
  bool timing = false;
  bool batched = false;  // created as a member of a batch (tile rule of batch members)

  femheat::Geom g{};
  bool cubic = false;
  int kind = 0;  // gather element kind: kElemBox, kElemCubic or kElemTet6
  bool nonzero_dirichlet = false;
  std::vector<double> sched;

  // element coefficients
  double* rhoc64 = nullptr;
  double* k64 = nullptr;
  float* rhoc32 = nullptr;
  float* k32 = nullptr;

  // node vectors, FP64
  double* F64 = nullptr;
  double* pinv64 = nullptr;
  double* b64 = nullptr;
  double* r64 = nullptr;
  double* q64 = nullptr;
  double* r64b = nullptr;  // one-reduction form: second residual and apply buffers
  double* q64b = nullptr;
  double* d64[2] = {nullptr, nullptr};
  double* pool[4] = {nullptr, nullptr, nullptr, nullptr};  // T^{n-1}, T^{n-2}, x ping-pong
  double* lift64 = nullptr;   // A_fD g (only with non-zero Dirichlet values)
  double* sink = nullptr;     // 256 scratch values for stores of lanes without a node
  double* noalloc_scratch = nullptr;  // device address of the library's static scratch on this device
  double ck_cached = -1.0;    // theta*dt of pinv/lift; < 0: none

  // Chebyshev preconditioner (FP64 solves): s = M^-1 r, the chain's residual
  // and direction ping-pong, 1/c and the step coefficients a_k, b_k
  double* s64 = nullptr;
  double* cr64 = nullptr;
  double* cd64[2] = {nullptr, nullptr};
  double ch_inv_c = 0.0, ch_hi = 0.0, ch_lo = 0.0;
  double ch_a[femheat::kChebMaxDegree] = {}, ch_b[femheat::kChebMaxDegree] = {};

  // node vectors, FP32 (mixed form)
  float* pinv32 = nullptr;
  float* e32[2] = {nullptr, nullptr};
  float* r32 = nullptr;
  float* q32 = nullptr;
  float* r32b = nullptr;  // one-reduction form of the inner solves: second residual and apply buffers
  float* q32b = nullptr;
  float* d32[2] = {nullptr, nullptr};
  float* rhs32 = nullptr;

  // relayed solve state: outer (FP64) and inner (FP32) solves
  femheat::RelayCtx outer, inner;
  uint32_t n_partials = 0;

  // per-run buffers
  double* xyz_dev = nullptr;
  double* traces_dev = nullptr;
  size_t traces_cap = 0;
  size_t xyz_cap = 0;

  femheat::GatherShape shape{};
  int32_t capacity = 1;   // blocks of the hot gather the device holds at once (tile rule of a simulation alone)
  bool tuned = false;     // the shape came from the autotuner's cache
  uint32_t upd_blocks64 = 0, upd_blocks32 = 0, start_blocks = 0;

  // element-by-element apply (test hook): 4 N partial sums, allocated on first use
  double* ebe_part = nullptr;
  hipEvent_t ev_apply[2] = {nullptr, nullptr};  // FEM_TIMING: around an apply's operator kernels

  fem_stats stats{};

  std::string err;
};

namespace femheat {

int solver_init(fem_heat* h, const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc);
// A handle for a validated problem; `batched` selects the tile rule of batch
// members.  On failure *why (may be NULL) receives the message.
int make_handle(const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc, const fem_opts& o,
                bool batched, fem_heat** out, std::string* why);
int solver_apply(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y);
// fem_heat_apply for device pointers with the library's static scratch: only
// kernel launches on the handle's stream (no allocation, copy or wait).
int solver_apply_noalloc(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y);
int noalloc_scratch_setup(fem_heat* h);
void solver_free(fem_heat* h);

// Time stepping (engine.hip): one handle, or a batch of handles advanced
// together (status[i] receives the outcome of sims[i]).
struct RunRequest {
  fem_heat* h;
  const double* T0;
  const double* T_prev;
  double dt, theta, rtol;
  int32_t nsteps;
  fem_out* out;
};
int solver_run(fem_heat* h, const double* T0, const double* T_prev, double dt, double theta, int32_t nsteps,
               double rtol, fem_out* out);
int engine_run(const RunRequest* reqs, int32_t n, hipStream_t stream, const fem_opts& opts, int32_t* status,
               std::string* err, bool one_kernel = false);

}  // namespace femheat
