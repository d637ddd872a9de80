// Opaque interface of the time-stepping engine (engine.hip) for host code
// that admits and retires simulations while others run (the server).
#pragma once

#include <hip/hip_runtime.h>

#include "solver.hpp"

namespace femheat {

class Engine;
struct Sim;

Engine* engine_new(hipStream_t stream, const fem_opts& opts, fem_heat* err);
void engine_delete(Engine* e);
// Prepares a simulation on its handle (whose stream must be the engine's);
// it joins the batch at the next epoch.
int engine_add(Engine* e, const RunRequest& r, Sim** out);
// One epoch: every member with steps left advances one step; *active is the
// number that did (0: nothing to do).  A failing HIP call fails the epoch.
int engine_step(Engine* e, int* active);
bool engine_sim_finished(const Sim* s);
int engine_sim_status(const Sim* s);
int32_t engine_sim_steps(const Sim* s);
// Writes a finished simulation's outputs (device_ms = ms) and removes it.
int engine_finish(Engine* e, Sim* s, double ms);
// Removes a simulation without outputs.
void engine_drop(Engine* e, Sim* s);

// Autotuner of the gather launch shape (fem_heat_tune).
int engine_tune(fem_heat* h, double dt, double theta, uint32_t flags, fem_tune_result* out);

// Device bytes a handle for this problem holds while it runs.
size_t handle_device_bytes(const fem_grid& grid, const fem_opts& opts, const fem_bc* bc, int32_t nsteps,
                           int32_t n_sensors);

}  // namespace femheat
