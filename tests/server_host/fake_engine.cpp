// A CPU fake of the time-stepping engine and of handle set-up, with the
// interface the serving loop calls (engine.hpp, solver.hpp).  It advances
// every member one step per epoch like the real engine, allocates and
// releases a handle's memory through the options' allocator on the lane's
// stream (the server's pool), and writes a finished simulation's outputs in
// engine_finish: T_final = T0 + nsteps, iters = 1 per step.  Each handle
// records the thread that created it; every later use must come from that
// thread (a lane owns its handles), which the fake checks.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "engine.hpp"

namespace femheat {

struct Sim {
  RunRequest rq;
  int32_t steps = 0;
};

class Engine {
 public:
  hipStream_t stream = nullptr;
  std::vector<Sim*> sims;
  std::thread::id owner;
  bool owned = false;
};

namespace {
struct FakeDev {
  void* block = nullptr;
  size_t bytes = 0;
  std::thread::id owner;
};

void check_owner(std::thread::id o, const char* what) {
  if (o != std::this_thread::get_id()) {
    std::fprintf(stderr, "fake engine: %s used from a thread that does not own it\n", what);
    std::abort();
  }
}
}  // namespace

int make_handle(const fem_grid* grid, const double*, const double*, const fem_bc*, const fem_opts& o, bool,
                fem_heat** out, std::string* why) {
  auto* h = new fem_heat();
  h->opts = o;
  h->stream = static_cast<hipStream_t>(o.hip_stream);
  h->g.nx = grid->nx;
  h->g.ny = grid->ny;
  h->g.nz = grid->nz;
  h->g.N = (uint32_t)((grid->nx + 1) * (grid->ny + 1) * (grid->nz + 1));
  auto* d = new FakeDev();
  d->owner = std::this_thread::get_id();
  d->bytes = 8 * (size_t)h->g.N;
  if (o.allocator) {
    if (o.allocator->alloc(o.allocator->ctx, &d->block, d->bytes, o.hip_stream) != 0) {
      if (why) *why = "fake allocation failed";
      delete d;
      delete h;
      return FEM_ENOMEM;
    }
  } else {
    d->block = std::malloc(d->bytes);
  }
  static_cast<char*>(d->block)[0] = 1;  // touch it
  h->sink = reinterpret_cast<double*>(d);  // the fake keeps its record in an unused field
  *out = h;
  return FEM_OK;
}

void solver_free(fem_heat* h) {
  auto* d = reinterpret_cast<FakeDev*>(h->sink);
  if (!d) return;
  check_owner(d->owner, "a handle");
  if (h->opts.allocator)
    h->opts.allocator->release(h->opts.allocator->ctx, d->block, h->stream);
  else
    std::free(d->block);
  delete d;
  h->sink = nullptr;
}

size_t handle_device_bytes(const fem_grid& grid, const fem_opts&, const fem_bc*, int32_t, int32_t) {
  return 8 * (size_t)(grid.nx + 1) * (grid.ny + 1) * (grid.nz + 1);
}

Engine* engine_new(hipStream_t stream, const fem_opts&, fem_heat*) {
  auto* e = new Engine();
  e->stream = stream;
  return e;
}

void engine_delete(Engine* e) {
  for (Sim* s : e->sims) delete s;
  delete e;
}

int engine_add(Engine* e, const RunRequest& r, Sim** out) {
  if (!e->owned) {
    e->owner = std::this_thread::get_id();
    e->owned = true;
  }
  check_owner(e->owner, "an engine");
  if (r.h->stream != e->stream) {
    std::fprintf(stderr, "fake engine: a handle on another stream joined the engine\n");
    std::abort();
  }
  auto* s = new Sim();
  s->rq = r;
  e->sims.push_back(s);
  *out = s;
  return FEM_OK;
}

int engine_step(Engine* e, int* active) {
  check_owner(e->owner, "an engine");
  int n = 0;
  for (Sim* s : e->sims)
    if (s->steps < s->rq.nsteps) {
      ++s->steps;
      ++n;
    }
  std::this_thread::sleep_for(std::chrono::microseconds(50 + 10 * n));
  *active = n;
  return FEM_OK;
}

bool engine_sim_finished(const Sim* s) { return s->steps >= s->rq.nsteps; }
int engine_sim_status(const Sim*) { return FEM_OK; }
int32_t engine_sim_steps(const Sim* s) { return s->steps; }

static void remove_sim(Engine* e, Sim* s) {
  for (size_t k = 0; k < e->sims.size(); ++k)
    if (e->sims[k] == s) {
      e->sims.erase(e->sims.begin() + (long)k);
      break;
    }
  delete s;
}

int engine_finish(Engine* e, Sim* s, double ms) {
  check_owner(e->owner, "an engine");
  fem_out* o = s->rq.out;
  if (o) {
    const uint32_t N = s->rq.h->g.N;
    if (o->T_final)
      for (uint32_t i = 0; i < N; ++i) o->T_final[i] = s->rq.T0[i] + s->rq.nsteps;
    if (o->iters)
      for (int32_t k = 0; k < s->rq.nsteps; ++k) o->iters[k] = 1;
    o->total_iters = s->rq.nsteps;
    o->device_ms = ms;
  }
  remove_sim(e, s);
  return FEM_OK;
}

void engine_drop(Engine* e, Sim* s) {
  check_owner(e->owner, "an engine");
  remove_sim(e, s);
}

}  // namespace femheat
