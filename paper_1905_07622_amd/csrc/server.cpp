// Serving loop: continuous batching of forward simulations on one GPU.
//
// Requests are grouped into size classes (the binary order of magnitude of
// their node count).  Each class has a lane: a worker thread with its own
// HIP stream and engine, so the classes' kernels run concurrently and a
// small request never waits for the epochs of a large one.  Each turn of a
// lane's loop is one epoch boundary: finished simulations retire (outputs,
// memory, completion stamp), cancelled ones leave, queued requests of the
// lane's class are admitted while their device footprint fits the free
// budget and a slot is free, and then every simulation of the lane advances
// one time step with the batched launches.  Admission follows arrival order
// across all classes: a request that does not fit blocks every later one,
// so large requests cannot starve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "server.hpp"

namespace {

using Clock = std::chrono::steady_clock;

// A request with its own copies of every input.
struct Request {
  uint64_t ticket = 0;
  fem_grid grid{};
  fem_bc bc{};
  std::vector<double> k_e, rhoc_e, T0, T_prev, sched, sensors;
  double dt = 0, theta = 0, rtol = 0;
  int32_t nsteps = 0;
  fem_out out{};                  // outputs point into the caller's arrays; inputs into ours
  fem_out* caller_out = nullptr;  // receives total_iters and device_ms
  fem_status st{};
  int key = 0;  // size class
  bool cancel = false;
  fem_heat* h = nullptr;
  femheat::Sim* sim = nullptr;
};

// Size class of a problem: floor(log2(node count)).
int size_class(const fem_grid& g) {
  const double n = (double)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  int k = 0;
  while ((double)(1ull << (k + 1)) <= n && k < 62) ++k;
  return k;
}

struct Lane;

}  // namespace

struct fem_server {
  fem_server_opts o{};
  // Device memory of admitted simulations: a stream-ordered pool of the
  // server (or the caller's allocator).  Each lane allocates and releases on
  // its own stream, so a retirement never synchronises the device -- hipFree
  // would wait for every lane's kernels -- and released blocks are reused by
  // later admissions without going back to the HIP runtime.
  hipMemPool_t pool = nullptr;
  fem_allocator pool_alloc{};
  std::string tune_cache;  // own copy of the options' tile-cache path

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;  // all classes, arrival order
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::map<int, std::unique_ptr<Lane>> lanes;
  uint64_t next_ticket = 1;
  uint64_t budget = 0, in_use = 0, peak = 0;
  int64_t submitted = 0, completed = 0, canceled = 0, failed = 0, epochs = 0;
  int32_t nrunning = 0;  // admitted and not yet finished, all lanes
  bool stop = false;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void finish(Request* r, int state, int status, bool charged);
  int open_lane(int key, std::string* err);
};

namespace {

// One size class: a stream, an engine and the worker that drives them.
struct Lane {
  fem_server* srv = nullptr;
  int key = 0;
  hipStream_t stream = nullptr;
  femheat::Engine* eng = nullptr;
  fem_heat errh;                  // receives the engine's messages
  std::vector<Request*> running;  // touched by the worker; counted under srv->mu
  bool dead = false;              // the worker stopped after an exception
  std::thread worker;
  void loop();
  void fail_all(int status);
};

}  // namespace

namespace {

int pool_alloc_fn(void* ctx, void** ptr, size_t bytes, void* stream) {
  auto* srv = static_cast<fem_server*>(ctx);
  if (hipMallocFromPoolAsync(ptr, bytes, srv->pool, static_cast<hipStream_t>(stream)) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return -1;
  }
  return 0;
}

void pool_release_fn(void*, void* ptr, void* stream) { (void)hipFreeAsync(ptr, static_cast<hipStream_t>(stream)); }

void free_handle(Request* r) {
  if (r->h) {
    femheat::solver_free(r->h);
    delete r->h;
    r->h = nullptr;
  }
  r->sim = nullptr;
}

}  // namespace

// Marks a request terminal and releases its budget if it was admitted
// (called with mu held).
void fem_server::finish(Request* r, int state, int status, bool charged) {
  r->st.state = state;
  r->st.status = status;
  r->st.t_done = now();
  if (charged) in_use -= r->st.bytes;
  if (state == FEM_REQ_CANCELED)
    ++canceled;
  else if (status == FEM_OK || status == FEM_ENOCONV)
    ++completed;
  else
    ++failed;
}

void Lane::loop() {
  fem_server& S = *srv;
  (void)hipSetDevice(S.o.opts.device);
  for (;;) {
    std::vector<Request*> admit, cancelled;
    bool stopping = false;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      // Admission in arrival order: a request is taken only if it fits
      // together with every request ahead of it (which other lanes take),
      // so the first one that does not fit blocks all later ones, of any
      // class, and a later request never takes the budget or the slot of an
      // earlier one.  `take` visits the requests of this class that fit.
      auto scan = [&](auto take) {
        uint64_t bytes = S.in_use;
        int32_t slots = S.nrunning;
        for (auto it = S.queue.begin(); it != S.queue.end();) {
          Request* r = *it;
          if (r->st.bytes > S.budget - std::min(S.budget, bytes) || slots >= S.o.max_slots) return;
          bytes += r->st.bytes;
          slots += 1;
          if (r->key == key) {
            if (!take(it)) return;
          } else {
            ++it;
          }
        }
      };
      auto admissible = [&] {
        bool any = false;
        scan([&](std::deque<Request*>::iterator&) { return !(any = true); });
        return any;
      };
      S.cv_work.wait(lk, [&] { return S.stop || !running.empty() || admissible(); });
      stopping = S.stop;
      if (stopping)
        for (Request* r : running) r->cancel = true;
      for (Request* r : running)
        if (r->cancel) cancelled.push_back(r);
      if (!S.stop) {
        scan([&](std::deque<Request*>::iterator& it) {
          admit.push_back(*it);
          it = S.queue.erase(it);
          return true;
        });
        // admitted requests leave the queue as RUNNING: a cancel from now on
        // is taken at the next epoch boundary, after their set-up below
        for (Request* r : admit) {
          r->st.state = FEM_REQ_RUNNING;
          r->st.t_admit = S.now();
          S.in_use += r->st.bytes;
        }
        S.peak = std::max(S.peak, S.in_use);
        S.nrunning += (int32_t)admit.size();
        // requests of other classes behind these may be admissible now
        if (!admit.empty()) S.cv_work.notify_all();
      }
    }
    // cancelled simulations leave without outputs
    for (Request* r : cancelled) {
      femheat::engine_drop(eng, r->sim);
      free_handle(r);
      std::lock_guard<std::mutex> lk(S.mu);
      running.erase(std::find(running.begin(), running.end(), r));
      --S.nrunning;
      S.finish(r, FEM_REQ_CANCELED, FEM_ECANCELED, true);
      S.cv_done.notify_all();
    }
    if (stopping) {
      std::lock_guard<std::mutex> lk(S.mu);
      if (running.empty()) return;
    }
    // admitted requests: device state and engine membership
    for (Request* r : admit) {
      fem_opts ho = S.o.opts;
      ho.hip_stream = stream;
      std::string why;
      fem_heat* h = nullptr;
      int rc = femheat::make_handle(&r->grid, r->k_e.data(), r->rhoc_e.data(), &r->bc, ho, true, &h, &why);
      if (rc == FEM_OK) {
        r->h = h;
        femheat::RunRequest rq{h, r->T0.data(), r->T_prev.empty() ? nullptr : r->T_prev.data(), r->dt, r->theta,
                               r->rtol, r->nsteps, &r->out};
        rc = femheat::engine_add(eng, rq, &r->sim);
      }
      std::lock_guard<std::mutex> lk(S.mu);
      if (rc != FEM_OK) {
        free_handle(r);
        --S.nrunning;
        S.finish(r, FEM_REQ_DONE, rc, true);
        S.cv_done.notify_all();
        continue;
      }
      running.push_back(r);
    }
    if (running.empty()) continue;
    // one epoch for every simulation of this lane
    int active = 0;
    const int rc = femheat::engine_step(eng, &active);
    std::vector<Request*> done;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      ++S.epochs;
      for (Request* r : running) {
        r->st.steps_done = femheat::engine_sim_steps(r->sim);
        if (rc != FEM_OK || femheat::engine_sim_finished(r->sim)) done.push_back(r);
      }
    }
    for (Request* r : done) {
      int status = rc != FEM_OK ? rc : femheat::engine_sim_status(r->sim);
      const double ms = (S.now() - r->st.t_admit) * 1e3;
      if (rc == FEM_OK) {
        const int wrc = femheat::engine_finish(eng, r->sim, ms);
        if (wrc != FEM_OK) status = wrc;
      } else {
        femheat::engine_drop(eng, r->sim);
      }
      if (r->caller_out && status != FEM_EDEVICE) {
        r->caller_out->total_iters = r->out.total_iters;
        r->caller_out->device_ms = r->out.device_ms;
      }
      free_handle(r);
      std::lock_guard<std::mutex> lk(S.mu);
      running.erase(std::find(running.begin(), running.end(), r));
      --S.nrunning;
      S.finish(r, FEM_REQ_DONE, status, true);
    }
    if (!done.empty()) {
      S.cv_done.notify_all();
      S.cv_work.notify_all();  // released budget or slots may admit other lanes' requests
    }
  }
}

// Ends this lane's requests with `status` (after an exception in its worker,
// whose engine state is then unknown); the lane admits nothing more.
void Lane::fail_all(int status) {
  std::lock_guard<std::mutex> lk(srv->mu);
  dead = true;
  for (Request* r : running) {
    free_handle(r);
    --srv->nrunning;
    srv->finish(r, FEM_REQ_DONE, status, true);
  }
  running.clear();
  for (auto it = srv->queue.begin(); it != srv->queue.end();) {
    if ((*it)->key == key) {
      srv->finish(*it, FEM_REQ_DONE, status, false);
      it = srv->queue.erase(it);
    } else {
      ++it;
    }
  }
  srv->cv_done.notify_all();
}

// Starts the lane of size class `key` (called with mu held).
int fem_server::open_lane(int key, std::string* err) {
  auto ln = std::make_unique<Lane>();
  ln->srv = this;
  ln->key = key;
  if (hipSetDevice(o.opts.device) != hipSuccess ||
      hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking) != hipSuccess) {
    *err = "hipStreamCreate failed";
    return FEM_EDEVICE;
  }
  fem_opts eo = o.opts;
  eo.hip_stream = ln->stream;
  ln->eng = femheat::engine_new(ln->stream, eo, &ln->errh);
  Lane* raw = ln.get();
  ln->worker = std::thread([raw] {
    try {
      raw->loop();
    } catch (const std::bad_alloc&) {
      raw->fail_all(FEM_ENOMEM);
    } catch (...) {
      raw->fail_all(FEM_EDEVICE);
    }
  });
  lanes[key] = std::move(ln);
  return FEM_OK;
}

namespace femheat {

int server_create(const fem_server_opts& o, fem_server** out, std::string* err) {
  auto s = std::make_unique<fem_server>();
  s->o = o;
  if (s->o.max_slots <= 0) s->o.max_slots = 256;
  if (hipSetDevice(o.opts.device) != hipSuccess) {
    *err = "hipSetDevice failed";
    return FEM_EDEVICE;
  }
  s->budget = o.hbm_budget_bytes;
  if (s->budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      *err = "hipMemGetInfo failed";
      return FEM_EDEVICE;
    }
    s->budget = free_b / 4 * 3;
  }
  if (!o.opts.allocator) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = o.opts.device;
    if (hipMemPoolCreate(&s->pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      *err = "hipMemPoolCreate failed";
      return FEM_EDEVICE;
    }
    // keep released blocks in the pool (at most what the budget admits at once)
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep);
    s->pool_alloc = fem_allocator{s.get(), pool_alloc_fn, pool_release_fn};
    s->o.opts.allocator = &s->pool_alloc;
  }
  if (o.opts.tune_cache) {
    s->tune_cache = o.opts.tune_cache;
    s->o.opts.tune_cache = s->tune_cache.c_str();
  }
  s->t0 = Clock::now();
  *out = s.release();
  return FEM_OK;
}

int server_submit(fem_server* s, const fem_request& q, uint64_t* ticket, std::string* err) {
  auto r = std::make_unique<Request>();
  const size_t E = (size_t)q.grid.nx * q.grid.ny * q.grid.nz;
  const size_t N = (size_t)(q.grid.nx + 1) * (q.grid.ny + 1) * (q.grid.nz + 1);
  r->grid = q.grid;
  r->k_e.assign(q.k_e, q.k_e + E);
  r->rhoc_e.assign(q.rhoc_e, q.rhoc_e + E);
  r->T0.assign(q.T0, q.T0 + N);
  if (q.T_prev) r->T_prev.assign(q.T_prev, q.T_prev + N);
  r->bc = q.bc;
  if (q.bc.flux_schedule && q.bc.n_schedule > 0) {
    r->sched.assign(q.bc.flux_schedule, q.bc.flux_schedule + q.bc.n_schedule);
    r->bc.flux_schedule = r->sched.data();
  } else {
    r->bc.flux_schedule = nullptr;
    r->bc.n_schedule = 0;
  }
  r->dt = q.dt;
  r->theta = q.theta;
  r->rtol = q.rtol;
  r->nsteps = q.nsteps;
  int32_t nsens = 0;
  if (q.out) {
    r->out = *q.out;
    r->caller_out = q.out;
    if (q.out->sensor_xyz && q.out->n_sensors > 0) {
      nsens = q.out->n_sensors;
      r->sensors.assign(q.out->sensor_xyz, q.out->sensor_xyz + 3 * (size_t)nsens);
      r->out.sensor_xyz = r->sensors.data();
    }
    r->out.first_step = q.out->first_step;
  }
  r->st.state = FEM_REQ_QUEUED;
  r->st.status = FEM_OK;
  r->st.t_admit = r->st.t_done = -1.0;
  r->st.bytes = handle_device_bytes(q.grid, s->o.opts, &q.bc, q.nsteps, nsens);
  r->key = size_class(q.grid);
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->st.bytes > s->budget) {
    *err = "request needs " + std::to_string(r->st.bytes) + " device bytes, budget " + std::to_string(s->budget);
    return FEM_ENOMEM;
  }
  if (s->stop) {
    *err = "server is stopping";
    return FEM_EBUSY;
  }
  if (!s->lanes.count(r->key)) {
    const int rc = s->open_lane(r->key, err);
    if (rc != FEM_OK) return rc;
  } else if (s->lanes[r->key]->dead) {
    *err = "the worker of this size class stopped after a device error";
    return FEM_EDEVICE;
  }
  r->ticket = s->next_ticket++;
  r->st.t_arrive = s->now();
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  ++s->submitted;
  s->cv_work.notify_all();
  return FEM_OK;
}

int server_poll(fem_server* s, uint64_t ticket, fem_status* st) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FEM_EINVAL;
  if (st) *st = it->second->st;
  return FEM_OK;
}

int server_wait(fem_server* s, uint64_t ticket, double timeout_s, fem_status* st) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FEM_EINVAL;
  Request* r = it->second.get();
  auto terminal = [r] { return r->st.state == FEM_REQ_DONE || r->st.state == FEM_REQ_CANCELED; };
  bool ok;
  if (timeout_s < 0) {
    s->cv_done.wait(lk, terminal);
    ok = true;
  } else {
    ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), terminal);
  }
  if (st) *st = r->st;
  return ok ? r->st.status : FEM_EBUSY;
}

int server_cancel(fem_server* s, uint64_t ticket) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FEM_EINVAL;
  Request* r = it->second.get();
  auto qi = std::find(s->queue.begin(), s->queue.end(), r);
  if (r->st.state == FEM_REQ_QUEUED && qi != s->queue.end()) {
    s->queue.erase(qi);
    s->finish(r, FEM_REQ_CANCELED, FEM_ECANCELED, false);
    s->cv_done.notify_all();
  } else if (r->st.state == FEM_REQ_RUNNING) {
    r->cancel = true;
    s->cv_work.notify_all();
  }
  return FEM_OK;
}

int server_info(fem_server* s, fem_server_info* info) {
  std::lock_guard<std::mutex> lk(s->mu);
  info->submitted = s->submitted;
  info->completed = s->completed;
  info->canceled = s->canceled;
  info->failed = s->failed;
  info->epochs = s->epochs;
  info->queued = (int32_t)s->queue.size();
  info->running = s->nrunning;
  info->budget_bytes = s->budget;
  info->bytes_in_use = s->in_use;
  info->peak_bytes_in_use = s->peak;
  info->now = s->now();
  return FEM_OK;
}

void server_destroy(fem_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (Request* r : s->queue) s->finish(r, FEM_REQ_CANCELED, FEM_ECANCELED, false);
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (auto& kv : s->lanes) {
    Lane& ln = *kv.second;
    if (ln.worker.joinable()) ln.worker.join();
    femheat::engine_delete(ln.eng);
    (void)hipStreamSynchronize(ln.stream);
    (void)hipStreamDestroy(ln.stream);
  }
  s->cv_done.notify_all();
  if (s->pool) (void)hipMemPoolDestroy(s->pool);
  delete s;
}

}  // namespace femheat
