// extern "C" entry points of include/fem_heat.h: argument validation, handle
// lifetime and error reporting.  The work itself is in solver.hip (set-up,
// operator hook) and engine.hip (time stepping, single and batched).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "server.hpp"
#include "solver.hpp"

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Reads n doubles from host or device memory for validation.
bool fetch(const double* src, size_t n, bool device, std::vector<double>& out) {
  out.resize(n);
  if (!device) {
    std::memcpy(out.data(), src, n * sizeof(double));
    return true;
  }
  return hipMemcpy(out.data(), src, n * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
}

thread_local std::string g_create_error;

int check_opts(const fem_opts* opts, fem_opts& o, std::string& why) {
  fem_heat_default_opts(&o);
  if (opts) o = *opts;
  auto bad = [&](const char* m) {
    why = m;
    return FEM_EINVAL;
  };
  if (o.precision != FEM_FP64 && o.precision != FEM_FP32_FP64DOT) return bad("unknown precision");
  if (o.max_iter < 0 || o.replace_every < 0 || o.max_refine < 0) return bad("negative iteration controls");
  if (o.guess != FEM_GUESS_EXTRAP && o.guess != FEM_GUESS_PREV) return bad("unknown guess rule");
  if (o.stop_rule != FEM_STOP_RHS && o.stop_rule != FEM_STOP_INITIAL) return bad("unknown stop rule");
  if (o.precision == FEM_FP32_FP64DOT && !finite_pos(o.inner_rtol)) return bad("inner_rtol must be > 0");
  if (o.element != FEM_ELEM_HEX8 && o.element != FEM_ELEM_TET6) return bad("unknown element");
  if (o.element == FEM_ELEM_TET6 && o.precond != FEM_PRECOND_JACOBI)
    return bad("the tetrahedral element runs with the Jacobi preconditioner");
  if (o.precond != FEM_PRECOND_JACOBI && o.precond != FEM_PRECOND_CHEBYSHEV) return bad("unknown preconditioner");
  if (o.precond == FEM_PRECOND_CHEBYSHEV) {
    if (o.precision != FEM_FP64 || (o.flags & FEM_ONE_REDUCTION))
      return bad("the Chebyshev preconditioner runs in the FP64 two-kernel form only");
    if (o.cheb_degree < 2 || o.cheb_degree > femheat::kChebMaxDegree) return bad("cheb_degree must be in 2..8");
    if (!(o.cheb_ratio > 1.0) || !std::isfinite(o.cheb_ratio)) return bad("cheb_ratio must be finite and > 1");
  }
  if (o.batch_groups < 0) return bad("batch_groups must be >= 0");
  if (o.tile_x < 0 || o.tile_y < 0 || o.tile_z < 0 || o.tile_x > femheat::kMaxBlockThreads ||
      o.tile_x * std::max(o.tile_y, 1) > femheat::kMaxBlockThreads)
    return bad("tile overrides out of range");
  // each thread of a gather block stages two entries of the (tx+2) x (ty+2)
  // plane tile and of the (tx+1) x (ty+1) coefficient tile; with tile_x given
  // and tile_y automatic, tile_y can shrink to 1, so that case must fit
  if (o.tile_x > 0) {
    const int tx = o.tile_x, ty = std::max(o.tile_y, 1);
    const int nthreads = ((tx * ty + 63) / 64) * 64;
    if ((tx + 2) * (ty + 2) > 2 * nthreads || (tx + 1) * (ty + 1) > 2 * nthreads)
      return bad("tile overrides too thin: the gather stages two plane entries per thread");
  } else if (o.tile_y > 0) {
    return bad("tile_y needs tile_x");
  }
  return FEM_OK;
}

// Grid, coefficients and boundary conditions of a problem.
int check_problem(const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc, const fem_opts& o,
                  std::string& why) {
  auto bad = [&](const char* m) {
    why = m;
    return FEM_EINVAL;
  };
  if (!grid || !k_e || !rhoc_e) return bad("grid, k_e and rhoc_e are required");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return bad("nx, ny, nz must be >= 1");
  const double N = (double)(grid->nx + 1) * (grid->ny + 1) * (grid->nz + 1);
  // kernels address FP64 node vectors with 32-bit byte offsets
  if (N >= 536870912.0) return bad("grid too large (N must be below 2^29 nodes)");
  if (!finite_pos(grid->hx) || !finite_pos(grid->hy) || !finite_pos(grid->hz)) return bad("h must be finite and > 0");
  if (o.element == FEM_ELEM_TET6 && !(grid->hx == grid->hy && grid->hy == grid->hz))
    return bad("the tetrahedral element needs cubic boxes (hx = hy = hz)");
  if (bc) {
    if ((bc->dirichlet_mask | bc->flux_mask) >= 64u) return bad("face masks have 6 bits");
    if (bc->dirichlet_mask & bc->flux_mask) return bad("a face is both Dirichlet and flux");
    for (int f = 0; f < 6; ++f)
      if (!std::isfinite(bc->dirichlet_value[f]) || !std::isfinite(bc->flux[f])) return bad("non-finite boundary value");
    if (bc->n_schedule < 0 || (bc->n_schedule > 0 && !bc->flux_schedule)) return bad("bad flux schedule");
    for (int32_t m = 0; m < bc->n_schedule; ++m)
      if (!std::isfinite(bc->flux_schedule[m])) return bad("non-finite flux schedule value");
  }
  const bool dev = (o.flags & FEM_DEVICE_PTRS) != 0;
  const size_t E = (size_t)grid->nx * grid->ny * grid->nz;
  if (dev && hipSetDevice(o.device) != hipSuccess) {
    why = "hipSetDevice failed";
    return FEM_EDEVICE;
  }
  std::vector<double> chk;
  if (!fetch(k_e, E, dev, chk)) {
    why = "reading k_e failed";
    return FEM_EDEVICE;
  }
  for (double v : chk)
    if (!(v >= 0.0) || !std::isfinite(v)) return bad("k_e must be finite and >= 0");
  if (!fetch(rhoc_e, E, dev, chk)) {
    why = "reading rhoc_e failed";
    return FEM_EDEVICE;
  }
  for (double v : chk)
    if (!finite_pos(v)) return bad("rhoc_e must be finite and > 0");
  return FEM_OK;
}

// Arguments of a run on grid g (only the sizes and spacings of g are used).
int check_run(const femheat::Geom& g, bool dev, const double* T0, double dt, double theta, double rtol,
              int32_t nsteps, const fem_out* out, std::string& why) {
  auto bad = [&](const char* m) {
    why = m;
    return FEM_EINVAL;
  };
  if (!T0) return bad("T0 is required");
  if (!finite_pos(dt)) return bad("dt must be finite and > 0");
  if (!(theta >= 0.0 && theta <= 1.0)) return bad("theta must be in [0, 1]");
  if (!finite_pos(rtol)) return bad("rtol must be finite and > 0");
  if (nsteps < 0) return bad("nsteps must be >= 0");
  if (out) {
    if (out->save_every < 0) return bad("save_every must be >= 0");
    if (out->n_sensors < 0 || (out->n_sensors > 0 && !out->sensor_xyz)) return bad("bad sensor points");
    if (out->n_sensors > 0) {
      std::vector<double> p;
      if (!fetch(out->sensor_xyz, 3 * (size_t)out->n_sensors, dev, p)) {
        why = "reading sensor points failed";
        return FEM_EDEVICE;
      }
      const double L[3] = {g.nx * g.hx, g.ny * g.hy, g.nz * g.hz};
      for (int32_t s = 0; s < out->n_sensors; ++s)
        for (int d = 0; d < 3; ++d) {
          const double v = p[3 * (size_t)s + d], tol = 1e-12 * L[d];
          if (!std::isfinite(v) || v < -tol || v > L[d] + tol) return bad("sensor point outside the domain");
        }
    }
  }
  return FEM_OK;
}

}  // namespace

extern "C" {

void fem_heat_default_opts(fem_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = FEM_FP64;
  o->max_iter = 10000;
  o->replace_every = 50;
  o->guess = FEM_GUESS_EXTRAP;
  o->stop_rule = FEM_STOP_RHS;
  o->max_refine = 4;
  o->inner_rtol = 1e-5;
  o->precond = FEM_PRECOND_JACOBI;
  o->cheb_degree = 3;
  o->cheb_ratio = 30.0;
}

const char* fem_strerror(int status) {
  switch (status) {
    case FEM_OK: return "ok";
    case FEM_EINVAL: return "invalid argument";
    case FEM_ENOMEM: return "out of memory";
    case FEM_ENOCONV: return "a step reached max_iter without converging";
    case FEM_EBREAKDOWN: return "conjugate gradient breakdown";
    case FEM_EDEVICE: return "HIP runtime error";
    case FEM_EBUSY: return "busy";
    case FEM_ECANCELED: return "cancelled";
    default: return "unknown status";
  }
}

const char* fem_last_error(const fem_heat* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int fem_heat_create(const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc,
                    const fem_opts* opts, fem_heat** out) {
  g_create_error.clear();
  if (!out) return FEM_EINVAL;
  *out = nullptr;
  fem_opts o;
  int rc = check_opts(opts, o, g_create_error);
  if (rc == FEM_OK) rc = check_problem(grid, k_e, rhoc_e, bc, o, g_create_error);
  if (rc != FEM_OK) return rc;
  return femheat::make_handle(grid, k_e, rhoc_e, bc, o, false, out, &g_create_error);
}

int fem_heat_run(fem_heat* h, const double* T0, const double* T_prev, double dt, double theta, int32_t nsteps,
                 double rtol, fem_out* out) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  const int rc = check_run(h->g, h->devptrs, T0, dt, theta, rtol, nsteps, out, h->err);
  if (rc != FEM_OK) return rc;
  try {
    return femheat::solver_run(h, T0, T_prev, dt, theta, nsteps, rtol, out);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return FEM_ENOMEM;
  } catch (...) {
    h->err = "unexpected exception";
    return FEM_EDEVICE;
  }
}

int fem_heat_run_batch(const fem_request* reqs, int32_t n, const fem_opts* opts, int32_t* status) {
  g_create_error.clear();
  if (n < 0 || (n > 0 && !reqs)) {
    g_create_error = "reqs and n >= 0 are required";
    return FEM_EINVAL;
  }
  if (n == 0) return FEM_OK;
  std::vector<int32_t> st((size_t)n, FEM_OK);
  fem_opts o;
  int rc = check_opts(opts, o, g_create_error);
  if (rc != FEM_OK) return rc;
  // validate every request before anything runs
  int first_bad = FEM_OK;
  for (int32_t i = 0; i < n && first_bad == FEM_OK; ++i) {
    const fem_request& r = reqs[i];
    std::string why;
    int v = check_problem(&r.grid, r.k_e, r.rhoc_e, &r.bc, o, why);
    if (v == FEM_OK) {
      femheat::Geom g{};
      g.nx = r.grid.nx;
      g.ny = r.grid.ny;
      g.nz = r.grid.nz;
      g.hx = r.grid.hx;
      g.hy = r.grid.hy;
      g.hz = r.grid.hz;
      v = check_run(g, (o.flags & FEM_DEVICE_PTRS) != 0, r.T0, r.dt, r.theta, r.rtol, r.nsteps, r.out, why);
    }
    if (v != FEM_OK) {
      st[(size_t)i] = v;
      first_bad = v;
      g_create_error = "request " + std::to_string(i) + ": " + why;
    }
  }
  if (first_bad != FEM_OK) {
    if (status) std::copy(st.begin(), st.end(), status);
    return first_bad;
  }
  if (hipSetDevice(o.device) != hipSuccess) {
    g_create_error = "hipSetDevice failed";
    return FEM_EDEVICE;
  }
  // G concurrent batches, simulations dealt round-robin, each batch on its
  // own stream and host thread: while one batch runs the last iterations of
  // its slowest member (few blocks), the others fill the device.  A
  // simulation's results do not depend on its batch, so the grouping changes
  // no result.
  // Automatic: one batch per 16 simulations and per 2^21 nodes, at most
  // three.  Measured on 64 x 48^3 in the mixed form (7.5M nodes), medians of
  // three: 92 solves/s as one batch, 105 as two, 108 as three, 92 as four
  // (the streams with the caller's then outnumber the four hardware queues a
  // process gets by default).  Batches of small simulations are bound by
  // launches, not by their tails, and stay whole: 32 x 19k nodes ran 20%
  // slower as two.
  uint64_t nodes = 0;
  for (int32_t i = 0; i < n; ++i)
    nodes += (uint64_t)(reqs[i].grid.nx + 1) * (uint64_t)(reqs[i].grid.ny + 1) * (uint64_t)(reqs[i].grid.nz + 1);
  const int auto_g = (int)std::min<uint64_t>({3u, (uint64_t)n / 16u, nodes >> 21});
  const int G = std::max(1, std::min<int>(n, o.batch_groups > 0 ? o.batch_groups : auto_g));
  hipStream_t caller = reinterpret_cast<hipStream_t>(o.hip_stream);
  std::vector<hipStream_t> gs((size_t)G, nullptr);
  std::vector<bool> own((size_t)G, false);
  hipEvent_t start = nullptr;
  for (int g = 0; g < G && rc == FEM_OK; ++g) {
    if (G == 1 && caller) {
      gs[0] = caller;
      break;
    }
    if (hipStreamCreateWithFlags(&gs[(size_t)g], hipStreamNonBlocking) != hipSuccess) {
      g_create_error = "hipStreamCreate failed";
      rc = FEM_EDEVICE;
      break;
    }
    own[(size_t)g] = true;
  }
  // the batches start after the work the caller enqueued on its stream
  if (rc == FEM_OK && caller && G > 1) {
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess || hipEventRecord(start, caller) != hipSuccess) {
      g_create_error = "hipEventRecord failed";
      rc = FEM_EDEVICE;
    }
    for (int g = 0; g < G && rc == FEM_OK; ++g)
      if (hipStreamWaitEvent(gs[(size_t)g], start, 0) != hipSuccess) {
        g_create_error = "hipStreamWaitEvent failed";
        rc = FEM_EDEVICE;
      }
  }
  std::vector<fem_heat*> hs((size_t)n, nullptr);
  std::vector<std::vector<femheat::RunRequest>> rq((size_t)G);
  std::vector<std::vector<int32_t>> idx((size_t)G), gst((size_t)G);
  std::vector<int> grc((size_t)G, FEM_OK);
  std::vector<std::string> gerr((size_t)G);
  try {
    for (int32_t i = 0; i < n && rc == FEM_OK; ++i) {
      const fem_request& r = reqs[i];
      const size_t g = (size_t)(i % G);
      fem_opts og = o;
      og.hip_stream = gs[g];
      rc = femheat::make_handle(&r.grid, r.k_e, r.rhoc_e, &r.bc, og, true, &hs[(size_t)i], &g_create_error);
      rq[g].push_back(femheat::RunRequest{hs[(size_t)i], r.T0, r.T_prev, r.dt, r.theta, r.rtol, r.nsteps, r.out});
      idx[g].push_back(i);
    }
    auto run_group = [&](size_t g) {
      fem_opts og = o;
      og.hip_stream = gs[g];
      gst[g].assign(rq[g].size(), FEM_OK);
      try {
        if (G > 1 && hipSetDevice(o.device) != hipSuccess) {
          gerr[g] = "hipSetDevice failed";
          grc[g] = FEM_EDEVICE;
          return;
        }
        grc[g] = femheat::engine_run(rq[g].data(), (int32_t)rq[g].size(), gs[g], og, gst[g].data(), &gerr[g]);
      } catch (const std::bad_alloc&) {
        gerr[g] = "host allocation failed";
        grc[g] = FEM_ENOMEM;
      } catch (...) {
        gerr[g] = "unexpected exception";
        grc[g] = FEM_EDEVICE;
      }
    };
    if (rc == FEM_OK) {
      if (G == 1) {
        run_group(0);
      } else {
        std::vector<std::thread> th;
        for (int g = 1; g < G; ++g) th.emplace_back(run_group, (size_t)g);
        run_group(0);
        for (auto& t : th) t.join();
      }
      for (int g = 0; g < G && rc == FEM_OK; ++g)
        if (grc[(size_t)g] != FEM_OK) {
          rc = grc[(size_t)g];
          g_create_error = gerr[(size_t)g];
        }
      for (int g = 0; g < G; ++g)
        for (size_t q = 0; q < idx[(size_t)g].size(); ++q) st[(size_t)idx[(size_t)g][q]] = gst[(size_t)g][q];
    }
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    rc = FEM_ENOMEM;
  } catch (...) {
    g_create_error = "unexpected exception";
    rc = FEM_EDEVICE;
  }
  for (fem_heat* h : hs) {
    if (!h) continue;
    femheat::solver_free(h);
    delete h;
  }
  for (int g = 0; g < G; ++g)
    if (own[(size_t)g]) {
      (void)hipStreamSynchronize(gs[(size_t)g]);
      (void)hipStreamDestroy(gs[(size_t)g]);
    }
  if (start) (void)hipEventDestroy(start);
  if (rc != FEM_OK) return rc;
  if (status) std::copy(st.begin(), st.end(), status);
  for (int32_t v : st)
    if (v != FEM_OK) return v;
  return FEM_OK;
}

int fem_heat_apply(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  const int op = which & 0xff;
  if ((which & ~(0xff | FEM_OP_FP32 | FEM_OP_ELEMENTWISE | FEM_OP_ROWWAVE)) || op > FEM_OP_LOAD) {
    h->err = "unknown operator";
    return FEM_EINVAL;
  }
  const int32_t form = which & (FEM_OP_ELEMENTWISE | FEM_OP_ROWWAVE);
  if (form && (form == (FEM_OP_ELEMENTWISE | FEM_OP_ROWWAVE) || (which & FEM_OP_FP32) ||
               (op != FEM_OP_A && op != FEM_OP_L) || h->opts.element != FEM_ELEM_HEX8)) {
    h->err = "the element-by-element and row-wavefront applies take one of FEM_OP_A, FEM_OP_L in FP64";
    return FEM_EINVAL;
  }
  if (!y || (op != FEM_OP_LOAD && !x)) {
    h->err = "x and y are required";
    return FEM_EINVAL;
  }
  if (!finite_pos(dt) || !(theta >= 0.0 && theta <= 1.0)) {
    h->err = "dt must be > 0 and theta in [0, 1]";
    return FEM_EINVAL;
  }
  try {
    return femheat::solver_apply(h, which, dt, theta, x, y);
  } catch (...) {
    h->err = "unexpected exception";
    return FEM_EDEVICE;
  }
}

int fem_heat_apply_noalloc(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  const int op = which & 0xff;
  if ((which & ~(0xff | FEM_OP_ELEMENTWISE)) || (op != FEM_OP_A && op != FEM_OP_L)) {
    h->err = "fem_heat_apply_noalloc takes FEM_OP_A or FEM_OP_L, optionally with FEM_OP_ELEMENTWISE";
    return FEM_EINVAL;
  }
  if ((which & FEM_OP_ELEMENTWISE) && h->opts.element != FEM_ELEM_HEX8) {
    h->err = "the element-by-element apply takes the hexahedral element";
    return FEM_EINVAL;
  }
  if (!x || !y) {
    h->err = "x and y are required";
    return FEM_EINVAL;
  }
  if (!finite_pos(dt) || !(theta >= 0.0 && theta <= 1.0)) {
    h->err = "dt must be > 0 and theta in [0, 1]";
    return FEM_EINVAL;
  }
  try {
    return femheat::solver_apply_noalloc(h, which, dt, theta, x, y);
  } catch (...) {
    h->err = "unexpected exception";
    return FEM_EDEVICE;
  }
}

int fem_heat_tune(fem_heat* h, double dt, double theta, uint32_t flags, fem_tune_result* out) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  if (!finite_pos(dt) || !(theta >= 0.0 && theta <= 1.0) || (flags & ~(uint32_t)FEM_TUNE_BATCH)) {
    h->err = "dt must be > 0, theta in [0, 1], flags FEM_TUNE_BATCH or 0";
    return FEM_EINVAL;
  }
  try {
    return femheat::engine_tune(h, dt, theta, flags, out);
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return FEM_ENOMEM;
  } catch (...) {
    h->err = "unexpected exception";
    return FEM_EDEVICE;
  }
}

int fem_server_create(const fem_server_opts* opts, fem_server** out) {
  g_create_error.clear();
  if (!out) return FEM_EINVAL;
  *out = nullptr;
  fem_server_opts so{};
  fem_heat_default_opts(&so.opts);
  if (opts) so = *opts;
  fem_opts o;
  int rc = check_opts(&so.opts, o, g_create_error);
  if (rc != FEM_OK) return rc;
  if (o.flags & (FEM_DEVICE_PTRS | FEM_TIMING)) {
    g_create_error = "the server takes host pointers and does not time kernels";
    return FEM_EINVAL;
  }
  if (so.max_slots < 0) {
    g_create_error = "max_slots must be >= 0";
    return FEM_EINVAL;
  }
  so.opts = o;
  try {
    return femheat::server_create(so, out, &g_create_error);
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return FEM_ENOMEM;
  } catch (...) {
    g_create_error = "unexpected exception";
    return FEM_EDEVICE;
  }
}

int fem_server_submit(fem_server* s, const fem_request* req, uint64_t* ticket) {
  g_create_error.clear();
  if (!s || !req || !ticket) {
    g_create_error = "server, request and ticket are required";
    return FEM_EINVAL;
  }
  fem_opts o;
  fem_heat_default_opts(&o);  // host pointers: validation reads them directly
  int rc = check_problem(&req->grid, req->k_e, req->rhoc_e, &req->bc, o, g_create_error);
  if (rc == FEM_OK) {
    femheat::Geom g{};
    g.nx = req->grid.nx;
    g.ny = req->grid.ny;
    g.nz = req->grid.nz;
    g.hx = req->grid.hx;
    g.hy = req->grid.hy;
    g.hz = req->grid.hz;
    rc = check_run(g, false, req->T0, req->dt, req->theta, req->rtol, req->nsteps, req->out, g_create_error);
  }
  if (rc != FEM_OK) return rc;
  try {
    return femheat::server_submit(s, *req, ticket, &g_create_error);
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return FEM_ENOMEM;
  }
}

int fem_server_poll(fem_server* s, uint64_t ticket, fem_status* st) {
  if (!s || !st) return FEM_EINVAL;
  return femheat::server_poll(s, ticket, st);
}

int fem_server_wait(fem_server* s, uint64_t ticket, double timeout_s, fem_status* st) {
  if (!s) return FEM_EINVAL;
  return femheat::server_wait(s, ticket, timeout_s, st);
}

int fem_server_cancel(fem_server* s, uint64_t ticket) {
  if (!s) return FEM_EINVAL;
  return femheat::server_cancel(s, ticket);
}

int fem_server_info_get(fem_server* s, fem_server_info* info) {
  if (!s || !info) return FEM_EINVAL;
  return femheat::server_info(s, info);
}

void fem_server_destroy(fem_server* s) {
  if (s) femheat::server_destroy(s);
}

int fem_heat_stats(const fem_heat* h, fem_stats* out) {
  if (!h || !out) return FEM_EINVAL;
  *out = h->stats;
  return FEM_OK;
}

void fem_heat_destroy(fem_heat* h) {
  if (!h) return;
  femheat::solver_free(h);
  delete h;
}

}  // extern "C"
