// extern "C" entry points of include/fem_heat.h: argument validation, handle
// lifetime and error reporting.  The work itself is in solver.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

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
  auto bad = [](const char* m) {
    g_create_error = m;
    return FEM_EINVAL;
  };
  if (!grid || !k_e || !rhoc_e) return bad("grid, k_e and rhoc_e are required");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return bad("nx, ny, nz must be >= 1");
  const double N = (double)(grid->nx + 1) * (grid->ny + 1) * (grid->nz + 1);
  if (N >= 2147483647.0) return bad("grid too large (N must fit in 31 bits)");
  if (!finite_pos(grid->hx) || !finite_pos(grid->hy) || !finite_pos(grid->hz)) return bad("h must be finite and > 0");
  fem_opts o;
  fem_heat_default_opts(&o);
  if (opts) o = *opts;
  if (o.precision != FEM_FP64 && o.precision != FEM_FP32_FP64DOT) return bad("unknown precision");
  if (o.max_iter < 0 || o.replace_every < 0 || o.max_refine < 0) return bad("negative iteration controls");
  if (o.guess != FEM_GUESS_EXTRAP && o.guess != FEM_GUESS_PREV) return bad("unknown guess rule");
  if (o.stop_rule != FEM_STOP_RHS && o.stop_rule != FEM_STOP_INITIAL) return bad("unknown stop rule");
  if (o.precision == FEM_FP32_FP64DOT && !finite_pos(o.inner_rtol)) return bad("inner_rtol must be > 0");
  if (o.tile_x < 0 || o.tile_y < 0 || o.tile_z < 0 || o.tile_x > 256 || o.tile_x * std::max(o.tile_y, 1) > 256)
    return bad("tile overrides out of range");
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
    g_create_error = "hipSetDevice failed";
    return FEM_EDEVICE;
  }
  std::vector<double> chk;
  if (!fetch(k_e, E, dev, chk)) {
    g_create_error = "reading k_e failed";
    return FEM_EDEVICE;
  }
  for (double v : chk)
    if (!(v >= 0.0) || !std::isfinite(v)) return bad("k_e must be finite and >= 0");
  if (!fetch(rhoc_e, E, dev, chk)) {
    g_create_error = "reading rhoc_e failed";
    return FEM_EDEVICE;
  }
  for (double v : chk)
    if (!finite_pos(v)) return bad("rhoc_e must be finite and > 0");

  fem_heat* h = new (std::nothrow) fem_heat();
  if (!h) return FEM_ENOMEM;
  h->opts = o;
  h->devptrs = dev;
  h->timing = (o.flags & FEM_TIMING) != 0;
  h->device = o.device;
  int rc = femheat::solver_init(h, grid, k_e, rhoc_e, bc);
  if (rc != FEM_OK) {
    g_create_error = h->err;
    femheat::solver_free(h);
    delete h;
    return rc;
  }
  *out = h;
  return FEM_OK;
}

int fem_heat_run(fem_heat* h, const double* T0, const double* T_prev, double dt, double theta, int32_t nsteps,
                 double rtol, fem_out* out) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  auto bad = [h](const char* m) {
    h->err = m;
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
      if (!fetch(out->sensor_xyz, 3 * (size_t)out->n_sensors, h->devptrs, p)) return FEM_EDEVICE;
      const double L[3] = {h->g.nx * h->g.hx, h->g.ny * h->g.hy, h->g.nz * h->g.hz};
      for (int32_t s = 0; s < out->n_sensors; ++s)
        for (int d = 0; d < 3; ++d) {
          const double v = p[3 * (size_t)s + d], tol = 1e-12 * L[d];
          if (!std::isfinite(v) || v < -tol || v > L[d] + tol) return bad("sensor point outside the domain");
        }
    }
  }
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

int fem_heat_apply(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  if (!h) return FEM_EINVAL;
  h->err.clear();
  const int op = which & 0xff;
  if ((which & ~(0xff | FEM_OP_FP32)) || op > FEM_OP_LOAD) {
    h->err = "unknown operator";
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
