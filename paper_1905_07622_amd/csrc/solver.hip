// Set-up, operator test hook and teardown of a solver handle (gfx950).
//
// One handle keeps a whole problem resident in HBM: coefficients, load
// vector, Jacobi preconditioner, the previous fields and the PCG vectors.
// Creating it uploads the coefficients and builds the boundary load vector
// (Sec. 3.1); the time stepping itself lives in engine.hip, which drives one
// handle or a batch of them.
#include <algorithm>
#include <array>
#include <new>
#include <cmath>
#include <cstring>
#include <mutex>

#include "ebe.hpp"
#include "engine.hpp"
#include "rowwave.hpp"
#include "runtime.hpp"
#include "tune.hpp"
#include "vector_kernels.hpp"

// Scratch of fem_heat_apply_noalloc, for callers that cannot allocate: the
// element-by-element form's 4 N partial sums (N <= kNoallocMaxNodes) and a
// sink for the gather's stores of lanes without a node (one value per thread
// of a block).  One copy
// per GPU, held until the process ends.  Host code never passes this name to
// a kernel (on the host it is only a stand-in); it uses the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocMaxNodes = size_t(1) << 20;
constexpr size_t kNoallocSink = femheat::kMaxBlockThreads;
static __device__ __align__(256) double scratch[4 * kNoallocMaxNodes + kNoallocSink];

namespace femheat {
namespace {

// Device address of `scratch` per device ordinal, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
std::array<double*, kMaxDevices> scratch_dev{};

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
template <typename V, int KIND>
hipError_t occupancy_of(int* n, int nthreads, size_t smem) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      n, reinterpret_cast<const void*>(&gather_kernel<V, KIND, ProDirection<V>, EpiQDot<V>>), nthreads, smem);
}

int resident_blocks(int kind, bool fp32, int nthreads, size_t smem) {
  int n = 0;
  hipError_t e;
  if (fp32)
    e = kind == kElemCubic ? occupancy_of<float, kElemCubic>(&n, nthreads, smem)
        : kind == kElemTet6 ? occupancy_of<float, kElemTet6>(&n, nthreads, smem)
                            : occupancy_of<float, kElemBox>(&n, nthreads, smem);
  else
    e = kind == kElemCubic ? occupancy_of<double, kElemCubic>(&n, nthreads, smem)
        : kind == kElemTet6 ? occupancy_of<double, kElemTet6>(&n, nthreads, smem)
                            : occupancy_of<double, kElemBox>(&n, nthreads, smem);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 2;
  }
  return std::max(n, 1);
}

// Launch shape of the gather: TX spans the x-row of nodes in as few equal
// pieces as possible, TY fills the block: pieces of at most 128 and blocks of
// at most 512 threads for a simulation alone (one block of eight waves per
// CU), of at most 64 and 256 threads for a batch member.  Unless given, TZ
// splits the columns of a simulation that has the GPU to itself into as
// many z-chunks as the chip holds blocks at once (`capacity`): the gather is
// latency-bound, so the launch should fill every CU to its occupancy limit
// in a single round -- a second, partial round of blocks costs a whole
// extra block time -- and longer z-marches pay the start-up of the plane
// pipeline less often.  capacity <= 0 selects the rule for members of a
// batch; wide = false the narrow blocks for a simulation alone too (the
// rule of a grid too small to give every CU a wide block).
GatherShape choose_shape(const Geom& g, const fem_opts& o, int capacity, bool wide = true) {
  GatherShape s{};
  const int px = g.px, py = g.py, pz = g.pz;
  const bool alone = capacity > 0;
  const int piece = alone && wide ? 128 : 64;
  int tx = o.tile_x > 0 ? o.tile_x : (px + (px + piece - 1) / piece - 1) / ((px + piece - 1) / piece);
  const int lim = alone && (wide || o.tile_x > 0) ? kMaxBlockThreads : kMaxBatchThreads;
  tx = std::max(1, std::min(tx, lim));
  int ty;
  if (o.tile_y > 0) {
    ty = o.tile_y;
  } else {
    const int tymax = std::max(1, lim / tx);
    const int nty = (py + tymax - 1) / tymax;
    ty = (py + nty - 1) / nty;
  }
  ty = std::max(1, std::min(ty, lim / tx));
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
  } else if (capacity <= 0) {
    // a member of a batch: the launch is filled by many simulations, so each
    // marches chunks of at most 32 planes (balanced); the rule depends on the
    // simulation's own grid only, which keeps its results independent of
    // what it shares the launch with
    const int nchunks = (pz + 31) / 32;
    tz = (pz + nchunks - 1) / nchunks;
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
void fill_classes(const Geom& g, GatherArgs<V>& ga, double cm, double ck, int kind) {
  if (kind == kElemCubic || kind == kElemTet6) {
    // cube of side h: hexahedron classes h^3/216 {8,4,2,1}, h/12 {4,0,-1,-1};
    // tetrahedra h^3/120 kTetM, h/6 kTetK
    const double h = g.hx;
    const bool tet = kind == kElemTet6;
    ga.sa = (V)(cm * h * h * h / (tet ? 120.0 : 216.0));
    ga.sb = (V)(ck * h / (tet ? 6.0 : 12.0));
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

Relay no_relay() { return Relay{nullptr, nullptr, nullptr, 0, nullptr, M_NONE, Ctl{0.0, 0, 0}, 0}; }

// Upper end of the Chebyshev interval: a bound of the spectrum of D^-1 A for
// every coefficient field on this element box.  x^T A x / x^T D x is a
// weighted mean of element quotients, each at most the larger of
// lambda_max(diag(M_e)^-1 M_e) and lambda_max(diag(K_e)^-1 K_e).  Both blocks
// have a constant diagonal (V/27 and (V/9) sum_d 1/h_d^2) and the eigenvectors
// of the tensor products of the 1-D blocks: per axis, the even mode gives the
// mass entry h/2 and stiffness 0, the odd mode h/6 and 2/h.  So the mass
// block's top is (V/8)/(V/27) = 27/8 and the stiffness block's the largest of
// sum_d s_d prod_{d' != d} m_d' over the 8 parity patterns.
double chebyshev_upper(const Geom& g) {
  const double h[3] = {g.hx, g.hy, g.hz};
  const double V = g.hx * g.hy * g.hz;
  const double kdiag = V / 9.0 * (1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]));
  double ktop = 0.0;
  for (int o = 0; o < 8; ++o) {
    double lam = 0.0;
    for (int d = 0; d < 3; ++d) {
      if (!((o >> d) & 1)) continue;  // even mode along d: the stiffness factor is 0
      double t = 2.0 / h[d];
      for (int e = 0; e < 3; ++e)
        if (e != d) t *= ((o >> e) & 1) ? h[e] / 6.0 : h[e] / 2.0;
      lam += t;
    }
    ktop = std::max(ktop, lam);
  }
  return std::max(27.0 / 8.0, ktop / kdiag);
}

// The Chebyshev preconditioner of degree m on [hi/ratio, hi]: with centre c,
// half-width w and sigma = c/w, rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1});
// step k of the chain forms d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / w) P^-1 res_k.
void chebyshev_coefficients(fem_heat* h) {
  const double hi = chebyshev_upper(h->g), lo = hi / h->opts.cheb_ratio;
  const double c = 0.5 * (hi + lo), w = 0.5 * (hi - lo), sigma = c / w;
  h->ch_hi = hi;
  h->ch_lo = lo;
  h->ch_inv_c = 1.0 / c;
  double rho = 1.0 / sigma;
  for (int k = 1; k < h->opts.cheb_degree && k <= kChebMaxDegree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    h->ch_a[k - 1] = rn * rho;
    h->ch_b[k - 1] = 2.0 * rn / w;
    rho = rn;
  }
}

}  // namespace

template <typename V>
GatherArgs<V> gather_args(const fem_heat* h, double cm, double ck) {
  GatherArgs<V> ga{};
  ga.g = h->g;
  ga.s = h->shape;
  if constexpr (sizeof(V) == 8) {
    ga.rhoc = h->rhoc64;
    ga.kc = h->k64;
  } else {
    ga.rhoc = h->rhoc32;
    ga.kc = h->k32;
  }
  ga.sink = reinterpret_cast<V*>(h->sink);
  fill_classes(h->g, ga, cm, ck, h->kind);
  return ga;
}
template GatherArgs<double> gather_args<double>(const fem_heat*, double, double);
template GatherArgs<float> gather_args<float>(const fem_heat*, double, double);

namespace {

// One gather of one handle outside the time stepping (set-up, test hook);
// `sink` (>= kMaxBlockThreads values) replaces the handle's sink when given.
template <typename V, class Pro, class Epi>
int launch_gather(fem_heat* h, double cm, double ck, Pro pro, Epi epi, const Relay& R, V* sink = nullptr) {
  GatherArgs<V> ga = gather_args<V>(h, cm, ck);
  if (sink) ga.sink = sink;
  const size_t smem = h->shape.smem_bytes(sizeof(V));
  if (h->kind == kElemCubic)
    hipLaunchKernelGGL((gather_kernel<V, kElemCubic, Pro, Epi>), dim3(h->shape.nblocks), dim3(h->shape.nthreads),
                       smem, h->stream, ga, pro, epi, R);
  else if (h->kind == kElemTet6)
    hipLaunchKernelGGL((gather_kernel<V, kElemTet6, Pro, Epi>), dim3(h->shape.nblocks), dim3(h->shape.nthreads),
                       smem, h->stream, ga, pro, epi, R);
  else
    hipLaunchKernelGGL((gather_kernel<V, kElemBox, Pro, Epi>), dim3(h->shape.nblocks), dim3(h->shape.nthreads), smem,
                       h->stream, ga, pro, epi, R);
  HIP_TRY(hipGetLastError());
  return FEM_OK;
}

// Element-by-element apply y = (M + ck K) x in two passes (comparison form)
// with its 4 N partial sums in `part`.
void launch_ebe(fem_heat* h, double ck, const double* x, double* part, double* y) {
  const uint32_t N = h->g.N;
  GatherArgs<double> ga{};
  fill_classes(h->g, ga, 1.0, ck, false);  // the general class entries hold for any box
  EbeArgs ea{};
  ea.nx = h->g.nx;
  ea.ny = h->g.ny;
  ea.nz = h->g.nz;
  ea.px = h->g.px;
  ea.py = h->g.py;
  ea.N = N;
  ea.nseg = (uint32_t)((h->g.nx + kEbeStore - 1) / kEbeStore);
  ea.x = x;
  ea.rhoc = h->rhoc64;
  ea.kc = h->k64;
  ea.part = part;
  for (int c = 0; c < 8; ++c) {
    ea.Mc[c] = ga.sa * ga.Mc[c];
    ea.Kc[c] = ga.sb * ga.Kc[c];
  }
  const uint64_t waves = (uint64_t)ea.nseg * (uint64_t)h->g.ny * (uint64_t)h->g.nz;
  hipLaunchKernelGGL(ebe_elements_kernel, dim3((uint32_t)((waves + 3) / 4)), dim3(256), 0, h->stream, ea);
  hipLaunchKernelGGL(ebe_sum_kernel, dim3(std::min<uint32_t>(nblk(N), 4096)), dim3(kT), 0, h->stream, ea, y);
}

}  // namespace

// Looks up the device address of `scratch` on the handle's device (current)
// the first time a handle is created there, and gives it to the handle.
int noalloc_scratch_setup(fem_heat* h) {
  const int dev = h->opts.device;
  if (dev < 0 || dev >= kMaxDevices) return fail(h, FEM_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[(size_t)dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(h, FEM_EDEVICE, "hipGetSymbolAddress(scratch) failed");
    }
    scratch_dev[(size_t)dev] = static_cast<double*>(p);
  }
  h->noalloc_scratch = scratch_dev[(size_t)dev];
  return FEM_OK;
}

int solver_apply_noalloc(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  const uint32_t N = h->g.N;
  const bool ebe = (which & FEM_OP_ELEMENTWISE) != 0;
  const int op = which & 0xff;
  if (ebe && (size_t)N > kNoallocMaxNodes)
    return fail(h, FEM_EINVAL, "the element-by-element form without allocation takes at most 2^20 nodes");
  double* part = h->noalloc_scratch;
  double* sink = h->noalloc_scratch + 4 * kNoallocMaxNodes;
  if (!part) return fail(h, FEM_EDEVICE, "scratch address not set up");
  HIP_TRY(hipSetDevice(h->opts.device));
  const double ck = op == FEM_OP_A ? theta * dt : -(1.0 - theta) * dt;
  if (ebe) {
    launch_ebe(h, ck, x, part, y);
  } else {
    RC_TRY(launch_gather<double>(h, 1.0, ck, ProPlain<double>{x}, EpiStore<double>{y}, no_relay(), sink));
  }
  HIP_TRY(hipGetLastError());
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
  if (h->opts.flags & FEM_ONE_REDUCTION) {
    RC_TRY(dalloc(h, &h->r32b, N));
    RC_TRY(dalloc(h, &h->q32b, N));
  }
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(E)), dim3(kT), 0, h->stream, h->rhoc64, h->rhoc32, E);
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(E)), dim3(kT), 0, h->stream, h->k64, h->k32, E);
  HIP_TRY(hipGetLastError());
  h->ck_cached = -1.0;  // pinv32 must be (re)built
  return FEM_OK;
}

// Jacobi preconditioner (Sec. 3.3) and, for non-zero Dirichlet values, the lifting
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
    RC_TRY(launch_gather<double>(h, 1.0, ck, ProPlain<double>{gext},
                                 EpiStore<double>{h->lift64}, no_relay()));
    hipLaunchKernelGGL(mask_free_kernel, dim3(nblk(N)), dim3(kT), 0, h->stream, h->pinv64, h->lift64, N);
    HIP_TRY(hipGetLastError());
  }
  h->ck_cached = ck;
  return FEM_OK;
}

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
  g.tet6 = h->opts.element == FEM_ELEM_TET6 ? 1 : 0;
  h->kind = g.tet6 ? kElemTet6 : (h->cubic ? kElemCubic : kElemBox);
  HIP_TRY(hipSetDevice(h->opts.device));
  RC_TRY(noalloc_scratch_setup(h));
  if (h->batched && h->opts.tile_x * std::max(h->opts.tile_y, 1) > kMaxBatchThreads)
    return fail(h, FEM_EINVAL, "tile overrides of batch members and served simulations: tile_x * tile_y <= 256");
  {
    // a tile the autotuner recorded for this grid, precision, element class
    // and launch kind (alone or in a batch) replaces the rule
    fem_opts so = h->opts;
    if (so.tune_cache && so.tile_x == 0 && so.tile_y == 0 && so.tile_z == 0) {
      int t[3];
      if (tune_lookup(so.tune_cache, tune_key(so.device, so.precision == FEM_FP32_FP64DOT, h->kind, h->batched,
                                              g.px, g.py, g.pz),
                      t)) {
        fem_opts probe_o = so;
        probe_o.tile_x = t[0];
        probe_o.tile_y = t[1];
        probe_o.tile_z = t[2];
        if (shape_stages(choose_shape(g, probe_o, 1))) {
          so = probe_o;
          h->tuned = true;
        }
      }
    }
    const bool fp32 = h->opts.precision == FEM_FP32_FP64DOT;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->opts.device));
    cus = std::max(1, cus);
    auto rule = [&](bool wide, int* capacity) {
      // the x-y tiling does not depend on the capacity: size the block first
      const GatherShape probe = choose_shape(g, so, 1, wide);
      // at most two blocks per CU: beyond that, the shorter z-marches pay the
      // plane pipeline's fill more often than the extra blocks hide latency
      // (measured for the FP32 gather, which could hold four); one block of
      // eight waves (blocks sharing a CU drift apart, the older one first)
      const int per_cu = std::min(probe.nthreads > kMaxBatchThreads ? 1 : 2,
                                  resident_blocks(h->kind, fp32, probe.nthreads, probe.smem_bytes(fp32 ? 4 : 8)));
      *capacity = cus * std::max(per_cu, 1);
      return choose_shape(g, so, h->batched ? 0 : *capacity, wide);
    };
    int cap = 0;
    h->shape = rule(true, &cap);
    // wide blocks only where they give (nearly) every CU one: a small grid
    // keeps narrow blocks, twice as many (measured at 49^3 nodes: 65 wide
    // blocks 13.0 us, 130 narrow ones 10.7 us per direction gather)
    if (!h->batched && so.tile_x == 0 && h->shape.nthreads > kMaxBatchThreads && 10 * h->shape.ntiles < 9u * cus)
      h->shape = rule(false, &cap);
    h->capacity = cap;
  }
  {
    const GatherShape& s = h->shape;
    if ((s.tx + 2) * (s.ty + 2) > kSlots * s.nthreads || (s.tx + 1) * (s.ty + 1) > kSlots * s.nthreads)
      return fail(h, FEM_EINVAL, "tile shape too thin for the staging scheme");
  }
  h->upd_blocks64 = std::max<uint32_t>(1, std::min<uint32_t>(nblk((g.N + 1) / 2), 512));
  h->upd_blocks32 = std::max<uint32_t>(1, std::min<uint32_t>(nblk((g.N + 3) / 4), 512));
  h->start_blocks = std::max<uint32_t>(1, std::min<uint32_t>(nblk(g.N), 1024));
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
  const bool one_red = (h->opts.flags & FEM_ONE_REDUCTION) != 0;
  if (one_red && h->opts.precision == FEM_FP64) {  // (the mixed form's FP32 set has its own, below)
    RC_TRY(dalloc(h, &h->r64b, N));
    RC_TRY(dalloc(h, &h->q64b, N));
  }
  RC_TRY(dalloc(h, &h->d64[0], N));
  RC_TRY(dalloc(h, &h->d64[1], N));
  for (auto& p : h->pool) RC_TRY(dalloc(h, &p, N));
  if (h->nonzero_dirichlet) RC_TRY(dalloc(h, &h->lift64, N));
  RC_TRY(dalloc(h, &h->sink, kMaxBlockThreads));
  h->n_partials = std::max({h->shape.nblocks, h->upd_blocks64, h->upd_blocks32, h->start_blocks});
  const size_t ncomp = one_red ? 4 : 1;  // the one-reduction direction kernel publishes four sums per block
  for (RelayCtx* c : {&h->outer, &h->inner})
    for (int k = 0; k < 2; ++k) {
      RC_TRY(dalloc(h, &c->S[k], 1));
      RC_TRY(dalloc(h, &c->P[k], ncomp * h->n_partials));
      HIP_TRY(hipMemsetAsync(c->S[k], 0, sizeof(Scalars), h->stream));
      HIP_TRY(hipMemsetAsync(c->P[k], 0, ncomp * h->n_partials * sizeof(double), h->stream));
    }
  if (h->opts.precond == FEM_PRECOND_CHEBYSHEV && h->opts.precision == FEM_FP64) {
    RC_TRY(dalloc(h, &h->s64, N));
    RC_TRY(dalloc(h, &h->cr64, N));
    RC_TRY(dalloc(h, &h->cd64[0], N));
    RC_TRY(dalloc(h, &h->cd64[1], N));
    chebyshev_coefficients(h);
  }
  RC_TRY(copy_in(h, h->rhoc64, rhoc_e, E));
  RC_TRY(copy_in(h, h->k64, k_e, E));
  hipLaunchKernelGGL(load_vector_kernel, dim3(nblk(N)), dim3(kT), 0, h->stream, g, h->F64);
  HIP_TRY(hipGetLastError());
  if (h->opts.precision == FEM_FP32_FP64DOT) RC_TRY(ensure_fp32(h));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FEM_OK;
}

int solver_apply(fem_heat* h, int32_t which, double dt, double theta, const double* x, double* y) {
  HIP_TRY(hipSetDevice(h->opts.device));
  const uint32_t N = h->g.N;
  const bool fp32 = (which & FEM_OP_FP32) != 0;
  const bool ebe = (which & FEM_OP_ELEMENTWISE) != 0;
  const bool rows = (which & FEM_OP_ROWWAVE) != 0;
  const int op = which & 0xff;
  double* xd = h->pool[0];
  double* yd = h->pool[1];
  if (op != FEM_OP_LOAD) RC_TRY(copy_in(h, xd, x, N));
  if (ebe && !h->ebe_part) RC_TRY(dalloc(h, &h->ebe_part, 4 * (size_t)N));
  if (h->timing) {
    for (auto& e : h->ev_apply)
      if (!e) HIP_TRY(hipEventCreate(&e));
    HIP_TRY(hipEventRecord(h->ev_apply[0], h->stream));
  }
  if ((op == FEM_OP_A || op == FEM_OP_L) && ebe) {
    const double ck = op == FEM_OP_A ? theta * dt : -(1.0 - theta) * dt;
    launch_ebe(h, ck, xd, h->ebe_part, yd);
  } else if ((op == FEM_OP_A || op == FEM_OP_L) && rows) {
    const double ck = op == FEM_OP_A ? theta * dt : -(1.0 - theta) * dt;
    GatherArgs<double> ga{};
    fill_classes(h->g, ga, 1.0, ck, kElemBox);
    RowArgs ra{};
    ra.nx = h->g.nx;
    ra.ny = h->g.ny;
    ra.nz = h->g.nz;
    ra.px = h->g.px;
    ra.py = h->g.py;
    ra.pz = h->g.pz;
    ra.nseg = (uint32_t)((h->g.px + kRowOwn - 1) / kRowOwn);
    ra.nwave = ra.nseg * (uint32_t)h->g.py * (uint32_t)h->g.pz;
    ra.nblk = (ra.nwave + 3) / 4;
    ra.share = (ra.nblk + 7) / 8;
    ra.x = xd;
    ra.rhoc = h->rhoc64;
    ra.kc = h->k64;
    ra.y = yd;
    for (int c = 0; c < 8; ++c) {
      ra.Mc[c] = ga.sa * ga.Mc[c];
      ra.Kc[c] = ga.sb * ga.Kc[c];
    }
    hipLaunchKernelGGL(rowwave_apply_kernel, dim3(8 * ra.share), dim3(256), 0, h->stream, ra);
  } else if (op == FEM_OP_A || op == FEM_OP_L) {
    const double ck = op == FEM_OP_A ? theta * dt : -(1.0 - theta) * dt;
    if (fp32) {
      RC_TRY(ensure_fp32(h));
      hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblk(N)), dim3(kT), 0, h->stream, xd, h->e32[0], N);
      RC_TRY(launch_gather<float>(h, 1.0, ck, ProPlain<float>{h->e32[0]}, EpiStore<float>{h->q32},
                                  no_relay()));
      hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nblk(N)), dim3(kT), 0, h->stream, h->q32, yd, N);
    } else {
      RC_TRY(launch_gather<double>(h, 1.0, ck, ProPlain<double>{xd}, EpiStore<double>{yd},
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
  if (h->timing) HIP_TRY(hipEventRecord(h->ev_apply[1], h->stream));
  RC_TRY(copy_out(h, y, yd, (size_t)N * sizeof(double)));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (h->timing) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev_apply[0], h->ev_apply[1]));
    h->stats.apply_calls += 1;
    h->stats.apply_ms += ms;
  }
  return FEM_OK;
}

// ---------------------------------------------------------------------------
// launch shapes for the autotuner

bool shape_stages(const GatherShape& s) {
  return s.tx >= 1 && s.ty >= 1 && s.tz >= 1 && s.tx * s.ty <= kMaxBlockThreads &&
         (s.tx + 2) * (s.ty + 2) <= kSlots * s.nthreads && (s.tx + 1) * (s.ty + 1) <= kSlots * s.nthreads;
}

GatherShape shape_with_tile(const fem_heat* h, int tx, int ty, int tz) {
  fem_opts o = h->opts;
  o.tile_x = tx;
  o.tile_y = ty;
  o.tile_z = tz;
  return choose_shape(h->g, o, h->batched ? 0 : h->capacity);
}

// Candidates: x pieces of the node row (1 to 4 equal pieces, and 16/32/64
// wide), block heights that the staging scheme holds in 256 threads (and,
// for a simulation alone, in 512: the largest, the one that splits the
// y-rows evenly, and half of it), and for each x-y tile a
// z-chunk length per target of resident blocks (1 to 4 per CU for a
// simulation alone; 8 to 32 planes or the whole column for batch members).
std::vector<GatherShape> tune_candidates(const fem_heat* h, int cus) {
  std::vector<GatherShape> out;
  // first the shape the launch kind gets without tuning: the handle's own
  // (the rule's, or the cached one) for a simulation alone, the batch rule's
  // for a batch member (a handle alone may have blocks wider than a batched
  // launch takes)
  out.push_back(h->batched ? choose_shape(h->g, h->opts, 0) : h->shape);
  const int px = h->g.px, py = h->g.py, pz = h->g.pz;
  std::vector<int> txs;
  for (int pieces = 1; pieces <= 4; ++pieces) {
    const int tx = (px + pieces - 1) / pieces;
    if (tx <= 128) txs.push_back(tx);
  }
  for (int tx : {16, 32, 64})
    if (tx < px) txs.push_back(tx);
  auto seen = [&](const GatherShape& s) {
    for (const GatherShape& o : out)
      if (o.tx == s.tx && o.ty == s.ty && o.tz == s.tz) return true;
    return false;
  };
  std::vector<std::pair<int, int>> txl;  // (tx, thread limit)
  for (int tx : txs) {
    txl.emplace_back(tx, kMaxBatchThreads);
    if (!h->batched) txl.emplace_back(tx, kMaxBlockThreads);
  }
  for (auto [tx, lim] : txl) {
    const int tymax = std::max(1, lim / tx);
    int fit = 0;
    for (int ty = std::min(tymax, py); ty >= 1; --ty) {
      const int nt = ((tx * ty + 63) / 64) * 64;
      if ((tx + 2) * (ty + 2) <= kSlots * nt && (tx + 1) * (ty + 1) <= kSlots * nt) {
        fit = ty;
        break;
      }
    }
    if (fit == 0 || (lim > kMaxBatchThreads && tx * fit <= kMaxBatchThreads)) continue;
    const int even = (py + ((py + fit - 1) / fit) - 1) / ((py + fit - 1) / fit);
    std::vector<int> tys = {fit, even, std::max(1, even / 2)};
    for (int ty : tys) {
      const int cols = ((px + tx - 1) / tx) * ((py + ty - 1) / ty);
      std::vector<int> tzs;
      if (h->batched) {
        tzs = {8, 12, 16, 24, 32};
        for (int c : {1, 2, 3, 4, 6}) tzs.push_back((pz + c - 1) / c);  // the column in c equal chunks
      } else {
        for (int per_cu = 1; per_cu <= 4; ++per_cu) {
          const int ntz = std::max(1, per_cu * cus / cols);
          tzs.push_back(std::max(2, (pz + ntz - 1) / ntz));
        }
      }
      for (int tz : tzs) {
        GatherShape s = shape_with_tile(h, tx, ty, std::min(std::max(tz, 1), pz));
        if (shape_stages(s) && !seen(s)) out.push_back(s);
      }
    }
  }
  return out;
}

int set_shape(fem_heat* h, const GatherShape& s) {
  if (!shape_stages(s)) return fail(h, FEM_EINVAL, "tile shape too thin for the staging scheme");
  if (s.nblocks > h->n_partials) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    const uint32_t n = s.nblocks;
    const size_t ncomp = (h->opts.flags & FEM_ONE_REDUCTION) ? 4 : 1;
    for (RelayCtx* c : {&h->outer, &h->inner})
      for (int k = 0; k < 2; ++k) {
        dfree(h, c->P[k]);
        RC_TRY(dalloc(h, &c->P[k], ncomp * n));
        HIP_TRY(hipMemsetAsync(c->P[k], 0, ncomp * n * sizeof(double), h->stream));
      }
    h->n_partials = n;
  }
  h->shape = s;
  h->stats.tile_x = s.tx;
  h->stats.tile_y = s.ty;
  h->stats.tile_z = s.tz;
  h->stats.grid_blocks = (int32_t)s.nblocks;
  return FEM_OK;
}

int make_handle(const fem_grid* grid, const double* k_e, const double* rhoc_e, const fem_bc* bc, const fem_opts& o,
                bool batched, fem_heat** out, std::string* why) {
  fem_heat* h = new (std::nothrow) fem_heat();
  if (!h) return FEM_ENOMEM;
  h->opts = o;
  h->devptrs = (o.flags & FEM_DEVICE_PTRS) != 0;
  h->timing = (o.flags & FEM_TIMING) != 0;
  h->device = o.device;
  h->batched = batched;
  const int rc = solver_init(h, grid, k_e, rhoc_e, bc);
  if (rc != FEM_OK) {
    if (why) *why = h->err;
    solver_free(h);
    delete h;
    return rc;
  }
  *out = h;
  return FEM_OK;
}

size_t handle_device_bytes(const fem_grid& grid, const fem_opts& opts, const fem_bc* bc, int32_t nsteps,
                           int32_t n_sensors) {
  const size_t N = (size_t)(grid.nx + 1) * (grid.ny + 1) * (grid.nz + 1);
  const size_t E = (size_t)grid.nx * grid.ny * grid.nz;
  bool lift = false;
  if (bc)
    for (int f = 0; f < 6; ++f)
      if (((bc->dirichlet_mask >> f) & 1u) && bc->dirichlet_value[f] != 0.0) lift = true;
  // FP64: coefficients; F, pinv, b, r, q, two directions, four fields (+ lift; + r, q ping-pong buffers of
  // the one-reduction form)
  const bool one_red = (opts.flags & FEM_ONE_REDUCTION) != 0;
  const bool mixed = opts.precision == FEM_FP32_FP64DOT;
  size_t bytes = 8 * (2 * E + (11 + (lift ? 1 : 0) + (one_red && !mixed ? 2 : 0)) * N);
  if (mixed) bytes += 4 * (2 * E + (8 + (one_red ? 2 : 0)) * N);  // FP32 set
  if (opts.precond == FEM_PRECOND_CHEBYSHEV && opts.precision == FEM_FP64) bytes += 8 * 4 * N;  // s, chain
  // relay state and partials (at most max(tiles, update blocks) per buffer) and the sink
  const size_t tiles_bound = N / 32 + 1024;
  bytes += 4 * (sizeof(Scalars) + 8 * tiles_bound * (one_red ? 4 : 1)) + 8 * kMaxBlockThreads;
  if (n_sensors > 0) bytes += 8 * (3 * (size_t)n_sensors + (size_t)std::max(nsteps, 1) * n_sensors);
  return bytes;
}

void solver_free(fem_heat* h) {
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  dfree(h, h->rhoc64);
  dfree(h, h->k64);
  dfree(h, h->rhoc32);
  dfree(h, h->k32);
  dfree(h, h->F64);
  dfree(h, h->pinv64);
  dfree(h, h->b64);
  dfree(h, h->r64);
  dfree(h, h->q64);
  dfree(h, h->r64b);
  dfree(h, h->q64b);
  for (auto& p : h->d64) dfree(h, p);
  for (auto& p : h->pool) dfree(h, p);
  dfree(h, h->lift64);
  dfree(h, h->sink);
  dfree(h, h->pinv32);
  for (auto& p : h->e32) dfree(h, p);
  dfree(h, h->r32);
  dfree(h, h->q32);
  dfree(h, h->r32b);
  dfree(h, h->q32b);
  for (auto& p : h->d32) dfree(h, p);
  dfree(h, h->rhs32);
  for (RelayCtx* c : {&h->outer, &h->inner})
    for (int k = 0; k < 2; ++k) {
      dfree(h, c->S[k]);
      dfree(h, c->P[k]);
    }
  dfree(h, h->s64);
  dfree(h, h->cr64);
  for (auto& p : h->cd64) dfree(h, p);
  dfree(h, h->xyz_dev);
  dfree(h, h->traces_dev);
  dfree(h, h->ebe_part);
  for (auto& e : h->ev_apply)
    if (e) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  h->stream = nullptr;
}

}  // namespace femheat
