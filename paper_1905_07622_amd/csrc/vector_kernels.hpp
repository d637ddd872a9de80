// Pointwise kernels of the solver (gfx950): the fused PCG residual update of
// Algorithm 1 (AXPY + DIMVM + VVM + Beta_update of App. A.2 in one pass),
// the setup kernels (Jacobi diagonal, boundary load vector, Dirichlet
// values), precision casts for the mixed form and sensor interpolation.
#pragma once

#include "common.hpp"
#include "gather.hpp"
#include "reduce.hpp"

namespace femheat {

template <typename V>
struct Vec;
template <>
struct Vec<double> {
  using T = double2;
  static constexpr int W = 2;
};
template <>
struct Vec<float> {
  using T = float4;
  static constexpr int W = 4;
};

// r -= alpha q (0 on Dirichlet rows) ; delta_new = r^T P^-1 r.  Dirichlet
// rows are recognised by P^-1 = 0.  (In the FP64 solve x += alpha d is
// deferred to the next direction gather.)
template <typename V>
__device__ inline void upd1(V& r, V q, V p, V alpha, double& acc) {
  V rr = fma(-alpha, q, r);
  rr = (p == V(0)) ? V(0) : rr;
  r = rr;
  acc += (double)rr * (double)(p * rr);
}

// Residual update of one solve by block `blk` of its `nblk` blocks (a
// grid-stride loop over the solve's own block count, so the partial sums do
// not depend on the launch the block belongs to).  Each thread loads kU
// strided vectors before it uses any, and the first kU before it settles
// alpha = delta / d^T q, so the partial sum runs while they are in flight.
// With kEarly (a launch for one simulation) those loads are issued even
// before the relayed state is read; otherwise the state comes first, so a
// finished solve loads nothing (in a lockstep batch most members are often
// finished).  When x and d are given (FP32 inner solves) the kernel also
// applies x += alpha d.  Vectors in flight per thread (kU): 4 in FP64, whose
// 1M-DOF launch is one round of blocks; 2 in FP32 for one simulation; 1 in
// FP32 batches, which run many rounds and need the occupancy of a small
// register count instead.
template <typename V, bool kEarly = false, int kU = (sizeof(V) == 8 ? 4 : 1)>
__device__ inline void update_body(V* __restrict__ r, const V* __restrict__ q, const V* __restrict__ pinv, uint32_t N,
                                   const Relay& R, uint32_t blk, uint32_t nblk, V* __restrict__ x = nullptr,
                                   const V* __restrict__ d = nullptr) {
  StageIn in;
  if constexpr (!kEarly) {
    in = stage_load<sizeof(V) == 8>(R);
    if (stage_idle(R, in, blk == 0)) return;
  }
  using VT = typename Vec<V>::T;
  constexpr int W = Vec<V>::W;
  const uint32_t nvec = N / W;
  const uint32_t stride = nblk * blockDim.x;
  const uint32_t tid = blk * blockDim.x + threadIdx.x;
  VT* rv = reinterpret_cast<VT*>(r);
  const VT* qv = reinterpret_cast<const VT*>(q);
  const VT* pv = reinterpret_cast<const VT*>(pinv);
  const bool withx = x != nullptr;  // uniform
  VT* xv = reinterpret_cast<VT*>(x);
  const VT* dv = reinterpret_cast<const VT*>(d);
  VT rr[kU], qq[kU], pp[kU], xx[kU], dd[kU];
  auto load = [&](uint32_t base) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = base + (uint32_t)u * stride;
      if (j < nvec) {
        rr[u] = gld(rv, j);
        qq[u] = gld(qv, j);
        pp[u] = gld(pv, j);
        if (withx) {
          xx[u] = gld(xv, j);
          dd[u] = gld(dv, j);
        }
      }
    }
  };
  load(tid);
  if constexpr (kEarly) {
    in = stage_load<sizeof(V) == 8>(R);
    if (stage_idle(R, in, blk == 0)) return;
  }
  Scalars st;
  if (!stage_finish(R, in, st, blk == 0)) return;
  const V alpha = (V)st.alpha;
  double acc = 0.0;
  for (uint32_t base = tid; base < nvec; base += kU * stride) {
    if (base != tid) load(base);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = base + (uint32_t)u * stride;
      if (j < nvec) {
        if constexpr (W == 2) {
          upd1(rr[u].x, qq[u].x, pp[u].x, alpha, acc);
          upd1(rr[u].y, qq[u].y, pp[u].y, alpha, acc);
        } else {
          upd1(rr[u].x, qq[u].x, pp[u].x, alpha, acc);
          upd1(rr[u].y, qq[u].y, pp[u].y, alpha, acc);
          upd1(rr[u].z, qq[u].z, pp[u].z, alpha, acc);
          upd1(rr[u].w, qq[u].w, pp[u].w, alpha, acc);
        }
        gst(rv, j, rr[u]);
        if (withx) {
          if constexpr (W == 2) {
            xx[u].x = fma(alpha, dd[u].x, xx[u].x);
            xx[u].y = fma(alpha, dd[u].y, xx[u].y);
          } else {
            xx[u].x = fma(alpha, dd[u].x, xx[u].x);
            xx[u].y = fma(alpha, dd[u].y, xx[u].y);
            xx[u].z = fma(alpha, dd[u].z, xx[u].z);
            xx[u].w = fma(alpha, dd[u].w, xx[u].w);
          }
          gst(xv, j, xx[u]);
        }
      }
    }
  }
  for (uint32_t i = nvec * W + tid; i < N; i += stride) {
    V rs = gld(r, i);
    upd1(rs, gld(q, i), gld(pinv, i), alpha, acc);
    gst(r, i, rs);
    if (withx) gst(x, i, fma(alpha, gld(d, i), gld(x, i)));
  }
  publish_partial(R, acc, blk);
}

// x += alpha d over a solve's nodes, by block `blk` of `nblk` (the deferred
// iterate update of a solve that finished in a decide kernel).
template <typename V>
__device__ inline void axpy_body(V* __restrict__ x, const V* __restrict__ d, V alpha, uint32_t N, uint32_t blk,
                                 uint32_t nblk) {
  const uint32_t stride = nblk * blockDim.x;
  for (uint32_t i = blk * blockDim.x + threadIdx.x; i < N; i += stride) gst(x, i, fma(alpha, gld(d, i), gld(x, i)));
}

// Start of an inner (FP32) solve of A e = r64 by block `blk` of `nblk`:
// rhs = r = (float) r64, e = 0, r0^T P^-1 r0 accumulated in FP64.  A solve
// relayed as M_IDLE is not needed and does nothing.
__device__ inline void inner_start_body(const double* __restrict__ r64, float* __restrict__ rhs,
                                        float* __restrict__ r, float* __restrict__ e,
                                        const float* __restrict__ pinv, uint32_t N, const Relay& R, uint32_t blk,
                                        uint32_t nblk) {
  Scalars st;
  if (!stage_entry(R, st, blk == 0)) return;
  double acc = 0.0;
  const uint32_t stride = nblk * blockDim.x;
  for (uint32_t i = blk * blockDim.x + threadIdx.x; i < N; i += stride) {
    const float v = (float)gld(r64, i);
    gst(rhs, i, v);
    gst(r, i, v);
    gst(e, i, 0.0f);
    acc += (double)v * (double)(gld(pinv, i) * v);
  }
  publish_partial(R, acc, blk);
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

__device__ inline void node_xyz(const Geom& g, uint32_t i, int& ix, int& iy, int& iz) {
  ix = (int)(i % (uint32_t)g.px);
  const uint32_t t = i / (uint32_t)g.px;
  iy = (int)(t % (uint32_t)g.py);
  iz = (int)(t / (uint32_t)g.py);
}

// Dirichlet test: the lowest-numbered Dirichlet face containing the node decides.
__device__ inline bool dirichlet_value(const Geom& g, int ix, int iy, int iz, double& val) {
  const bool on[6] = {ix == 0, ix == g.nx, iy == 0, iy == g.ny, iz == 0, iz == g.nz};
#pragma unroll
  for (int f = 0; f < 6; ++f)
    if (((g.dir_mask >> f) & 1u) && on[f]) {
      val = g.dir_val[f];
      return true;
    }
  return false;
}

// Jacobi preconditioner P = diag(A), A = M + ck*K (Sec. 3.3, Jacobi_A of App. A.2),
// summed over the elements around each node: every diagonal entry of the
// trilinear element blocks is M_aa = V/27 and K_aa = (V/9)(1/hx^2+1/hy^2+1/hz^2).
// Stored as P^-1, 0 on Dirichlet nodes.
template <typename V>
__global__ void jacobi_kernel(Geom g, const double* __restrict__ rhoc, const double* __restrict__ kc, double ck,
                              V* __restrict__ pinv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int ix, iy, iz;
  node_xyz(g, i, ix, iy, iz);
  double gv;
  if (dirichlet_value(g, ix, iy, iz, gv)) {
    pinv[i] = V(0);
    return;
  }
  const double vol = g.hx * g.hy * g.hz;
  const double md = vol / 27.0;
  const double kd = vol / 9.0 * (1.0 / (g.hx * g.hx) + 1.0 / (g.hy * g.hy) + 1.0 / (g.hz * g.hz));
  double P = 0.0;
  for (int oz = 0; oz < 2; ++oz)
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        const int ex = ix - 1 + ox, ey = iy - 1 + oy, ez = iz - 1 + oz;
        if (ex < 0 || ex >= g.nx || ey < 0 || ey >= g.ny || ez < 0 || ez >= g.nz) continue;
        const uint32_t e = (uint32_t)ex + (uint32_t)g.nx * ((uint32_t)ey + (uint32_t)g.ny * (uint32_t)ez);
        if (g.tet6) {  // the node is corner a of this box; the tetrahedra's diagonal entries differ by corner
          const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
          P += rhoc[e] * (g.hx * g.hx * g.hx / 120.0 * kTetM[a][a]) + ck * kc[e] * (g.hx / 6.0 * kTetK[a][a]);
        } else {
          P += rhoc[e] * md + ck * kc[e] * kd;
        }
      }
  pinv[i] = (V)(1.0 / P);
}

// Boundary load F_i = sum over flux faces f containing i of q_f * integral of
// the bilinear face shape function = q_f * (h_u h_v / 4) * (face elements at i).
[[maybe_unused]] static __global__ void load_vector_kernel(Geom g, double* __restrict__ F) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int idx[3];
  node_xyz(g, i, idx[0], idx[1], idx[2]);
  const int n[3] = {g.nx, g.ny, g.nz};
  const double h[3] = {g.hx, g.hy, g.hz};
  double f = 0.0;
  for (int face = 0; face < 6; ++face) {
    if (!((g.flux_mask >> face) & 1u)) continue;
    const int d = face >> 1;
    if (idx[d] != ((face & 1) ? n[d] : 0)) continue;
    const int u = (d + 1) % 3, v = (d + 2) % 3;
    if (g.tet6) {
      // the face's triangles split every face square along its (0,0)-(1,1)
      // diagonal: a node at that diagonal of a square gets q hu hv / 3 from
      // it (two triangles), at the other diagonal q hu hv / 6 (one)
      double w = 0.0;
      for (int su = idx[u] - 1; su <= idx[u]; ++su)
        for (int sv = idx[v] - 1; sv <= idx[v]; ++sv) {
          if (su < 0 || su >= n[u] || sv < 0 || sv >= n[v]) continue;
          w += ((idx[u] - su) == (idx[v] - sv)) ? 1.0 / 3.0 : 1.0 / 6.0;
        }
      f += g.flux[face] * h[u] * h[v] * w;
      continue;
    }
    const int cu = (idx[u] > 0) + (idx[u] < n[u]);
    const int cv = (idx[v] > 0) + (idx[v] < n[v]);
    f += g.flux[face] * 0.25 * h[u] * h[v] * (double)(cu * cv);
  }
  F[i] = f;
}

// Overwrite Dirichlet nodes of T with their boundary value.
template <typename V>
__global__ void apply_dirichlet_kernel(Geom g, V* __restrict__ T) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int ix, iy, iz;
  node_xyz(g, i, ix, iy, iz);
  double gv;
  if (dirichlet_value(g, ix, iy, iz, gv)) T[i] = (V)gv;
}

// g_ext: boundary value on Dirichlet nodes, 0 elsewhere.
[[maybe_unused]] static __global__ void dirichlet_field_kernel(Geom g, double* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int ix, iy, iz;
  node_xyz(g, i, ix, iy, iz);
  double gv = 0.0;
  out[i] = dirichlet_value(g, ix, iy, iz, gv) ? gv : 0.0;
}

// lift_i = (A g_ext)_i on free rows, 0 on Dirichlet rows (computed in place on y).
[[maybe_unused]] static __global__ void mask_free_kernel(const double* __restrict__ pinv, double* __restrict__ y, uint32_t N) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && pinv[i] == 0.0) y[i] = 0.0;
}

template <typename A, typename B>
__global__ void cast_kernel(const A* __restrict__ in, B* __restrict__ out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (B)in[i];
}

template <typename V>
__global__ void fill_kernel(V* __restrict__ out, V v, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}

template <typename V>
__global__ void scale_kernel(const V* __restrict__ a, const V* __restrict__ x, double* __restrict__ y, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)(a[i] * (V)x[i]);
}

// Field value at points: trilinear interpolation in the containing element
// (lowest-index element on shared faces).  Traces row-major [step][sensor].
[[maybe_unused]] static __global__ void sensor_kernel(Geom g, const double* __restrict__ T, const double* __restrict__ xyz, int32_t S,
                              double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int n[3] = {g.nx, g.ny, g.nz};
  const double h[3] = {g.hx, g.hy, g.hz};
  int e[3];
  double xi[3];
  for (int d = 0; d < 3; ++d) {
    const double t = xyz[3 * s + d] / h[d];
    int k = (int)ceil(t) - 1;
    k = k < 0 ? 0 : (k > n[d] - 1 ? n[d] - 1 : k);
    double loc = t - (double)k;
    loc = loc < 0.0 ? 0.0 : (loc > 1.0 ? 1.0 : loc);
    e[d] = k;
    xi[d] = loc;
  }
  double v = 0.0;
  if (g.tet6) {
    // the tetrahedron 0, e_p, e_p + e_q, 7 with xi_p >= xi_q >= xi_r contains
    // the point; barycentrics 1 - xi_p, xi_p - xi_q, xi_q - xi_r, xi_r
    int o[3] = {0, 1, 2};
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2 - i; ++j)
        if (xi[o[j]] < xi[o[j + 1]]) {
          const int t = o[j];
          o[j] = o[j + 1];
          o[j + 1] = t;
        }
    const double lam[4] = {1.0 - xi[o[0]], xi[o[0]] - xi[o[1]], xi[o[1]] - xi[o[2]], xi[o[2]]};
    int a = 0;
    for (int k = 0; k < 4; ++k) {
      if (k > 0) a |= 1 << o[k - 1];
      const uint32_t i = (uint32_t)(e[0] + (a & 1)) +
                         (uint32_t)g.px * ((uint32_t)(e[1] + ((a >> 1) & 1)) + (uint32_t)g.py * (uint32_t)(e[2] + (a >> 2)));
      v += lam[k] * T[i];
    }
    out[s] = v;
    return;
  }
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const double w = (ax ? xi[0] : 1.0 - xi[0]) * (ay ? xi[1] : 1.0 - xi[1]) * (az ? xi[2] : 1.0 - xi[2]);
    const uint32_t i = (uint32_t)(e[0] + ax) + (uint32_t)g.px * ((uint32_t)(e[1] + ay) + (uint32_t)g.py * (uint32_t)(e[2] + az));
    v += w * T[i];
  }
  out[s] = v;
}

}  // namespace femheat
