// Node-centred gather apply of the assembly-free operator (gfx950).
//
// For every node i the kernel evaluates
//     y_i = sum over the (up to 8) elements e around i of
//           sum_b (cm*rhoc_e*M_ref[a,b] + ck*k_e*K_ref[a,b]) * v_{node(e,b)}
// which is the DoF-by-DoF reading of the assembly operator (eq. EbEvsDbD,
// eq. DbD, Sec. 3.2 and 4.2.2): one thread owns one output node, so there is
// no second pass, no partial-sum buffer and no atomics.  With (cm, ck) =
// (1, theta*dt) it is A = M + theta*dt*K, with (1, -(1-theta)*dt) it is L.
//
// Entries of the 8x8 reference blocks of a trilinear hexahedron depend only
// on which axes separate the two corners (c = a xor b): M[c] is the product
// of the 1-D mass entries h/3 (same) or h/6 (differ), K[c] sums over the axes
// the 1-D stiffness entry +-1/h times the two 1-D mass entries.  For cubic
// elements they depend on popcount(c) only: M = h^3/216 {8,4,2,1},
// K = h/12 {4,0,-1,-1}.
//
// Memory schedule (the paper's Impl. 2 lost to uncoalesced strips; here every
// global access is a coalesced row segment): a block owns a TX x TY column
// tile and marches along z through TZ planes.  Each step stages one plane of
// the input vector with a one-node halo and one layer of element
// coefficients into double-buffered LDS, then every thread combines the
// 3x3 neighbourhood of the new plane (9 LDS reads) with the 4 elements of the
// layer (8 LDS reads) for the two nodes of its column that the layer touches.
// Plane quantities are kept in registers for the next layer.  Out-of-grid
// nodes are staged as 0 and out-of-grid elements carry zero coefficients, so
// boundaries need no branches in the arithmetic.
//
// A prologue functor produces the input value at every staged node (and
// writes it back for owned nodes: fused search-direction or x updates), an
// epilogue functor consumes the result at owned nodes (q, residual, RHS) and
// returns the node's contribution to a block dot product that is reduced on
// the device.
#pragma once

#include "common.hpp"
#include "reduce.hpp"

namespace femheat {

template <typename V>
struct GatherArgs {
  Geom g;
  GatherShape s;
  const V* rhoc;   // per-element rho*C
  const V* kc;     // per-element k
  V sa, sb;        // cubic: cm*h^3/216, ck*h/12 ; general: cm, ck
  V Mc[8], Kc[8];  // general elements: class entries M[c], K[c]
};

// 3x3 neighbourhood of one plane around a column: centre, x-/x+, y-/y+, and
// the four diagonal corners b[sy*2+sx] (s = 0: minus side, 1: plus side).
template <typename V>
struct PlaneQ {
  V c, xm, xp, ym, yp, b[4];
};

template <typename V>
__device__ inline void read_plane(const V* P, int pw, int lx, int ly, PlaneQ<V>& q) {
  const V* row0 = P + ly * pw + lx;  // (lx-1+1, ly-1+1) is the centre at row0[pw+1]
  q.b[0] = row0[0];
  q.ym = row0[1];
  q.b[1] = row0[2];
  q.xm = row0[pw];
  q.c = row0[pw + 1];
  q.xp = row0[pw + 2];
  q.b[2] = row0[2 * pw];
  q.yp = row0[2 * pw + 1];
  q.b[3] = row0[2 * pw + 2];
}

template <typename V, bool CUBIC, class Pro, class Epi>
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs<V> ga, Pro pro, Epi epi, Relay R) {
  Scalars st;
  if (!stage_entry(R, st)) return;  // uniform: the solve is done (or broke down)
  pro.init(st);
  epi.init(st);

  extern __shared__ unsigned char smem_raw[];
  const int TX = ga.s.tx, TY = ga.s.ty, TZ = ga.s.tz;
  const int PW = TX + 2, PH = TY + 2, CW = TX + 1, CH = TY + 1;
  V* plane = reinterpret_cast<V*>(smem_raw);  // [2][PH*PW]
  V* ca = plane + 2 * PW * PH;               // [2][CH*CW]
  V* cb = ca + 2 * CW * CH;                  // [2][CH*CW]

  const int px = ga.g.px, py = ga.g.py, pz = ga.g.pz;
  const int nx = ga.g.nx, ny = ga.g.ny, nz = ga.g.nz;

  // XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs,
  // so block b runs on XCD b%8.  Logical tile = (b%8)*share + b/8 gives every
  // XCD a contiguous range of tiles with z fastest, so the z-halo planes that
  // neighbouring chunks share are reused from the same L2.
  const uint32_t share = ga.s.nblocks >> 3;
  const uint32_t logical = (blockIdx.x & 7u) * share + (blockIdx.x >> 3);
  const bool idle = logical >= ga.s.ntiles;
  double dot = 0.0;

  if (!idle) {
    uint32_t b = logical;
    const int tz = (int)(b % (uint32_t)ga.s.ntz);
    b /= (uint32_t)ga.s.ntz;
    const int tyi = (int)(b % (uint32_t)ga.s.nty);
    const int txi = (int)(b / (uint32_t)ga.s.nty);
    const int x0 = txi * TX, y0 = tyi * TY, z0 = tz * TZ;
    const int z1 = min(z0 + TZ, pz);

    const int t = threadIdx.x;
    const int nthr = blockDim.x;
    const bool has_col = t < TX * TY;
    const int ltx = has_col ? t % TX : 0, lty = has_col ? t / TX : 0;
    const int gx = x0 + ltx, gy = y0 + lty;
    const bool col_ok = has_col && gx < px && gy < py;

    auto stage_plane = [&](int z, int buf) {
      V* P = plane + buf * PW * PH;
      const bool zin = z >= 0 && z < pz;
      const bool zown = z >= z0 && z < z1;
      for (int s = t; s < PW * PH; s += nthr) {
        const int ly = s / PW, lx = s - ly * PW;
        const int x = x0 - 1 + lx, y = y0 - 1 + ly;
        V v = V(0);
        if (zin && x >= 0 && x < px && y >= 0 && y < py) {
          const uint32_t i = (uint32_t)x + (uint32_t)px * ((uint32_t)y + (uint32_t)py * (uint32_t)z);
          const bool owned = zown && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
          v = pro.load(i, owned);
        }
        P[s] = v;
      }
    };
    auto stage_coef = [&](int l, int buf) {
      V* A = ca + buf * CW * CH;
      V* B = cb + buf * CW * CH;
      const bool lin = l >= 0 && l < nz;
      for (int s = t; s < CW * CH; s += nthr) {
        const int ly = s / CW, lx = s - ly * CW;
        const int ex = x0 - 1 + lx, ey = y0 - 1 + ly;
        V a = V(0), bb = V(0);
        if (lin && ex >= 0 && ex < nx && ey >= 0 && ey < ny) {
          const uint32_t e = (uint32_t)ex + (uint32_t)nx * ((uint32_t)ey + (uint32_t)ny * (uint32_t)l);
          a = ga.sa * ga.rhoc[e];
          bb = ga.sb * ga.kc[e];
        }
        A[s] = a;
        B[s] = bb;
      }
    };

    PlaneQ<V> lo, hi;
    stage_plane(z0 - 1, 0);
    __syncthreads();
    read_plane(plane, PW, ltx, lty, lo);
    V acc_lo = V(0);
    int buf = 1;
    for (int l = z0 - 1; l < z1; ++l) {
      stage_plane(l + 1, buf);
      stage_coef(l, buf);
      __syncthreads();
      read_plane(plane + buf * PW * PH, PW, ltx, lty, hi);
      const V* A = ca + buf * CW * CH;
      const V* B = cb + buf * CW * CH;
      V acc_hi = V(0);
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          const int ci = (lty + sy) * CW + ltx + sx;
          const V a = A[ci], bk = B[ci];
          const V xl = sx ? lo.xp : lo.xm, yl = sy ? lo.yp : lo.ym, bl = lo.b[sy * 2 + sx];
          const V xh = sx ? hi.xp : hi.xm, yh = sy ? hi.yp : hi.ym, bh = hi.b[sy * 2 + sx];
          if (CUBIC) {
            // classes by popcount: c0 = 8a+4b, c1 = 4a, c2 = 2a-b, c3 = a-b
            const V c0 = V(8) * a + V(4) * bk, c1 = V(4) * a, c2 = V(2) * a - bk, c3 = a - bk;
            const V al = xl + yl, ah = xh + yh;
            acc_lo += c0 * lo.c + c1 * (al + hi.c) + c2 * (bl + ah) + c3 * bh;
            acc_hi += c0 * hi.c + c1 * (ah + lo.c) + c2 * (bh + al) + c3 * bl;
          } else {
            V k[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) k[c] = a * ga.Mc[c] + bk * ga.Kc[c];
            acc_lo += k[0] * lo.c + k[1] * xl + k[2] * yl + k[3] * bl + k[4] * hi.c + k[5] * xh + k[6] * yh + k[7] * bh;
            acc_hi += k[0] * hi.c + k[1] * xh + k[2] * yh + k[3] * bh + k[4] * lo.c + k[5] * xl + k[6] * yl + k[7] * bl;
          }
        }
      }
      if (l >= z0 && col_ok) {
        const uint32_t i = (uint32_t)gx + (uint32_t)px * ((uint32_t)gy + (uint32_t)py * (uint32_t)l);
        dot += epi.store(i, acc_lo, lo.c);
      }
      acc_lo = acc_hi;
      lo = hi;
      buf ^= 1;
    }
  }
  if (R.pout) publish_partial(R, dot);
}

// ---------------------------------------------------------------------------
// prologues: value of the gathered vector at node i (and write-back when owned)
// ---------------------------------------------------------------------------

template <typename V>
struct ProPlain {  // v = src
  const V* src;
  __device__ void init(const Scalars&) {}
  __device__ V load(uint32_t i, bool) const { return src[i]; }
};

template <typename V>
struct ProDirection {  // d_new = P^-1 r + beta d_old   (Algorithm 1: s <- P^-1 r, d <- s + beta d)
  const V* r;
  const V* pinv;
  const V* dold;
  V* dnew;
  V beta;
  __device__ void init(const Scalars& S) { beta = (V)S.beta; }
  __device__ V load(uint32_t i, bool owned) const {
    const V v = pinv[i] * r[i] + beta * dold[i];
    if (owned) dnew[i] = v;
    return v;
  }
};

template <typename V, typename W>
struct ProAxpy {  // x_new = x + alpha d  (alpha from the solve's scalars, or 1 for a correction)
  const V* x;
  const W* d;
  V* xnew;
  int32_t unit_alpha;
  V alpha;
  __device__ void init(const Scalars& S) { alpha = unit_alpha ? V(1) : (V)S.alpha; }
  __device__ V load(uint32_t i, bool owned) const {
    const V v = x[i] + alpha * (V)d[i];
    if (owned) xnew[i] = v;
    return v;
  }
};

template <typename V>
struct ProGuess {  // x0 = 2 T1 - T2 (u0_update, App. A.2) or T1; 0 on free nodes for a zero RHS
  const V* t1;
  const V* t2;
  const V* pinv;
  V* x;
  int32_t prev;
  int32_t zero;
  __device__ void init(const Scalars& S) { zero = S.zero_rhs; }
  __device__ V load(uint32_t i, bool owned) const {
    V v = prev ? t1[i] : V(2) * t1[i] - t2[i];
    if (zero) v = (pinv[i] == V(0)) ? t1[i] : V(0);
    if (owned) x[i] = v;
    return v;
  }
};

// ---------------------------------------------------------------------------
// epilogues: consume y_i at an owned node, return the dot-product contribution
// ---------------------------------------------------------------------------

template <typename V>
struct EpiStore {  // y = A v
  V* y;
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V) const {
    y[i] = acc;
    return 0.0;
  }
};

template <typename V>
struct EpiQDot {  // q = A d ; contribution d_i q_i to d^T q
  V* q;
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V v) const {
    q[i] = acc;
    return (double)v * (double)acc;
  }
};

template <typename V>
struct EpiResidual {  // r = b - A x (0 on Dirichlet rows); contribution r_i P^-1_i r_i
  const V* b;
  const V* pinv;
  V* r;
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V) const {
    const V p = pinv[i];
    const V rr = (p == V(0)) ? V(0) : b[i] - acc;
    r[i] = rr;
    return (double)rr * (double)(p * rr);
  }
};

template <typename V>
struct EpiRhs {  // b = L T + dt*s*F ; contribution (b - lift)_i P^-1_i (b - lift)_i over free rows
  V* b;
  const V* F;
  const V* pinv;
  const V* lift;  // A_fD g for non-zero Dirichlet values, or nullptr
  V fs;           // dt * s_n
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V) const {
    const V bb = acc + fs * F[i];
    b[i] = bb;
    const V bh = lift ? bb - lift[i] : bb;
    return (double)bh * (double)(pinv[i] * bh);
  }
};

}  // namespace femheat
