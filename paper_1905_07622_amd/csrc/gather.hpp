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
// nodes are staged from clamped addresses and out-of-grid elements carry zero
// coefficients, so boundaries need no branches in the arithmetic.
//
// Neighbouring z-chunks march in opposite directions, so they read the halo
// planes they share at the same time, from the same L2.
//
// A prologue functor produces the input value at every staged node (and
// writes it back for owned nodes: fused search-direction or x updates, the
// deferred x += alpha d of the previous iteration, or the advanced residual
// of the one-reduction form), an epilogue functor consumes the result at
// owned nodes (q, residual, RHS) and returns the node's contribution to a
// block dot product that is reduced on the device.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "gmem.hpp"
#include "reduce.hpp"

namespace femheat {

// Element kinds of the gather (template argument KIND): a trilinear
// hexahedron on a general box (8 class entries), on a cube (4 popcount
// classes), or a cube split into six linear tetrahedra (the paper's element).
constexpr int kElemBox = 0, kElemCubic = 1, kElemTet6 = 2;

// Box matrices of the six-tetrahedron split of a cube of side h (tetrahedra
// 0, e_i, e_i + e_j, 7 for each order of the axes: the split around the 0-7
// diagonal, conforming across boxes).  From the linear tetrahedron's closed
// forms M_t = V/20 (1 + delta_ij) and K_t = V grad l_i . grad l_j with
// V = h^3/6: M = h^3/120 * kTetM and K = h/6 * kTetK (corner a = ax + 2ay + 4az).
// Pairs joined by no tetrahedron edge are 0, and K reduces to the 7-point
// Laplacian stencil once assembled.
constexpr int kTetM[8][8] = {{12, 2, 2, 2, 2, 2, 2, 6}, {2, 4, 0, 1, 0, 1, 0, 2}, {2, 0, 4, 1, 0, 0, 1, 2},
                             {2, 1, 1, 4, 0, 0, 0, 2}, {2, 0, 0, 0, 4, 1, 1, 2}, {2, 1, 0, 0, 1, 4, 0, 2},
                             {2, 0, 1, 0, 1, 0, 4, 2}, {6, 2, 2, 2, 2, 2, 2, 12}};
constexpr int kTetK[8][8] = {{6, -2, -2, 0, -2, 0, 0, 0}, {-2, 4, 0, -1, 0, -1, 0, 0}, {-2, 0, 4, -1, 0, 0, -1, 0},
                             {0, -1, -1, 4, 0, 0, 0, -2}, {-2, 0, 0, 0, 4, -1, -1, 0}, {0, -1, 0, 0, -1, 4, 0, -2},
                             {0, 0, -1, 0, -1, 0, 4, -2}, {0, 0, 0, -2, 0, -2, -2, 6}};

template <typename V>
struct GatherArgs {
  Geom g;
  GatherShape s;
  const V* rhoc;   // per-element rho*C
  const V* kc;     // per-element k
  V sa, sb;        // cubic: cm*h^3/216, ck*h/12 ; tetrahedra: cm*h^3/120, ck*h/6 ; general: cm, ck
  V Mc[8], Kc[8];  // general elements: class entries M[c], K[c]
  V* sink;         // >= kMaxBlockThreads scratch values: stores of lanes without a node land here
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

// Staging slots: thread t stages LDS entries t and t + nthreads of a plane
// tile (and of a coefficient tile); the launch guarantees both tiles fit.
constexpr int kSlots = 2;

// Layers between issuing a plane's global loads and staging it in LDS: 2
// keeps two register sets of loads in flight, 1 one set (fewer registers).
#ifndef FEMHEAT_GATHER_DEPTH
#define FEMHEAT_GATHER_DEPTH 2
#endif
constexpr int kDepth = FEMHEAT_GATHER_DEPTH;

// XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs,
// so block b runs on XCD b%8.  Work item (b%8)*share + b/8 gives every XCD a
// contiguous range of tiles (z fastest, then x, then y), so the halo planes,
// columns and rows that neighbouring tiles share are mostly reused from the
// same L2.  `nblocks` is a multiple of 8.
__device__ inline uint32_t xcd_work_item(uint32_t b, uint32_t nblocks) {
  return (b & 7u) * (nblocks >> 3) + (b >> 3);
}

// A prologue that also owns the iterate: it applies the previous iteration's
// deferred x += alpha d at the block's own nodes (see ProDirection).
template <class P>
struct CarriesIterate {
  static constexpr bool value = false;
};

// A prologue of the one-reduction form: it also advances the residual and
// stages it (and P^-1) for the node's own dot products.
template <class P>
struct AdvancesResidual {
  static constexpr bool value = false;
};

// An epilogue that reads per-node inputs (b, P^-1, F, ...) declares them as
// its Raw and loads them in fetch(i); the march requests them at the start of
// the layer that completes the own node, before that layer issues the next
// planes' loads, and hands the values to store() (or keep()).  (Loads issued
// after the planes' and used in the same layer would make the wave wait for
// every load before them, the prefetched planes included.)
template <class E, class = void>
struct EpiFetches {
  static constexpr bool value = false;
};
template <class E>
struct EpiFetches<E, std::void_t<typename E::Raw>> {
  static constexpr bool value = true;
};
struct NoRaw {};
template <class E, bool = EpiFetches<E>::value>
struct EpiRawOf {
  using type = NoRaw;
};
template <class E>
struct EpiRawOf<E, true> {
  using type = typename E::Raw;
};

// An epilogue that keeps the result at the block's own nodes on chip (in
// LDS, for a later phase of the same kernel) instead of storing it: it has
// keep(zl, acc, v, live, raw), zl the node's plane within the block's
// z-chunk, raw what its fetch(i) read at the node (see EpiFetches).
template <class E, class = void>
struct EpiKeeps {
  static constexpr bool value = false;
};
template <class E>
struct EpiKeeps<E, std::void_t<decltype(E::kKeeps)>> {
  static constexpr bool value = E::kKeeps;
};

// What a gather leaves for a later phase of the same kernel (out-parameter
// of gather_tile): the state it evaluated (valid when `settled`) and, when
// the relay has no partial buffer, the thread's share of the dot product.
struct TileOut {
  Scalars st;
  double dot;
  bool settled;
};

// One block's share of a gather: tile `logical` of the solve that `ga`, the
// functors and the relay describe.  The block's dot-product partial is
// stored at index `logical`, and tile 0 publishes the relayed state.
// kD: prefetch depth in layers.  The FP64 one-reduction direction kernel stages a fourth vector and
// keeps four accumulators; with one layer of prefetch it fits 164 VGPRs instead of 256 with a spill
// (in FP32 two layers fit in 169).
template <typename V, int KIND, class Pro, class Epi, bool kFour = AdvancesResidual<Pro>::value,
          int kD = (AdvancesResidual<Pro>::value && sizeof(V) == 8 ? 1 : kDepth)>
__device__ inline void gather_tile(const GatherArgs<V>& ga, Pro pro, Epi epi, const Relay& R, uint32_t logical,
                                   TileOut* out = nullptr) {
  const StageIn in = stage_load<sizeof(V) == 8>(R);
  if (out) {
    out->st = in.t;
    out->dot = 0.0;
    out->settled = false;
  }
  if (stage_idle(R, in, logical == 0)) return;  // uniform: a finished solve
  Scalars st;

  extern __shared__ unsigned char smem_raw[];
  const int TX = ga.s.tx, TY = ga.s.ty, TZ = ga.s.tz;
  const int NW = TX + 2, PH = TY + 2, NC = TX + 1, CH = TY + 1;  // tile widths (nodes, elements)
  const int PW = ga.s.pw, CW = ga.s.cw;                          // LDS row pitches (bank-conflict padding)
  // Coefficient tiles: the scaled rho*c and k of each element of a layer.
  // (Staging the four cubic class coefficients instead saves arithmetic but
  // doubles these tiles, and measured slower.)
  const int CS = CW * CH;
  V* plane = reinterpret_cast<V*>(smem_raw);  // [2][PH*PW]
  V* coef = plane + 2 * PW * PH;             // [2][2][CH*CW]: rho*c, k
  constexpr bool FU = AdvancesResidual<Pro>::value;
  V* rpl = coef + 4 * CS;    // one-reduction form: [2][PH*PW] advanced residual
  V* ppl = rpl + 2 * PW * PH;  //                    [2][PH*PW] P^-1

  const int px = ga.g.px, py = ga.g.py, pz = ga.g.pz;
  const int nx = ga.g.nx, ny = ga.g.ny, nz = ga.g.nz;
  const uint32_t pstride = (uint32_t)px * (uint32_t)py, lstride = (uint32_t)nx * (uint32_t)ny;

  if (logical >= ga.s.ntiles) {  // a padding block: partial 0 (never the writer)
    const bool go = stage_finish<kFour>(R, in, st, false);
    if (out) {
      out->st = st;
      out->settled = true;
    }
    if (go && R.pout) {
      if constexpr (AdvancesResidual<Pro>::value) {
        const double z[4] = {0.0, 0.0, 0.0, 0.0};
        publish_partial4(R, z, logical);
      } else {
        publish_partial(R, 0.0, logical);
      }
    }
    return;
  }
  double dot = 0.0;
  double dots[4] = {0.0, 0.0, 0.0, 0.0};  // one-reduction form: d^T q, q^T P^-1 r, q^T P^-1 q, r^T P^-1 r
  {
    // tile order: z-chunk fastest, then x, then y -- the tiles that split a
    // row in x are neighbours in the order and so share an XCD (and its L2),
    // which serves the cache lines and halo columns they both read
    uint32_t b = logical;
    const int tz = (int)(b % (uint32_t)ga.s.ntz);
    b /= (uint32_t)ga.s.ntz;
    const int txi = (int)(b % (uint32_t)ga.s.ntx);
    const int tyi = (int)(b / (uint32_t)ga.s.ntx);
    const int x0 = txi * TX, y0 = tyi * TY, z0 = tz * TZ;
    const int z1 = min(z0 + TZ, pz);

    const int t = threadIdx.x;
    const int nthr = blockDim.x;
    const bool has_col = t < TX * TY;
    const int ltx = has_col ? t % TX : 0, lty = has_col ? t / TX : 0;
    const int gx = x0 + ltx, gy = y0 + lty;
    const bool col_ok = has_col && gx < px && gy < py;

    // Per-slot staging coordinates, fixed for the whole z march.  Node
    // addresses are clamped into the grid: a value staged outside the grid
    // only ever meets elements outside the grid, whose coefficients are 0, so
    // any finite value is exact there.  Element coefficients outside the grid
    // are stored as 0 explicitly.  Unused slots load a valid dummy address.
    // Every global load and store of the z march is unconditional, so the
    // compiler can count outstanding memory operations exactly and the loads
    // issued two layers ahead stay in flight while the current layer computes.
    int pl[kSlots], cl[kSlots];
    uint32_t pxy[kSlots], cxy[kSlots];
    bool cin[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      const int idx = t + k * nthr;
      const int ly = idx / NW, lx = idx - ly * NW;
      const bool pv = idx < NW * PH;
      pl[k] = pv ? ly * PW + lx : -1;
      const int x = x0 - 1 + lx, y = y0 - 1 + ly;
      pxy[k] = pv ? (uint32_t)min(max(x, 0), px - 1) + (uint32_t)px * (uint32_t)min(max(y, 0), py - 1) : 0u;
      const int ey_ = idx / NC, ex_ = idx - ey_ * NC;
      const bool cv = idx < NC * CH;
      cl[k] = cv ? ey_ * CW + ex_ : -1;
      const int ex = x0 - 1 + ex_, ey = y0 - 1 + ey_;
      cin[k] = cv && ex >= 0 && ex < nx && ey >= 0 && ey < ny;
      cxy[k] = cv ? (uint32_t)min(max(ex, 0), nx - 1) + (uint32_t)nx * (uint32_t)min(max(ey, 0), ny - 1) : 0u;
    }
    const uint32_t col_xy = col_ok ? (uint32_t)gx + (uint32_t)px * (uint32_t)gy : 0u;

    // Two register sets hold the planes l+1 and l+2 (and coefficient layers
    // l and l+1) while layer l computes.
    constexpr bool XI = CarriesIterate<Pro>::value;
    constexpr bool EF = EpiFetches<Epi>::value;
    struct Stage {
      typename Pro::Raw p[kSlots];
      V a[kSlots], b[kSlots];
      V xo, dold;  // iterate and old direction at this column's node emitted with this stage
    };
    auto fetch = [&](Stage& S, int z, int l, int zown) {  // plane z, coefficient layer l, own node zown (clamped)
      const uint32_t zo = pstride * (uint32_t)min(max(z, 0), pz - 1);
      const uint32_t lo_ = lstride * (uint32_t)min(max(l, 0), nz - 1);
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        S.p[k] = pro.fetch(pxy[k] + zo);
        S.a[k] = gld(ga.rhoc, cxy[k] + lo_);
        S.b[k] = gld(ga.kc, cxy[k] + lo_);
      }
      if constexpr (XI) {
        const uint32_t io = col_xy + pstride * (uint32_t)min(max(zown, 0), pz - 1);
        S.xo = gld(pro.x, io);
        S.dold = gld(pro.dold, io);
      }
    };
    auto store = [&](const Stage& S, int l, int buf) {  // LDS only
      V* P = plane + buf * PW * PH;
      V* C = coef + buf * 2 * CS;
      const bool lin = l >= 0 && l < nz;
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        if constexpr (FU) {
          if (pl[k] >= 0) {
            const V rn = pro.residual(S.p[k]);
            P[pl[k]] = pro.direction(S.p[k], rn);
            rpl[buf * PW * PH + pl[k]] = rn;
            ppl[buf * PW * PH + pl[k]] = S.p[k].p;
          }
        } else {
          if (pl[k] >= 0) P[pl[k]] = pro.finish(S.p[k]);
        }
        if (cl[k] >= 0) {
          const bool ok = lin && cin[k];
          const V a = ok ? ga.sa * S.a[k] : V(0), bk = ok ? ga.sb * S.b[k] : V(0);
          C[cl[k]] = a;
          C[CS + cl[k]] = bk;
        }
      }
    };

    // The march visits planes vis(0..n) and the n layers between consecutive
    // ones; node vis(k) is owned for 1 <= k <= n-1.  Odd z-chunks march
    // down, even ones up, so two neighbouring chunks read the planes and the
    // coefficient layer they share at the same end of their marches, while
    // both are in the same L2 (with one direction, one chunk reads them first
    // and its neighbour a whole march later, from memory again).
    const bool down = (tz & 1) != 0;
    const int n = z1 - z0 + 1;
    auto vis = [&](int k) { return down ? z1 - k : z0 - 1 + k; };
    auto lay = [&](int k) { return down ? z1 - 1 - k : z0 - 1 + k; };  // layer between vis(k) and vis(k+1)

    PlaneQ<V> lo, hi;
    V carry = V(0);
    V rn_lo = V(0), pp_lo = V(0), rn_hi = V(0), pp_hi = V(0);  // one-reduction form: own node's r, P^-1
    // Contributions of one layer's 4 elements to the two nodes of this
    // column that the layer joins: `lo` on plane `lp` (other plane `hp`) and
    // `hi` on `hp`.  A node's value is the sum of the contributions of its two
    // layers, each computed here from zero (explicit FMAs in a fixed order;
    // the library is built without automatic contraction) -- so it does not
    // depend on the tiling or on the direction of the march.  Each element's
    // coefficients serve both nodes and are then dead.
    auto contributions = [&](const PlaneQ<V>& lp, const PlaneQ<V>& hp, const V* C, V& lo_sum, V& hi_sum) {
      V plo[4], phi[4];
      // the tetrahedra are not symmetric under z-reflection: their corners
      // are taken on the physical bottom and top planes of the layer (which
      // are hp and lp when the chunk marches down)
      PlaneQ<V> bot, top;
      if constexpr (KIND == kElemTet6) {
        bot = down ? hp : lp;
        top = down ? lp : hp;
      }
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          const int e = sy * 2 + sx;
          const int ci = (lty + sy) * CW + ltx + sx;
          const V xl = sx ? lp.xp : lp.xm, yl = sy ? lp.yp : lp.ym, bl = lp.b[e];
          const V xh = sx ? hp.xp : hp.xm, yh = sy ? hp.yp : hp.ym, bh = hp.b[e];
          if constexpr (KIND == kElemTet6) {
            // rows of the bottom node (corner ax + 2ay) and the top node (+4)
            // of this element against its 8 corner values, zero entries skipped
            const V a = C[ci], bk = C[CS + ci];
            const int ax = 1 - sx, ay = 1 - sy;
            V val[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
              const PlaneQ<V>& P = (b >> 2) ? top : bot;
              const bool dx = (b & 1) != ax, dy = ((b >> 1) & 1) != ay;
              val[b] = dx ? (dy ? P.b[e] : (sx ? P.xp : P.xm)) : (dy ? (sy ? P.yp : P.ym) : P.c);
            }
            V rows[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
              const int arow = ax + 2 * ay + 4 * r;
              V acc = V(0);
#pragma unroll
              for (int b = 0; b < 8; ++b) {
                const int m = kTetM[arow][b], kk = kTetK[arow][b];
                if (m == 0 && kk == 0) continue;
                const V c = m == 0 ? bk * V(kk) : (kk == 0 ? a * V(m) : fma(a, V(m), bk * V(kk)));
                acc = fma(c, val[b], acc);
              }
              rows[r] = acc;
            }
            plo[e] = down ? rows[1] : rows[0];
            phi[e] = down ? rows[0] : rows[1];
          } else if constexpr (KIND == kElemCubic) {
            // classes by popcount: c0 = 8a+4b, c1 = 4a, c2 = 2a-b, c3 = a-b
            const V a = C[ci], bk = C[CS + ci];
            const V c0 = fma(V(8), a, V(4) * bk), c1 = V(4) * a, c2 = fma(V(2), a, -bk), c3 = a - bk;
            V u = c0 * lp.c;
            u = fma(c1, (xl + yl) + hp.c, u);
            u = fma(c2, bl + (xh + yh), u);
            plo[e] = fma(c3, bh, u);
            V w = c0 * hp.c;
            w = fma(c1, (xh + yh) + lp.c, w);
            w = fma(c2, bh + (xl + yl), w);
            phi[e] = fma(c3, bl, w);
          } else {
            const V a = C[ci], bk = C[CS + ci];
            const V vl[8] = {lp.c, xl, yl, bl, hp.c, xh, yh, bh};  // corner differing by class c
            const V vh[8] = {hp.c, xh, yh, bh, lp.c, xl, yl, bl};
            V c = fma(a, ga.Mc[0], bk * ga.Kc[0]);
            V u = c * vl[0], w = c * vh[0];
#pragma unroll
            for (int k = 1; k < 8; ++k) {
              c = fma(a, ga.Mc[k], bk * ga.Kc[k]);
              u = fma(c, vl[k], u);
              w = fma(c, vh[k], w);
            }
            plo[e] = u;
            phi[e] = w;
          }
        }
      }
      lo_sum = (plo[0] + plo[1]) + (plo[2] + plo[3]);
      hi_sum = (phi[0] + phi[1]) + (phi[2] + phi[3]);
    };
    // Layer k: completes node vis(k) (its other layer was layer k-1) and
    // starts node vis(k+1).  Loads for plane vis(k+3) and layer k+2 are issued
    // here (clamped to the march: past its end they re-read the last ones).
    auto layer = [&](int k, int buf, Stage& S, auto emit) {
      store(S, lay(k), buf);
      if constexpr (XI) {
        // The deferred x += alpha d_old at node vis(k), whose x and d_old came
        // with this stage: stored before the stage's registers take the next
        // loads, so no value of a load still in flight has to be kept (a copy
        // of it would make the wave wait for that load).
        if (decltype(emit)::value && pro.corr) {
          const uint32_t i = col_xy + pstride * (uint32_t)vis(k);
          const V xn = fma(pro.alpha, S.dold, S.xo);
          gst_at(col_ok ? pro.x + i : ga.sink + threadIdx.x, xn);
        }
      }
      // The epilogue's inputs at node vis(k) are requested before the next
      // planes, so the wait for them at the end of the layer leaves those
      // planes in flight.  (Carried over from an earlier layer in registers,
      // they would cross the loop's back edge as copies of loads still in
      // flight, which wait for every load.)
      typename EpiRawOf<Epi>::type eo{};
      if constexpr (EF)
        if (decltype(emit)::value) eo = epi.fetch(col_xy + pstride * (uint32_t)vis(k));
      __syncthreads();
      fetch(S, vis(min(k + 1 + kD, n)), lay(min(k + kD, n - 1)), vis(min(k + kD, n)));
      read_plane(plane + buf * PW * PH, PW, ltx, lty, hi);
      if constexpr (FU) {  // the new plane's centre: this column's node vis(k+1)
        const int c = (lty + 1) * PW + ltx + 1;
        rn_hi = rpl[buf * PW * PH + c];
        pp_hi = ppl[buf * PW * PH + c];
      }
      V p_lo, p_hi;
      contributions(lo, hi, coef + buf * 2 * CS, p_lo, p_hi);
      if (decltype(emit)::value) {  // node vis(k) is owned by this block
        const uint32_t i = col_xy + pstride * (uint32_t)vis(k);
        pro.write(i, lo.c, col_ok, ga.sink);
        if constexpr (FU) {
          if (pro.corr) gst_at(col_ok ? pro.rnew + i : ga.sink + threadIdx.x, rn_lo);
          const V qv = carry + p_lo;
          gst_at(col_ok ? epi.q + i : ga.sink + threadIdx.x, qv);
          if (col_ok) {
            dots[0] += (double)lo.c * (double)qv;
            dots[1] += (double)qv * (double)(pp_lo * rn_lo);
            dots[2] += (double)qv * (double)(pp_lo * qv);
            dots[3] += (double)rn_lo * (double)(pp_lo * rn_lo);
          }
        } else if constexpr (EpiKeeps<Epi>::value) {
          dot += epi.keep(vis(k) - z0, carry + p_lo, lo.c, col_ok, eo);
        } else if constexpr (EF) {
          dot += epi.store(i, carry + p_lo, lo.c, col_ok, ga.sink, eo);
        } else {
          dot += epi.store(i, carry + p_lo, lo.c, col_ok, ga.sink);
        }
      }
      carry = p_hi;
      lo = hi;
      if constexpr (FU) {
        rn_lo = rn_hi;
        pp_lo = pp_hi;
      }
    };

    // Prologue: the first three planes and the first two coefficient layers
    // are requested at once, before the relayed partial sum, so that sum and
    // the fill of the plane pipeline overlap.  (Issuing them before the
    // relayed state is read as well measured slower.)
    Stage SA, SB;
    {
      Stage S0;
      fetch(S0, vis(0), lay(0), vis(0));
      fetch(SB, vis(1), lay(0), vis(0));
      if constexpr (kD == 2) fetch(SA, vis(min(2, n)), lay(min(1, n - 1)), vis(1));
      const bool go = stage_finish<kFour>(R, in, st, logical == 0);
      if (out) {
        out->st = st;
        out->settled = true;
      }
      if (!go) {  // uniform
        if constexpr (XI) {
          // the solve finished in this kernel's evaluation: the last
          // iteration's deferred iterate update is still due at own nodes
          if (R.mode == M_DIR && in.pending && st.status == 0 && pro.corr && col_ok) {
            const V al = (V)st.alpha;
            for (int z = z0; z < z1; ++z) {
              const uint32_t i = col_xy + pstride * (uint32_t)z;
              const V xn = fma(al, gld(pro.dold, i), gld(pro.x, i));
              gst(pro.x, i, xn);
            }
          }
        }
        return;
      }
      pro.init(st);
      epi.init(st);
      store(S0, -1, 0);  // plane vis(0) into buffer 0 (its coefficient slots are rewritten before use)
    }
    __syncthreads();
    read_plane(plane, PW, ltx, lty, lo);
    if constexpr (FU) {
      const int c = (lty + 1) * PW + ltx + 1;
      rn_lo = rpl[c];
      pp_lo = ppl[c];
    }
    using no = std::integral_constant<bool, false>;
    using yes = std::integral_constant<bool, true>;
    layer(0, 1, SB, no{});  // node vis(0) belongs to the neighbouring chunk
    if constexpr (kD == 2) {
      int k = 1;
      for (; k + 1 < n; k += 2) {  // two register sets alternate: indices stay compile-time
        layer(k, 0, SA, yes{});
        layer(k + 1, 1, SB, yes{});
      }
      if (k < n) layer(k, 0, SA, yes{});
    } else {
      for (int k = 1; k < n; ++k) layer(k, (k + 1) & 1, SB, yes{});
    }
  }
  if constexpr (FU) {
    if (R.pout) publish_partial4(R, dots, logical);
  } else {
    if (R.pout) publish_partial(R, dot, logical);
    if (out) out->dot = dot;
  }
}

// A gather of one solve: one block per tile (grid = ga.s.nblocks).
template <typename V, int KIND, class Pro, class Epi>
__global__ void __launch_bounds__(kMaxBlockThreads) gather_kernel(GatherArgs<V> ga, Pro pro, Epi epi, Relay R) {
  gather_tile<V, KIND>(ga, pro, epi, R, xcd_work_item(blockIdx.x, ga.s.nblocks));
}

// ---------------------------------------------------------------------------
// prologues: value of the gathered vector at node i (and write-back when owned)
// ---------------------------------------------------------------------------

// A prologue has fetch(i) -> Raw (the global loads of one node, issued two
// layers early), finish(raw) -> value (pure arithmetic, also for halo nodes)
// and write(i, v, live, sink): the write-back of the value at an owned node
// (lanes without a node store to the sink instead of branching).

template <typename V>
struct ProPlain {  // v = src
  const V* src;
  struct Raw {
    V a;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(src, i)}; }
  __device__ V finish(const Raw& w) const { return w.a; }
  __device__ void write(uint32_t, V, bool, V*) const {}
};

// The iterate update x += alpha d of Algorithm 1 is deferred to the next
// iteration's direction gather, which reads d_old anyway: at its own nodes it
// applies x += alpha_prev d_old when `corr` is set (the previous iteration
// ended with a plain update, not a residual replacement, which updates x
// itself).  The x/r update kernel then streams r, q and P^-1 only.
template <typename V>
struct ProDirection {  // d_new = P^-1 r + beta d_old   (Algorithm 1: s <- P^-1 r, d <- s + beta d)
  const V* r;
  const V* pinv;
  const V* dold;
  V* dnew;
  V* x;          // iterate, updated in place at own nodes
  int32_t corr;  // apply the deferred x += alpha d_old
  V beta;
  V alpha;
  struct Raw {
    V r, p, d;
  };
  __device__ void init(const Scalars& S) {
    beta = (V)S.beta;
    alpha = (V)S.alpha;
  }
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(r, i), gld(pinv, i), gld(dold, i)}; }
  __device__ V finish(const Raw& w) const { return fma(beta, w.d, w.p * w.r); }
  __device__ void write(uint32_t i, V v, bool live, V* sink) const { gst_at(live ? dnew + i : sink + threadIdx.x, v); }
};

// Only the FP64 direction kernel carries the iterate: in the FP32 inner
// solves of the mixed form the update kernel keeps x += alpha d (moving those
// bytes into the gather measured slower there, in batches above all).
template <>
struct CarriesIterate<ProDirection<double>> {
  static constexpr bool value = true;
};

// One-reduction form of an iteration (one kernel, one set of partial sums):
// when `corr` is set the kernel first completes the previous iteration's
// update, r -= alpha q (0 on Dirichlet rows, as in the update kernel) and
// x += alpha d_old (own nodes), then forms d = P^-1 r + beta d_old and
// q = A d.  Its partials are d^T q, q^T P^-1 r, q^T P^-1 q and r^T P^-1 r of
// the advanced r (see PH_AFTER_FUSED).  The residual ping-pongs (the halo of
// a tile reads r values that another tile advances).
template <typename V>
struct ProFused {
  const V* r;     // residual this kernel starts from
  const V* qold;  // q of the previous iteration (read always; used when corr)
  const V* pinv;
  const V* dold;
  V* dnew;
  V* x;           // iterate, updated in place at own nodes
  V* rnew;        // advanced residual, written at own nodes when corr
  int32_t corr;
  V beta;
  V alpha;
  struct Raw {
    V r, q, p, d;
  };
  __device__ void init(const Scalars& S) {
    beta = (V)S.beta;
    alpha = (V)S.alpha;
  }
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(r, i), gld(qold, i), gld(pinv, i), gld(dold, i)}; }
  __device__ V residual(const Raw& w) const {
    if (!corr) return w.r;
    const V rr = fma(-alpha, w.q, w.r);
    return (w.p == V(0)) ? V(0) : rr;
  }
  __device__ V direction(const Raw& w, V rn) const { return fma(beta, w.d, w.p * rn); }
  __device__ V finish(const Raw& w) const { return direction(w, residual(w)); }
  __device__ void write(uint32_t i, V v, bool live, V* sink) const { gst_at(live ? dnew + i : sink + threadIdx.x, v); }
};

template <typename V>
struct CarriesIterate<ProFused<V>> {
  static constexpr bool value = true;
};

template <typename V>
struct AdvancesResidual<ProFused<V>> {
  static constexpr bool value = true;
};

// Search direction from a preconditioned residual held as a vector (the
// Chebyshev preconditioner): d_new = s + beta d_old, with the deferred
// x += alpha d_old at own nodes as in ProDirection.
template <typename V>
struct ProDirectionS {
  const V* s;
  const V* dold;
  V* dnew;
  V* x;
  int32_t corr;
  V beta;
  V alpha;
  struct Raw {
    V s, d;
  };
  __device__ void init(const Scalars& S) {
    beta = (V)S.beta;
    alpha = (V)S.alpha;
  }
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(s, i), gld(dold, i)}; }
  __device__ V finish(const Raw& w) const { return fma(beta, w.d, w.s); }
  __device__ void write(uint32_t i, V v, bool live, V* sink) const { gst_at(live ? dnew + i : sink + threadIdx.x, v); }
};

template <>
struct CarriesIterate<ProDirectionS<double>> {
  static constexpr bool value = true;
};

// First step of the Chebyshev preconditioner applied to r_in (minus the
// Dirichlet lifting when given): the gathered vector is d_0 = P^-1 (r_in -
// lift) / c, c the centre of the interval.
template <typename V>
struct ProChebStart {
  const V* r;
  const V* lift;  // or nullptr
  const V* pinv;
  V inv_c;
  struct Raw {
    V r, l, p;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(r, i), lift ? gld(lift, i) : V(0), gld(pinv, i)}; }
  __device__ V finish(const Raw& w) const { return (w.p * (w.r - w.l)) * inv_c; }
  __device__ void write(uint32_t, V, bool, V*) const {}
};

// Step k of the Chebyshev preconditioner, at own nodes, after the gather
// formed (A d_{k-1})_i: res_k = res_{k-1} - A d_{k-1}, z = P^-1 res_k,
// d_k = a_k d_{k-1} + b_k z, y_{k+1} = y_k + d_k (y_1 = d_0).  The last step
// writes only y (= s, the preconditioned vector) and returns the node's
// contribution r_in_i s_i; the others carry res, d and y to the next step.
template <typename V>
struct EpiCheb {
  const V* rprev;  // res_{k-1}: r_in (k = 1) or the chain's residual
  const V* lift;   // k = 1 with a lifted right-hand side, or nullptr
  const V* pinv;
  const V* yprev;  // y_k, or nullptr for k = 1 (y_1 = d_0, the gathered value)
  const V* rin;    // the chain's input (for the last step's dot product)
  const V* rlift;  // its lifting, or nullptr
  V* rnext;        // res_k (not on the last step)
  V* dnext;        // d_k (not on the last step)
  V* y;            // y_{k+1}
  V a, b;
  int32_t last;
  struct Raw {  // loaded values only: the arithmetic waits for them in store()
    V rp, l, p, y, ri, rl;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const {
    Raw w;
    w.rp = gld(rprev, i);
    w.l = lift ? gld(lift, i) : V(0);
    w.p = gld(pinv, i);
    w.y = yprev ? gld(yprev, i) : V(0);
    w.ri = last ? gld(rin, i) : V(0);
    w.rl = (last && rlift) ? gld(rlift, i) : V(0);
    return w;
  }
  __device__ double store(uint32_t i, V acc, V v, bool live, V* sink, const Raw& w) const {
    const V rp = lift ? w.rp - w.l : w.rp;
    const V rk = rp - acc;
    const V dk = fma(a, v, b * (w.p * rk));
    const V yk = (yprev ? w.y : v) + dk;
    gst_at(live ? y + i : sink + threadIdx.x, yk);
    if (last) {
      const V ri = rlift ? w.ri - w.rl : w.ri;
      return live ? (double)ri * (double)yk : 0.0;
    }
    gst_at(live ? rnext + i : sink + threadIdx.x, rk);
    gst_at(live ? dnext + i : sink + threadIdx.x, dk);
    return 0.0;
  }
};

template <typename V, typename W>
struct ProAxpy {  // x_new = x + alpha d  (alpha from the solve's scalars, or 1 for a correction)
  const V* x;
  const W* d;
  V* xnew;
  int32_t unit_alpha;
  V alpha;
  struct Raw {
    V x;
    W d;
  };
  __device__ void init(const Scalars& S) { alpha = unit_alpha ? V(1) : (V)S.alpha; }
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(x, i), gld(d, i)}; }
  __device__ V finish(const Raw& w) const { return fma(alpha, (V)w.d, w.x); }
  __device__ void write(uint32_t i, V v, bool live, V* sink) const { gst_at(live ? xnew + i : sink + threadIdx.x, v); }
};

template <typename V>
struct ProGuess {  // x0 = 2 T1 - T2 (u0_update, App. A.2) or T1; 0 on free nodes for a zero RHS
  const V* t1;
  const V* t2;
  const V* pinv;
  V* x;
  int32_t prev;
  int32_t zero;
  struct Raw {
    V a, b, p;
  };
  __device__ void init(const Scalars& S) { zero = S.zero_rhs; }
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(t1, i), gld(t2, i), gld(pinv, i)}; }
  __device__ V finish(const Raw& w) const {
    V v = prev ? w.a : fma(V(2), w.a, -w.b);
    if (zero) v = (w.p == V(0)) ? w.a : V(0);
    return v;
  }
  __device__ void write(uint32_t i, V v, bool live, V* sink) const { gst_at(live ? x + i : sink + threadIdx.x, v); }
};

// ---------------------------------------------------------------------------
// epilogues: consume y_i at an owned node, return the dot-product contribution
// ---------------------------------------------------------------------------

// An epilogue consumes y_i at an owned node and returns the node's dot
// contribution; lanes without a node (live = false) store to the sink.

template <typename V>
struct EpiStore {  // y = A v
  V* y;
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V, bool live, V* sink) const {
    gst_at(live ? y + i : sink + threadIdx.x, acc);
    return 0.0;
  }
};

template <typename V>
struct EpiQDot {  // q = A d ; contribution d_i q_i to d^T q
  V* q;
  __device__ void init(const Scalars&) {}
  __device__ double store(uint32_t i, V acc, V v, bool live, V* sink) const {
    gst_at(live ? q + i : sink + threadIdx.x, acc);
    return live ? (double)v * (double)acc : 0.0;
  }
};

template <typename V>
struct EpiQ {  // q = A d (one-reduction form: the kernel forms its four dot products itself)
  V* q;
  __device__ void init(const Scalars&) {}
};

template <typename V>
struct EpiResidual {  // r = b - A x (0 on Dirichlet rows); contribution r_i P^-1_i r_i
  const V* b;
  const V* pinv;
  V* r;
  struct Raw {
    V b, p;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(b, i), gld(pinv, i)}; }
  __device__ double store(uint32_t i, V acc, V, bool live, V* sink, const Raw& w) const {
    const V rr = (w.p == V(0)) ? V(0) : w.b - acc;
    gst_at(live ? r + i : sink + threadIdx.x, rr);
    return live ? (double)rr * (double)(w.p * rr) : 0.0;
  }
};

template <typename V>
struct EpiRhs {  // b = L T + dt*s*F ; contribution (b - lift)_i P^-1_i (b - lift)_i over free rows
  V* b;
  const V* F;
  const V* pinv;
  const V* lift;  // A_fD g for non-zero Dirichlet values, or nullptr
  V fs;           // dt * s_n
  struct Raw {
    V F, p, l;
  };
  __device__ void init(const Scalars&) {}
  __device__ Raw fetch(uint32_t i) const { return Raw{gld(F, i), gld(pinv, i), lift ? gld(lift, i) : V(0)}; }
  __device__ double store(uint32_t i, V acc, V, bool live, V* sink, const Raw& w) const {
    const V bb = fma(fs, w.F, acc);
    gst_at(live ? b + i : sink + threadIdx.x, bb);
    const V bh = lift ? bb - w.l : bb;
    return live ? (double)bh * (double)(w.p * bh) : 0.0;
  }
};

}  // namespace femheat
