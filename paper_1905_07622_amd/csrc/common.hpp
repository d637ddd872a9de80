// Definitions shared by the gfx950 kernels and the host runtime of the
// assembly-free theta-scheme heat solver (arXiv:1905.07622).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace femheat {

// Grid description used by every kernel.  Node i = ix + px*(iy + py*iz),
// element e = ex + nx*(ey + ny*ez) (x fastest, the paper's fixed grid, Sec. 4.1).
struct Geom {
  int32_t nx, ny, nz;  // elements per axis
  int32_t px, py, pz;  // nodes per axis (n + 1)
  uint32_t N, E;
  double hx, hy, hz;
  uint32_t dir_mask;   // Dirichlet faces (bit f: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z)
  double dir_val[6];
  uint32_t flux_mask;
  double flux[6];
  int32_t tet6;        // 1: every box is six linear tetrahedra (cubes only), else a trilinear hexahedron
};

// State of one PCG solve (Algorithm 1), all scalars in FP64, relayed from
// kernel to kernel on the device.
struct Scalars {
  double delta;      // r^T P^-1 r of the current residual (delta_new)
  double delta_old;
  double delta0;     // value at the start of the solve
  double delta_b;    // b^T P^-1 b over free rows (stopping reference)
  double tol;        // loop continues while delta > tol
  double dq;         // d^T q
  double alpha;
  double beta;
  double mu, nu;     // one-reduction form: q^T P^-1 r and q^T P^-1 q of the last direction
  int32_t iter;      // completed iterations of the current solve
  int32_t done;      // 1: every further iteration kernel is a no-op
  int32_t status;    // 0 or a negative status (breakdown)
  int32_t zero_rhs;  // b^T P^-1 b == 0 with the RHS stop rule
  int32_t phase;     // which scalar update the latest partials complete
  int32_t fresh;     // one-reduction form: the last direction kernel also advanced r
};

// Controls of one solve.
struct Ctl {
  double rtol2;      // squared relative tolerance
  int32_t max_iter;
  int32_t stop_rule; // 0: relative to b^T P^-1 b, 1: relative to the initial residual
};

enum Phase : int32_t {
  PH_NONE = 0,
  PH_AFTER_INIT = 1,   // partials hold r0^T P^-1 r0
  PH_AFTER_UPD = 2,    // partials hold r^T P^-1 r after an update
  PH_AFTER_CHECK = 3,  // partials hold the FP64 residual norm of a refinement sweep
  PH_DECIDED = 4,
  PH_AFTER_FUSED = 5   // partials hold d^T q, q^T P^-1 r, q^T P^-1 q, r^T P^-1 r (one-reduction form)
};

// Role of a kernel in the relay.
enum Mode : int32_t {
  M_NONE = 0,    // no solve state (test hooks, setup)
  M_RHS = 1,     // right-hand side of a new step
  M_INIT = 2,    // initial guess and residual (reads b^T P^-1 b)
  M_START = 3,   // initial residual of an inner solve
  M_DIR = 4,     // settles delta/beta/stop, then direction + apply
  M_UPD = 5,     // settles alpha, then x/r update (or replacement)
  M_CORR = 6,    // FP64 correction of a refinement sweep
  M_DECIDE = 7,  // settles the pending decision only
  M_SKIP = 8,    // relays the state unchanged and does no work
  M_IDLE = 9,    // an inner solve that is not needed: starts done, zero iterations
  // one-reduction form: settle the pending update, then
  M_FDIR = 10,   //   direction + apply with the residual as it is (after the initial residual or a replacement)
  M_FUPD = 11,   //   r -= alpha q, x += alpha d, then direction + apply
  M_FREPL = 12,  //   residual replacement x += alpha d, r = b - A x
  // the next step's right-hand side and initial residual, launched before the
  // host knows whether the current solve has finished: they run only if it has
  M_RHS_NEXT = 13,   // as M_RHS if the solve ended well with the iterate buffer predicted
  M_INIT_NEXT = 14,  // as M_INIT if the M_RHS_NEXT before it ran
  // a kernel of the preconditioner chain (Chebyshev): relays the state
  // unchanged, leaves the pending update for the kernel after the chain
  // (whose partials, from the chain's last kernel, complete it); idle once done
  M_PASS = 15
};

constexpr int32_t kStatusBreakdown = -4;

// Highest degree of the Chebyshev preconditioner (m - 1 gathers per application).
constexpr int kChebMaxDegree = 8;

// Threads of a gather block: up to 512 for a simulation alone (one block of
// eight waves per CU holds a whole x-row of a 101-node grid in 101 x 5
// tiles: every wave of the CU then marches in step with the others, where
// two blocks of four waves drift apart, the older one issuing first), up to
// 256 for batch members (two or more per CU).
constexpr int kMaxBlockThreads = 512;
constexpr int kMaxBatchThreads = 256;

// Launch shape of the gather apply: a block owns a TX x TY column tile of
// nodes and marches TZ planes in z.
struct GatherShape {
  int32_t tx, ty, tz;
  int32_t ntx, nty, ntz;
  int32_t nthreads;   // TX*TY rounded up to a multiple of 64
  int32_t pw, cw;     // LDS row pitches of the plane tile (>= TX+2) and coefficient tile (>= TX+1)
  uint32_t ntiles;    // ntx*nty*ntz
  uint32_t nblocks;   // ntiles rounded up to a multiple of 8 (one share per XCD)
  // LDS of a gather: `planes` double-buffered node planes and two
  // double-buffered coefficient tiles.
  size_t smem_bytes(size_t vbytes, int planes = 1) const {
    return vbytes * (2 * (size_t)planes * pw * (ty + 2) + 4 * (size_t)cw * (ty + 1));
  }
};

}  // namespace femheat
