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
};

// Device-resident scalars of one PCG solve (Algorithm 1), all in FP64.
struct Scalars {
  double delta;      // r^T P^-1 r of the current residual (delta_new)
  double delta_old;
  double delta0;     // value at the start of the solve
  double delta_b;    // b^T P^-1 b over free rows (stopping reference)
  double tol;        // loop continues while delta > tol
  double dq;         // d^T q
  double alpha;
  double beta;
  double aux;        // scratch for test hooks
  int32_t iter;      // completed iterations of the current solve
  int32_t done;      // 1: every further iteration kernel is a no-op
  int32_t status;    // 0 or a negative status (breakdown)
  int32_t zero_rhs;  // b^T P^-1 b == 0 with the RHS stop rule
  uint32_t ticket;   // arrival counter of the last-block reduction
  int32_t pad[3];
};

// Controls of one solve.
struct Ctl {
  double rtol2;      // squared relative tolerance
  int32_t max_iter;
  int32_t stop_rule; // 0: relative to b^T P^-1 b, 1: relative to the initial residual
};

enum Finalize : int32_t {
  FIN_NONE = 0,
  FIN_RHS = 1,    // delta_b = sum
  FIN_INIT = 2,   // delta = delta0 = sum; tol; done test before the first iteration
  FIN_ALPHA = 3,  // dq = sum; alpha = delta / dq (breakdown test)
  FIN_DELTA = 4,  // delta_old = delta; delta = sum; beta; iter++; done test
  FIN_CHECK = 5,  // delta = sum; done test (outer refinement check)
  FIN_STORE = 6   // aux = sum
};

constexpr int32_t kStatusBreakdown = -4;

// Launch shape of the gather apply: a block owns a TX x TY column tile of
// nodes and marches TZ planes in z.
struct GatherShape {
  int32_t tx, ty, tz;
  int32_t ntx, nty, ntz;
  int32_t nthreads;   // TX*TY rounded up to a multiple of 64
  uint32_t ntiles;    // ntx*nty*ntz
  uint32_t nblocks;   // ntiles rounded up to a multiple of 8 (one share per XCD)
  size_t smem_bytes(size_t vbytes) const {
    return vbytes * (2 * (size_t)(tx + 2) * (ty + 2) + 4 * (size_t)(tx + 1) * (ty + 1));
  }
};

}  // namespace femheat
