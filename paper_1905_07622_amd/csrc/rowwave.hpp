// Node-centred operator apply y = (cm M + ck K) x with one wavefront per node
// row and no block barrier, kept beside the LDS-tiled gather for comparison.
//
// Wavefront w takes x-segment `seg` of node row (y, z) (rows x fastest, then
// y, then z).  Lane L holds node x = 62 seg - 1 + L; lanes 1..62 own theirs,
// lanes 0 and 63 are the x-halo.  Each lane loads the nine rows (y + dy,
// z + dz), dy, dz in {-1, 0, 1}, at its x (coalesced; rows and nodes outside
// the grid read as 0) and takes the x-neighbours from lanes L - 1 and L + 1 by
// shuffles; it loads the coefficients of the four elements (x, y - 1..y,
// z - 1..z) and takes those of the four elements at x - 1 from lane L - 1.
// For each of the 8 elements around its node (corner a of the element) it
// adds sum_b (rho_e cm M[a^b] + k_e ck K[a^b]) x_b, with the entry classes of
// the element block (c = a xor b, bit d set when the corners differ along
// axis d).  Nothing is staged in LDS and no wavefront waits for another.
// Blocks (4 wavefronts) take an XCD-aware order: block b runs on XCD b mod 8
// and takes block (b mod 8) * share + b / 8 of the row order, so each XCD
// works through a contiguous slab of rows and the nine-row neighbourhoods
// meet in its L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace femheat {

constexpr int kRowOwn = 62;  // nodes a wavefront owns

struct RowArgs {
  int32_t nx, ny, nz, px, py, pz;
  uint32_t nseg;   // x-segments per node row: ceil(px / 62)
  uint32_t nwave;  // nseg * py * pz
  uint32_t nblk;   // blocks of 4 wavefronts covering nwave
  uint32_t share;  // ceil(nblk / 8); the launch has 8 * share blocks
  const double* x;
  const double* rhoc;  // per element, dense (ex fastest)
  const double* kc;
  double* y;
  double Mc[8], Kc[8];  // cm M[c] and ck K[c] for entry class c
};

__global__ void __launch_bounds__(256) rowwave_apply_kernel(RowArgs a) {
  const uint32_t blk = (blockIdx.x & 7u) * a.share + (blockIdx.x >> 3);
  if (blk >= a.nblk) return;
  const uint32_t w = blk * 4u + (threadIdx.x >> 6);
  if (w >= a.nwave) return;  // whole wavefronts
  const int lane = (int)(threadIdx.x & 63u);
  const uint32_t seg = w % a.nseg;
  const uint32_t row = w / a.nseg;
  const int y = (int)(row % (uint32_t)a.py);
  const int z = (int)(row / (uint32_t)a.py);
  const int x = (int)seg * kRowOwn - 1 + lane;
  const bool xin = x >= 0 && x <= a.nx;
  const int xc = min(max(x, 0), a.nx);
  // the nine node rows, index (dy + 1) + 3 (dz + 1); x-1 and x+1 from the neighbouring lanes
  double D[9], Dl[9], Dr[9];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int ry = y + dy, rz = z + dz;
      const bool ok = xin && ry >= 0 && ry <= a.ny && rz >= 0 && rz <= a.nz;
      const uint32_t i = (uint32_t)xc + (uint32_t)a.px * ((uint32_t)min(max(ry, 0), a.ny) +
                                                          (uint32_t)a.py * (uint32_t)min(max(rz, 0), a.nz));
      const double v = a.x[i];
      D[(dy + 1) + 3 * (dz + 1)] = ok ? v : 0.0;
    }
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    Dl[r] = __shfl_up(D[r], 1u);
    Dr[r] = __shfl_down(D[r], 1u);
  }
  const bool eok_x = x >= 0 && x < a.nx;
  const int exc = min(max(x, 0), a.nx - 1);
  double q = 0.0;
#pragma unroll
  for (int oz = -1; oz <= 0; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 0; ++oy) {
      const int ey = y + oy, ez = z + oz;
      const bool eok = eok_x && ey >= 0 && ey < a.ny && ez >= 0 && ez < a.nz;
      const uint32_t e = (uint32_t)exc + (uint32_t)a.nx * ((uint32_t)min(max(ey, 0), a.ny - 1) +
                                                           (uint32_t)a.ny * (uint32_t)min(max(ez, 0), a.nz - 1));
      const double rc0 = a.rhoc[e], kk0 = a.kc[e];
      const double rc = eok ? rc0 : 0.0, kk = eok ? kk0 : 0.0;
      const double rcl = __shfl_up(rc, 1u), kkl = __shfl_up(kk, 1u);
#pragma unroll
      for (int ox = -1; ox <= 0; ++ox) {
        const double re = ox < 0 ? (lane > 0 ? rcl : 0.0) : rc;
        const double ke = ox < 0 ? (lane > 0 ? kkl : 0.0) : kk;
        const int corner = (-ox) + 2 * (-oy) + 4 * (-oz);  // this node's corner of the element
        double C[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) C[c] = fma(ke, a.Kc[c], re * a.Mc[c]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int sx = ox + (b & 1), sy = oy + ((b >> 1) & 1), sz = oz + (b >> 2);  // -1..1 from the node
          const int r = (sy + 1) + 3 * (sz + 1);
          const double dv = sx < 0 ? Dl[r] : (sx == 0 ? D[r] : Dr[r]);
          q = fma(C[corner ^ b], dv, q);
        }
      }
    }
  if (xin && lane >= 1 && lane <= kRowOwn)
    a.y[(uint32_t)x + (uint32_t)a.px * ((uint32_t)y + (uint32_t)a.py * (uint32_t)z)] = q;
}

}  // namespace femheat
