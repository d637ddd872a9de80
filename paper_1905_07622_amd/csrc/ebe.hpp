// Element-by-element operator apply in two passes, y = (cm M + ck K) x, kept
// beside the node-centred gather for comparison.  It follows the structure of
// the paper's coalesced element-by-element method (Section 4.3, third
// implementation: a work group loads the four node rows along the x-edges of a
// row of elements with coalesced reads, integrates every element of that row,
// sums what it can locally and leaves the rest to a second pass), on 8-node
// hexahedra and 64-wide wavefronts instead of tetrahedra and 32-wide warps.
//
// Pass 1: one wavefront per (x-segment, ey, ez).  Lane L holds node
// x = 62 seg + L of the four node rows (ey + dy, ez + dz), dy, dz in {0, 1};
// lanes 0..62 integrate element x (when x < nx): its 8 x 8 block from the
// entry classes (c = a xor b, bit d set when corners a and b differ along
// axis d) times its 8 corner values, the +x corners taken from lane L + 1.
// A node's two x-neighbouring elements are summed through a lane shuffle, and
// lanes 1..62 (lane 0 too in the first segment) store the four node rows into
// partial buffer s = dy + 2 dz (the row's place in the element row).
// Pass 2: y_i is the sum of the partials of the up to four element rows
// around node row (y, z), in the fixed order s = 0..3.
// Memory moved per apply (FP64): pass 1 reads x four times (each node row
// belongs to four element rows) and the two coefficient arrays, and writes
// 4 N partials; pass 2 reads them and writes y: (13 N + 2 E) * 8 bytes,
// against (2 N + 2 E) * 8 for the gather.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace femheat {

constexpr int kEbeStore = 62;  // nodes of a node row one segment stores

struct EbeArgs {
  int32_t nx, ny, nz, px, py;
  uint32_t N;
  uint32_t nseg;        // x-segments per element row: ceil(nx / 62)
  const double* x;
  const double* rhoc;   // per element, dense (ex fastest)
  const double* kc;
  double* part;         // 4 N partial sums, part[s N + i]
  double Mc[8], Kc[8];  // cm M[c] and ck K[c] for entry class c
};

__global__ void __launch_bounds__(256) ebe_elements_kernel(EbeArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= a.nseg * (uint32_t)a.ny * (uint32_t)a.nz) return;  // whole wavefronts
  const uint32_t seg = w % a.nseg;
  const uint32_t row = w / a.nseg;
  const int ey = (int)(row % (uint32_t)a.ny);
  const int ez = (int)(row / (uint32_t)a.ny);
  const int x = (int)(seg * kEbeStore + lane);
  const bool node_ok = x <= a.nx;
  const bool elem_ok = lane < 63u && x < a.nx;
  const int xc = min(x, a.nx);  // loads stay inside the node array
  double d[4];                  // node rows r = dy + 2 dz
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t i = (uint32_t)xc + (uint32_t)a.px * ((uint32_t)(ey + (r & 1)) + (uint32_t)a.py * (uint32_t)(ez + (r >> 1)));
    d[r] = a.x[i];
  }
  double rc = 0.0, kk = 0.0;
  if (elem_ok) {
    const uint32_t e = (uint32_t)x + (uint32_t)a.nx * ((uint32_t)ey + (uint32_t)a.ny * (uint32_t)ez);
    rc = a.rhoc[e];
    kk = a.kc[e];
  }
  // corner b = bx + 2 by + 4 bz lies in node row r = by + 2 bz, at this lane
  // (bx = 0) or the next one (bx = 1)
  double u[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    u[2 * r] = d[r];
    u[2 * r + 1] = __shfl_down(d[r], 1u);
  }
  double C[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) C[c] = fma(kk, a.Kc[c], rc * a.Mc[c]);
  double v[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    double s = C[p] * u[0];
#pragma unroll
    for (int b = 1; b < 8; ++b) s = fma(C[p ^ b], u[b], s);
    v[p] = elem_ok ? s : 0.0;
  }
  const bool store = node_ok && ((lane >= 1u && lane <= (uint32_t)kEbeStore) || (lane == 0u && seg == 0u));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    // this element's -x corner of row r, plus the +x corner of the element
    // on the left (lane L - 1; none left of node 0)
    const double left = __shfl_up(v[2 * r + 1], 1u);
    const double sum = lane > 0u ? v[2 * r] + left : v[2 * r];
    if (store) {
      const uint32_t i = (uint32_t)x + (uint32_t)a.px * ((uint32_t)(ey + (r & 1)) + (uint32_t)a.py * (uint32_t)(ez + (r >> 1)));
      a.part[(size_t)r * a.N + i] = sum;
    }
  }
}

__global__ void __launch_bounds__(256) ebe_sum_kernel(EbeArgs a, double* __restrict__ y) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
    const uint32_t t = i / (uint32_t)a.px;
    const int yy = (int)(t % (uint32_t)a.py);
    const int z = (int)(t / (uint32_t)a.py);
    const bool y0 = yy < a.ny, y1 = yy >= 1, z0 = z < a.nz, z1 = z >= 1;
    double s = 0.0;
    if (y0 && z0) s = a.part[i];
    if (y1 && z0) s += a.part[(size_t)a.N + i];
    if (y0 && z1) s += a.part[2 * (size_t)a.N + i];
    if (y1 && z1) s += a.part[3 * (size_t)a.N + i];
    y[i] = s;
  }
}

}  // namespace femheat
