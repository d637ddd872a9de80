/*
 * CPU oracle for the assembly-free transient heat-flow method (arXiv:1905.07622).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  See
 * fem_oracle.h for the layout conventions.
 *
 * What it computes, in the paper's order:
 *  - element matrices M_e, K_e of the trilinear hexahedron by Gauss quadrature
 *    (Sec. 3.2, "FE Formulation II");
 *  - the assembled system A = M + theta*dt*K and right-hand operator
 *    L = M - (1-theta)*dt*K with per-element rho*C and k (Sec. 3.1/3.2);
 *  - the boundary load vector F from the flux condition k dT/dn = f (Sec. 3.1);
 *  - per time step b = L U^{i-1} + dt*F and Jacobi-preconditioned CG
 *    (Algorithm 1) on A U^i = b.
 * Readings where the paper is silent or ambiguous (each one is repeated where
 * it is used):
 *  - delta_old is set to delta_new just before delta_new is recomputed;
 *  - the loop continues while delta_new > rtol^2 * delta_b, where
 *    delta_b = b^T P^-1 b over free rows (a relative residual test; the
 *    experiments of Sec. 5.1 quote a relative tolerance);
 *  - residual replacement r = b - A x happens when i mod 50 == 0 with i
 *    counted from 0 before its increment, as printed;
 *  - the load is dt*s_n*F (the dt of the displayed system, not the "+F" of
 *    the abbreviated form), s_n a per-step schedule value;
 *  - Dirichlet faces (not in the paper, which has flux conditions only) are
 *    imposed by symmetric elimination;
 *  - the initial guess is the linear extrapolation 2 T^{n-1} - T^{n-2} of the
 *    u0_update kernel (App. A.2) with the two previous fields kept separately.
 */
#include "fem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 4096

/* ------------------------------------------------------------------------- */
/* indexing                                                                   */
/* ------------------------------------------------------------------------- */

static int64_t n_nodes(const oracle_problem *p) {
  return (int64_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1);
}
static int64_t n_elems(const oracle_problem *p) {
  return (int64_t)p->nx * p->ny * p->nz;
}
static int64_t node_id(const oracle_problem *p, int ix, int iy, int iz) {
  return ix + (int64_t)(p->nx + 1) * (iy + (int64_t)(p->ny + 1) * iz);
}
static int64_t elem_id(const oracle_problem *p, int ex, int ey, int ez) {
  return ex + (int64_t)p->nx * (ey + (int64_t)p->ny * ez);
}

/* ------------------------------------------------------------------------- */
/* element matrices (Sec. 3.2)                                                */
/* ------------------------------------------------------------------------- */

/* 1-D linear shape functions on [0,1]: phi_0 = 1-t, phi_1 = t. */
static double phi(int a, double t) { return a ? t : 1.0 - t; }
static double dphi(int a) { return a ? 1.0 : -1.0; }

void oracle_element_matrices(double hx, double hy, double hz, double *M, double *K) {
  const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  const double h[3] = {hx, hy, hz};
  const double jac = hx * hy * hz;
  memset(M, 0, 64 * sizeof(double));
  memset(K, 0, 64 * sizeof(double));
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {g[qx], g[qy], g[qz]};
        const double w = 0.125 * jac; /* weights 1/2 per axis on [0,1] */
        double N[8], dN[8][3];
        for (int a = 0; a < 8; ++a) {
          const int ab[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
          N[a] = phi(ab[0], xi[0]) * phi(ab[1], xi[1]) * phi(ab[2], xi[2]);
          for (int d = 0; d < 3; ++d) {
            double v = dphi(ab[d]) / h[d];
            for (int e = 0; e < 3; ++e)
              if (e != d) v *= phi(ab[e], xi[e]);
            dN[a][d] = v;
          }
        }
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            M[a * 8 + b] += w * N[a] * N[b];
            K[a * 8 + b] += w * (dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2]);
          }
      }
}

/* The paper's element (Sec. 4.1): every box of the fixed grid split into six
 * linear tetrahedra.  Which six is not stated; the split taken here is the one
 * around the box diagonal from corner 0 to corner 7, tetrahedron
 * 0 -> 0 + e_i -> 0 + e_i + e_j -> 7 for each order (i, j, k) of the axes,
 * which gives the same diagonal on the shared face of every two neighbouring
 * boxes, so the mesh is conforming. */
static const int kTet6[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};

static void corner_xyz(int a, const double h[3], double x[3]) {
  x[0] = (a & 1) * h[0];
  x[1] = ((a >> 1) & 1) * h[1];
  x[2] = ((a >> 2) & 1) * h[2];
}

/* Barycentric gradients of a tetrahedron with vertices X[4][3] and its volume:
 * grad l_k for k = 1..3 are the rows of J^-1 with J = [X1-X0, X2-X0, X3-X0]
 * (columns), grad l_0 = -(sum of the others). */
static double tet_gradients(const double X[4][3], double G[4][3]) {
  double J[3][3];
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 3; ++k) J[d][k] = X[k + 1][d] - X[0][d];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int d = 0; d < 3; ++d) {
    G[0][d] = 0.0;
    for (int k = 0; k < 3; ++k) {
      G[k + 1][d] = inv[k][d];
      G[0][d] -= inv[k][d];
    }
  }
  return fabs(det) / 6.0;
}

/* 8x8 box matrices of the six-tetrahedron split: the sum of the 4x4
 * tetrahedron matrices M_t = int l_i l_j (4-point Gauss rule, exact for
 * quadratics) and K_t = int grad l_i . grad l_j (constant gradients). */
void oracle_tet6_matrices(double hx, double hy, double hz, double *M, double *K) {
  const double h[3] = {hx, hy, hz};
  const double qa = 0.5854101966249685, qb = 0.1381966011250105; /* (5 +- 3 sqrt 5)/20 */
  memset(M, 0, 64 * sizeof(double));
  memset(K, 0, 64 * sizeof(double));
  for (int t = 0; t < 6; ++t) {
    double X[4][3], G[4][3];
    for (int k = 0; k < 4; ++k) corner_xyz(kTet6[t][k], h, X[k]);
    const double V = tet_gradients(X, G);
    for (int q = 0; q < 4; ++q) {
      double l[4];
      for (int k = 0; k < 4; ++k) l[k] = (k == q) ? qa : qb;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) M[kTet6[t][i] * 8 + kTet6[t][j]] += 0.25 * V * l[i] * l[j];
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        K[kTet6[t][i] * 8 + kTet6[t][j]] += V * (G[i][0] * G[j][0] + G[i][1] * G[j][1] + G[i][2] * G[j][2]);
  }
}

/* The 8x8 blocks of one box of the problem's element kind. */
static void box_matrices(const oracle_problem *p, double *M, double *K) {
  if (p->element == ORACLE_ELEM_TET6)
    oracle_tet6_matrices(p->hx, p->hy, p->hz, M, K);
  else
    oracle_element_matrices(p->hx, p->hy, p->hz, M, K);
}

/* ------------------------------------------------------------------------- */
/* assembly into CSR (Sec. 3.2, the assembly operator)                        */
/* ------------------------------------------------------------------------- */

static int64_t find_col(const int32_t *col, int64_t lo, int64_t hi, int64_t j) {
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (col[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

int oracle_assemble(const oracle_problem *p, double cm, double ck, oracle_csr *out, int nthreads) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = n_nodes(p);
  double M[64], K[64];
  box_matrices(p, M, K);
  int64_t *rowptr = (int64_t *)malloc((size_t)(N + 1) * sizeof(int64_t));
  if (!rowptr) return ORACLE_ENOMEM;
  rowptr[0] = 0;
  for (int iz = 0; iz <= nz; ++iz)
    for (int iy = 0; iy <= ny; ++iy)
      for (int ix = 0; ix <= nx; ++ix) {
        const int cx = 1 + (ix > 0) + (ix < nx), cy = 1 + (iy > 0) + (iy < ny), cz = 1 + (iz > 0) + (iz < nz);
        const int64_t i = node_id(p, ix, iy, iz);
        rowptr[i + 1] = rowptr[i] + cx * cy * cz;
      }
  const int64_t nnz = rowptr[N];
  int32_t *col = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
  double *val = (double *)malloc((size_t)nnz * sizeof(double));
  if (!col || !val) {
    free(rowptr);
    free(col);
    free(val);
    return ORACLE_ENOMEM;
  }
  (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < N; ++i) {
    const int ix = (int)(i % (nx + 1));
    const int iy = (int)((i / (nx + 1)) % (ny + 1));
    const int iz = (int)(i / ((int64_t)(nx + 1) * (ny + 1)));
    int64_t pos = rowptr[i];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
          if (jx < 0 || jx > nx || jy < 0 || jy > ny || jz < 0 || jz > nz) continue;
          col[pos] = (int32_t)node_id(p, jx, jy, jz);
          val[pos] = 0.0;
          ++pos;
        }
    /* sum the element contributions A_e[a][b] over the elements around node i */
    for (int oz = 0; oz < 2; ++oz)
      for (int oy = 0; oy < 2; ++oy)
        for (int ox = 0; ox < 2; ++ox) {
          const int ex = ix - 1 + ox, ey = iy - 1 + oy, ez = iz - 1 + oz;
          if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
          const int64_t e = elem_id(p, ex, ey, ez);
          const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
          const double sm = cm * p->rhoc_e[e], sk = ck * p->k_e[e];
          for (int b = 0; b < 8; ++b) {
            const int64_t j = node_id(p, ex + (b & 1), ey + ((b >> 1) & 1), ez + ((b >> 2) & 1));
            const int64_t s = find_col(col, rowptr[i], rowptr[i + 1], j);
            val[s] += sm * M[a * 8 + b] + sk * K[a * 8 + b];
          }
        }
  }
  out->n = N;
  out->nnz = nnz;
  out->rowptr = rowptr;
  out->col = col;
  out->val = val;
  return ORACLE_OK;
}

void oracle_csr_free(oracle_csr *a) {
  free(a->rowptr);
  free(a->col);
  free(a->val);
  a->rowptr = NULL;
  a->col = NULL;
  a->val = NULL;
}

void oracle_spmv(const oracle_csr *a, const double *x, double *y, int nthreads) {
  (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t i = 0; i < a->n; ++i) {
    double s = 0.0;
    for (int64_t k = a->rowptr[i]; k < a->rowptr[i + 1]; ++k) s += a->val[k] * x[a->col[k]];
    y[i] = s;
  }
}

void oracle_element_loop(const oracle_problem *p, double cm, double ck, const double *x, double *y) {
  double M[64], K[64];
  box_matrices(p, M, K);
  memset(y, 0, (size_t)n_nodes(p) * sizeof(double));
  for (int ez = 0; ez < p->nz; ++ez)
    for (int ey = 0; ey < p->ny; ++ey)
      for (int ex = 0; ex < p->nx; ++ex) {
        const int64_t e = elem_id(p, ex, ey, ez);
        int64_t nodes[8];
        for (int a = 0; a < 8; ++a) nodes[a] = node_id(p, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
        for (int a = 0; a < 8; ++a) {
          double s = 0.0;
          for (int b = 0; b < 8; ++b)
            s += (cm * p->rhoc_e[e] * M[a * 8 + b] + ck * p->k_e[e] * K[a * 8 + b]) * x[nodes[b]];
          y[nodes[a]] += s;
        }
      }
}

/* ------------------------------------------------------------------------- */
/* boundary data                                                              */
/* ------------------------------------------------------------------------- */

void oracle_load_vector(const oracle_problem *p, double *F) {
  const int n[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->hx, p->hy, p->hz};
  const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  memset(F, 0, (size_t)n_nodes(p) * sizeof(double));
  for (int f = 0; f < 6; ++f) {
    if (!(p->flux_mask & (1u << f))) continue;
    const double q = p->flux[f];
    const int d = f / 2;                 /* normal axis */
    const int u = (d + 1) % 3, v = (d + 2) % 3; /* in-face axes */
    const int fixed = (f % 2) ? n[d] : 0;
    const double area = h[u] * h[v];
    if (p->element == ORACLE_ELEM_TET6) {
      /* the faces of the tetrahedra on a box face: two triangles split by the
       * diagonal from its low corner (0,0) to its high corner (1,1) in the two
       * in-face axes; each vertex gets the integral of its linear function by
       * the 3-point edge-midpoint rule (exact for quadratics) */
      const int tri[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {0, 1}, {1, 1}}};
      for (int eu = 0; eu < n[u]; ++eu)
        for (int ev = 0; ev < n[v]; ++ev)
          for (int t = 0; t < 2; ++t)
            for (int k = 0; k < 3; ++k) {
              double s = 0.0;
              for (int m = 0; m < 3; ++m) { /* midpoint of the edge opposite to vertex m */
                double lk = 0.0;
                for (int j = 0; j < 3; ++j)
                  if (j != m) lk += (j == k) ? 0.5 : 0.0;
                s += (0.5 * area / 3.0) * lk;
              }
              int idx[3];
              idx[d] = fixed;
              idx[u] = eu + tri[t][k][0];
              idx[v] = ev + tri[t][k][1];
              F[node_id(p, idx[0], idx[1], idx[2])] += q * s;
            }
      continue;
    }
    for (int eu = 0; eu < n[u]; ++eu)
      for (int ev = 0; ev < n[v]; ++ev)
        for (int c = 0; c < 4; ++c) {
          const int cu = c & 1, cv = (c >> 1) & 1;
          double s = 0.0; /* integral of the bilinear corner function over the face element */
          for (int qu = 0; qu < 2; ++qu)
            for (int qv = 0; qv < 2; ++qv) s += 0.25 * area * phi(cu, g[qu]) * phi(cv, g[qv]);
          int idx[3];
          idx[d] = fixed;
          idx[u] = eu + cu;
          idx[v] = ev + cv;
          F[node_id(p, idx[0], idx[1], idx[2])] += q * s;
        }
  }
}

void oracle_dirichlet(const oracle_problem *p, uint8_t *is_dir, double *g) {
  for (int iz = 0; iz <= p->nz; ++iz)
    for (int iy = 0; iy <= p->ny; ++iy)
      for (int ix = 0; ix <= p->nx; ++ix) {
        const int64_t i = node_id(p, ix, iy, iz);
        const int on[6] = {ix == 0, ix == p->nx, iy == 0, iy == p->ny, iz == 0, iz == p->nz};
        is_dir[i] = 0;
        g[i] = 0.0;
        for (int f = 0; f < 6; ++f) /* lowest-numbered Dirichlet face decides the value */
          if ((p->dirichlet_mask & (1u << f)) && on[f]) {
            is_dir[i] = 1;
            g[i] = p->dirichlet_value[f];
            break;
          }
      }
}

void oracle_sensors(const oracle_problem *p, const double *T, const double *xyz, int32_t n, double *out) {
  const int nn[3] = {p->nx, p->ny, p->nz};
  const double h[3] = {p->hx, p->hy, p->hz};
  for (int32_t s = 0; s < n; ++s) {
    int e[3];
    double xi[3];
    for (int d = 0; d < 3; ++d) {
      const double t = xyz[3 * s + d] / h[d];
      int k = (int)ceil(t) - 1; /* lowest-index element on a shared face */
      if (k < 0) k = 0;
      if (k > nn[d] - 1) k = nn[d] - 1;
      double loc = t - k;
      if (loc < 0) loc = 0;
      if (loc > 1) loc = 1;
      e[d] = k;
      xi[d] = loc;
    }
    double v = 0.0;
    if (p->element == ORACLE_ELEM_TET6) {
      /* the tetrahedron whose barycentric coordinates of the point are all
       * >= 0 (the first one, on shared faces), the field linear in it */
      const double hu[3] = {1.0, 1.0, 1.0};
      int found = 0;
      for (int t = 0; t < 6 && !found; ++t) {
        double X[4][3], G[4][3], l[4];
        for (int k = 0; k < 4; ++k) corner_xyz(kTet6[t][k], hu, X[k]);
        (void)tet_gradients(X, G);
        double mn = 1.0;
        for (int k = 1; k < 4; ++k) {
          l[k] = G[k][0] * (xi[0] - X[0][0]) + G[k][1] * (xi[1] - X[0][1]) + G[k][2] * (xi[2] - X[0][2]);
        }
        l[0] = 1.0 - l[1] - l[2] - l[3];
        for (int k = 0; k < 4; ++k) mn = l[k] < mn ? l[k] : mn;
        if (mn < -1e-12) continue;
        found = 1;
        for (int k = 0; k < 4; ++k) {
          const int a = kTet6[t][k];
          v += l[k] * T[node_id(p, e[0] + (a & 1), e[1] + ((a >> 1) & 1), e[2] + ((a >> 2) & 1))];
        }
      }
    } else {
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        v += phi(ax, xi[0]) * phi(ay, xi[1]) * phi(az, xi[2]) * T[node_id(p, e[0] + ax, e[1] + ay, e[2] + az)];
      }
    }
    out[s] = v;
  }
}

/* ------------------------------------------------------------------------- */
/* vector helpers                                                             */
/* ------------------------------------------------------------------------- */

/* sum_i a_i*b_i in fixed chunks summed in chunk order: thread-count invariant */
static double dot(const double *a, const double *b, int64_t n, int nthreads) {
  const int64_t nc = (n + CHUNK - 1) / CHUNK;
  double *part = (double *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(double));
  (void)nthreads;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t lo = c * CHUNK, hi = lo + CHUNK < n ? lo + CHUNK : n;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += a[i] * b[i];
    part[c] = s;
  }
  double s = 0.0;
  for (int64_t c = 0; c < nc; ++c) s += part[c];
  free(part);
  return s;
}

static void diag_of(const oracle_csr *A, double *P) {
  for (int64_t i = 0; i < A->n; ++i) {
    P[i] = 0.0;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
      if (A->col[k] == i) P[i] = A->val[k];
  }
}

/* ------------------------------------------------------------------------- */
/* Chebyshev-accelerated Jacobi preconditioner (not in the paper, whose GPU   */
/* method uses Jacobi only, Sec. 3.3; a polynomial preconditioner is the kind */
/* that stays element-wise and matrix-free on the device)                     */
/* ------------------------------------------------------------------------- */

/* Largest eigenvalue of the symmetric 8x8 matrix D^-1/2 X D^-1/2 (D = diag X)
 * by power iteration from a fixed generic start: plain and slow, 8x8 only. */
static double scaled_top_eigenvalue(const double *X) {
  double v[8], w[8], lam = 0.0;
  for (int a = 0; a < 8; ++a) v[a] = 1.0 + 0.1 * a + 0.01 * a * a;
  for (int it = 0; it < 2000; ++it) {
    double n = 0.0;
    for (int a = 0; a < 8; ++a) {
      double t = 0.0;
      for (int b = 0; b < 8; ++b) t += X[a * 8 + b] / sqrt(X[a * 8 + a] * X[b * 8 + b]) * v[b];
      w[a] = t;
      n += t * t;
    }
    n = sqrt(n);
    lam = 0.0;
    for (int a = 0; a < 8; ++a) {
      lam += v[a] * w[a];
      v[a] = w[a] / n;
    }
  }
  return lam;
}

/* For A = sum_e (rho_e M_e + c k_e K_e) with rho_e > 0, c k_e >= 0 and D its
 * diagonal, the Rayleigh quotient x^T A x / x^T D x is a weighted mean of the
 * element quotients x_e^T M_e x_e / x_e^T diag(M_e) x_e and the same for K_e,
 * so the spectrum of D^-1 A lies below the larger of the two element maxima,
 * for every coefficient field (Dirichlet elimination keeps it below). */
double oracle_cheb_upper(double hx, double hy, double hz) {
  double M[64], K[64];
  oracle_element_matrices(hx, hy, hz, M, K);
  const double lm = scaled_top_eigenvalue(M), lk = scaled_top_eigenvalue(K);
  return lm > lk ? lm : lk;
}

/* s = M^-1 r for the preconditioner defined by m steps of the Chebyshev
 * iteration for D^-1 A x = D^-1 r from x = 0 on the interval [lo, hi]:
 * with c = (hi+lo)/2, w = (hi-lo)/2 and sigma = c/w,
 *   x = 0, res = r, rho = 1/sigma, d = D^-1 res / c;
 *   repeat m times: x += d; stop after the m-th; res -= A d;
 *                   rho' = 1/(2 sigma - rho); d = rho' rho d + (2 rho'/w) D^-1 res; rho = rho'.
 * The result is q(D^-1 A) D^-1 r where 1 - lambda q(lambda) is the Chebyshev
 * polynomial of degree m shifted to [lo, hi] and scaled to 1 at 0: it lies in
 * (0, 2) on [lo, hi] and in (0, 1] below lo, so M^-1 is symmetric positive
 * definite whenever hi bounds the spectrum.  Rows with P = 0 give s = 0. */
void oracle_cheb_apply(const oracle_csr *A, const double *P, int32_t m, double lo, double hi, const double *r,
                       double *s, int nthreads) {
  const int64_t n = A->n;
  double *res = (double *)malloc((size_t)n * sizeof(double));
  double *d = (double *)malloc((size_t)n * sizeof(double));
  double *w = (double *)malloc((size_t)n * sizeof(double));
  const double c = 0.5 * (hi + lo), wd = 0.5 * (hi - lo), sigma = c / wd;
  double rho = 1.0 / sigma;
  for (int64_t i = 0; i < n; ++i) {
    s[i] = 0.0;
    res[i] = r[i];
    d[i] = P[i] > 0.0 ? res[i] / P[i] / c : 0.0;
  }
  for (int32_t k = 1; k <= m; ++k) {
    for (int64_t i = 0; i < n; ++i) s[i] += d[i];
    if (k == m) break;
    oracle_spmv(A, d, w, nthreads);
    const double rn = 1.0 / (2.0 * sigma - rho);
    for (int64_t i = 0; i < n; ++i) {
      res[i] -= w[i];
      d[i] = rn * rho * d[i] + (2.0 * rn / wd) * (P[i] > 0.0 ? res[i] / P[i] : 0.0);
    }
    rho = rn;
  }
  free(res);
  free(d);
  free(w);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1: preconditioned conjugate gradient                             */
/* ------------------------------------------------------------------------- */

/* s = preconditioner applied to r: P^-1 r (Jacobi, Sec. 3.3) or the
 * Chebyshev polynomial above (pc != NULL).  Rows with P = 0 (eliminated
 * Dirichlet rows of a caller that marks them so) give 0. */
static void precondition(const oracle_csr *A, const double *P, const oracle_precond *pc, const double *r, double *s,
                         int nthreads) {
  if (pc && pc->kind == ORACLE_PRECOND_CHEBYSHEV) {
    oracle_cheb_apply(A, P, pc->degree, pc->lo, pc->hi, r, s, nthreads);
  } else {
    for (int64_t k = 0; k < A->n; ++k) s[k] = P[k] > 0.0 ? r[k] / P[k] : 0.0;
  }
}

int oracle_pcg_prec(const oracle_csr *A, const double *b, double *x, int32_t max_iter, double tol_scale,
                    int32_t relative_to_initial, int32_t replace_every, int32_t locked, const oracle_precond *pc,
                    const double *Pdiag, double *delta_out, double *tol_out, int nthreads) {
  const int64_t n = A->n;
  double *P = (double *)malloc((size_t)n * sizeof(double));
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *d = (double *)malloc((size_t)n * sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  double *s = (double *)malloc((size_t)n * sizeof(double));
  if (!P || !r || !d || !q || !s) {
    free(P); free(r); free(d); free(q); free(s);
    return ORACLE_ENOMEM;
  }
  if (Pdiag)
    memcpy(P, Pdiag, (size_t)n * sizeof(double));
  else
    diag_of(A, P);
  int status = 0;
  int32_t i = 0;
  /* r <- b - A x ; d <- M^-1 r ; delta_new <- r^T d */
  oracle_spmv(A, x, r, nthreads);
  for (int64_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
  precondition(A, P, pc, r, d, nthreads);
  double delta_new = dot(r, d, n, nthreads);
  const double tol = relative_to_initial ? tol_scale * delta_new : tol_scale;
  *tol_out = tol;
  for (;;) {
    if (locked >= 0) {
      if (i >= locked) break;
    } else if (!(i < max_iter && delta_new > tol)) {
      break;
    }
    oracle_spmv(A, d, q, nthreads);                 /* q <- A d */
    const double dq = dot(d, q, n, nthreads);
    if (!(dq > 0.0) || !isfinite(dq)) {
      status = ORACLE_EBREAKDOWN;
      break;
    }
    const double alpha = delta_new / dq;            /* alpha <- delta_new / d^T q */
    for (int64_t k = 0; k < n; ++k) x[k] += alpha * d[k];
    if (replace_every > 0 && i % replace_every == 0) {
      oracle_spmv(A, x, r, nthreads);               /* r <- b - A x */
      for (int64_t k = 0; k < n; ++k) r[k] = b[k] - r[k];
    } else {
      for (int64_t k = 0; k < n; ++k) r[k] -= alpha * q[k];
    }
    precondition(A, P, pc, r, s, nthreads);         /* s <- M^-1 r */
    const double delta_old = delta_new;             /* delta_old is not assigned in the listing */
    delta_new = dot(r, s, n, nthreads);
    if (!isfinite(delta_new)) {
      status = ORACLE_EBREAKDOWN;
      break;
    }
    const double beta = delta_new / delta_old;
    for (int64_t k = 0; k < n; ++k) d[k] = s[k] + beta * d[k];
    ++i;
  }
  *delta_out = delta_new;
  free(P); free(r); free(d); free(q); free(s);
  return status ? status : i;
}

int oracle_pcg(const oracle_csr *A, const double *b, double *x, int32_t max_iter, double tol_scale,
               int32_t relative_to_initial, int32_t replace_every, int32_t locked, double *delta_out,
               double *tol_out, int nthreads) {
  return oracle_pcg_prec(A, b, x, max_iter, tol_scale, relative_to_initial, replace_every, locked, NULL, NULL,
                         delta_out, tol_out, nthreads);
}

/* ------------------------------------------------------------------------- */
/* the theta-scheme time loop (Sec. 3.1)                                      */
/* ------------------------------------------------------------------------- */

static int valid(const oracle_problem *p, const oracle_controls *c) {
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
  if (p->element != ORACLE_ELEM_HEX8 && p->element != ORACLE_ELEM_TET6) return 0;
  if (c && c->precond == ORACLE_PRECOND_CHEBYSHEV && p->element != ORACLE_ELEM_HEX8) return 0;
  if (!(p->hx > 0) || !(p->hy > 0) || !(p->hz > 0)) return 0;
  if ((p->dirichlet_mask | p->flux_mask) >= 64u || (p->dirichlet_mask & p->flux_mask)) return 0;
  for (int64_t e = 0; e < n_elems(p); ++e) {
    if (!(p->k_e[e] >= 0) || !isfinite(p->k_e[e])) return 0;
    if (!(p->rhoc_e[e] > 0) || !isfinite(p->rhoc_e[e])) return 0;
  }
  if (c) {
    if (!(c->dt > 0) || !(c->theta >= 0 && c->theta <= 1) || !(c->rtol > 0) || c->nsteps < 0) return 0;
    if (c->max_iter < 0 || c->replace_every < 0) return 0;
    if (c->precond != ORACLE_PRECOND_JACOBI && c->precond != ORACLE_PRECOND_CHEBYSHEV) return 0;
    if (c->precond == ORACLE_PRECOND_CHEBYSHEV && (c->cheb_degree < 2 || !(c->cheb_ratio > 1.0))) return 0;
  }
  return 1;
}

static double schedule(const oracle_problem *p, int64_t m) {
  if (!p->flux_schedule) return 1.0;
  if (m < 1 || m > p->n_schedule) return 0.0;
  return p->flux_schedule[m - 1];
}

int oracle_run(const oracle_problem *p, const double *T0, const double *T_prev, const oracle_controls *c,
               oracle_outputs *o) {
  if (!valid(p, c)) return ORACLE_EINVAL;
  const int nt = c->nthreads;
  const int64_t N = n_nodes(p);
  int status = ORACLE_OK;
  oracle_csr A = {0}, L = {0};
  int rc = oracle_assemble(p, 1.0, c->theta * c->dt, &A, nt);
  if (rc) return rc;
  rc = oracle_assemble(p, 1.0, -(1.0 - c->theta) * c->dt, &L, nt);
  if (rc) {
    oracle_csr_free(&A);
    return rc;
  }
  double *F = (double *)malloc((size_t)N * sizeof(double));
  double *g = (double *)malloc((size_t)N * sizeof(double));
  uint8_t *dir = (uint8_t *)malloc((size_t)N);
  double *lift = (double *)calloc((size_t)N, sizeof(double));
  double *P = (double *)malloc((size_t)N * sizeof(double));
  double *T1 = (double *)malloc((size_t)N * sizeof(double));
  double *T2 = (double *)malloc((size_t)N * sizeof(double));
  double *x = (double *)malloc((size_t)N * sizeof(double));
  double *b = (double *)malloc((size_t)N * sizeof(double));
  double *w = (double *)malloc((size_t)N * sizeof(double));
  double *Pm = NULL, *bf = NULL;
  if (!F || !g || !dir || !lift || !P || !T1 || !T2 || !x || !b || !w) {
    status = ORACLE_ENOMEM;
    goto done;
  }
  oracle_load_vector(p, F);
  oracle_dirichlet(p, dir, g);

  /* symmetric elimination: lift_f = A_fD g_D, then zero the Dirichlet rows and
   * columns of A and put 1 on their diagonal */
  for (int64_t i = 0; i < N; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      const int64_t j = A.col[k];
      if (dir[i]) {
        A.val[k] = (j == i) ? 1.0 : 0.0;
      } else if (dir[j]) {
        lift[i] += A.val[k] * g[j];
        A.val[k] = 0.0;
      }
    }
  diag_of(&A, P);
  /* Chebyshev preconditioner: interval [hi/ratio, hi] from the bound of the
   * spectrum of D^-1 A; the diagonal it scales by is 0 on Dirichlet rows, so
   * they stay out of every preconditioned vector */
  const int cheb = c->precond == ORACLE_PRECOND_CHEBYSHEV;
  oracle_precond pc = {ORACLE_PRECOND_JACOBI, 0, 0.0, 0.0};
  if (cheb) {
    Pm = (double *)malloc((size_t)N * sizeof(double));
    bf = (double *)malloc((size_t)N * sizeof(double));
    if (!Pm || !bf) {
      status = ORACLE_ENOMEM;
      goto done;
    }
    pc.kind = ORACLE_PRECOND_CHEBYSHEV;
    pc.degree = c->cheb_degree;
    pc.hi = oracle_cheb_upper(p->hx, p->hy, p->hz);
    pc.lo = pc.hi / c->cheb_ratio;
    for (int64_t i = 0; i < N; ++i) Pm[i] = dir[i] ? 0.0 : P[i];
  }

  for (int64_t i = 0; i < N; ++i) {
    T1[i] = dir[i] ? g[i] : T0[i];
    T2[i] = dir[i] ? g[i] : (T_prev ? T_prev[i] : T0[i]);
  }

  for (int32_t n = 1; n <= c->nsteps; ++n) {
    const double s_n = schedule(p, (int64_t)c->first_step + n);
    /* b = L T^{n-1} + dt*s_n*F, lifted */
    oracle_spmv(&L, T1, b, nt);
    for (int64_t i = 0; i < N; ++i) {
      b[i] += c->dt * s_n * F[i];
      b[i] = dir[i] ? g[i] : b[i] - lift[i];
      w[i] = dir[i] ? 0.0 : b[i] / P[i];
    }
    double delta_b;
    if (cheb) {  /* b^T M^-1 b over the free rows, M^-1 the Chebyshev preconditioner */
      for (int64_t i = 0; i < N; ++i) bf[i] = dir[i] ? 0.0 : b[i];
      oracle_cheb_apply(&A, Pm, pc.degree, pc.lo, pc.hi, bf, w, nt);
      delta_b = dot(bf, w, N, nt);
    } else {
      delta_b = dot(b, w, N, nt);
    }
    for (int64_t i = 0; i < N; ++i)
      x[i] = (c->guess == ORACLE_GUESS_PREV) ? T1[i] : 2.0 * T1[i] - T2[i];
    int it;
    double delta = 0.0, tol = 0.0;
    const int32_t locked = c->locked_iters ? c->locked_iters[n - 1] : -1;
    if (c->stop_rule == ORACLE_STOP_RHS && delta_b == 0.0 && locked <= 0) {
      for (int64_t i = 0; i < N; ++i) x[i] = dir[i] ? g[i] : 0.0; /* zero right-hand side */
      it = 0;
    } else {
      const double rt2 = c->rtol * c->rtol;
      it = oracle_pcg_prec(&A, b, x, c->max_iter, c->stop_rule == ORACLE_STOP_RHS ? rt2 * delta_b : rt2,
                           c->stop_rule == ORACLE_STOP_INITIAL, c->replace_every, locked, cheb ? &pc : NULL,
                           cheb ? Pm : NULL, &delta, &tol, nt);
      if (it < 0) {
        status = it;
        goto done;
      }
      if (locked < 0 && it >= c->max_iter && delta > tol) status = ORACLE_ENOCONV;
    }
    double *tmp = T2;
    T2 = T1;
    T1 = x;
    x = tmp;
    if (o->iters) o->iters[n - 1] = it;
    if (o->relres) o->relres[n - 1] = delta_b > 0 ? sqrt(delta / delta_b) : 0.0;
    if (o->T_saved && o->save_every > 0 && n % o->save_every == 0)
      memcpy(o->T_saved + (size_t)(n / o->save_every - 1) * N, T1, (size_t)N * sizeof(double));
    if (o->traces && o->sensor_xyz && o->n_sensors > 0)
      oracle_sensors(p, T1, o->sensor_xyz, o->n_sensors, o->traces + (size_t)(n - 1) * o->n_sensors);
  }
  if (o->T_final) memcpy(o->T_final, T1, (size_t)N * sizeof(double));

done:
  oracle_csr_free(&A);
  oracle_csr_free(&L);
  free(F); free(g); free(dir); free(lift); free(P); free(T1); free(T2); free(x); free(b); free(w);
  free(Pm); free(bf);
  return status;
}
