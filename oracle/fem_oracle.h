/*
 * CPU oracle for the assembly-free transient heat-flow method of Loeb & Earls,
 * "Analysis of heterogeneous computing approaches to simulating heat transfer
 * in heterogeneous material" (arXiv:1905.07622).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial-by-construction FP64
 * implementation of what the method computes, written from the paper with an
 * ASSEMBLED sparse matrix (CSR), element matrices integrated by Gauss
 * quadrature and textbook preconditioned CG.  It exists so that the GPU
 * library can be checked against an independent implementation.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the GPU library never links, includes or calls it.
 *
 * Optional OpenMP threads split rows (sparse products) and fixed 4096-entry
 * chunks (dot products, summed in chunk order), so results are bitwise the same
 * for any thread count.
 *
 * Layout: nodes i = ix + (nx+1)*(iy + (ny+1)*iz) (x fastest, Sec. 4.1);
 * elements e = ex + nx*(ey + ny*ez); local hexahedron corner
 * a = ax + 2*ay + 4*az.  Faces 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.
 */
#ifndef FEM_ORACLE_H
#define FEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
  ORACLE_ENOMEM = -2,
  ORACLE_ENOCONV = -3,
  ORACLE_EBREAKDOWN = -4
};

enum { ORACLE_GUESS_EXTRAP = 0, ORACLE_GUESS_PREV = 1 };
enum { ORACLE_STOP_RHS = 0, ORACLE_STOP_INITIAL = 1 };
enum { ORACLE_ELEM_HEX8 = 0, ORACLE_ELEM_TET6 = 1 };
enum { ORACLE_PRECOND_JACOBI = 0, ORACLE_PRECOND_CHEBYSHEV = 1 };

/* A preconditioner for oracle_pcg_prec: Jacobi (Sec. 3.3), or the Chebyshev
 * polynomial of `degree` on [lo, hi] in the Jacobi-scaled operator. */
typedef struct {
  int32_t kind;
  int32_t degree;
  double lo, hi;
} oracle_precond;

typedef struct {
  int32_t nx, ny, nz;
  double hx, hy, hz;
  const double *k_e;     /* E conductivities */
  const double *rhoc_e;  /* E heat capacities (rho*C) */
  uint32_t dirichlet_mask;
  double dirichlet_value[6];
  uint32_t flux_mask;
  double flux[6];          /* inward flux q per face */
  const double *flux_schedule; /* s_m for global step m = 1..n_schedule; NULL: s = 1 */
  int32_t n_schedule;
  int32_t element;         /* ORACLE_ELEM_HEX8: one trilinear hexahedron per box; ORACLE_ELEM_TET6: six
                              linear tetrahedra per box around its 0-7 diagonal (Sec. 4.1) */
} oracle_problem;

typedef struct {
  double dt, theta, rtol;
  int32_t nsteps;
  int32_t max_iter;       /* i_max of Algorithm 1 */
  int32_t replace_every;  /* residual replacement period (50 in Algorithm 1); 0: never */
  int32_t guess;          /* ORACLE_GUESS_* */
  int32_t stop_rule;      /* ORACLE_STOP_* */
  int32_t first_step;     /* global index of the step before the first one of this run */
  const int32_t *locked_iters; /* NULL: stop by the tolerance; else run exactly these counts */
  int32_t nthreads;
  int32_t precond;        /* ORACLE_PRECOND_*; the stop rule's norm is the preconditioner's */
  int32_t cheb_degree;    /* Chebyshev: polynomial degree m >= 2 (m - 1 operator applies) */
  double cheb_ratio;      /* Chebyshev: interval [hi/ratio, hi], hi = oracle_cheb_upper */
} oracle_controls;

typedef struct {
  double *T_final;            /* N */
  double *T_saved;            /* (nsteps/save_every) * N, or NULL */
  int32_t save_every;
  const double *sensor_xyz;   /* 3*S points, or NULL */
  int32_t n_sensors;
  double *traces;             /* nsteps * S, row-major [step][sensor] */
  int32_t *iters;             /* nsteps, or NULL */
  double *relres;             /* nsteps, or NULL */
} oracle_outputs;

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *rowptr;
  int32_t *col;
  double *val;
} oracle_csr;

/* Element mass and stiffness matrices (8x8, row-major) of the trilinear
 * hexahedron hx*hy*hz by 2x2x2 Gauss-Legendre quadrature (Sec. 3.2). */
void oracle_element_matrices(double hx, double hy, double hz, double *M, double *K);

/* 8x8 box matrices of the six-tetrahedron split (sum of the six linear
 * tetrahedra of the box, mass by a 4-point Gauss rule). */
void oracle_tet6_matrices(double hx, double hy, double hz, double *M, double *K);

/* Assembled CSR of  sum_e (cm*rhoc_e*M_e + ck*k_e*K_e)  (no boundary rows
 * modified).  Returns ORACLE_OK or ORACLE_ENOMEM. */
int oracle_assemble(const oracle_problem *p, double cm, double ck, oracle_csr *out, int nthreads);
void oracle_csr_free(oracle_csr *a);
void oracle_spmv(const oracle_csr *a, const double *x, double *y, int nthreads);

/* Brute-force element loop y = sum_e (cm*rhoc_e*M_e + ck*k_e*K_e) x_e with no
 * assembled matrix (the EbE reading of the assembly operator, eq. EbEvsDbD). */
void oracle_element_loop(const oracle_problem *p, double cm, double ck, const double *x, double *y);

/* Boundary load vector F_i = sum over flux faces of integral q*N_i ds by 2x2
 * Gauss quadrature on every face element (Sec. 3.1). */
void oracle_load_vector(const oracle_problem *p, double *F);

/* 1 where node i is a Dirichlet node, with its value in g (0 elsewhere). */
void oracle_dirichlet(const oracle_problem *p, uint8_t *is_dir, double *g);

/* Field value at points by trilinear interpolation in the containing element. */
void oracle_sensors(const oracle_problem *p, const double *T, const double *xyz, int32_t n, double *out);

/* Full theta-scheme run (Sec. 3.1) with Jacobi-PCG per step (Algorithm 1). */
int oracle_run(const oracle_problem *p, const double *T0, const double *T_prev,
               const oracle_controls *c, oracle_outputs *o);

/* One PCG solve of A x = b with Jacobi preconditioner P = diag(A)
 * (Algorithm 1).  The loop runs while delta_new > tol and i < max_iter, where
 * tol = tol_scale, or tol_scale * delta_0 when relative_to_initial is set
 * (delta_0 = r0^T P^-1 r0).  If locked >= 0 it runs exactly `locked`
 * iterations instead.  Returns the iteration count (>= 0) or
 * ORACLE_EBREAKDOWN; *delta_out gets the final r^T P^-1 r and *tol_out the
 * threshold that was used. */
int oracle_pcg(const oracle_csr *A, const double *b, double *x, int32_t max_iter,
               double tol_scale, int32_t relative_to_initial, int32_t replace_every,
               int32_t locked, double *delta_out, double *tol_out, int nthreads);

/* Upper bound of the spectrum of D^-1 A (D = diag A) for every coefficient
 * field on this element box: the larger of the element maxima for the mass
 * and the stiffness block, each by power iteration on the 8x8 block. */
double oracle_cheb_upper(double hx, double hy, double hz);

/* s = q(D^-1 A) D^-1 r: m steps of the Chebyshev iteration on [lo, hi] from 0
 * (m - 1 products with A); rows with P[i] = 0 give s[i] = 0. */
void oracle_cheb_apply(const oracle_csr *A, const double *P, int32_t m, double lo, double hi, const double *r,
                       double *s, int nthreads);

/* oracle_pcg with a preconditioner (pc NULL: Jacobi) and optionally the
 * diagonal it scales by (Pdiag NULL: diag A).  delta = r^T M^-1 r. */
int oracle_pcg_prec(const oracle_csr *A, const double *b, double *x, int32_t max_iter, double tol_scale,
                    int32_t relative_to_initial, int32_t replace_every, int32_t locked, const oracle_precond *pc,
                    const double *Pdiag, double *delta_out, double *tol_out, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
