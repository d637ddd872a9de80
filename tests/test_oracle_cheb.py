"""Pins for the oracle's Chebyshev-accelerated Jacobi preconditioner.

The preconditioner is not in the paper (its GPU method uses Jacobi only,
Sec. 3.3); it is the polynomial kind a matrix-free GPU path can apply with the
same element-wise operator.  M^-1 = q(D^-1 A) D^-1 with 1 - lambda q(lambda) the
Chebyshev polynomial of degree m on [lo, hi], scaled to 1 at lambda = 0.  The
oracle applies it by the three-term Chebyshev iteration; these tests pin it
to things it does not compute that way:

* the closed form: q evaluated on the eigenvalues of D^-1/2 A D^-1/2 from a
  dense eigendecomposition (numpy), with T_m(x) = cos(m arccos x) or
  cosh(m arccosh x);
* the interval bound: hi >= the largest eigenvalue of D^-1 A for any
  coefficients, equal to 27/8 (the constant mode of the trilinear mass block)
  on a single cubic element without stiffness, and to 3/2 for the stiffness
  block alone (the tensor-product modes of the 1-D blocks);
* M^-1 symmetric positive definite (built column by column);
* PCG with it solves the system (dense solve), in fewer iterations than with
  Jacobi on a stiff problem; degree 1 is Jacobi up to a scale, which leaves
  the CG iterates unchanged;
* whole runs keep the exact discrete decay of a separable mode.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1905_07622_amd import workloads as wl


def cheb_T(m, x):
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


def closed_form_minv(A, m, lo, hi):
    d = np.diag(A)
    S = A / np.sqrt(np.outer(d, d))
    lam, V = np.linalg.eigh(S)
    c, w = (hi + lo) / 2, (hi - lo) / 2
    resid = cheb_T(m, (c - lam) / w) / cheb_T(m, np.array([c / w]))[0]
    q = (1.0 - resid) / lam
    Dm = np.diag(1.0 / np.sqrt(d))
    return Dm @ V @ np.diag(q) @ V.T @ Dm


@pytest.mark.parametrize("m", [2, 3, 5])
@pytest.mark.parametrize("ck", [1e-3, 0.3])
def test_cheb_apply_equals_closed_form_polynomial(m, ck):
    prob = wl.random_problem(4, 3, 5, seed=61, hx=0.2, hy=0.3, hz=0.25)
    A = oracle.CSR(prob, 1.0, ck)
    D = A.to_dense()
    hi = oracle.cheb_upper(prob.hx, prob.hy, prob.hz)
    lo = hi / 20.0
    r = wl.random_vector(prob.n_nodes, 62)
    s = A.cheb_apply(r, m, lo, hi)
    ref = closed_form_minv(D, m, lo, hi) @ r
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("h", [(0.1, 0.1, 0.1), (0.3, 0.7, 1.9), (0.05, 0.2, 0.1)])
def test_cheb_upper_bounds_the_spectrum_for_any_coefficients(h):
    hi = oracle.cheb_upper(*h)
    for seed, ck in ((63, 1e-4), (64, 1e-1), (65, 10.0)):
        prob = wl.random_problem(3, 4, 3, seed=seed, hx=h[0], hy=h[1], hz=h[2], k_range=(1e-3, 1e3),
                                 rhoc_range=(1e-2, 1e2))
        D = oracle.CSR(prob, 1.0, ck).to_dense()
        d = np.diag(D)
        top = np.linalg.eigvalsh(D / np.sqrt(np.outer(d, d)))[-1]
        assert top <= hi * (1 + 1e-12), (top, hi)


def test_cheb_upper_closed_forms_on_one_element():
    # cubic box: mass block D_M^-1 M has top eigenvalue 27/8 (constant mode);
    # stiffness block D_K^-1 K has 3/2 (one axis odd, two even: (2/h)(h/2)^2 / (h/3))
    assert abs(oracle.cheb_upper(0.4, 0.4, 0.4) - 27.0 / 8.0) < 1e-12
    M, K = oracle.element_matrices(0.4, 0.4, 0.4)
    top_k = np.linalg.eigvalsh(K / np.sqrt(np.outer(np.diag(K), np.diag(K))))[-1]
    assert abs(top_k - 1.5) < 1e-12
    # a single element with mass only attains the bound
    prob = wl.random_problem(1, 1, 1, seed=66, hx=0.4, hy=0.4, hz=0.4, dirichlet_mask=0)
    D = oracle.CSR(prob, 1.0, 0.0).to_dense()
    d = np.diag(D)
    assert abs(np.linalg.eigvalsh(D / np.sqrt(np.outer(d, d)))[-1] - 27.0 / 8.0) < 1e-12


def test_cheb_preconditioner_is_symmetric_positive_definite():
    prob = wl.random_problem(3, 3, 3, seed=67, k_range=(1e-2, 1e2))
    A = oracle.CSR(prob, 1.0, 0.05)
    hi = oracle.cheb_upper(prob.hx, prob.hy, prob.hz)
    Minv = np.column_stack([A.cheb_apply(e, 4, hi / 30, hi) for e in np.eye(prob.n_nodes)])
    np.testing.assert_allclose(Minv, Minv.T, atol=1e-12 * np.abs(Minv).max())
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T))[0] > 0


def test_pcg_cheb_solves_and_needs_fewer_iterations():
    prob = wl.lognormal_cube(10, seed=68, nsteps=1)
    A = oracle.CSR(prob, 1.0, 0.5)  # stiff: theta dt k / h^2 ~ 50
    b = wl.random_vector(prob.n_nodes, 69)
    ref = np.linalg.solve(A.to_dense(), b)
    hi = oracle.cheb_upper(prob.hx, prob.hy, prob.hz)
    xj, ij, _ = A.pcg(b, np.zeros_like(b), tol=1e-26, replace_every=0)
    xc, ic, _ = A.pcg_cheb(b, np.zeros_like(b), degree=4, lo=hi / 30, hi=hi, tol=1e-26, replace_every=0)
    np.testing.assert_allclose(xc, ref, atol=1e-10 * np.abs(ref).max())
    np.testing.assert_allclose(xj, ref, atol=1e-10 * np.abs(ref).max())
    assert ic < ij / 2, (ic, ij)


def test_degree_one_is_scaled_jacobi_with_the_same_iterates():
    prob = wl.random_problem(5, 4, 4, seed=70)
    A = oracle.CSR(prob, 1.0, 0.02)
    b = wl.random_vector(prob.n_nodes, 71)
    hi = oracle.cheb_upper(prob.hx, prob.hy, prob.hz)
    for n in (3, 7):
        xj, _, _ = A.pcg(b, np.zeros_like(b), locked=n, replace_every=0)
        xc, _, _ = A.pcg_cheb(b, np.zeros_like(b), degree=1, lo=hi / 10, hi=hi, locked=n, replace_every=0)
        np.testing.assert_allclose(xc, xj, atol=1e-13 * np.abs(xj).max())


@pytest.mark.parametrize("theta,dt", [(1.0, 1e-2), (0.5, 5e-3)])
def test_cheb_runs_keep_exact_discrete_mode_decay(theta, dt):
    from test_oracle_solver import mode_problem
    prob, g = mode_problem(6, 5, 7, 1 / 6, 0.2, 1 / 7, 1, 2, 1, theta, dt)
    out = oracle.run(prob, save_every=1, max_iter=2000, precond=oracle.PRECOND_CHEBYSHEV, cheb_degree=3)
    assert out["status"] == 0
    for n in range(prob.nsteps):
        np.testing.assert_allclose(out["T_saved"][n], g ** (n + 1) * prob.T0, atol=1e-11 * np.abs(prob.T0).max())


def test_cheb_run_matches_jacobi_run_and_counts_drop():
    prob = wl.lognormal_cube(12, seed=72, nsteps=3).replace(dt=5e-2, theta=1.0, rtol=1e-10)
    j = oracle.run(prob, save_every=1)
    c = oracle.run(prob, save_every=1, precond=oracle.PRECOND_CHEBYSHEV, cheb_degree=3, cheb_ratio=30.0)
    assert j["status"] == 0 and c["status"] == 0
    for n in range(prob.nsteps):
        assert np.linalg.norm(c["T_saved"][n] - j["T_saved"][n]) <= 1e-8 * np.linalg.norm(j["T_saved"][n])
    assert c["iters"].sum() < j["iters"].sum()
    bad = oracle.run(prob, precond=oracle.PRECOND_CHEBYSHEV, cheb_degree=1)
    assert bad["status"] == oracle.EINVAL
