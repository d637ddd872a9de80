"""Pins for the oracle's stopping rule (Algorithm 1's loop condition, read as a
relative residual test; Sec. 5 runs use a relative residual tolerance).

The rule: the loop of one time step continues while delta = r^T P^-1 r exceeds
rtol^2 * delta_b, with delta_b = b^T P^-1 b over the free rows of the lifted
right-hand side (or rtol^2 * delta_0 for the "initial residual" variant).  The
oracle evaluates delta from its recursively updated residual; these tests
rebuild everything the rule depends on densely, from the closed-form element
blocks and face weights written here, and check the returned iterate against
the rule with its TRUE residual b - A x:

  * after the oracle's own count k the rule holds, and
  * after k - 1 iterations (same oracle, iteration-locked) it does not.

One time step is used, so the count of that step alone decides the field.  The
cases are chosen so that the plausible slips move the stopping iteration: a
non-zero Dirichlet value makes the lifting A_fD g large (delta_b on the
unlifted b, or with Dirichlet rows included, is then far off), and a rough
guess makes delta_0 differ from delta_b by orders of magnitude (a test
relative to the wrong reference stops far too early or too late).
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1905_07622_amd import workloads as wl


def _m1(h):
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


def _s1(h):
    return 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])


def dense_operator(p, cm, ck):
    """sum_e cm*rhoc_e*M_e + ck*k_e*K_e with the tensor-product blocks of
    1-D linear elements (corner a = ax + 2ay + 4az; kron puts z slowest)."""
    hx, hy, hz = p.hx, p.hy, p.hz
    M = np.kron(_m1(hz), np.kron(_m1(hy), _m1(hx)))
    K = (np.kron(_s1(hz), np.kron(_m1(hy), _m1(hx))) + np.kron(_m1(hz), np.kron(_s1(hy), _m1(hx)))
         + np.kron(_m1(hz), np.kron(_m1(hy), _s1(hx))))
    N = p.n_nodes
    A = np.zeros((N, N))
    px, py = p.nx + 1, p.ny + 1
    for ez in range(p.nz):
        for ey in range(p.ny):
            for ex in range(p.nx):
                e = ex + p.nx * (ey + p.ny * ez)
                idx = np.array([(ex + (a & 1)) + px * ((ey + ((a >> 1) & 1)) + py * (ez + (a >> 2)))
                                for a in range(8)])
                A[np.ix_(idx, idx)] += cm * p.rhoc_e[e] * M + ck * p.k_e[e] * K
    return A


def face_load(p):
    """F_i = sum over flux faces of q * (face element area / 4) * (face elements at i)."""
    F = np.zeros((p.nz + 1, p.ny + 1, p.nx + 1))
    n = (p.nx, p.ny, p.nz)
    h = (p.hx, p.hy, p.hz)
    for face in range(6):
        if not (p.flux_mask >> face) & 1:
            continue
        d = face >> 1
        u, v = (d + 1) % 3, (d + 2) % 3
        cu = np.full(n[u] + 1, 2.0)
        cu[0] = cu[-1] = 1.0
        cv = np.full(n[v] + 1, 2.0)
        cv[0] = cv[-1] = 1.0
        w = p.flux[face] * 0.25 * h[u] * h[v] * np.outer(cu, cv)  # [iu, iv]
        level = n[d] if face & 1 else 0
        # F indexed [z, y, x]; axis of coordinate c is 2 - c
        sl = [slice(None)] * 3
        sl[2 - d] = level
        block = F[tuple(sl)]  # remaining axes in order (z, y, x) minus d
        axes = [c for c in (2, 1, 0) if c != d]  # coordinates of block's axes
        ww = w if axes == [u, v] else w.T
        block += ww
    return F.ravel()


def dirichlet_nodes(p):
    """Mask and values; where faces meet, the lowest-numbered face sets the value."""
    Z, Y, X = np.meshgrid(np.arange(p.nz + 1), np.arange(p.ny + 1), np.arange(p.nx + 1), indexing="ij")
    on = [X == 0, X == p.nx, Y == 0, Y == p.ny, Z == 0, Z == p.nz]
    mask = np.zeros(Z.shape, dtype=bool)
    val = np.zeros(Z.shape)
    for f in range(6):
        if (p.dirichlet_mask >> f) & 1:
            new = on[f] & ~mask
            val[new] = p.dirichlet_value[f]
            mask |= on[f]
    return mask.ravel(), val.ravel()


def step_system(p, T0):
    """Lifted system of the first step: A_ff x_f = bhat_f, its Jacobi diagonal,
    and the Dirichlet data."""
    A = dense_operator(p, 1.0, p.theta * p.dt)
    L = dense_operator(p, 1.0, -(1.0 - p.theta) * p.dt)
    s1 = 1.0 if p.flux_schedule is None else float(p.flux_schedule[0])
    dmask, g = dirichlet_nodes(p)
    T = np.where(dmask, g, T0)
    b = L @ T + p.dt * s1 * face_load(p)
    f = ~dmask
    bhat = b[f] - A[np.ix_(f, dmask)] @ g[dmask]
    Aff = A[np.ix_(f, f)]
    return Aff, bhat, np.diag(Aff).copy(), f, g, T


def pnorm2(r, P):
    return float(r @ (r / P))


def make_case(seed, *, g0, prev_noise, dt):
    """One step from a smooth T0; the field "before" T0 is T0 plus noise of
    amplitude prev_noise, so the extrapolated guess 2 T0 - T_prev is as far
    from the solution as that noise."""
    rng = np.random.default_rng(seed)
    p = wl.random_problem(5, 4, 6, seed=seed, theta=0.5, dt=dt, nsteps=1, rtol=1e-6,
                          dirichlet_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP),
                          dirichlet_value=[0, 0.5, 0, 0, g0, 0],
                          flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, 2.0])
    X, Y, Z = wl.node_coords(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz)
    T0 = (1.0 + np.cos(2.0 * X) * np.sin(1.5 * Y + 0.3) * (0.5 + Z)).ravel()
    T_prev = T0 + prev_noise * rng.standard_normal(p.n_nodes)
    return p.replace(T0=T0), T_prev


def first_guess(p, T_prev, f, g):
    """x0 = 2 T0 - T_prev (Dirichlet values imposed on both fields first)."""
    T1 = np.where(f, p.T0, g)
    T2 = np.where(f, T_prev, g)
    return 2.0 * T1 - T2


CASES = [(41, 5.0, 0.0, 1e-3), (42, 5.0, 10.0, 4e-2), (43, -2.0, 10.0, 4e-2), (47, 0.0, 10.0, 4e-2),
         (48, 0.0, 0.0, 1e-3)]


@pytest.mark.parametrize("seed,g0,prev_noise,dt", CASES)
def test_stop_rule_rhs_reference_true_residual(seed, g0, prev_noise, dt):
    p, T_prev = make_case(seed, g0=g0, prev_noise=prev_noise, dt=dt)
    Aff, bhat, P, f, g, T = step_system(p, p.T0)
    delta_b = pnorm2(bhat, P)
    x0 = first_guess(p, T_prev, f, g)
    delta_0 = pnorm2(bhat - Aff @ x0[f], P)
    # precondition for the test's power: a test relative to delta_0 would
    # stop at a clearly different iteration
    assert delta_0 / delta_b > 30 or delta_0 / delta_b < 1 / 30, delta_0 / delta_b
    out = oracle.run(p, T_prev=T_prev)
    k = int(out["iters"][0])
    assert out["status"] == 0 and k >= 2
    x = out["T_final"]
    r = bhat - Aff @ x[f]
    ratio = pnorm2(r, P) / delta_b
    assert ratio <= p.rtol ** 2 * (1 + 1e-6), (k, ratio)
    # the relative residual the oracle reports is this ratio's square root
    assert abs(out["relres"][0] - np.sqrt(ratio)) <= 1e-6 * p.rtol
    # one iteration fewer does not meet the rule
    prev = oracle.run(p, T_prev=T_prev, locked_iters=[k - 1])
    rp = bhat - Aff @ prev["T_final"][f]
    assert pnorm2(rp, P) / delta_b > p.rtol ** 2, k
    # Dirichlet values are held exactly
    assert np.array_equal(x[~f], g[~f])


@pytest.mark.parametrize("seed,g0,prev_noise,dt", CASES)
def test_stop_rule_initial_reference_true_residual(seed, g0, prev_noise, dt):
    p, T_prev = make_case(seed, g0=g0, prev_noise=prev_noise, dt=dt)
    Aff, bhat, P, f, g, T = step_system(p, p.T0)
    x0 = first_guess(p, T_prev, f, g)
    delta_0 = pnorm2(bhat - Aff @ x0[f], P)
    out = oracle.run(p, T_prev=T_prev, stop_rule=oracle.STOP_INITIAL)
    k = int(out["iters"][0])
    assert out["status"] == 0 and k >= 2
    r = bhat - Aff @ out["T_final"][f]
    assert pnorm2(r, P) / delta_0 <= p.rtol ** 2 * (1 + 1e-6)
    prev = oracle.run(p, T_prev=T_prev, stop_rule=oracle.STOP_INITIAL, locked_iters=[k - 1])
    rp = bhat - Aff @ prev["T_final"][f]
    assert pnorm2(rp, P) / delta_0 > p.rtol ** 2


def test_stop_rule_zero_rhs_gives_zero_free_field_without_iterations():
    # T0 = 0, no flux, zero Dirichlet value: b = 0, so delta_b = 0 and the free
    # part of the solution is exactly 0 after no iterations
    p = wl.random_problem(4, 3, 3, seed=46, nsteps=2, rtol=1e-8).replace(T0=np.zeros(80))
    out = oracle.run(p)
    assert out["status"] == 0 and np.all(out["iters"] == 0)
    assert np.all(out["T_final"] == 0.0)


def test_face_load_helper_matches_area():
    # the helper itself: the loads of a face sum to q * area (A.5 of the derivation)
    p, _ = make_case(41, g0=5.0, prev_noise=0.0, dt=1e-3)
    assert abs(face_load(p).sum() - 2.0 * p.nx * p.hx * p.ny * p.hy) < 1e-14
    F = oracle.load_vector(p)
    np.testing.assert_allclose(face_load(p), F, rtol=0, atol=1e-15)
