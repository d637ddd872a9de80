"""Pins for the oracle's six-tetrahedron element (the paper's element, Sec. 4.1).

Every box of the fixed grid is split into six linear tetrahedra around its
0-7 diagonal (tetrahedron 0, e_i, e_i + e_j, 7 for each order of the axes).
The oracle integrates their matrices by quadrature; these tests pin it to the
closed forms of the linear tetrahedron written here (M_t = V/20 (1 + delta_ij),
K_t = V grad l_i . grad l_j), to the assembled stencil that split is known to
give (on cubes, h times the 7-point Laplacian), to a dense brute-force
assembly, to invariants, to exact reproduction of linear fields, and to whole
runs with exact answers (layered steady state, energy balance, uniform fields).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle
from paper_1905_07622_amd import workloads as wl


def kuhn_tets():
    out = []
    for perm in itertools.permutations(range(3)):
        a, v = 0, [0]
        for ax in perm:
            a |= 1 << ax
            v.append(a)
        out.append(v)
    return out


def closed_form_box(hx, hy, hz):
    h = np.array([hx, hy, hz])
    M = np.zeros((8, 8))
    K = np.zeros((8, 8))
    for t in kuhn_tets():
        X = np.array([[(a >> d) & 1 for d in range(3)] for a in t], dtype=float) * h
        E = (X[1:] - X[0]).T
        V = abs(np.linalg.det(E)) / 6
        Gi = np.linalg.inv(E)  # rows: gradients of l_1..l_3
        G = np.vstack([-Gi.sum(axis=0), Gi])
        idx = np.ix_(t, t)
        M[idx] += V / 20 * (np.ones((4, 4)) + np.eye(4))
        K[idx] += V * G @ G.T
    return M, K


def tet_problem(nx, ny, nz, seed, **kw):
    return wl.random_problem(nx, ny, nz, seed, **kw).replace(element=oracle.ELEM_TET6)


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.1, 0.1, 0.1), (0.3, 0.7, 1.9)])
def test_tet6_box_matrices_match_closed_form(h):
    M, K = oracle.tet6_matrices(*h)
    Mc, Kc = closed_form_box(*h)
    np.testing.assert_allclose(M, Mc, rtol=0, atol=1e-14 * np.abs(Mc).max())
    np.testing.assert_allclose(K, Kc, rtol=0, atol=1e-13 * np.abs(Kc).max())


def test_tet6_box_invariants():
    hx, hy, hz = 0.2, 0.5, 0.9
    M, K = oracle.tet6_matrices(hx, hy, hz)
    assert abs(M.sum() - hx * hy * hz) < 1e-15
    np.testing.assert_allclose(K @ np.ones(8), 0.0, atol=1e-13)
    np.testing.assert_allclose(M, M.T, atol=0)
    np.testing.assert_allclose(K, K.T, atol=1e-15)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-12 and ev[1] > 1e-3
    assert np.linalg.eigvalsh(M)[0] > 0
    # corner pairs joined by no tetrahedron edge do not couple
    for a, b in ((1, 6), (2, 5), (3, 4)):
        assert M[a, b] == 0 and K[a, b] == 0


def test_tet6_cube_stiffness_is_h_times_seven_point_laplacian():
    h = 0.125
    p = tet_problem(5, 4, 6, seed=1, hx=h, hy=h, hz=h)
    K = oracle.CSR(p.replace(k_e=np.ones(p.n_elems)), 0.0, 1.0).to_dense()
    i = 2 + 6 * (2 + 5 * 3)  # an interior node
    row = K[i]
    expect = np.zeros_like(row)
    expect[i] = 6 * h
    for off in (1, -1, 6, -6, 30, -30):
        expect[i + off] = -h
    np.testing.assert_allclose(row, expect, atol=1e-15)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (4, 3, 2)])
def test_tet6_csr_equals_element_loop_equals_dense(dims):
    p = tet_problem(*dims, seed=3, hx=0.3, hy=0.2, hz=0.4)
    Mc, Kc = closed_form_box(p.hx, p.hy, p.hz)
    N = p.n_nodes
    A = np.zeros((N, N))
    nx, ny = p.nx, p.ny
    for ez in range(p.nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                nodes = [(ex + (a & 1)) + (nx + 1) * ((ey + ((a >> 1) & 1)) + (ny + 1) * (ez + (a >> 2)))
                         for a in range(8)]
                A[np.ix_(nodes, nodes)] += 1.0 * p.rhoc_e[e] * Mc + 0.3 * p.k_e[e] * Kc
    x = wl.random_vector(N, 4)
    csr = oracle.operator_apply(p, 1.0, 0.3, x)
    loop = oracle.element_loop(p, 1.0, 0.3, x)
    np.testing.assert_allclose(csr, A @ x, atol=1e-13 * np.abs(A @ x).max())
    np.testing.assert_allclose(loop, A @ x, atol=1e-13 * np.abs(A @ x).max())


def test_tet6_stiffness_annihilates_linear_fields_inside():
    p = tet_problem(5, 4, 4, seed=5, hx=0.2, hy=0.3, hz=0.25)
    X, Y, Z = wl.node_coords(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz)
    T = (0.3 + 1.1 * X - 0.7 * Y + 2.0 * Z).ravel()
    KT = oracle.operator_apply(p.replace(k_e=np.ones(p.n_elems)), 0.0, 1.0, T).reshape(p.nz + 1, p.ny + 1, p.nx + 1)
    np.testing.assert_allclose(KT[1:-1, 1:-1, 1:-1], 0.0, atol=1e-13)


def test_tet6_face_loads():
    p = tet_problem(3, 2, 2, seed=6, hx=0.5, hy=0.25, hz=0.4, dirichlet_mask=0,
                    flux_mask=(1 << wl.FACE_ZM) | (1 << wl.FACE_XP), flux=[0, 2.0, 0, 0, 1.5, 0])
    F = oracle.load_vector(p).reshape(p.nz + 1, p.ny + 1, p.nx + 1)
    # z = 0 face: per face square, its (0,0) and (1,1) corners get q h_x h_y / 3, the others / 6
    q, a = 1.5, 0.5 * 0.25
    ref = np.zeros((p.ny + 1, p.nx + 1))
    for ey in range(p.ny):
        for ex in range(p.nx):
            ref[ey, ex] += q * a / 3
            ref[ey + 1, ex + 1] += q * a / 3
            ref[ey, ex + 1] += q * a / 6
            ref[ey + 1, ex] += q * a / 6
    xp = np.zeros((p.nz + 1, p.ny + 1))
    qx, ax = 2.0, 0.25 * 0.4  # +x face, in-face axes y (u) and z (v)
    for ez in range(p.nz):
        for ey in range(p.ny):
            xp[ez, ey] += qx * ax / 3
            xp[ez + 1, ey + 1] += qx * ax / 3
            xp[ez, ey + 1] += qx * ax / 6
            xp[ez + 1, ey] += qx * ax / 6
    full = np.zeros_like(F)
    full[0] += ref
    full[:, :, p.nx] += xp
    np.testing.assert_allclose(F, full, atol=1e-15)
    assert abs(F.sum() - (q * p.nx * p.hx * p.ny * p.hy + qx * p.ny * p.hy * p.nz * p.hz)) < 1e-14


def test_tet6_sensors_exact_for_linear_fields():
    p = tet_problem(4, 3, 5, seed=7, hx=0.25, hy=0.3, hz=0.2)
    X, Y, Z = wl.node_coords(p.nx, p.ny, p.nz, p.hx, p.hy, p.hz)
    f = lambda x, y, z: 0.5 - 1.2 * x + 0.4 * y + 3.0 * z
    T = f(X, Y, Z).ravel()
    rng = np.random.default_rng(8)
    pts = rng.uniform(0, 1, (50, 3)) * np.array([p.nx * p.hx, p.ny * p.hy, p.nz * p.hz])
    out = oracle.sensors(p, T, pts)
    np.testing.assert_allclose(out, f(pts[:, 0], pts[:, 1], pts[:, 2]), atol=1e-13)


def test_tet6_layered_steady_state():
    nx = ny = 3
    nz = 6
    h = 1.0 / nz
    kz = np.where(np.arange(nz) < 2, 1.0, 4.0)
    q = 0.8
    p = wl.Problem(name="layers", nx=nx, ny=ny, nz=nz, hx=h, hy=h, hz=h, k_e=np.repeat(kz, nx * ny),
                   rhoc_e=np.ones(nx * ny * nz), T0=np.zeros((nx + 1) * (ny + 1) * (nz + 1)), dt=1e8, theta=1.0,
                   nsteps=1, rtol=1e-14, dirichlet_mask=1 << wl.FACE_ZM, flux_mask=1 << wl.FACE_ZP,
                   flux=np.array([0, 0, 0, 0, 0, q]), element=oracle.ELEM_TET6)
    out = oracle.run(p)
    expect = q * np.concatenate([[0.0], np.cumsum(h / kz)])
    T = out["T_final"].reshape(nz + 1, ny + 1, nx + 1)
    for iz in range(nz + 1):
        np.testing.assert_allclose(T[iz], expect[iz], rtol=1e-6, atol=1e-9)


def test_tet6_energy_balance_and_uniform_field():
    q = 1.7
    p = tet_problem(5, 4, 3, seed=9, theta=0.5, dt=2e-3, nsteps=5, rtol=1e-13, dirichlet_mask=0,
                    flux_mask=1 << wl.FACE_ZP, flux=[0, 0, 0, 0, 0, q])
    out = oracle.run(p, save_every=1)
    Mass = oracle.CSR(p, 1.0, 0.0).to_dense()
    ones = np.ones(p.n_nodes)
    E0 = ones @ Mass @ p.T0
    area = p.nx * p.hx * p.ny * p.hy
    for n in range(p.nsteps):
        assert abs(ones @ Mass @ out["T_saved"][n] - (E0 + (n + 1) * p.dt * q * area)) < 1e-11
    u = oracle.run(p.replace(flux_mask=0, T0=np.full(p.n_nodes, 2.5)), save_every=1)
    np.testing.assert_allclose(u["T_saved"], 2.5, atol=1e-12)
