"""Pins for the oracle's element matrices and assembled operators.

The oracle integrates the trilinear-hexahedron matrices by Gauss quadrature
(Sec. 3.2).  These tests pin it to the independent tensor-product closed form
of linear 1-D elements, to invariants of the mass and stiffness operators, and
to a brute-force dense assembly written here from the closed form.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle
from paper_1905_07622_amd import workloads as wl


def m1(h):
    return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])


def s1(h):
    return 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])


def closed_form(hx, hy, hz):
    """M = m_z (x) m_y (x) m_x and K = s_z m_y m_x + m_z s_y m_x + m_z m_y s_x for
    local corner a = ax + 2 ay + 4 az (kron puts z slowest)."""
    M = np.kron(m1(hz), np.kron(m1(hy), m1(hx)))
    K = (np.kron(s1(hz), np.kron(m1(hy), m1(hx))) + np.kron(m1(hz), np.kron(s1(hy), m1(hx)))
         + np.kron(m1(hz), np.kron(m1(hy), s1(hx))))
    return M, K


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.01, 0.01, 0.01), (0.3, 0.7, 1.9)])
def test_element_matrices_match_tensor_closed_form(h):
    M, K = oracle.element_matrices(*h)
    Mc, Kc = closed_form(*h)
    np.testing.assert_allclose(M, Mc, rtol=1e-14, atol=1e-14 * np.abs(Mc).max())
    np.testing.assert_allclose(K, Kc, rtol=1e-14, atol=1e-14 * np.abs(Kc).max())


def test_cubic_element_entries_by_hamming_distance():
    # cubic h: M = h^3/216 {8,4,2,1}, K = h/12 {4,0,-1,-1} by popcount(a^b)
    h = 0.25
    M, K = oracle.element_matrices(h, h, h)
    mv = np.array([8, 4, 2, 1]) * h ** 3 / 216
    kv = np.array([4, 0, -1, -1]) * h / 12
    for a, b in itertools.product(range(8), repeat=2):
        d = bin(a ^ b).count("1")
        assert abs(M[a, b] - mv[d]) < 1e-16
        assert abs(K[a, b] - kv[d]) < 1e-15


def test_element_matrix_invariants():
    hx, hy, hz = 0.2, 0.5, 0.9
    M, K = oracle.element_matrices(hx, hy, hz)
    assert abs(M.sum() - hx * hy * hz) < 1e-15          # sum M = volume
    np.testing.assert_allclose(K @ np.ones(8), 0.0, atol=1e-13)  # constants in the kernel of K
    np.testing.assert_allclose(M, M.T, atol=0)
    np.testing.assert_allclose(K, K.T, atol=0)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-12 and ev[1] > 1e-3           # PSD, one-dimensional kernel
    assert np.linalg.eigvalsh(M)[0] > 0                  # SPD


def dense_bruteforce(prob, cm, ck):
    """Dense assembly written from the closed form with explicit loops."""
    Mc, Kc = closed_form(prob.hx, prob.hy, prob.hz)
    N = prob.n_nodes
    A = np.zeros((N, N))
    nx, ny = prob.nx, prob.ny
    for ez in range(prob.nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                nodes = [(ex + (a & 1)) + (nx + 1) * ((ey + ((a >> 1) & 1)) + (ny + 1) * (ez + (a >> 2)))
                         for a in range(8)]
                Ae = cm * prob.rhoc_e[e] * Mc + ck * prob.k_e[e] * Kc
                for a in range(8):
                    for b in range(8):
                        A[nodes[a], nodes[b]] += Ae[a, b]
    return A


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (5, 4, 3)])
def test_csr_equals_element_loop_equals_dense(dims):
    prob = wl.random_problem(*dims, seed=11, hx=0.3, hy=0.2, hz=0.45)
    cm, ck = 1.0, 0.37
    D = dense_bruteforce(prob, cm, ck)
    A = oracle.CSR(prob, cm, ck)
    np.testing.assert_allclose(A.to_dense(), D, rtol=1e-14, atol=1e-15 * np.abs(D).max())
    x = wl.random_vector(prob.n_nodes, 5)
    y_ref = D @ x
    scale = np.abs(y_ref).max()
    np.testing.assert_allclose(A.matvec(x), y_ref, atol=1e-14 * scale)
    np.testing.assert_allclose(oracle.element_loop(prob, cm, ck, x), y_ref, atol=1e-14 * scale)
    # same operator with a negative stiffness scale (the right-hand operator L)
    np.testing.assert_allclose(oracle.operator_apply(prob, 1.0, -0.6, x),
                               dense_bruteforce(prob, 1.0, -0.6) @ x, atol=1e-13 * scale)


def test_assembled_stiffness_annihilates_constants_and_mass_sums_to_weighted_volume():
    prob = wl.random_problem(4, 3, 5, seed=3)
    K = oracle.CSR(prob, 0.0, 1.0)
    np.testing.assert_allclose(K.matvec(np.ones(prob.n_nodes)), 0.0, atol=1e-12)
    M = oracle.CSR(prob, 1.0, 0.0)
    vol = prob.hx * prob.hy * prob.hz
    assert abs(M.matvec(np.ones(prob.n_nodes)).sum() - prob.rhoc_e.sum() * vol) < 1e-13


def test_assembled_operator_symmetric_positive_definite():
    prob = wl.random_problem(3, 2, 3, seed=7, zero_k_fraction=0.3)
    A = oracle.CSR(prob, 1.0, 0.8).to_dense()
    np.testing.assert_allclose(A, A.T, atol=0)
    np.linalg.cholesky(A)  # raises if not SPD
    K = oracle.CSR(prob, 0.0, 1.0).to_dense()
    assert np.linalg.eigvalsh(K)[0] > -1e-12


def test_homogeneous_interior_stencil():
    # interior node of a homogeneous cubic grid: the neighbour shares 8/4/2/1 elements
    n, h = 4, 0.5
    prob = wl.random_problem(n, n, n, seed=0).replace(
        hx=h, hy=h, hz=h, k_e=np.ones(n ** 3), rhoc_e=np.ones(n ** 3))
    K = oracle.CSR(prob, 0.0, 1.0).to_dense()
    M = oracle.CSR(prob, 1.0, 0.0).to_dense()
    i = 2 + 5 * (2 + 5 * 2)
    kv = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}
    mv = {0: 8 * h ** 3 / 27, 1: 2 * h ** 3 / 27, 2: h ** 3 / 54, 3: h ** 3 / 216}
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        j = (2 + dx) + 5 * ((2 + dy) + 5 * (2 + dz))
        c = abs(dx) + abs(dy) + abs(dz)
        assert abs(K[i, j] - kv[c]) < 1e-14
        assert abs(M[i, j] - mv[c]) < 1e-15
    assert abs(K[i].sum()) < 1e-13 and abs(M[i].sum() - h ** 3) < 1e-15


def test_load_vector_face_weights():
    n = 4
    h = 0.25
    q = 2.5
    prob = wl.random_problem(n, n, n, seed=1).replace(flux_mask=1 << wl.FACE_ZP, dirichlet_mask=0,
                                                       flux=np.array([0, 0, 0, 0, 0, q]))
    F = oracle.load_vector(prob).reshape(n + 1, n + 1, n + 1)
    assert abs(F.sum() - q * 1.0) < 1e-14            # sum F = q * face area
    top = F[n]
    assert np.all(F[:n] == 0)
    assert abs(top[2, 2] - q * h * h) < 1e-15          # interior face node
    assert abs(top[0, 2] - q * h * h / 2) < 1e-15      # face edge
    assert abs(top[0, 0] - q * h * h / 4) < 1e-15      # face corner


def test_load_vector_every_face():
    prob = wl.random_problem(3, 4, 2, seed=1, hx=0.2, hy=0.3, hz=0.5).replace(
        dirichlet_mask=0, flux_mask=0b111111, flux=np.arange(1.0, 7.0))
    F = oracle.load_vector(prob)
    lx, ly, lz = 3 * 0.2, 4 * 0.3, 2 * 0.5
    areas = [ly * lz, ly * lz, lx * lz, lx * lz, lx * ly, lx * ly]
    assert abs(F.sum() - sum(q * a for q, a in zip(range(1, 7), areas))) < 1e-13


def test_dirichlet_mask_counts():
    prob = wl.two_phase_sphere_cube()
    d, g = oracle.dirichlet(prob)
    assert d.sum() == 17 * 17 and np.all(g == 0)
    d3 = d.reshape(17, 17, 17)
    assert d3[0].all() and not d3[1:].any()


def test_sensor_interpolation_exact_for_trilinear_fields():
    prob = wl.random_problem(3, 5, 4, seed=2, hx=0.3, hy=0.2, hz=0.25)
    X, Y, Z = wl.node_coords(prob.nx, prob.ny, prob.nz, prob.hx, prob.hy, prob.hz)

    def f(x, y, z):
        return 0.3 + 1.5 * x - 2 * y + 0.7 * z + 0.4 * x * y - 1.1 * y * z + 0.9 * x * y * z

    # globally trilinear only within each element; a product of linear
    # functions is trilinear on every element, so nodal interpolation is exact
    T = f(X, Y, Z).ravel()
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 1, (50, 3)) * np.array([0.9, 1.0, 1.0])
    pts = np.vstack([pts, [[0.3, 0.2, 0.25], [0.0, 0.0, 0.0], [0.9, 1.0, 1.0]]])
    np.testing.assert_allclose(oracle.sensors(prob, T, pts), f(*pts.T), atol=1e-13)
