"""Seeded input generators: determinism and the stated shapes and statistics."""
import numpy as np

from paper_1905_07622_amd import workloads as wl


def test_sphere_cube_geometry():
    p = wl.two_phase_sphere_cube()
    assert p.n_nodes == 4913 and p.n_elems == 4096
    assert (p.k_e == 10).sum() == 280 and np.all((p.k_e == 10) == (p.rhoc_e == 2))
    # no element centroid lies within 2.9e-3 (squared distance) of the sphere surface
    cx, cy, cz = wl.element_centroids(16, 16, 16, 1 / 16, 1 / 16, 1 / 16)
    d2 = (cx - 0.5) ** 2 + (cy - 0.5) ** 2 + (cz - 0.5) ** 2
    assert np.abs(d2 - 0.0625).min() > 2.9e-3


def test_lognormal_cube_statistics_and_determinism():
    a = wl.lognormal_cube(40, seed=2)
    b = wl.lognormal_cube(40, seed=2)
    c = wl.lognormal_cube(40, seed=3)
    assert np.array_equal(a.k_e, b.k_e) and not np.array_equal(a.k_e, c.k_e)
    z = np.log(a.k_e)
    assert abs(z.mean()) < 0.1 and abs(z.std() - 1.0) < 0.05
    z3 = z.reshape(40, 40, 40)
    corr1 = np.corrcoef(z3[:, :, :-1].ravel(), z3[:, :, 1:].ravel())[0, 1]
    corr4 = np.corrcoef(z3[:, :, :-4].ravel(), z3[:, :, 4:].ravel())[0, 1]
    assert corr1 > 0.5 and abs(corr4) < 0.1
    assert a.rhoc_e.min() >= 0.8 and a.rhoc_e.max() <= 1.2
    assert a.n_nodes == 41 ** 3


def test_full_size_configs_shapes():
    p = wl.lognormal_cube()
    assert p.n_nodes == 1_030_301 and p.theta == 0.5 and p.nsteps == 200
    s = wl.defect_slab()
    assert s.n_nodes == 201 * 201 * 26 and s.sensors.shape == (256, 3)
    assert np.isclose(s.nz * s.hz, 0.125) and s.flux_schedule[:10].sum() == 10
    assert s.flux_schedule[10:].sum() == 0
    assert set(np.unique(s.k_e)) <= {0.01, 1.0, 5.0} and (s.k_e == 0.01).any()


def test_proposals_and_requests_are_seeded():
    p0, p0b, p1 = wl.sphere_proposal(0), wl.sphere_proposal(0), wl.sphere_proposal(1)
    assert np.array_equal(p0.k_e, p0b.k_e) and not np.array_equal(p0.k_e, p1.k_e)
    k = p0.k_e
    frac = (k != 1.0).mean()
    assert 0.05 <= frac <= 0.6 and 2 <= k.max() <= 50
    r = [wl.serve_request(i) for i in range(12)]
    assert all(x.nx in wl.SERVE_EDGES and 50 <= x.nsteps <= 300 and x.theta in (0.5, 1.0) for x in r)
    t = wl.poisson_arrivals(1000, rate=10.0)
    assert np.all(np.diff(t) > 0) and abs(1000 / t[-1] - 10.0) < 1.0
