"""The coefficient-inverse sampler (Section 5.4) without a GPU.

Pins of the reference (oracle/inverse_ref.py):
  * the per-pixel likelihood of the camera model (Gaussian noise, then
    rounding to the nearest q) against direct quadrature of the normal density
    over the rounding bin, centre and both tails;
  * the Metropolis-Hastings step against a posterior known in closed form: a
    Gaussian log-likelihood in theta under a wide uniform prior, whose long
    chains must reproduce its mean and standard deviation (a wrong acceptance
    ratio, sign or prior test biases them).
Host logic of the driver (paper_1905_07622_amd/inverse.py) against the pinned
reference: the same log-likelihoods, and bit-identical chains for the same
draws and likelihood.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import inverse_ref as ref
from paper_1905_07622_amd import inverse as inv
from paper_1905_07622_amd import workloads as wl


@pytest.mark.parametrize("m,o", [(5.0, 5.0), (5.0, 5.1), (5.03, 4.9), (1.0, 1.5), (2.0, 1.4), (0.0, 0.3)])
def test_reference_pixel_likelihood_matches_quadrature(m, o):
    sigma, q = 0.1, 0.1
    p, _ = integrate.quad(lambda t: math.exp(-0.5 * ((t - m) / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi)),
                          o - q / 2, o + q / 2, epsabs=0, epsrel=1e-13)
    assert ref.bin_log_prob(m, o, sigma, q) == pytest.approx(math.log(p), rel=1e-10, abs=1e-10)


def test_reference_pixel_likelihood_sums_to_one_over_bins():
    """The bins of all observable values partition the line: their probabilities add to 1."""
    m, sigma, q = 3.04, 0.1, 0.1
    total = sum(math.exp(ref.bin_log_prob(m, round(k * q, 10), sigma, q)) for k in range(20, 41))
    assert total == pytest.approx(1.0, abs=1e-12)


def test_reference_sampler_reproduces_a_known_posterior():
    mu, s = 0.3, 0.05  # posterior N(mu, s^2) (prior [-10, 10] is flat over it)
    normals, uniforms = wl.mh_draws(11, 20000, 4)
    out = ref.metropolis([0.0, 0.1, 0.5, 0.9], normals, uniforms, 0.08,
                         lambda th: [-0.5 * ((t - mu) / s) ** 2 for t in th], -10.0, 10.0)
    x = np.array(out["samples"][2000:]).ravel()
    assert x.mean() == pytest.approx(mu, abs=0.006)
    assert x.std() == pytest.approx(s, rel=0.06)
    rate = np.mean(out["accepted"])
    assert 0.2 < rate < 0.9


def test_reference_sampler_respects_the_prior():
    normals, uniforms = wl.mh_draws(12, 3000, 2)
    out = ref.metropolis([0.05, 0.95], normals, uniforms, 0.3, lambda th: [0.0] * len(th), 0.0, 1.0)
    x = np.array(out["samples"])
    assert x.min() >= 0.0 and x.max() <= 1.0
    # a flat likelihood inside the prior: every candidate inside is accepted, none outside
    for i, row in enumerate(out["accepted"]):
        for c, ok in enumerate(row):
            cand = out["samples"][i][c] + 0.3 * normals[i][c]
            assert ok == (0.0 <= cand <= 1.0)


def test_driver_likelihood_matches_reference():
    rng = np.random.Generator(np.random.PCG64(5))
    pred = rng.uniform(4.0, 6.0, 200)
    obs = inv.camera(pred + rng.uniform(-0.4, 0.4, 200), wl.camera_noise(3, 200))
    got = inv.log_likelihood(pred, obs)
    want = ref.log_likelihood(pred, obs)
    assert got == pytest.approx(want, rel=1e-12)
    assert np.allclose(np.round(obs / 0.1) * 0.1, obs, rtol=0, atol=1e-12)  # rounded to the quantum


def test_driver_chain_is_the_reference_chain():
    normals, uniforms = wl.mh_draws(13, 400, 3)

    def ll(th):
        return [-0.5 * ((t - 0.2) / 0.07) ** 2 + 0.1 * math.sin(40 * t) for t in th]

    a = inv.metropolis([0.1, 0.2, 0.3], normals, uniforms, 0.05, lambda th: np.array(ll(th)), 0.0, 0.5)
    b = ref.metropolis([0.1, 0.2, 0.3], normals, uniforms, 0.05, ll, 0.0, 0.5)
    assert np.array_equal(a["samples"], np.array(b["samples"]))
    assert np.array_equal(a["accepted"], np.array(b["accepted"]))
    assert np.array_equal(a["proposed"], np.array(b["proposed"]))
    assert a["evaluated"] == b["evaluated"]


def test_corroded_plate_is_continuous_in_depth():
    """Element coefficients move continuously with the depth (share of each element's
    z-extent below the channel profile), and the plate is intact at depth 0."""
    p0 = wl.corroded_plate(0.0)
    assert np.all(p0.k_e == 1.0)
    a, b = wl.corroded_plate(0.03), wl.corroded_plate(0.03 + 1e-6)
    assert 0 < np.abs(a.k_e - b.k_e).max() < 1e-3
