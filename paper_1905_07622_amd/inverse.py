"""Coefficient-inverse driver (paper Section 5.4): Metropolis-Hastings over a
defect's penetration depth, every proposal a forward solve through the batched
path (fem_heat_run_batch), several chains advancing together so that each
iteration is one batched launch sequence.

Camera model: i.i.d. Gaussian pixel noise (sigma = 0.1) then rounding to the
nearest 0.1 (Section 5.4).  The likelihood of an observed frame D given a
predicted frame m is therefore the probability that each noisy pixel landed in
its observed rounding bin, prod_p [Phi((o_p + q/2 - m_p)/sigma) -
Phi((o_p - q/2 - m_p)/sigma)]; it is evaluated in log form, each factor in the
tail where it does not cancel.  The prior is uniform on [lo, hi]; a candidate
theta_hat = theta + s*xi is accepted with probability
min(1, p(D|theta_hat)/p(D|theta)) and one outside the prior is rejected without
a solve.  The random numbers come in as arguments.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np
from scipy.special import log_ndtr

SIGMA = 0.1
QUANTUM = 0.1


def camera(frame: np.ndarray, noise: np.ndarray, sigma: float = SIGMA, quantum: float = QUANTUM) -> np.ndarray:
    """An observed frame: the predicted one plus sigma * noise, rounded to the nearest quantum."""
    return np.round((np.asarray(frame) + sigma * np.asarray(noise)) / quantum) * quantum


def pixel_log_prob(pred, observed, sigma: float = SIGMA, quantum: float = QUANTUM) -> np.ndarray:
    """log p(o | m) per pixel.  For a bin above the mean the two normal CDFs are near 1 and would
    cancel, so the mirrored bin of the upper tail is used there."""
    m = np.asarray(pred, dtype=np.float64)
    o = np.asarray(observed, dtype=np.float64)
    a = (o - 0.5 * quantum - m) / sigma
    b = (o + 0.5 * quantum - m) / sigma
    up = a > 0.0
    lo_ = np.where(up, -b, a)
    hi_ = np.where(up, -a, b)
    lh = log_ndtr(hi_)
    return lh + np.log1p(-np.exp(log_ndtr(lo_) - lh))


def log_likelihood(pred, observed, sigma: float = SIGMA, quantum: float = QUANTUM) -> float:
    return float(np.sum(pixel_log_prob(pred, observed, sigma, quantum)))


def metropolis(theta0: Sequence[float], normals: np.ndarray, uniforms: np.ndarray, scale: float,
               loglik: Callable[[np.ndarray], np.ndarray], lo: float, hi: float) -> dict:
    """Chains side by side.  loglik(thetas) -> log-likelihoods of those thetas (one call per
    iteration, for the candidates inside the prior).  normals, uniforms: (n_iter, n_chains).
    Returns samples and log-likelihoods (n_iter + 1, n_chains), accept flags and the candidates'
    log-likelihoods (-inf outside the prior; n_iter, n_chains) and the number of likelihood
    evaluations (forward solves)."""
    theta = np.array(theta0, dtype=np.float64)
    cur = np.asarray(loglik(theta), dtype=np.float64).copy()
    n_iter, K = np.shape(normals)
    samples = np.empty((n_iter + 1, K))
    logls = np.empty((n_iter + 1, K))
    accepted = np.zeros((n_iter, K), dtype=bool)
    proposed = np.full((n_iter, K), -np.inf)
    samples[0], logls[0] = theta, cur
    evaluated = K
    for i in range(n_iter):
        prop = theta + scale * np.asarray(normals[i], dtype=np.float64)
        inside = np.flatnonzero((prop >= lo) & (prop <= hi))
        new = np.full(K, -np.inf)
        if inside.size:
            new[inside] = np.asarray(loglik(prop[inside]), dtype=np.float64)
            evaluated += inside.size
        ok = np.zeros(K, dtype=bool)
        ok[inside] = np.log(np.asarray(uniforms[i], dtype=np.float64)[inside]) < new[inside] - cur[inside]
        theta = np.where(ok, prop, theta)
        cur = np.where(ok, new, cur)
        accepted[i] = ok
        proposed[i] = new
        samples[i + 1], logls[i + 1] = theta, cur
    return {"samples": samples, "loglik": logls, "accepted": accepted, "proposed": proposed,
            "evaluated": int(evaluated)}


def batched_frames(make_problem: Callable[[float], object], **run_kw) -> Callable[[np.ndarray], np.ndarray]:
    """A forward model for the sampler: the camera frames (field at the pixel points after the last
    step) of the problems make_problem(theta) for all thetas, in one fem_heat_run_batch call."""
    from . import femheat as fh

    def frames(thetas: np.ndarray) -> np.ndarray:
        probs = [make_problem(float(t)) for t in thetas]
        st, res = fh.run_batch(probs, sensors=True, **run_kw)
        if st != fh.FEM_OK:
            raise fh.FemError(st, "forward solves of the proposals failed")
        return np.stack([np.asarray(r["traces"])[-1] for r in res])

    return frames


def likelihood_of(frames: Callable[[np.ndarray], np.ndarray], observed: np.ndarray,
                  sigma: float = SIGMA, quantum: float = QUANTUM) -> Callable[[np.ndarray], np.ndarray]:
    """loglik(thetas) for the sampler from a batched forward model and the observed frame."""
    def loglik(thetas: np.ndarray) -> np.ndarray:
        f = frames(np.asarray(thetas))
        return np.array([log_likelihood(row, observed, sigma, quantum) for row in f])

    return loglik
