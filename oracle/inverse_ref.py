"""Reference coefficient-inverse sampler (paper Section 5.4).
TEST INFRASTRUCTURE ONLY: used by the test-suite (and nothing the GPU library
loads).  Plain loops in FP64, written from the paper's description, with the
forward model taken from the CPU oracle.

Camera model (Section 5.4): each pixel of the predicted frame m is
contaminated with i.i.d. Gaussian noise of standard deviation sigma and
rounded to the nearest q, so an observed value o is the rounding bin
[o - q/2, o + q/2) that m + sigma*xi fell into:
    p(o | m) = Phi((o + q/2 - m)/sigma) - Phi((o - q/2 - m)/sigma),
    Phi(x) = erfc(-x/sqrt(2))/2,
and the likelihood of a frame is the product over pixels.

Metropolis-Hastings (Section 5.4): from theta_i a candidate
theta_hat = theta_i + s*xi is drawn; under a uniform prior on [lo, hi] it is
taken as theta_{i+1} with probability min(1, p(D|theta_hat)/p(D|theta_i))
(here: when log u < log p(D|theta_hat) - log p(D|theta_i)), and rejected
outright outside the prior; otherwise theta_i repeats.  Several chains run
side by side and share one forward call per iteration.
"""
from __future__ import annotations

import math

from . import oracle


def _Phi(x: float) -> float:
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def bin_log_prob(m: float, o: float, sigma: float, q: float) -> float:
    """log p(o | m) for one pixel (both tails written so the two terms do not cancel)."""
    a = (o - 0.5 * q - m) / sigma
    b = (o + 0.5 * q - m) / sigma
    if a > 0.0:  # upper tail: Phi(b) - Phi(a) = Phi(-a) - Phi(-b)
        p = _Phi(-a) - _Phi(-b)
    else:
        p = _Phi(b) - _Phi(a)
    return math.log(p)


def log_likelihood(pred, obs, sigma: float = 0.1, q: float = 0.1) -> float:
    s = 0.0
    for m, o in zip(pred, obs):
        s += bin_log_prob(float(m), float(o), sigma, q)
    return s


def metropolis(theta0, normals, uniforms, scale: float, loglik, lo: float, hi: float) -> dict:
    """Chains side by side.  loglik(list of thetas) -> list of log-likelihoods (one call per
    iteration, for the candidates inside the prior).  normals and uniforms: (n_iter, n_chains).
    "proposed" holds each candidate's log-likelihood (-inf outside the prior)."""
    K = len(theta0)
    theta = [float(t) for t in theta0]
    cur = list(loglik(theta))
    samples = [list(theta)]
    logls = [list(cur)]
    accepted = []
    proposed = []
    evaluated = K
    for i in range(len(normals)):
        prop = [theta[c] + scale * float(normals[i][c]) for c in range(K)]
        inside = [c for c in range(K) if lo <= prop[c] <= hi]
        got = dict(zip(inside, loglik([prop[c] for c in inside]))) if inside else {}
        evaluated += len(inside)
        proposed.append([got.get(c, -math.inf) for c in range(K)])
        row = []
        for c in range(K):
            ok = c in got and math.log(float(uniforms[i][c])) < got[c] - cur[c]
            if ok:
                theta[c] = prop[c]
                cur[c] = got[c]
            row.append(ok)
        accepted.append(row)
        samples.append(list(theta))
        logls.append(list(cur))
    return {"samples": samples, "loglik": logls, "accepted": accepted, "proposed": proposed,
            "evaluated": evaluated}


def frame(problem, nthreads: int = 1):
    """The camera frame the oracle predicts: the field at the pixel points after the last step."""
    r = oracle.run(problem, sensor_xyz=problem.sensors, nthreads=nthreads)
    return list(r["traces"][-1])
