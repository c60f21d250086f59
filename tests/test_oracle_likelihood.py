"""Pins of the likelihood-ratio algebra (CPU only).

* The theorem of Section III-A (with Gamma^-1 = Sigma^-1 - Lambda^-1, Lambda = A'Sigma A,
  the reading that makes the completed square of its proof close) against Gaussian
  log-densities computed by scipy.
* The oracle's q-tilde control terms (Section III-C special case) against the log
  ratio of the natural and the sampling control densities, under the noise-cost
  coupling R = lambda Sigma^-1 of Section II.
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal as mvn

from oracle import mppi


def _spd(rng, d):
    X = rng.standard_normal((d, d))
    return X @ X.T + d * np.eye(d)


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_theorem_against_gaussian_densities(d):
    rng = np.random.default_rng(d)
    for _ in range(20):
        S = _spd(rng, d)
        A = np.eye(d) * rng.uniform(1.2, 3.0) + 0.1 * rng.standard_normal((d, d))
        Lam = A.T @ S @ A
        dt = rng.uniform(0.01, 0.2)
        mu = rng.standard_normal(d)
        z = rng.standard_normal(d) * 3
        lhs = mvn.logpdf(z, np.zeros(d), S / dt) - mvn.logpdf(z, mu, Lam / dt)
        Gi = np.linalg.inv(S) - np.linalg.inv(Lam)
        Si = np.linalg.inv(S)
        Q = (z - mu) @ Gi @ (z - mu) + 2 * mu @ Si @ (z - mu) + mu @ Si @ mu
        rhs = np.log(abs(np.linalg.det(A))) - 0.5 * dt * Q
        assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("m,nu,lam", [(1, 2.0, 1.0), (2, 5.0, 0.3), (4, 1.0, 7.0), (3, 150.0, 2.0)])
def test_q_tilde_is_the_log_likelihood_ratio(m, nu, lam):
    rng = np.random.default_rng(m)
    Sig = _spd(rng, m) / m
    R = lam * np.linalg.inv(Sig)
    U = rng.standard_normal(m)
    du = rng.standard_normal((50, m)) * 2
    v = U + du
    log_ratio = mvn.logpdf(v, np.zeros(m), Sig) - mvn.logpdf(v, U, nu * Sig)
    cost = mppi.likelihood_ratio_cost(du, U, R, nu)
    assert np.allclose(log_ratio, -cost / lam + 0.5 * m * np.log(nu), rtol=1e-10, atol=1e-10)


def test_q_tilde_at_nu_one_is_girsanov_only():
    rng = np.random.default_rng(0)
    R = _spd(rng, 2)
    U = rng.standard_normal(2)
    du = rng.standard_normal((10, 2))
    c = mppi.likelihood_ratio_cost(du, U, R, 1.0)
    assert np.allclose(c, du @ R @ U + 0.5 * U @ R @ U, rtol=1e-14)


@pytest.mark.parametrize("m,lam", [(2, 1.0), (4, 3.0), (3, 0.5)])
def test_per_dimension_covariance_change(m, lam):
    """Diagonal A = diag(sqrt(nu_j)) (the general A_t of Section III-A): the generalised
    q-tilde control terms are the log ratio of N(0, Sigma) and N(u, A Sigma A), up to
    log|A|, under the coupling R = lambda Sigma^-1; a scalar nu reduces to Section III-C."""
    rng = np.random.default_rng(10 + m)
    Sig = _spd(rng, m) / m
    R = lam * np.linalg.inv(Sig)
    nu = rng.uniform(1.0, 20.0, m)
    A = np.diag(np.sqrt(nu))
    U = rng.standard_normal(m)
    du = rng.standard_normal((40, m)) * 2
    v = U + du
    log_ratio = mvn.logpdf(v, np.zeros(m), Sig) - mvn.logpdf(v, U, A @ Sig @ A)
    cost = mppi.likelihood_ratio_cost(du, U, R, nu)
    assert np.allclose(log_ratio, -cost / lam + np.log(np.linalg.det(A)), rtol=1e-10, atol=1e-10)
    same = mppi.likelihood_ratio_cost(du, U, R, np.full(m, 3.0))
    assert np.allclose(same, mppi.likelihood_ratio_cost(du, U, R, 3.0), rtol=1e-13)


def test_per_dimension_noise_covariance():
    from oracle import noise
    sigma = np.array([[0.5, 0.1], [0.1, 0.3]])
    nu = np.array([2.0, 9.0])
    du = noise.control_noise(4, 0, 100_000, 4, sigma, nu).reshape(-1, 2)
    A = np.diag(np.sqrt(nu))
    assert np.allclose(np.cov(du.T), A @ sigma @ A, rtol=0.02, atol=0.01)
