"""Exploration noise of one MPPI iteration (test infrastructure only).

The special case of Section III-C draws the control perturbation du from a Gaussian
whose covariance is the natural one scaled by nu (A = sqrt(nu) I).  Algorithm 1 does
not say how du is drawn; this oracle fixes the draw so that any implementation can
reproduce it exactly from (seed, iteration):

* Philox4x32-10 block for counter (g, k, iteration_lo, iteration_hi), key = seed,
  supplies the four standard normals with flat indices 4g .. 4g+3 of sample k, where
  the flat index of control component j at time step i is i*m + j;
* uniforms u = ((x >> 8) + 1) * 2^-24 in (0, 1] (exact in FP32 and FP64);
* Box-Muller (Box & Muller 1958) on output pairs (0, 1) and (2, 3):
  eps_a = sqrt(-2 ln u_a) cos(2 pi u_b),  eps_b = sqrt(-2 ln u_a) sin(2 pi u_b);
* du_{k,i} = sqrt(nu) * L eps_{k,i}, L = chol(Sigma)   (variance nu * Sigma).
"""
import numpy as np

from .philox import philox4x32_10, key_words


def uniforms_from_bits(x):
    """uint32 -> (0, 1]: top 24 bits plus one, times 2^-24."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 1.0) * (2.0 ** -24)


def box_muller(ua, ub):
    r = np.sqrt(-2.0 * np.log(ua))
    t = 2.0 * np.pi * ub
    return r * np.cos(t), r * np.sin(t)


def standard_normals(seed: int, iteration: int, K: int, T: int, m: int, k_offset: int = 0):
    """eps[k, i, j] for k in [k_offset, k_offset + K), FP64, shape (K, T, m)."""
    n_flat = T * m
    n_groups = (n_flat + 3) // 4
    k0, k1 = key_words(seed)
    it = int(iteration) & 0xFFFFFFFFFFFFFFFF
    g = np.arange(n_groups, dtype=np.uint64)[None, :]
    k = (np.arange(K, dtype=np.uint64) + np.uint64(k_offset))[:, None]
    g, k = np.broadcast_arrays(g, k)
    o0, o1, o2, o3 = philox4x32_10(g, k, it & 0xFFFFFFFF, it >> 32, k0, k1)
    e0, e1 = box_muller(uniforms_from_bits(o0), uniforms_from_bits(o1))
    e2, e3 = box_muller(uniforms_from_bits(o2), uniforms_from_bits(o3))
    flat = np.stack([e0, e1, e2, e3], axis=-1).reshape(K, n_groups * 4)[:, :n_flat]
    return flat.reshape(K, T, m)


def control_noise(seed: int, iteration: int, K: int, T: int, sigma, nu, k_offset: int = 0):
    """du[k, i, :] = A chol(sigma) eps[k, i, :] with A = sqrt(nu) I for a scalar nu, or
    A = diag(sqrt(nu_j)) for per-dimension factors (the covariance change A_t of the
    likelihood-ratio theorem, Section III-A): du ~ N(0, A sigma A)."""
    sigma = np.atleast_2d(np.asarray(sigma, dtype=np.float64))
    m = sigma.shape[0]
    eps = standard_normals(seed, iteration, K, T, m, k_offset)
    L = cholesky_psd(sigma)
    if np.ndim(nu) == 0:
        return np.sqrt(nu) * np.einsum("jl,ktl->ktj", L, eps)
    A = np.diag(np.sqrt(np.asarray(nu, dtype=np.float64)))
    return np.einsum("jl,ktl->ktj", A @ L, eps)


def cholesky_psd(sigma):
    """Lower Cholesky factor; a zero covariance (no noise) gives L = 0."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if not np.any(sigma):
        return np.zeros_like(sigma)
    return np.linalg.cholesky(sigma)
