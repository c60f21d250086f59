"""One MPPI iteration and one MPC control step, FP64 (test infrastructure only).

Follows Algorithm 1 (Section IV) with the likelihood-ratio running cost of the
special case in Section III-C and the Monte-Carlo update law that precedes it.
The readings taken where the paper is silent or inconsistent are:

* transitions i = 0 .. T-1 (every u_i is used), one explicit Euler step each;
* the running cost is evaluated at the post-transition state x_{i+1} and is added
  per step without a dt factor (as Algorithm 1 adds q-tilde); phi(x_T) at the end;
* one total path cost per sample weights every time step (the forward-accumulated
  cost of Algorithm 1); the cost-to-go variant is ``iteration_cost_to_go``;
* the weights are shifted by the minimum cost before exponentiating -- any
  sample-independent factor cancels between numerator and denominator of the
  update law (Section III-B), so this changes nothing but the range;
* a non-finite path cost counts as +inf (weight 0); if every sample is non-finite
  the iteration leaves U unchanged and reports status NUMERIC.
"""
import dataclasses

import numpy as np

from . import systems as _systems
from .noise import control_noise

STATUS_OK = 0
STATUS_NUMERIC = -5


@dataclasses.dataclass
class IterationResult:
    U: np.ndarray          # updated nominal sequence (T, m)
    S: np.ndarray          # per-sample path cost with likelihood-ratio terms (K,)
    w: np.ndarray          # normalised weights (K,)
    eta: float             # normaliser sum_k exp(-(S_k - rho) / lam)
    rho: float             # min_k S_k
    dU: np.ndarray         # weighted average of the perturbations (T, m)
    du: np.ndarray         # perturbations (K, T, m)
    status: int


def likelihood_ratio_cost(du, U_i, R, nu):
    """Control part of q-tilde.  Special case A = sqrt(nu) I (Section III-C):
    (1 - 1/nu)/2 du^T R du + u^T R du + 1/2 u^T R u, per sample.  For per-dimension factors
    A = diag(sqrt(nu_j)) the same derivation (the theorem of Section III-A with the noise-cost
    coupling of Section II) gives 1/2 du^T (R - A^-1 R A^-1) du + u^T R du + 1/2 u^T R u."""
    lin = du @ (R @ U_i)
    const = 0.5 * U_i @ R @ U_i
    if np.ndim(nu) == 0:
        quad = np.einsum("kj,jl,kl->k", du, R, du)
        return 0.5 * (1.0 - 1.0 / nu) * quad + lin + const
    Ai = np.diag(1.0 / np.sqrt(np.asarray(nu, dtype=np.float64)))
    M = R - Ai @ R @ Ai
    return 0.5 * np.einsum("kj,jl,kl->k", du, M, du) + lin + const


def transition(system, x, v, dt, crashed):
    """One Euler transition of all samples and the crash term of the step's cost.  With a
    crash indicator (Section V-C: C = 1 once the vehicle hits the ground or an obstacle) a
    crashed sample stops simulating and stays where it is for the rest of the horizon,
    paying crash_cost at every step from the one that crashed on."""
    x_new = _systems.euler_step(system, x, v, dt)
    cc = getattr(system, "crash_cost", 0.0)
    if not cc:
        return x_new, crashed, 0.0
    x_new = np.where(crashed[:, None], x, x_new)
    crashed = crashed | system.crashed(x_new)
    return x_new, crashed, np.where(crashed, cc, 0.0)


def rollout_costs(system, x0, U, du, dt, R, nu, observer=None):
    """Path costs S-tilde for all samples: the K-loop of Algorithm 1.
    ``observer(i, x)``, if given, sees the states x_{i+1} of all samples (tests only)."""
    K, T, m = du.shape
    x = np.repeat(np.asarray(x0, float)[None, :], K, axis=0)
    crashed = np.zeros(K, dtype=bool)
    S = np.zeros(K)
    for i in range(T):
        v = U[i][None, :] + du[:, i, :]
        x, crashed, c_cost = transition(system, x, v, dt, crashed)
        if observer is not None:
            observer(i, x)
        S = S + (system.q(x) + c_cost + likelihood_ratio_cost(du[:, i, :], U[i], R, nu))
    S = S + system.phi(x)
    S[~np.isfinite(S)] = np.inf
    return S


def weights_and_update(S, du, lam):
    """Min-shifted exponential weights and the Monte-Carlo update law (Section III-C):
    dU_i = sum_k exp(-S_k / lam) du_{k,i} / sum_k exp(-S_k / lam)."""
    rho = float(np.min(S))
    K, T, m = du.shape
    if not np.isfinite(rho):
        return np.zeros(K), 0.0, rho, np.zeros((T, m)), STATUS_NUMERIC
    e = np.exp(-(S - rho) / lam)
    eta = float(np.sum(e))
    w = e / eta
    dU = np.einsum("k,ktj->tj", w, du)
    return w, eta, rho, dU, STATUS_OK


def iteration(wl, x0, U, iteration_index, system=None, nu=None, du=None, observer=None):
    """One MPPI iteration on workload ``wl`` from state x0 around sequence U."""
    system = system or _systems.make(wl)
    nu = wl.nu if nu is None else nu
    U = np.asarray(U, float)
    if du is None:
        du = control_noise(wl.seed, iteration_index, wl.K, wl.T, wl.sigma, nu)
    S = rollout_costs(system, x0, U, du, wl.dt, np.asarray(wl.R, float), nu, observer)
    w, eta, rho, dU, status = weights_and_update(S, du, wl.lam)
    return IterationResult(U=U + dU, S=S, w=w, eta=eta, rho=rho, dU=dU, du=du, status=status)


def shift(U, u_init):
    """Warm start of Algorithm 1: drop u_0, move everything one step up, append u_init."""
    out = np.empty_like(U)
    out[:-1] = U[1:]
    out[-1] = u_init
    return out


def control_step(wl, x0, U, iteration_start, system=None, observer=None):
    """``n_iters`` iterations, emit u0, shift.  Returns (u0, U_shifted, next_iteration, results)."""
    system = system or _systems.make(wl)
    results = []
    it = iteration_start
    for _ in range(wl.n_iters):
        r = iteration(wl, x0, U, it, system=system, observer=observer)
        results.append(r)
        U = r.U
        it += 1
    u0 = U[0].copy()
    return u0, shift(U, wl.u_init), it, results


def plant_step(wl, x, u, system=None):
    """Deterministic same-model plant: one noise-free Euler step with the emitted control."""
    system = system or _systems.make(wl)
    return _systems.euler_step(system, np.asarray(x, float)[None, :], np.asarray(u, float)[None, :], wl.dt)[0]


def initial_sequence(wl):
    return np.repeat(np.asarray(wl.u_init, float)[None, :], wl.T, axis=0)


def plain_mppi_iteration(wl, x0, U, iteration_index, system=None):
    """MPPI with the mean-shift (Girsanov-only) importance weights and the natural noise:
    no exploration factor at all.  S = sum_i [q(x_{i+1}) + u_i^T R du_i + 1/2 u_i^T R u_i] + phi.
    Written separately from ``iteration`` so that nu = 1 can be checked against it."""
    system = system or _systems.make(wl)
    R = np.asarray(wl.R, float)
    du = control_noise(wl.seed, iteration_index, wl.K, wl.T, wl.sigma, 1.0)
    K = wl.K
    x = np.repeat(np.asarray(x0, float)[None, :], K, axis=0)
    S = np.zeros(K)
    for i in range(wl.T):
        x = x + wl.dt * system.xdot(x, U[i][None, :] + du[:, i, :])
        S = S + (system.q(x) + (du[:, i, :] @ (R @ U[i]) + 0.5 * U[i] @ R @ U[i]))
    S = S + system.phi(x)
    S[~np.isfinite(S)] = np.inf
    e = np.exp(-(S - S.min()) / wl.lam)
    return U + np.einsum("k,ktj->tj", e / e.sum(), du), S


def iteration_cost_to_go(wl, x0, U, iteration_index, system=None, du=None):
    """Per-time-step weighting by the cost-to-go from time i onward (the literal reading of
    the update law's S(tau_{i,k})): u_i += sum_k w_{k,i} du_{k,i} with w_{.,i} the min-shifted
    softmax of the tail sums of q-tilde."""
    system = system or _systems.make(wl)
    R = np.asarray(wl.R, float)
    U = np.asarray(U, float)
    if du is None:
        du = control_noise(wl.seed, iteration_index, wl.K, wl.T, wl.sigma, wl.nu)
    K, T, m = du.shape
    x = np.repeat(np.asarray(x0, float)[None, :], K, axis=0)
    crashed = np.zeros(K, dtype=bool)
    qt = np.zeros((K, T))
    for i in range(T):
        x, crashed, c_cost = transition(system, x, U[i][None, :] + du[:, i, :], wl.dt, crashed)
        qt[:, i] = system.q(x) + c_cost + likelihood_ratio_cost(du[:, i, :], U[i], R, wl.nu)
    qt[:, -1] += system.phi(x)
    tail = np.cumsum(qt[:, ::-1], axis=1)[:, ::-1]
    dU = np.zeros((T, m))
    for i in range(T):
        s = tail[:, i]
        s = np.where(np.isfinite(s), s, np.inf)
        e = np.exp(-(s - s.min()) / wl.lam)
        dU[i] = (e / e.sum()) @ du[:, i, :]
    return U + dU


def merge_shards(parts, lam):
    """Exact combination of per-shard partial sums (rho_g, eta_g, N_g) where
    eta_g = sum exp(-(S - rho_g)/lam) and N_g = sum exp(-(S - rho_g)/lam) du over shard g:
    the sample-independent factor exp(-(rho_g - rho)/lam) rescales each shard."""
    rho = min(p[0] for p in parts)
    alpha = [np.exp(-(p[0] - rho) / lam) for p in parts]
    eta = sum(a * p[1] for a, p in zip(alpha, parts))
    N = sum(a * p[2] for a, p in zip(alpha, parts))
    return N / eta


def effective_sample_size(w):
    return 1.0 / np.sum(np.asarray(w) ** 2)
