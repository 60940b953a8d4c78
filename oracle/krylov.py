"""Alg. 1 of the paper ("Krylov-method"), written out plainly in NumPy/SciPy, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows the paper: A = -iH, Krylov vectors v_1..v_m (here V[:, 0..]),
Hessenberg matrix M (anti-Hermitian, tridiagonal), residual norm ``no``,
h = h_{m+1,m}, tol_rate = err_max / t (eq. errorRate), step t_step (eq. stepSize).

Readings adopted where the paper is silent, ambiguous or garbled:
  R1  Orthogonalisation: Alg. 1 prints the three-term recurrence and the text
      names modified Gram-Schmidt; the hot path requires full Gram-Schmidt.  The
      step here is Alg. 1's recurrence followed by one modified Gram-Schmidt
      pass against every stored vector.  M keeps Alg. 1's tridiagonal entries;
      the extra coefficients only orthogonalise (identical in exact arithmetic).
  R2  Inner products are conjugate-linear in the first slot: M_jj = v_j^H p.
  R3  Lucky breakdown when no < tol_rate (Alg. 1), with h := no; the Krylov
      dimension is then k = j and the step runs to the end of the interval.
  R4  The substep loop integrates [t_step + (n-1) s, t_step + n s] and accepts
      with a strict '<'; the garbled bounds of Alg. 1 would skip the first
      substep interval.  Halving uses a strict '>' (accept '<=').
  R5  N_SUBSTEPS = 10; the first restart starts from t_step = 0.1 and doubles
      while the doubled step still obeys the rate and fits the interval; later
      restarts start from 0.97 times the previous step.  Every candidate is
      clipped to the remaining time, and a step that ends within one substep of
      the end is extended to the end when the whole remaining interval still
      obeys the rate.
  R6  Halving is capped at 64 times (StepUnderflow); with m >= 2 the rate
      E(tau)/tau vanishes as tau -> 0 so the cap is never hit in practice.
  R7  Roundoff estimate (eq. numericalError): d * ||H||_1 * 2^-52 per restart,
      accumulated over restarts and compared with the accumulated bound.
  R8  The initial vector is normalised once; restart vectors are used as they
      come (no renormalisation), and the result is scaled back by ||v0||.
  R10 Quadrature stop test (eq. errorIntegral evaluated per Sec. "Description of
      Program"): relative change below 1e-3 after at least 3 levels, or an
      absolute change below (b - a) * h * k * 2^-52, the rounding-noise floor of
      f = h |sum_n c_n exp(-i lam_n tau)| with sum_n |c_n| <= 1.
  R9  tol = err_max bounds the 2-norm of the final error; the reported bound is
      the sum of the per-step integrals (unitarity makes local errors add).
  R14 The fast integration option (Sec. "Description of Program": a non-adaptive Gauss
      scheme) is the n-point Gauss-Legendre rule on each integration interval, n chosen by
      the user (the paper gives no count); it has no error estimate, so the bound it yields
      is an approximation of the rigorous one.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .quadrature import gauss_legendre, tanh_sinh

WARN_NUMERICAL = 1
WARN_QUADRATURE = 2
UNIT_ROUNDOFF = 2.0 ** -52


class StepUnderflow(RuntimeError):
    """The halving loop of step 2 did not reach an admissible step."""


@dataclass
class Options:
    n_substeps: int = 10
    t_init: float = 0.1
    shrink: float = 0.97
    quad_rel_tol: float = 1e-3
    quad_max_level: int = 15
    quad_min_level: int = 3
    max_halvings: int = 64
    quad_gauss_points: int = 0   # > 0: the paper's fast non-adaptive Gauss option (R14)


@dataclass
class ArnoldiResult:
    V: np.ndarray       # d x k orthonormal Krylov basis
    M: np.ndarray       # k x k anti-Hermitian tridiagonal Hessenberg matrix
    h: float            # h_{k+1,k}: norm of the last residual
    k: int              # Krylov dimension reached
    breakdown: bool     # lucky breakdown (no < tol_rate)


@dataclass
class StepRecord:
    tau: float
    err: float
    k: int
    breakdown: bool
    quad_converged: bool


@dataclass
class EvolveResult:
    v: np.ndarray
    steps: int
    matvecs: int
    err_bound: float
    num_err_estimate: float
    warnings: int
    breakdown_dim: int
    t_reached: float
    trace: List[StepRecord] = field(default_factory=list)
    samples: Optional[np.ndarray] = None        # [n_times, d]: states at the sample times
    sample_bounds: Optional[np.ndarray] = None  # bound at the end of the step holding each time


def spmv(H, x: np.ndarray) -> np.ndarray:
    """y = H x for a workloads.CSR (or any object with to_scipy) or a scipy matrix."""
    mat = H.to_scipy() if hasattr(H, "to_scipy") else H
    return mat @ x


def arnoldi(H, u: np.ndarray, m: int, tol_rate: float, three_term: bool = False) -> ArnoldiResult:
    """Step 1 of Alg. 1 (eq. arnoldi) on A = -iH with full re-orthogonalisation (R1-R3).

    ``three_term``: the recurrence exactly as printed in eq. arnoldi / Alg. 1 (subtract the
    previous vector, project on the current one, normalise), without the full pass; V then
    loses orthogonality as j grows, while the Arnoldi relation holds to rounding."""
    mat = H.to_scipy() if hasattr(H, "to_scipy") else H
    d = u.shape[0]
    k_max = min(m, d)
    V = np.zeros((d, k_max), dtype=np.complex128)
    M = np.zeros((k_max, k_max), dtype=np.complex128)
    V[:, 0] = u
    h = 0.0
    for j in range(k_max):
        p = -1j * (mat @ V[:, j])                    # p := A v_j
        if j > 0:
            p = p - M[j - 1, j] * V[:, j - 1]        # p := p - M_{j-1,j} v_{j-1}
        M[j, j] = np.vdot(V[:, j], p)                # M_jj := v_j^H p
        p = p - M[j, j] * V[:, j]
        if not three_term:
            for i in range(j + 1):                   # full Gram-Schmidt pass (R1)
                p = p - np.vdot(V[:, i], p) * V[:, i]
        no = float(np.linalg.norm(p))
        if no < tol_rate:                            # lucky breakdown (R3)
            return ArnoldiResult(V[:, :j + 1], M[:j + 1, :j + 1], no, j + 1, True)
        if j < k_max - 1:
            M[j, j + 1] = -no
            M[j + 1, j] = no
            V[:, j + 1] = p / no
        else:
            h = no
    return ArnoldiResult(V, M, h, k_max, False)


def hessenberg_from_lanczos(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """The anti-Hermitian M of Alg. 1 for a Lanczos run on H with real diagonal alpha and
    off-diagonal beta: in the basis v_j^(A) = (-i)^(j-1) v_j^(H), M_jj = -i alpha_j and
    M_{j+1,j} = -M_{j,j+1} = beta_j."""
    k = alpha.shape[0]
    M = np.diag(-1j * np.asarray(alpha, dtype=np.float64)).astype(np.complex128)
    for j in range(k - 1):
        M[j + 1, j] = beta[j]
        M[j, j + 1] = -beta[j]
    return M


def hessenberg_eig(M: np.ndarray):
    """Diagonalise the small Hessenberg matrix once per restart (Sec. "Pseudocode", first
    remark): X = iM is Hermitian, X = U diag(lam) U^H, so exp(M tau) = U exp(-i lam tau) U^H."""
    X = 1j * M
    X = 0.5 * (X + X.conj().T)
    lam, U = np.linalg.eigh(X)
    return lam, U


def bound_integrand(lam: np.ndarray, U: np.ndarray, h: float):
    """f(tau) = h |e_k^T exp(M tau) e_1| (Alg. 1 step 2; eq. errorIntegral)."""
    k = lam.shape[0]
    coef = U[k - 1, :] * np.conj(U[0, :])

    def f(tau):
        tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
        phases = np.exp(-1j * np.outer(tau, lam))
        return h * np.abs(phases @ coef)

    return f


def step_size(f, tol_rate: float, t_rem: float, first: bool, tau_prev: float, breakdown: bool,
              opts: Optional[Options] = None, noise_rate: float = 0.0):
    """Step 2 of Alg. 1 (eq. stepSize) with readings R4-R6 and R10.

    ``noise_rate`` is the integrand's rounding floor h * k * 2^-52 (R10).
    Returns (tau, err, quadrature_converged)."""
    opts = opts or Options()
    ok = [True]

    def integral(a, b):
        if opts.quad_gauss_points > 0:
            return gauss_legendre(f, a, b, opts.quad_gauss_points).value
        res = tanh_sinh(f, a, b, opts.quad_rel_tol, opts.quad_max_level, opts.quad_min_level,
                        noise_rate * (b - a))
        ok[0] &= res.converged
        return res.value

    if breakdown:
        tau = t_rem
        return tau, integral(0.0, tau), ok[0]
    if first:
        tau = min(opts.t_init, t_rem)
        err = integral(0.0, tau)
        while err <= tol_rate * tau and 2.0 * tau <= t_rem:
            err2 = integral(0.0, 2.0 * tau)
            if err2 <= tol_rate * 2.0 * tau:
                tau, err = 2.0 * tau, err2
            else:
                break
    else:
        tau = min(opts.shrink * tau_prev, t_rem)
        err = integral(0.0, tau)
    halvings = 0
    while err > tol_rate * tau:
        if halvings == opts.max_halvings:
            raise StepUnderflow("no admissible step after %d halvings" % halvings)
        tau = tau / 2.0
        err = integral(0.0, tau)
        halvings += 1
    s = tau / opts.n_substeps
    n = 1
    while True:
        b = tau + n * s
        if b > t_rem:
            break
        delta = integral(tau + (n - 1) * s, b)
        if err + delta < tol_rate * b:
            err += delta
            n += 1
        else:
            break
    tau = tau + (n - 1) * s
    if tau < t_rem and t_rem - tau < s:
        err_full = integral(0.0, t_rem)
        if err_full <= tol_rate * t_rem:
            tau, err = t_rem, err_full
    return tau, err, ok[0]


def krylov_coefficients(lam: np.ndarray, U: np.ndarray, tau: float) -> np.ndarray:
    """omega = exp(M tau) e_1 (Alg. 1 step 2, last line), through the diagonalisation."""
    return U @ (np.exp(-1j * lam * tau) * np.conj(U[0, :]))


def evolve(H, v0: np.ndarray, t: float, tol: float, m: int, opts: Optional[Options] = None,
           norm1: Optional[float] = None, max_steps: Optional[int] = None,
           three_term: bool = False, sample_times=None, on_step=None) -> EvolveResult:
    """Alg. 1: approximate exp(-iHt) v0 with the a-posteriori bound of eq. errorIntegral.

    ``max_steps`` (harness use only, e.g. timing a bounded sample) stops after that many
    restarts and returns the state reached at t_reached < t.  ``three_term``: step 1 with the
    printed recurrence only (see ``arnoldi``).  ``sample_times`` (ascending, in [0, t]): the
    states at those times from the basis and the small matrix of the step holding each of them
    (second remark after Alg. 1): for t_now <= t_s <= t_now + t_step, v(t_s) = V exp(M (t_s -
    t_now)) e_1; each comes with the bound accumulated up to the end of its step."""
    opts = opts or Options()
    if not (np.isfinite(t) and t >= 0.0) or not (np.isfinite(tol) and tol > 0.0) or m < 2:
        raise ValueError("need t >= 0 finite, tol > 0 finite, m >= 2")
    v0 = np.asarray(v0, dtype=np.complex128)
    if not np.all(np.isfinite(v0)):
        raise ValueError("non-finite initial vector")
    d = v0.shape[0]
    beta0 = float(np.linalg.norm(v0))
    ts = None if sample_times is None else np.asarray(sample_times, dtype=np.float64)
    if ts is not None and (ts.ndim != 1 or np.any(ts < 0) or np.any(ts > t) or np.any(np.diff(ts) < 0)):
        raise ValueError("sample times must be ascending and within [0, t]")
    if t == 0.0 or beta0 == 0.0:
        smp = None if ts is None else np.repeat(v0[None, :], ts.size, axis=0)
        return EvolveResult(v0.copy(), 0, 0, 0.0, 0.0, 0, 0, t, [], smp,
                            None if ts is None else np.zeros(ts.size))
    samples = None if ts is None else np.zeros((ts.size, d), dtype=np.complex128)
    sample_bounds = None if ts is None else np.zeros(ts.size)
    next_sample = 0
    if norm1 is None:
        norm1 = H.norm1() if hasattr(H, "norm1") else float(abs(H).sum(axis=0).max())
    w = v0 / beta0                                   # R8
    tol_rate = tol / t                               # eq. errorRate
    t_now = 0.0
    err_acc = 0.0
    num_acc = 0.0
    warnings = 0
    steps = matvecs = 0
    first = True
    tau_prev = opts.t_init
    breakdown_dim = 0
    trace: List[StepRecord] = []
    while t_now < t:
        t_rem = t - t_now
        ar = arnoldi(H, w, m, tol_rate, three_term)  # step 1
        matvecs += ar.k
        lam, U = hessenberg_eig(ar.M)                # step 2
        f = bound_integrand(lam, U, ar.h)
        tau, err, quad_ok = step_size(f, tol_rate, t_rem, first, tau_prev, ar.breakdown, opts,
                                      ar.h * ar.k * UNIT_ROUNDOFF)
        if not quad_ok:
            warnings |= WARN_QUADRATURE
        err_acc += err
        num_acc += d * norm1 * UNIT_ROUNDOFF          # R7
        if num_acc > err_acc:
            warnings |= WARN_NUMERICAL
        omega = krylov_coefficients(lam, U, tau)
        t_end = t if (tau == t_rem or ar.breakdown) else t_now + tau
        while ts is not None and next_sample < ts.size and ts[next_sample] <= t_end:
            om_s = krylov_coefficients(lam, U, ts[next_sample] - t_now)
            samples[next_sample] = beta0 * (ar.V @ om_s)
            sample_bounds[next_sample] = beta0 * err_acc
            next_sample += 1
        w = ar.V @ omega                             # step 3
        t_now = t if tau == t_rem else t_now + tau
        steps += 1
        trace.append(StepRecord(tau, err, ar.k, ar.breakdown, quad_ok))
        tau_prev = tau
        first = False
        if ar.breakdown:
            breakdown_dim = ar.k
            t_now = t
        if on_step is not None:
            on_step(steps, t_now, beta0 * err_acc)
        if max_steps is not None and steps >= max_steps:
            break
    return EvolveResult(beta0 * w, steps, matvecs, beta0 * err_acc, beta0 * num_acc, warnings,
                        breakdown_dim, t_now, trace, samples, sample_bounds)
