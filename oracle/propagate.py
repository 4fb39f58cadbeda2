"""Time propagation (oracle): adaptive Lanczos exponential and Magnus-2 step.

* Sec. 2.6, eq. (AdaptiveKrylov): exp(-i tau Hbar) psi ~ ||psi|| Q_k exp(-i tau T_k) e_1,
  with Q_k the Lanczos vectors of Hbar started from psi and T_k tridiagonal.
  The section gives the three-term recurrence; in floating point the vectors
  lose orthogonality once Ritz values converge, so two ways of keeping them
  orthogonal are provided (both reduce to the recurrence in exact arithmetic):
  - "full" (default, the plain scheme every stored reference is made with): the
    three-term step, then two classical Gram-Schmidt passes against all previous
    vectors;
  - "partial": the three-term recurrence itself, with alpha_j the
    q_j coefficient of A q_j (computed) and beta_{j-1} the previous norm (known);
    Simon's omega recurrence (Simon 1984,
    "The Lanczos algorithm with partial reorthogonalization") estimates
    omega_{j+1,k} ~ q_{j+1}^H q_k from alpha, beta alone, and when an estimate
    exceeds sqrt(eps) the vector, and the next one, get a Gram-Schmidt pass
    against all previous vectors (semi-orthogonality, which keeps T_k the
    projected operator to working accuracy); a pass is also made when the
    local one cancelled most of the vector.
  exp(-i tau T_k) e_1 by eigendecomposition of T_k.
* eq. (AdaptiveKrylovErr): the error estimate of the k-dimensional
  approximation is |tau| beta_k ||psi|| |[exp(-i tau T_k)]_{k,1}|, where beta_k is
  the next off-diagonal entry (the factor |tau| converts the Lanczos data of Hbar
  into those of -i tau Hbar).  The iteration stops at the first k whose estimate
  is at most tol ||psi||, or at an invariant subspace (beta_k <= 1e-14 ||T_k||).
* Sec. 2.5, eq. (ApproxMagnus): psi(t+dt) = exp(-i dt Hbar[rho(t+dt/2)]) psi(t),
  with the midpoint Hamiltonian from a second-order predictor-corrector: a
  predictor step with Hbar[rho(t), t], rho_mid = (rho(t) + rho_pred)/2, field at
  t + dt/2, one corrector step.
* delta kick: psi <- exp(i kappa Zbar_d) psi with the Loewdin position operator.
* Sec. 2.5 names a second way to the midpoint Hamiltonian: extrapolation from
  m > 2 previous steps.  Scheme "extrap" takes m = 3: the density at t + dt/2 is
  the quadratic through rho(t), rho(t - dt), rho(t - 2 dt) evaluated there
  (weights 15/8, -10/8, 3/8), Hbar is evaluated at that density with the field
  at t + dt/2, and one exponential makes the step.  Until three densities of the
  current dt are known (after a refresh or a change of dt) a step is a
  predictor-corrector step.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
import scipy.linalg as sla


class NoConvergence(RuntimeError):
    pass


def tridiag_exp_e1(alpha, beta, tau):
    """u = exp(-i tau T) e_1 for the symmetric tridiagonal T(alpha, beta)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    if len(alpha) == 1:
        return np.array([np.exp(-1j * tau * alpha[0])])
    lam, V = sla.eigh_tridiagonal(alpha, np.asarray(beta, dtype=np.float64))
    return V @ (np.exp(-1j * tau * lam) * V[0, :])


EPS = float(np.finfo(np.float64).eps)
SQRT_EPS = math.sqrt(EPS)
CANCEL_ETA = 1e-3      # a local pass leaving less than this fraction of w triggers a full pass


def omega_next(alpha, beta, b_j, om_j, om_jm1, anorm):
    """Simon's recurrence: estimates omega_{j+1,k} ~ q_{j+1}^H q_k, k = 1..j+1.

    beta_j omega_{j+1,k} = beta_k omega_{j,k+1} + (alpha_k - alpha_j) omega_{j,k}
                           + beta_{k-1} omega_{j,k-1} - beta_{j-1} omega_{j-1,k}
    for k < j, plus a rounding term 2 eps ||A|| of the sign of the sum; omega_{j+1,j}
    = eps ||A|| / beta_j (the explicit local orthogonalisation) and omega_{j+1,j+1} = 1.
    alpha = [alpha_1..alpha_j], beta = [beta_1..beta_{j-1}], b_j = beta_j,
    om_j[k-1] = omega_{j,k} (k = 1..j), om_jm1[k-1] = omega_{j-1,k} (k = 1..j-1)."""
    j = len(alpha)
    a_j = alpha[-1]
    out = np.zeros(j + 1)
    for k in range(1, j):
        t = beta[k - 1] * om_j[k] + (alpha[k - 1] - a_j) * om_j[k - 1]
        if k > 1:
            t += beta[k - 2] * om_j[k - 2]
        t -= beta[j - 2] * om_jm1[k - 1]
        t += math.copysign(2.0 * EPS * anorm, t)
        out[k - 1] = t / b_j
    out[j - 1] = EPS * anorm / b_j
    out[j] = 1.0
    return out


def _lanczos_column(tau, v, tol, kmax, k_force: Optional[int] = None, reorth: str = "full",
                    stats: Optional[dict] = None):
    """One column as a generator: yields each Lanczos vector q_j and is sent A q_j;
    returns (exp(-i tau A) v approximation, k, error estimate)."""
    if reorth not in ("partial", "full"):
        raise ValueError(f"unknown reorthogonalisation {reorth!r}")
    beta0 = float(np.linalg.norm(v))
    if beta0 == 0.0:
        return np.zeros_like(v), 0, 0.0
    Q = [v / beta0]
    alpha, beta = [], []
    om_j, om_jm1 = np.array([1.0]), None
    anorm, force = 0.0, False
    for j in range(1, kmax + 1):
        q = Q[-1]
        w = yield q
        if reorth == "full":
            a = float(np.real(np.vdot(q, w)))
            alpha.append(a)
            w = w - a * q
            if j > 1:
                w = w - beta[-1] * Q[-2]
            Qm = np.stack(Q, axis=1)
            for _ in range(2):                       # two CGS passes
                h = Qm.conj().T @ w
                w = w - Qm @ h
            b = float(np.linalg.norm(w))
        else:
            # three-term step: the q_j coefficient from w, the q_{j-1} one the known beta_{j-1}
            w0 = float(np.linalg.norm(w))
            h = np.vdot(q, w)
            w = w - h * q
            if j > 1:
                w = w - beta[-1] * Q[-2]
            a = float(np.real(h))
            alpha.append(a)
            b = float(np.linalg.norm(w))
            anorm = max(anorm, abs(a) + b + (beta[-1] if beta else 0.0))
            if b > 0.0:
                om_new = omega_next(alpha, beta, b, om_j, om_jm1, anorm)
                exceed = j > 1 and float(np.max(np.abs(om_new[:j - 1]))) > SQRT_EPS
            else:
                om_new, exceed = np.zeros(j + 1), False
            if b > 0.0 and (exceed or force or b < CANCEL_ETA * w0):
                Qm = np.stack(Q, axis=1)
                w = w - Qm @ (Qm.conj().T @ w)
                b = float(np.linalg.norm(w))
                om_new[:j] = EPS
                if stats is not None:
                    stats["reorth"] = stats.get("reorth", 0) + 1
            force = exceed
            om_jm1, om_j = om_j, om_new
        u = tridiag_exp_e1(alpha, beta, tau)
        err = abs(tau) * b * beta0 * abs(u[-1])
        tnorm = max(abs(alpha[i]) + (beta[i - 1] if i > 0 else 0.0) + (beta[i] if i < len(beta) else 0.0)
                    for i in range(len(alpha))) + b
        if k_force is not None:
            done = j >= k_force
        else:
            done = err <= tol * beta0 or b <= 1e-14 * tnorm
        if done:
            return beta0 * (np.stack(Q, axis=1) @ u), j, err
        beta.append(b)
        Q.append(w / b)
    raise NoConvergence(f"Lanczos did not reach tol {tol} within {kmax} vectors")


def lanczos_expm_column(Aop, tau, v, tol, kmax, k_force: Optional[int] = None, reorth: str = "full",
                        stats: Optional[dict] = None):
    """One column: returns (exp(-i tau A) v approximation, k, error estimate)."""
    gen = _lanczos_column(tau, v, tol, kmax, k_force, reorth, stats)
    try:
        q = next(gen)
        while True:
            q = gen.send(Aop(q))
    except StopIteration as stop:
        return stop.value


def lanczos_expm(A, tau, X, tol=1e-10, kmax=64, k_force: Optional[Sequence[int]] = None, reorth: str = "full",
                 stats: Optional[dict] = None, block=False, block_cols=None):
    """exp(-i tau A) X, one Krylov space per column.  A: matrix (sparse/dense) or callable.

    block=False: the columns one after another.  block=True (A callable on an
    (n, m) block): the columns' recurrences advance together and A is applied once
    per iteration to the block of the still-running columns' vectors; each column
    runs the same steps as alone (the columns are independent problems).  With
    block_cols, at most that many columns advance together (bounds the memory of
    the Krylov vectors held at once)."""
    if block and block_cols is not None and X.shape[1] > block_cols:
        X = np.asarray(X, dtype=np.complex128)
        Y = np.empty_like(X)
        ks = np.zeros(X.shape[1], dtype=np.int32)
        errs = np.zeros(X.shape[1])
        for c0 in range(0, X.shape[1], block_cols):
            c1 = min(c0 + block_cols, X.shape[1])
            kf = None if k_force is None else k_force[c0:c1]
            Y[:, c0:c1], ks[c0:c1], errs[c0:c1] = lanczos_expm(A, tau, X[:, c0:c1], tol, kmax, kf, reorth, stats,
                                                              block=True)
        return Y, ks, errs
    X = np.asarray(X, dtype=np.complex128)
    Y = np.empty_like(X)
    ks = np.zeros(X.shape[1], dtype=np.int32)
    errs = np.zeros(X.shape[1])
    if not block:
        Aop = A if callable(A) else (lambda q: A @ q)
        for a in range(X.shape[1]):
            kf = None if k_force is None else int(k_force[a])
            Y[:, a], ks[a], errs[a] = lanczos_expm_column(Aop, tau, X[:, a], tol, kmax, kf, reorth, stats)
        return Y, ks, errs
    Ablk = A if callable(A) else (lambda B: A @ B)
    gens, qs = {}, {}
    for a in range(X.shape[1]):
        kf = None if k_force is None else int(k_force[a])
        g = _lanczos_column(tau, X[:, a], tol, kmax, kf, reorth, stats)
        try:
            qs[a] = next(g)
            gens[a] = g
        except StopIteration as stop:
            Y[:, a], ks[a], errs[a] = stop.value
    while gens:
        cols = sorted(gens)
        W = Ablk(np.stack([qs[a] for a in cols], axis=1))
        for i, a in enumerate(cols):
            try:
                qs[a] = gens[a].send(W[:, i])
            except StopIteration as stop:
                Y[:, a], ks[a], errs[a] = stop.value
                del gens[a], qs[a]
    return Y, ks, errs


# quadratic extrapolation to t + dt/2 from the values at t, t - dt, t - 2 dt
EXTRAP3 = (15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0)


def extrapolate_midpoint(history):
    """Value at t + dt/2 of the quadratic through history = [f(t - 2dt), f(t - dt), f(t)]."""
    return EXTRAP3[0] * history[-1] + EXTRAP3[1] * history[-2] + EXTRAP3[2] * history[-3]


class Propagator:
    """Magnus-2 propagation of the orbital block (eq. ApproxMagnus); the midpoint
    Hamiltonian by predictor-corrector (scheme "pc") or by extrapolation from the
    three previous densities (scheme "extrap")."""

    def __init__(self, model, X, t=0.0, field=None, tol=None, kmax=None, scheme="pc", reorth="full",
                 matrix_free=False, block_cols=None):
        """matrix_free: Hbar as `EFEModel.operator` (cell blocks and coupling applied
        without assembly, Hartree by fast diagonalisation) and the Lanczos columns
        advanced together, at most block_cols at a time (for large meshes);
        otherwise the assembled matrix."""
        if scheme not in ("pc", "extrap"):
            raise ValueError(f"unknown scheme {scheme!r}")
        self.reorth = reorth
        self.matrix_free = matrix_free
        self.block_cols = block_cols
        self.model = model
        self.X = np.asarray(X, dtype=np.complex128).copy()
        self.t = float(t)
        self.field = field
        self.tol = model.spec.krylov_tol if tol is None else tol
        self.kmax = model.spec.kmax if kmax is None else kmax
        self.scheme = scheme
        self.refresh()

    def refresh(self):
        """(Re)build rho and Hbar for the current orbitals and time; the density
        history restarts from rho."""
        self.rho = self.model.density(self.X)
        self.H = self._ham(self.rho, self.t)
        self.hist, self.hist_dt = [self.rho], None

    def _ham(self, rho, t):
        if self.matrix_free:
            return self.model.operator_from_density(rho, t, self.field)
        return self.model.hamiltonian_from_density(rho, t, self.field)

    def _expm(self, A, tau, X, k_force):
        return lanczos_expm(A, tau, X, self.tol, self.kmax, k_force, reorth=self.reorth, block=self.matrix_free,
                            block_cols=self.block_cols)

    def kick(self, kappa, direction=2):
        """psi <- exp(i kappa Zbar_d) psi, then refresh the Hamiltonian."""
        self.H = None                              # released before the next operator is built
        Z = self.model.position_operator_free(direction) if self.matrix_free else \
            self.model.position_operator(direction)
        self.X, k, _ = self._expm(Z, -kappa, self.X, None)
        del Z
        self.refresh()
        return k

    def step(self, dt, k_force=None):
        """One Magnus-2 step; returns (mu, k_pred, k_corr) (k_pred = 0 for an
        extrapolated step, which has no predictor)."""
        m = self.model
        kp_f = None if k_force is None else k_force[0]
        kc_f = None if k_force is None else k_force[1]
        hist = self.hist if self.hist_dt == dt else [self.rho]
        if self.scheme == "extrap" and len(hist) >= 3:
            rho_mid = extrapolate_midpoint(hist)
            kp = np.zeros(self.X.shape[1], dtype=np.int32)
        else:
            Xp, kp, _ = self._expm(self.H, dt, self.X, kp_f)
            rho_mid = 0.5 * (self.rho + m.density(Xp))
            del Xp
        self.H = None                                  # rebuilt at the end of the step
        Hmid = self._ham(rho_mid, self.t + 0.5 * dt)
        self.X, kc, _ = self._expm(Hmid, dt, self.X, kc_f)
        del Hmid
        self.t += dt
        self.rho = m.density(self.X)
        self.H = None
        self.H = self._ham(self.rho, self.t)
        self.hist, self.hist_dt = (hist + [self.rho])[-3:], dt
        return m.dipole(self.rho), kp, kc

    def run(self, dt, nsteps, k_force=None):
        mus, ks = [], []
        for n in range(nsteps):
            mu, kp, kc = self.step(dt, None if k_force is None else k_force[n])
            mus.append(mu)
            ks.append((kp, kc))
        return np.array(mus), np.array(ks)


def scf_ground_state(model, tol=1e-11, mix=0.5, maxit=200, verbose=False):
    """Self-consistent ground state by dense diagonalisation of Hbar.

    Start from the Hamiltonian without Hartree and xc terms, take the lowest
    norb eigenvectors, mix densities linearly, stop when max |rho_out - rho_in| < tol.
    Returns (X, eigenvalues, iterations).
    """
    norb = model.spec.norb
    active = np.concatenate([model.interior, model.mesh.n_nodes + np.arange(model.nk)])
    v0 = model.v_nuc + model.v_trap
    H = model.hamiltonian(v0)
    rho_in = None
    for it in range(1, maxit + 1):
        Ha = H[active][:, active].toarray()
        lam, V = sla.eigh(Ha, subset_by_index=[0, norb - 1])
        X = np.zeros((model.n_rows, norb), dtype=np.complex128)
        X[active] = V
        rho_out = model.density(X)
        if rho_in is not None:
            dmax = float(np.max(np.abs(rho_out - rho_in)))
            if verbose:
                print(f"scf {it}: max|drho| = {dmax:.3e}  eps = {lam}")
            if dmax < tol:
                return X, lam, it
            rho_in = (1.0 - mix) * rho_in + mix * rho_out
        else:
            rho_in = rho_out
        H = model.hamiltonian_from_density(rho_in)
    raise NoConvergence("SCF did not converge")
