"""Pins for the oracle's Lanczos exponential and Magnus-2 step.

* Lanczos against dense exp(-i tau Hbar) (eigendecomposition) on the tiny Hbar;
  a 2x2 closed form; an eigenvector input stops at k = 1 with the exact phase;
  the a-posteriori estimate of eq. (AdaptiveKrylovErr) tracks the true error.
* Magnus: norm and orthonormality conservation; time reversibility with a frozen
  Hamiltonian; a self-consistent ground state is stationary (density constant,
  orbitals acquire exp(-i eps t)); second-order convergence in dt (paper: q = 1.99);
  harmonic-potential (Kohn) theorem mu_z(t) = N kappa sin(w t)/w in a trap;
  linear response mu/kappa independent of kappa; inversion symmetry: mu odd in kappa.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.model import EFEModel
from oracle.propagate import (lanczos_expm, lanczos_expm_column, Propagator, tridiag_exp_e1,
                              NoConvergence)
from workloads import tiny, trap

TRAP_ARGS = dict(omega=1.0, ncell=4, half=6.0, degree=4)


@pytest.fixture(scope="module")
def tiny_model():
    return EFEModel(tiny())


@pytest.fixture(scope="module")
def tiny_gs(golden_dir):
    return np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))


def test_tridiag_exp_closed_form():
    a, b, d = 0.3, 0.7, -1.1
    tau = 0.9
    u = tridiag_exp_e1([a, d], [b], tau)
    mu, om = 0.5 * (a + d), math.hypot(0.5 * (a - d), b)
    A = np.array([[a, b], [b, d]])
    E = np.exp(-1j * tau * mu) * (math.cos(tau * om) * np.eye(2)
                                  - 1j * math.sin(tau * om) / om * (A - mu * np.eye(2)))
    np.testing.assert_allclose(u, E[:, 0], atol=1e-15)


def test_lanczos_2x2_exact():
    A = np.array([[0.3, 0.7], [0.7, -1.1]])
    v = np.array([0.6, 0.8j])
    y, k, err = lanczos_expm_column(lambda q: A @ q, 0.9, v, 1e-14, 4)
    w, V = np.linalg.eigh(A)
    exact = V @ (np.exp(-0.9j * w) * (V.T @ v))
    np.testing.assert_allclose(y, exact, atol=1e-15)
    assert k == 2


def test_lanczos_matches_dense_expm(tiny_model):
    m = tiny_model
    H = m.hamiltonian(m.v_nuc)
    act = np.concatenate([m.interior, m.mesh.n_nodes + np.arange(m.nk)])
    Ha = H[act][:, act].toarray()
    lam, V = np.linalg.eigh(Ha)
    rng = np.random.default_rng(0)
    X = np.zeros((m.n_rows, 3), dtype=np.complex128)
    X[act] = rng.standard_normal((len(act), 3)) + 1j * rng.standard_normal((len(act), 3))
    X /= np.linalg.norm(X, axis=0)
    tau, tol = 0.05, 1e-10
    Y, ks, errs = lanczos_expm(H, tau, X, tol=tol, kmax=200)
    exact = np.zeros_like(X)
    exact[act] = V @ (np.exp(-1j * tau * lam)[:, None] * (V.T @ X[act]))
    e = np.linalg.norm(Y - exact, axis=0)
    assert np.all(e <= 10 * tol), (e, ks)
    # unitarity
    np.testing.assert_allclose(np.linalg.norm(Y, axis=0), 1.0, atol=1e-13)
    # the estimate is within two orders of magnitude of the truth at a fixed k
    for k in (4, 6, 8):
        Yk, _, ek = lanczos_expm(H, tau, X[:, :1], tol=tol, kmax=200, k_force=[k])
        true = np.linalg.norm(Yk[:, 0] - exact[:, 0])
        assert 1e-2 < ek[0] / true < 1e2, (k, ek, true)


def _spread_operator(n=500, seed=1):
    """Hermitian A = U diag(lam) U^H: a dense cluster in [0, 1] and six isolated large
    eigenvalues, whose Ritz values converge within a few steps (the situation in which
    the three-term recurrence loses orthogonality)."""
    rng = np.random.default_rng(seed)
    lam = np.concatenate([np.linspace(0.0, 1.0, n - 6), [200.0, 400.0, 600.0, 800.0, 1000.0, 1200.0]])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return U, lam, v / np.linalg.norm(v)


def _plain_lanczos_loss(A, v, k):
    """Largest |q_i^H q_l| (i != l) of k steps of the bare three-term recurrence."""
    Q = [v]
    beta = 0.0
    for j in range(k):
        w = A @ Q[-1]
        a = np.real(np.vdot(Q[-1], w))
        w = w - a * Q[-1] - (beta * Q[-2] if j > 0 else 0.0)
        beta = np.linalg.norm(w)
        Q.append(w / beta)
    Qm = np.stack(Q, axis=1)
    G = Qm.conj().T @ Qm
    return float(np.max(np.abs(G - np.eye(len(Q)))))


@pytest.mark.parametrize("tau", [0.02, 0.1])
def test_partial_reorth_matches_exact_and_full(tau):
    """Simon's partial reorthogonalisation: the exponential agrees with the exact one
    to the Krylov tolerance and with full reorthogonalisation to rounding, while the
    bare recurrence on the same operator loses orthogonality to O(1e-3) and more."""
    U, lam, v = _spread_operator()
    A = (U * lam) @ U.conj().T
    exact = U @ (np.exp(-1j * tau * lam) * (U.conj().T @ v))
    st = {}
    y, k, _ = lanczos_expm_column(lambda q: A @ q, tau, v, 1e-10, 200, reorth="partial", stats=st)
    yf, kf, _ = lanczos_expm_column(lambda q: A @ q, tau, v, 1e-10, 200, reorth="full")
    assert k == kf
    assert st.get("reorth", 0) >= 2                       # the estimates did trigger
    assert np.linalg.norm(y - exact) < 10 * 1e-10
    assert np.linalg.norm(y - yf) < 1e-13
    assert _plain_lanczos_loss(A, v, k) > 1e-3


def test_omega_estimates_bound_the_loss():
    """The omega recurrence tracks the actual loss of orthogonality of the bare
    recurrence from above (within a few orders) until it passes sqrt(eps)."""
    from oracle.propagate import omega_next, SQRT_EPS
    U, lam, v = _spread_operator()
    A = (U * lam) @ U.conj().T
    Q, alpha, beta = [v], [], []
    om_j, om_jm1, anorm = np.array([1.0]), None, 0.0
    checked = 0
    for j in range(1, 40):
        w = A @ Q[-1]
        h = np.vdot(Q[-1], w)
        w = w - h * Q[-1] - (beta[-1] * Q[-2] if j > 1 else 0.0)
        alpha.append(float(np.real(h)))
        b = float(np.linalg.norm(w))
        anorm = max(anorm, abs(alpha[-1]) + b + (beta[-1] if beta else 0.0))
        om = omega_next(alpha, beta, b, om_j, om_jm1, anorm)
        q = w / b
        true = np.abs(np.stack(Q, axis=1).conj().T @ q)[:-1] if j > 1 else np.zeros(0)
        est = np.abs(om[:j - 1])
        if j > 1 and est.max() < SQRT_EPS:
            assert true.max() <= 10 * est.max() + 1e-15, (j, true.max(), est.max())
            checked += 1
        if j > 1 and true.max() > SQRT_EPS:
            assert est.max() > 0.1 * SQRT_EPS, (j, true.max(), est.max())
            break
        beta.append(b)
        Q.append(q)
        om_jm1, om_j = om_j, om
    assert checked >= 5


def test_partial_reorth_on_the_tiny_hamiltonian(tiny_model):
    """On Hbar of the tiny system the partial and full variants agree to rounding with
    the same k, and the exact exponential to the tolerance."""
    m = tiny_model
    H = m.hamiltonian(m.v_nuc)
    act = np.concatenate([m.interior, m.mesh.n_nodes + np.arange(m.nk)])
    lam, V = np.linalg.eigh(H[act][:, act].toarray())
    rng = np.random.default_rng(4)
    X = np.zeros((m.n_rows, 2), dtype=np.complex128)
    X[act] = rng.standard_normal((len(act), 2)) + 1j * rng.standard_normal((len(act), 2))
    X /= np.linalg.norm(X, axis=0)
    tau = 0.2
    st = {}
    Yp, kp, _ = lanczos_expm(H, tau, X, tol=1e-10, kmax=200, reorth="partial", stats=st)
    Yf, kf, _ = lanczos_expm(H, tau, X, tol=1e-10, kmax=200, reorth="full")
    exact = np.zeros_like(X)
    exact[act] = V @ (np.exp(-1j * tau * lam)[:, None] * (V.T @ X[act]))
    assert list(kp) == list(kf)
    assert np.max(np.linalg.norm(Yp - Yf, axis=0)) < 1e-13
    assert np.max(np.linalg.norm(Yp - exact, axis=0)) < 10 * 1e-10


def test_lanczos_eigenvector_one_step(tiny_model):
    m = tiny_model
    H = m.hamiltonian(m.v_nuc)
    act = np.concatenate([m.interior, m.mesh.n_nodes + np.arange(m.nk)])
    lam, V = sla.eigh(H[act][:, act].toarray(), subset_by_index=[0, 0])
    x = np.zeros((m.n_rows, 1), dtype=np.complex128)
    x[act, 0] = V[:, 0]
    Y, ks, _ = lanczos_expm(H, 0.3, x, tol=1e-10)
    assert ks[0] == 1
    np.testing.assert_allclose(Y, np.exp(-0.3j * lam[0]) * x, atol=1e-12)


def test_lanczos_kmax_raises(tiny_model):
    m = tiny_model
    H = m.hamiltonian(m.v_nuc)
    rng = np.random.default_rng(1)
    x = np.zeros((m.n_rows, 1), dtype=np.complex128)
    x[m.interior, 0] = rng.standard_normal(len(m.interior))
    with pytest.raises(NoConvergence):
        lanczos_expm(H, 0.5, x, tol=1e-12, kmax=3)


def test_frozen_time_reversibility(tiny_model, tiny_gs):
    m = tiny_model
    H = m.hamiltonian(m.v_nuc + 0.05 * m.qpts[:, 2])
    X0 = tiny_gs["X"]
    X = X0.copy()
    n, tol = 10, 1e-10
    for _ in range(n):
        X, _, _ = lanczos_expm(H, 0.05, X, tol=tol)
    for _ in range(n):
        X, _, _ = lanczos_expm(H, -0.05, X, tol=tol)
    assert np.abs(X - X0).max() < 2 * n * tol


def test_ground_state_is_stationary(tiny_model, tiny_gs):
    m = tiny_model
    X0, eps = tiny_gs["X"], tiny_gs["eps"]
    P = Propagator(m, X0)
    rho0 = P.rho.copy()
    dt, n = 0.05, 3
    for _ in range(n):
        P.step(dt)
    assert np.abs(P.rho - rho0).max() < 1e-8 * np.abs(rho0).max()
    phase = np.exp(-1j * eps * dt * n)
    np.testing.assert_allclose(P.X, X0 * phase[None, :], atol=1e-8)
    G = P.X.conj().T @ P.X
    np.testing.assert_allclose(G, np.eye(2), atol=1e-12)


def test_symmetry_and_linear_response(tiny_model, tiny_gs):
    m = tiny_model
    X0 = tiny_gs["X"]
    assert np.abs(m.dipole(m.density(X0))).max() < 1e-10     # inversion symmetry
    traces = {}
    for kappa in (1e-3, -1e-3, 1e-4):
        P = Propagator(m, X0)
        P.kick(kappa, 2)
        traces[kappa] = np.array([P.step(0.05)[0] for _ in range(3)])
    a, b, c = traces[1e-3], traces[-1e-3], traces[1e-4]
    # odd in the field
    np.testing.assert_allclose(a[:, 2], -b[:, 2], rtol=1e-7, atol=1e-15)
    assert np.abs(a[:, :2]).max() < 1e-12
    # linear response: mu / kappa agrees to O(kappa)
    np.testing.assert_allclose(a[:, 2] / 1e-3, c[:, 2] / 1e-4, rtol=1e-3)
    # orthonormality conserved
    P = Propagator(m, X0)
    P.kick(1e-2, 2)
    for _ in range(3):
        P.step(0.05)
    np.testing.assert_allclose(P.X.conj().T @ P.X, np.eye(2), atol=1e-11)


@pytest.fixture(scope="module")
def trap_setup(golden_dir):
    m = EFEModel(trap(**TRAP_ARGS))
    X0 = np.load(os.path.join(golden_dir, "trap_ground_state.npz"))["X"]
    return m, X0


def test_kohn_theorem_in_trap(trap_setup):
    """Harmonic-potential theorem: mu_z(t) = N kappa sin(w t)/w, with Hartree + Slater."""
    m, X0 = trap_setup
    P = Propagator(m, X0, tol=1e-12)
    kappa, w, N = 1e-3, 1.0, 2.0
    P.kick(kappa, 2)
    ts, mu = [], []
    for _ in range(16):
        mu.append(P.step(0.1)[0][2])
        ts.append(P.t)
    exact = N * kappa * np.sin(w * np.array(ts)) / w
    err = np.abs(np.array(mu) - exact).max() / np.abs(exact).max()
    assert err < 0.05, err        # discretisation-limited (h = 3, p = 4)


def test_second_order_in_dt(trap_setup):
    """Slope of log error vs log dt is 2 (the paper measures 1.99)."""
    m, X0 = trap_setup
    T = 0.8

    def mu_at(dt):
        P = Propagator(m, X0, tol=1e-13, kmax=100)
        P.kick(1e-2, 2)
        for _ in range(int(round(T / dt))):
            mu = P.step(dt)[0]
        return mu[2]

    ref = mu_at(0.0125)
    e = [abs(mu_at(dt) - ref) for dt in (0.2, 0.1)]
    slope = math.log(e[0] / e[1]) / math.log(2.0)
    assert 1.8 < slope < 2.3, (e, slope)


# ---- extrapolated midpoint Hamiltonian (Sec. 2.5, m = 3 previous steps) ----------

def test_extrapolation_weights_reproduce_quadratics():
    """The midpoint value of a quadratic is exact; a cubic leaves an O(dt^3) error."""
    from oracle.propagate import extrapolate_midpoint
    rng = np.random.default_rng(5)
    a, b, c, d = rng.standard_normal((4, 50))
    t, dt = 0.7, 0.05
    quad = lambda s: a + b * s + c * s * s
    hist = [quad(t - 2 * dt), quad(t - dt), quad(t)]
    np.testing.assert_allclose(extrapolate_midpoint(hist), quad(t + 0.5 * dt), rtol=1e-13, atol=1e-13)
    errs = []
    for h in (0.1, 0.05):
        cub = lambda s: d * s ** 3
        e = extrapolate_midpoint([cub(t - 2 * h), cub(t - h), cub(t)]) - cub(t + 0.5 * h)
        errs.append(np.abs(e).max())
    # error of the quadratic through t-2h, t-h, t at t+h/2: f'''/6 (1/2)(3/2)(5/2) h^3 = (15/8) d h^3
    np.testing.assert_allclose(errs[0], 15.0 / 8.0 * np.abs(d).max() * 0.1 ** 3, rtol=1e-10)
    assert 7.9 < errs[0] / errs[1] < 8.1


def test_extrap_starts_with_predictor_corrector_steps(tiny_model, tiny_gs):
    m = tiny_model
    X0 = tiny_gs["X"]
    Pa, Pb = Propagator(m, X0), Propagator(m, X0, scheme="extrap")
    for P in (Pa, Pb):
        P.kick(1e-3, 2)
    for n in range(3):
        ra, rb = Pa.step(0.05), Pb.step(0.05)
        if n < 2:
            assert np.array_equal(Pa.X, Pb.X) and np.all(rb[1] > 0)
        else:
            assert np.all(rb[1] == 0) and not np.array_equal(Pa.X, Pb.X)
            # both are second-order approximations of the same midpoint
            assert abs(ra[0][2] - rb[0][2]) < 1e-3 * abs(ra[0][2])
    # a new dt restarts the history: the next step is again a predictor-corrector step
    assert np.all(Pb.step(0.025)[1] > 0)
    np.testing.assert_allclose(Pb.X.conj().T @ Pb.X, np.eye(2), atol=1e-11)


def test_extrap_kohn_theorem_in_trap(trap_setup):
    m, X0 = trap_setup
    P = Propagator(m, X0, tol=1e-12, scheme="extrap")
    kappa, w, N = 1e-3, 1.0, 2.0
    P.kick(kappa, 2)
    ts, mu = [], []
    for _ in range(16):
        mu.append(P.step(0.1)[0][2])
        ts.append(P.t)
    exact = N * kappa * np.sin(w * np.array(ts)) / w
    err = np.abs(np.array(mu) - exact).max() / np.abs(exact).max()
    assert err < 0.05, err


def test_extrap_second_order_in_dt(trap_setup):
    """Both schemes converge to the same solution; the extrapolated one at order 2."""
    m, X0 = trap_setup
    T = 0.8

    def mu_at(dt, scheme):
        P = Propagator(m, X0, tol=1e-13, kmax=100, scheme=scheme)
        P.kick(1e-2, 2)
        for _ in range(int(round(T / dt))):
            mu = P.step(dt)[0]
        return mu[2]

    ref = mu_at(0.0125, "pc")
    e = [abs(mu_at(dt, "extrap") - ref) for dt in (0.1, 0.05)]
    slope = math.log(e[0] / e[1]) / math.log(2.0)
    assert 1.7 < slope < 2.4, (e, slope)


def test_extrap_second_order_with_field(trap_setup):
    """Field-driven (no kick): the field enters at t + dt/2, so the order stays 2."""
    from oracle.model import Field
    m, X0 = trap_setup
    field = Field(direction=2, A=np.array([0.02]), w=np.array([2.0]), phi=np.array([0.3]), t0=0.4, s=0.5)
    T = 0.8

    def mu_at(dt, scheme):
        P = Propagator(m, X0, tol=1e-13, kmax=100, field=field, scheme=scheme)
        for _ in range(int(round(T / dt))):
            mu = P.step(dt)[0]
        return mu[2]

    ref = mu_at(0.0125, "pc")
    e = [abs(mu_at(dt, "extrap") - ref) for dt in (0.1, 0.05)]
    slope = math.log(e[0] / e[1]) / math.log(2.0)
    assert 1.7 < slope < 2.4, (e, slope)
