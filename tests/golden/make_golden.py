"""Write the stored expected values under tests/golden/ (calls only the oracle).

Usage: python tests/golden/make_golden.py [tiny_gs] [trap_gs] [tiny_traj] [tiny_extrap] [na8] [adjoint_tiny]
       [tiny_graded_gs] [tiny_graded_traj] [na8_graded] [na8_step] [na2_traj]

Every file written here is produced by the FP64 oracle from the seeded inputs of
``workloads``; nothing comes from the GPU library.  Every stored trajectory and
gradient uses the oracle's plain Lanczos scheme (Sec. 2.6, eq. (AdaptiveKrylov):
the three-term step followed by two classical Gram-Schmidt passes against all
previous vectors, reorth="full"), never the partial reorthogonalisation the GPU
library runs by default; the files record the scheme under "lanczos".
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import (tiny, tiny_graded, trap, na8 as na8_spec, na8_graded as na8_graded_spec,  # noqa: E402
                       na_cluster, adjoint_field_params, ADJOINT_TINY)
from oracle.model import EFEModel  # noqa: E402
from oracle.propagate import scf_ground_state, Propagator  # noqa: E402

TRAP_ARGS = dict(omega=1.0, ncell=4, half=6.0, degree=4)


def tiny_gs():
    m = EFEModel(tiny())
    X, eps, it = scf_ground_state(m, tol=1e-11, mix=0.5)
    np.savez_compressed(os.path.join(HERE, "tiny_ground_state.npz"), X=X, eps=eps, iterations=it)
    print("tiny ground state:", eps, it)


def trap_gs():
    m = EFEModel(trap(**TRAP_ARGS))
    X, eps, it = scf_ground_state(m, tol=1e-11, mix=0.5)
    np.savez_compressed(os.path.join(HERE, "trap_ground_state.npz"), X=X, eps=eps, iterations=it)
    print("trap ground state:", eps, it)


def tiny_traj():
    """Kick 1e-3 along z, then 200 Magnus-2 steps of 0.05 au at tol 1e-10."""
    spec = tiny()
    m = EFEModel(spec)
    X0 = np.load(os.path.join(HERE, "tiny_ground_state.npz"))["X"]
    P = Propagator(m, X0, tol=spec.krylov_tol, kmax=spec.kmax, reorth="full")
    mu0 = m.dipole(P.rho)
    k_kick = P.kick(spec.kick, spec.kick_dir)
    mus = [m.dipole(P.rho)]
    ks = []
    t0 = time.time()
    for n in range(spec.nsteps):
        mu, kp, kc = P.step(spec.dt)
        mus.append(mu)
        ks.append(np.stack([kp, kc]))
        if n % 20 == 0:
            print(f"step {n} mu_z={mu[2]:.6e} k={kp},{kc} ({time.time() - t0:.0f}s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "tiny_traj.npz"), mu_ground=mu0, mu=np.array(mus),
                        k=np.array(ks, dtype=np.int32), k_kick=k_kick, X_final=P.X,
                        rho_final=P.rho, dt=spec.dt, kick=spec.kick, lanczos="full")


def tiny_extrap():
    """Kick 1e-3 along z, then 100 steps of 0.05 au with the midpoint Hamiltonian
    extrapolated from the last three steps (the first two steps predictor-corrector)."""
    spec = tiny()
    m = EFEModel(spec)
    X0 = np.load(os.path.join(HERE, "tiny_ground_state.npz"))["X"]
    P = Propagator(m, X0, tol=spec.krylov_tol, kmax=spec.kmax, scheme="extrap", reorth="full")
    k_kick = P.kick(spec.kick, spec.kick_dir)
    mus = [m.dipole(P.rho)]
    ks = []
    t0 = time.time()
    for n in range(100):
        mu, kp, kc = P.step(spec.dt)
        mus.append(mu)
        ks.append(np.stack([kp, kc]))
        if n % 20 == 0:
            print(f"step {n} mu_z={mu[2]:.6e} k={kp},{kc} ({time.time() - t0:.0f}s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "tiny_extrap.npz"), mu=np.array(mus), k=np.array(ks, dtype=np.int32),
                        k_kick=k_kick, X_final=P.X, dt=spec.dt, kick=spec.kick, lanczos="full")


def tiny_graded_gs():
    m = EFEModel(tiny_graded())
    X, eps, it = scf_ground_state(m, tol=1e-11, mix=0.5)
    np.savez_compressed(os.path.join(HERE, "tiny_graded_ground_state.npz"), X=X, eps=eps, iterations=it)
    print("tiny_graded ground state:", eps, it)


def tiny_graded_traj():
    """The tiny system on its graded mesh: kick 1e-3 along z, then 50 Magnus-2 steps of 0.05 au."""
    spec = tiny_graded()
    m = EFEModel(spec)
    X0 = np.load(os.path.join(HERE, "tiny_graded_ground_state.npz"))["X"]
    P = Propagator(m, X0, tol=spec.krylov_tol, kmax=spec.kmax, reorth="full")
    k_kick = P.kick(spec.kick, spec.kick_dir)
    mus = [m.dipole(P.rho)]
    ks = []
    for n in range(50):
        mu, kp, kc = P.step(spec.dt)
        mus.append(mu)
        ks.append(np.stack([kp, kc]))
    np.savez_compressed(os.path.join(HERE, "tiny_graded_traj.npz"), mu=np.array(mus),
                        k=np.array(ks, dtype=np.int32), k_kick=k_kick, X_final=P.X, dt=spec.dt, kick=spec.kick,
                        lanczos="full")
    print("tiny_graded trajectory: mu_z(50) =", mus[-1][2])


def na8(spec=None, name="na8_sampled.npz"):
    """Na8 reference values at sampled rows/points for the full-size GPU parity test.

    Initial orbitals X0 (enrichment directions + seeded noise, Loewdin
    orthonormalised), rho(X0) at sampled quadrature points, the dipole, the
    Hartree potential at sampled nodes, and (Hbar[rho(X0), t=0] X0) at sampled
    node rows and at every enrichment row.
    """
    spec = na8_spec() if spec is None else spec
    t0 = time.time()
    m = EFEModel(spec)
    print(f"na8 model {time.time() - t0:.0f}s", flush=True)
    X0 = m.enrichment_noise_state()
    print(f"initial state {time.time() - t0:.0f}s", flush=True)
    rho = m.density(X0)
    mu = m.dipole(rho)
    print(f"density {time.time() - t0:.0f}s  mu={mu}", flush=True)
    phi = m.hartree(rho, solver="fdm")
    v = m.ks_potential(rho, m.interpolate_nodal(phi), 0.0, None)
    print(f"hartree {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(2024)
    N = m.mesh.n_nodes
    near = np.nonzero(np.any(m.c != 0.0, axis=1))[0]
    rows = np.unique(np.concatenate([rng.choice(m.interior, 96, replace=False), rng.choice(near, 96, replace=False)]))
    Yr, YE = m.hamiltonian_rows(v, X0, rows)
    print(f"Hbar rows {time.time() - t0:.0f}s", flush=True)
    q_idx = np.sort(rng.choice(m.mesh.n_quad, 8192, replace=False))
    ph_idx = np.sort(rng.choice(N, 2048, replace=False))
    np.savez_compressed(os.path.join(HERE, name), rows=rows, X0_rows=X0[rows], X0_E=X0[N:],
                        Y_rows=Yr, Y_E=YE, q_idx=q_idx, rho_q=rho[q_idx], rho_sum=float(np.sum(m.qw * rho)),
                        mu=mu, phi_idx=ph_idx, phi=phi[ph_idx], nk=m.nk)
    print("na8 done", flush=True)


def na8_graded():
    """The same sampled values for Na8 in its 70-bohr box on the sinh-graded mesh."""
    na8(na8_graded_spec(), "na8_graded_sampled.npz")


def cluster_steps(spec, nsteps, name):
    """Kicked Magnus-2 steps of a sodium cluster by the oracle's matrix-free route
    (cell blocks and coupling applied without assembly, Lanczos columns advanced
    together, Hartree by fast diagonalisation; the plain Lanczos scheme).

    Stores the dipole before and after the kick and after every step, the Krylov
    dimension of every column (kick, predictor, corrector), and the orbitals at
    sampled node rows and at every enrichment row after the kick and each step."""
    t0 = time.time()
    m = EFEModel(spec)
    print(f"{name}: model {time.time() - t0:.0f}s", flush=True)
    X0 = m.enrichment_noise_state()
    P = Propagator(m, X0, tol=spec.krylov_tol, kmax=spec.kmax, reorth="full", matrix_free=True, block_cols=11)
    mu0 = m.dipole(P.rho)
    print(f"{name}: initial state and Hamiltonian {time.time() - t0:.0f}s  mu0={mu0}", flush=True)
    k_kick = P.kick(spec.kick, spec.kick_dir)
    N = m.mesh.n_nodes
    rng = np.random.default_rng(2025)
    near = np.nonzero(np.any(m.c != 0.0, axis=1))[0]
    rows = np.unique(np.concatenate([rng.choice(m.interior, 64, replace=False), rng.choice(near, 64, replace=False)]))
    mus, ks, Xr, XE, secs = [m.dipole(P.rho)], [], [P.X[rows]], [P.X[N:]], []
    print(f"{name}: kick k={k_kick} {time.time() - t0:.0f}s  mu={mus[-1]}", flush=True)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except ImportError:
        threads = os.cpu_count()
    cpu = "unknown"
    with open("/proc/cpuinfo") as f:
        for line in f:
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    for n in range(nsteps):
        ts = time.time()
        mu, kp, kc = P.step(spec.dt)
        secs.append(time.time() - ts)
        mus.append(mu)
        ks.append(np.stack([kp, kc]))
        Xr.append(P.X[rows])
        XE.append(P.X[N:])
        print(f"{name}: step {n} k={kp},{kc} {time.time() - t0:.0f}s  mu={mu}", flush=True)
        # written after every step: the steps done so far are kept if a later one is cut short
        np.savez_compressed(os.path.join(HERE, name), mu_ground=mu0, mu=np.array(mus),
                            k=np.array(ks, dtype=np.int32), k_kick=k_kick, rows=rows, X_rows=np.array(Xr),
                            X_E=np.array(XE), dt=spec.dt, kick=spec.kick, kick_dir=spec.kick_dir, lanczos="full",
                            step_seconds=np.array(secs), threads=threads, cpu_model=cpu)
    print(f"{name}: done {time.time() - t0:.0f}s", flush=True)


def na8_step():
    """Na8 (the benchmark system): z kick 1e-3 and two Magnus-2 steps of 0.02 au."""
    cluster_steps(na8_spec(), 2, "na8_step.npz")


def na2_traj():
    """Na2 (seed 2; a member of the batched workload): x kick 1e-3 and ten steps."""
    cluster_steps(na_cluster(2, seed=2, kick=1e-3, kick_dir=0), 10, "na2_traj.npz")


def adjoint_tiny():
    """Field-parameter gradient on the tiny system (oracle central differences, k replayed)."""
    from oracle.adjoint import fd_gradient, run_dipole, field_from_params
    cfg = ADJOINT_TINY
    m = EFEModel(tiny())
    X0 = np.load(os.path.join(HERE, "tiny_ground_state.npz"))["X"]
    theta = adjoint_field_params(cfg["seed"], cfg["ncomp"])
    theta_star = adjoint_field_params(cfg["seed_target"], cfg["ncomp"])
    t0 = time.time()
    mus_star, _ = run_dipole(m, X0, field_from_params(theta_star, cfg["t0"], cfg["s"]), cfg["dt"], cfg["nsteps"])
    mu_target = mus_star[:, 2]
    print(f"target run {time.time() - t0:.0f}s", flush=True)
    g, L, mus, ks = fd_gradient(m, X0, theta, cfg["t0"], cfg["s"], cfg["dt"], cfg["nsteps"], mu_target)
    print(f"gradient {time.time() - t0:.0f}s  L={L:.6e}  g={g}", flush=True)
    np.savez_compressed(os.path.join(HERE, "adjoint_tiny.npz"), theta=theta, theta_star=theta_star,
                        mu_target=mu_target, mus=mus, L=L, g_fd=g, ks=np.asarray(ks, dtype=np.int32), h=1e-6,
                        lanczos="full")


if __name__ == "__main__":
    jobs = sys.argv[1:] or ["tiny_gs", "trap_gs", "tiny_traj"]
    for j in jobs:
        globals()[j]()
