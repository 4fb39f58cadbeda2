"""Device-driven, graph-captured Magnus steps and batched propagations (GPU).

The captured step runs the same kernels as magnus_step with the stopping
decisions taken on the device, so each replay must reproduce the host-driven
step: same Krylov dimension per column, orbitals and dipole to rounding.  The
graph is replayed several times with eager library and torch work in between,
and every replay is checked.  A batch steps independent systems (different
kick directions, and a second mesh) as concurrent branches of one graph; each
member must match the same system stepped alone.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def tiny_gs(golden_dir):
    return np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]


def _kicked(ctx, X0, direction="z", kick=1e-3):
    Psi = _dev(X0)
    ctx.lanczos_expm(Psi, -kick, op=direction)
    ctx.set_hamiltonian(Psi, 0.0)
    return Psi


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def test_graph_step_matches_host_step(tiny_gs):
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    print("tiny graph vs host step", flush=True)
    ca, cb = Context(spec, kmax=40), Context(spec, kmax=40)
    try:
        Pa, Pb = _kicked(ca, tiny_gs), _kicked(cb, tiny_gs)
        t = 0.0
        for n in range(6):
            sa = ca.magnus_step(Pa, t, spec.dt)
            sb = cb.magnus_step(Pb, t, spec.dt, graph=True)
            t += spec.dt
            assert list(sa["k_pred"]) == list(sb["k_pred"]) and list(sa["k_corr"]) == list(sb["k_corr"])
            assert sa["cg_iters"] == sb["cg_iters"]
            e = _rel(Pb, Pa)
            dmu = np.max(np.abs(sb["mu"] - sa["mu"])) / np.max(np.abs(sa["mu"]))
            print(f"step {n}: k {sb['k_pred']} {sb['k_corr']} |dPsi| {e:.2e} |dmu| {dmu:.2e}", flush=True)
            assert e < 1e-12 and dmu < 1e-12
            # eager work between replays: library calls on the graph's context and plain torch work
            mu_eager = cb.dipole(Pb)
            np.testing.assert_allclose(mu_eager, sb["mu"], rtol=1e-12, atol=1e-14)
            _ = (Pb.real * 2.0).sum().item()
    finally:
        ca.close()
        cb.close()


def test_graph_recaptures_on_new_block(tiny_gs):
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    ca, cb = Context(spec, kmax=40), Context(spec, kmax=40)
    try:
        Pa, Pb = _kicked(ca, tiny_gs), _kicked(cb, tiny_gs)
        ca.magnus_step(Pa, 0.0, spec.dt)
        cb.magnus_step(Pb, 0.0, spec.dt, graph=True)
        Pb2 = Pb.clone()                      # different pointer: the step is captured again
        cb.set_hamiltonian(Pb2, spec.dt)
        ca.set_hamiltonian(Pa, spec.dt)
        sa = ca.magnus_step(Pa, spec.dt, spec.dt)
        sb = cb.magnus_step(Pb2, spec.dt, spec.dt, graph=True)
        assert list(sa["k_corr"]) == list(sb["k_corr"])
        assert _rel(Pb2, Pa) < 1e-12
    finally:
        ca.close()
        cb.close()


def test_graph_recaptures_after_new_options(tiny_gs):
    """A captured step holds its Krylov settings: after set_options (here the full
    reorthogonalisation and a tighter tolerance) the next graph step is recorded
    again and equals a host-driven step with the new settings."""
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    ca, cb = Context(spec, kmax=40, reorth="full", tol=1e-12), Context(spec, kmax=40)
    try:
        Pa, Pb = _kicked(ca, tiny_gs), _kicked(cb, tiny_gs)
        cb.magnus_step(Pb, 0.0, spec.dt, graph=True)          # captured with the default settings
        cb.set_options(reorth="full", tol=1e-12)
        Pb2 = _kicked(cb, tiny_gs)
        Pb.copy_(Pb2)
        cb.set_hamiltonian(Pb, 0.0)
        sa = ca.magnus_step(Pa, 0.0, spec.dt)
        sb = cb.magnus_step(Pb, 0.0, spec.dt, graph=True)
        assert list(sa["k_pred"]) == list(sb["k_pred"]) and list(sa["k_corr"]) == list(sb["k_corr"])
        assert _rel(Pb, Pa) < 1e-12
    finally:
        ca.close()
        cb.close()


def test_batch_matches_members_alone(tiny_gs):
    from workloads import tiny, trap
    from paper_2210_14421_amd.efe import Context, Batch
    spec = tiny()
    tspec = trap(omega=1.0, ncell=4, half=6.0, degree=4)
    dirs = ["x", "y", "z"]
    print("batch: tiny x/y/z kicks + harmonic trap", flush=True)
    alone = [Context(spec, kmax=40) for _ in dirs] + [Context(tspec, kmax=40)]
    members = [Context(spec, kmax=40) for _ in dirs] + [Context(tspec, kmax=40)]
    batch = None
    try:
        Xt = np.load(os.path.join(os.path.dirname(__file__), "golden", "trap_ground_state.npz"))["X"]
        assert Xt.shape == (alone[3].n_rows, tspec.norb)
        P_alone = [_kicked(c, tiny_gs, d) for c, d in zip(alone[:3], dirs)] + [_kicked(alone[3], Xt, "z")]
        P_mem = [_kicked(c, tiny_gs, d) for c, d in zip(members[:3], dirs)] + [_kicked(members[3], Xt, "z")]
        batch = Batch(members)
        t = 0.0
        for n in range(4):
            ref = [c.magnus_step(P, t, spec.dt) for c, P in zip(alone, P_alone)]
            got = batch.step(P_mem, t, spec.dt)
            t += spec.dt
            for i in range(4):
                assert list(ref[i]["k_pred"]) == list(got[i]["k_pred"])
                assert list(ref[i]["k_corr"]) == list(got[i]["k_corr"])
                e = _rel(P_mem[i], P_alone[i])
                print(f"step {n} member {i}: |dPsi| {e:.2e}", flush=True)
                assert e < 1e-12
                np.testing.assert_allclose(got[i]["mu"], ref[i]["mu"], rtol=1e-11, atol=1e-14)
            _ = sum(float(P.abs().sum()) for P in P_mem)   # eager work between replays
    finally:
        if batch is not None:
            batch.close()
        for c in alone + members:
            c.close()


def test_batch_recaptures_after_member_options(tiny_gs):
    """A batch graph holds every member's Krylov settings: after set_options on one
    member (full reorthogonalisation, tighter tolerance) the next batch step is
    recorded again and that member equals its host-driven step with the new
    settings, while the other member is unchanged."""
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context, Batch
    spec = tiny()
    print("batch re-capture after set_options", flush=True)
    ref_new = Context(spec, kmax=40, reorth="full", tol=1e-12)
    ref_old = Context(spec, kmax=40)
    members = [Context(spec, kmax=40), Context(spec, kmax=40)]
    batch = None
    try:
        Pn, Po = _kicked(ref_new, tiny_gs, "z"), _kicked(ref_old, tiny_gs, "x")
        P_mem = [_kicked(members[0], tiny_gs, "z"), _kicked(members[1], tiny_gs, "x")]
        batch = Batch(members)
        batch.step(P_mem, 0.0, spec.dt)                       # captured with the default settings
        ref_old.magnus_step(Po, 0.0, spec.dt)
        members[0].set_options(reorth="full", tol=1e-12)
        P_mem[0].copy_(_kicked(members[0], tiny_gs, "z"))
        members[0].set_hamiltonian(P_mem[0], 0.0)
        got = batch.step(P_mem, 0.0, spec.dt)                 # no field: t enters nothing
        sn = ref_new.magnus_step(Pn, 0.0, spec.dt)
        assert list(got[0]["k_pred"]) == list(sn["k_pred"]) and list(got[0]["k_corr"]) == list(sn["k_corr"])
        e0 = _rel(P_mem[0], Pn)
        print(f"member 0 (new settings): k {got[0]['k_corr']} |dPsi| {e0:.2e}", flush=True)
        assert e0 < 1e-12
        so = ref_old.magnus_step(Po, spec.dt, spec.dt)
        assert list(got[1]["k_corr"]) == list(so["k_corr"])
        e1 = _rel(P_mem[1], Po)
        print(f"member 1 (old settings): |dPsi| {e1:.2e}", flush=True)
        assert e1 < 1e-12
    finally:
        if batch is not None:
            batch.close()
        for c in members + [ref_new, ref_old]:
            c.close()


def test_graph_step_na8():
    """One captured step at the full Na8 size equals the host-driven step."""
    from workloads import na8
    from paper_2210_14421_amd.efe import Context
    spec = na8()
    print("na8 graph vs host step", flush=True)
    ca, cb = Context(spec, kmax=24), Context(spec, kmax=24)
    try:
        Pa = ca.initial_state()
        Pb = cb.initial_state()
        for c, P in ((ca, Pa), (cb, Pb)):
            c.lanczos_expm(P, -spec.kick, op="z")
            c.set_hamiltonian(P, 0.0)
        for n in range(2):
            sa = ca.magnus_step(Pa, n * spec.dt, spec.dt)
            sb = cb.magnus_step(Pb, n * spec.dt, spec.dt, graph=True)
            assert list(sa["k_pred"]) == list(sb["k_pred"]) and list(sa["k_corr"]) == list(sb["k_corr"])
            e = _rel(Pb, Pa)
            print(f"Na8 step {n}: |dPsi| {e:.2e}", flush=True)
            assert e < 1e-12
            np.testing.assert_allclose(sb["mu"], sa["mu"], rtol=1e-12)
    finally:
        ca.close()
        cb.close()
