"""The captured step (magnus_step_graph: device-driven Lanczos with a fixed trip
count, replayed from a hipGraph) against the host-driven step on systems
outside the workloads' shapes: the tiny system at degree 6, with 60 orbitals
and on 1 x 2 x 5 cells, and lattice13 (52 enrichment functions).

Two contexts start from the same seeded orthonormal block; four steps each,
one host-driven and one replayed, with eager library and torch work between
the replays: identical Krylov dimensions and CG iteration counts, orbitals
and dipoles within 1e-12.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _spec(case):
    from workloads import tiny, lattice13
    if case == "degree6":
        return dataclasses.replace(tiny(), degree=6)
    if case == "orbitals60":
        return dataclasses.replace(tiny(), occ=np.concatenate([[2.0, 1.0], np.zeros(58)]))
    if case == "thin":
        return dataclasses.replace(tiny(), ncell=(1, 2, 5))
    return lattice13()


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("case", ["degree6", "lattice13", "orbitals60", "thin"])
def test_graph_step_matches_host_step(case):
    from oracle.fe import Mesh
    from paper_2210_14421_amd.efe import Context
    spec = _spec(case)
    print(f"{case}: graph vs host step", flush=True)
    ca, cb = Context(spec, kmax=40), Context(spec, kmax=40)
    try:
        n, N = ca.n_rows, ca.n_nodes
        mesh = Mesh(spec.ncell, spec.lo, spec.hi, spec.degree)
        act = np.concatenate([np.nonzero(~mesh.boundary_mask())[0], N + np.arange(n - N)])
        rng = np.random.default_rng(5)
        Z = rng.standard_normal((len(act), spec.norb)) + 1j * rng.standard_normal((len(act), spec.norb))
        X0 = np.zeros((n, spec.norb), dtype=np.complex128)
        X0[act] = np.linalg.qr(Z)[0]
        Pa = torch.from_numpy(X0).to("cuda")
        Pb = Pa.clone()
        ca.set_hamiltonian(Pa, 0.0)
        cb.set_hamiltonian(Pb, 0.0)
        t = 0.0
        for step in range(4):
            sa = ca.magnus_step(Pa, t, spec.dt)
            sb = cb.magnus_step(Pb, t, spec.dt, graph=True)
            t += spec.dt
            assert list(sa["k_pred"]) == list(sb["k_pred"]) and list(sa["k_corr"]) == list(sb["k_corr"])
            assert sa["cg_iters"] == sb["cg_iters"]
            e = _rel(Pb, Pa)
            dmu = float(np.max(np.abs(sb["mu"] - sa["mu"])) / np.max(np.abs(sa["mu"])))
            print(f"{case} step {step}: k {sorted(set(sb['k_corr'].tolist()))} |dPsi| {e:.1e} |dmu| {dmu:.1e}",
                  flush=True)
            assert e < 1e-12 and dmu < 1e-12
            np.testing.assert_allclose(cb.dipole(Pb), sb["mu"], rtol=1e-12, atol=1e-14)
            _ = (Pb.real * 2.0).sum().item()
    finally:
        ca.close()
        cb.close()
