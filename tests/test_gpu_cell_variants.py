"""Every dense kernel shape of the cell products gives the same bits.

The autotuner picks one shape per problem; all shapes (chunks in flight, k-rows per
chunk, register budget, 64- and 32-column workgroups, sixteen-wave workgroups for FP32
blocks; for BF16 blocks eight or twelve waves, two or three stages of block rows, block
rows through LDS copies or through registers) add
the k terms of each output in the same order, so each must reproduce the default
shape's Hbar X bit for bit.  Each shape is selected through the autotuner's
cache (a forced run writes the problem's entry; the test rewrites its choice and a fresh
context reads it back).  Systems: tiny (125-node cells) with 3 orbitals and Na2 (216-node
cells) with its 11; FP64, FP32, BF16 and split BF16 blocks (the reduced-precision ones on
the FP32 / BF16 rows of the propagation).
"""
import dataclasses
import json
import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _boundary(spec):
    nn = [spec.ncell[d] * spec.degree + 1 for d in range(3)]
    g = np.arange(nn[0] * nn[1] * nn[2])
    ix, iy, iz = g % nn[0], (g // nn[0]) % nn[1], g // (nn[0] * nn[1])
    return (ix == 0) | (ix == nn[0] - 1) | (iy == 0) | (iy == nn[1] - 1) | (iz == 0) | (iz == nn[2] - 1)


def _block(ctx, spec, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ctx.n_rows, spec.norb)) + 1j * rng.standard_normal((ctx.n_rows, spec.norb))
    X[:ctx.n_nodes][_boundary(spec)] = 0.0
    X /= np.linalg.norm(X, axis=0)
    return torch.from_numpy(X).to("cuda")


def _systems():
    from workloads import tiny, na_cluster
    return [("tiny", dataclasses.replace(tiny(), occ=np.array([2.0, 1.0, 1.0]))), ("Na2", na_cluster(2, seed=2))]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("which", [0, 1])
def test_every_dense_shape_same_bits(dtype, which, tmp_path):
    from paper_2210_14421_amd.efe import Context
    name, spec = _systems()[which]
    cache = tmp_path / "tune.json"
    base = Context(spec, dtype=dtype, kmax=8)
    try:
        X, B = _block(base, spec, 1), _block(base, spec, 2)
        base.set_hamiltonian(X, 0.0)
        Yref = base.apply_H(B)
        r = base.autotune(cache=cache, force=True)
        shapes = [n for n in sorted(r["times_us"]) if n != "sum_factorised"]
        print(f"{name} {dtype}: {r['times_us']}", flush=True)
        if dtype == "f32":
            assert any(n.endswith("_16w") for n in shapes)
        if dtype == "bf16":
            assert sum(n.endswith("_a3") for n in shapes) == 2 and sum(n.endswith("_ra") for n in shapes) == 2
        text = cache.read_text()
        assert len(json.loads(text)) == 1
        for shape in shapes:
            cache.write_text(re.sub(r'"choice": "[^"]*"', f'"choice": "{shape}"', text))
            ctx = Context(spec, dtype=dtype, kmax=8)
            try:
                ctx.set_hamiltonian(X, 0.0)
                r2 = ctx.autotune(cache=cache)
                assert r2["cached"] and r2["choice"] == shape
                Y = ctx.apply_H(B)
                torch.cuda.synchronize()
                print(f"{name} {dtype}: {shape}: equal {torch.equal(Y, Yref)}", flush=True)
                assert torch.equal(Y, Yref)
            finally:
                ctx.close()
    finally:
        base.close()
