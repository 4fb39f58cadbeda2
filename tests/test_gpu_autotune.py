"""Autotuner of the cell products (efe_autotune, GPU).

Every dense kernel shape adds the k terms of a cell product in the same order, so
the tuned context must give the same bits as the default one: Hbar X and a whole
Magnus step are compared bit for bit (sum factorisation, when chosen for FP64
blocks, within 1e-12).  The choice is written to a JSON cache and a second
context of the same system takes it from there without timing; a forced run
times again.  On Na8 the table of every block type is printed.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _kicked(ctx, spec, X0):
    Psi = torch.from_numpy(np.ascontiguousarray(X0)).cuda()
    ctx.lanczos_expm(Psi, -spec.kick, op="z")
    ctx.set_hamiltonian(Psi, 0.0)
    return Psi


def test_autotune_tiny_same_bits_and_cache(tmp_path, golden_dir):
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context
    spec = tiny()
    X0 = np.load(os.path.join(golden_dir, "tiny_ground_state.npz"))["X"]
    cache = tmp_path / "tune.json"
    print("autotune: tiny FP64", flush=True)
    ca, cb, cc = Context(spec, kmax=40), Context(spec, kmax=40), Context(spec, kmax=40)
    try:
        Pa, Pb = _kicked(ca, spec, X0), _kicked(cb, spec, X0)
        Ya = ca.apply_H(Pa)
        r = cb.autotune(cache=cache)
        print(f"tiny: {r}", flush=True)
        assert not r["cached"] and len(r["times_us"]) >= 2 and r["choice"] in r["times_us"] and not r["rejected"]
        Yb = cb.apply_H(Pb)
        sf = r["choice"] == "sum_factorised"
        if sf:
            assert float((Yb - Ya).abs().max() / Ya.abs().max()) < 1e-12
        else:
            assert torch.equal(Yb, Ya)
        sa = ca.magnus_step(Pa, 0.0, spec.dt)
        sb = cb.magnus_step(Pb, 0.0, spec.dt)
        assert list(sa["k_corr"]) == list(sb["k_corr"])
        if not sf:
            assert torch.equal(Pa, Pb)
        # the cache: one entry, read back by a second context without timing
        entries = json.loads(cache.read_text())
        assert len(entries) == 1 and list(entries.values())[0]["choice"] == r["choice"]
        _kicked(cc, spec, X0)
        r2 = cc.autotune(cache=cache)
        assert r2["cached"] and r2["choice"] == r["choice"] and not r2["times_us"]
        r3 = cc.autotune(cache=cache, force=True)
        assert not r3["cached"] and len(json.loads(cache.read_text())) == 1
    finally:
        for c in (ca, cb, cc):
            c.close()


def test_autotune_needs_hamiltonian():
    from workloads import tiny
    from paper_2210_14421_amd.efe import Context, EfeError, EFE_ERR_STATE
    ctx = Context(tiny(), kmax=8)
    try:
        with pytest.raises(EfeError) as e:
            ctx.autotune()
        assert e.value.status == EFE_ERR_STATE
    finally:
        ctx.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16x3"])
def test_autotune_na8(dtype, tmp_path):
    from workloads import na8
    from paper_2210_14421_amd.efe import Context
    spec = na8()
    print(f"autotune: Na8 {dtype}", flush=True)
    ca, cb = Context(spec, dtype=dtype, kmax=20), Context(spec, dtype=dtype, kmax=20)
    try:
        Pa, Pb = ca.initial_state(), cb.initial_state()
        for c, P in ((ca, Pa), (cb, Pb)):
            c.lanczos_expm(P, -spec.kick, op="z")
            c.set_hamiltonian(P, 0.0)
        r = cb.autotune(cache=tmp_path / "tune.json")
        table = ", ".join(f"{k} {v:.0f} us" for k, v in sorted(r["times_us"].items(), key=lambda kv: kv[1]))
        print(f"Na8 {dtype}: choice {r['choice']}; per Hbar X (cell part): {table}", flush=True)
        assert not r["rejected"]
        sa = ca.magnus_step(Pa, 0.0, spec.dt)
        sb = cb.magnus_step(Pb, 0.0, spec.dt)
        assert list(sa["k_corr"]) == list(sb["k_corr"])
        if r["choice"] == "sum_factorised":
            assert float((Pb - Pa).abs().max()) < 1e-11
        else:
            assert torch.equal(Pa, Pb)
    finally:
        ca.close()
        cb.close()
