"""Benchmark: Magnus-2 steps/s on the Na8 workload on one MI355X.

Workload (one GPU): 8 Na atoms at seeded positions in a ball of radius 6 bohr,
box [-20, 20]^3 with 24^3 cells of degree 5 (1,771,561 nodes), 48 enrichment
functions, 44 doubly occupied orbitals from enrichment directions plus seeded
low-frequency noise, ALDA (Slater + PW92), z kick 1e-3, dt = 0.02 au, Lanczos
tolerance 1e-10.  A step is one full predictor-corrector Magnus-2 step (two
adaptive Lanczos exponentials, two densities, two Poisson solves, two
Hamiltonian rebuilds, one dipole), orbitals resident in HBM.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Magnus steps/s at Na8 (44 orbitals) + H.X roofline fraction, mixed vs plain FP64"
HBM_GBS = 8000.0


TUNE_CACHE = os.environ.get("EFE_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "efe_tune.json"))


def run_gpu(spec, dtype, steps, warmup, kmax, scheme="pc", reorth="partial", autotune=True):
    import numpy as np
    import torch
    from paper_2210_14421_amd.efe import Context
    t0 = time.time()
    ctx = Context(spec, dtype=dtype, kmax=kmax, reorth=reorth)
    Psi = ctx.initial_state()
    ctx.lanczos_expm(Psi, -spec.kick, op="z")
    ctx.set_hamiltonian(Psi, 0.0)
    tune = ctx.autotune(cache=TUNE_CACHE) if autotune else None
    if tune is not None:
        print(f"[bench] {dtype}: autotuned cell products: {tune}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    print(f"[bench] {dtype}: setup + initial state + kick {setup_s:.1f} s", file=sys.stderr, flush=True)
    t = 0.0
    # the extrapolated scheme needs three densities of the step: its first two steps are warm-up
    for i in range(max(warmup, 2) if scheme == "extrap" else warmup):
        ctx.magnus_step(Psi, t, spec.dt, scheme=scheme, keep_ham=False)
        t += spec.dt
    ctx.enable_timing(True)
    stage = {}
    ks = []
    mus = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        st = ctx.magnus_step(Psi, t, spec.dt, scheme=scheme, keep_ham=False)
        t += spec.dt
        tm = ctx.timing()
        for k, v in tm.items():
            stage[k] = stage.get(k, 0) + v
        ks.append((float(np.mean(st["k_pred"])), float(np.mean(st["k_corr"]))))
        mus.append(st["mu"].tolist())
        print(f"[bench] {dtype} {scheme} step {i}: mu_z={st['mu'][2]:.9e} k={ks[-1]} total {tm['total']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    G = Psi.conj().T @ Psi
    orth = float((G - torch.eye(spec.norb, dtype=G.dtype, device=G.device)).abs().max())
    dims = dict(n_union_rows=ctx.n_union_rows, n_kept=ctx.n_kept)
    ctx.close()
    return dict(wall=wall, stage=stage, k=ks, mu=mus, orth=orth, setup_s=setup_s, tune=tune, dims=dims)


def traffic_summary(dtype):
    """HBM traffic of one cell-product launch from the committed rocprofv3 summary.

    The summary records FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by
    the same counter's reading for a plain copy of known size, and the sha256 of
    the kernel source it was taken with; it is used only while that source is
    unchanged (otherwise traffic is reported as null)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "cell_apply_na8_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in ("kernels_cell.hip", "kernels_cell_bf16.hip"):
        with open(os.path.join(ROOT, "paper_2210_14421_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    if rec.get("kernel_source_sha256") != sha or dtype not in rec.get("per_launch_bytes", {}):
        return None
    b = rec["per_launch_bytes"][dtype]
    return {"total": b["fetch"] + b["write"], "fetch": b["fetch"], "write": b["write"],
            "algorithmic": b.get("algorithmic"), "source": os.path.relpath(path, ROOT)}


def run_apply_mode(spec, dtype, n_apply):
    """Counter-collection workload: Na8 set-up, n_apply Hbar X in the form the
    propagation runs them, then a 1 GiB copy (the calibration kernel of known size
    for FETCH_SIZE / WRITE_SIZE).  With FP64 blocks that form is a Lanczos run with
    k = n_apply (the cell kernel then also sums each cell's share of x^H Hbar x);
    otherwise efe_apply_H, which runs the same kernels as the propagation."""
    import numpy as np
    import torch
    from paper_2210_14421_amd.efe import Context
    # FP64: kmax = k, so that no iteration past the last is enqueued (its kernels would
    # return at once and count as launches)
    ctx = Context(spec, dtype=dtype, kmax=n_apply if dtype == "f64" else 4)
    Psi = ctx.initial_state()
    ctx.set_hamiltonian(Psi, 0.0)
    tune = ctx.autotune(cache=TUNE_CACHE)        # the kernel shape the timed steps use
    print(f"[bench] apply {dtype}: {tune}", file=sys.stderr, flush=True)
    if dtype == "f64":
        ctx.lanczos_expm(Psi, spec.dt, k_force=np.full(spec.norb, n_apply, dtype=np.int32))
    else:
        Y = torch.empty_like(Psi)
        for _ in range(n_apply):
            ctx.apply_H(Psi, Y)
    a = torch.full((1 << 27,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"mode": "apply", "dtype": dtype, "n_apply": n_apply, "calibration_copy_bytes": a.numel() * 8}))


# arithmetic each stored-block type is multiplied in: the MFMA peak of that instruction
MFMA_OF = {"f64": ("f64", 78.6), "f32": ("f32", 157.3), "bf16": ("bf16", 2500.0), "bf16x3": ("bf16", 2500.0 / 3)}
BLOCK_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "bf16x3": 4}
# bytes per real element of the orbital rows the cell products read (X: the FP64 Lanczos
# vector, or its FP32 / BF16 copy) and write (Y: FP64, or the FP32 product block)
X_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "bf16x3": 4}
Y_BYTES = {"f64": 8, "f32": 4, "bf16": 4, "bf16x3": 4}


def roofline(spec, res, dtype):
    """Cell-product kernel against the lower of its roofs, per Hbar X.

    One Hbar X is one launch per cell colour (parity class); the launches multiply
    the nloc x nloc blocks of every cell into the 2 N_orb real columns of the
    orbital block: 2 nloc^2 (2 N_orb) flops per cell.  Algorithmic bytes of one
    Hbar X are the unique ones: the orbital block read once, the result written
    once and every stored block read once (the gathers of nodes shared between
    cells and the read-modify-write of later colours are not algorithmic).  The
    roof is the MFMA peak of the instruction the blocks are multiplied with, or the
    arithmetic intensity times the HBM bandwidth, whichever is lower; the achieved
    figure is flops or unique bytes over the time of all colour launches of one
    Hbar X (HIP events of the library on its stream).  The per-launch figures with
    the gathered bytes are kept as secondary keys, and so is the stricter fraction
    on the kernel's own unique bytes (reduced-precision products read an FP32 or
    BF16 copy of X and write an FP32 Y, fewer bytes than the FP64 rows counted
    above).  With FP64 blocks the kernel of the propagation also leaves each cell's
    share of the Lanczos coefficient x^H Hbar x (it reads the cell's X rows again), in
    place of a dot pass over two orbital blocks per Lanczos step; the same shape without
    that work, as the autotuner timed it live before the steps, is kept under apply_only."""
    P = spec.degree + 1
    nloc = P ** 3
    ncells = spec.ncell[0] * spec.ncell[1] * spec.ncell[2]
    ncolour = 1
    for n in spec.ncell:
        ncolour *= min(2, n)
    ncolr = 2 * spec.norb
    nn = [n * spec.degree + 1 for n in spec.ncell]
    n_nodes = nn[0] * nn[1] * nn[2]
    flop_hx = 2.0 * nloc * nloc * ncolr * ncells
    n_hx = res["stage"]["n_hx"]
    hx_s = res["stage"]["cell_hx"] * 1e-3 / n_hx
    esz = BLOCK_BYTES[dtype]
    row = ncolr * 8
    unique_hx = 2.0 * n_nodes * row + ncells * nloc * nloc * esz
    ai = flop_hx / unique_hx
    inst, mfma_peak = MFMA_OF[dtype]
    if mfma_peak <= ai * HBM_GBS / 1e3:        # the MFMA roof is the lower one
        bound, achieved, peak, unit = "mfma", flop_hx / hx_s / 1e12, mfma_peak, "TFLOP/s"
    else:
        bound, achieved, peak, unit = "hbm", unique_hx / hx_s / 1e9, HBM_GBS, "GB/s"
    # per launch, with the gathered rows and the later colours' reads of Y
    incid = 1
    for a in range(3):
        incid *= nn[a] + spec.ncell[a] - 1
    yreads = (incid - n_nodes) / ncolour
    cells_l = ncells / ncolour
    xrow, yrow = ncolr * X_BYTES[dtype], ncolr * Y_BYTES[dtype]
    bytes_launch = cells_l * nloc * nloc * esz + cells_l * nloc * (xrow + yrow) + yreads * yrow
    kernel_unique_hx = n_nodes * (xrow + yrow) + ncells * nloc * nloc * esz
    launch_s = hx_s / ncolour
    tr = traffic_summary(dtype)
    # enrichment coupling of the same Hbar X: Y_C[R] += G X_E and Y_E = G^T X[R] (+ the
    # small H^ee X_E), G the n_R x n_k block; unique bytes: G, the X rows of R and the Y
    # rows of R read and written, in the element types the kernels use (FP64 X rows with
    # BF16 blocks)
    nr, nk = res["dims"]["n_union_rows"], res["dims"]["n_kept"]
    cp_s = res["stage"]["coupling"] * 1e-3 / n_hx
    gsz = 8 if dtype == "f64" else 4
    cxsz = 8 if dtype in ("f64", "bf16") else 4
    cp_flop = 4.0 * nr * nk * ncolr
    cp_bytes = nr * nk * gsz + nr * ncolr * (cxsz + 2 * Y_BYTES[dtype])
    whole_s = hx_s + cp_s
    if bound == "mfma":
        whole_frac = (flop_hx + cp_flop) / whole_s / 1e12 / peak
    else:
        whole_frac = (unique_hx + cp_bytes) / whole_s / 1e9 / peak
    apply_only = None
    tune = res.get("tune") or {}
    t_us = (tune.get("times_us") or {}).get(tune.get("choice"))
    if t_us:
        a_s = t_us * 1e-6
        a_ach = flop_hx / a_s / 1e12 if bound == "mfma" else unique_hx / a_s / 1e9
        apply_only = {"shape": tune.get("choice"), "hx_us": t_us, "achieved": a_ach, "frac": a_ach / peak}
    coupling = {"us_per_hx": cp_s * 1e6, "flop_per_hx": cp_flop, "unique_bytes_per_hx": cp_bytes,
                "GBps": cp_bytes / cp_s / 1e9, "frac_of_hbm": cp_bytes / cp_s / 1e9 / HBM_GBS,
                "n_union_rows": nr, "n_k": nk}
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": None if tr is None else tr["total"] * ncolour,
            "kernel": "k_cell_bf16" if dtype in ("bf16", "bf16x3") else "k_cell_apply", "mfma_instruction": inst, "flop_per_hx": flop_hx,
            "unique_bytes_per_hx": unique_hx, "arithmetic_intensity": ai, "hx_us": hx_s * 1e6,
            "tflops": flop_hx / hx_s / 1e12, "unique_GBps": unique_hx / hx_s / 1e9,
            "launches_per_hx": ncolour, "launch_avg_us": launch_s * 1e6,
            "per_launch_bytes_with_gathers": bytes_launch, "per_launch_GBps_with_gathers": bytes_launch / launch_s / 1e9,
            "hx_per_step": n_hx / max(1, len(res["k"])), "traffic_detail": tr,
            "kernel_unique_bytes_per_hx": kernel_unique_hx,
            "kernel_unique_GBps": kernel_unique_hx / hx_s / 1e9,
            "frac_of_hbm_on_kernel_unique_bytes": kernel_unique_hx / hx_s / 1e9 / HBM_GBS,
            "coupling": coupling, "whole_hx_us": whole_s * 1e6, "whole_hx_frac": whole_frac,
            "apply_only": apply_only}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_tiny_steps(nsteps=2):
    """Complete oracle Magnus-2 steps of the tiny system (assembled route, plain
    Lanczos), kicked from the stored ground state, at one BLAS thread and at all:
    seconds per step for each."""
    import numpy as np
    from threadpoolctl import threadpool_limits, threadpool_info
    from oracle.model import EFEModel
    from oracle.propagate import Propagator
    from workloads import tiny
    spec = tiny()
    X0 = np.load(os.path.join(ROOT, "tests", "golden", "tiny_ground_state.npz"))["X"]
    m = EFEModel(spec)
    out = {}
    allc = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    for label, nthr in (("1_thread", 1), ("all_cores", allc)):
        with threadpool_limits(limits=nthr):
            P = Propagator(m, X0, tol=spec.krylov_tol, kmax=spec.kmax)
            P.kick(spec.kick, spec.kick_dir)
            t0 = time.perf_counter()
            for _ in range(nsteps):
                P.step(spec.dt)
            out[label] = {"threads": nthr, "s_per_step": (time.perf_counter() - t0) / nsteps,
                          "steps_per_s": nsteps / (time.perf_counter() - t0)}
    return out


def cpu_baseline(spec, hx_per_step):
    """The FP64 oracle timed on this host's cores.

    value (Na8 steps/s, an ESTIMATE and an upper bound): one pass of the oracle's
    cell route (`EFEModel.cell_block` over all 13,824 cells, each block multiplied
    into the 88 real columns: the cell part of one Hbar X) is timed at all cores and
    scaled by the Hbar X count per step measured on the GPU; the coupling, Lanczos
    vector work, densities, Poisson solves and rebuilds are not in the sample.
    measured: complete oracle Magnus steps of the tiny system at one thread and at
    all cores.  reference_run: the complete Na8 oracle steps of the stored reference
    (tests/golden/na8_step.npz), timed where that file was written."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle.model import EFEModel
    t_setup = time.perf_counter()
    m = EFEModel(spec)
    t_setup = time.perf_counter() - t_setup
    mesh = m.mesh
    rng = np.random.default_rng(0)
    X = rng.standard_normal((mesh.n_nodes, 2 * spec.norb))
    Y = np.zeros_like(X)
    v = m.v_nuc
    t0 = time.perf_counter()
    for c in range(mesh.n_cells):
        nodes = mesh.cell_nodes(c)
        Y[nodes] += m.cell_block(c, v) @ X[nodes]
    dt = time.perf_counter() - t0
    cores = int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    flop_hx = 2.0 * mesh.n_cells * float(spec.degree + 1) ** 6 * 2 * spec.norb
    out = {"value": 1.0 / (dt * hx_per_step), "unit": "steps/s", "cores": cores, "kind": "oracle",
           "estimate": True, "cpu_model": _cpu_model(),
           "hx_cell_gflops": flop_hx / dt / 1e9,
           "sample": f"Na8 estimate (upper bound): oracle cell part of one Hbar X ({mesh.n_cells} cells, {dt:.1f} s "
                     f"at {cores} threads; set-up {t_setup:.0f} s untimed) scaled to {hx_per_step:.0f} Hbar X per "
                     f"step; coupling, vector work, densities, Poisson and rebuilds excluded"}
    out["measured_tiny"] = oracle_tiny_steps()
    ref = os.path.join(ROOT, "tests", "golden", "na8_step.npz")
    if os.path.exists(ref):
        z = np.load(ref)
        if "step_seconds" in z:
            out["reference_run_na8"] = {"s_per_step": [float(x) for x in z["step_seconds"]],
                                        "threads": int(z["threads"]), "cpu_model": str(z["cpu_model"]),
                                        "note": "complete matrix-free oracle steps (plain Lanczos) where the "
                                                "stored Na8 reference was written"}
    return out


def batch_members(n24=True):
    """The batched workload: Na2, Na4 and Na6 (seeds 2, 4, 6) each kicked along
    x, y, z with 1e-4 and 1e-3, plus Na8 kicked along x, y, z with 1e-3 (21
    propagations as enumerated) and, with n24, Na8 along x, y, z at 1e-4 as well
    (24: the stated count); FP32 products, FP64 Krylov."""
    out = []
    for natom, seed in ((2, 2), (4, 4), (6, 6)):
        for kick in (1e-4, 1e-3):
            for d in "xyz":
                out.append((natom, seed, d, kick))
    for kick in ((1e-4, 1e-3) if n24 else (1e-3,)):
        for d in "xyz":
            out.append((8, 0, d, kick))
    return out


def run_batch(steps, warmup, kmax, dtype="f32"):
    import numpy as np
    import torch
    from workloads import na_cluster
    from paper_2210_14421_amd.efe import Context, Batch
    t0 = time.time()
    specs = {}
    ctxs, Psis = [], []
    members = batch_members()
    tuned = {}
    for natom, seed, d, kick in members:
        spec = specs.setdefault((natom, seed), na_cluster(natom, seed=seed))
        c = Context(spec, dtype=dtype, kmax=kmax)
        P = c.initial_state()
        c.lanczos_expm(P, -kick, op=d)
        c.set_hamiltonian(P, 0.0)
        # cell-product shape per cluster (the cache key is the problem shape: one tuning per cluster)
        tuned[natom] = c.autotune(cache=TUNE_CACHE)["choice"]
        ctxs.append(c)
        Psis.append(P)
    torch.cuda.synchronize()
    print(f"[bench] batch of {len(ctxs)}: set-up {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    batch = Batch(ctxs)
    dt = specs[(8, 0)].dt
    t = 0.0
    for _ in range(max(1, warmup)):      # the first step captures the graph
        batch.step(Psis, t, dt)
        t += dt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ks = []
    for i in range(steps):
        st = batch.step(Psis, t, dt)
        t += dt
        ks.append([float(np.mean(x["k_corr"])) for x in st])
        print(f"[bench] batch step {i}: {1e3 * (time.perf_counter() - t1) / (i + 1):.1f} ms/step", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    free_b, total_b = torch.cuda.mem_get_info()      # every member alive
    batch.close()
    # the same members stepped one after another by the host-driven magnus_step, each timed
    # alone: its cell-product work per second is what the GPU gives that member by itself
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    alone = {}
    for (natom, _, _, _), c, P in zip(members, ctxs, Psis):
        ta = time.perf_counter()
        st = c.magnus_step(P, t, dt)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - ta)
        nhx = float(np.mean(st["k_pred"]) + np.mean(st["k_corr"]))
        flop = 2.0 * (c.spec.degree + 1) ** 6 * int(np.prod(c.spec.ncell)) * 2 * c.norb * nhx
        alone.setdefault(f"Na{natom}", []).append((ms, flop))
    seq_ms = 1e3 * (time.perf_counter() - t2)
    for c in ctxs:
        c.close()
    n = len(ctxs)
    # the members' cell-product work at the best rate any member reaches alone: the time a
    # launch shared by all members could at best approach if it ran every member at that rate
    rates = {k: sum(f for _, f in v) / sum(m for m, _ in v) for k, v in alone.items()}
    best = max(rates, key=rates.get)
    total_flop = sum(f for v in alone.values() for _, f in v)
    bound_ms = total_flop / rates[best]
    return {"metric": f"batched Magnus steps/s ({n} independent Na2/Na4/Na6/Na8 propagations, one hipGraph per step)",
            "value": n * steps / wall, "unit": "propagation-steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": 1e3 * wall / steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 products, f64 Krylov", "data": "synthetic",
            "device_memory_used_GB": (total_b - free_b) / 1e9, "device_memory_total_GB": total_b / 1e9,
            "config": {"workload": "{Na2, Na4, Na6, Na8} x {x,y,z} x {1e-4,1e-3}, dt 0.02, tol 1e-10",
                       "members": n, "kmax": kmax, "cell_product_shapes": {f"Na{k}": v for k, v in tuned.items()}},
            "sequential_ms_per_step": seq_ms, "speedup_vs_sequential": seq_ms / (1e3 * wall / steps),
            "alone_ms_per_step": {k: [round(m, 2) for m, _ in v] for k, v in alone.items()},
            "alone_cell_gflop_per_s": {k: r / 1e6 for k, r in rates.items()},
            "ms_per_step_at_best_alone_rate": bound_ms, "best_alone_rate_member": best,
            "batch_over_best_alone_rate": (1e3 * wall / steps) / bound_ms,
            "krylov_k_mean_last": ks[-1] if ks else None}


def run_adjoint(steps, kmax):
    """Na8 driven by the sum-of-sines field along z (seed 7 parameters, t0 = 4,
    s = 2; no kick): forward steps, then the reverse sweep over them with the
    checkpointed driver.  Reports ms per forward step and per adjoint step."""
    import numpy as np
    import torch
    from workloads import na8, adjoint_field_params
    from paper_2210_14421_amd.efe import Context, make_field
    spec = na8()
    theta = adjoint_field_params(7, 8, (1e-3, 1e-2), (0.05, 0.5))
    m = len(theta) // 3
    field, keep = make_field(2, theta[:m], theta[m:2 * m], theta[2 * m:], 4.0, 2.0)
    ctx = Context(spec, dtype="f64", kmax=kmax)
    Psi = ctx.initial_state()
    ctx.set_hamiltonian(Psi, 0.0, field)
    states = [Psi.clone()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(steps):
        ctx.magnus_step(Psi, n * spec.dt, spec.dt, field)
        states.append(Psi.clone())
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / steps
    Psibar = ctx.dipole_adjoint(states[-1], (0.0, 0.0, 1.0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for n in range(steps - 1, -1, -1):
        ctx.magnus_adjoint(states[n], Psibar, n * spec.dt, spec.dt, field, (0.0, 0.0, 1.0))
        print(f"[bench] adjoint step {n}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    adj = (time.perf_counter() - t1) / steps
    ctx.close()
    del keep
    return {"metric": "adjoint Magnus step time at Na8 (field-driven, dL/dmu_z = 1 at every step)",
            "value": 1e3 * adj, "unit": "ms per adjoint step", "n_gpus": 1, "steps": steps,
            "higher_is_better": False, "forward_ms_per_step": 1e3 * fwd, "adjoint_over_forward": adj / fwd,
            "dtype": "f64", "data": "synthetic", "config": {"workload": "Na8, field of 8 sines (seed 7), t0 4, s 2"}}


def run_spectrum_timing(reps=5):
    """Absorption spectrum on the GPU at the paper's run length: three runs of 20 fs
    (8,270 samples of 0.1 au), 2,000 frequencies; synthetic traces (a sum of damped modes)."""
    import numpy as np
    import torch
    from paper_2210_14421_amd.efe import absorption_spectrum
    dt, nt, nw = 0.1, 8270, 2000
    t = dt * np.arange(nt + 1)
    rng = np.random.default_rng(11)
    traces = np.zeros((3, nt + 1, 3))
    for d in range(3):
        for w0, f in zip(rng.uniform(0.1, 1.5, 6), rng.uniform(0.1, 1.0, 6)):
            traces[d, :, d] += 1e-3 * f * np.sin(w0 * t) / w0
    mu = torch.from_numpy(traces).cuda()
    w = torch.linspace(0.0, 2.0, nw, dtype=torch.float64, device="cuda")
    pulse = dict(kind="kick", kappa=1e-3)
    absorption_spectrum(mu, [0, 1, 2], dt, w, 100.0, pulse)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        absorption_spectrum(mu, [0, 1, 2], dt, w, 100.0, pulse)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"runs": 3, "samples": nt + 1, "frequencies": nw, "ms": ms,
            "sample_frequency_pairs_per_s": 3 * (nt + 1) * nw / (ms * 1e-3)}


def run_hhg(max_steps=None, graph=False):
    """High-harmonic workload of Sec. 3.5 on the tiny system (one atom at the centre, inversion
    symmetric): kappa sin(pi t/T) sin(omega t) along z with kappa 0.01, omega 0.03, T five periods,
    dt 0.1, Krylov tol 1e-7 (the paper's settings), steps over [0, T] (host-driven by default: with
    k of about 8 the captured step's fixed kmax trip count costs more than the host round trips), then the
    dipole power spectrum (Gaussian window, tau 1e5) at 2,000 frequencies up to 20 omega."""
    import numpy as np
    import torch
    from workloads import tiny, hhg_field
    from paper_2210_14421_amd.efe import Context, make_field, power_spectrum
    here = os.path.dirname(os.path.abspath(__file__))
    spec = tiny()
    p = hhg_field(kappa=0.01, omega=0.03, ncycles=5, direction=2)
    dt = 0.1
    nsteps = int(round(p["T"] / dt)) if max_steps is None else max_steps
    f, keep = make_field(p["direction"], p["A"], p["w"], p["phi"], p["t0"], p["s"])
    X0 = np.load(os.path.join(here, "tests", "golden", "tiny_ground_state.npz"))["X"]
    ctx = Context(spec, kmax=40, tol=1e-7)
    Psi = torch.from_numpy(np.ascontiguousarray(X0)).cuda()
    ctx.set_hamiltonian(Psi, 0.0, field=f)
    mus = [ctx.dipole(Psi)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = 0.0
    for n in range(nsteps):
        st = ctx.magnus_step(Psi, t, dt, field=f, graph=graph)
        t += dt
        mus.append(st["mu"])
        if n % 2000 == 0:
            print(f"[bench] hhg step {n}/{nsteps}: mu_z={st['mu'][2]:.6e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    mu = torch.from_numpy(np.array(mus)).cuda()
    w = torch.linspace(0.0, 20 * 0.03, 2000, dtype=torch.float64, device="cuda")
    power_spectrum(mu, 2, dt, w, 1e5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P = power_spectrum(mu, 2, dt, w, 1e5)
    e1.record()
    torch.cuda.synchronize()
    P = P.cpu().numpy()
    wn = w.cpu().numpy()
    harm = {}
    for k in range(1, 16):
        sel = np.abs(wn - k * 0.03) <= 0.5 * 0.03 / 2
        harm[k] = float(P[sel].max())
    _ = keep
    return {"metric": "driven Magnus steps/s (tiny system, sinusoidal pulse of the high-harmonic study)",
            "value": nsteps / wall, "unit": "steps/s", "n_gpus": 1, "steps": nsteps, "ms_per_step": 1e3 * wall / nsteps,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "tiny (Z = 3 at the centre), kappa 0.01, omega 0.03, T = 5 periods, dt 0.1, tol 1e-7",
                       "steps": "graph-captured" if graph else "host-driven"},
            "power_spectrum_ms": e0.elapsed_time(e1), "samples": nsteps + 1, "frequencies": 2000,
            "harmonic_peaks": harm, "graph": graph}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kmax", type=int, default=40)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extrap", action="store_true")
    ap.add_argument("--no-graded", action="store_true")
    ap.add_argument("--graph", action="store_true", help="hhg workload: graph-captured steps")
    ap.add_argument("--workload", default="na8",
                    choices=["na8", "na8_graded", "tiny", "na2", "batch", "adjoint", "hhg"])
    ap.add_argument("--mode", default="step", choices=["step", "apply"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16", "bf16x3", "f64sf"])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the orbitals would be sharded across GPUs, which is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from workloads import na8, na8_graded, tiny, na_cluster
    torch.cuda.set_device(0)
    if args.workload == "batch":
        print(json.dumps(run_batch(args.steps, args.warmup, min(args.kmax, 17))))
        return
    if args.workload == "hhg":
        print(json.dumps(run_hhg(graph=args.graph)))
        return
    if args.workload == "adjoint":
        print(json.dumps(run_adjoint(args.steps, min(args.kmax, 24))))
        return
    spec = {"na8": na8, "na8_graded": na8_graded, "tiny": tiny,
            "na2": lambda: na_cluster(2, seed=2)}[args.workload]()
    if args.mode == "apply":
        run_apply_mode(spec, args.dtype, max(1, args.steps))
        return
    # the headline run is FP64; --dtype gives another product type for profiling runs
    res = run_gpu(spec, args.dtype, args.steps, args.warmup, args.kmax)
    value = args.steps / res["wall"]
    roof = roofline(spec, res, args.dtype if args.dtype in MFMA_OF else "f64")
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * res["wall"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{spec.name}: {spec.natom} atoms, {spec.ncell[0]}^3 cells degree {spec.degree}, "
                               f"{(spec.ncell[0] * spec.degree + 1) ** 3} nodes, {spec.norb} orbitals, "
                               f"dt {spec.dt}, Krylov tol {spec.krylov_tol}, z kick {spec.kick}",
                   "precision": ("FP64" if args.dtype == "f64" else args.dtype.upper()) + " products, FP64 Lanczos",
                   "lanczos_reorthogonalisation": "partial (Simon's omega recurrence)"},
        "roofline": roof, "autotune": res["tune"],
        "stage_ms_per_step": {k: v / args.steps for k, v in res["stage"].items() if k != "n_hx"},
        "krylov_k_mean": res["k"], "orthonormality_error": res["orth"],
    }
    if not args.no_mixed:
        mres = run_gpu(spec, "f32", args.steps, args.warmup, args.kmax)
        mroof = roofline(spec, mres, "f32")
        mv = args.steps / mres["wall"]
        import numpy as np
        dmu = np.max(np.linalg.norm(np.array(mres["mu"]) - np.array(res["mu"]), axis=1)) / \
            np.max(np.linalg.norm(np.array(res["mu"]), axis=1))
        out["mixed"] = {"dtype": "f32 products, FP64 Lanczos", "value": mv, "unit": "steps/s",
                        "ms_per_step": 1e3 * mres["wall"] / args.steps, "speedup_vs_f64": mv / value,
                        "roofline": mroof, "autotune": mres["tune"], "dipole_rel_diff_vs_f64": float(dmu), "krylov_k_mean": mres["k"],
                        "stage_ms_per_step": {k: v / args.steps for k, v in mres["stage"].items() if k != "n_hx"}}
    if not args.no_mixed:
        bres = run_gpu(spec, "bf16", args.steps, args.warmup, args.kmax)
        broof = roofline(spec, bres, "bf16")
        bv = args.steps / bres["wall"]
        import numpy as np
        dmu = np.max(np.linalg.norm(np.array(bres["mu"]) - np.array(res["mu"]), axis=1)) / \
            np.max(np.linalg.norm(np.array(res["mu"]), axis=1))
        out["mixed_bf16"] = {"dtype": "bf16 products (blocks and orbital rows in BF16, BF16 MFMA), FP64 Lanczos",
                             "value": bv, "unit": "steps/s",
                             "ms_per_step": 1e3 * bres["wall"] / args.steps, "speedup_vs_f64": bv / value,
                             "roofline": broof, "autotune": bres["tune"], "dipole_rel_diff_vs_f64": float(dmu), "krylov_k_mean": bres["k"],
                             "stage_ms_per_step": {k: v / args.steps for k, v in bres["stage"].items() if k != "n_hx"}}
    if not args.no_mixed:
        xres = run_gpu(spec, "bf16x3", args.steps, args.warmup, args.kmax)
        xroof = roofline(spec, xres, "bf16x3")
        xv = args.steps / xres["wall"]
        import numpy as np
        dmu = np.max(np.linalg.norm(np.array(xres["mu"]) - np.array(res["mu"]), axis=1)) / \
            np.max(np.linalg.norm(np.array(res["mu"]), axis=1))
        out["mixed_bf16x3"] = {"dtype": "split bf16 products (hi/lo pairs, three BF16 MFMAs), FP64 Lanczos",
                               "value": xv, "unit": "steps/s", "ms_per_step": 1e3 * xres["wall"] / args.steps,
                               "speedup_vs_f64": xv / value, "roofline": xroof, "autotune": xres["tune"], "krylov_k_mean": xres["k"],
                               "dipole_rel_diff_vs_f64": float(dmu),
                               "stage_ms_per_step": {k: v / args.steps for k, v in xres["stage"].items() if k != "n_hx"}}
    if not args.no_extrap:
        # one exponential per step: the midpoint Hamiltonian at the density extrapolated from three steps
        eres = run_gpu(spec, "f64", args.steps, args.warmup, args.kmax, scheme="extrap")
        ev = args.steps / eres["wall"]
        out["extrap"] = {"scheme": "midpoint Hamiltonian at the density extrapolated from the last three steps",
                         "dtype": "f64", "value": ev, "unit": "steps/s", "ms_per_step": 1e3 * eres["wall"] / args.steps,
                         "speedup_vs_predictor_corrector": ev / value, "orthonormality_error": eres["orth"],
                         "stage_ms_per_step": {k: v / args.steps for k, v in eres["stage"].items() if k != "n_hx"}}
    if not args.no_mixed:
        # the same FP64 operator applied by sum factorisation (no stored cell blocks)
        sres = run_gpu(spec, "f64sf", args.steps, args.warmup, args.kmax)
        sv = args.steps / sres["wall"]
        import numpy as np
        dmu = np.max(np.linalg.norm(np.array(sres["mu"]) - np.array(res["mu"]), axis=1)) / \
            np.max(np.linalg.norm(np.array(res["mu"]), axis=1))
        out["sum_factorised"] = {"dtype": "f64, sum-factorised cell products, no stored blocks", "value": sv,
                                 "unit": "steps/s", "ms_per_step": 1e3 * sres["wall"] / args.steps,
                                 "speedup_vs_f64": sv / value, "dipole_rel_diff_vs_f64": float(dmu),
                                 "stage_ms_per_step": {k: v / args.steps for k, v in sres["stage"].items()
                                                       if k != "n_hx"}}
    if not args.no_graded and args.workload == "na8":
        # the same step with a Gram-Schmidt pass against every previous Lanczos vector at each iteration
        fres = run_gpu(spec, "f64", args.steps, args.warmup, args.kmax, reorth="full")
        fv = args.steps / fres["wall"]
        import numpy as np
        dmu = np.max(np.linalg.norm(np.array(fres["mu"]) - np.array(res["mu"]), axis=1)) / \
            np.max(np.linalg.norm(np.array(res["mu"]), axis=1))
        out["full_reorth"] = {"dtype": "f64", "value": fv, "unit": "steps/s", "ms_per_step": 1e3 * fres["wall"] / args.steps,
                              "partial_speedup": value / fv, "dipole_rel_diff_vs_partial": float(dmu),
                              "orthonormality_error": fres["orth"],
                              "stage_ms_per_step": {k: v / args.steps for k, v in fres["stage"].items() if k != "n_hx"}}
        # the same cluster in a 70-bohr box on a sinh-graded mesh with the same node count
        gspec = na8_graded()
        gres = run_gpu(gspec, "f64", args.steps, args.warmup, args.kmax)
        gv = args.steps / gres["wall"]
        out["graded"] = {"workload": "Na8 in [-35, 35]^3, 24^3 sinh-graded cells (1.68 .. 5.44 bohr) of degree 5",
                         "dtype": "f64", "value": gv, "unit": "steps/s", "ms_per_step": 1e3 * gres["wall"] / args.steps,
                         "ratio_vs_uniform_box": gv / value,
                         "mean_krylov_dim": [float(sum(k[0] for k in gres["k"]) / len(gres["k"])),
                                             float(sum(k[1] for k in gres["k"]) / len(gres["k"]))],
                         "orthonormality_error": gres["orth"],
                         "stage_ms_per_step": {k: v / args.steps for k, v in gres["stage"].items() if k != "n_hx"}}
    if not args.no_extrap:
        out["spectrum"] = run_spectrum_timing()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, roof["hx_per_step"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
