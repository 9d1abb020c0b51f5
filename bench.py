#!/usr/bin/env python3
"""Throughput of the real-time TDKS time step on one MI355X.

Workload: the 8-atom diamond cell on a 20^3 grid with 16 doubly occupied
orbitals at 8^3 = 512 Monkhorst-Pack k-points, s+p Kleinman-Bylander
projectors, Hartree + PZ81 LDA, x kick (|A0|/c = 1e-3), dt = 0.04 a.u.
(the 0.08 of the run description exceeds the fourth-order Taylor stability
bound on this grid; the library refuses it). Inputs are seeded synthetic
arrays resident in HBM before the timed region.

One step = the whole path: four Horner stages with the nonlocal projections,
the observables and nonlocal current, the density, FFT Poisson, LDA and the
current reduction. value = orbital x k-point x grid-point steps per second
(og-steps/s) of the mixed path (complex FP32 orbitals and stencil, FP64
reductions, Poisson and projector products); the complex128 path is timed
beside it. The JSON line also carries the roofline of the dominant kernel
(the LDS-resident whole-step update k_fused, HIP events around back-to-back
launches on the library's stream) and the CPU oracle timed on the host cores
(one worker process per core) on a bounded sample of the same workload.
Further lines run the other workloads at their stated shapes: the 96^3
cluster with all 512 orbitals (mixed, and a complex128 twin), the 64-cell
uneven batch with 8-64 orbitals and 1-64 k-points, and the multiscale slab of
256 cells (16^3, 16 orbitals, 64 k-points); a plain device copy gives the
streaming rate of the box.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "orbital·gridpoint Taylor steps/s (FP64 vs mixed/batched), % HBM peak"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
FP32_VALU_PACKED_TFLOPS = 157.3  # MI355X FP32 vector as published: 256 CU x 2.4 GHz x 256 flop/clk,
                                 # which counts two packed FP32 FMAs per lane and clock
# 256 CU x 4 SIMD x 16 lanes x 2 flop (one FMA per lane and clock) x 2.4 GHz: the FP32
# vector rate of code built without packed FP32 instructions, as this library is
FP32_VALU_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def time_path(system, precision, steps, warmup):
    import torch
    from paper_1804_01404_amd.binding import (KERNEL_DENSITY, KERNEL_FUSED, KERNEL_OBSERVE,
                                              KERNEL_PROJECT, KERNEL_STAGE, TDDFT, TDDFTError)
    A = system.A
    with TDDFT(system, precision=precision) as t:
        t.set_potential()
        if warmup:
            t.propagate(A[: warmup + 1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = t.propagate(A[warmup: warmup + steps + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dev_ms = t.last_timing_ms()
        kern = {
            "stage_ms": t.time_kernel(KERNEL_STAGE, 50),
            "project_ms": t.time_kernel(KERNEL_PROJECT, 50),
            "observe_ms": t.time_kernel(KERNEL_OBSERVE, 20),
            "density_ms": t.time_kernel(KERNEL_DENSITY, 20),
        }
        try:
            kern["fused_ms"] = t.time_kernel(KERNEL_FUSED, 20)
        except TDDFTError:
            kern["fused_ms"] = None   # this shape takes the per-stage kernels
        kern["report"] = t.report()
    return (t1 - t0) / steps * 1e3, dev_ms, kern, J


def step_flops_per_og(system):
    """Algorithmic real flops of one time step per orbital x k-point x grid
    point: 152 per Horner stage for the 25-point h (Laplacian and gradient,
    kappa term, diagonal, Horner update), four stages, plus the projection and
    add-back of the nonlocal term, 2 x 8 flops per projector and sphere point
    and stage, spread over the grid."""
    sphere = sum(p.beta.shape[0] * p.npts for p in system.projectors)
    return 4 * 152 + 4 * 16 * sphere / system.n_grid


def stored_traffic(kernel_source, kernel_name, workload):
    """HBM bytes per launch from the committed profiler counters, if they were
    taken on the current source of the kernel; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_name}_{workload}_traffic.txt")
    src = os.path.join(ROOT, "paper_1804_01404_amd", "csrc", kernel_source)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != digest:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---- the oracle on the host cores: one worker process per core, each owning a
# block of k-points for the Taylor step, its density and its current; the
# density and current are summed in block order in the parent, which then
# forms the Hartree and LDA potential. Runs in a child process that never
# touches the GPU.

def _oracle_worker(conn, ks):
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import tdks
    s = _POOL["system"]
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    projs = [tdks.Projector(p.idx, p.x, p.beta, p.e_kb) for p in s.projectors]
    psi = np.array(s.psi0[ks], dtype=np.complex128)
    kpts, kw = s.kpts[ks], s.kw[ks]
    with threadpool_limits(limits=1):
        while True:
            msg = conn.recv()
            if msg is None:
                break
            V, A0, A1 = msg
            shift = 0.5 * (A0 + A1) / tdks.C_LIGHT
            for i, k in enumerate(kpts):
                kap = k + shift
                psi[i] = tdks.taylor_step(psi[i], s.dt, lambda X, kap=kap: tdks.apply_h(X, kap, V, projs, grid))
            conn.send((tdks.density(psi, kw, grid), tdks.current(psi, kpts, kw, A1, projs, grid)))


_POOL = {}


def bench_sample(nk, nsteps):
    """The bench cell restricted to its first nk k-points (equal weights)."""
    import copy
    import numpy as np
    import synth
    s = synth.single_cell_config(1, nsteps=nsteps)
    if nk >= s.n_k:
        return s
    sub = copy.copy(s)
    sub.kpts = s.kpts[:nk]
    sub.kw = np.full(nk, 1.0 / nk)
    sub.psi0 = s.psi0[:nk]
    return sub


def oracle_pool_run(steps, workers, nk):
    """The bench cell's first nk k-points on `workers` processes: one untimed
    step, then `steps` timed ones. Returns the density and current after the
    last step and the timing."""
    import multiprocessing as mp
    import numpy as np
    from oracle import tdks
    s = bench_sample(nk, steps + 1)
    _POOL["system"] = s
    o = tdks.TDKS.from_system(s)          # the potential of the initial density
    blocks = [b for b in np.array_split(np.arange(s.n_k), workers) if b.size]
    ctx = mp.get_context("fork")
    procs, conns = [], []
    for b in blocks:
        a, c = ctx.Pipe()
        p = ctx.Process(target=_oracle_worker, args=(c, b))
        p.start()
        procs.append(p)
        conns.append(a)
    grid = o.grid
    V = o.v_ks
    J = np.zeros((steps + 1, 3))
    t0 = None
    for n in range(steps + 1):
        if n == 1:
            t0 = time.perf_counter()
        for c in conns:
            c.send((V, s.A[n], s.A[n + 1]))
        parts = [c.recv() for c in conns]
        rho = parts[0][0].copy()
        cur = parts[0][1].copy()
        for r, j in parts[1:]:
            rho += r
            cur += j
        J[n] = cur
        vh = tdks.hartree_periodic(rho, grid)
        vxc, _ = tdks.lda_pz81(rho)
        V = s.v_loc + vh + vxc
    el = time.perf_counter() - t0
    for c in conns:
        c.send(None)
    for p in procs:
        p.join()
    return {"rho": rho, "J": J, "seconds": el, "og": s.og, "steps": steps, "workers": len(blocks)}


def cpu_baseline(steps=6, nk=512):
    """The oracle as it stands on the host cores (one process per core, BLAS
    threads pinned to 1 per worker), on a bounded sample of the bench cell:
    its first nk of 512 k-points (all of them by default; all 16 orbitals, the
    whole grid), one untimed step, then `steps` timed steps (Taylor + density
    + current + Hartree + LDA), about 10 s of work on 16 cores. The same steps then run on the GPU (complex128 and mixed)
    and their errors against the oracle are reported beside the timing."""
    import subprocess
    import numpy as np
    from paper_1804_01404_amd.binding import TDDFT
    host = os.cpu_count() or 1
    try:
        host = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    workers = max(1, min(16, host))
    import tempfile
    out_npz = os.path.join(tempfile.gettempdir(), f"oracle_pool_{os.getpid()}.npz")
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-pool-child", str(steps), str(workers), str(nk),
           out_npz]
    t_wall = time.perf_counter()
    r = subprocess.run(cmd, capture_output=True, text=True)
    t_wall = time.perf_counter() - t_wall
    if r.returncode != 0:
        return {"error": r.stderr[-2000:]}
    res = np.load(out_npz)
    os.remove(out_npz)
    og, el = float(res["og"]), float(res["seconds"])
    parity = {}
    s = bench_sample(nk, steps + 1)
    for prec in ("c128", "mixed"):
        with TDDFT(s, precision=prec) as t:
            t.set_potential()
            J = t.propagate(s.A[:steps + 2])
            rho, _ = t.density_current()
        parity[prec] = {"density_l2_error": float(np.linalg.norm(rho - res["rho"]) / np.linalg.norm(res["rho"])),
                        "current_error": float(np.max(np.abs(J - res["J"])) / np.max(np.abs(res["J"])))}
    return {"value": og * steps / el, "unit": "og-steps/s", "cores": int(res["workers"]), "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"the bench cell's first {s.n_k} of 512 k-points x {s.n_orb} orbitals x {s.n_grid} points, "
                      f"1 untimed + {steps} timed full steps (Taylor + density + current + Hartree + LDA) "
                      f"in {el:.1f} s, NumPy FP64 on {int(res['workers'])} worker processes over k-point "
                      f"blocks, one BLAS thread each; child process wall time {t_wall:.1f} s",
            "gpu_vs_oracle_on_sample": parity}


def accuracy_report():
    """Errors of the mixed path against the complex128 path over 1000 steps
    (the complex128 path is pinned to the oracle by the parity tests and by
    the cpu_baseline leg), and the field-free energy drift per 1000 steps
    from the ground state, both precisions."""
    import numpy as np
    import synth
    from paper_1804_01404_amd.binding import TDDFT

    def run(s, prec, psi=None, every=0):
        with TDDFT(s, precision=prec) as t:
            t.set_potential()
            if psi is not None:
                t.set_orbitals(psi)
            Es = [t.energy()]
            J = None
            if every:
                for i in range(0, s.A.shape[0] - 1, every):
                    t.propagate(s.A[i:i + every + 1])
                    Es.append(t.energy())
            else:
                J = t.propagate(s.A)
            rho, _ = t.density_current()
            d = t.dipole()
        return J, rho, d, np.array(Es)
    out = {}
    s = synth.single_cell_config(1, nk=2, nsteps=1000)
    J64, r64, _, _ = run(s, "c128")
    J32, r32, _, _ = run(s, "mixed")
    out["periodic_20^3_k8_1000_steps"] = {
        "current_error": float(np.max(np.max(np.abs(J32 - J64), axis=0) / np.max(np.abs(J64), axis=0))),
        "density_l2_error": float(np.linalg.norm(r32 - r64) / np.linalg.norm(r64))}
    c = synth.single_cell_config(2, n=40, n_orb=32, n_fcc=1, nsteps=1000)
    _, _, d64, _ = run(c, "c128")
    _, _, d32, _ = run(c, "mixed")
    out["isolated_40^3_32orb_1000_steps"] = {
        "dipole_error": float(np.max(np.abs(d32 - d64)) / np.max(np.abs(d64)))}
    g = synth.single_cell_config(0, nsteps=1000, kick=0.0)
    with TDDFT(g, precision="c128") as t:
        t.set_potential()
        t.ground_state(600, 0.035)
        psi = t.orbitals()
    drift = {}
    for prec in ("c128", "mixed"):
        _, _, _, E = run(g, prec, psi=psi, every=100)
        tt = np.arange(E.shape[0]) * 100
        drift[prec] = float(np.polyfit(tt, E, 1)[0] * 1000 / abs(E[0]))
    out["energy_drift_per_1000_steps_16^3_ground_state"] = drift
    return out


def bench_mgga(system, precision, lda_ms, steps=60, warmup=10):
    """The same cell and path with the Tran-Blaha exchange (Sec. 4.1): step time,
    its ratio to the LDA step, and the density pass that also forms tau."""
    import copy
    import numpy as np
    s = copy.copy(system)
    s.xc = "tb09"
    # the field table is sized for the main line's steps: stay within it
    avail = s.A.shape[0] - 1
    warmup = min(warmup, avail // 4)
    steps = min(steps, avail - warmup)
    ms, dev_ms, kern, J = time_path(s, precision, steps, warmup)
    return {"xc": "tb09", "ms_per_step": ms, "device_ms_per_step": dev_ms, "lda_ms_per_step": lda_ms,
            "ratio_to_lda": ms / lda_ms, "density_tau_ms": kern["density_ms"],
            "fused_ms": kern["fused_ms"], "current_finite": bool(np.all(np.isfinite(J)))}


def mfma_projection(system, project_ms, esz):
    """MFMA work of one stage-mode projection launch (per-stage path): one
    four-block 4x4x4 FP64 MFMA (512 flops) per four sphere entries, per atom
    and group of eight orbitals; every product is used except the padding of
    the last orbital group and of the last four entries of a sphere. The
    launch is bound by the sphere gathers (one orbital value per entry and
    orbital, esz bytes), reported as gather_GBs."""
    n_tot = system.n_orb * system.n_k
    n_groups = (n_tot + 7) // 8
    issued = sum(n_groups * -(-p.npts // 4) * 512 for p in system.projectors)
    useful = sum(n_tot * 2 * kmax * p.npts * 2 for p in system.projectors for kmax in (4,))
    gathered = sum(n_tot * p.npts * esz for p in system.projectors)
    t = project_ms * 1e-3
    return {"instruction": "v_mfma_f64_4x4x4f64", "issued_tflops": issued / t / 1e12,
            "useful_tflops": useful / t / 1e12, "peak": FP64_MFMA_PEAK_TFLOPS,
            "frac_issued": issued / t / 1e12 / FP64_MFMA_PEAK_TFLOPS,
            "frac_useful": useful / t / 1e12 / FP64_MFMA_PEAK_TFLOPS,
            "gather_GBs": gathered / t / 1e9, "ms_per_launch": project_ms}


def per_stage_figures(system, kern, esz, traffic_workload=None):
    """HBM fractions of the per-stage kernels from their algorithmic bytes:
    a middle stage reads u_s and w and writes u_{s-1} (3 esz per og), the
    observe pass reads w once (esz per og). stage_ms is the middle-stage
    kernel alone (the tuner's time for the chosen plan, or the isolated timing
    with the nonlocal add-back when no plan was tuned); stage_with_addback_ms
    adds the nonlocal add-back launches of the stage."""
    og = system.og
    plan = kern["report"].get("stage") or {}
    st_ms = plan.get("ms") or kern["stage_ms"]
    st = 3 * esz * og / (st_ms * 1e-3) / 1e9
    ob = esz * og / (kern["observe_ms"] * 1e-3) / 1e9
    out = {"stage_ms": st_ms, "stage_GBs": st, "stage_frac_hbm": st / HBM_PEAK_GBS,
           "stage_with_addback_ms": kern["stage_ms"],
           "observe_ms": kern["observe_ms"], "observe_GBs": ob, "observe_frac_hbm": ob / HBM_PEAK_GBS,
           "project_ms": kern["project_ms"], "tuner": kern["report"].get("stage"),
           "tuner_source": kern["report"].get("source")}
    if traffic_workload:
        out["stage_traffic_counters"] = stored_traffic("k_stage.hip", "k_stage", traffic_workload)
    return out


def bench_cluster(steps=5, warmup=2, n_orb=512):
    """The isolated-cluster workload at its stated size: 96^3 box, 256 atoms
    with s+p projectors, all 512 orbitals, length gauge, Gaussian-envelope
    pulse; the orbital does not fit in LDS, so this is the per-stage path with
    the tuned decomposition."""
    import numpy as np
    import synth
    t0 = time.perf_counter()
    s = synth.single_cell_config(2, n_orb=n_orb, nsteps=steps + warmup)
    t_gen = time.perf_counter() - t0
    ms, dev_ms, kern, J = time_path(s, "mixed", steps, warmup)
    out = {"workload": f"cluster-96^3: 256 atoms, {n_orb} orbitals, Gamma, length gauge, dt 0.02",
           "og_per_step": s.og, "ms_per_step": ms, "device_ms_per_step": dev_ms,
           "value": s.og / (ms * 1e-3), "unit": "og-steps/s",
           "steps": steps, "warmup": warmup, "input_generation_s": t_gen,
           "current_finite": bool(np.all(np.isfinite(J)))}
    out.update(per_stage_figures(s, kern, 8, "cluster96_orb512" if n_orb == 512 else None))
    out["mfma_projection"] = mfma_projection(s, kern["project_ms"], 8)
    # the complex128 twin of the same cell (three timed steps)
    log("  cluster complex128 twin")
    ms64, dev64, kern64, _ = time_path(s, "c128", 3, 1)
    out["c128"] = {"ms_per_step": ms64, "device_ms_per_step": dev64, "value": s.og / (ms64 * 1e-3),
                   "stage_ms": kern64["stage_ms"], "steps": 3, "warmup": 1}
    out["speedup_mixed_over_c128"] = ms64 / ms
    return out


def copy_bandwidth(mib=2048, reps=10):
    """A plain device-to-device copy of mib MiB (torch's copy kernel), timed
    with HIP events: the streaming rate this machine reaches, beside which the
    kernels' HBM fractions can be read."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    del src, dst
    return {"bytes_per_copy": 2 * n * 4, "ms": ms, "GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}


def bench_batch(steps=12, warmup=6):
    """The uneven-batch workload at its stated ranges: 64 seeded periodic
    cells, grids {12, 16, 20, 24, 32}^3 at h 0.55, 8-64 orbitals, 1-64
    k-points, 2-16 atoms, each with its own cos^2 pulse; mixed and
    complex128. The first steps of the mixed run include the tuner's
    candidate steps (warm-up)."""
    import torch
    import synth
    from paper_1804_01404_amd.binding import TDDFTBatch
    t0 = time.perf_counter()
    cells = synth.batch_cells(64, nsteps=warmup + steps)
    t_gen = time.perf_counter() - t0
    og = sum(c.og for c in cells)
    out = {"workload": "batch-64cells: 64 periodic cells, grids {12,16,20,24,32}^3 at h 0.55, "
                       "8-64 orbitals, 1-64 k-points, 2-16 atoms, own cos^2 pulse each, dt 0.02",
           "og_per_step": og, "input_generation_s": t_gen, "steps": steps, "warmup": warmup}
    for prec in ("mixed", "c128"):
        with TDDFTBatch(cells, precision=prec) as b:
            b.propagate([c.A[: warmup + 1] for c in cells])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.propagate([c.A[warmup: warmup + steps + 1] for c in cells])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[prec] = {"value": og * steps / el, "ms_per_step": el / steps * 1e3,
                         "device_ms_per_step": b.last_timing_ms()}
            if prec == "mixed":
                out["plan"] = b.report()
    out["speedup_mixed_over_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    return out


def bench_multiscale():
    """Learned multiscale coupling, small slab: 16 points of 12^3 diamond-like
    cells (8 orbitals, 2^3 k-points, converged ground state) under a 1.55 eV
    pulse, run with a cell at every point (complex128 and mixed) and through
    the surrogate with two sentinel cells checked every 50 steps at the stated
    spot-check error 1e-3. The network (window 300, 16 hidden) is trained here
    by the library: least-squares linear part on the weak-field trajectories,
    then Adam (cosine schedule) on 256 batch-path trajectories (192 varied
    fields, 64 random cos^2 pulses)."""
    import numpy as np
    import synth
    from paper_1804_01404_amd import pipeline
    n_sub, dt, T = 4, 0.32, 300
    cell = synth.multiscale_cell(nk=2, n=12, n_orb=8, dt=dt / n_sub)
    t0 = time.perf_counter()
    psi, _ = pipeline.ground_state(cell, n_iter=12000, tau=0.06)
    t_gs = time.perf_counter() - t0
    P, _ = synth.random_pulse_tables(64, T, dt, 3, e0_range=(1e-4, 1e-2), ev_range=(0.5, 3.0),
                                     t_range=(40.0, 200.0))
    A_tr = np.vstack([synth.random_field_tables(192, T, dt, 1, a_max=12.0), P])
    J_tr, t_gen = pipeline.trajectories(cell, psi, A_tr, n_sub=n_sub, axis=0)
    a_scale, j_scale = float(np.abs(A_tr).max()), float(np.abs(J_tr).max())
    t0 = time.perf_counter()
    nn, losses = pipeline.train(A_tr, J_tr, synth.surrogate_init(T, 16, 1), window=T, hidden=16,
                                a_scale=a_scale, j_scale=j_scale, epochs=60, batch=256, seed=1, lr=2e-3,
                                a_fit=a_scale / 8, cosine=True)
    t_train = time.perf_counter() - t0
    dx, n_mat, n_vac = 147.6, 16, 12
    n_x = n_mat + 2 * n_vac
    inc = synth.incident_table(T, dt, dx, delay=0.0, E0=3e-3, omega=1.55 / 27.211386245988, T=100.0)
    kw = dict(n_x=n_x, x0=n_vac, n_mat=n_mat, dx=dx, dt=dt, n_sub=n_sub, axis=0)
    A64, _, t64, _ = pipeline.run_slab(cell, psi, inc, precision="c128", **kw)
    A32, _, t32, _ = pipeline.run_slab(cell, psi, inc, precision="mixed", **kw)
    with nn:
        An, _, tn, st = pipeline.run_slab(cell, psi, inc, precision="mixed", nn=nn, a_max=a_scale,
                                          sentinels=[0, n_mat // 2], check_every=50, tol=1e-3, **kw)
    ref = np.max(np.abs(A64))
    og_run = cell.og * n_mat * T * n_sub
    return {"workload": f"slab of {n_mat} cells (12^3, 8 orbitals, 8 k-points) + {2 * n_vac} vacuum "
                        f"points, dX 147.6, dt 0.32 = 4 cell steps, {T} steps, 1.55 eV pulse E0 3e-3",
            "cells_c128_s": t64, "cells_mixed_s": t32, "surrogate_s": tn,
            "cells_c128_og_steps_per_s": og_run / t64, "cells_mixed_og_steps_per_s": og_run / t32,
            "speedup_surrogate_over_c128_cells": t64 / tn, "speedup_mixed_over_c128_cells": t64 / t32,
            "sentinel_tol": 1e-3,
            "field_error_mixed_cells": float(np.max(np.abs(A32 - A64)) / ref),
            "field_error_surrogate": float(np.max(np.abs(An - A64)) / ref),
            "surrogate_status": st, "train_s": t_train, "trajectories_s": t_gen, "ground_state_s": t_gs,
            "loss_first_last": [float(losses[0]), float(losses[-1])]}


def sentinel_error_scan(cell, psi, nn, kw, n_mat, e0, dt, dx, n_macro=4000, every=25):
    """The coupled run over n_macro macroscopic steps under a 20 fs cos^2 pulse
    of peak field e0 through the network, with the spot-check threshold and the
    amplitude gate out of reach (so it never falls back): the sentinel error
    met at each check (every `every` steps), relative to the output scale."""
    import numpy as np
    import torch
    import synth
    from paper_1804_01404_amd.binding import Multiscale
    T20 = 20.0 * 41.341373335
    inc = synth.incident_table(n_macro, dt, dx, delay=0.0, E0=e0, omega=1.55 / 27.211386245988, T=T20)
    errs = []
    with Multiscale(cell, psi, precision="mixed", **kw) as ms:
        ms.attach_surrogate(nn, a_max=1e30, sentinels=[0, n_mat // 2], check_every=every, tol=1e30)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(0, n_macro, every):
            ms.step(every, inc[c:c + every + 1])
            errs.append(ms.status()["last_check"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    over = [i for i, e in enumerate(errs) if e > 1e-3]
    return {"macro_steps": n_macro, "pulse": f"cos^2, 1.55 eV, T = 20 fs, E0 {e0:g}", "checks": len(errs),
            "max_error": max(errs), "checks_over_1e-3": len(over),
            "first_step_over_1e-3": (over[0] + 1) * every if over else None,
            "ms_per_macro_step": el / n_macro * 1e3}


def bench_multiscale_cfg5(n_macro=600, timed_cells=8, n_traj=64, e0=5.34e-3, a_train=16.0):
    """The multiscale workload at its cell shape and point count: 256 medium
    points (plus 64 vacuum points on each side), each a 16^3 diamond cell with
    16 orbitals and 4^3 = 64 k-points (mixed), dX 147.6, macroscopic dt 0.32
    = 4 cell steps of 0.08, on a window of n_macro steps with a 100 a.u.
    1.55 eV pulse of peak field e0 (the 4000-step, 20 fs run is not repeated
    here). Reported:
    the cells path per macroscopic step (timed_cells steps), and the coupled
    run through a network with a 512-step window trained on n_traj
    trajectories of this cell (batch path), two sentinel cells checked every
    25 steps at the spot-check error 1e-3, with its fallback status; then the
    stated 4000-step run under the 20 fs pulse through the same network as a
    scan of the sentinel errors it meets (no fallback taken)."""
    import numpy as np
    import torch
    import synth
    from paper_1804_01404_amd import pipeline
    from paper_1804_01404_amd.binding import Multiscale
    n_sub, dt, W = 4, 0.32, 512
    cell = synth.multiscale_cell(dt=dt / n_sub)
    t0 = time.perf_counter()
    log("  cfg5 cell: ground state")
    psi, E = pipeline.ground_state(cell, imag_time=2880.0)
    t_gs = time.perf_counter() - t0
    log("  cfg5 cell: training trajectories")
    # training fields up to |A| = a_train (the incident pulse's peak |A| is
    # c e0 / omega = 12.8 at e0 = 5.34e-3 and 1.55 eV)
    P, _ = synth.random_pulse_tables(n_traj // 4, n_macro, dt, 13, e0_range=(1e-4, 1.2 * e0), ev_range=(1.0, 3.0),
                                     t_range=(40.0, 200.0))
    A_tr = np.vstack([synth.random_field_tables(n_traj - n_traj // 4, n_macro, dt, 11, a_max=a_train), P])
    J_tr, t_gen = pipeline.trajectories(cell, psi, A_tr, n_sub=n_sub, axis=0)
    a_scale, j_scale = float(np.abs(A_tr).max()), float(np.abs(J_tr).max())
    J0, _ = pipeline.trajectories(cell, psi, np.zeros((1, 32)), n_sub=n_sub, axis=0)
    t0 = time.perf_counter()
    log("  cfg5 cell: training")
    nn, losses = pipeline.train(A_tr, J_tr, synth.surrogate_init(W, 16, 2), window=W, hidden=16,
                                a_scale=a_scale, j_scale=j_scale, epochs=60, batch=256, seed=1, lr=2e-3,
                                a_fit=a_scale / 8, cosine=True)
    t_train = time.perf_counter() - t0
    dx, n_mat, n_vac = 147.6, 256, 64
    n_x = n_mat + 2 * n_vac
    inc = synth.incident_table(n_macro, dt, dx, delay=0.0, E0=e0, omega=1.55 / 27.211386245988, T=100.0)
    kw = dict(n_x=n_x, x0=n_vac, n_mat=n_mat, dx=dx, dt=dt, n_sub=n_sub, axis=0)
    og_macro = cell.og * n_mat * n_sub
    log("  cfg5 slab: cells path")
    with Multiscale(cell, psi, precision="mixed", **kw) as ms:
        ms.step(1, inc[:2])                              # creates and warms the 256 cells
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms.step(timed_cells, inc[1:timed_cells + 2])
        torch.cuda.synchronize()
        t_cells = (time.perf_counter() - t0) / timed_cells
    log("  cfg5 slab: network path")
    with nn:
        An, _, tn, st = pipeline.run_slab(cell, psi, inc, precision="mixed", nn=nn, a_max=a_scale,
                                          sentinels=[0, n_mat // 2], check_every=25, tol=1e-3, **kw)
        log("  cfg5 slab: 4000-step sentinel error scan (20 fs pulse)")
        long_scan = sentinel_error_scan(cell, psi, nn, kw, n_mat, e0, dt, dx)
    return {"workload": f"multiscale-256X: {n_mat} cells (16^3, 16 orbitals, 64 k-points, mixed) + "
                        f"{2 * n_vac} vacuum points, dX 147.6, dt 0.32 = 4 cell steps of 0.08",
            "og_per_macro_step": og_macro, "cells_ms_per_macro_step": t_cells * 1e3,
            "cells_og_steps_per_s": og_macro / t_cells,
            "surrogate_run": {"macro_steps": n_macro, "window": W, "seconds": tn,
                              "ms_per_macro_step": tn / n_macro * 1e3,
                              "speedup_over_cells_per_step": t_cells / (tn / n_macro), "status": st,
                              "sentinel_tol": 1e-3, "pulse": f"cos^2, 1.55 eV, T = 100 a.u., E0 {e0:g}"},
            "long_run_sentinel_scan": long_scan,
            "ground_state_s": t_gs, "zero_field_current_rel": float(np.max(np.abs(J0)) / j_scale),
            "training_a_max": a_scale, "trajectories": n_traj, "trajectory_steps": n_macro, "trajectories_s": t_gen, "train_s": t_train,
            "loss_first_last": [float(losses[0]), float(losses[-1])]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "c128"])
    ap.add_argument("--no-twin", action="store_true", help="skip the complex128 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch line")
    ap.add_argument("--no-multiscale", action="store_true", help="skip the learned multiscale lines")
    ap.add_argument("--no-multiscale-small", action="store_true", help="skip the small-slab multiscale line")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the 1000-step accuracy report")
    ap.add_argument("--no-mgga", action="store_true", help="skip the Tran-Blaha exchange line")
    ap.add_argument("--no-cluster", action="store_true", help="skip the 96^3 cluster line")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    ap.add_argument("--oracle-pool-child", nargs=4, metavar=("STEPS", "WORKERS", "NK", "OUT"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_pool_child:
        import numpy as np
        steps, workers, nk = (int(v) for v in args.oracle_pool_child[:3])
        out = args.oracle_pool_child[3]
        res = oracle_pool_run(steps, workers, nk)
        np.savez(out, rho=res["rho"], J=res["J"], seconds=res["seconds"], og=res["og"], workers=res["workers"])
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the multi-GPU sharding of the step is a design "
              "(orbital/k-point split, density all-reduce) and is not built; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    total = args.steps + args.warmup
    log("main line: diamond-20^3-k512")
    s = synth.single_cell_config(1, nsteps=total)
    og = s.og
    ms, dev_ms, kern, J = time_path(s, args.precision, args.steps, args.warmup)
    value = og / (ms * 1e-3)
    esz = 8 if args.precision == "mixed" else 16
    if kern["fused_ms"] is not None:
        # dominant kernel: the LDS-resident whole-step update (four stages and the
        # nonlocal term per orbital); the orbital is read and written once, so the
        # plain arithmetic bounds it
        flops = og * step_flops_per_og(s)
        achieved = flops / (kern["fused_ms"] * 1e-3) / 1e12
        peak = FP32_VALU_PEAK_TFLOPS if args.precision == "mixed" else FP64_VALU_PEAK_TFLOPS
        traffic = stored_traffic("k_fused.hip", "k_fused", "diamond20_k512") if args.precision == "mixed" else None
        t_launch = kern["fused_ms"] * 1e-3
        roofline = {"bound": "alu", "kernel": "k_fused (whole step, LDS-resident)",
                    "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                    "traffic": traffic,
                    "peak_note": "FP32 vector without packed instructions (256 CU x 4 SIMD x 16 lanes x "
                                 "2 flop x 2.4 GHz); the library is built without packed FP32"
                                 if args.precision == "mixed" else "FP64 vector",
                    "published_fp32_peak_packed": FP32_VALU_PACKED_TFLOPS,
                    "frac_of_published_packed": achieved / FP32_VALU_PACKED_TFLOPS,
                    "flops_per_launch": flops, "algorithmic_bytes_per_launch": 2 * esz * og,
                    "hbm_frac_algorithmic": 2 * esz * og / t_launch / 1e9 / HBM_PEAK_GBS,
                    "hbm_frac_counters": (traffic / t_launch / 1e9 / HBM_PEAK_GBS) if traffic else None,
                    "ms_per_launch": kern["fused_ms"]}
    else:
        # dominant kernel: a middle Horner stage, read u_s, read w, write u_{s-1}
        stage_bytes = 3 * esz * og
        achieved = stage_bytes / (kern["stage_ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "k_stage (middle Horner stage)",
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": stored_traffic("k_stage.hip", "k_stage", "diamond20_k512"),
                    "bytes_per_launch": stage_bytes, "ms_per_launch": kern["stage_ms"]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "og-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if args.precision == "mixed" else "c128",
        "data": "synthetic",
        "config": {
            "workload": "diamond-20^3-k512: 8-atom diamond cell, 20^3 grid, 16 orbitals, "
                        "8^3 k-points, s+p projectors, Hartree+PZ81, x kick, dt 0.04",
            "og_per_step": og,
            "precision": args.precision,
        },
        "roofline": roofline,
        "device_ms_per_step": dev_ms,
        "flops_per_og_step": step_flops_per_og(s),
        "kernels_ms": kern,
        "per_stage_path": per_stage_figures(s, kern, esz),
        "mfma_projection": mfma_projection(s, kern["project_ms"], esz),
        "current_finite": bool(np.all(np.isfinite(J))),
    }
    log("copy bandwidth")
    out["copy_bandwidth"] = copy_bandwidth()
    if not args.no_twin:
        log("complex128 twin")
        other = "c128" if args.precision == "mixed" else "mixed"
        ms2, dev2, kern2, _ = time_path(s, other, args.steps, args.warmup)
        out["twin"] = {"precision": other, "value": og / (ms2 * 1e-3), "ms_per_step": ms2,
                       "kernels_ms": kern2,
                       "stage_GBs": 3 * (16 if other == "c128" else 8) * og / (kern2["stage_ms"] * 1e-3) / 1e9}
    if not args.no_mgga:
        log("Tran-Blaha line")
        out["mgga"] = bench_mgga(s, args.precision, ms)
    if not args.no_cluster:
        log("cluster line (96^3, 512 orbitals)")
        out["cluster"] = bench_cluster()
    if not args.no_accuracy:
        log("accuracy report")
        out["accuracy"] = accuracy_report()
    if not args.no_batch:
        log("batch line (64 cells)")
        out["batched"] = bench_batch()
    if not args.no_multiscale:
        if not args.no_multiscale_small:
            log("multiscale line (small slab, surrogate gain)")
            out["multiscale"] = bench_multiscale()
        log("multiscale line (256 points of the 16^3 x 64-k cell)")
        out["multiscale_cfg5"] = bench_multiscale_cfg5()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host cores)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
