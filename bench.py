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
(a middle Horner stage, HIP events around back-to-back launches) and the
CPU oracle timed on a bounded sample of the same workload.
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
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (256 CU x 2.4 GHz x 256 flop/clk, packed issue)
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector


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


def cpu_baseline(system, target_s=12.0):
    """The oracle as it stands, on a bounded sample: the same cell, grid,
    orbitals and projectors with a subset of the k-points, one BLAS thread.
    The same sample then runs on the GPU (complex128 and mixed) and the
    errors against the oracle's steps are reported beside the timing."""
    import copy
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import tdks
    from paper_1804_01404_amd.binding import TDDFT
    s = system
    nk = 2

    def make(nk):
        return tdks.TDKS(s.n, s.cell, s.boundary, s.kpts[:nk], np.full(nk, 1.0 / nk), s.psi0[:nk], s.dt,
                         s.v_loc, s.projectors, hartree=s.hartree, xc=s.xc, gauge=s.gauge)
    with threadpool_limits(limits=1):
        while True:
            o = make(nk)
            t0 = time.perf_counter()
            o.step(s.A[0], s.A[1])
            o.current()
            one = time.perf_counter() - t0
            if one * 3 >= target_s or nk >= s.n_k:
                break
            nk = min(s.n_k, max(nk + 1, int(nk * target_s / (3 * one))))
        steps = max(1, min(5, int(target_s / max(one, 1e-3))))
        o = make(nk)
        J_o = np.empty((steps, 3))
        t0 = time.perf_counter()
        for n in range(steps):
            o.step(s.A[n], s.A[n + 1])
            J_o[n] = o.current()
        el = time.perf_counter() - t0
    og = s.n_orb * nk * s.n_grid
    sub = copy.copy(s)
    sub.kpts = s.kpts[:nk]
    sub.kw = np.full(nk, 1.0 / nk)
    sub.psi0 = s.psi0[:nk]
    parity = {}
    for prec in ("c128", "mixed"):
        with TDDFT(sub, precision=prec) as t:
            t.set_potential()
            J = t.propagate(s.A[:steps + 1])
            rho, _ = t.density_current()
        parity[prec] = {"density_l2_error": float(np.linalg.norm(rho - o.rho) / np.linalg.norm(o.rho)),
                        "current_error": float(np.max(np.abs(J - J_o)) / np.max(np.abs(J_o)))}
    return {"value": og * steps / el, "unit": "og-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{nk} of {s.n_k} k-points x {s.n_orb} orbitals x {s.n_grid} points, "
                      f"{steps} full steps (Taylor + density + current + Hartree + LDA), "
                      f"{el:.1f} s, NumPy FP64 with one BLAS thread",
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


def bench_cluster(steps=10, warmup=3, n_orb=64):
    """The isolated-cluster shape (96^3 box, 256 atoms with s+p projectors,
    length gauge) on the per-stage path, with n_orb of its 512 orbitals: step
    rate and the middle Horner stage against the HBM roof."""
    import numpy as np
    import synth
    s = synth.single_cell_config(2, n_orb=n_orb, nsteps=steps + warmup)
    ms, dev_ms, kern, J = time_path(s, "mixed", steps, warmup)
    stage_bytes = 3 * 8 * s.og
    return {"workload": f"cluster-96^3: 256 atoms, {n_orb} of 512 orbitals, Gamma, length gauge",
            "og_per_step": s.og, "ms_per_step": ms, "value": s.og / (ms * 1e-3), "unit": "og-steps/s",
            "stage_ms": kern["stage_ms"], "stage_GBs": stage_bytes / (kern["stage_ms"] * 1e-3) / 1e9,
            "stage_frac_hbm": stage_bytes / (kern["stage_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "observe_ms": kern["observe_ms"], "project_ms": kern["project_ms"],
            "current_finite": bool(np.all(np.isfinite(J)))}


def bench_batch(steps=30, warmup=8):
    """The uneven-batch path on 64 seeded cells (grids 12..32, up to 32
    orbitals and 8 k-points each: the 64-cell workload with the orbital and
    k-point ranges cut so that the host can generate the initial orbitals in
    seconds), mixed and complex128."""
    import torch
    import synth
    from paper_1804_01404_amd.binding import TDDFTBatch
    cells = synth.batch_cells(64, nsteps=warmup + steps, max_orb=32, max_k=8)
    og = sum(c.og for c in cells)
    out = {"workload": "batch-64cells: 64 periodic cells, grids {12,16,20,24,32}^3 at h 0.55, "
                       "8-32 orbitals, 1-8 k-points, 2-16 atoms, own cos^2 pulse each, dt 0.02",
           "og_per_step": og}
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
    out["speedup_mixed_over_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    return out


def bench_multiscale():
    """Learned multiscale coupling: a 16-point slab of 12^3 diamond-like cells
    (8 orbitals, 2^3 k-points, ground state) under a 1.55 eV pulse, run with a
    cell at every point (complex128 and mixed) and through the trained
    surrogate with two sentinel cells; the network is trained here by the
    library's kernels on 48 batch-path trajectories."""
    import numpy as np
    import synth
    from paper_1804_01404_amd import pipeline
    n_sub, dt, T = 4, 0.32, 300
    cell = synth.multiscale_cell(nk=2, n=12, n_orb=8, dt=dt / n_sub)
    psi, _ = pipeline.ground_state(cell, n_iter=3000, tau=0.06)
    A_tr = synth.random_field_tables(48, T, dt, 1, a_max=12.0)
    J_tr, t_gen = pipeline.trajectories(cell, psi, A_tr, n_sub=n_sub, axis=0)
    a_scale, j_scale = float(np.abs(A_tr).max()), float(np.abs(J_tr).max())
    t0 = time.perf_counter()
    nn, losses = pipeline.train(A_tr, J_tr, synth.surrogate_init(T, 16, 1), window=T, hidden=16,
                                a_scale=a_scale, j_scale=j_scale, epochs=150, batch=256, seed=1, lr=2e-3)
    t_train = time.perf_counter() - t0
    dx, n_mat, n_vac = 147.6, 16, 12
    n_x = n_mat + 2 * n_vac
    inc = synth.incident_table(T, dt, dx, delay=0.0, E0=3e-3, omega=1.55 / 27.211386245988, T=100.0)
    kw = dict(n_x=n_x, x0=n_vac, n_mat=n_mat, dx=dx, dt=dt, n_sub=n_sub, axis=0)
    A64, _, t64, _ = pipeline.run_slab(cell, psi, inc, precision="c128", **kw)
    A32, _, t32, _ = pipeline.run_slab(cell, psi, inc, precision="mixed", **kw)
    with nn:
        An, _, tn, st = pipeline.run_slab(cell, psi, inc, precision="mixed", nn=nn, a_max=a_scale,
                                          sentinels=[0, n_mat // 2], check_every=50, tol=0.1, **kw)
    ref = np.max(np.abs(A64))
    og_run = cell.og * n_mat * T * n_sub
    return {"workload": f"slab of {n_mat} cells (12^3, 8 orbitals, 8 k-points) + {2 * n_vac} vacuum "
                        f"points, dX 147.6, dt 0.32 = 4 cell steps, {T} steps, 1.55 eV pulse E0 3e-3",
            "cells_c128_s": t64, "cells_mixed_s": t32, "surrogate_s": tn,
            "cells_c128_og_steps_per_s": og_run / t64, "cells_mixed_og_steps_per_s": og_run / t32,
            "speedup_surrogate_over_c128_cells": t64 / tn, "speedup_mixed_over_c128_cells": t64 / t32,
            "field_error_mixed_cells": float(np.max(np.abs(A32 - A64)) / ref),
            "field_error_surrogate": float(np.max(np.abs(An - A64)) / ref),
            "surrogate_status": st, "train_s": t_train, "trajectories_s": t_gen,
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
    ap.add_argument("--no-multiscale", action="store_true", help="skip the learned multiscale line")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the 1000-step accuracy report")
    ap.add_argument("--no-mgga", action="store_true", help="skip the Tran-Blaha exchange line")
    ap.add_argument("--no-cluster", action="store_true", help="skip the 96^3 cluster line")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    args = ap.parse_args()
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
        roofline = {"bound": "alu", "kernel": "k_fused (whole step, LDS-resident)",
                    "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                    "traffic": stored_traffic("k_fused.hip", "k_fused", "diamond20_k512"),
                    "flops_per_launch": flops, "algorithmic_bytes_per_launch": 2 * esz * og,
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
    # issued MFMA work of one projection launch (per-stage path): one 16x16x4
    # FP64 MFMA per four sphere entries, per atom and group of eight orbitals
    n_groups = (s.n_orb * s.n_k + 7) // 8
    mfma_flops = sum(n_groups * -(-p.npts // 4) * 2 * 16 * 16 * 4 for p in s.projectors)
    mfma_tflops = mfma_flops / (kern["project_ms"] * 1e-3) / 1e12

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
        "mfma_projection": {"issued_tflops": mfma_tflops, "peak": FP64_MFMA_PEAK_TFLOPS,
                            "frac": mfma_tflops / FP64_MFMA_PEAK_TFLOPS},
        "current_finite": bool(np.all(np.isfinite(J))),
    }
    if not args.no_twin:
        other = "c128" if args.precision == "mixed" else "mixed"
        ms2, dev2, kern2, _ = time_path(s, other, args.steps, args.warmup)
        out["twin"] = {"precision": other, "value": og / (ms2 * 1e-3), "ms_per_step": ms2,
                       "kernels_ms": kern2,
                       "stage_GBs": 3 * (16 if other == "c128" else 8) * og / (kern2["stage_ms"] * 1e-3) / 1e9}
    if not args.no_mgga:
        out["mgga"] = bench_mgga(s, args.precision, ms)
    if not args.no_cluster:
        out["cluster"] = bench_cluster()
    if not args.no_accuracy:
        out["accuracy"] = accuracy_report()
    if not args.no_batch:
        out["batched"] = bench_batch()
    if not args.no_multiscale:
        out["multiscale"] = bench_multiscale()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
