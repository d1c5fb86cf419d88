#!/usr/bin/env python3
"""Throughput of the screened Fock-like exchange operator on one MI355X.

A step is one full application V_x[u] u over every (k, i, k', j) pair of the
workload (kernel tables resident, orbitals already in HBM), in the fused FP32
form (complex64 pair FFTs; FP32 partial sums over at most 16 bands, added into
Neumaier-compensated FP64 sums; at 32^3 each target split over two CUs, and,
since the targets are the sources, each pair of k-points transformed once: the
W of (k', j) on (k, i) is the conjugate of that of (k, i) on (k', j)).
The plain FP64 path runs the same orbitals for the speed-up and the per-k
error of the FP32 form; the FP64 oracle runs a bounded sample on the host.

Prints one JSON line. Default workload: 32^3 grid, 6x6x6 k-mesh, 16 bands
(11,943,936 pairs per step).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VALU_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E

# Device-memory traffic of one fused 32^3 launch, from two rocprofv3 --pmc runs of
# this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
# the same counter reads for a 1 GiB device copy in the same run. Valid only for
# the kernel sources whose digest is recorded; a changed kernel reports null.
COUNTER_TRAFFIC = {
    "sources_sha256": "ed3c6062830b6c85389eb1575f4bbd0ce3d19419dcf04a584a62100051d25fd3",
    "workload": 2,
    "fetch_kib": 1353198492.3125, "write_kib": 3354108010.0,
    "fetch_scale": 1048576 / 524319.625, "write_scale": 1.0,
}
# the sources of the dominant 32^3 kernel (split32_kernel) whose dispatches the counters measured
KERNEL_SOURCES = ("paper_1507_05156_amd/csrc/split32.hip", "paper_1507_05156_amd/csrc/fft_reg.hpp",
                  "paper_1507_05156_amd/csrc/fused_common.hpp", "paper_1507_05156_amd/csrc/kernels.hpp")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(workload: int):
    """Scaled read + write bytes per launch, or None when the record does not
    belong to these kernel sources and this workload."""
    c = COUNTER_TRAFFIC
    if c["sources_sha256"] != kernel_sources_digest() or c["workload"] != workload or c["fetch_kib"] is None:
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def symmetric_pair_ffts(n: int, nk: int, nb: int) -> int | None:
    """Pairs whose FFTs the 32^3 split kernel runs when it uses the pair symmetry
    (u as targets and sources, at least 3 k-points): each target runs the source
    k-points k + d, d = 0 .. nk/2. None when the kernel runs every pair."""
    if n != 32 or nk < 3 or os.environ.get("FOCKMI_SPLIT_SYM", "1") == "0":
        return None
    return nk * nb * (nk // 2 + 1) * nb


def flops_per_pair(nr: int) -> float:
    """Nominal algorithmic flops of one pair: two complex 3D FFTs (5 N log2 N each)
    plus pair product (6), kernel multiply (2) and multiply-accumulate (8) per point."""
    return 10.0 * nr * math.log2(nr) + 16.0 * nr


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_SAMPLE = {}


def _oracle_worker_init(shm_name, shape, kp, cell, omega):
    """Pool worker: one BLAS thread, the oracle imported, the shared sample attached."""
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    import numpy as np
    from multiprocessing import shared_memory

    import oracle  # noqa: F401
    shm = shared_memory.SharedMemory(name=shm_name)
    _ORACLE_SAMPLE.update(shm=shm, u=np.ndarray(shape, dtype=np.complex128, buffer=shm.buf), kp=kp, cell=cell,
                          omega=omega)


def _oracle_worker_row(row):
    import oracle
    s = _ORACLE_SAMPLE
    oracle.fock_apply(s["u"], s["u"], s["kp"], s["cell"], s["omega"], rows=[row])
    return row


def cpu_baseline(u, kp, cell, omega, nsrc, workers):
    """The FP64 oracle, unmodified, on output rows of the workload against its first nsrc
    source k-points: one row on one thread, then `workers` rows at once, one per process
    (each with one BLAS thread), over a shared copy of the sample. Returns a dict."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits

    us = np.ascontiguousarray(u[:nsrc])
    kps = np.ascontiguousarray(kp[:nsrc])
    nb = u.shape[1]
    pairs_row = nsrc * nb
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.fock_apply(us, us, kps, cell, omega, rows=[(0, 0)])
        dt1 = time.perf_counter() - t0
    rows = [(k, i) for k in range(nsrc) for i in range(nb)][:workers]
    shm = shared_memory.SharedMemory(create=True, size=us.nbytes)
    try:
        np.ndarray(us.shape, dtype=us.dtype, buffer=shm.buf)[...] = us
        ctx = mp.get_context("spawn")
        with ctx.Pool(len(rows), initializer=_oracle_worker_init,
                      initargs=(shm.name, us.shape, kps, cell, omega)) as pool:
            pool.map(_oracle_worker_row, [(0, 0)] * len(rows), chunksize=1)  # every worker started and warm
            t0 = time.perf_counter()
            pool.map(_oracle_worker_row, rows, chunksize=1)
            dtp = time.perf_counter() - t0
    finally:
        shm.close()
        shm.unlink()
    return {"value": len(rows) * pairs_row / dtp, "unit": "pairs/s", "cores": len(rows), "kind": "oracle",
            "sample": f"{len(rows)} output rows (k, i) at once, one per process, each against {nsrc} source k-points x "
                      f"{nb} bands = {pairs_row} pairs of the workload, {dtp:.1f} s",
            "one_thread_pairs_per_s": pairs_row / dt1, "one_thread_sample_s": dt1,
            "host_cpu_count": os.cpu_count(), "host": host_cpu_model()}


def copy_bandwidth(torch, dev, mib=1024, reps=5):
    """Best device-to-device copy rate (bytes read + written per second, GB/s)
    of a mib-MiB buffer: the HBM rate a plain copy kernel reaches."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2.0 * (mib << 20) / best / 1e9


def _timed(fn, reps, torch):
    """Average wall seconds of fn() over reps calls, bracketed by device synchronisation."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def extra_legs(torch, np, synth, Plan, omega, dev, ud_c2, plan32_c2):
    """Timings of the other calls on the path, each on its own workload:
    the batched launch over three uneven cells in each of its forms (against the
    same cells launched one by one, and against the plain FP64 path for the error), the FP64
    adjoint and Taylor-4 step at 24^3 / 64 k / 16 bands, and E_x (FP32 form) and
    the FP64 orthonormalisation on the bench workload, the down-sampled sum as
    the paper runs it (12^3 k-points, 4^3 source sub-mesh, 16 bands), the
    work of the field against the energy functional at two time steps, and the
    eigenstates after a pulse with the excited-electron density."""
    out = {}
    # ------------------------------------------- batched launch (three cells), every form
    cells, us = [], []
    for ci in range(3):
        a, kp, u = synth.workload(4, ci)
        cells.append(dict(n=u.shape[2], a=a, kpts=kp, nb=u.shape[1], omega=omega))
        us.append(torch.from_numpy(u).to(dev))
    pairs = sum((c["kpts"].shape[0] * c["nb"]) ** 2 for c in cells)
    pb = Plan(cells, prec="fp32")
    pb.apply_batched(us)
    t_batched = _timed(lambda: pb.apply_batched(us), 3, torch)
    t_cells = _timed(lambda: [pb.apply(us[ci], cell=ci) for ci in range(3)], 3, torch)
    outs = pb.apply_batched(us)
    # every form of the batched launch, forced through a tuning cache
    import tempfile
    forms = {}
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "tune.json")
        Plan(cells, prec="fp32", tune_cache=path).apply_batched(us)
        data = json.load(open(path))
        key = [k for k in data if "/batched/" in k][0]
        tuned = dict(data[key])
        for name, form in (("persistent_kernel", 0), ("forked_cells", 1), ("cells_in_sequence", 2)):
            data[key].update(form=form, wg_per_cu=1)
            json.dump(data, open(path, "w"))
            pf = Plan(cells, prec="fp32", tune_cache=path)
            pf.apply_batched(us)
            forms[name + "_ms"] = _timed(lambda: pf.apply_batched(us), 3, torch) * 1e3
            del pf
    errs = []
    for ci, c in enumerate(cells):
        p64 = Plan(c, prec="fp64")
        ref = p64.apply(us[ci])
        nk = c["kpts"].shape[0]
        rel = ((outs[ci] - ref).reshape(nk, -1).norm(dim=1) / ref.reshape(nk, -1).norm(dim=1)).max().item()
        errs.append(rel)
        del p64, ref
    out["batched_3cells"] = {
        "cells": "16^3/27 k/8 b + 20^3/64 k/12 b + 24^3/125 k/16 b", "pairs": pairs,
        "batched_graph_pairs_per_s": pairs / t_batched, "batched_graph_ms": t_batched * 1e3,
        "default_form": "forked cells (each cell's fused kernel on its own stream, one captured graph)",
        "forms_ms": forms, "tuner_choice": tuned,
        "per_cell_launches_pairs_per_s": pairs / t_cells, "per_cell_launches_ms": t_cells * 1e3,
        "max_rel_err_per_k_vs_fp64": max(errs), "rel_err_per_cell": errs}
    del pb, us, outs
    print(f"[bench] batched 3 cells: {pairs / t_batched:.4e} pairs/s (per-cell launches {pairs / t_cells:.4e})",
          file=sys.stderr, flush=True)
    # ------------------------------------------------ FP64 adjoint and Taylor-4 step, 24^3
    a, kp, u = synth.workload(3)
    nk, nb = u.shape[0], u.shape[1]
    p3 = (nk * nb) ** 2
    u3 = torch.from_numpy(u).to(dev)
    plan = Plan(dict(n=u.shape[2], a=a, kpts=kp, nb=nb, omega=omega), prec="fp64")
    g = torch.from_numpy(synth.random_fields(u.shape, seed=7)).to(dev)
    plan.vjp(u3, u3, g)
    t_vjp = _timed(lambda: plan.vjp(u3, u3, g), 1, torch)
    psi = u3.clone()
    t_step = _timed(lambda: plan.taylor_step(psi, [0.0, 0.0, 0.01], 0.02, 0.25), 1, torch)
    t_apply = _timed(lambda: plan.apply(u3), 1, torch)
    ref = plan.apply(u3)
    out["fp64_24cube_64k_16b"] = {
        "pairs_per_apply": p3, "apply_ms": t_apply * 1e3, "apply_pairs_per_s": p3 / t_apply,
        "vjp_ms": t_vjp * 1e3, "vjp_pair_ffts_per_s": 3 * p3 / t_vjp,
        "taylor4_step_ms": t_step * 1e3, "taylor4_pair_ffts_per_s": 4 * p3 / t_step}
    print(f"[bench] fp64 24^3: apply {t_apply * 1e3:.0f} ms, vjp {t_vjp * 1e3:.0f} ms, "
          f"taylor step {t_step * 1e3:.0f} ms", file=sys.stderr, flush=True)
    del plan, psi
    # the same calls through the fused FP64 form
    planf = Plan(dict(n=u.shape[2], a=a, kpts=kp, nb=nb, omega=omega), prec="fp64f")
    got = planf.apply(u3)
    rel = ((got - ref).reshape(nk, -1).norm(dim=1) / ref.reshape(nk, -1).norm(dim=1)).max().item()
    planf.vjp(u3, u3, g)
    t_vjpf = _timed(lambda: planf.vjp(u3, u3, g), 1, torch)
    psi = u3.clone()
    t_stepf = _timed(lambda: planf.taylor_step(psi, [0.0, 0.0, 0.01], 0.02, 0.25), 1, torch)
    t_applyf = _timed(lambda: planf.apply(u3, out=got), 3, torch)
    out["fp64_fused_24cube_64k_16b"] = {
        "apply_ms": t_applyf * 1e3, "apply_pairs_per_s": p3 / t_applyf, "speedup_vs_plain": t_apply / t_applyf,
        "max_rel_err_per_k_vs_plain": rel,
        "vjp_ms": t_vjpf * 1e3, "taylor4_step_ms": t_stepf * 1e3}
    print(f"[bench] fp64 fused 24^3: apply {t_applyf * 1e3:.0f} ms ({t_apply / t_applyf:.2f}x plain), "
          f"vjp {t_vjpf * 1e3:.0f} ms, taylor step {t_stepf * 1e3:.0f} ms", file=sys.stderr, flush=True)
    del planf, u3, g, psi, got, ref
    # ------------------- down-sampling as the paper runs it: 12^3 k-mesh, 4^3 source sub-mesh
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(12, cell)
    src = synth.submesh(12, 3)
    u = synth.orbitals(16, cell, kp, 16, seed=synth.seed_for(5, 0))
    ud = torch.from_numpy(u).to(dev)
    del u
    desc = dict(n=16, a=cell, kpts=kp, nb=16, omega=omega, src=src)
    pairs_ds = (len(kp) * 16) * (len(src) * 16)
    p32 = Plan(desc, prec="fp32")
    o32 = p32.apply(ud)
    t32 = _timed(lambda: p32.apply(ud, out=o32), 3, torch)
    p64 = Plan(desc, prec="fp64")
    o64 = p64.apply(ud)
    t64 = _timed(lambda: p64.apply(ud, out=o64), 1, torch)
    nk = len(kp)
    rel = ((o32 - o64).reshape(nk, -1).norm(dim=1) / o64.reshape(nk, -1).norm(dim=1)).max().item()
    del p64
    p64f = Plan(desc, prec="fp64f")
    o64f = p64f.apply(ud)
    t64f = _timed(lambda: p64f.apply(ud, out=o64f), 3, torch)
    rel64f = ((o64f - o64).reshape(nk, -1).norm(dim=1) / o64.reshape(nk, -1).norm(dim=1)).max().item()
    del p64f, o64f
    out["downsampled_12cube_k_4cube_q"] = {
        "grid": "16^3", "k_points": nk, "source_k_points": len(src), "bands": 16, "pairs": pairs_ds,
        "fp32_pairs_per_s": pairs_ds / t32, "fp32_ms": t32 * 1e3,
        "fp64_plain_pairs_per_s": pairs_ds / t64, "fp64_plain_ms": t64 * 1e3,
        "fp64_fused_pairs_per_s": pairs_ds / t64f, "fp64_fused_ms": t64f * 1e3,
        "fp64_fused_max_rel_err_per_k_vs_plain": rel64f,
        "fp32_max_rel_err_per_k_vs_fp64": rel,
        "pairs_without_downsampling": (nk * 16) ** 2}
    del p32, o32, o64, ud
    print(f"[bench] down-sampled 12^3 k / 4^3 q at 16^3: fp32 {pairs_ds / t32:.4e} pairs/s, "
          f"fp64 plain {pairs_ds / t64:.4e}, fp64 fused {pairs_ds / t64f:.4e}", file=sys.stderr, flush=True)
    # ---------------- work of the field vs the energy functional (Eqs. (23)-(24)), two steps
    from paper_1507_05156_amd import dynamics
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = torch.from_numpy(synth.orbitals(16, cell, kp, 4, seed=synth.seed_for(6, 0))).to(dev)
    pw = Plan(dict(n=16, a=cell, kpts=kp, nb=4, omega=omega), prec="fp64")
    leg = {"pulse": "A0 = 0.5 (A/c), T_d = 0.8 a.u., 1.55 eV, alpha = 1/4, FP64"}
    for pc in (False, True):
        runs = {}
        for dt_w in (0.02, 0.01):
            nsteps = int(round(0.8 / dt_w))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e_ex, ow, _ = dynamics.work_and_energy(pw, u, 0.5, dt_w, nsteps, predictor_corrector=pc)
            torch.cuda.synchronize()
            runs[dt_w] = (e_ex, ow, (time.perf_counter() - t0) / nsteps)
        (e1, w1, s1), (e2, w2, s2) = runs[0.02], runs[0.01]
        leg["predictor_corrector" if pc else "h_at_t"] = {
            "dt_0.02": {"E_ex": e1, "Omega_W": w1, "ms_per_step_with_current": s1 * 1e3},
            "dt_0.01": {"E_ex": e2, "Omega_W": w2, "ms_per_step_with_current": s2 * 1e3},
            "gap_ratio": abs(w1 - e1) / abs(w2 - e2),
            "extrapolated_E_ex": 2 * e2 - e1, "extrapolated_Omega_W": 2 * w2 - w1}
    out["work_vs_energy_16cube_8k_4b"] = leg
    del pw, u
    # ------------- excited electrons after a pulse (Sec. IV B, Eqs. (25)-(26)): 16^3, 8 k, 16 bands
    cell = synth.cubic_cell()
    kp = synth.gamma_mesh(2, cell)
    u = torch.from_numpy(synth.orbitals(16, cell, kp, 16, seed=synth.seed_for(7, 0))).to(dev)
    v = torch.from_numpy(synth.model_vloc(16)).to(dev)
    px = Plan(dict(n=16, a=cell, kpts=kp, nb=16, omega=omega), prec="fp64f")
    px.eigensolve(u, vloc=v, tol=1e-4, maxit=5)  # warm-up (allocations, tables)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi0, eps0, res0, it0, conv0 = px.eigensolve(u, vloc=v, alpha=0.25, tol=1e-8, maxit=400)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    leg = {"setting": "silicon model potential, alpha = 1/4, FP64 fused form; psi(0) = the 16 lowest states of "
                      "h[u] for seeded orbitals u; 40 Taylor steps of dt = 0.02 under the 1.55 eV pulse; "
                      "eigenstates of h(t_f) from psi(t_f), tol 1e-8",
           "eigensolve_ms": t_eig * 1e3, "eigensolve_iterations": it0, "eigensolve_converged": conv0,
           "ms_per_iteration": t_eig * 1e3 / max(it0, 1), "pairs_per_h_application": (len(kp) * 16) ** 2,
           "valence_density": 2.0 * 16 / abs(np.linalg.det(cell))}
    for A0 in (0.0, 0.5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nex, _, it, conv, _, _ = dynamics.excited_density_after_pulse(px, psi0, A0, 0.02, 40, vloc=v, tol=1e-8)
        torch.cuda.synchronize()
        leg[f"A0_{A0}"] = {"n_ex": nex, "eigensolve_iterations": it, "converged": conv,
                           "seconds_propagation_and_eigensolve": time.perf_counter() - t0}
    out["excited_16cube_8k_16b"] = leg
    print(f"[bench] excited density 16^3/8k/16b: eigensolve {t_eig * 1e3:.0f} ms ({it0} iterations), "
          f"n_ex {leg['A0_0.0']['n_ex']:.3e} (no pulse) / {leg['A0_0.5']['n_ex']:.3e} (A0 = 0.5)",
          file=sys.stderr, flush=True)
    del px, u, v, psi0
    # ------------- one GPU's share of an 8-GPU k-point decomposition of the bench workload
    nk2 = ud_c2.shape[0]
    share = nk2 // 8
    part = plan32_c2.apply_krange(ud_c2, 0, share)
    t_share = _timed(lambda: plan32_c2.apply_krange(ud_c2, 0, share, out=part), 1, torch)
    pairs_share = share * ud_c2.shape[1] * nk2 * ud_c2.shape[1]
    out["shard_of_8_32cube"] = {"output_k_points": share, "pairs": pairs_share, "ms": t_share * 1e3,
                                "pairs_per_s": pairs_share / t_share}
    print(f"[bench] one of 8 k-point shards at 32^3 ({share} k): {t_share * 1e3:.0f} ms, "
          f"{pairs_share / t_share:.4e} pairs/s", file=sys.stderr, flush=True)
    del part
    # ------------------------------------- E_x and orthonormalisation, the bench workload
    t_e = _timed(lambda: plan32_c2.energy(ud_c2), 1, torch)
    psi = ud_c2.clone()
    t_o = _timed(lambda: plan32_c2.orthonormalize(psi), 1, torch)
    out["energy_fp32_ms"] = t_e * 1e3
    out["orthonormalize_fp64_ms"] = t_o * 1e3
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, help="2: 32^3/216k/16b (default); 1: 24^3/64k/16b")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed plain FP64 applications (0 = skip)")
    ap.add_argument("--fp64-form", choices=["plain", "fused"], default="plain",
                    help="FP64 comparison path: the plain staged path (the reference of the speed-up), or the "
                         "fused FP64 form (cubic 16^3-24^3 grids)")
    ap.add_argument("--cpu-sources", type=int, default=96, help="source k-points in the oracle sample (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes run at once (default: the host's CPU count, at most 16)")
    ap.add_argument("--extras", type=int, default=1, help="1: also time the batched launch, adjoint, Taylor step, a device copy, "
                    "energy and orthonormalisation")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (a known-size kernel for HBM counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU decomposition is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1507_05156_amd import synth
    from paper_1507_05156_amd.api import Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    omega = synth.OMEGA_HSE
    t_gen = time.perf_counter()
    cell, kp, u = synth.workload(args.workload)
    nk, nb, n = u.shape[0], u.shape[1], u.shape[2]
    nr = n ** 3
    pairs = (nk * nb) ** 2
    print(f"[bench] workload {args.workload}: {n}^3 grid, {nk} k, {nb} bands, {pairs} pairs/step "
          f"(inputs generated in {time.perf_counter() - t_gen:.1f}s)", file=sys.stderr, flush=True)
    ud = torch.from_numpy(u).to(dev)
    desc = dict(n=n, a=cell, kpts=kp, nb=nb, omega=omega)
    if args.calibrate_copy_mb > 0:
        src = torch.ones(args.calibrate_copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------------------------------------------------------- FP32 form
    plan32 = Plan(desc, prec="fp32")
    out32 = torch.empty_like(ud)
    for _ in range(args.warmup):
        plan32.apply(ud, out=out32)
    torch.cuda.synchronize()
    first = out32.clone() if args.warmup > 0 else None
    plan32.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        plan32.apply(ud, out=out32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = plan32.profile_read()
    repeat_equal = bool((first == out32).all()) if first is not None else None
    del first
    plan32.profile(False)
    elapsed = t1 - t0
    value = args.steps * pairs / elapsed
    kern_avg_s = kern_ms / 1e3 / max(launches, 1)
    achieved_tflops = flops_per_pair(nr) * pairs / kern_avg_s / 1e12
    alg_bytes = pairs * nr * 8.0   # one complex64 orbital streamed per pair
    achieved_gbs = alg_bytes / kern_avg_s / 1e9
    traffic = counter_traffic(args.workload)
    sym_pairs = symmetric_pair_ffts(n, nk, nb)
    print(f"[bench] fp32: {elapsed / args.steps * 1e3:.1f} ms/step, {value:.4e} pairs/s, "
          f"kernel {kern_avg_s * 1e3:.1f} ms", file=sys.stderr, flush=True)
    e32 = plan32.energy(ud)

    # ---------------------------------------------------------- plain FP64 path
    fp64 = {}
    if args.fp64_steps > 0:
        plan64 = Plan(desc, prec="fp64" if args.fp64_form == "plain" else "fp64f")
        out64 = torch.empty_like(ud)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            plan64.apply(ud, out=out64)
        torch.cuda.synchronize()
        dt64 = (time.perf_counter() - t0) / args.fp64_steps
        diff = (out32 - out64).reshape(nk, -1).norm(dim=1)
        refn = out64.reshape(nk, -1).norm(dim=1)
        rel = (diff / refn).cpu().numpy()
        w = (2.0 / 2.0) / nk * abs(np.linalg.det(cell)) / nr
        e64 = (w * torch.vdot(ud.reshape(-1), out64.reshape(-1))).item()
        tag = "fp64_plain" if args.fp64_form == "plain" else "fp64_fused"
        fp64 = {f"{tag}_pairs_per_s": pairs / dt64, f"{tag}_ms_per_step": dt64 * 1e3,
                f"speedup_fp32_vs_{tag}": value / (pairs / dt64)}
        fp64.update(dict(fp32_max_rel_err_per_k_vs_fp64=float(rel.max()),
                         fp32_median_rel_err_per_k_vs_fp64=float(np.median(rel)),
                         ex_fp32=e32.real, ex_fp64=e64.real,
                         ex_rel_err_fp32_vs_fp64=abs(e32.real - e64.real) / abs(e64.real)))
        print(f"[bench] {tag.replace('_', ' ')}: {dt64 * 1e3:.1f} ms/step, max per-k rel err of fp32 {rel.max():.2e}",
              file=sys.stderr, flush=True)
        del plan64, out64

    extras = extra_legs(torch, np, synth, Plan, omega, dev, ud, plan32) if args.extras else None
    copy_gbs = copy_bandwidth(torch, dev) if args.extras else None

    # ------------------------------------------------------------ CPU baseline
    cpu = None
    if args.cpu_sources > 0:
        nsrc = min(args.cpu_sources, nk)
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(u, kp, cell, omega, nsrc, workers)
        print(f"[bench] cpu oracle: {cpu['value']:.1f} pairs/s on {cpu['cores']} processes "
              f"({cpu['one_thread_pairs_per_s']:.1f} on one thread; host has {cpu['host_cpu_count']} CPUs)",
              file=sys.stderr, flush=True)

    rec = {
        "metric": "Fock pair-FFTs/s: FP64 plain vs FP32 batched at \u22641e-6 rel err; % HBM peak",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "accumulate_dtype": "f64 (Neumaier-compensated sums of FP32 partial sums over at most 16 bands)",
        "data": "synthetic seeded orbitals",
        "config": {"workload": f"{n}^3 grid, {round(nk ** (1 / 3))}^3 Gamma-centred k-mesh ({nk} k), {nb} bands, "
                               f"a=10.26 bohr cubic, omega={omega} bohr^-1",
                   "pairs_per_step": pairs, "ffts_per_step": 2 * (sym_pairs or pairs),
                   "pairs_transformed_per_step": sym_pairs or pairs,
                   "kernel": ("split FP32 pair kernel (each target on two CUs of one XCD"
                              + ("; pair symmetry: each pair of k-points transformed once)" if sym_pairs else ")"))
                   if n == 32 else "fused FP32 pair kernel"},
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "split32_kernel" if n == 32 else f"fused_apply_kernel<{n}>", "kernel_ms_avg": kern_avg_s * 1e3, "launches": launches,
                     "alg_bytes_per_pair": nr * 8, "alg_bytes_per_launch": alg_bytes, "pairs_per_launch": pairs,
                     "traffic_bytes_per_pair": traffic / pairs if traffic else None,
                     "traffic_GBs": traffic / kern_avg_s / 1e9 if traffic else None,
                     "valu_achieved_TFLOPs": achieved_tflops, "valu_peak_TFLOPs": FP32_VALU_PEAK_TFLOPS,
                     "valu_frac": achieved_tflops / FP32_VALU_PEAK_TFLOPS,
                     "valu_peak_unpacked_TFLOPs": FP32_VALU_PEAK_TFLOPS / 2,
                     "valu_frac_unpacked": achieved_tflops / (FP32_VALU_PEAK_TFLOPS / 2),
                     "flops_per_pair": flops_per_pair(nr),
                     "valu_executed_TFLOPs": flops_per_pair(nr) * (sym_pairs or pairs) / kern_avg_s / 1e12,
                     "note": ("achieved counts the application's algorithmic bytes, one complex64 orbital per "
                              "(target, source) pair; with the pair symmetry the kernel transforms "
                              f"{sym_pairs} of the {pairs} pairs" if sym_pairs else None),
                     "copy_GBs_measured": copy_gbs,
                     "frac_of_measured_copy": achieved_gbs / copy_gbs if copy_gbs else None},
        "ffts_per_s": 2 * (sym_pairs or pairs) * args.steps / elapsed,
        "fp32_repeat_bitwise_equal": repeat_equal,
        "cpu_baseline": cpu,
    }
    rec.update(fp64)
    if extras is not None:
        rec["other_calls"] = extras
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
