#!/usr/bin/env python3
"""Throughput of the TENO residual hot path on one MI355X.

One step = one SSP-RK3 step of the whole hot path on the device: the
constant-CFL time step, then three stages of (reconstruction with TENO
selection -> HLL face fluxes -> residual gather -> stage update).  The
headline workload is 5th-order TENO on a jittered periodic 512 x 512 x 2
mesh (524,288 triangles) with the seeded four-region random-line state.

Prints ONE JSON line (see the end of main()).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell-updates/s per RK stage (5th-order, Euler) + HBM GB/s %peak; "
          "adjoint/forward time")
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hpp", "tables.h"):
        with open(os.path.join(ROOT, "paper_2105_02127_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_stage(order: int) -> int:
    """Bytes one cell must move per RK stage, the fused minimum of the
    method: its least-squares operators (3 small 5 x 11 + the large
    nu x nl, FP64), its stencil indices (33 + nl int32), its state, U^n and
    U^(k+1) (32 B each), and its share of the face geometry (1.5 faces x
    (normal, |A|, two cell ids) + its face list and |V|: 68 B).  Stencil
    gathers served from cache and intermediates are not counted: 2,100 /
    3,060 / 4,980 / 8,340 B at orders 3-6."""
    r = order - 1
    nu = (r + 1) * (r + 2) // 2 - 1
    nl = (r + 1) * (r + 2) - 1
    ops = 8 * (3 * 5 * 11 + nu * nl)
    idx = 4 * (33 + nl)
    return ops + idx + 3 * 32 + 68


def traffic_from_profiles(workload: str):
    """HBM bytes per reconstruction launch from the committed rocprofv3 PMC
    summary, or None when the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"k_reconstruct_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stream_triad_gbs(torch, n=1 << 26, reps=20):
    """Achievable HBM bandwidth on this GPU for context: a = b + s c over
    three 512 MiB FP64 arrays (torch's elementwise kernel), 3 x 8 n bytes per
    pass, best of `reps` passes timed with events."""
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    for _ in range(3):
        torch.add(b, c, alpha=0.5, out=a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.add(b, c, alpha=0.5, out=a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b, c
    return 3 * 8 * n / (best * 1e-3) / 1e9


def cpu_baseline(mesh, U, order, fallback, steps=1, single=True):
    """The CPU oracle (as it stands) on the same mesh and state: one full
    SSP-RK3 step over every cell, set-up excluded, all host threads; then
    (single) one residual evaluation on one thread."""
    import oracle
    threads = oracle.get_threads()
    om = oracle.OracleMesh(mesh.xy, mesh.tri)
    t0 = time.perf_counter()
    om.setup(oracle.params(order=order, fallback=fallback))
    t_setup = time.perf_counter() - t0
    dt = om.dt(U, 0.4)
    t0 = time.perf_counter()
    Uc = U
    for _ in range(steps):
        Uc = om.rk_step(Uc, dt)["U"]
    t = time.perf_counter() - t0
    out = {"value": mesh.n_cell * 3 * steps / t, "unit": "cell-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{steps} full SSP-RK3 step(s) ({3 * steps} stages) over all {mesh.n_cell} cells "
                     f"of the same mesh and state; oracle set-up ({t_setup:.1f} s) excluded",
           "seconds": t}
    if single:
        # one host thread, one residual evaluation (one stage) over every cell
        # of a 128x128x2 mesh of the same kind (the cost per cell does not
        # depend on the mesh size; the full mesh would take about half a
        # minute on one thread)
        from paper_2105_02127_amd import inputs
        ms = inputs.jittered_periodic_mesh(128, mesh.seed)
        Us = inputs.random_lines(ms)
        oms = oracle.OracleMesh(ms.xy, ms.tri)
        oms.setup(oracle.params(order=order, fallback=fallback))
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oms.residual(Us)
        t1 = time.perf_counter() - t0
        oracle.set_threads(threads)
        out["single_thread"] = {"value": ms.n_cell / t1, "unit": "cell-updates/s", "cores": 1,
                                "sample": f"one residual evaluation over the {ms.n_cell} cells of a "
                                          f"128x128x2 mesh of the same kind", "seconds": t1}
    return out


def adjoint_timing(torch, teno, inputs, steps=200, checkpoint_every=20):
    """Forward rollout versus backward on the adjoint workload (TENO4,
    256x256x2 cells, 200 steps).  Two memory plans: every step kept by the
    forward pass (17.5 GB here, no recompute; the headline ratio), and a
    checkpoint every 20 steps with each segment recomputed in the backward
    pass.  The ratio divides by the plain forward rollout, a simulation that
    keeps nothing."""
    from paper_2105_02127_amd import adjoint
    w, mesh, U0 = inputs.make_workload(4)
    lm = teno.Mesh(mesh.xy, mesh.tri).setup(order=w["order"], fallback=1)
    sv = teno.Solver(lm)
    U0d = torch.as_tensor(U0[lm.perm], device="cuda")
    center, radius = inputs.adjoint_loss_disc(mesh)
    v = inputs.unwrapped_vertices(mesh)
    e1, e2 = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    wts = torch.as_tensor((area * inputs.disc_mask(mesh, center, radius))[lm.perm], device="cuda")
    adjoint.forward_rollout(sv, U0d, 5)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    adjoint.forward_rollout(sv, U0d, steps, checkpoint_every=checkpoint_every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0

    def run(K, warm):
        # a first untimed run of the same size lets the later one take its
        # stage and face-state buffers from torch's caching allocator
        for _ in range(2 if warm else 1):
            x = U0d.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            UT, _ = adjoint.rollout(sv, x, steps, checkpoint_every=K)
            loss = adjoint.pressure_squared_loss(UT, wts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            g = x.grad
            del x, UT, loss
        return t1 - t0, t2 - t1, g

    f_keep, b_keep, g_keep = run(None, True)
    f_ck, b_ck, g_ck = run(checkpoint_every, True)
    same = bool(torch.equal(g_keep, g_ck))
    del g_keep, g_ck
    torch.cuda.empty_cache()
    return {"workload": w["name"], "n_cell": mesh.n_cell, "steps": steps,
            "forward_s": t_fwd, "backward_s": b_keep, "adjoint_over_forward": b_keep / t_fwd,
            "memory_plan": "every step kept (stages, flags, face states), no recompute",
            "forward_keeping_s": f_keep,
            "checkpointed": {"checkpoint_every": checkpoint_every, "forward_s": f_ck,
                             "backward_s": b_ck, "adjoint_over_forward": b_ck / t_fwd,
                             "note": "backward recomputes each segment from its checkpoint"},
            "gradients_bitwise_equal": same}


# Tab. runtime analysis (Sec. 5.10), KHI on 577,416 triangles, 56 CPU threads:
# t_norm = reconstruction seconds per iteration per element, as printed.
PAPER_KHI_T_NORM = {"TENO3": 1.32e-6, "TENO4": 1.66e-6, "TENO5": 1.90e-6, "TENO6": 2.20e-6,
                    "CWENO5": 1.88e-6, "CWENO6": 2.17e-6}


def khi_timing(torch, teno, inputs, steps=10, warmup=2):
    """The paper's KHI timing workload (Sec. 5.7, 5.10) at its size: TENO3-6
    and CWENO5-6 on the 537x537x2 mesh (576,738 cells), per-stage throughput
    and the reconstruction time per RK3 step per element beside the paper's
    t_norm (CPU hardware; context only).  The *_char schemes select in
    characteristic variables, edge by edge (Sec. 2.3); the paper gives no
    timing for them."""
    w, mesh, U0 = inputs.make_workload(6)
    out = {"workload": "kelvin_helmholtz_N537", "n_cell": mesh.n_cell, "steps": steps, "schemes": {}}
    for name, order, variant, chr_ in (("TENO3", 3, 0, 0), ("TENO4", 4, 0, 0), ("TENO5", 5, 0, 0),
                                       ("TENO6", 6, 0, 0), ("CWENO5", 5, 2, 0), ("CWENO6", 6, 2, 0),
                                       ("TENO5_char", 5, 0, 1), ("TENO6_char", 6, 0, 1),
                                       ("CWENO5_char", 5, 2, 1)):
        lm = teno.Mesh(mesh.xy, mesh.tri).setup(order=order, fallback=1, variant=variant,
                                                characteristic=chr_)
        sv = teno.Solver(lm)
        U = torch.as_tensor(U0[lm.perm], device="cuda")
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
        torch.cuda.synchronize()
        sv.profile_read(reset=True)
        sv.profile_enable(True, kinds=("reconstruct",))
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sv.profile_enable(False)
        prof = sv.profile_read(reset=True)
        rec_ms = prof.ms["reconstruct"] / max(1, prof.launches["reconstruct"])
        out["schemes"][name] = {
            "value": mesh.n_cell * 3 * steps / el, "unit": "cell-updates/s",
            "ms_per_step": el * 1e3 / steps,
            "recon_s_per_step_per_element": 3 * rec_ms * 1e-3 / mesh.n_cell,
            "paper_t_norm_cpu": PAPER_KHI_T_NORM.get(name)}
        del sv, lm, U
    return out


# Tab. runtime analysis (Sec. 5.10), DMR on 369,794 triangles, 56 CPU threads.
PAPER_DMR_T_NORM = {"TENO3": 1.36e-6, "TENO4": 1.66e-6, "TENO5": 1.96e-6, "TENO6": 2.24e-6,
                    "CWENO5": 1.98e-6, "CWENO6": 2.20e-6}


def dmr_timing(torch, teno, inputs, steps=10, warmup=2):
    """The paper's DMR timing workload (Sec. 5.8, 5.10) at its size: a Mach 10
    shock on [0, 4] x [0, 1] with 860 x 215 x 2 = 369,800 cells (paper:
    369,794), reflective wall, prescribed inflow and moving-shock top,
    transmissive outflow.  The top boundary follows the exact shock position
    at the start of every step (its states are computed on the device from
    the device-resident time)."""
    w, mesh, U0 = inputs.make_workload(7)
    out = {"workload": "double_mach_860x215", "n_cell": mesh.n_cell, "steps": steps, "schemes": {}}
    for name, order, variant in (("TENO3", 3, 0), ("TENO4", 4, 0), ("TENO5", 5, 0), ("TENO6", 6, 0),
                                 ("CWENO5", 5, 2), ("CWENO6", 6, 2)):
        lm = teno.Mesh(mesh.xy, mesh.tri, period=mesh.period)
        verts, _ = lm.boundary_faces()
        kind, state = inputs.double_mach_boundary(mesh, verts, 0.0)
        lm.set_boundary(kind, state)
        lm.setup(order=order, fallback=1, variant=variant)
        sv = teno.Solver(lm)
        mid, side = inputs.face_sides(mesh, verts)
        top = torch.as_tensor((side == 3)[:, None], device="cuda")
        xmid = torch.as_tensor(mid[:, :1], device="cuda")
        post = torch.as_tensor(inputs.conservative(*inputs.DMR_POST), device="cuda")
        pre = torch.as_tensor(inputs.conservative(*inputs.DMR_PRE), device="cuda")
        base = torch.as_tensor(state, device="cuda")
        U = torch.as_tensor(U0[lm.perm], device="cuda")
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        t = torch.zeros(1, dtype=torch.float64, device="cuda")

        def step():
            xs = 1.0 / 6.0 + (1.0 + 20.0 * t) / 3.0 ** 0.5
            sv.set_boundary_states(torch.where(top, torch.where(xmid < xs, post, pre), base))
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
            t.add_(dt)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        sv.profile_read(reset=True)
        sv.profile_enable(True, kinds=("reconstruct",))
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sv.profile_enable(False)
        prof = sv.profile_read(reset=True)
        diag = sv.diagnostics(reset=True)
        rec_ms = prof.ms["reconstruct"] / max(1, prof.launches["reconstruct"])
        out["schemes"][name] = {
            "value": mesh.n_cell * 3 * steps / el, "unit": "cell-updates/s",
            "ms_per_step": el * 1e3 / steps,
            "recon_s_per_step_per_element": 3 * rec_ms * 1e-3 / mesh.n_cell,
            "paper_t_norm_cpu": PAPER_DMR_T_NORM.get(name),
            "fallback_cells": int(diag["fallbacks"]),
            "finite": bool(torch.isfinite(U).all().item())}
        del sv, lm, U
    return out


def algorithmic_bytes_stage3(order: int) -> int:
    """Tetrahedra: bytes one cell must move per RK stage, the fused minimum
    as for triangles: its least-squares operators (4 small 9 x 19 + the
    large nu x nl, FP64), stencil indices (76 + nl int32), its state, U^n and
    U^(k+1) (40 B each) and its share of the face geometry (2 faces x
    (normal, |A|, two cell ids) + its face list and |V|: 104 B): 7,444 /
    12,084 / 25,044 / 55,284 B at orders 3-6."""
    r = order - 1
    nu = (r + 1) * (r + 2) * (r + 3) // 6 - 1
    nl = 2 * (nu + 1) - 1
    ops = 8 * (4 * 9 * 19 + nu * nl)
    idx = 4 * (4 * 19 + nl)
    return ops + idx + 3 * 40 + 104


def tet_timing(torch, steps=10, warmup=2):
    """Tetrahedra (the method in three reference coordinates): TENO3-6 on the
    jittered periodic 32^3 x 6 = 196,608-cell cube with random planes, and
    the paper's 3D explosion (Sec. 5.9, edge h ~ 1/30) with TENO4 on
    [-1, 1]^3 split into 60^3 x 6 = 1,296,000 tetrahedra with transmissive
    sides; per-stage throughput and the roofline of the reconstruction."""
    from paper_2105_02127_amd import inputs3, teno3
    out = {"schemes": {}}
    for name, wl, order in (("TENO3_planes_N32", "teno4_planes_N32", 3),
                            ("TENO4_planes_N32", "teno4_planes_N32", 4),
                            ("TENO5_planes_N32", "teno4_planes_N32", 5),
                            ("TENO6_planes_N32", "teno4_planes_N32", 6),
                            ("TENO4_explosion3_N60", "explosion3_N60", 4)):
        w, mesh, U0 = inputs3.make_workload3(wl)
        t0 = time.perf_counter()
        lm = teno3.TetMesh(mesh.xyz, mesh.tet, period=mesh.period).setup(
            order=order, fallback=w["fallback"])
        t_setup = time.perf_counter() - t0
        sv = teno3.TetSolver(lm)
        U = torch.as_tensor(U0[lm.perm], device="cuda")
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
        torch.cuda.synchronize()
        sv.diagnostics(reset=True)
        sv.profile_read(reset=True)
        sv.profile_enable(kinds=("reconstruct",))
        t0 = time.perf_counter()
        for _ in range(steps):
            sv.max_dt(U, 0.4, dt)
            sv.rk_step(U, dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sv.profile_enable(kinds=())
        prof = sv.profile_read(reset=True)
        diag = sv.diagnostics(reset=True)
        rec_ms = prof.ms["reconstruct"] / max(1, prof.launches["reconstruct"])
        bytes_stage = algorithmic_bytes_stage3(order) * mesh.n_cell
        achieved = bytes_stage / (rec_ms * 1e-3) / 1e9 if rec_ms > 0 else None
        step_gbs = 3 * bytes_stage / (el / steps) / 1e9
        out["schemes"][name] = {
            "workload": wl, "n_cell": mesh.n_cell, "order": order, "steps": steps,
            "value": mesh.n_cell * 3 * steps / el, "unit": "cell-updates/s",
            "ms_per_step": el * 1e3 / steps, "setup_s": t_setup,
            "recon_avg_launch_ms": rec_ms,
            "algorithmic_bytes_per_cell": algorithmic_bytes_stage3(order),
            "recon_achieved_gbs": achieved,
            "recon_frac": achieved / HBM_PEAK_GBS if achieved else None,
            "whole_step_gbs": step_gbs, "whole_step_frac": step_gbs / HBM_PEAK_GBS,
            "fallback_cells": int(diag["fallbacks"]),
            "finite": bool(torch.isfinite(U).all().item())}
        print(f"[tet] {name}: {out['schemes'][name]['value']:.3e} cell-updates/s, "
              f"recon {rec_ms:.3f} ms, setup {t_setup:.1f} s", file=sys.stderr, flush=True)
        del sv, lm, U
    return out


def batch_timing(torch, teno, inputs, steps=100):
    """Batched workload: 64 seeded jittered periodic meshes, N ~ U{32..316},
    order ~ U{3..6}, random-line states; one step = per-mesh dt + one
    SSP-RK3 step of every mesh (one replay of the captured step graph).
    All 100 steps of the workload are timed, for the autotuned batched
    schedule and for the same meshes stepped one solver at a time."""
    from paper_2105_02127_amd.batch import Batch, autotune
    specs = inputs.batch_specs()
    solvers, U0 = [], []
    t0 = time.perf_counter()
    for n, p, seed in specs:
        m = inputs.jittered_periodic_mesh(n, seed)
        lm = teno.Mesh(m.xy, m.tri).setup(order=p, fallback=1)
        solvers.append(teno.Solver(lm))
        U0.append(torch.as_tensor(inputs.random_lines(m)[lm.perm], device="cuda"))
    t_setup = time.perf_counter() - t0
    cells = sum(s.n_cell for s in solvers)
    by_order = {}
    for s in solvers:
        by_order[s.order] = by_order.get(s.order, 0) + s.n_cell
    b = Batch(solvers)
    dt = b.max_dt(U0, 0.4)
    best, timings = autotune(b, U0, dt, steps=3)
    tuned = b.stats                 # the tuned schedule's graph is captured below
    U = [u.clone() for u in U0]
    for _ in range(2):
        b.max_dt(U, 0.4, dt)
        b.rk_step(U, dt)
    torch.cuda.synchronize()
    before = b.stats
    t0 = time.perf_counter()
    for _ in range(steps):
        b.max_dt(U, 0.4, dt)
        b.rk_step(U, dt)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    after = b.stats
    timed = {k: after[k] - before[k] for k in after}
    finite = all(bool(torch.isfinite(u).all().item()) for u in U)
    # the same meshes, one solver at a time
    U = [u.clone() for u in U0]
    dts = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in solvers]
    for _ in range(2):
        for s, u, d in zip(solvers, U, dts):
            s.max_dt(u, 0.4, d)
            s.rk_step(u, d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, u, d in zip(solvers, U, dts):
            s.max_dt(u, 0.4, d)
            s.rk_step(u, d)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    return {"workload": "64 meshes, N~U{32..316}, order~U{3..6}, random lines", "meshes": len(solvers),
            "n_cell": cells, "cells_by_order": by_order, "steps": steps,
            "value": cells * 3 * steps / t_batch, "unit": "cell-updates/s",
            "ms_per_step": t_batch * 1e3 / steps,
            "single_mesh_sequential_value": cells * 3 * steps / t_seq,
            "batched_over_sequential": t_seq / t_batch,
            "tuning": best, "setup_s": t_setup,
            "graph": {"captures_of_tuned_schedule": after["captures"] - tuned["captures"],
                      "captures_in_timed_steps": timed["captures"],
                      "replays_in_timed_steps": timed["replays"],
                      "descriptor_writes_in_timed_steps": timed["descriptor_writes"]},
            "finite": finite}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, help="2 = TENO5 512^2 lines, 3 = TENO6 1024^2")
    ap.add_argument("--n", type=int, default=None, help="override mesh size N (N x N x 2 cells)")
    ap.add_argument("--fallback", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-single", action="store_true",
                    help="skip the single-thread oracle timing")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the stream-triad bandwidth measured for context")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-khi", action="store_true", help="skip the KHI TENO3-6 timings")
    ap.add_argument("--khi-steps", type=int, default=10, help="timed steps per KHI/DMR scheme")
    ap.add_argument("--khi-warmup", type=int, default=2, help="warm-up steps per KHI/DMR scheme")
    ap.add_argument("--no-dmr", action="store_true", help="skip the DMR TENO3-6 timings")
    ap.add_argument("--no-tet", action="store_true", help="skip the tetrahedral timings")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time the steps without per-launch HIP events (no roofline figures)")
    ap.add_argument("--breakdown-steps", type=int, default=5,
                    help="extra steps after the timed ones, every kernel timed by events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (a single mesh "
              "would shard by domain decomposition with one ghost exchange per stage).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_02127_amd import inputs, teno

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w, mesh, U0 = inputs.make_workload(args.workload, n=args.n)
    order = w["order"]
    t0 = time.perf_counter()
    lm = teno.Mesh(mesh.xy, mesh.tri).setup(order=order, fallback=args.fallback)
    t_setup = time.perf_counter() - t0
    sv = teno.Solver(lm)
    info = lm.info()
    Ud = torch.as_tensor(U0[lm.perm], device="cuda")
    dt = torch.empty(1, dtype=torch.float64, device="cuda")

    # a step = one SSP-RK3 step whose last stage also forms the next step's
    # CFL dt from the states it writes (teno_rk_step_dt); the first step's
    # dt comes from teno_max_dt
    def step():
        sv.rk_step_dt(Ud, dt, 0.4)

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    sv.max_dt(Ud, 0.4, dt)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sv.diagnostics(reset=True)
    sv.profile_read(reset=True)
    # events only around the reconstruction launches (the roofline kernel):
    # events around every launch cost about 2.5% of the step
    sv.profile_enable(not args.no_kernel_events, kinds=("reconstruct",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sv.profile_enable(False)
    prof = sv.profile_read(reset=True)
    diag = sv.diagnostics(reset=True)
    # per-kernel breakdown on a few extra (untimed) steps, every launch timed
    sv.profile_enable(args.breakdown_steps > 0)
    for _ in range(args.breakdown_steps):
        step()
    torch.cuda.synchronize()
    sv.profile_enable(False)
    brk = sv.profile_read(reset=True)

    n_cell = mesh.n_cell
    stages = 3 * args.steps
    value = n_cell * stages / elapsed
    nq = info.n_quad
    k1_ms = prof.ms["reconstruct"] / max(1, prof.launches["reconstruct"])
    per_launch = {k: brk.ms[k] / brk.launches[k] for k in ("reconstruct", "flux_update", "dt")
                  if brk.launches[k]}
    bytes_stage = algorithmic_bytes_stage(order) * n_cell
    achieved = bytes_stage / (k1_ms * 1e-3) / 1e9 if k1_ms > 0 else None
    step_gbs = 3 * bytes_stage / (elapsed / args.steps) / 1e9
    traffic = traffic_from_profiles(w["name"])
    out = {
        "metric": METRIC if order == 5 else f"cell-updates/s per RK stage ({order}th-order, Euler)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_cell": n_cell, "order": order, "n_quad": nq,
                   "ic": w["ic"], "seed": w["seed"], "cfl": 0.4,
                   "positivity_fallback": bool(args.fallback),
                   "nonphysical_cells_in_timed_stages": int(diag["nonphysical"]),
                   "fallback_cells_in_timed_stages": int(diag["fallbacks"]),
                   "note": ("the random-line states are not physical everywhere at the seams of "
                            "the lines: the first-order fallback (not in the paper) replaces the "
                            "face states of the cells counted above, after their full "
                            "reconstruction") if diag["fallbacks"] else None,
                   "stage": "reconstruct + HLL flux + gather + RK update; dt once per step, "
                            "formed by the last stage's update"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": traffic,
                     "kernel": "k_reconstruct",
                     "algorithmic_bytes_per_launch": bytes_stage,
                     "algorithmic_bytes_per_cell": algorithmic_bytes_stage(order),
                     "avg_launch_ms": k1_ms,
                     "whole_step_gbs": step_gbs,
                     "whole_step_frac": step_gbs / HBM_PEAK_GBS},
        "kernels_ms_per_launch": per_launch,
        "diagnostics": diag,
        "setup_s": t_setup,
    }
    if achieved and not args.no_stream:
        triad = stream_triad_gbs(torch)
        out["roofline"]["stream_triad_gbs"] = triad
        out["roofline"]["frac_of_stream_triad"] = achieved / triad
    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing(torch, teno, inputs)
    if not args.no_batch:
        out["batched"] = batch_timing(torch, teno, inputs)
    if not args.no_khi:
        out["khi"] = khi_timing(torch, teno, inputs, args.khi_steps, args.khi_warmup)
    if not args.no_dmr:
        out["dmr"] = dmr_timing(torch, teno, inputs, args.khi_steps, args.khi_warmup)
    if not args.no_tet:
        out["tetrahedra"] = tet_timing(torch, args.khi_steps, args.khi_warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, U0, order, args.fallback, args.cpu_steps,
                                           single=not args.no_cpu_single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
