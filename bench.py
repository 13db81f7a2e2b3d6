"""Benchmark: element updates per second of the anelastic ADER-DG LTS forward
solve on one MI355X.

Workload (synthetic, seeded): the layered 20 x 20 x 10 km box, 996,558
jittered Kuhn tetrahedra (67 x 67 columns; 4 x 100 m, 3 x 200 m, 30 x 300 m
layers), order 5 (35 basis functions), 3 relaxation mechanisms (27
quantities), FP32, clustered rate-2 LTS with N_c = 3 and a searched lambda,
free surface on top and absorbing elsewhere, layered vs 800-3500 m/s with
vp/vs = 1.8, +-5% Gaussian perturbations, Qs = 50 vs[km/s], Qp = 2 Qs, one
Ricker moment-tensor source (fc = 2 Hz), 64 surface receivers.

One step = one LTS cycle (the coarsest cluster's time step; every element
advances by its own steps).  The timed region is one edg_advance_to call over
`steps` cycles, bracketed by device synchronisation; its element updates per
second is the value.  The roofline entry uses the per-launch durations of
the element-update kernel from HIP events recorded on the library's stream
during the same timed region.  The CPU baseline times the FP64 oracle on a
bounded sample (a 6 x 6-column box of the same construction, three cycles).

The "fused" entry runs 16 independent runs of the same workload in one
context (one launch per LTS level for all runs), each with its own Ricker
source (fc uniform in 1-3 Hz, random moment tensor, uniform location in the
top 5 km), and reports run-element updates per second against the plain
single-run value.

Extra workload lines (--configs): "c3_basin" the 7.88M-tet graded basin
(O=5, N_c=5, 400 subfaults, 256 receivers; a few timed cycles, the wall time
of 10 simulated seconds extrapolated), "c4_fused_o4" 16 runs at O=4 against
the plain O=4 run, "c5_gradient_o4" the 201,720-tet gradient workload (O=4,
N_c=2, elastic and anelastic, 4 s, a checkpoint every 50 cycles).

The "adjoint" entry times the gradient of a receiver misfit with respect to
rho, vp, vs over a short window: the checkpointed forward plus the reverse
sweep, against the plain forward of the same cycles.  Its main figure keeps
the window as one checkpoint segment (the forward records every level's
state, the sweep replays nothing); "checkpoint_per_cycle" stores one
checkpoint per cycle instead and replays all but the last.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 peak (vector and matrix cores alike): the roofline's
# compute ceiling
FP32_PEAK_TFLOPS = 157.3
# issue-rate diagnostic only: FP32 FMA on the vector ALUs without packed-FP32
# instructions (which this build does not emit), 256 CUs x 4 SIMDs x 16 lanes
# x 2 flop x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# the paper's flop count per element update at O=5, m=3 when every zero of the
# sparse matrices is skipped (Sec. VII-B (LOH.3, Performance), Table speedups_flops_loh3 discussion)
PAPER_FLOPS_ALL_SPARSITY = 212688
# HBM traffic of the element-update kernel: rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by what the counter reads for a device copy of known
# size, summed over the four launches of a steady-state LTS cycle and divided by
# the cycle's element updates.  Valid only for the kernel sources it was taken
# on (their SHA-256 below); after any change the roofline reports null.
TRAFFIC_BYTES_PER_UPDATE = 15205.8
TRAFFIC_SOURCES_SHA256 = "7040d603ed30fff0dff05585c1f7d86a489cf101fb7ba88823768f9ad6130018"
KERNEL_SOURCES = ["kernels.hip", "kernels.hpp", "device_common.hpp", "gen_refmats.cpp", "basis.cpp", "basis.hpp"]
METRIC = "elem-updates/s on 1 GPU at order 5 (plain vs 16-fused vs fwd+adjoint); % roofline"


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2202_10313_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def face_neighbours(tet_verts):
    """[K,4] neighbour across the face opposite each local vertex (-1 = none)."""
    K = tet_verts.shape[0]
    faces = []
    for i in range(4):
        others = [m for m in range(4) if m != i]
        f = np.sort(tet_verts[:, others], axis=1)
        faces.append(np.concatenate([f, np.arange(K)[:, None], np.full((K, 1), i)], axis=1))
    F = np.concatenate(faces)
    order = np.lexsort((F[:, 2], F[:, 1], F[:, 0]))
    F = F[order]
    same = np.all(F[1:, :3] == F[:-1, :3], axis=1)
    nbr = -np.ones((K, 4), dtype=np.int64)
    idx = np.nonzero(same)[0]
    a, b = F[idx], F[idx + 1]
    nbr[a[:, 3], a[:, 4]] = b[:, 3]
    nbr[b[:, 3], b[:, 4]] = a[:, 3]
    return nbr


def algorithmic_bytes_per_update(cl, nbr, order, m, n_clusters, word=4):
    """Bytes an element update must move, averaged over the updates of one
    cycle: Q read and written once (2 Nq B), the element's own B1 written and
    every buffer read once (ideal reuse), B2 written where a finer neighbour
    needs it, B3 read-modify-written where a coarser one does, plus 48 words
    of per-element parameters (inverse Jacobian, |det J|, rho/lambda/mu, the
    anelastic weights, four faces of normal, area ratio and neighbour id)."""
    B = order * (order + 1) * (order + 2) // 6
    nq = 9 + 6 * m
    ncl = np.where(nbr >= 0, cl[np.maximum(nbr, 0)], cl[:, None])
    b2 = np.any(ncl < cl[:, None], axis=1).astype(float)
    b3 = np.any(ncl > cl[:, None], axis=1).astype(float)
    per = word * (2 * nq * B + 9 * B * (1 + b2 + 1.5 * b3) + 9 * B * (1 + b2 + b3)) + 4 * 48
    weight = 2.0 ** (n_clusters - cl)           # updates per cycle of an element of cluster cl (1-based)
    return float(np.sum(per * weight) / np.sum(weight))


def fractions(rate, bytes_per_update, flops_per_update):
    """HBM, FP32 and combined roofline fractions of an element-update rate."""
    hbm = rate * bytes_per_update / (HBM_PEAK_GBS * 1e9)
    fp32 = rate * flops_per_update / (FP32_PEAK_TFLOPS * 1e12) if flops_per_update else 0.0
    return {"hbm": hbm, "fp32": fp32 if flops_per_update else None, "combined": max(hbm, fp32)}


def _oracle_sample(cycles):
    """One oracle run of the CPU-baseline sample (runs in a worker process):
    returns (element updates, wall seconds, CPU seconds)."""
    from oracle.solver import Oracle
    dz = [100.0] * 4 + [200.0] * 3 + [300.0] * 30
    h = 20000.0 / 67
    n = 6
    mesh = synth.layered_box(n, n, dz, n * h, n * h, jitter=0.15, seed=20)
    mat = synth.layered_materials(mesh, 21)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    orc = Oracle(mesh, mat, 5, attn=attn, n_clusters=3, lam=None)
    orc.set_initial(synth.random_state(1, orc.K, 27, orc.B))
    c0, t0 = time.process_time(), time.perf_counter()
    orc.run(cycles * orc.sync_dt)
    t1, c1 = time.perf_counter(), time.process_time()
    return orc.K, orc.updates, t1 - t0, c1 - c0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cycles=3, workers=None):
    """The oracle (FP64 NumPy, as it stands) on a 6 x 6-column box of the
    workload's construction (same spacing, layering and material recipe),
    `cycles` LTS cycles, run as one independent instance per host core (up
    to 16, the host share of one GPU; NumPy's element-wise work is
    single-threaded, so the host's throughput is the sum over instances).
    About 15 s of wall time."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = workers or max(1, min(16, os.cpu_count() or 1))
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:
        os.environ[k] = "1"          # one thread per instance (the children inherit it)
    try:
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(n, mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_sample, [cycles] * n))
        wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    K = res[0][0]
    upd = sum(r[1] for r in res)
    run_wall = max(r[2] for r in res)
    cpu_s = sum(r[3] for r in res)
    return {"value": upd / run_wall, "unit": "elem-updates/s",
            "cores": max(1, round(cpu_s / run_wall)), "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"FP64 oracle, {n} independent instances (one per core) of a {K}-tet 6x6-column box of the "
                      f"same construction, O=5, m=3, N_c=3, {cycles} LTS cycles each ({upd} element updates, "
                      f"slowest instance {run_wall:.1f} s, pool wall {wall:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fused-runs", type=int, default=16, help="runs of the fused batch line (<= 1: skip it)")
    ap.add_argument("--fused-steps", type=int, default=4)
    ap.add_argument("--adjoint-steps", type=int, default=2,
                    help="cycles of the forward + adjoint (gradient) line (0: skip it)")
    ap.add_argument("--configs", default="c3,c4,c5",
                    help="extra workload lines: c3 (7.88M-tet basin, N_c=5), c4 (16 fused runs at O=4), "
                         "c5 (200k-tet gradient workload); '' for none")
    ap.add_argument("--c3-cycles", type=int, default=3, help="timed LTS cycles of the basin line")
    ap.add_argument("--c4-steps", type=int, default=4, help="timed LTS cycles of the O=4 fused line")
    ap.add_argument("--c5-seconds", type=float, default=4.0, help="simulated time of the gradient line")
    ap.add_argument("--no-graph", dest="graph", action="store_false", help="launch every level eagerly")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false", help="keep the default launch plan")
    ap.add_argument("--trace-mfma", action="store_true",
                    help="form the traces of faces 0 and 1 on the matrix cores (launch-plan option trace_mfma)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 2 GiB (profiler calibration of FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2202_10313_amd import FLAG_GRAPH, Context, STF_RICKER

    if args.copy_calibration:
        n = 1 << 29                                   # 2 GiB of float32
        a = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 3}))
        return

    print("[bench] generating the workload", file=sys.stderr, flush=True)
    mesh = synth.loh_like_box("full", seed=20)
    K = mesh["tet_verts"].shape[0]
    mat = synth.layered_materials(mesh, 21)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    src = synth.ricker_sources(22, 1, ((5000.0, 15000.0), (5000.0, 15000.0)), (1000.0, 5000.0), fc_range=(2.0, 2.0))
    rec = synth.surface_receivers(23, 64, ((1000.0, 19000.0), (1000.0, 19000.0)))
    torch.cuda.init()
    stream = torch.cuda.current_stream()

    def measure(order, runs, steps, warmup):
        """Advance `runs` runs of the workload (run r with its own Ricker
        source): the autotuner's cycles (one per candidate launch plan), then
        warmup + steps LTS cycles, timing the last `steps` (full cycles
        replayed as captured HIP graphs)."""
        ctx = Context(order, mechanisms=3, n_clusters=3, fp64=False, cfl=0.5, lam=None, stream=stream.cuda_stream,
                      n_runs=runs, flags=FLAG_GRAPH if args.graph else 0)
        ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
        ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
        ctx.upload_clusters(None)
        info = ctx.get_clusters()
        sync = info["sync_dt"]
        for r in range(runs):
            s = src if runs == 1 else synth.ricker_sources(40 + r, 1, ((0.0, 20000.0), (0.0, 20000.0)), (0.0, 5000.0),
                                                           fc_range=(1.0, 3.0))
            ctx.set_sources(s["xyz"], s["moment"], STF_RICKER, s["stf_params"], run=r)
        total_t = (warmup + steps + 16) * sync
        ctx.set_receivers(rec, 0.005, int(total_t / 0.005) + 2)
        plan, tuned_ms = ctx.autotune(cycles=1) if args.autotune else (ctx.get_plan(), None)
        if args.trace_mfma:
            plan = dict(plan, trace_mfma=1)
            ctx.set_plan(**plan)
        print(f"[bench] launch plan {plan} ({tuned_ms} ms per cycle while tuning)", file=sys.stderr, flush=True)
        t_start = ctx.time()
        ctx.advance_to(t_start + warmup * sync)
        u0 = ctx.element_updates()
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.advance_to(t_start + (warmup + steps) * sync)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = dict(updates=ctx.element_updates() - u0, wall=t1 - t0, ks=ctx.kernel_stats(), info=info, plan=plan)
        for r in range(runs):
            if not np.all(np.isfinite(ctx.read_receivers(run=r))):
                raise RuntimeError(f"non-finite seismograms in run {r}")
        ctx.close()
        return res

    def measure_adjoint(order, steps, every):
        """Gradient of J = 1/2 sum_r,s |seis|^2 dt_sample with respect to rho,
        vp, vs over `steps` LTS cycles: the checkpointed forward (a checkpoint
        every `every` cycles; the final segment records its level states) plus
        the reverse sweep (replay of every other segment from its checkpoint,
        adjoint kernels backwards).  One untimed cycle first."""
        ctx = Context(order, mechanisms=3, n_clusters=3, fp64=False, cfl=0.5, lam=None, stream=stream.cuda_stream,
                      flags=FLAG_GRAPH if args.graph else 0)
        ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
        ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
        ctx.upload_clusters(None)
        sync = ctx.get_clusters()["sync_dt"]
        # t0 = 0: the source radiates from the first step, so the gradient of
        # the short window is not zero
        ctx.set_sources(src["xyz"], src["moment"], STF_RICKER, np.array([[2.0, 0.0]]))
        dts = 0.005
        ctx.set_receivers(rec, dts, int((steps + 2) * sync / dts) + 2)
        ctx.set_checkpointing(every)
        out = {}
        for phase, n in (("warm", 1), ("timed", steps)):
            ctx.rewind()
            ctx.set_initial(np.zeros((K, ctx.nq, ctx.B)))
            u0 = ctx.element_updates()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance_to(n * sync)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = ctx.adjoint(dj_dseis=ctx.read_receivers() * dts, want_q0=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            out = dict(updates=ctx.element_updates() - u0, fwd=t1 - t0, adj=t2 - t1)
        if not all(np.all(np.isfinite(g[k])) for k in ("g_rho", "g_vp", "g_vs")):
            raise RuntimeError("non-finite gradient")
        ctx.close()
        return out

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    def line_c3():
        """The graded basin (one GPU's share of a high-frequency run): 7.88M
        tets, O=5, m=3, N_c=5, FP32, 400 Hann subfaults, 256 receivers; one
        untimed cycle, then --c3-cycles timed; the wall time of the 10 s
        simulation is extrapolated from the timed cycles."""
        say("c3: generating the 7.88M-tet basin")
        bm = synth.basin_box("full", seed=30)
        bmat = synth.basin_materials(bm, 31)
        battn = synth.attenuation_inputs(bmat, 3, 0.1, 10.0)
        fault = synth.kinematic_fault(32, (2000.0, -1500.0, -7000.0))
        brec = synth.surface_receivers(33, 256, ((-20000.0, 20000.0), (-20000.0, 20000.0)))
        ctx = Context(5, mechanisms=3, n_clusters=5, fp64=False, cfl=0.5, lam=None, stream=stream.cuda_stream,
                      flags=FLAG_GRAPH if args.graph else 0)
        ctx.upload_mesh(bm["tet_verts"], bm["tet_xyz"], bm["face_bc"])
        ctx.upload_materials(bmat["rho"], bmat["vp"], bmat["vs"], battn["omega"], battn["yp"], battn["ys"])
        say("c3: clustering and uploading")
        ctx.upload_clusters(None)
        inf = ctx.get_clusters()
        sy = inf["sync_dt"]
        ctx.set_sources(fault["xyz"], fault["moment"], fault["stf_kind"], fault["stf_params"])
        ctx.set_receivers(brec, 0.01, 1001)
        ctx.set_plan(xcd_remap=1)
        ctx.advance_to(sy)
        u0 = ctx.element_updates()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.advance_to((1 + args.c3_cycles) * sy)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        upd = ctx.element_updates() - u0
        if not np.all(np.isfinite(ctx.read_receivers())):
            raise RuntimeError("non-finite seismograms in the basin line")
        ctx.close()
        bcl = inf["clusters"].astype(np.int64)
        bpu = algorithmic_bytes_per_update(bcl, face_neighbours(bm["tet_verts"]), 5, 3, 5)
        rate = upd / wall
        cycles_10s = 10.0 / sy
        say(f"c3: {rate:.4g} element updates/s, {wall / args.c3_cycles * 1e3:.1f} ms per cycle")
        return {"workload": f"graded basin, {bm['tet_verts'].shape[0]} tets, O=5, m=3, N_c=5, FP32, 400 Hann "
                            f"subfaults, 256 receivers; step = one LTS cycle ({2 ** 4} finest levels)",
                "value": rate, "unit": "elem-updates/s", "steps": args.c3_cycles,
                "ms_per_step": wall / args.c3_cycles * 1e3, "lambda": inf["lam"],
                "cluster_sizes": np.bincount(bcl, minlength=6)[1:].tolist(),
                "theoretical_lts_speedup": inf["speedup"],
                "gts_equivalent_rate": bm["tet_verts"].shape[0] * (args.c3_cycles * sy / inf["dt_min"]) / wall,
                "simulated_10s": {"cycles": cycles_10s, "wall_s_extrapolated": cycles_10s * wall / args.c3_cycles},
                "algorithmic_bytes_per_update": bpu,
                "roofline": fractions(rate, bpu, PAPER_FLOPS_ALL_SPARSITY)}

    def line_c4():
        """16 independent runs at O=4 in one context against the plain O=4 run
        (the rate of 16 sequential plain runs is 16 runs x the plain rate)."""
        say(f"c4: plain O=4, 1 run, warmup 1, {args.c4_steps} cycles")
        pl = measure(4, 1, args.c4_steps, 1)
        say(f"c4: fused O=4, 16 runs, warmup 1, {args.c4_steps} cycles")
        fu = measure(4, 16, args.c4_steps, 1)
        pv, fv = pl["updates"] / pl["wall"], fu["updates"] / fu["wall"]
        bpu4 = algorithmic_bytes_per_update(cl, nbr, 4, 3, 3)
        say(f"c4: {fv:.4g} run-element updates/s against {pv:.4g} plain ({fv / pv:.2f}x)")
        return {"workload": f"16 runs of the layered box, {K} tets, O=4, m=3, N_c=3, FP32, one Ricker per run",
                "runs": 16, "value": fv, "unit": "run-elem-updates/s", "plain_value": pv,
                "ratio_vs_16_sequential_plain_runs": fv / pv, "steps": args.c4_steps,
                "ms_per_step": fu["wall"] * 1e3 / args.c4_steps, "plain_ms_per_step": pl["wall"] * 1e3 / args.c4_steps,
                "launch_plan": fu["plan"], "plain_launch_plan": pl["plan"],
                "algorithmic_bytes_per_update": bpu4, "roofline_plain": fractions(pv, bpu4, None),
                "roofline_fused": fractions(fv, bpu4, None)}

    def line_c5():
        """The gradient workload: 201,720 tets, O=4, N_c=2, FP32, elastic and
        anelastic; misfit J = 1/2 sum (s - d)^2 dt against data d from a
        +-3% perturbed model over --c5-seconds; forward with a checkpoint
        every 50 LTS cycles (all but the final segment replayed by the
        sweep) plus the reverse sweep, against the plain forward."""
        dm = synth.differentiation_box("full", seed=50)
        dmat = synth.layered_materials(dm, 51)
        dattn = synth.attenuation_inputs(dmat, 3, 0.05, 5.0)
        dsrc = synth.ricker_sources(52, 1, ((3000.0, 7000.0), (3000.0, 7000.0)), (1000.0, 3000.0), fc_range=(2.0, 2.0))
        drec = synth.surface_receivers(53, 32, ((500.0, 9500.0), (500.0, 9500.0)))
        rng = np.random.default_rng(54)
        Kd = dm["tet_verts"].shape[0]
        pert = {k: dmat[k] * (1 + rng.uniform(-0.03, 0.03, Kd)) for k in ("rho", "vp", "vs")}
        out = {"workload": f"layered 10x10x5 km box, {Kd} tets, O=4, N_c=2, FP32, 1 Ricker, 32 receivers, "
                           f"{args.c5_seconds} s; misfit against a +-3% perturbed model",
               "checkpoint_every_cycles": 50}
        for mech in (0, 3):
            ctx = Context(4, mechanisms=mech, n_clusters=2, fp64=False, cfl=0.5, lam=None, stream=stream.cuda_stream,
                          flags=FLAG_GRAPH if args.graph else 0)
            ctx.upload_mesh(dm["tet_verts"], dm["tet_xyz"], dm["face_bc"])
            extra = (dattn["omega"], dattn["yp"], dattn["ys"]) if mech else ()
            ctx.upload_materials(dmat["rho"], dmat["vp"], dmat["vs"], *extra)
            ctx.upload_clusters(None)
            inf = ctx.get_clusters()
            sy = inf["sync_dt"]
            ncyc = max(1, int(round(args.c5_seconds / sy)))
            dts = 0.005
            ctx.set_sources(dsrc["xyz"], dsrc["moment"], STF_RICKER, dsrc["stf_params"])
            ctx.set_receivers(drec, dts, int(ncyc * sy / dts) + 2)
            say(f"c5 m={mech}: data from the perturbed model, {ncyc} cycles")
            ctx.upload_materials(pert["rho"], pert["vp"], pert["vs"], *extra)
            ctx.advance_to(ncyc * sy)
            d = ctx.read_receivers()
            ctx.upload_materials(dmat["rho"], dmat["vp"], dmat["vs"], *extra)
            ctx.rewind()
            u0 = ctx.element_updates()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance_to(ncyc * sy)
            torch.cuda.synchronize()
            plain = time.perf_counter() - t0
            upd = ctx.element_updates() - u0
            ctx.rewind()
            ctx.set_checkpointing(50)
            say(f"c5 m={mech}: checkpointed forward + reverse sweep")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.advance_to(ncyc * sy)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s_ = ctx.read_receivers()
            g = ctx.adjoint(dj_dseis=(s_ - d) * dts, want_q0=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if not all(np.all(np.isfinite(g[k])) and np.any(g[k] != 0) for k in ("g_rho", "g_vp", "g_vs")):
                raise RuntimeError("non-finite or zero gradient in the gradient line")
            ctx.close()
            out["anelastic" if mech else "elastic"] = {
                "cycles": ncyc, "lambda": inf["lam"], "cluster_sizes": np.bincount(inf["clusters"], minlength=3)[1:].tolist(),
                "plain_forward_s": plain, "plain_rate": upd / plain,
                "forward_checkpointed_s": t1 - t0, "reverse_sweep_s": t2 - t1,
                "cost_vs_plain_forward": (t2 - t0) / plain, "reverse_vs_plain_forward": (t2 - t1) / plain,
                "misfit": 0.5 * float(np.sum((s_ - d) ** 2) * dts)}
            say(f"c5 m={mech}: forward + gradient {(t2 - t0) / plain:.2f}x the plain forward ({plain:.2f} s)")
        return out

    print(f"[bench] plain: 1 run, O={args.order}, warmup {args.warmup}, {args.steps} cycles", file=sys.stderr, flush=True)
    m = measure(args.order, 1, args.steps, args.warmup)
    info, ks, wall, updates = m["info"], m["ks"], m["wall"], m["updates"]
    sync = info["sync_dt"]
    value = updates / wall
    print(f"[bench] timed {args.steps} cycles: {wall * 1e3:.1f} ms, {updates} element updates", file=sys.stderr, flush=True)

    cl = info["clusters"].astype(np.int64)
    nbr = face_neighbours(mesh["tet_verts"])
    bpu = algorithmic_bytes_per_update(cl, nbr, args.order, 3, 3)
    kern_s = ks["total_ms"] / 1e3
    per_launch_ms = ks["total_ms"] / max(ks["launches"], 1)
    upd_per_launch = ks["element_updates"] / max(ks["launches"], 1)
    achieved_gbs = ks["element_updates"] * bpu / kern_s / 1e9
    # the paper's flop count is for O=5, m=3 only; other orders report HBM alone
    flops = PAPER_FLOPS_ALL_SPARSITY if args.order == 5 else None
    achieved_tf = ks["element_updates"] * flops / kern_s / 1e12 if flops else 0.0
    frac_hbm = achieved_gbs / HBM_PEAK_GBS
    frac_fp32 = achieved_tf / FP32_PEAK_TFLOPS
    # combined: rate x max(bytes / HBM peak, flops / FP32 peak)
    frac = max(frac_hbm, frac_fp32)
    counts = np.bincount(cl, minlength=4)[1:]
    traffic = None
    if args.order == 5 and kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256:
        traffic = TRAFFIC_BYTES_PER_UPDATE * upd_per_launch
    hbm_bound = frac_hbm >= frac_fp32
    roofline = {
        "bound": "hbm" if hbm_bound else "alu",
        "achieved": achieved_gbs if hbm_bound else achieved_tf,
        "peak": HBM_PEAK_GBS if hbm_bound else FP32_PEAK_TFLOPS,
        "unit": "GB/s" if hbm_bound else "TFLOP/s",
        "frac": frac,
        "traffic": traffic,
        "traffic_unit": "bytes/launch",
        "kernel": f"k_level2<float,{args.order},3,FUSED>" if args.order >= 4 else f"k_level<float,{args.order},3>",
        "launches": ks["launches"],
        "launch_plan": m["plan"],
        "graph": bool(args.graph),
        "avg_launch_ms": per_launch_ms,
        "element_updates_per_launch": upd_per_launch,
        "algorithmic_bytes_per_update": bpu,
        "combined": {"frac": frac, "definition": "rate x max(bytes / 8 TB/s, flops / 157.3 TFLOP/s)"},
        "hbm": {"achieved_GBs": achieved_gbs, "peak_GBs": HBM_PEAK_GBS, "frac": frac_hbm},
        "fp32": {"achieved_TFLOPs": achieved_tf, "peak_TFLOPs": FP32_PEAK_TFLOPS, "frac": frac_fp32,
                 "flops_per_update": flops} if flops else None,
        "valu_issue_diagnostic": {"peak_TFLOPs": VALU_FP32_PEAK_TFLOPS, "frac": achieved_tf / VALU_FP32_PEAK_TFLOPS,
                                  "note": "non-packed FP32 FMA issue rate of the vector ALUs"} if flops else None,
    }
    fused = None
    if args.fused_runs > 1:
        print(f"[bench] fused: {args.fused_runs} runs, O={args.order}, warmup 1, {args.fused_steps} cycles",
              file=sys.stderr, flush=True)
        f = measure(args.order, args.fused_runs, args.fused_steps, 1)
        fv = f["updates"] / f["wall"]
        fused = {"runs": args.fused_runs, "value": fv, "unit": "run-elem-updates/s", "ratio_vs_plain": fv / value,
                 "steps": args.fused_steps, "ms_per_step": f["wall"] * 1e3 / args.fused_steps,
                 "avg_launch_ms": f["ks"]["total_ms"] / max(f["ks"]["launches"], 1),
                 "launch_plan": f["plan"],
                 "sources": "one Ricker per run: fc U[1,3] Hz, random moment tensor, uniform in the top 5 km"}
        print(f"[bench] fused: {fv:.4g} run-element updates/s ({fv / value:.2f}x plain)", file=sys.stderr, flush=True)
    adjoint = None
    if args.adjoint_steps > 0:
        print(f"[bench] forward + adjoint: O={args.order}, {args.adjoint_steps} cycles", file=sys.stderr, flush=True)
        # one segment over the window (its level states recorded by the
        # forward, no replay), then a checkpoint per cycle (less memory; every
        # segment but the last replayed)
        a = measure_adjoint(args.order, args.adjoint_steps, args.adjoint_steps)
        a1 = measure_adjoint(args.order, args.adjoint_steps, 1) if args.adjoint_steps > 1 else a
        wall_plain = wall / args.steps * args.adjoint_steps          # plain forward of the same cycles
        av = a["updates"] / (a["fwd"] + a["adj"])
        adjoint = {"value": av, "unit": "elem-updates/s (forward updates per second of forward + gradient)",
                   "steps": args.adjoint_steps, "ms_per_step": (a["fwd"] + a["adj"]) * 1e3 / args.adjoint_steps,
                   "forward_checkpointed_ms": a["fwd"] * 1e3, "reverse_sweep_ms": a["adj"] * 1e3,
                   "cost_vs_plain_forward": (a["fwd"] + a["adj"]) / wall_plain,
                   "reverse_vs_plain_forward": a["adj"] / wall_plain,
                   "checkpoint_every_cycles": args.adjoint_steps,
                   "regime": "one checkpoint segment over the window: the forward records every level's state and "
                             "the sweep replays nothing (the no-replay best case; checkpoint_per_cycle replays "
                             "every segment but the last, and c5_gradient_o4 a checkpoint every 50 cycles)",
                   "checkpoint_per_cycle": {"forward_checkpointed_ms": a1["fwd"] * 1e3,
                                            "reverse_sweep_ms": a1["adj"] * 1e3,
                                            "cost_vs_plain_forward": (a1["fwd"] + a1["adj"]) / wall_plain},
                   "misfit": "1/2 sum |seismogram|^2 dt_sample over the 64 receivers; gradient w.r.t. rho, vp, vs"}
        print(f"[bench] forward + adjoint: {av:.4g} element updates/s, {adjoint['cost_vs_plain_forward']:.2f}x the "
              f"plain forward", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "elem-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"anelastic LTS forward: layered 20x20x10 km box, {K} tets, O={args.order}, m=3, "
                        f"N_c=3, FP32, 1 Ricker source, 64 receivers; step = one LTS cycle",
            "tets": K, "order": args.order, "mechanisms": 3, "n_clusters": 3,
            "lambda": info["lam"], "cluster_sizes": counts.tolist(),
            "theoretical_lts_speedup": info["speedup"],
            "gts_equivalent_rate": K * (args.steps * sync / info["dt_min"]) / wall,
        },
        "roofline": roofline,
    }
    if fused is not None:
        out["fused"] = fused
    if adjoint is not None:
        out["adjoint"] = adjoint
    extra = [c.strip() for c in args.configs.split(",") if c.strip()]
    if "c4" in extra:
        out["c4_fused_o4"] = line_c4()
    if "c5" in extra:
        out["c5_gradient_o4"] = line_c5()
    if "c3" in extra:
        out["c3_basin"] = line_c3()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
