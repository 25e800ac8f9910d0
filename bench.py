"""Surfactant-step throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c1i|c0|c2|c3|c4]

A step is one pass of the whole path (redistancing of the moving interface,
the fused transport kernel, the FP64 reductions) over the workload's grid.
The default workload is the 1024^2 FP32 soluble expanding circle.  Inputs
(the VoF field at every step, the face velocities, the initial state) are
generated before the timed region and resident in HBM.

Timed regions:
  1. the K steps replayed from one HIP graph (captured after W eager steps):
     `value` (Gcell-updates/s) and `ms_per_step`;
  2. the same K steps launched eagerly with the library's per-launch HIP
     events: average duration of the fused transport kernel -> `roofline`.
The FP64 CPU oracle is timed on a bounded sample of the same workload on the
host (`cpu_baseline`).

Other workloads (one JSON line each, not the default):
  c2  the 256^3 translating sphere (inputs generated on the GPU, all steps
      resident before the timed region);
  c2f the sphere of c2 with the 3D interfacial forces taken every step;
  c2a the sphere of c2 on the ACDI interface (phi advanced by ACDI, each
      next ACDI step prepared during the transport, re-initialized from the
      VoF every 50 steps; the ACDI bound sets dt = 3.5e-4);
  c3  the 64-instance ensemble in the batched form (one persistent launch
      per step, HIP-graph replay), against the same instances stepped one by
      one with the plain path;
  c4  the 128^3 adjoint sphere: forward steps and checkpointed adjoint steps;
  c1a the 1024^2 soluble expanding circle on the ACDI interface (phi advanced
      by ACDI, re-initialized from the VoF every 50 steps), with the ACDI
      steps timed in a burst (`acdi`);
  c2x the translating sphere of c2 on axisymmetric rings, 512 x 1024 (run it
      with --steps 100: its inputs are generated on the host);
  c1m the 1024^2 soluble expanding circle with substep 2 implicit (48 times
      the explicit step, at most 100 steps): steps launched eagerly (the host
      paces the CG launches; --implicit-graph adds a graph replay),
      the CG iteration kernel timed in a burst (`roofline`), the iterations
      of every linear solve, and the implicit oracle on a 256^2 sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector issue peak in VALU lane operations per second: 157.3 TFLOP/s
# (256 CUs at 2.4 GHz) counts an FMA as two flops; one lane of one VALU
# instruction is one lane operation
VALU_PEAK_LANE_OPS = 157.3e12 / 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c1",
                    choices=["c0", "c1", "c1i", "c1a", "c1f", "c1m", "c1v", "c2", "c2a", "c2f", "c2x",
                             "c3", "c4"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--implicit-graph", action="store_true",
                    help="c1m: also replay the steps from a HIP graph (every capped CG launch "
                         "is captured; eagerly the host stops enqueuing once a solve converged)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="2D moving interface: run each step's geometry on the step's own "
                         "stream instead of preparing it during the previous transport")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy kernel of MIB MiB (counter calibration)")
    return ap.parse_args()


def workload(name, K, W):
    from paper_2605_27534_amd import configs as C
    if name == "c0":
        return C.c0_static_circle()
    if name == "c1":
        return C.c1_expanding_circle(soluble=True)
    if name == "c1i":
        return C.c1_expanding_circle(soluble=False)
    if name == "c1a":
        return C.c1_acdi()
    if name == "c1f":
        return C.c1_forces()
    if name == "c1v":
        return C.c1_variants()
    if name == "c2x":
        return C.c2_axisymmetric()
    if name == "c2a":
        return C.c2_acdi()
    if name == "c2f":
        return C.c2_forces()
    return C.c2_translating_sphere()


def transport_kernel(cfg):
    """Name of the transport kernel the library runs for the workload."""
    p = cfg["prob"]
    if p.get("flux_form", 0) != 0:
        return "k_step" if p["dim"] == 3 else "k_step2d"
    return "k_col3d" if p["dim"] == 3 else "k_col2d"


def algorithmic_bytes(cfg, es):
    """(transport-kernel bytes per cell, whole-step bytes per cell): every
    compulsory field counted once, read or written.  The transport reads chi,
    the state and the face velocities and writes the state and sigma; a
    moving interface adds the VoF read and the level-set write, done by the
    geometry kernels before it."""
    p = cfg["prob"]
    dim = p["dim"]
    bulk = p.get("bulk_enabled", 1)
    has_u = cfg.get("u") is not None or cfg.get("u_seq") is not None
    fields = 2 if bulk else 1
    words = 1 + fields + (dim if has_u else 0) + fields + 1  # chi, state, u | state, sigma
    step_words = words + (2 if cfg.get("vof_seq") else 0)     # + vof read, chi write
    return words * es, step_words * es


# committed counter summaries (rocprofv3 FETCH_SIZE / WRITE_SIZE): the
# workload, the file and the sources of the kernel they were taken on
TRAFFIC = {
    "expanding circle 1024^2 fp32 soluble": (
        "k_col2d_expanding_circle_1024_counters.md",
        ("surf_common.hpp", "surf_kernels.hpp", "surf_col2d.hpp")),
    "translating sphere 256^3 fp32": (
        "k_col3d_translating_sphere_256_counters.md",
        ("surf_common.hpp", "surf_kernels.hpp", "surf_col2d.hpp", "surf_col3d.hpp")),
    "expanding circle 1024^2 fp32 soluble implicit": (
        "k_cg_iter_expanding_circle_implicit_1024_traffic.md",
        ("surf_common.hpp", "surf_kernels.hpp", "surf_col2d.hpp", "surf_implicit.hpp")),
}


def kernel_source_digest(sources):
    import hashlib
    hs = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2605_27534_amd", "csrc", f), "rb") as fh:
            hs.update(fh.read())
    return hs.hexdigest()[:16]


# the same for the Marangoni face force (surf_force)
FORCE_COUNTERS = {
    "expanding circle 1024^2 fp32 soluble": (
        "k_force2_expanding_circle_1024_counters.md", ("surf_common.hpp", "surf_kernels.hpp")),
    "translating sphere 256^3 fp32": (
        "k_force3_translating_sphere_256_counters.md", ("surf_common.hpp", "surf_kernels.hpp")),
}

# the same for the interfacial-force kernel of the c1f workload
IFACE_TRAFFIC = {
    "expanding circle 1024^2 fp32 soluble forces": (
        "k_iface_force_expanding_circle_forces_1024_traffic.md",
        ("surf_common.hpp", "surf_kernels.hpp", "surf_capillary.hpp")),
}


def kernel_counters(workload_name, table=None):
    """The machine-readable fields of the committed rocprofv3 counter summary
    of the workload's dominant kernel (or of the kernel `table` covers), or
    {} when there is none for this workload or the kernel source changed
    since the counters were taken."""
    table = TRAFFIC if table is None else table
    if workload_name not in table:
        return {}
    fname, sources = table[workload_name]
    try:
        txt = open(os.path.join(ROOT, "profiles", fname)).read()
    except OSError:
        return {}
    kv = {}
    for line in txt.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    if (kv.get("workload") != workload_name
            or kv.get("kernel_source_digest") != kernel_source_digest(sources)):
        return {}
    return kv


def roofline_of(kernel, alg_bytes, launch_ms, ctr):
    """The roofline of one launch: the algorithmic bytes against 8 TB/s, and,
    with a counter summary, the counted VALU lane operations against the
    FP32 vector issue peak; the larger of the two floors (the time each
    would take at its peak) names the bound.  Without counters the bound is
    the HBM one."""
    t = launch_ms * 1e-3
    hbm_ach = alg_bytes / t / 1e9
    hbm = {"achieved": round(hbm_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(hbm_ach / HBM_PEAK_GBS, 4)}
    traffic = float(ctr["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in ctr else None
    out = {"bound": "hbm", "kernel": kernel, **hbm, "traffic": traffic}
    if "valu_insts_per_launch" in ctr:
        lane_ops = float(ctr["valu_insts_per_launch"]) * 64
        v_ach = lane_ops / t / 1e12
        valu = {"achieved": round(v_ach, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
                "unit": "Tlane-op/s", "frac": round(v_ach * 1e12 / VALU_PEAK_LANE_OPS, 4),
                "lane_ops_per_launch": lane_ops}
        if lane_ops / VALU_PEAK_LANE_OPS > alg_bytes / (HBM_PEAK_GBS * 1e9):
            out.update({"bound": "alu", "achieved": valu["achieved"], "peak": valu["peak"],
                        "unit": valu["unit"], "frac": valu["frac"]})
        out["hbm"] = hbm
        out["valu"] = valu
    return out


def measured_traffic(workload_name, table=None):
    """HBM-side bytes per launch of the workload's dominant kernel (or of the
    kernel `table` covers) from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none
    for this workload or the kernel source changed since the counters were
    taken."""
    table = TRAFFIC if table is None else table
    if workload_name not in table:
        return None
    fname, sources = table[workload_name]
    try:
        txt = open(os.path.join(ROOT, "profiles", fname)).read()
    except OSError:
        return None
    kv = {}
    for line in txt.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip().strip("`")
    if (kv.get("workload") != workload_name
            or kv.get("kernel_source_digest") != kernel_source_digest(sources)):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mb):
    """A plain device copy of `mb` MiB (read mb, write mb) repeated 5 times,
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "c3":
        return bench_batch(args)
    if args.workload == "c4":
        return bench_adjoint(args)
    if args.workload == "c1m":
        return bench_implicit(args)
    import numpy as np
    import torch
    from paper_2605_27534_amd import surf as S

    K, W = args.steps, args.warmup
    cfg = workload(args.workload, K, W)
    prob, prec = dict(cfg["prob"]), cfg["precision"]
    prob["hj_iters_step"] = cfg.get("hj_step", 8)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    side = torch.cuda.Stream(dev)
    ncell = int(np.prod(prob["n"]))
    es = 8 if prec == 1 else 4

    with torch.cuda.stream(side):
        s = S.Surf(prob, cfg["dt"], prec)
        tens = s.tensor
        print("# generating inputs: %s, %d steps" % (cfg["name"], W + K), file=sys.stderr, flush=True)
        dev_gen = cfg.get("vof_seq_dev") is not None
        vof0 = tens(cfg["vof0_dev"](dev)) if dev_gen else tens(cfg["vof0"]())
        vofs = None
        reinit = cfg.get("reinit_every")  # ACDI: a VoF field only every `reinit` steps
        if cfg.get("vof_seq"):
            vofs = [None if reinit and (k + 1) % reinit else
                    tens(cfg["vof_seq_dev"](k, dev)) if dev_gen else tens(cfg["vof_seq"](k))
                    for k in range(W + K)]
        u_static = [tens(x) for x in cfg["u"]()] if cfg.get("u") else None
        u_list = None
        if cfg.get("u_seq"):
            u_list = [[tens(x) for x in (cfg["u_seq_dev"](k, dev) if dev_gen else cfg["u_seq"](k))]
                      for k in range(W + K)]
        c0v = cfg["c0"]() if cfg.get("c0") else None  # None: constant c0 (or no bulk)
        c0 = tens(c0v) if c0v is not None else None
        bulk = prob.get("bulk_enabled", 1)
        bufs = [[s.empty() if bulk else None, s.empty()] for _ in range(2)]
        sig = s.empty()
        hist = torch.zeros((W + K, 16), dtype=torch.float64, device=dev)
        forces = None
        if cfg.get("forces"):  # capillary and Marangoni face arrays
            forces = tuple([torch.empty(s.face_shape(d), dtype=s.dtype, device=dev)
                            for d in range(prob["dim"])] for _ in range(2))

        def reset():
            s.set_geometry(vof0, full=True)
            F, P = s.init_state(c0, cfg.get("c0_const", 1.0), cfg.get("gamma0", 0.0))
            if F is not None:
                bufs[0][0].copy_(F)
            bufs[0][1].copy_(P)

        def do_step(k):
            a, b = bufs[k % 2], bufs[(k + 1) % 2]
            u = u_list[k] if u_list is not None else u_static
            v = vofs[k] if vofs is not None else None
            s.step(a[0], a[1], b[0], b[1], u=u, vof_next=v, sigma_out=sig, totals=hist[k])
            if forces is not None:
                s.interface_force(v if v is not None else vof0, sig, out=forces)

        # 2D moving interface: step k+1's geometry is prepared on `aux` while
        # step k's transport runs on `side`; every run of steps ends with no
        # geometry pending
        pipelined = (vofs is not None and prob.get("flux_form", 0) == 0
                     and not args.no_pipeline and not reinit)
        # ACDI: each next ACDI step is prepared on `aux` during the transport
        # (steps that re-initialize from a VoF field run it in the step)
        pipelined_acdi = (bool(reinit) and prob.get("flux_form", 0) == 0
                          and not args.no_pipeline)
        aux = torch.cuda.Stream(dev)

        def run_steps(k0, k1):
            for k in range(k0, k1):
                do_step(k)
                if pipelined and k + 1 < k1:
                    s.prepare_geometry(vofs[k + 1], aux)
                elif pipelined_acdi and k + 1 < k1 and vofs[k + 1] is None:
                    s.prepare_phase(u_list[k + 1] if u_list is not None else u_static, aux)

        # ---- region 1: graph replay of K steps
        reset()
        run_steps(0, W)
        torch.cuda.synchronize()
        graph = None
        if not args.no_graph:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=side):
                run_steps(W, W + K)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record(side)
        if graph is not None:
            graph.replay()
        else:
            run_steps(W, W + K)
        t1.record(side)
        side.synchronize()
        wall = time.perf_counter() - wall0
        ms_total = t0.elapsed_time(t1)
        h1 = hist.cpu().numpy()
        assert np.all(np.isfinite(h1[W:W + K, S.T_MTOT])), "non-finite totals"
        status = s.status()

        # ---- region 2: eager K steps with per-launch events
        reset()
        run_steps(0, W)
        torch.cuda.synchronize()
        s.profile_read()
        s.profile(True)
        run_steps(W, W + K)
        torch.cuda.synchronize()
        step_ms, step_n, geom_ms, geom_n = s.profile_read()
        s.profile(False)
        h2 = hist.cpu().numpy()

        # ---- region 3: the transport kernel alone, a burst of back-to-back
        # launches between two HIP events (an event pair around one launch
        # also counts the launch's dispatch latency, about 3 us)
        burst_ms, burst_reps = None, 0
        if prob.get("flux_form", 0) == 0:
            burst_reps = 200 if ncell <= (1 << 22) else 40
            a, b = bufs[(W + K) % 2], bufs[(W + K + 1) % 2]
            u = u_list[W + K - 1] if u_list is not None else u_static
            burst_ms = s.time_transport(a[0], a[1], b[0], b[1], u=u, sigma_out=sig,
                                        reps=burst_reps)
        acdi_ms, acdi_reps = None, 200 if ncell <= (1 << 22) else 40
        if reinit:
            acdi_ms = s.time_acdi(u=u_static if u_list is None else u_list[W + K - 1],
                                  reps=acdi_reps)
        # the Marangoni face force (surf_force) on the last step's sigma, a
        # burst of back-to-back calls between HIP events
        mforce_ms = None
        if prob.get("flux_form", 0) == 0 and not prob.get("axisym"):
            fout = [torch.empty(s.face_shape(d), dtype=s.dtype, device=dev)
                    for d in range(prob["dim"])]
            reps = 200 if ncell <= (1 << 22) else 40
            for _ in range(5):
                s.force(sig, out=fout)
            f0 = torch.cuda.Event(enable_timing=True)
            f1 = torch.cuda.Event(enable_timing=True)
            f0.record(side)
            for _ in range(reps):
                s.force(sig, out=fout)
            f1.record(side)
            side.synchronize()
            mforce_ms = f0.elapsed_time(f1) / reps
        force_ms = None
        if forces is not None:  # the force kernel alone, back to back
            v_last = vofs[W + K - 1] if vofs is not None else vof0
            force_reps = FORCE_REPS if ncell <= (1 << 22) else 20
            for _ in range(3):
                s.interface_force(v_last, sig, out=forces)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(side)
            for _ in range(force_reps):
                s.interface_force(v_last, sig, out=forces)
            e1.record(side)
            side.synchronize()
            force_ms = e0.elapsed_time(e1) / force_reps

    ms_per_step = ms_total / K
    value = ncell * K / (ms_total * 1e-3) / 1e9
    kbytes, sbytes = algorithmic_bytes(cfg, es)
    k_step_ms = step_ms / max(step_n, 1)
    k_avg_ms = burst_ms if burst_ms is not None else k_step_ms
    step_gbs = sbytes * ncell / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "surfactant-step Gcell-updates/s (+ % HBM roofline)",
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "cells": ncell, "dt": cfg["dt"],
                   "hj_sweeps_per_step": prob["hj_iters_step"] if vofs is not None else 0,
                   "graph": graph is not None,
                   "pipelined_geometry": pipelined or pipelined_acdi},
        "roofline": {
            **roofline_of(transport_kernel(cfg), kbytes * ncell, k_avg_ms,
                          kernel_counters(cfg["name"])),
            "bytes_per_cell": kbytes, "avg_launch_us": round(k_avg_ms * 1e3, 3),
            "launch_timing": ("%d back-to-back launches between HIP events" % burst_reps
                              if burst_ms is not None else "HIP events around each launch"),
            "avg_launch_us_in_steps": round(k_step_ms * 1e3, 3),
            "step_bytes_per_cell": sbytes, "step_frac": round(step_gbs / HBM_PEAK_GBS, 4),
            "geometry_us_per_step": round(geom_ms / K * 1e3, 3),
        },
        "status": status,
        "wall_s": round(wall, 4),
    }
    if mforce_ms is not None:
        fbpc = (2 + prob["dim"]) * es  # reads chi, sigma; writes the dim face arrays
        out["force"] = {
            **roofline_of("k_force%d" % prob["dim"], fbpc * ncell, mforce_ms,
                          kernel_counters(cfg["name"], FORCE_COUNTERS)),
            "avg_launch_us": round(mforce_ms * 1e3, 3),
            "timing": "back-to-back surf_force calls between HIP events",
            "bytes_per_cell": fbpc}
    if acdi_ms is not None:
        ab = ACDI_WORDS_PER_CELL * es
        out["config"]["acdi_reinit_every"] = reinit
        out["acdi"] = {
            "kernels": "k_acdi_adv + k_acdi_reg", "avg_step_us": round(acdi_ms * 1e3, 3),
            "timing": "%d back-to-back ACDI steps between HIP events" % acdi_reps,
            "bytes_per_cell": ab, "achieved": round(ab * ncell / (acdi_ms * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ab * ncell / (acdi_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if force_ms is not None:
        three = prob["dim"] == 3
        # 2D: reads the VoF, writes four face arrays; 3D: reads the VoF, chi
        # and sigma, writes six
        fb = (9 if three else FORCE_WORDS_PER_CELL) * es
        out["config"]["interface_forces"] = True
        out["iface"] = {
            "kernel": "k_iface3_cells + k_iface3_faces" if three else "k_iface_force",
            "avg_launch_us": round(force_ms * 1e3, 3),
            "timing": "%d back-to-back calls between HIP events" % force_reps,
            "bytes_per_cell": fb, "achieved": round(fb * ncell / (force_ms * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(fb * ncell / (force_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(cfg["name"], IFACE_TRAFFIC)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baselines(cpu_baseline, cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """The 64-instance ensemble: batched form against the plain path."""
    import numpy as np
    import torch
    from paper_2605_27534_amd import configs as C
    from paper_2605_27534_amd import surf as S
    from paper_2605_27534_amd.batch import Batch
    K, W = args.steps, args.warmup
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ens = C.c3_ensemble()
    side = torch.cuda.Stream(dev)
    cells = sum(int(np.prod(e["prob"]["n"])) for e in ens)
    print("# generating inputs: 64 instances, %d cells" % cells, file=sys.stderr, flush=True)
    vofs = [torch.as_tensor(e["vof0"]()).to(dev, torch.float32) for e in ens]
    with torch.cuda.stream(side):
        b = Batch([e["prob"] for e in ens], [e["dt"] for e in ens], S.SURF_F32)
        for i, e in enumerate(ens):
            b.set_geometry(i, vofs[i].reshape(b.shapes[i]).contiguous())
            b.init_state(i, None, e["c0_const"], e["gamma0"])
        choice, times = b.tune()
        tot = torch.zeros((len(ens), 16), dtype=torch.float64, device=dev)
        b.step(W, tot)
        side.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.step(K, tot)  # records the graphs of K steps from both buffer parities
        b.step(K, tot)
        side.synchronize()
        t0.record(side)
        b.step(K, tot)  # replays it
        t1.record(side)
        side.synchronize()
        ms_batch = t0.elapsed_time(t1)
        # plain path: the same instances one after the other, K steps each
        plain = []
        for i, e in enumerate(ens):
            s = S.Surf(e["prob"], e["dt"], S.SURF_F32)
            s.set_geometry(vofs[i].reshape(b.shapes[i]).contiguous(), full=True)
            F, P = s.init_state(None, e["c0_const"], e["gamma0"])
            F2, P2, sg = s.empty(), s.empty(), s.empty()
            plain.append([s, F, P, F2, P2, sg])
        side.synchronize()

        def plain_steps(k):
            for st in plain:
                s, F, P, F2, P2, sg = st
                for _ in range(k):
                    s.step(F, P, F2, P2, sigma_out=sg)
                    F, F2, P, P2 = F2, F, P2, P
                st[1:5] = [F, P, F2, P2]

        plain_steps(W)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            plain_steps(K)
        side.synchronize()
        t0.record(side)
        g.replay()
        t1.record(side)
        side.synchronize()
        ms_plain = t0.elapsed_time(t1)
    value = cells * K / (ms_batch * 1e-3) / 1e9
    kern_us = times[choice] if 0 <= choice < len(times) else None
    bpc = 24  # FP32, no flow: reads chi, F, psi; writes F, psi, sigma
    out = {"metric": "surfactant-step Gcell-updates/s (batched form)", "value": round(value, 4),
           "unit": "Gcell-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": round(ms_batch / K, 6), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "ensemble of 64 static circles fp32", "cells": cells,
                      "tuned_choice": choice},
           "plain": {"value": round(cells * K / (ms_plain * 1e-3) / 1e9, 4),
                     "ms_per_step": round(ms_plain / K, 6),
                     "note": "the same 64 instances stepped one after the other with surf_step, "
                             "replayed from one HIP graph"},
           "batched_over_plain": round(ms_plain / ms_batch, 3)}
    if kern_us:
        ach = bpc * cells / (kern_us * 1e-6) / 1e9
        out["roofline"] = {"bound": "hbm", "kernel": "k_batch_col2d", "achieved": round(ach, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                           "traffic": None, "bytes_per_cell": bpc,
                           "avg_launch_us": round(kern_us, 3),
                           "launch_timing": "3 back-to-back launches between HIP events (the "
                                            "tuner's measurement of its choice)",
                           "tuner_times_us": [round(t, 2) for t in times if t > 0]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baselines(cpu_baseline_ensemble, ens, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_ensemble(ens, seconds):
    """The oracle on one instance of each grid size of the ensemble, the same
    number of steps each (about `seconds` in all), scaled by cell count."""
    import math
    import numpy as np
    from oracle import oracle as O
    picked = {}
    for e in ens:
        picked.setdefault(e["prob"]["n"][0], e)
    insts = [picked[k] for k in sorted(picked)]
    state = []
    for e in insts:
        prob = e["prob"]
        q = O.full(prob)
        iters = 2 * int(math.ceil(q["chi_max_eps"] * q["eps"] / (q["h"] / q["dim"]) - 1e-9))
        chi = O.geometry(prob, e["vof0"](), iters)
        F, P = O.init_state(prob, chi, c0_const=e["c0_const"], gamma0=e["gamma0"])
        state.append([chi, F, P, np.zeros(16)])
    cells = sum(int(np.prod(e["prob"]["n"])) for e in insts)
    el, k = 0.0, 0
    while (el < seconds or k == 0) and k < 200:
        t = time.perf_counter()
        for e, st in zip(insts, state):
            st[1], st[2], _, st[3] = O.step(e["prob"], st[0], None, st[1], st[2], e["dt"], st[3])
        el += time.perf_counter() - t
        k += 1
    return {"value": round(cells * k / el / 1e9, 6), "unit": "Gcell-updates/s", "kind": "oracle",
            "sample": "one instance of each size (%s), %d steps each, FP64, %.1f s"
                      % (", ".join("%d^2" % n for n in sorted(picked)), k, el)}


def bench_adjoint(args):
    """The 128^3 adjoint sphere: forward and checkpointed adjoint steps."""
    import numpy as np
    import torch
    from paper_2605_27534_amd import configs as C
    from paper_2605_27534_amd import surf as S
    from paper_2605_27534_amd.adjoint import Rollout
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = C.c4_adjoint()
    N = args.steps
    Kc = min(cfg["checkpoint"], N)  # the workload's checkpoint interval (50)
    print("# generating inputs: %s" % cfg["name"], file=sys.stderr, flush=True)
    ro = Rollout(cfg["prob"], cfg["dt"], S.SURF_F32, vof=cfg["vof0"](), u=cfg["u"](),
                 gamma0=cfg["gamma0"], nsteps=N, checkpoint=Kc)
    th = torch.tensor(cfg["theta_nominal"], dtype=torch.float64, device=dev)
    c0 = ro.s.tensor(cfg["c0"]())
    tg = torch.full((N,), 0.95, dtype=torch.float64, device=dev)
    ro.forward(th, c0, tg)  # warm-up
    torch.cuda.synchronize()
    t0, t1, t2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t0.record()
    loss, tot, w, ck = ro.forward(th, c0, tg)
    t1.record()
    ro.backward(w, ck, tot)
    t2.record()
    torch.cuda.synchronize()
    ms_f, ms_b = t0.elapsed_time(t1), t1.elapsed_time(t2)
    cells = int(np.prod(cfg["prob"]["n"]))
    # one adjoint step alone, a burst of back-to-back calls between HIP
    # events (same inputs; the dtheta accumulator only grows)
    s = ro.s
    F0, P0 = ck[0]
    lF, lP, nF, nP = s.empty(), s.empty(), s.empty(), s.empty()
    lF.zero_()
    lP.fill_(1e-3)
    dth = torch.zeros(4, dtype=torch.float64, device=dev)
    # the backward pass's form of the step: with the advected state the
    # recomputation kept, or advecting again where the context has none
    star = None
    if ro.keep_advected:
        star = (s.empty(), s.empty())
        s.step(F0, P0, s.empty(), s.empty(), u=ro.u, totals=torch.zeros(16, dtype=torch.float64,
                                                                       device=dev), star=star)
    reps = 50
    for _ in range(3):
        s.adjoint_step(F0, P0, lF, lP, nF, nP, dth, u=ro.u, w=w[0:1], star=star)
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record()
    for _ in range(reps):
        s.adjoint_step(F0, P0, lF, lP, nF, nP, dth, u=ro.u, w=w[0:1], star=star)
    a1.record()
    torch.cuda.synchronize()
    adj_us = a0.elapsed_time(a1) / reps * 1e3
    # FP32 reads of chi, u (3), F, psi, lambda (2) and, when kept, the
    # advected F and psi; writes of lambda (2)
    bpc = 48 if star is not None else 40
    out = {"metric": "surfactant-step Gcell-updates/s (adjoint form)",
           "value": round(cells * N / (ms_b * 1e-3) / 1e9, 4), "unit": "Gcell-updates/s",
           "n_gpus": 1, "steps": N, "warmup": 1, "ms_per_step": round(ms_b / N, 6),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": cfg["name"], "cells": cells, "checkpoint": Kc,
                      "note": "backward = recomputation of each checkpoint segment + the adjoint "
                              "steps, launched eagerly"},
           "forward": {"value": round(cells * N / (ms_f * 1e-3) / 1e9, 4),
                       "ms_per_step": round(ms_f / N, 6)},
           "adjoint_over_forward_time": round(ms_b / ms_f, 3)}
    ach = bpc * cells / (adj_us * 1e-6) / 1e9
    kern = ("adjoint step (k_adj_src, k_adj_adv, k_adj_final) on the kept advected state"
            if star is not None else "adjoint step (k_adv_star, k_adj_src, k_adj_adv, k_adj_final)")
    out["roofline"] = {"bound": "hbm", "kernel": kern,
                       "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                       "bytes_per_cell": bpc, "avg_launch_us": round(adj_us, 3),
                       "launch_timing": "%d back-to-back adjoint steps between HIP events" % reps}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baselines(cpu_baseline_adjoint, cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(cfg, seconds):
    """The oracle's forward and adjoint steps on the 128^3 sphere (the first
    S forward steps, then S adjoint steps back over them)."""
    import numpy as np
    from oracle import oracle as O
    prob = cfg["prob"]
    chi = O.geometry(prob, cfg["vof0"](), 108)
    u = cfg["u"]()
    q = O.with_theta(prob, cfg["theta_nominal"])
    F, P = O.init_state(q, chi, c0=cfg["c0"](), gamma0=cfg["gamma0"])
    cells = int(np.prod(prob["n"]))
    states, el, k = [(F, P)], 0.0, 0
    while (el < 0.25 * seconds or k == 0) and k < 20:
        t = time.perf_counter()
        F, P, _, _ = O.step(q, chi, u, F, P, cfg["dt"])
        el += time.perf_counter() - t
        states.append((F, P))
        k += 1
    lF, lP = np.zeros_like(F), np.full_like(P, 1e-3)
    ea = 0.0
    for n in range(k - 1, -1, -1):
        t = time.perf_counter()
        lF, lP, _ = O.adjoint_step(q, chi, u, states[n][0], states[n][1], cfg["dt"], lF, lP)
        ea += time.perf_counter() - t
    return {"value": round(cells * k / ea / 1e9, 6), "unit": "Gcell-updates/s", "kind": "oracle",
            "sample": "%d forward steps (%.1f s, %.4f Gcell-updates/s), then %d adjoint steps "
                      "(%.1f s; the value), FP64" % (k, el, cells * k / el / 1e9, k, ea)}


# ACDI: k_acdi_adv reads phi and the d face velocities, writes phi* and s;
# k_acdi_reg reads phi* and s, writes phi and chi (2D: 5 + 4 words)
ACDI_WORDS_PER_CELL = 9
# interfacial forces (2D): read the VoF, write the capillary and Marangoni
# forces on the x and y faces (about one face per cell and axis); the level
# set and sigma are read only in tiles that hold interface
FORCE_WORDS_PER_CELL = 5
FORCE_REPS = 200
CG_ITER_BYTES_PER_CELL = 13 * 8  # reads x p r w z minv dg w_face, writes x p r w z


def bench_implicit(args):
    """The 1024^2 soluble expanding circle with substep 2 implicit."""
    import numpy as np
    import torch
    from paper_2605_27534_amd import configs as C
    from paper_2605_27534_amd import surf as S
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    side = torch.cuda.Stream(dev)
    cfg = C.c1_implicit()
    K, W = min(args.steps, cfg["steps"]), args.warmup
    prob = dict(cfg["prob"])
    prob["hj_iters_step"] = cfg["hj_step"]
    ncell = int(np.prod(prob["n"]))
    print("# generating inputs: %s, %d steps" % (cfg["name"], W + K), file=sys.stderr, flush=True)
    with torch.cuda.stream(side):
        s = S.Surf(prob, cfg["dt"], S.SURF_F32)
        T = s.tensor
        vof0 = T(cfg["vof0"]())
        vofs = [T(cfg["vof_seq"](k)) for k in range(W + K)]
        u = [T(x) for x in cfg["u"]()]
        c0 = T(cfg["c0"]())
        bufs = [[s.empty(), s.empty()] for _ in range(2)]
        sig = s.empty()
        hist = torch.zeros((W + K, 16), dtype=torch.float64, device=dev)
        forces = None
        if cfg.get("forces"):  # capillary and Marangoni face arrays
            forces = tuple([torch.empty(s.face_shape(d), dtype=s.dtype, device=dev)
                            for d in range(prob["dim"])] for _ in range(2))

        def reset():
            s.set_geometry(vof0, full=True)
            F, P = s.init_state(c0, 1.0, cfg["gamma0"])
            bufs[0][0].copy_(F)
            bufs[0][1].copy_(P)

        def do_step(k):
            a, b = bufs[k % 2], bufs[(k + 1) % 2]
            s.step(a[0], a[1], b[0], b[1], u=u, vof_next=vofs[k], sigma_out=sig, totals=hist[k])

        reset()
        warm_iters = []
        for k in range(W):
            do_step(k)
            warm_iters.append(s.solver_iterations())
        torch.cuda.synchronize()
        print("# warm-up solves (iterations per solve): %s" % warm_iters, file=sys.stderr, flush=True)
        # ---- region 1: K steps launched eagerly
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record(side)
        for k in range(W, W + K):
            do_step(k)
        t1.record(side)
        side.synchronize()
        wall = time.perf_counter() - wall0
        ms_eager = t0.elapsed_time(t1)
        last_iters = s.solver_iterations()
        h1 = hist.cpu().numpy()
        assert np.all(np.isfinite(h1[W:W + K, S.T_MTOT])), "non-finite totals"
        status = s.status()
        print("# eager: %.3f ms/step, status %d" % (ms_eager / K, status), file=sys.stderr,
              flush=True)
        # ---- region 2: the same K steps replayed from a HIP graph
        ms_graph = None
        if args.implicit_graph:
            reset()
            for k in range(W):
                do_step(k)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=side):
                for k in range(W, W + K):
                    do_step(k)
            torch.cuda.synchronize()
            t0.record(side)
            graph.replay()
            t1.record(side)
            side.synchronize()
            ms_graph = t0.elapsed_time(t1)
            status |= s.status()
            del graph
            print("# graph: %.3f ms/step" % (ms_graph / K), file=sys.stderr, flush=True)
        # ---- region 3: the CG iteration kernel alone (bulk problem)
        reps = 200
        it_ms = s.time_solver(1, reps)
    ms_total = min(ms_eager, ms_graph) if ms_graph is not None else ms_eager
    achieved = CG_ITER_BYTES_PER_CELL * ncell / (it_ms * 1e-3) / 1e9
    out = {
        "metric": "surfactant-step Gcell-updates/s (+ % HBM roofline)",
        "value": round(ncell * K / (ms_total * 1e-3) / 1e9, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms_total / K, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 state, f64 solver", "data": "synthetic",
        "config": {"workload": cfg["name"], "cells": ncell, "dt": cfg["dt"],
                   "picard_sweeps": prob["picard_iters"], "cg_tol": prob["cg_tol"],
                   "cg_max_iters": prob["cg_max_iters"],
                   "timing": "graph replay" if ms_total == ms_graph else "eager launches"},
        "ms_per_step_eager": round(ms_eager / K, 6),
        "ms_per_step_graph": round(ms_graph / K, 6) if ms_graph is not None else None,
        "simulated_time_per_s": round(cfg["dt"] * K / (ms_total * 1e-3), 6),
        "solve_iterations_last_step": last_iters,
        "solve_iterations_warmup": warm_iters,
        "roofline": {
            "bound": "hbm", "kernel": "k_cg_iter", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(cfg["name"]), "bytes_per_cell": CG_ITER_BYTES_PER_CELL,
            "avg_launch_us": round(it_ms * 1e3, 3),
            "launch_timing": "%d back-to-back iteration launches between HIP events" % reps,
            "cg_share_of_step": round(sum(last_iters) * it_ms / (ms_total / K), 4),
        },
        "status": status,
        "wall_s": round(wall, 4),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baselines(cpu_baseline_implicit, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline_implicit(seconds):
    """The implicit FP64 oracle (sparse direct solves) on the same workload at
    256^2 (the 1024^2 factorizations take minutes)."""
    import math
    import numpy as np
    from oracle import implicit as I
    from oracle import oracle as O
    from paper_2605_27534_amd import configs as C
    cfg = C.c1_implicit(n=256)
    prob = dict(cfg["prob"])
    q = O.full(prob)
    ncell = int(np.prod(q["n"]))
    iters = 2 * int(math.ceil(q["chi_max_eps"] * q["eps"] / (q["h"] / q["dim"]) - 1e-9))
    chi = O.geometry(prob, cfg["vof0"](), iters)
    F, P = O.init_state(prob, chi, c0=cfg["c0"](), gamma0=cfg["gamma0"])
    u = cfg["u"]()
    tot = np.zeros(16)
    el, k = 0.0, 0
    while el < seconds and k < 50:
        vk = cfg["vof_seq"](k)
        t = time.perf_counter()
        chi = O.geometry(prob, vk, cfg["hj_step"], chi=chi)
        F, P, _, tot = I.implicit_step(prob, chi, u, F, P, cfg["dt"], picard=prob["picard_iters"],
                                       totals=tot)
        el += time.perf_counter() - t
        k += 1
    return {"value": round(ncell * k / el / 1e9, 6), "unit": "Gcell-updates/s",
            "kind": "oracle",
            "sample": "first %d steps of the same workload at 256^2 (geometry warm start + "
                      "implicit step with sparse direct solves), FP64, %.1f s" % (k, el)}


def cpu_baselines(fn, *args):
    """The oracle's rate on all host cores (`cpu_baseline`), with the
    single-core rate of the same sample beside it."""
    from oracle import oracle as O
    cores = O.set_threads(None)
    O.set_threads(cores)
    allc = fn(*args)
    allc["cores"] = cores
    O.set_threads(1)
    one = fn(*args)
    O.set_threads(None)
    allc["one_core"] = {"value": one["value"], "sample": one["sample"]}
    return allc


def cpu_baseline(cfg, seconds):
    """The FP64 oracle as it stands on a bounded sample of the same workload:
    the first S steps (the interface step + the surfactant step), S chosen
    from a one-step probe to take about `seconds`."""
    import math
    import numpy as np
    from oracle import oracle as O
    prob = dict(cfg["prob"])
    q = O.full(prob)
    ncell = int(np.prod(q["n"]))
    vof0 = cfg["vof0"]()
    iters = 2 * int(math.ceil(q["chi_max_eps"] * q["eps"] / (q["h"] / q["dim"]) - 1e-9))
    chi = O.geometry(prob, vof0, iters)
    c0 = cfg["c0"]() if cfg.get("c0") else None
    F, P = O.init_state(prob, chi, c0=c0, c0_const=cfg.get("c0_const", 1.0),
                        gamma0=cfg.get("gamma0", 0.0))
    u = cfg["u"]() if cfg.get("u") else None
    hj = cfg.get("hj_step", 8)
    reinit = cfg.get("reinit_every")
    st = {"chi": chi}
    if reinit:
        from oracle import acdi as A
        st["phi"] = A.phi_of_chi(prob, chi)

    def inputs(k):
        # inputs of step k, generated outside the timed part
        vk = None
        if cfg.get("vof_seq") and (not reinit or (k + 1) % reinit == 0):
            vk = cfg["vof_seq"](k)
        uk = cfg["u_seq"](k) if cfg.get("u_seq") else u
        return vk, uk

    def one(vk, uk, F, P, tot):
        if reinit:
            if vk is not None:
                st["chi"] = O.geometry(prob, vk, hj, chi=st["chi"])
                st["phi"] = A.phi_of_chi(prob, st["chi"])
            else:
                st["phi"] = A.acdi_step(prob, st["phi"], uk, cfg["dt"], prob["acdi_zeta"])
                st["chi"] = A.chi_of_phi(prob, st["phi"])
        elif vk is not None:
            st["chi"] = O.geometry(prob, vk, hj, chi=st["chi"])
        F, P, S, tot = O.step(prob, st["chi"], uk, F, P, cfg["dt"], tot)
        if cfg.get("forces"):
            K.forces(prob, vk if vk is not None else vof0, st["chi"], S)
        return F, P, tot

    if cfg.get("forces"):
        from oracle import capillary as K
    tot = np.zeros(16)
    vk, uk = inputs(0)
    t = time.perf_counter()
    F, P, tot = one(vk, uk, F, P, tot)
    probe = time.perf_counter() - t
    if probe >= seconds:  # one step is already the sample
        nsteps, el = 1, probe
    else:
        nsteps = max(1, min(200, int(seconds / max(probe, 1e-6))))
        el = 0.0
        for k in range(1, nsteps + 1):
            vk, uk = inputs(k)
            t = time.perf_counter()
            F, P, tot = one(vk, uk, F, P, tot)
            el += time.perf_counter() - t
    what = ("ACDI step" if reinit else "geometry warm start") + " + step"
    if cfg.get("forces"):
        what += " + interfacial forces"
    return {"value": round(ncell * nsteps / el / 1e9, 6), "unit": "Gcell-updates/s",
            "kind": "oracle",
            "sample": "first %d steps of the same workload (%s), FP64, %.1f s"
                      % (nsteps, what, el)}


if __name__ == "__main__":
    main()
