"""Benchmark of the shallow-water step on one MI355X.

Workload: the 10,000,000-triangle water drop (jittered split-square mesh of a 10 km x 5 km box,
sloping bed with 64 Gaussian bumps, Manning n ~ U(0.015, 0.06), Gaussian hump of water at the
centre, walls, Morton-ordered cells).  A "step" is one explicit step of the whole path:
reconstruction + HLLC on every cell's three edges, update, friction and the CFL dt reduction.

Prints one JSON line: cell-updates/s of the FP64 step (the paper's precision) as `value`, the
FP32 step under `variants`, the HBM roofline of the step kernel from its algorithmic bytes, and
the CPU oracle timed on this host on a bounded sample of the same workload.
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

HBM_PEAK_GBPS = 8000.0     # MI355X HBM3E, public specification
KERNELS = {"tiled": "tile_step_kernel", "cell": "step_kernel"}   # step kernel of each variant
PROFILED_KERNEL = "tile_step_kernel"   # the kernel whose counters profiles/ holds


def algorithmic_bytes(n_cells: int, n_nodes: int, word: int) -> int:
    """Compulsory HBM bytes of one step: every array read or written once.

    Per cell: U in (3 words), U out (3), bed (1), roughness (1), three neighbour ids and three
    node ids (int32); per node: two double coordinates."""
    return n_cells * (8 * word + 24) + n_nodes * 16


def kernel_source_hash() -> str:
    """sha256[:16] of the step kernels' source with comments and blank lines removed: a
    committed counter run stays valid across comment edits, not across code changes."""
    import re
    p = os.path.join(ROOT, "paper_1807_00672_amd", "csrc", "swe_kernels.hip")
    with open(p) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    code = "\n".join(ln.rstrip() for ln in src.splitlines() if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def load_counter(dtype: str, n_cells: int, what: str = "bytes_per_launch"):
    """A per-launch counter figure of the step kernel (HBM bytes, VALU instructions) from
    committed counter runs, if they were taken on the current kernel source for this
    workload; else None."""
    p = os.path.join(ROOT, "profiles", "tile_step_kernel_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_sha") != kernel_source_hash() or d.get("n_cells") != n_cells:
        return None
    return d.get(what, {}).get(dtype)


# VALU issue: one wave64 instruction takes 4 cycles of a 16-lane SIMD; 256 CUs x 4 SIMDs at
# 2.4 GHz (MI355X).
N_SIMD, CLOCK_HZ = 1024, 2.4e9


def valu_issue_s(valu_insts):
    return valu_insts * 4 / N_SIMD / CLOCK_HZ


def alu_view(r):
    """The step's second ceiling: its counted VALU instructions issued at full rate on every
    SIMD, against the measured step time."""
    v = r.get("valu_insts_per_launch")
    if v is None:
        return None
    t = valu_issue_s(v)
    return {"valu_insts_per_launch": v, "valu_issue_us_at_full_rate": t * 1e6,
            "frac_of_step_time": t / (r["ms_per_step"] * 1e-3),
            "source": "SQ_INSTS_VALU of the committed counter run (profiles/)"}


# swe_run replays groups of 8 steps from one captured graph once a run has at least 16 steps:
# a warm-up of that length captures it, so no timed window pays for the capture.
GRAPH_WARMUP = 16
# Device time the warm-up keeps the GPU stepping before the first timed window: a short
# warm-up leaves the first windows several per cent slow while the device's clocks settle.
SETTLE_S = 0.25


def time_gpu(solver, steps, warmup, stream, windows=5):
    """Median over `windows` timed windows of exactly `steps` steps each.  Before them, an
    untimed warm-up on the same stream: max(warmup, GRAPH_WARMUP) steps, then more untimed
    windows of `steps` steps until the warm-up has kept the device busy for SETTLE_S.  HIP
    events on the stream that runs the steps bracket each window.  Returns (ms of the median
    window, rc, stats, warm-up steps run, every timed window's ms)."""
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    warm = max(warmup, GRAPH_WARMUP)
    with torch.cuda.stream(stream):
        ev0.record(stream)
        solver.run(warm, sync=False, stream=stream)
        ev1.record(stream)
    torch.cuda.synchronize()
    busy = ev0.elapsed_time(ev1) * 1e-3
    chunk = max(steps, GRAPH_WARMUP)
    while busy < SETTLE_S:
        with torch.cuda.stream(stream):
            ev0.record(stream)
            solver.run(chunk, sync=False, stream=stream)
            ev1.record(stream)
        torch.cuda.synchronize()
        busy += ev0.elapsed_time(ev1) * 1e-3
        warm += chunk
    times = []
    for _ in range(windows):
        with torch.cuda.stream(stream):
            ev0.record(stream)
            solver.run(steps, sync=False, stream=stream)
            ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    ms = float(np.median(times))
    rc, st = solver.stats(stream=stream)
    return ms, rc, st, warm, times


def bench_ensemble(dtype: str, steps: int, warmup: int, stream) -> dict:
    """Config 4: 256 scenarios (5e3 to 2e5 triangles, own inflow and roughness, own CFL dt)
    stepped by one launch per step, against the same scenarios each run on its own."""
    import torch

    import gen
    import paper_1807_00672_amd as swe
    cases = gen.ensemble(256)
    meshes = [swe.Mesh(c.xy, c.tri, c.edge_tag) for c in cases]
    batch = swe.Batch(meshes)
    bs = swe.BatchSolver(batch, cases, dtype=dtype)
    bs.run(warmup)   # at least 16 steps: captures the batch's graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        bs.run(steps, sync=False, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) * 1e-3
    rc, st = bs.run(0, stream=stream)
    assert rc == 0 and all(x["steps"] == warmup + steps for x in st), (rc, st[:2])
    singles = [swe.Solver(m, c.z, c.n, c.h, c.hu, c.hv, dtype=dtype, inflow_q=c.inflow_q)
               for m, c in zip(meshes, cases)]
    for sv in singles:
        sv.run(warmup, sync=False)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for sv in singles:
            sv.run(steps, sync=False, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t_single = e0.elapsed_time(e1) * 1e-3
    same = True
    for k, sv in enumerate(singles):
        rc1, st1 = sv.stats(stream=stream)
        a, b = sv.numpy_state(), bs.numpy_state(k)
        same &= rc1 == 0 and st1["t"] == st[k]["t"] and all(np.array_equal(x, y) for x, y in zip(a, b))
    # the same separate runs spread over several streams (default priority), so that the
    # small scenarios' kernels may overlap
    n_str = 8
    streams = [torch.cuda.Stream() for _ in range(n_str)]
    multi = [swe.Solver(m, c.z, c.n, c.h, c.hu, c.hv, dtype=dtype, inflow_q=c.inflow_q)
             for m, c in zip(meshes, cases)]
    for k, sv in enumerate(multi):
        sv.run(warmup, sync=False, stream=streams[k % n_str])
    torch.cuda.synchronize()
    done = [torch.cuda.Event() for _ in range(n_str)]
    with torch.cuda.stream(stream):
        e0.record(stream)
        for q in streams:
            q.wait_event(e0)
        for k, sv in enumerate(multi):
            sv.run(steps, sync=False, stream=streams[k % n_str])
        for q, ev in zip(streams, done):
            ev.record(q)
            stream.wait_event(ev)
        e1.record(stream)
    torch.cuda.synchronize()
    t_multi = e0.elapsed_time(e1) * 1e-3
    for k, sv in enumerate(multi):
        rc1, st1 = sv.stats(stream=streams[k % n_str])
        a, b = sv.numpy_state(), bs.numpy_state(k)
        same &= rc1 == 0 and st1["t"] == st[k]["t"] and all(np.array_equal(x, y) for x, y in zip(a, b))
    n_cells = int(batch.n_cells)
    t_sep = min(t_single, t_multi)
    return {"scenarios": len(cases), "n_cells": n_cells, "steps": steps,
            "batched_cell_updates_per_s": n_cells * steps / t_batch,
            "separate_cell_updates_per_s": n_cells * steps / t_sep,
            "batched_s": t_batch, "separate_one_stream_s": t_single,
            f"separate_{n_str}_streams_s": t_multi, "speedup": t_sep / t_batch,
            "bitwise_equal_to_separate": bool(same),
            "separate": "the faster of the runs one after another on one stream and spread "
                        f"over {n_str} streams"}


def bench_shards(mesh, case, stream, parts: int = 8, steps: int = 100) -> dict:
    """One GPU's share of the 10M-cell mesh split over `parts` devices: a contiguous Morton
    range of T/parts cells with its halo, stepped on its own (the kernel at its real shape);
    and all the shards stepped in turn on this device with their halo exchanges (pack, copy,
    unpack) and the dt all-reduce, FP64."""
    import torch

    import paper_1807_00672_amd as swe
    sh = swe.ShardedSolver(mesh, parts, case.z, case.n, case.h, case.hu, case.hv, dtype="f64")
    q = parts // 2
    m = sh.meshes[q]
    one = swe.Solver(m, *[np.asarray(a, np.float64)[mesh.perm][m.global_ids]
                          for a in (case.z, case.n, case.h, case.hu, case.hv)], dtype="f64")
    ms_one, rc, st, _, _ = time_gpu(one, steps, 10, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sh.step(5)
    torch.cuda.synchronize()
    e0.record()
    sh.step(steps // 5)
    e1.record()
    torch.cuda.synchronize()
    ms_all = e0.elapsed_time(e1) / (steps // 5)
    e0.record()
    for _ in range(steps // 5):
        sh.exchange()
    e1.record()
    torch.cuda.synchronize()
    us_x = e0.elapsed_time(e1) * 1e3 / (steps // 5)
    halos = [mm.n_cells - mm.n_owned for mm in sh.meshes]
    return {"parts": parts, "shard": q, "n_owned": m.n_owned, "n_halo": m.n_cells - m.n_owned,
            "shard_ms_per_step": ms_one / steps,
            "shard_cell_updates_per_s": m.n_owned * steps / (ms_one * 1e-3),
            "all_shards_on_one_gpu_ms_per_step": ms_all,
            "exchange_us_per_step": us_x, "halo_cells_total": int(sum(halos))}


def bench_configs(stream, dtypes, tiles) -> dict:
    """Configs 1 (10,000-cell dam break, 200 steps) and 2 (1,000,000-cell wet/dry bumps, 1,000
    steps) in full on the GPU, each precision on the tile size the autotuner picks among
    `tiles` for its size class."""
    import torch

    import gen
    import paper_1807_00672_amd as swe
    out = {}
    for k in (1, 2):
        case = gen.config(k)
        r = {"n_cells": case.n_cells, "steps": case.steps}
        for dt in dtypes:
            by_tile = None
            tile = tiles[0]
            if len(tiles) > 1:
                tile, per_tile = swe.tune.tune_tiles(case.xy, case.tri, case.z, case.n, case.h,
                                                     case.hu, case.hv, case.edge_tag, dtype=dt,
                                                     steps=20, tiles=tiles, order="morton")
                by_tile = {str(t): min(v for v in q["ms_per_step"].values() if v > 0)
                           for t, q in per_tile.items()}
            mesh = swe.Mesh(case.xy, case.tri, case.edge_tag, tile=tile)
            solver = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dt)
            ms, rc, st, warm, _ = time_gpu(solver, case.steps, 0, stream)
            if rc != swe.SWE_OK or st["steps"] != warm + 5 * case.steps:
                raise RuntimeError(f"config {k} {dt}: rc={rc} stats={st}")
            r[dt] = {"cell_updates_per_s": case.n_cells * case.steps / (ms * 1e-3),
                     "ms_per_step": ms / case.steps, "tile": tile,
                     "tuner_ms_per_step_by_tile": by_tile}
            del solver, mesh
            torch.cuda.empty_cache()
        out[f"config{k}"] = r
    return out


def bench_adjoint(stream, steps: int = 2000) -> dict:
    """Config 5: the gauge-misfit adjoint (checkpointing forward + reverse sweep) of 2,000 FP64
    steps on the 250,000-cell calibration setup, against the plain forward run of the same
    steps with the same replayed dt sequence; then the same adjoint storing every step
    (ckpt_every = 1, no recompute), whose gradients must equal the checkpointed ones bit for
    bit."""
    import torch

    import gen
    import paper_1807_00672_amd as swe
    from paper_1807_00672_amd import _abi as A
    from paper_1807_00672_amd.solver import _ptr, _stream_handle
    case = gen.calibration(steps=steps)
    ex = case.extra
    mesh = swe.Mesh(case.xy, case.tri)
    inv = np.empty(mesh.n_cells, np.int64)
    inv[mesh.perm] = np.arange(mesh.n_cells)
    g_mesh = torch.as_tensor(inv[ex["gauges"]], device=mesh.device)
    # observations: the hidden roughness with the CFL dt, h at the gauges every obs_every steps
    sv = swe.Solver(mesh, case.z, ex["n_hidden"], case.h, case.hu, case.hv, dtype="f64")
    dts, obs = [], []
    for k in range(steps):
        dts.append(sv.stats()[1]["dt_next"])
        sv.step()
        if (k + 1) % ex["obs_every"] == 0:
            obs.append(sv.device_state()[0][g_mesh].cpu().numpy())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dt_dev = torch.as_tensor(np.array(dts, np.float64), device=mesh.device)

    def forward():
        fw = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype="f64")
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            e0.record(stream)
            fw.run(steps, dt_seq=dt_dev, sync=False, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    def adjoint(calib):
        sa = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype="f64")
        out = [torch.empty(mesh.n_cells, dtype=torch.float64, device=mesh.device)
               for _ in range(5)]
        grads = A.swe_grads(*[_ptr(o) for o in out])
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            e0.record(stream)
            j = A.swe_adjoint(mesh.handle, mesh.dev, sa.params, sa.state, steps, _ptr(calib.dt),
                              calib.loss, calib.ckpt_every, grads, _ptr(calib.ws),
                              calib.ws.numel(), _stream_handle(stream))
            e1.record(stream)
        torch.cuda.synchronize()
        fwd_ms, rev_ms = A.swe_adjoint_timings()
        return e0.elapsed_time(e1) * 1e-3, fwd_ms * 1e-3, rev_ms * 1e-3, j, out

    forward()
    t_fwd = min(forward() for _ in range(3))
    res, grads = {}, {}
    for k in (ex["ckpt_every"], 1):
        calib = swe.Calibration(mesh, np.array(dts), ex["gauges"], np.array(obs), ex["obs_every"],
                                ckpt_every=k)
        adjoint(calib)
        runs = sorted((adjoint(calib) for _ in range(3)), key=lambda r: r[0])
        t_adj, t_ckpt, t_rev, loss, out = runs[0]
        grads[k] = [o.cpu() for o in out]
        res[k] = {"ckpt_every": k, "workspace_GB": calib.ws.numel() / 1e9,
                  "adjoint_s": t_adj, "adjoint_forward_pass_s": t_ckpt,
                  "adjoint_reverse_sweep_s": t_rev, "reverse_over_forward": t_rev / t_fwd,
                  "adjoint_over_forward": t_adj / t_fwd, "loss": loss}
        del calib, out, runs
        torch.cuda.empty_cache()
    # the same adjoint through torch.autograd with device tensors (AdjointLoss: inputs permuted
    # to mesh order and gradients back on the device), against swe_adjoint alone
    calib = swe.Calibration(mesh, np.array(dts), ex["gauges"], np.array(obs), ex["obs_every"],
                            ckpt_every=ex["ckpt_every"])
    ins = [torch.tensor(np.asarray(a, np.float64), device=mesh.device, requires_grad=True)
           for a in (case.n, case.z, case.h, case.hu, case.hv)]

    def autograd_once():
        for t in ins:
            t.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = swe.AdjointLoss.apply(calib, *ins)
        loss.backward()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    sa = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype="f64")
    outs = [torch.empty(mesh.n_cells, dtype=torch.float64, device=mesh.device) for _ in range(5)]
    g_raw = A.swe_grads(*[_ptr(o) for o in outs])

    def raw_once():   # the C call alone on prepared device arrays; it synchronises (loss out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A.swe_adjoint(mesh.handle, mesh.dev, sa.params, sa.state, steps, _ptr(calib.dt),
                      calib.loss, calib.ckpt_every, g_raw, _ptr(calib.ws), calib.ws.numel(),
                      _stream_handle(None))
        return time.perf_counter() - t0

    autograd_once()
    raw_once()
    t_auto = min(autograd_once() for _ in range(3))
    t_raw = min(raw_once() for _ in range(3))
    res[ex["ckpt_every"]]["autograd_s"] = t_auto
    res[ex["ckpt_every"]]["autograd_over_swe_adjoint"] = t_auto / t_raw
    del calib, ins, sa, outs
    torch.cuda.empty_cache()
    k0 = ex["ckpt_every"]
    record = res[1]
    record["gradients_bitwise_equal_to_checkpointed"] = bool(
        record["loss"] == res[k0]["loss"] and
        all(torch.equal(a, b) for a, b in zip(grads[1], grads[k0])))
    return {"n_cells": mesh.n_cells, "steps": steps, "forward_s": t_fwd, **res[k0],
            "record_every_step": record,
            "timing": "best of 3 after one warm-up, HIP events on the stream. forward_s: swe_run "
                      "of the steps with the replayed dt. adjoint_s: the whole swe_adjoint call; "
                      "its forward pass (checkpoints, or every state) and its reverse sweep "
                      "(segment recompute, if any, and adjoint steps) from swe_adjoint_timings. "
                      "autograd_s: AdjointLoss.apply and backward on device tensors, host wall "
                      "clock between synchronisations, against the swe_adjoint call alone"}


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """Plain device copy: achieved GB/s (read + write) as a measured ceiling for context."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), and how many logical CPUs it lists."""
    names, n = [], 0
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    n += 1
                    nm = ln.split(":", 1)[1].strip()
                    if nm not in names:
                        names.append(nm)
    except OSError:
        return "unknown"
    return f"{' / '.join(names) or 'unknown'} ({n} logical CPUs listed)"


def cpu_baseline(case, budget_s=12.0, single_budget_s=8.0, config_ks=()):
    """The oracle, as it is, on this host: a bounded number of steps of the same workload, on
    all its OpenMP threads (`value`) and on one thread (`single_thread`, the paper's one-core
    reference point); and the configurations `config_ks` run in full (`configs`)."""
    import gen
    import oracle
    t0 = time.perf_counter()
    mesh = oracle.Mesh(case.xy, case.tri, case.edge_tag)
    build_s = time.perf_counter() - t0

    def timed(budget, max_steps):
        t0 = time.perf_counter()
        rc, *_ = oracle.run_case(case, steps=1, mesh=mesh)
        one = time.perf_counter() - t0
        steps = int(max(1, min(max_steps, budget / max(one, 1e-3))))
        t0 = time.perf_counter()
        rc, *_ = oracle.run_case(case, steps=steps, mesh=mesh)
        el = time.perf_counter() - t0
        assert rc == 0, rc
        return steps, el

    nth = oracle.threads()
    steps, el = timed(budget_s, 50)
    oracle.set_threads(1)
    try:
        steps1, el1 = timed(single_budget_s, 20)
    finally:
        oracle.set_threads(nth)
    configs = {}
    for k in config_ks:   # the small configurations in full, beside the GPU's
        c = gen.config(k)
        om = oracle.Mesh(c.xy, c.tri, c.edge_tag)
        t0 = time.perf_counter()
        rc, *_ = oracle.run_case(c, mesh=om)
        ek = time.perf_counter() - t0
        assert rc == 0, rc
        configs[f"config{k}"] = {"value": c.n_cells * c.steps / ek, "cores": nth,
                                 "sample": f"{c.n_cells} cells, all {c.steps} steps ({ek:.1f} s)"}
    return {"value": case.n_cells * steps / el, "unit": "cell-updates/s", "cores": nth,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{case.n_cells} cells, {steps} steps from the initial state "
                      f"({el:.1f} s on {nth} OpenMP threads; mesh build {build_s:.1f} s untimed)",
            "single_thread": {"value": case.n_cells * steps1 / el1, "cores": 1,
                              "sample": f"{steps1} steps ({el1:.1f} s)"},
            "configs": configs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", default="full", choices=["full", "small"],
                    help="small: the same recipe at 1e5 cells (quick checks)")
    ap.add_argument("--dtypes", default="f64,f32")
    ap.add_argument("--tiles", default="64,128,256,512",
                    help="tile sizes the autotuner compares (one mesh each)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ensemble-steps", type=int, default=2000,
                    help="steps of the 256-scenario ensemble (0: skip it)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the FP64 run with correctly rounded division and square root")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 10,000- and 1,000,000-cell configurations")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the 250,000-cell adjoint timing (0: skip it)")
    ap.add_argument("--probe", choices=["copy"], default=None,
                    help="copy: run only a plain 2 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import torch

    import gen
    import paper_1807_00672_amd as swe
    swe.require_gpu()

    if args.probe == "copy":
        gbps = copy_bandwidth()
        # two more kernels of known traffic for the counter calibration: a read-only sum and a
        # write-only fill of the same 2 GiB
        a = torch.ones((2 << 30) // 8, dtype=torch.float64, device="cuda")
        total = float(a.sum())
        a.fill_(2.0)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_per_copy": 2 << 30, "GBps": gbps,
                          "sum_of_ones": total}), flush=True)
        return

    t_gen = time.perf_counter()
    case = gen.config(3) if args.size == "full" else gen.water_drop(nx=250, ny=200,
                                                                    lx=2000.0, ly=1600.0)
    t_gen = time.perf_counter() - t_gen
    t_mesh = time.perf_counter()
    meshes = {swe.SWE_TILE: swe.Mesh(case.xy, case.tri, morton=True)}
    t_mesh = time.perf_counter() - t_mesh
    print(f"# {case.name}: {case.n_cells} cells, {case.n_nodes} nodes; generate {t_gen:.1f} s, "
          f"mesh build {t_mesh:.1f} s", file=sys.stderr, flush=True)
    tiles = tuple(int(x) for x in args.tiles.split(","))

    def mesh_of(tile):
        if tile not in meshes:
            meshes[tile] = swe.Mesh(case.xy, case.tri, morton=True, tile=tile)
        return meshes[tile]

    stream = torch.cuda.Stream()
    results = {}
    tuning = {}
    runs = [(dt, dt, False) for dt in args.dtypes.split(",")]
    if "f64" in args.dtypes.split(",") and not args.no_exact:
        runs.append(("f64_exact", "f64", True))   # correctly rounded FP64 division and sqrt
    for key, dt, exact in runs:
        if dt not in tuning:
            # the autotuner picks the tile size (one mesh per size), then the step variant and
            # workgroup order that SWE_AUTO runs on it
            best, per_tile = swe.tune.tune_tiles(case.xy, case.tri, case.z, case.n, case.h,
                                                 case.hu, case.hv, dtype=dt, steps=20,
                                                 tiles=tiles)
            tuning[dt] = {"tile": best, **per_tile[best],
                          "ms_per_step_by_tile": {
                              str(t): min(v for v in r["ms_per_step"].values() if v > 0)
                              for t, r in per_tile.items()},
                          "by_tile": {str(t): r for t, r in per_tile.items()}}
            print(f"# tuned {dt}: tile {best}; best ms/step by tile "
                  f"{tuning[dt]['ms_per_step_by_tile']}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        mesh = mesh_of(tuning[dt]["tile"])
        solver = swe.Solver(mesh, case.z, case.n, case.h, case.hu, case.hv, dtype=dt,
                            exact=exact)
        ms, rc, st, warm, windows = time_gpu(solver, args.steps, args.warmup, stream)
        if rc != swe.SWE_OK or st["steps"] != warm + 5 * args.steps:
            raise RuntimeError(f"{key}: run failed rc={rc} stats={st}")
        word = 8 if dt == "f64" else 4
        per_step_s = ms * 1e-3 / args.steps
        alg = algorithmic_bytes(case.n_cells, case.n_nodes, word)
        kernel = KERNELS[tuning[dt]["variant"]]
        results[key] = {
            "value": case.n_cells * args.steps / (ms * 1e-3),
            "ms_per_step": ms / args.steps,
            "window_ms_per_step": [w / args.steps for w in windows],
            "warmup_steps_run": warm,
            "alg_bytes_per_step": alg,
            "achieved_GBps": alg / per_step_s / 1e9,
            "kernel": kernel,
            "math": "correctly rounded" if exact else ("newton" if dt == "f64" else "hardware"),
            "traffic": (load_counter(key, case.n_cells) if kernel == PROFILED_KERNEL else None),
            "valu_insts_per_launch": (load_counter(key, case.n_cells, "valu_insts_per_launch")
                                      if kernel == PROFILED_KERNEL else None),
            "t_end_state": st["t"],
        }
        print(f"# {key}: {ms / args.steps:.4f} ms/step, {results[key]['value'] / 1e9:.2f} G "
              f"cell-updates/s, {results[key]['achieved_GBps']:.0f} GB/s algorithmic",
              file=sys.stderr, flush=True)
        del solver
        torch.cuda.empty_cache()

    ensemble = {}
    if args.ensemble_steps > 0 and args.size == "full":
        for dt in args.dtypes.split(","):
            ensemble[dt] = bench_ensemble(dt, args.ensemble_steps, 16, stream)
            e = ensemble[dt]
            print(f"# ensemble {dt}: {e['n_cells']} cells in {e['scenarios']} scenarios, batched "
                  f"{e['batched_cell_updates_per_s'] / 1e9:.2f} G/s vs separate "
                  f"{e['separate_cell_updates_per_s'] / 1e9:.2f} G/s (x{e['speedup']:.2f}), "
                  f"bitwise equal {e['bitwise_equal_to_separate']}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()

    shards = {}
    if args.size == "full" and not args.no_configs:
        shards = bench_shards(mesh_of(tuning.get("f64", {}).get("tile", swe.SWE_TILE)), case,
                              stream)
        print(f"# shard {shards['shard']} of {shards['parts']}: {shards['n_owned']} owned + "
              f"{shards['n_halo']} halo cells, {shards['shard_ms_per_step']:.4f} ms/step alone; "
              f"all shards in turn {shards['all_shards_on_one_gpu_ms_per_step']:.4f} ms/step, "
              f"exchange {shards['exchange_us_per_step']:.0f} us/step",
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    configs = {}
    if args.size == "full" and not args.no_configs:
        configs = bench_configs(stream, args.dtypes.split(","), tiles)
        for k, v in configs.items():
            print(f"# {k}: {v['n_cells']} cells x {v['steps']} steps: " +
                  ", ".join(f"{dt} {v[dt]['cell_updates_per_s'] / 1e9:.2f} G/s (tile {v[dt]['tile']})"
                            for dt in args.dtypes.split(",")), file=sys.stderr, flush=True)

    adjoint = {}
    if args.adjoint_steps > 0 and args.size == "full":
        adjoint = bench_adjoint(stream, args.adjoint_steps)
        rec = adjoint["record_every_step"]
        print(f"# adjoint: {adjoint['n_cells']} cells, {adjoint['steps']} steps: forward "
              f"{adjoint['forward_s']:.3f} s, adjoint {adjoint['adjoint_s']:.3f} s "
              f"(x{adjoint['adjoint_over_forward']:.2f}; reverse sweep "
              f"x{adjoint['reverse_over_forward']:.2f}); every step stored "
              f"({rec['workspace_GB']:.1f} GB): {rec['adjoint_s']:.3f} s "
              f"(x{rec['adjoint_over_forward']:.2f}; reverse sweep x{rec['reverse_over_forward']:.2f}), "
              f"gradients bitwise equal {rec['gradients_bitwise_equal_to_checkpointed']}; "
              f"through AdjointLoss x{adjoint['autograd_over_swe_adjoint']:.3f} of swe_adjoint",
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    copy_gbps = copy_bandwidth()
    main_dt = "f64" if "f64" in results else next(iter(results))   # default FP64 arithmetic
    r = results[main_dt]
    line = {
        "metric": "cell-updates/s at 10M triangles (FP64 step; FP32 under variants)",
        "value": r["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_dt,
        "data": "synthetic",
        "config": {"workload": f"water drop, {case.n_cells} triangles, jittered split-square "
                               f"mesh 10 km x 5 km, Morton order, walls",
                   "n_cells": case.n_cells, "n_nodes": case.n_nodes, "parallelism": "none"},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": r["achieved_GBps"] / HBM_PEAK_GBPS,
                     "traffic": r["traffic"], "kernel": r["kernel"],
                     "timed": "whole step (step kernel + dt fold kernel) per step",
                     "alg_bytes_per_launch": r["alg_bytes_per_step"],
                     "copy_GBps_measured": copy_gbps,
                     "frac_of_measured_copy": r["achieved_GBps"] / copy_gbps,
                     "alu": alu_view(r)},
        "variants": {k: {kk: vv for kk, vv in v.items() if kk != "t_end_state"}
                     for k, v in results.items()},
        "tuning": tuning,
        "configs": configs,
        "shards": shards,
        "ensemble": ensemble,
        "adjoint": adjoint,
        "copy_GBps_measured": copy_gbps,
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(
            case, config_ks=(1, 2) if args.size == "full" and not args.no_configs else ())
        for k, v in line["cpu_baseline"]["configs"].items():
            print(f"# oracle {k}: {v['value'] / 1e6:.0f} M cell-updates/s ({v['sample']})",
                  file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
