#!/usr/bin/env python3
"""Throughput benchmark of the fused fluctuating two-species D2Q9 step.

One "step" advances every replica of the workload by one lattice-Boltzmann
time step (collision with forcing and noise, streaming, walls) with the
structure-factor and pressure sampling fused in at its configured cadence.

Default workload (N = 1): the batched ensemble of 96 replicas with L in
{32, 64, 128, 256}, Lx = 2L, FP32-deviation storage, sampled every 10 steps.
Printed as one JSON line:
  value        MLUPS over the whole batch (one update = both species at one node)
  value_without_sampling
               the same batch with sampling off
  roofline     the step kernel alone (sampling off): algorithmic bytes per
               launch (18 reads + 18 writes per node and step, times the steps
               one launch advances) / measured launch time; measured HBM bytes
               per launch from the committed counter record (ensemble only,
               while the kernel and its sources match it); a plain device-copy
               ceiling measured in the same run
  compare      plain FP64 storage on the same batch and on the single 512 x 256
               lattice, and the agreement of the two storage forms
  adjoint      one gradient of the S(q) misfit on 256 x 128 (FP64, 2000 steps)
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published peak


def _events_time(lat, nsteps):
    """Elapsed ms of nsteps steps between two HIP events on the library's stream."""
    import torch
    s = lat.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lat.step(nsteps)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1)


def copy_ceiling_gbs(mib: int = 1024, reps: int = 20) -> float:
    """Read + write bandwidth of a plain device-to-device copy of `mib` MiB
    (torch's copy kernel), timed with HIP events: the practical streaming
    ceiling of the box, beside the published peak."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    del src, dst
    return 2 * n * 4 * reps / sec / 1e9


def storage_agreement(F, reps, every: int, steps: int = 200) -> dict:
    """The same replicas (same seeds) advanced `steps` steps with FP32-deviation
    and with FP64 storage: largest relative differences over all replicas of
    S(q) of both fields (|dS(q)| against mean S + |<Phi(q)>|^2), of the time
    sums of the mean pressure and its row profile (against the largest row
    mean), and of the populations' deviations from the rest state."""
    import numpy as np
    a = F.Lattice(reps, precision=F.FP32_DEV, sample_every=every)
    b = F.Lattice(reps, precision=F.FP64, sample_every=every)
    a.step(steps)
    b.step(steps)
    dS = dP = 0.0
    for i in range(len(reps)):
        for fld in range(2):
            a2, re, im, n = a.read_structure_factor(i, fld)
            b2, bre, bim, _ = b.read_structure_factor(i, fld)
            Sa = a2 / n - (re / n) ** 2 - (im / n) ** 2
            Sb = b2 / n - (bre / n) ** 2 - (bim / n) ** 2
            m2 = (bre / n) ** 2 + (bim / n) ** 2
            dS = max(dS, float((np.abs(Sa - Sb) / (np.abs(Sb).mean() + m2)).max()))
        pa, _, proa, _ = a.read_pressure(i)
        pb, _, prob, _ = b.read_pressure(i)
        scale = max(np.abs(prob).max(), 1e-300)
        dP = max(dP, abs(pa - pb) / scale, float(np.abs(proa - prob).max() / scale))
    # populations: a few replicas of each size (the read-back is host work)
    df = 0.0
    for i in range(0, len(reps), max(1, len(reps) // 8)):
        fa, fb = a.read_populations(i), b.read_populations(i)
        rest = F.Lattice([reps[i]], precision=F.FP64)
        f0 = rest.read_populations(0)
        df = max(df, float(np.abs(fa - fb).max() / np.abs(fb - f0).max()))
        rest.close()
    a.close()
    b.close()
    return {"steps": steps, "S_rel": float(f"{dS:.3g}"), "P_rel": float(f"{dP:.3g}"),
            "populations_rel": float(f"{df:.3g}")}


def equal_error(F, reps, every: int, warm: int = 500, n_blocks: int = 10,
                block_samples: int = 20) -> dict:
    """The survey's "equal S(q) error" check on the benchmark's own replicas.
    Both storage forms run the same replicas with the same seeds (the same
    noise).  After `warm` steps the accumulators are cleared; then
    `n_blocks` blocks of `block_samples` samples each are summed separately.
    From the FP64 blocks, eps_S is the relative standard error of the block
    means of S_c(q_x, 0) (k_z = 0), averaged over the band k_x >= 1 of every
    replica.  The FP32-deviation result over the same blocks must differ from
    the FP64 one by much less: `max_rel_diff` is the largest
    |S32 - S64| / S64 over that band (block means), `ratio` = that / eps_S,
    and the bar is 0.1."""
    import numpy as np
    lats = {p: F.Lattice(reps, precision=p, sample_every=every) for p in (F.FP64, F.FP32_DEV)}
    blocks = {p: [] for p in lats}
    for p, lat in lats.items():
        lat.step(warm)
        lat.reset_accumulators()
        for _ in range(n_blocks):
            lat.step(block_samples * every)
            row = []
            for i in range(len(reps)):
                a2, re, im, n = lat.read_structure_factor(i, F.FIELD_C)
                S = a2 / n - (re / n) ** 2 - (im / n) ** 2
                row.append(S[0, 1:].copy())
            blocks[p].append(row)
            lat.reset_accumulators()
        lat.close()
    rel_se, diff = [], []
    for i in range(len(reps)):
        b64 = np.array([blk[i] for blk in blocks[F.FP64]])      # [block][k_x]
        b32 = np.array([blk[i] for blk in blocks[F.FP32_DEV]])
        m64 = b64.mean(axis=0)
        se = b64.std(axis=0, ddof=1) / np.sqrt(n_blocks)
        rel_se.append(se / m64)
        diff.append(np.abs(b32.mean(axis=0) - m64) / m64)
    eps = float(np.mean(np.concatenate(rel_se)))
    dmax = float(np.max(np.concatenate(diff)))
    return {"eps_S": float(f"{eps:.3g}"), "max_rel_diff": float(f"{dmax:.3g}"),
            "ratio": float(f"{dmax / eps:.3g}"), "bar": 0.1,
            "blocks": n_blocks, "samples_per_block": block_samples, "warm_steps": warm,
            "field": "S_c(q_x, 0), k_x >= 1, every replica"}


def adjoint_leg(F, W, reps_done: int = 3) -> dict:
    """Time of one gradient of the structure-factor misfit by the adjoint
    (256 x 128 FP64, horizon 2000 sampled every 10, checkpoints every 100),
    against the forward run of the same horizon.  The target spectrum comes
    from a GPU twin run at (tau_s, tau_d, G) x (1.05, 0.95, 1.1)."""
    import dataclasses
    import numpy as np
    import torch
    rep, H, every, K = W.adjoint_256x128(), 2000, 10, 100
    twin = dataclasses.replace(rep, tau_s=rep.tau_s * 1.05, tau_d=rep.tau_d * 0.95,
                               G=rep.G * 1.1)
    lt = F.Lattice([twin], precision=F.FP64, sample_every=every)
    lt.step(H)
    S_t = lt.structure_factor(0, F.FIELD_C)
    del lt
    w = np.ones_like(S_t)
    w[:, 0] = 0.0
    lat = F.Lattice([rep], precision=F.FP64, sample_every=every)
    lat.sq_misfit_gradient(S_t, w, H, ckpt_every=K)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps_done):
        J, g = lat.sq_misfit_gradient(S_t, w, H, ckpt_every=K)
    t_grad = (time.perf_counter() - t0) / reps_done
    fwd = F.Lattice([rep], precision=F.FP64, sample_every=every)
    fwd.step(H)
    ms_fwd = _events_time(fwd, H)
    return {"workload": "adjoint 256x128 fp64, horizon 2000, sample every 10, checkpoint every 100",
            "ms_per_gradient": round(t_grad * 1e3, 2), "forward_ms": round(ms_fwd, 2),
            "gradient_over_forward": round(t_grad * 1e3 / ms_fwd, 2),
            "grad": [float(x) for x in g], "J": float(J)}


# the sources each step kernel is compiled from
_STEP_HEADERS = ("fnlb_node.hpp", "fnlb_device.hpp", "fnlb_internal.hpp", "fnlb_state.hpp")
STEP_SOURCES = {"k_step": ("k_step.hip",) + _STEP_HEADERS,
                "k_step2": ("k_step2.hip",) + _STEP_HEADERS}
# SQ counters of the one --pmc pass behind profiles/counters_batched96_fp32dev.md
PMC_SET = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
           "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_step_batched96_fp32dev.json")
# the step kernels as rocprofv3 names them: (plain, sampling) variants and the
# steps one launch advances
STEP_KERNELS = {"k_step2": ("k_step2<0>", "k_step2<1>", 2),
                "k_step": ("k_step<float, float, 0,", "k_step<float, float, 1,", 1)}


def _step_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for n in STEP_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1808_05168_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic_from_profiles(kernel: str):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, if it was taken on this kernel and the current kernel sources
    (else None)."""
    try:
        with open(TRAFFIC_JSON) as fh:
            d = json.load(fh)
        if d.get("kernel") != kernel or d.get("source_sha256") != _step_source_hash(kernel):
            return None
        return d["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def summarize_trace(trace_dir, out_md, title, command, top=16):
    """Kernel-trace statistics of a rocprofv3 run as a short Markdown summary."""
    import csv
    stats = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    lines = [f"# {title}", "", "Command (run from the repository root; <out> is any output "
             "directory):", "", "```", command.strip(), "```", "",
             "| kernel | calls | average us | share % |", "|---|---|---|---|"]
    for r in stats[:top]:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_timeline(trace_dir, out_md, title, command):
    """Where a sample's time goes in graph replays, from the start and end
    timestamps and queue ids of a rocprofv3 kernel trace (no --stats needed):
    per sample, the sampling launch over a plain one, the idle time between
    the step launches before and after it, what the row pass and the column
    pass add to the plain launches they run beside, and the sum, against the
    measured time between sampling launches."""
    import csv
    rows = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))

    def kind(name):
        for k, tag in (("k_step2<1>", "S"), ("k_step2<0>", "P"), ("k_row_fft", "R"),
                       ("k_col_fft", "C"), ("k_advance_time", "A")):
            if k in name:
                return tag
        return None

    ev = [(kind(r["Kernel_Name"]), int(r["Queue_Id"]), int(r["Start_Timestamp"]) / 1e3,
           int(r["End_Timestamp"]) / 1e3) for r in rows]
    ev = [e for e in ev if e[0]]
    first_s = next(i for i, e in enumerate(ev) if e[0] == "S")
    ev = ev[first_s:]
    # the step launches (and the time-counter node at a graph's end) form one
    # chain, whatever queues they run on
    chain = [e for e in ev if e[0] in "SPA"]
    passes = [e for e in ev if e[0] in "RC"]

    def overlaps(a, b):
        return a[2] < b[3] and b[2] < a[3]

    def mean(v):
        return sum(v) / len(v) if v else float("nan")

    alone = [e[3] - e[2] for e in chain if e[0] == "P" and
             not any(overlaps(p, e) for p in passes)]
    plain = mean(alone)
    gap_before, gap_after, s_extra, periods = [], [], [], []
    s_idx = [i for i, e in enumerate(chain) if e[0] == "S"]
    for i in s_idx:
        e = chain[i]
        if i == 0 or i + 1 >= len(chain) or chain[i - 1][0] == "A":
            continue  # samples inside a replay only (not at a graph's first node)
        gap_before.append(e[2] - chain[i - 1][3])
        gap_after.append(chain[i + 1][2] - e[3])
        s_extra.append(e[3] - e[2] - plain)
    cols = [p for p in passes if p[0] == "C"]
    for a, b in zip(s_idx, s_idx[1:]):
        span = (None, None, chain[a][2], chain[b][2])
        if not any(chain[k][0] == "A" for k in range(a, b)) and \
                not any(overlaps(c, span) for c in cols):
            periods.append((chain[b][2] - chain[a][2], b - a))
    n_r = sum(e[0] == "R" for e in ev)
    beside_r = [e[3] - e[2] - plain for e in chain if e[0] == "P" and
                any(p[0] == "R" and overlaps(p, e) for p in passes) and
                not any(p[0] == "C" and overlaps(p, e) for p in passes)]
    beside_c = [e[3] - e[2] - plain for e in chain if e[0] == "P" and
                any(p[0] == "C" and overlaps(p, e) for p in passes)]
    col_per_sample = sum(beside_c) / n_r if n_r else float("nan")
    per_sample = (mean(s_extra) + mean(gap_before) + mean(gap_after) + mean(beside_r) +
                  col_per_sample)
    launches = mean([n for _, n in periods])
    period_extra = mean([t for t, _ in periods]) - launches * plain
    queues = {k: sorted(set(e[1] for e in ev if e[0] == k)) for k in "SPRC"}
    lines = [f"# {title}", "", "Command (run from the repository root; <out> is any output "
             "directory):", "", "```", command.strip(), "```", "",
             "Launches from the first sampling launch on. Hardware queues: " +
             ", ".join(f"{n} {queues[k]}" for k, n in
                       (("S", "sampling launches"), ("P", "plain launches"),
                        ("R", "row passes"), ("C", "column passes"))) + ".", "",
             f"A plain launch with nothing beside it: {plain:.1f} us ({len(alone)} launches).",
             "", "| per sample | us | from |", "|---|---|---|",
             f"| sampling launch over a plain one | {mean(s_extra):.1f} | {len(s_extra)} "
             "sampling launches inside replays |",
             f"| idle before the sampling launch | {mean(gap_before):.1f} | the same |",
             f"| idle after the sampling launch | {mean(gap_after):.1f} | the same |",
             f"| row pass: what the plain launch beside it takes over a plain one | "
             f"{mean(beside_r):.1f} | {len(beside_r)} launches (row passes average "
             f"{mean([e[3] - e[2] for e in ev if e[0] == 'R']):.1f} us) |",
             f"| column pass: what the plain launches beside it take over plain ones, per "
             f"sample | {col_per_sample:.1f} | {len(beside_c)} launches, {n_r} samples |",
             f"| sum | {per_sample:.1f} | |",
             f"| measured: time between sampling launches in a replay over the same number of "
             f"plain launches | {period_extra:.1f} | {len(periods)} periods of {launches:.0f} "
             "launches (no column pass) |"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return dict(plain=plain, sampling_extra=mean(s_extra), gap_before=mean(gap_before),
                gap_after=mean(gap_after), beside_row=mean(beside_r),
                col_per_sample=col_per_sample, per_sample=per_sample,
                period_extra=period_extra)


# steps of the roofline leg before its timed launches (clock ramp, then a probe
# of 20 steps that sizes the timed part)
ROOFLINE_LEAD_STEPS = 120


def summarize_profile(trace_dir, fetch_dir, write_dir, out_md, command):
    """Turns rocprofv3 outputs of this benchmark into the committed summary:
    kernel-trace statistics, the average duration of the step kernel in the
    roofline leg (the plain launches at the timed grid size before the first
    sampling step, less the leg's first ROOFLINE_LEAD_STEPS steps of clock
    ramp and probe; in the sampled run the transforms of a sample overlap the
    plain steps that follow it, and autotuning trials use other grids), and HBM bytes
    per step launch from FETCH_SIZE and WRITE_SIZE scaled by what the same
    counters read for the plain 1 GiB copies that --copy-calibration-mb 1024
    runs first."""
    import csv
    from collections import Counter, defaultdict
    stats = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    rows = sorted(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))),
                  key=lambda r: int(r["Start_Timestamp"]))
    # the step kernel of the run: the two-step kernel if it ran, else the
    # one-step kernel (template arguments: compute type, storage type, mode)
    kernel = "k_step2" if any(STEP_KERNELS["k_step2"][0] in r["Kernel_Name"] for r in rows) \
        else "k_step"
    step_name, sample_name, spl = STEP_KERNELS[kernel]
    trace = [r for r in rows if step_name in r["Kernel_Name"]]
    grid = Counter(r["Grid_Size_X"] for r in trace).most_common(1)[0][0]
    first_sample = min((int(r["Start_Timestamp"]) for r in rows
                        if sample_name in r["Kernel_Name"]), default=1 << 62)
    leg = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace
           if r["Grid_Size_X"] == grid and int(r["Start_Timestamp"]) < first_sample]
    durs = leg[ROOFLINE_LEAD_STEPS // spl:]
    avg_us = sum(durs) / len(durs) / 1e3

    def counters(d, name):
        step, copy = [], []
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            if r["Counter_Name"] != name:
                continue
            if step_name in r["Kernel_Name"] and r["Grid_Size"] == grid:
                step.append(float(r["Counter_Value"]))
            elif "copyBuffer" in r["Kernel_Name"]:
                copy.append(float(r["Counter_Value"]))
        big = [v for v in copy if v >= 0.5 * max(copy)]
        return sum(step) / len(step), sum(big) / len(big), len(step)

    f_step, f_copy, nf = counters(fetch_dir, "FETCH_SIZE")
    w_step, w_copy, nw = counters(write_dir, "WRITE_SIZE")
    copy_kib = 1024 * 1024
    f_scale, w_scale = copy_kib / f_copy, copy_kib / w_copy
    rd = f_step * f_scale * 1024
    wr = w_step * w_scale * 1024
    import workloads as W
    nodes = sum(r.Lx * r.Lz for r in W.batched_ensemble(96))
    alg = 144 * nodes * spl
    title = ("k_step2 (two fused collide-stream steps per pass)" if spl == 2
             else "k_step (fused collide-stream)")
    lines = [f"# {title}, batched 96-replica FP32-deviation workload", "",
             "Commands (run from the repository root; <out> is any output directory):", "",
             "```", command, "```", "",
             "## Kernel trace (rocprofv3 --stats)", "",
             "| kernel | calls | average us | share % |", "|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    lines += ["", "In the sampled run the transforms of each sample run beside the plain steps "
              "that follow it, so the averages above include that overlap.", "",
              f"Step kernel `{kernel}` in the roofline leg ({spl} step(s) per launch; plain "
              f"launches, grid {grid} threads, {len(durs)} dispatches): average "
              f"{avg_us:.1f} us per launch, {avg_us / spl:.1f} us per step.", "",
              "## HBM traffic per step launch", "",
              f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch, {nf} and {nw} step dispatches) "
              f"scaled by the 1 GiB copy: FETCH x{f_scale:.4f}, WRITE x{w_scale:.4f}.", "",
              f"- read {rd/1e6:.1f} MB, write {wr/1e6:.1f} MB, total {(rd+wr)/1e6:.1f} MB",
              f"- algorithmic (144 B/node-step x {nodes} nodes x {spl} step(s)): "
              f"{alg/1e6:.1f} MB",
              f"- ratio {(rd+wr)/alg:.3f}"]
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump({"kernel": kernel, "steps_per_launch": spl,
                   "bytes_per_launch": round(rd + wr), "read_bytes": round(rd),
                   "write_bytes": round(wr), "algorithmic_bytes": alg,
                   "step_avg_us": round(avg_us, 2), "grid": int(grid),
                   "source_sha256": _step_source_hash(kernel), "command": command}, fh, indent=1)
    print("\n".join(lines))


def summarize_counters(pmc_dir, out_md, command):
    """Per-kernel averages of the SQ counters of one rocprofv3 --pmc pass over
    this benchmark, with the derived figures quoted in the design notes:
    VALU instructions per node (wavefront instructions x 64 / nodes), the share
    of wave-resident cycles spent issuing VALU work and waiting, and LDS bank
    conflict cycles per LDS instruction."""
    import csv
    from collections import defaultdict
    import workloads as W
    nodes = sum(r.Lx * r.Lz for r in W.batched_ensemble(96))
    agg = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))):
        name = r["Kernel_Name"].replace("fnlb::(anonymous namespace)::", "")
        name = name.replace("HIP_vector_type<float, 2u>", "float2")
        name = name.replace("HIP_vector_type<double, 2u>", "double2")
        name = name.split("(")[0] if "k_step" not in name else name.split("(fnlb")[0]
        agg[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["# SQ counters, batched 96-replica FP32-deviation workload", "",
             "Command (run from the repository root; <out> is any output directory):", "",
             "```", command.strip(), "```", "",
             "Averages per dispatch of the library's kernels. VALU/node = SQ_INSTS_VALU x 64 "
             "/ 4,177,920 nodes, per step (the two-step kernel's dispatches are divided by "
             "their two steps; a column-pass dispatch adds every sample kept in the "
             "spectrum slots, up to 16). The next two columns are raw ratios of counters to "
             "SQ_WAVE_CYCLES (SQ_ACTIVE_INST_VALU, SQ_WAIT_ANY), summed over the wavefronts "
             "of a dispatch; their cycle units need not match. The last column is "
             "SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS.", "",
             "| kernel | waves | VALU/node | ACTIVE_INST_VALU / WAVE_CYCLES | "
             "WAIT_ANY / WAVE_CYCLES | LDS instr | bank-conflict cycles per LDS instr |",
             "|---|---|---|---|---|---|---|"]
    for name, c in sorted(agg.items()):
        m = {k: sum(v) / len(v) for k, v in c.items()}
        if not any(k in name for k in ("k_step", "transform", "_fft", "pressure")):
            continue
        wc = max(m.get("SQ_WAVE_CYCLES", 1.0), 1.0)
        per = 2 if "k_step2" in name else 1
        lines.append(
            f"| {name} | {m['SQ_WAVES']:.0f} | {m['SQ_INSTS_VALU'] * 64 / nodes / per:.0f} | "
            f"{m['SQ_ACTIVE_INST_VALU'] / wc:.2f} | {m['SQ_WAIT_ANY'] / wc:.2f} | "
            f"{m['SQ_INSTS_LDS']:.3g} | "
            f"{m['SQ_LDS_BANK_CONFLICT'] / max(m['SQ_INSTS_LDS'], 1.0):.2f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def host_threads() -> int:
    """Threads the oracle runs on: OMP_NUM_THREADS where it is set (the host's
    CPU share for one GPU on a shared machine), else every CPU this process may
    run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_rate(O, reps, steps, t0=0, acc=None, every=0):
    """Node updates per second of the oracle over `steps` steps of each replica
    (each from its rest state), and the elapsed seconds."""
    f = [O.init_state(r) for r in reps]
    t = time.perf_counter()
    for r, fr in zip(reps, f):
        O.run(r, fr, t0, steps, acc, sample_every=every)
    dt = time.perf_counter() - t
    return sum(r.Lx * r.Lz for r in reps) * steps / dt, dt


def cpu_baseline(reps, c4_steps: int = 50, steps: int = 200, steps_1thread: int = 20):
    """The oracle as it stands (plain FP64 C++ at -O2, OpenMP over rows), on the
    host's cores and on one thread.

    value: one replica of each lattice size of the benchmark's ensemble, `steps`
    steps each, no sampling (the rate of the timed workload's mix of sizes).
    protocol: the 64 x 32 run end to end (5000 steps sampled every 10) with the
    time of its sampling (the direct Fourier sums) reported apart from the
    rate; 512 x 256 over `steps` steps; 4096 x 1024 over `c4_steps` steps; the
    ensemble sample on one thread over `steps_1thread` steps.  Every figure is a
    measured rate over the stated steps; nothing is extrapolated."""
    import workloads as W
    from oracle import oracle as O
    threads = host_threads()
    O.set_threads(threads)
    seen, sample = set(), []
    for r in reps:
        if (r.Lx, r.Lz) not in seen:
            seen.add((r.Lx, r.Lz))
            sample.append(r)
    rate, dt = _oracle_rate(O, sample, steps)
    proto = {}
    c1 = W.parity_small()
    acc = O.Accum(c1.Lx, c1.Lz)
    r_s, t_s = _oracle_rate(O, [c1], 5000, acc=acc, every=10)
    r_p, t_p = _oracle_rate(O, [c1], 5000)
    proto["c1_64x32_5000_steps"] = {"mlups_sampled": round(r_s / 1e6, 3), "seconds": round(t_s, 2),
                                    "mlups_without_sampling": round(r_p / 1e6, 3),
                                    "sampling_seconds": round(t_s - t_p, 2),
                                    "samples": acc.n_samples}
    r2, t2 = _oracle_rate(O, [W.single_512x256()], steps)
    proto["c2_512x256"] = {"mlups": round(r2 / 1e6, 3), "steps": steps, "seconds": round(t2, 2)}
    r4, t4 = _oracle_rate(O, [W.large_4096x1024()], c4_steps)
    proto["c4_4096x1024"] = {"mlups": round(r4 / 1e6, 3), "steps": c4_steps,
                             "seconds": round(t4, 2)}
    O.set_threads(1)
    r1, t1 = _oracle_rate(O, sample, steps_1thread)
    O.set_threads(threads)
    proto["ensemble_sample_1thread"] = {"mlups": round(r1 / 1e6, 3), "steps": steps_1thread,
                                        "seconds": round(t1, 2)}
    return {"value": round(rate / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "value_1thread": round(r1 / 1e6, 3),
            "host_cpus_visible": os.cpu_count(),
            "sample": f"{len(sample)} replicas (one per size of the ensemble: "
                      + ", ".join(f"{r.Lx}x{r.Lz}" for r in sample)
                      + f"), {steps} steps each from rest, FP64, no sampling, {dt:.1f} s on "
                      f"{threads} threads",
            "protocol": proto}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="batched96",
                    choices=["batched96", "large4096x1024", "single512x256"])
    ap.add_argument("--cpu-c4-steps", type=int, default=50,
                    help="steps of the 4096 x 1024 oracle run in cpu_baseline.protocol")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg (for its kernel trace)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device copy of this size (3 times), the "
                         "reference for scaling HBM byte counters")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step directly instead of replaying the captured "
                         "sampling period (a kernel trace then times the transforms of a "
                         "sample without the steps running beside them)")
    ap.add_argument("--tune-cache", default="",
                    help="tuning file: load the stored choices first, save them after "
                         "tuning; the line reports whether the new pick reproduces the "
                         "stored one")
    ap.add_argument("--kernel", choices=["auto", "one", "two"], default="auto",
                    help="step kernel: one or two steps per launch (auto: the autotuner's "
                         "choice)")
    ap.add_argument("--chunk-rows", type=int, default=0,
                    help="fixed rows per work item (skips the autotuner); profiles use it "
                         "so that every pass times the same launch configuration")
    ap.add_argument("--summarize-profile", nargs=3, metavar=("TRACE", "FETCH", "WRITE"),
                    help="summarise rocprofv3 output directories into profiles/ (CPU only)")
    ap.add_argument("--profile-command", default="")
    ap.add_argument("--summarize-counters", metavar="PMC_DIR",
                    help="write profiles/counters_batched96_fp32dev.md from a --pmc pass "
                         "with the counters of PMC_SET")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE", "NAME", "TITLE"),
                    help="summarise a rocprofv3 kernel trace into profiles/NAME.md (CPU only)")
    ap.add_argument("--summarize-timeline", metavar="TRACE",
                    help="write profiles/sample_timeline_batched96_fp32dev.md from a "
                         "rocprofv3 kernel trace of graph replays (CPU only)")
    args = ap.parse_args()

    if args.summarize_timeline:
        d = args.summarize_timeline
        summarize_timeline(
            d, os.path.join(ROOT, "profiles", "sample_timeline_batched96_fp32dev.md"),
            "A sample in graph replays, batched 96-replica FP32-deviation workload, "
            "two-step kernel",
            "rocprofv3 --kernel-trace --output-format csv -d <out>/tl -o run -- python3 "
            "bench.py --steps 2000 --warmup 20 --no-cpu-baseline --no-compare --no-adjoint "
            "--kernel two --chunk-rows 32\n"
            "python3 bench.py --summarize-timeline <out>/tl")
        return

    if args.summarize_counters:
        d = args.summarize_counters
        summarize_counters(d, os.path.join(ROOT, "profiles", "counters_batched96_fp32dev.md"),
                           f"rocprofv3 --pmc {' '.join(PMC_SET)} --output-format csv -d <out>/pc "
                           f"-o run -- python3 bench.py --steps 20 --warmup 2 --no-cpu-baseline "
                           f"--no-compare --no-adjoint --kernel two --chunk-rows 32\n"
                           f"python3 bench.py --summarize-counters <out>/pc")
        return
    if args.summarize_trace:
        d, name, title = args.summarize_trace
        # the run each committed trace summary is taken from
        runs = {"sample_passes_batched96_fp32dev":
                ("ps", "--steps 300 --warmup 20 --no-cpu-baseline --no-compare --no-adjoint "
                       "--kernel two --chunk-rows 32 --no-graph")}
        sub, run_args = runs.get(name, ("pa", "--adjoint-only"))
        cmd = args.profile_command or (
            f"rocprofv3 --kernel-trace --stats --output-format csv -d <out>/{sub} -o run -- "
            f"python3 bench.py {run_args}\n"
            f"python3 bench.py --summarize-trace <out>/{sub} {name} \"{title}\"")
        summarize_trace(d, os.path.join(ROOT, "profiles", name + ".md"), title, cmd)
        return

    if args.summarize_profile:
        out = os.path.join(ROOT, "profiles", "step_batched96_fp32dev.md")
        leg = "--no-cpu-baseline --no-compare --no-adjoint --kernel two --chunk-rows 32"
        cmd = args.profile_command or "\n".join([
            "rocprofv3 --kernel-trace --stats --output-format csv -d <out>/pt -o run -- "
            f"python3 bench.py --steps 200 --warmup 20 {leg}",
            "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/pf -o run -- "
            f"python3 bench.py --steps 10 --warmup 2 {leg} --copy-calibration-mb 1024",
            "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/pw -o run -- "
            f"python3 bench.py --steps 10 --warmup 2 {leg} --copy-calibration-mb 1024",
            "python3 bench.py --summarize-profile <out>/pt <out>/pf <out>/pw"])
        summarize_profile(*args.summarize_profile, out, cmd)
        return

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(replicas, and z-slabs of a single lattice, would shard across GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1808_05168_amd as F
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(F, W)}), flush=True)
        return

    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    every = 10
    if args.workload == "batched96":
        reps, prec = W.batched_ensemble(96), F.FP32_DEV
        desc = "96 replicas, L = 32*2^(i%4), Lx = 2L, G in {0, 0.5}, grad_c0 in [0, 1e-3]"
    elif args.workload == "large4096x1024":
        reps, prec, every = [W.large_4096x1024()], F.FP32_DEV, 50
        desc = "single 4096 x 1024 lattice, G = 0.5, grad_c0 = 5e-4"
    else:
        reps, prec = [W.single_512x256()], F.FP64
        desc = "single 512 x 256 lattice, G = 0.5, grad_c0 = 1e-3"
    nodes = sum(r.Lx * r.Lz for r in reps)
    store_bytes = 4 if prec == F.FP32_DEV else 8
    bytes_per_node = 36 * store_bytes

    flags = F.DEFAULT_FLAGS | (F.NO_GRAPH if args.no_graph else 0)
    flags |= {"auto": 0, "one": F.ONE_STEP, "two": F.TWO_STEP}[args.kernel]
    if args.tune_cache and os.path.exists(args.tune_cache):
        F.tune_cache_load(args.tune_cache)
    stored = F.tune_lookup(reps, prec)
    lat = F.Lattice(reps, precision=prec, sample_every=every, flags=flags,
                    chunk_rows=args.chunk_rows)
    tuned = args.chunk_rows <= 0 and not args.no_autotune
    if tuned:
        lat.autotune(50)
        if args.tune_cache:
            F.tune_cache_save(args.tune_cache)
    # the launch configuration the timed steps use (kernel and row ranges)
    spl, chunk = lat.launch_config()
    tuning = {"autotuned": tuned, "stored": list(stored) if stored else None,
              "reproduces_stored": (tuple(stored) == (spl, chunk)) if (stored and tuned)
              else None}
    # roofline leg: the step kernel alone (no sampling), same batch and launch
    # configuration; one launch advances spl steps, so its algorithmic bytes
    # are spl x 144 B (FP32) per node.  It runs first, for about 0.3 s: the
    # GPU lowers its clocks within milliseconds of idling and takes about
    # 0.2 s of load to raise them again, so the timed steps that follow it
    # (after their own warm-up steps) see the clocks a long run sees.
    kflag = F.TWO_STEP if spl == 2 else F.ONE_STEP
    lat_r = F.Lattice(reps, precision=prec, sample_every=0,
                      flags=(flags & ~(F.ONE_STEP | F.TWO_STEP)) | kflag, chunk_rows=chunk)
    assert lat_r.launch_config() == (spl, chunk)
    lat_r.step(ROOFLINE_LEAD_STEPS - 20)
    ms_probe = _events_time(lat_r, 20)
    nr = max(50, int(300.0 / max(ms_probe / 20, 1e-3)))
    nr += nr % spl
    ms_r = _events_time(lat_r, nr)
    t_step = ms_r / 1e3 / nr
    t_launch = t_step * spl
    alg_launch = bytes_per_node * nodes * spl
    achieved = alg_launch / t_launch / 1e9
    kernel = "k_step2" if spl == 2 else "k_step"

    # the clock starts where the W warm-up steps end on a sampling-period
    # boundary, so that the K timed steps replay whole captured periods, as a
    # long run does, however short K is (the time only keys the noise and the
    # sampling schedule: same steps, same samples per step)
    t_start = (-args.warmup) % every
    if t_start + args.warmup == 0:
        t_start = every
    lat.time = t_start
    lat.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = _events_time(lat, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sec = ms / 1e3
    mlups = nodes * args.steps / sec / 1e6
    del lat_r       # freed after the timed steps: its teardown would idle the GPU

    # the counter record is of the ensemble's step kernel
    traffic = _traffic_from_profiles(kernel) if args.workload == "batched96" else None
    copy_gbs = copy_ceiling_gbs()

    out = {
        "metric": "MLUPS (both species)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == F.FP32_DEV else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "nodes": nodes,
                   "storage": "fp32-deviation" if prec == F.FP32_DEV else "fp64",
                   "sample_every": every, "kernel": kernel, "steps_per_launch": spl,
                   "chunk_rows": chunk, "tuning": tuning, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": ("k_step2 (two fused collide-stream steps per pass)" if spl == 2
                                else "k_step (fused collide-stream)"),
                     "steps_per_launch": spl,
                     "launch_ms": round(t_launch * 1e3, 5),
                     "algorithmic_bytes_per_launch": alg_launch,
                     "copy_ceiling_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "wall_s": round(wall, 3),
        # the same batch with sampling off (the roofline leg)
        "value_without_sampling": round(nodes / t_step / 1e6, 1),
    }

    if not args.no_compare and prec == F.FP32_DEV:
        # the same workload with plain FP64 storage, and the FP64 single lattice
        out["compare"] = {}
        for name, creps in (("fp64_same_workload_mlups", reps),
                            ("fp64_single_512x256_mlups", [W.single_512x256()])):
            lat64 = F.Lattice(creps, precision=F.FP64, sample_every=every)
            if not args.no_autotune:
                lat64.autotune(20)
            lat64.step(args.warmup)
            n64 = args.steps
            ms64 = _events_time(lat64, n64)
            n_nodes = sum(r.Lx * r.Lz for r in creps)
            out["compare"][name] = round(n_nodes * n64 / (ms64 / 1e3) / 1e6, 1)
            del lat64
        out["compare"]["fp32_vs_fp64_storage"] = storage_agreement(F, reps, every)
        out["compare"]["equal_error"] = equal_error(F, reps, every)
        out["compare"]["speedup_vs_fp64_single_512x256"] = round(
            out["value"] / out["compare"]["fp64_single_512x256_mlups"], 2)
        out["compare"]["note"] = (f"plain FP64 storage, sampled every {every} steps; both "
                                  "storage forms give S(q) within 1e-5 of the FP64 oracle "
                                  "(parity tests) and of each other (fp32_vs_fp64_storage), far "
                                  "below the statistical error of any finite run, so equal S(q) "
                                  "error means equal step counts")

    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(F, W)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(reps, c4_steps=args.cpu_c4_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
