#!/usr/bin/env python
"""Throughput of the SplitSolve hot path on one MI355X: (E, k) solves per second.

One step = the whole hot path for every (E, k) instance of the workload, inputs resident in HBM:
lead self-energies (decimation), Q = first/last block columns of (E S - H)^{-1} (Alg. 1 with
pivoted LU), the 2s x 2s open-boundary correction with psi for m injected columns and the corner of
G^R, and the Caroli transmission T_LR, T_RL.

Modes: fp64 (plain SplitSolve in FP64, T from the corner of G^R) and mixed (recursion products in
FP32 on the matrix cores, FP64 LU, injection b' = [W_L; 0] from the left lead, FP64 iterative
refinement of psi on the full open system, T from the refined psi).

Workloads (synthetic, seeded; see synth/):
  dft512   s = 512 (8x8x8 lattice slab), nb = 40, 64 energies in [-5, 5] eV x 4 momenta
           k in {pi/8, 3pi/8, 5pi/8, 7pi/8}, seed 1, crystal device, complex128   (default)
  chain16  s = 16 random chain cell, nb = 32, 64 energies in [-3, 3], seed 0, complex128
  dft1024  s = 1024 (8x8x16 slab), nb = 60, 32 energies in [-5, 5] eV, k = pi/3, seed 2
  uneven256  256 instances, each its own lattice-slab crystal: s uniform in {128, 256, 384, 512, 768},
           nb uniform in [16, 64], E uniform in [-5, 5] eV, k uniform in [0, pi); instance i draws from
           numpy default_rng([3, i]); run as one plan (per-size groups, graph replay, autotuned)
  learned  self-energies of the s = 256 (4x8x8) lead cell, seed 4: a perceptron (35 -> 512 -> 512 -> 512
           -> 4 s^2, FP32) trained on 10^4 decimation solves (E uniform in [-5, 5] eV, k on a 64-point grid
           of [0, pi)) and evaluated on 2048 held-out points: cold decimation vs warm start (network +
           Newton + judge + fallback) vs continuation from the nearest training point

Prints one JSON line.  --gpus > 1 is refused: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix, datasheet
HBM_PEAK_GBS = 8000.0

# absorb: the absorbing boundary of Step 1 (i*absorb*I on the first and last diagonal blocks, moved from
# the self-energies into A; see ss_precompute_columns), in the units of H (eV for the lattice slabs)
WORKLOADS = {
    "dft512": dict(s=512, nb=40, n_e=64, e_lo=-5.0, e_hi=5.0, ks=[np.pi / 8, 3 * np.pi / 8, 5 * np.pi / 8, 7 * np.pi / 8],
                   seed=1, eta=1e-8, m=32, chunk=256, absorb=1.0),
    "chain16": dict(s=16, nb=32, n_e=64, e_lo=-3.0, e_hi=3.0, ks=[0.0], seed=0, eta=1e-8, m=4, chunk=64, absorb=1.0),
    "dft1024": dict(s=1024, nb=60, n_e=32, e_lo=-5.0, e_hi=5.0, ks=[np.pi / 3], seed=2, eta=1e-8, m=32, chunk=32,
                    absorb=1.0),
}
# oracle transmissions of every instance, written by tests/golden/make_golden_slab.py (oracle only)
GOLDEN_T = {w: os.path.join(ROOT, "tests", "golden", f"{w}_transmission.txt") for w in ("dft512", "dft1024")}
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix, datasheet
# kernel families of the first/last-column recursion (Step 1)
RECURSION_FAMILIES = ",form,chain,panel,lu_gemm,trsm,"
UNEVEN = dict(n=256, sizes=(128, 256, 384, 512, 768), nb_lo=16, nb_hi=64, e_lo=-5.0, e_hi=5.0, seed=3, eta=1e-8,
              m=32, absorb=1.0)


def sweep_flops(nb: int, s: int) -> float:
    """Algorithmic flops of Q for one instance (both recursions + chains), 8mnk per complex GEMM,
    8/3 n^3 per complex LU, 8 n^2 k per triangular pair with k right-hand sides."""
    per_step = 8 * s**3 + 8.0 / 3 * s**3 + 8 * s**3  # D update, LU, solve with s RHS
    chain = 8 * s**3
    return 2 * (nb * per_step - 8 * s**3 + (nb - 1) * chain)


def dec_flops(s: int, iters: float) -> float:
    """Decimation pass: LU of eps, solve with 2s RHS, four s^3 products; plus the final Sigma solves."""
    return iters * (8.0 / 3 * s**3 + 16 * s**3 + 32 * s**3)


def obc_flops(nb: int, s: int, m: int) -> float:
    n = 2 * s
    cq = 8 * n * n * s
    lu = 8.0 / 3 * n**3 + 8 * n * n * (n + m)
    gc = 8 * n**3
    psi = 8 * nb * s * n * m + 8 * n * n * m
    return cq + lu + gc + psi


def build_inputs(name: str):
    import synth

    w = WORKLOADS[name]
    s, nb = w["s"], w["nb"]
    if name == "chain16":
        cells = [synth.chain_cell(s, w["seed"])]
    else:
        base = synth.DFTLikeCell(synth.SLAB_SHAPES[s], w["seed"])
        cells = [base.at(k) for k in w["ks"]]
    insts = [synth.device_from_cell(c, nb) for c in cells]
    energies = np.linspace(w["e_lo"], w["e_hi"], w["n_e"])
    E = np.tile(energies, len(cells))
    kidx = np.repeat(np.arange(len(cells), dtype=np.int32), len(energies))
    inj = np.stack([synth.injection_block(s, w["m"], 1000 + b) for b in range(len(E))])
    return w, insts, E, kidx, inj


# HBM traffic per launch of a kernel family, from rocprofv3 FETCH_SIZE/WRITE_SIZE runs calibrated with a
# plain copy (profiles/<family>_traffic_dft512.txt); null once the kernel's sources have changed since.
TRAFFIC_SOURCES = {
    "dec_update": ("paper_1812_01396_amd/csrc/selfenergy.hip", "paper_1812_01396_amd/csrc/tile.hpp"),
    "lu_gemm": ("paper_1812_01396_amd/csrc/lu.hip", "paper_1812_01396_amd/csrc/tile.hpp"),
}


def measured_traffic(family: str, workload: str):
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{family}_traffic_{workload}.txt")
    if family not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[family]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, insts, E, kidx, inj, sample: int, T_gpu):
    """The oracle, untuned, timed on the host: all cores (BLAS threads = the host's cores) on `sample`
    instances and one core on one instance.  The sample is the instances whose GPU Caroli pair T_LR, T_RL
    disagrees most (the likeliest to be off), then evenly spaced ones; returns (JSON object, worst T error
    of the GPU over the sample)."""
    import threadpoolctl

    from oracle import transport

    d = np.abs(T_gpu[:, 0] - T_gpu[:, 1])
    idx = [int(i) for i in np.argsort(-d)[: max(1, sample // 2)]]
    for i in np.linspace(0, len(E) - 1, sample).round().astype(int):
        if len(idx) < sample and int(i) not in idx:
            idx.append(int(i))
    errs = []

    def solve(b):
        inst = insts[kidx[b]]
        ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                       inst.S01, float(E[b]), w["eta"], inj=inj[b])
        errs.append(max(abs(T_gpu[b, 0] - ref["t_lr"]) / max(1.0, abs(ref["t_lr"])),
                        abs(T_gpu[b, 1] - ref["t_rl"]) / max(1.0, abs(ref["t_rl"]))))

    ncpu = os.cpu_count() or 1
    with threadpoolctl.threadpool_limits(ncpu):
        t0 = time.perf_counter()
        for b in idx:
            solve(b)
        dt_all = time.perf_counter() - t0
        cores = max((p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()), default=ncpu)
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        solve(idx[0])
        dt_one = time.perf_counter() - t0
    return dict(value=len(idx) / dt_all, unit="solves/s", cores=int(cores), kind="oracle",
                sample=f"{len(idx)} of {len(E)} instances (indices {idx}), same inputs, {dt_all:.1f} s wall "
                       f"with {cores} BLAS threads",
                single_core=dict(value=1.0 / dt_one, unit="solves/s", cores=1,
                                 sample=f"instance {idx[0]}, {dt_one:.1f} s wall"),
                cpu_model=cpu_model(), host_cpus=ncpu), float(max(errs))


def golden_errors(workload: str, T_gpu):
    """Worst |T - T_oracle| / max(1, T_oracle) over every instance, from the stored oracle transmissions
    (both Caroli directions), or None without a stored file."""
    path = GOLDEN_T.get(workload)
    if path is None or not os.path.exists(path):
        return None
    ref = np.loadtxt(path, comments="#")
    if ref.shape[0] != T_gpu.shape[0]:
        return None
    err = np.abs(T_gpu - ref[:, 3:5]) / np.maximum(1.0, np.abs(ref[:, 3:5]))
    worst = int(np.argmax(err.max(axis=1)))
    return dict(max=float(err.max()), instances=int(ref.shape[0]), worst_instance=worst,
                over_1e_8=int((err.max(axis=1) > 1e-8).sum()), over_1e_10=int((err.max(axis=1) > 1e-10).sum()))


def trace_queue_stats(path: str, pattern: str):
    """Per queue: (launches, average duration in us) of the kernels matching `pattern` in a rocprofv3
    kernel-trace CSV (the stream a kernel was launched on maps to one queue)."""
    import csv
    import re

    per = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if re.search(pattern, r["Kernel_Name"]):
                d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                per.setdefault(int(r["Queue_Id"]), []).append(d)
    return {q: (len(v), float(np.mean(v)) / 1e3) for q, v in sorted(per.items())}


def summarize_trace(path: str, steps: int = 1, top: int = 25) -> str:
    """Per-kernel summary of a rocprofv3 kernel trace: the SQLite database that rocprofv3 writes by default
    (`*_results.db`, read through its `kernels` view) or a `*kernel_trace.csv`.  Kernels are grouped by
    name with template arguments kept; per group: launches, total and average duration, share of the
    summed kernel time; then the busy time (union of all kernel intervals) against the summed time, which
    shows how much kernels overlap.  `steps` divides the totals (launches and ms per step)."""
    import csv
    import sqlite3

    rows = []  # (name, start_ns, end_ns)
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        for name, st, en in con.execute("select name, start, end from kernels"):
            rows.append((name, int(st), int(en)))
        con.close()
    else:
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                rows.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    if not rows:
        return "no kernels in " + path
    agg = {}
    for name, st, en in rows:
        n, t = agg.get(name, (0, 0))
        agg[name] = (n + 1, t + (en - st))
    total = sum(t for _, t in agg.values())
    iv = sorted((st, en) for _, st, en in rows)
    busy, cur_s, cur_e = 0, iv[0][0], iv[0][1]
    for st, en in iv[1:]:
        if st > cur_e:
            busy += cur_e - cur_s
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
    busy += cur_e - cur_s
    span = iv[-1][1] - iv[0][0]
    lines = [f"# kernel summary of {os.path.basename(path)}: {len(rows)} launches, {steps} step(s)",
             f"# summed kernel time {total / 1e6 / steps:.1f} ms per step; busy (any kernel running) "
             f"{busy / 1e6 / steps:.1f} ms per step; first start to last end {span / 1e6:.1f} ms",
             f"{'share':>6} {'ms/step':>9} {'launches/step':>13} {'avg_us':>9}  kernel"]
    for name, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{100.0 * t / total:5.1f}% {t / 1e6 / steps:9.2f} {n / steps:13.1f} {t / n / 1e3:9.1f}  {name}")
    return "\n".join(lines)


def counter_means(path: str, pattern: str):
    """Per queue: (launches, mean, max) of the counter values (KiB per dispatch) that a rocprofv3 --pmc run
    wrote to its *_counter_collection.csv, over the kernels whose name matches `pattern`."""
    import csv
    import re

    per = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if re.search(pattern, r["Kernel_Name"]):
                per.setdefault(int(r["Queue_Id"]), []).append(float(r["Counter_Value"]))
    return {q: (len(v), float(np.mean(v)), float(np.max(v))) for q, v in sorted(per.items())}


# kernel families of the SQ counter report: (label, name pattern)
SQ_FAMILIES = [("k_lu_gemm 64x64", r"k_lu_gemm<ss::TileCfg<64, 64"),
               ("k_lu_gemm 64x64 G3", r"k_lu_gemm<ss::TileCfgG3<64, 64"), ("k_lu_gemm 64x32", r"k_lu_gemm<ss::TileCfg<64, 32"),
               ("k_lu_gemm 32x128", r"k_lu_gemm<ss::TileCfg<32, 128"), ("k_panel32", r"k_panel32<"),
               ("k_lu_leaf2x", r"k_lu_leaf2x<"), ("k_form", r"k_form<"), ("k_chain", r"k_chain<"),
               ("k_dec_update", r"k_dec_update")]
MI355X_SIMDS = 256 * 4
MI355X_XCDS = 8


def sq_report(paths) -> str:
    """Per-dispatch means of the SQ/GRBM counters that rocprofv3 --pmc wrote (one or more
    *_counter_collection.csv files, one row per dispatch and counter), per kernel family, with derived
    ratios: the share of wave time spent waiting to issue (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES, both in
    quad-cycles), instructions per wave, the matrix-core busy share (SQ_VALU_MFMA_BUSY_CYCLES summed over
    the 1024 SIMDs / (1024 x the per-XCD clock cycles, GRBM_GUI_ACTIVE being summed over the 8 XCDs: it
    reads 8 x 2.38 cycles per ns of dispatch)) and the FP64 matrix flops the hardware counted
    (MOPS_F64 x 512) per second of the dispatch's duration."""
    import csv
    import re

    disp = {}
    for path in paths:
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                key = (path, r["Dispatch_Id"])
                d = disp.setdefault(key, {"name": r["Kernel_Name"], "ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
                d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = ["family | dispatches | mean us | waves | wait/wave-cycles | VALU/wave | MFMA/wave | LDS/wave | "
             "MFMA busy | FP64 MFMA TF/s (counted)"]
    for label, pat in SQ_FAMILIES:
        rows = [d for d in disp.values() if re.search(pat, d["name"])]
        if not rows:
            continue
        m = lambda c: float(np.mean([d.get(c, np.nan) for d in rows]))  # noqa: E731
        us = m("ns") / 1e3
        waves = m("SQ_WAVES")
        wait = m("SQ_WAIT_INST_ANY") / max(m("SQ_WAVE_CYCLES"), 1.0)
        busy = m("SQ_VALU_MFMA_BUSY_CYCLES") / max(m("GRBM_GUI_ACTIVE") / MI355X_XCDS * MI355X_SIMDS, 1.0)
        tfs = m("SQ_INSTS_VALU_MFMA_MOPS_F64") * 512.0 / max(m("ns"), 1.0) / 1e3
        lines.append(f"{label} | {len(rows)} | {us:.1f} | {waves:.0f} | {wait:.3f} | {m('SQ_INSTS_VALU') / waves:.0f} | "
                     f"{m('SQ_INSTS_MFMA') / waves:.0f} | {m('SQ_INSTS_LDS') / waves:.0f} | {busy:.3f} | {tfs:.1f}")
    return "\n".join(lines)


def traffic_report(family: str, workload: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str,
                   copy_write_csv: str, queue: int, algorithmic_bytes: float, commands: str) -> str:
    """The text of profiles/<family>_traffic_<workload>.txt: FETCH_SIZE and WRITE_SIZE per dispatch of the
    family's kernel (queue `queue`: the stream whose launches the roofline covers), each scaled by what the
    counter reads for a plain 1 GiB device copy, beside the algorithmic bytes per launch and the SHA-256
    of the kernel's sources (bench.py uses the traffic only while the sources are unchanged)."""
    import hashlib

    kern = {"lu_gemm": r"k_lu_gemm<", "dec_update": r"k_dec_update"}[family]
    copy_bytes = float(1 << 30)
    cf = counter_means(copy_fetch_csv, r"copyBuffer")
    cw = counter_means(copy_write_csv, r"copyBuffer")
    f_fetch = copy_bytes / (1024.0 * next(iter(cf.values()))[1])
    f_write = copy_bytes / (1024.0 * next(iter(cw.values()))[1])
    fm, wm = counter_means(fetch_csv, kern), counter_means(write_csv, kern)
    rd = fm[queue][1] * 1024.0 * f_fetch
    wr = wm[queue][1] * 1024.0 * f_write
    h = hashlib.sha256()
    for fsrc in TRAFFIC_SOURCES[family]:
        with open(os.path.join(ROOT, fsrc), "rb") as fh:
            h.update(fh.read())
    lines = [f"HBM traffic of k_{family}, {workload} workload", "",
             "commands (from the repository root, on one MI355X; one counter per run):", commands, "",
             "report: python3 bench.py --traffic-report " + family + " ... (bench.traffic_report)",
             f"copy calibration: FETCH_SIZE reads {1.0 / f_fetch:.4f} of the bytes a plain 1 GiB copy reads "
             f"(factor {f_fetch:.4f}), WRITE_SIZE {1.0 / f_write:.4f} of the bytes written (factor {f_write:.4f})"]
    for q in sorted(set(fm) | set(wm)):
        n1, m1, x1 = fm.get(q, (0, 0.0, 0.0))
        n2, m2, x2 = wm.get(q, (0, 0.0, 0.0))
        lines.append(f"  queue {q}: {n1} launches; FETCH_SIZE mean {m1:.1f} KiB (max {x1:.1f}), "
                     f"WRITE_SIZE mean {m2:.1f} KiB (max {x2:.1f})")
    lines += ["", f"roofline queue: {queue}",
              f"traffic_read_bytes_per_launch: {rd:.6e}",
              f"traffic_write_bytes_per_launch: {wr:.6e}",
              f"traffic_bytes_per_launch: {rd + wr:.6e}",
              f"algorithmic_bytes_per_launch: {algorithmic_bytes:.6e}",
              f"traffic_over_algorithmic: {(rd + wr) / algorithmic_bytes:.3f}",
              f"kernel_source_sha256: {h.hexdigest()}"]
    return "\n".join(lines) + "\n"


def uneven_specs(n: int = UNEVEN["n"], seed: int = UNEVEN["seed"]):
    """(s, nb, E, k, cell_seed) of every instance of the uneven batch; instance i from default_rng([seed, i])."""
    u = UNEVEN
    out = []
    for i in range(n):
        rng = np.random.default_rng([seed, i])
        s = int(rng.choice(u["sizes"]))
        nb = int(rng.integers(u["nb_lo"], u["nb_hi"] + 1))
        E = float(rng.uniform(u["e_lo"], u["e_hi"]))
        k = float(rng.uniform(0.0, np.pi))
        out.append((s, nb, E, k, int(rng.integers(2**31))))
    return out


def uneven_cell(spec):
    import synth
    s, nb, E, k, cs = spec
    return synth.DFTLikeCell(synth.SLAB_SHAPES[s], cs).at(k)


class UnevenPipeline:
    """The uneven batch as one ss_plan: crystal devices (every block a copy of the instance's own cell,
    materialised on the GPU), psi for m columns per instance; run() is one plan execution."""

    def __init__(self, n: int = UNEVEN["n"], use_graph: bool = True, autotune: bool = True, mem_gib: float = 0.0,
                 absorb: float | None = None):
        import torch

        import paper_1812_01396_amd as ss

        self.ss, self.torch = ss, torch
        self.specs = uneven_specs(n)
        self.w = dict(UNEVEN, n=n)
        if absorb is not None:
            self.w["absorb"] = absorb
        m = self.w["m"]
        dev = torch.device("cuda", 0)
        self.ctx = ss.Context(0)
        self.instances = []
        t0 = time.perf_counter()
        for i, spec in enumerate(self.specs):
            if i % 32 == 0:
                print(f"uneven256: building instance {i} of {len(self.specs)} ({time.perf_counter() - t0:.0f} s)",
                      file=sys.stderr, flush=True)
            s, nb, E, k, _ = spec
            h00, h01, s00, s01 = (torch.as_tensor(a).to(dev) for a in uneven_cell(spec))
            x = ss.Instance(h00.expand(nb, s, s).contiguous(), h01.expand(nb - 1, s, s).contiguous(),
                            s00.expand(nb, s, s).contiguous(), s01.expand(nb - 1, s, s).contiguous(),
                            h00, h01, s00, s01, E, torch.zeros(nb, s, m, dtype=torch.complex128, device=dev))
            self.instances.append(x)
        torch.cuda.synchronize()
        print(f"uneven256: inputs resident ({time.perf_counter() - t0:.0f} s); creating the plan", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        if mem_gib <= 0:  # the device memory left after the inputs, less a margin
            free, _ = torch.cuda.mem_get_info(dev)
            mem_gib = max(8.0, free / (1 << 30) - 4.0)
        self.mem_gib = mem_gib
        self.plan = ss.Plan(self.ctx, self.instances, self.w["eta"], m=m, use_graph=use_graph, autotune=autotune,
                            mem_bytes=int(mem_gib * (1 << 30)), absorb=self.w["absorb"])
        torch.cuda.synchronize()
        self.create_s = time.perf_counter() - t0
        print(f"uneven256: plan created in {self.create_s:.1f} s, graph nodes {self.plan.graph_nodes}", file=sys.stderr,
              flush=True)

    def run(self):
        self.plan.execute()


def run_uneven(args):
    import torch

    pipe = UnevenPipeline(use_graph=not args.no_graph, autotune=not args.no_autotune, mem_gib=args.plan_mem_gib,
                          absorb=None if args.absorb < 0 else args.absorb)
    for _ in range(args.warmup):
        pipe.run()
    torch.cuda.synchronize()
    print("uneven256: warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"uneven256: {args.steps} steps in {elapsed:.2f} s", file=sys.stderr, flush=True)
    T = pipe.plan.T.cpu().numpy()
    info = pipe.plan.info.cpu().numpy()
    m = pipe.w["m"]
    f_step = sum(sweep_flops(nb, s) + dec_flops(s, float(info[i, 3])) + obc_flops(nb, s, m)
                 for i, (s, nb, _, _, _) in enumerate(pipe.specs))
    f_sweep = sum(sweep_flops(nb, s) for (s, nb, _, _, _) in pipe.specs)
    ms_per_step = elapsed * 1e3 / args.steps
    achieved = f_step / (ms_per_step * 1e-3) / 1e12
    cpu, t_err = None, None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        from oracle import transport
        import synth
        # the smallest instances keep the oracle's share of the run bounded
        order = sorted(range(len(pipe.specs)), key=lambda i: pipe.specs[i][0] ** 3 * pipe.specs[i][1])
        idx = order[: args.cpu_sample]
        t0 = time.perf_counter()
        errs = []
        for i in idx:
            s, nb, E, k, _ = pipe.specs[i]
            inst = synth.device_from_cell(uneven_cell(pipe.specs[i]), nb)
            ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00,
                                           inst.S01, E, pipe.w["eta"], want_q=False)
            errs.append(max(abs(T[i, 0] - ref["t_lr"]), abs(T[i, 1] - ref["t_rl"])) / max(1.0, abs(ref["t_lr"])))
        dt = time.perf_counter() - t0
        try:
            import threadpoolctl
            cores = max(p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()) or os.cpu_count()
        except Exception:
            cores = os.cpu_count()
        cpu = dict(value=len(idx) / dt, unit="solves/s", cores=int(cores), kind="oracle",
                   sample=f"{len(idx)} smallest of {len(pipe.specs)} instances (indices {idx}), {dt:.1f} s wall; "
                          "not representative of the mean instance")
        t_err = float(max(errs))
    groups = pipe.plan.groups()
    out = {
        "metric": "(E,k) solves/sec",
        "value": round(len(pipe.specs) * args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "uneven256", "instances": len(pipe.specs), "sizes": list(UNEVEN["sizes"]),
                   "nb_range": [UNEVEN["nb_lo"], UNEVEN["nb_hi"]], "m_inj": m, "eta": UNEVEN["eta"],
                   "graph": not args.no_graph, "autotune": not args.no_autotune, "plan_mem_gib": round(pipe.mem_gib, 1),
                   "precision": "fp64", "absorb": pipe.w["absorb"]},
        "tflops_step": round(achieved, 3),
        "sweep_tflop": round(f_sweep / 1e12, 2),
        "step_tflop": round(f_step / 1e12, 2),
        "roofline": dict(bound="mfma", achieved=round(achieved, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                         frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=None, kernel="whole step"),
        "plan_create_s": round(pipe.create_s, 2),
        "graph_nodes": pipe.plan.graph_nodes,
        "graph_segments": pipe.plan.graph_segments,
        "groups": groups,
        "decimation_iters": [int(info[:, 3].min()), int(info[:, 3].max())],
        "nonzero_info": int((info[:, :3] != 0).sum()),
        "t_lr_minus_t_rl_max": float(np.abs(T[:, 0] - T[:, 1]).max()),
        "t_minus_integer_max": float(np.abs(T - np.round(T)).max()),
        "cpu_baseline": cpu,
        "t_err_vs_oracle": t_err,
    }
    print(json.dumps(out))


LEARNED = dict(s=256, seed=4, n_train=10000, n_eval=2048, nk=64, eta=1e-8, width=512, steps=2000, batch=256,
               lr=1e-3)


def run_learned(args):
    """cfg of the learned warm start: training on the GPU, then cold / warm / continuation solves."""
    import torch

    import paper_1812_01396_amd as ss
    import synth

    w = LEARNED
    s, dev = w["s"], torch.device("cuda", 0)
    rng = np.random.default_rng(w["seed"])
    n_all = w["n_train"] + w["n_eval"]
    E = rng.uniform(-5.0, 5.0, n_all)
    kgrid = (np.arange(w["nk"]) + 0.5) * np.pi / w["nk"]
    ki = rng.integers(0, w["nk"], n_all).astype(np.int32)
    base = synth.DFTLikeCell(synth.SLAB_SHAPES[s], w["seed"])
    cells = [base.at(k) for k in kgrid]
    lead = [torch.as_tensor(np.stack([c[j] for c in cells])).to(dev) for j in range(4)]
    ctx = ss.Context(0)
    Ed = torch.as_tensor(E).to(dev)
    kd = torch.as_tensor(kgrid[ki]).to(dev)
    kid = torch.as_tensor(ki).to(dev)
    tr, ev = slice(0, w["n_train"]), slice(w["n_train"], n_all)
    log = lambda msg: print(f"learned: {msg}", file=sys.stderr, flush=True)  # noqa: E731

    # training data from the decimation
    t0 = time.perf_counter()
    sig = torch.empty(n_all, 2, s, s, dtype=torch.complex128, device=dev)
    it_dec = torch.empty(n_all, dtype=torch.int32, device=dev)
    for c0 in range(0, w["n_train"], 1024):
        c1 = min(c0 + 1024, w["n_train"])
        ss.ss_lead_selfenergy(ctx, *lead, Ed[c0:c1].contiguous(), w["eta"], kidx=kid[c0:c1].contiguous(),
                              sigma=sig[c0:c1], iters=it_dec[c0:c1])
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"training data {t_data:.1f} s")
    X = ss.ss_warm_features(ctx, Ed, kd)
    mean, std = ss.ss_sigma_moments(ctx, sig[tr].contiguous(), std_floor=1e-6)
    Y = ss.ss_sigma_encode(ctx, sig[tr].contiguous(), mean, std)
    dims = [X.shape[1], w["width"], w["width"], w["width"], 4 * s * s]
    net = ss.MLP(ctx, dims, seed=w["seed"])
    g = torch.Generator(device="cpu").manual_seed(w["seed"])
    t0 = time.perf_counter()
    losses = []
    for step in range(w["steps"]):
        idx = torch.randint(0, w["n_train"], (w["batch"],), generator=g).to(dev)
        xb, yb = X[idx].contiguous(), Y[idx].contiguous()
        acts, _ = net.forward(xb)
        loss = net.backward(xb, acts, yb)
        net.adam(w["lr"])
        if step % 100 == 0 or step == w["steps"] - 1:
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"training {t_train:.1f} s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    del Y

    Ee, ke, kie = Ed[ev].contiguous(), kd[ev].contiguous(), kid[ev].contiguous()
    ne = w["n_eval"]

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    # cold: the decimation
    (cold, _, _, info_c), t_cold = timed(lambda: ss.ss_lead_selfenergy(ctx, *lead, Ee, w["eta"], kidx=kie,
                                                                       iters=it_dec[ev]))
    ref = cold.clone()
    it_cold = it_dec[ev].cpu().numpy()

    # warm: features -> network -> Sigma -> Newton (judge, fallback)
    def warm():
        Xe = ss.ss_warm_features(ctx, Ee, ke)
        _, pred = net.forward(Xe)
        init = ss.ss_sigma_decode(ctx, pred.contiguous(), mean, std, s)
        return init, ss.ss_lead_selfenergy_warm(ctx, *lead, Ee, w["eta"], init, kidx=kie)
    (init_w, (sig_w, itn_w, itd_w, _, info_w)), t_warm = timed(warm)

    # continuation: Newton from the self-energy of the nearest training point at the same momentum
    E_np, ki_np = E, ki
    near = np.empty(ne, dtype=np.int64)
    for j in range(ne):
        cand = np.nonzero(ki_np[tr] == ki_np[w["n_train"] + j])[0]
        near[j] = cand[np.argmin(np.abs(E_np[cand] - E_np[w["n_train"] + j]))]
    init_c = sig[torch.as_tensor(near).to(dev)].contiguous()
    (sig_c, itn_c, itd_c, _, info_c2), t_cont = timed(
        lambda: ss.ss_lead_selfenergy_warm(ctx, *lead, Ee, w["eta"], init_c, kidx=kie))

    def rel_err(a, b):
        d = (a - b).reshape(a.shape[0], -1).norm(dim=1) / b.reshape(b.shape[0], -1).norm(dim=1)
        return d.cpu().numpy()

    err_pred = rel_err(init_w, ref)
    err_cont_start = rel_err(init_c, ref)
    info_w, info_c2 = info_w.cpu().numpy(), info_c2.cpu().numpy()
    out = {
        "metric": "(E,k) self-energy solves/sec",
        "value": round(ne / t_warm, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(t_warm * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (network fp32)",
        "data": "synthetic",
        "config": {"workload": "learned", "s": s, "n_train": w["n_train"], "n_eval": ne, "k_grid": w["nk"],
                   "eta": w["eta"], "dims": dims, "train_steps": w["steps"], "batch": w["batch"]},
        "cold_decimation": {"solves_per_s": round(ne / t_cold, 3), "iters": [int(it_cold.min()), int(it_cold.max())],
                            "nonzero_info": int((info_c.cpu().numpy() != 0).sum())},
        "warm_start": {"solves_per_s": round(ne / t_warm, 3), "accepted": int((info_w == 0).sum()),
                       "fallback": int((info_w == -2).sum()), "newton_iters_max": int(itn_w.max()),
                       "prediction_rel_err_median": float(np.median(err_pred)),
                       "max_rel_diff_vs_cold": float(rel_err(sig_w, ref).max())},
        "continuation": {"solves_per_s": round(ne / t_cont, 3), "accepted": int((info_c2 == 0).sum()),
                         "start_rel_err_median": float(np.median(err_cont_start)),
                         "max_rel_diff_vs_cold": float(rel_err(sig_c, ref).max())},
        "training": {"data_s": round(t_data, 2), "train_s": round(t_train, 2), "loss_first": losses[0],
                     "loss_last": losses[-1]},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


class Pipeline:
    """The whole hot path for every instance of a workload, inputs resident on the GPU.

    run() enqueues one step: self-energies on a second stream (overlapping the first chunk's
    recursion), then per chunk of instances Q, the open-boundary correction with psi and the corner
    of G^R, and T.  Outputs stay on the device (sigma, iters, resid, psi, gc, T, info_*).
    """

    def __init__(self, workload: str, chunk: int = 0, mode: str = "fp64", refine_tol: float = 1e-10,
                 accept_tol: float = 1e-10, absorb: float | None = None, m: int = 0, lanes: int = 1,
                 lu_tile: int = 0):
        import torch

        import paper_1812_01396_amd as ss

        self.ss, self.torch = ss, torch
        self.mode = mode
        self.prec = {"fp64": ss.SS_PREC_FP64, "mixed": ss.SS_PREC_FP32, "mixed-lu": ss.SS_PREC_FP32_LU,
                     "mixed-bf16": ss.SS_PREC_BF16}[mode]
        self.refine_tol = refine_tol
        self.accept_tol = accept_tol  # refined residual above this: the instance is redone in FP64
        self.fallback = 0
        w, insts, E_np, kidx_np, inj_np = build_inputs(workload)
        w = dict(w)
        if absorb is not None:
            w["absorb"] = absorb
        if m > 0 and mode != "fp64":  # columns of the injection factor W_L (the seeded b' of FP64 mode keeps its m)
            w["m"] = m
        self.absorb = w["absorb"]
        self.w, self.insts, self.E_np, self.kidx_np, self.inj_np = w, insts, E_np, kidx_np, inj_np
        s, nb, m = w["s"], w["nb"], w["m"]
        self.n = nb_inst = len(E_np)
        # lanes > 1: the instances split into that many lanes, each with a context, stream and host thread
        # of its own running its whole path (Step 1, corner, refinement, T) beside the others
        self.lanes = max(1, int(lanes))
        self.chunk = -(-nb_inst // self.lanes) if self.lanes > 1 else (chunk or w["chunk"])
        dev = self.dev = torch.device("cuda", 0)

        def t(a, dt=torch.complex128):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)

        self.Hd = t(np.stack([i.Hd for i in insts]))
        self.Hu = t(np.stack([i.Hu for i in insts]))
        self.Sd = t(np.stack([i.Sd for i in insts]))
        self.Su = t(np.stack([i.Su for i in insts]))
        self.lead = [t(np.stack([getattr(i, f) for i in insts])) for f in ("H00", "H01", "S00", "S01")]
        self.E = t(E_np, torch.float64)
        self.kidx = t(kidx_np, torch.int32)
        # FP64 mode injects the seeded b'; the mixed modes write W_L of their own width here
        self.inj = t(inj_np) if mode == "fp64" else torch.zeros(nb_inst, 2 * s, m, dtype=torch.complex128, device=dev)
        c128 = torch.complex128
        self.sigma = torch.empty(nb_inst, 2, s, s, dtype=c128, device=dev)
        self.iters = torch.empty(nb_inst, dtype=torch.int32, device=dev)
        self.resid = torch.empty(nb_inst, 2, dtype=torch.float64, device=dev)
        self.info_s = torch.empty(nb_inst, dtype=torch.int32, device=dev)
        self.Qbuf = torch.empty(self.chunk, nb, s, 2 * s, dtype=c128, device=dev)
        self.psi = torch.empty(nb_inst, nb, s, m, dtype=c128, device=dev)
        self.gc = torch.empty(nb_inst, 2 * s, 2 * s, dtype=c128, device=dev)
        self.T = torch.empty(nb_inst, 2, dtype=torch.float64, device=dev)
        self.info_q = torch.empty(nb_inst, dtype=torch.int32, device=dev)
        self.info_o = torch.empty(nb_inst, dtype=torch.int32, device=dev)
        self.T_psi = torch.empty(nb_inst, dtype=torch.float64, device=dev)
        # mixed: last block row of the unrefined psi (with gc it carries the part of Gamma_L outside W_L)
        self.psi0 = torch.empty(nb_inst, s, m, dtype=c128, device=dev) if mode != "fp64" else None
        self.rank = torch.zeros(nb_inst, dtype=torch.int32, device=dev)
        self.ir_iters = torch.zeros(nb_inst, dtype=torch.int32, device=dev)
        self.ir_resid = torch.zeros(nb_inst, dtype=torch.float64, device=dev)
        self.stream_main = torch.cuda.current_stream(dev)
        self.stream_sig = torch.cuda.Stream(dev)  # default priority
        self.ctx = ss.Context(0, self.stream_main)
        self.ctx_s = ss.Context(0, self.stream_sig)
        self.lane_streams, self.lane_ctx, self.lane_Q = [self.stream_main], [self.ctx], [self.Qbuf]
        for _ in range(1, self.lanes):
            st = torch.cuda.Stream(dev)  # default priority
            self.lane_streams.append(st)
            self.lane_ctx.append(ss.Context(0, st))
            self.lane_Q.append(torch.empty(self.chunk, nb, s, 2 * s, dtype=c128, device=dev))
        for c in self.lane_ctx + [self.ctx_s]:  # tile of the LU's general block products
            c.set_lu_tile(lu_tile)
        ss.splitsolve._check_kidx(self.kidx, len(insts))  # once: the step itself never reads back to the host

    def close(self):
        """Release the pipeline's contexts (their device workspaces); the tensors go with the object."""
        for c in self.lane_ctx + [self.ctx_s]:
            c.close()

    def run(self, recursion_ms=None):
        """One step.  recursion_ms: a list that receives the summed duration (ms) of the recursion's
        kernels of each chunk (HIP events on the main stream; synchronizes after each chunk's recursion)."""
        if self.lanes > 1:
            return self._run_lanes(recursion_ms)
        ss, torch, w = self.ss, self.torch, self.w
        # the previous step's readers of sigma (main stream) finish before sigma is overwritten
        prev = torch.cuda.Event()
        prev.record(self.stream_main)
        done = torch.cuda.Event()
        err = []

        def run_sigma():
            try:
                with torch.cuda.stream(self.stream_sig):
                    self.stream_sig.wait_event(prev)
                    ss.ss_lead_selfenergy(self.ctx_s, *self.lead, self.E, w["eta"], kidx=self.kidx, sigma=self.sigma,
                                          iters=self.iters, resid=self.resid, info=self.info_s, validate=False)
                    done.record(self.stream_sig)
            except Exception as e:  # surfaced after join
                err.append(e)

        th = threading.Thread(target=run_sigma)
        th.start()
        mixed = self.mode != "fp64"
        for c0 in range(0, self.n, self.chunk):
            c1 = min(c0 + self.chunk, self.n)
            q = self.Qbuf[: c1 - c0]
            if recursion_ms is not None:
                self.ctx.kernel_timer(RECURSION_FAMILIES)
            ss.ss_precompute_columns(self.ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E[c0:c1],
                                     kidx=self.kidx[c0:c1], Q=q, info=self.info_q[c0:c1], validate=False,
                                     prec=self.prec, keep_factors=mixed,
                                     absorb=self.absorb)
            if recursion_ms is not None:
                recursion_ms.append(self.ctx.kernel_timer_read()[0])
                self.ctx.kernel_timer(None)
            if c0 == 0:
                th.join()
                if err:
                    raise err[0]
                self.stream_main.wait_event(done)
            sig = self.sigma[c0:c1]
            if mixed:
                ss.ss_injection_left(self.ctx, sig, w["m"], inj=self.inj[c0:c1], rank=self.rank[c0:c1])
            ss.ss_apply_obc(self.ctx, q, sig, inj=self.inj[c0:c1], psi=self.psi[c0:c1], gc=self.gc[c0:c1],
                            info=self.info_o[c0:c1], absorb=self.absorb)
            if mixed:
                self.psi0[c0:c1].copy_(self.psi[c0:c1, -1])
                ss.ss_refine_psi(self.ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E[c0:c1], q, sig,
                                 self.inj[c0:c1], self.psi[c0:c1], kidx=self.kidx[c0:c1], tol=self.refine_tol,
                                 iters=self.ir_iters[c0:c1], resid=self.ir_resid[c0:c1])
                self._fp64_fallback(c0, c1)
                ss.ss_transmission_psi(self.ctx, self.psi[c0:c1], sig, T=self.T_psi[c0:c1], psi0=self.psi0[c0:c1],
                                       gc=self.gc[c0:c1])
            else:
                ss.ss_transmission(self.ctx, self.gc[c0:c1], sig, T=self.T[c0:c1])

    def recursion_alone(self, family=RECURSION_FAMILIES, with_flops=False):
        """Step 1 by itself (no self-energies beside it): wall time (ms) of ss_precompute_columns over
        all instances, and the summed duration of the launches of `family` (HIP events; all of the
        recursion's kernels by default); with_flops: also their launch count and algorithmic flops."""
        ss, torch = self.ss, self.torch
        mixed = self.mode != "fp64"
        torch.cuda.synchronize()
        self.ctx.kernel_timer(family)
        t0 = time.perf_counter()
        for c0 in range(0, self.n, self.chunk):
            c1 = min(c0 + self.chunk, self.n)
            ss.ss_precompute_columns(self.ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E[c0:c1],
                                     kidx=self.kidx[c0:c1], Q=self.Qbuf[: c1 - c0], info=self.info_q[c0:c1],
                                     validate=False, prec=self.prec,
                                     keep_factors=mixed, absorb=self.absorb)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        rd = self.ctx.kernel_timer_read(with_flops=with_flops)
        self.ctx.kernel_timer(None)
        if with_flops:
            return wall, rd[0], rd[1], rd[2]
        return wall, rd[0]

    def observables(self):
        """Orbital density and bond currents of every instance's psi (ss_observables, after a step), timed
        with HIP events on the main stream, and their energy integral with trapezoid weights and a Fermi
        occupation at mu = 0, kT = 0.025 (the quadrature is an input of the library call).  Current
        conservation is reported as the largest spread of J_i over the interfaces of one instance."""
        ss, torch, w = self.ss, self.torch, self.w
        s, nb, m = w["s"], w["nb"], w["m"]
        dE = float(self.E_np[1] - self.E_np[0]) if len(self.E_np) > 1 else 1.0
        ne = w["n_e"]
        wt = np.full(len(self.E_np), dE / (2 * np.pi) / len(w["ks"]))
        wt[np.arange(len(self.E_np)) % ne == 0] *= 0.5
        wt[np.arange(len(self.E_np)) % ne == ne - 1] *= 0.5
        wt *= 0.5 * (1.0 - np.tanh(0.5 * self.E_np / 0.025))
        wt_d = torch.as_tensor(wt, dtype=torch.float64, device=self.dev)
        torch.cuda.synchronize()
        self.ctx.kernel_timer("obs")
        dens, cur = ss.ss_observables(self.ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E, self.psi, kidx=self.kidx)
        ms, launches = self.ctx.kernel_timer_read()[:2]
        self.ctx.kernel_timer(None)
        n_int = ss.ss_energy_integral(self.ctx, wt_d, dens)
        torch.cuda.synchronize()
        cur_np = cur.cpu().numpy()
        spread = float(np.max((cur_np.max(axis=1) - cur_np.min(axis=1)) / np.maximum(np.abs(cur_np).max(axis=1), 1e-300)))
        n_b = self.n
        # density: the diagonal and off-diagonal S blocks times psi (3 nb - 2 products of s x s x m per
        # instance); current: nb - 1 products
        flops = 8.0 * s * s * m * n_b * ((3 * nb - 2) + (nb - 1))
        return dict(ms=round(ms, 3), launches=int(launches), tflops=round(flops / (ms * 1e-3) / 1e12, 3),
                    frac_fp64_peak=round(flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                    current_spread_max=spread, integrated_density_sum=float(n_int.sum().item()))

    def _run_lanes(self, recursion_ms=None):
        """One step with the instances split into lanes: the self-energies of all instances on their own
        stream as in run(), and every lane's Step 1, corner correction, refinement and T on its own context
        and stream from a host thread of its own (the refinement's convergence polls wait for that lane's
        stream only), so one lane's latency-bound tail overlaps the other lanes' work.  recursion_ms receives
        the summed duration of lane 0's recursion kernels (self.chunk instances)."""
        ss, torch, w = self.ss, self.torch, self.w
        prevs = []
        for st in self.lane_streams:  # the previous step's readers of sigma finish before it is overwritten
            e = torch.cuda.Event()
            e.record(st)
            prevs.append(e)
        done = torch.cuda.Event()
        sig_ready = threading.Event()
        err = []

        def run_sigma():
            try:
                with torch.cuda.stream(self.stream_sig):
                    for e in prevs:
                        self.stream_sig.wait_event(e)
                    ss.ss_lead_selfenergy(self.ctx_s, *self.lead, self.E, w["eta"], kidx=self.kidx, sigma=self.sigma,
                                          iters=self.iters, resid=self.resid, info=self.info_s, validate=False)
                    done.record(self.stream_sig)
            except Exception as e:  # surfaced after join
                err.append(e)
            finally:
                sig_ready.set()

        def run_lane(li):
            try:
                c0 = li * self.chunk
                c1 = min(c0 + self.chunk, self.n)
                if c0 >= c1:
                    return
                ctx, st, q = self.lane_ctx[li], self.lane_streams[li], self.lane_Q[li][: c1 - c0]
                with torch.cuda.stream(st):
                    self._path(ctx, q, c0, c1, sig_ready, done, err, recursion_ms if li == 0 else None)
            except Exception as e:
                err.append(e)

        ths = [threading.Thread(target=run_sigma)] + [threading.Thread(target=run_lane, args=(li,))
                                                       for li in range(self.lanes)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        if err:
            raise err[0]
        for st in self.lane_streams[1:]:  # later work on the main stream follows every lane
            e = torch.cuda.Event()
            e.record(st)
            self.stream_main.wait_event(e)

    def _path(self, ctx, q, c0, c1, sig_ready, done, err, recursion_ms=None):
        """Step 1 and the post-processing of instances [c0, c1) on ctx (and the current stream, ctx's)."""
        ss, w = self.ss, self.w
        mixed = self.mode != "fp64"
        if recursion_ms is not None:
            ctx.kernel_timer(RECURSION_FAMILIES)
        ss.ss_precompute_columns(ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E[c0:c1], kidx=self.kidx[c0:c1], Q=q,
                                 info=self.info_q[c0:c1], validate=False, prec=self.prec, keep_factors=mixed,
                                 absorb=self.absorb)
        if recursion_ms is not None:
            recursion_ms.append(ctx.kernel_timer_read()[0])
            ctx.kernel_timer(None)
        sig_ready.wait()
        if err:
            return
        self.torch.cuda.current_stream().wait_event(done)
        sig = self.sigma[c0:c1]
        if mixed:
            ss.ss_injection_left(ctx, sig, w["m"], inj=self.inj[c0:c1], rank=self.rank[c0:c1])
        ss.ss_apply_obc(ctx, q, sig, inj=self.inj[c0:c1], psi=self.psi[c0:c1], gc=self.gc[c0:c1],
                        info=self.info_o[c0:c1], absorb=self.absorb)
        if mixed:
            self.psi0[c0:c1].copy_(self.psi[c0:c1, -1])
            ss.ss_refine_psi(ctx, self.Hd, self.Hu, self.Sd, self.Su, self.E[c0:c1], q, sig, self.inj[c0:c1],
                             self.psi[c0:c1], kidx=self.kidx[c0:c1], tol=self.refine_tol,
                             iters=self.ir_iters[c0:c1], resid=self.ir_resid[c0:c1])
            self._fp64_fallback(c0, c1, ctx, q)
            ss.ss_transmission_psi(ctx, self.psi[c0:c1], sig, T=self.T_psi[c0:c1], psi0=self.psi0[c0:c1],
                                   gc=self.gc[c0:c1])
        else:
            ss.ss_transmission(ctx, self.gc[c0:c1], sig, T=self.T[c0:c1])

    def _fp64_fallback(self, c0, c1, ctx=None, qbuf=None):
        """Instances whose refinement from the FP32-product factors did not reach the tolerance (pivot
        blocks too ill-conditioned for FP32 products) are solved again with FP64 products and refined."""
        ss, torch = self.ss, self.torch
        ctx = ctx if ctx is not None else self.ctx
        qbuf = qbuf if qbuf is not None else self.Qbuf
        bad = torch.nonzero(~(self.ir_resid[c0:c1] <= self.accept_tol)).flatten()
        nbad = int(bad.numel())  # one host read per chunk
        self.fallback += nbad
        if nbad == 0:
            return
        idx = bad + c0
        E_b, k_b = self.E[idx].contiguous(), self.kidx[idx].contiguous()
        sig_b, inj_b = self.sigma[idx].contiguous(), self.inj[idx].contiguous()
        q = qbuf[:nbad]
        info_b = torch.zeros(nbad, dtype=torch.int32, device=self.dev)
        ss.ss_precompute_columns(ctx, self.Hd, self.Hu, self.Sd, self.Su, E_b, kidx=k_b, Q=q, info=info_b,
                                 validate=False, prec=ss.SS_PREC_FP64, keep_factors=True, absorb=self.absorb)
        self.info_q[idx] = info_b
        psi_b, gc_b, info_ob = ss.ss_apply_obc(ctx, q, sig_b, inj=inj_b, absorb=self.absorb)
        self.psi0[idx] = psi_b[:, -1]
        it_b = torch.zeros(nbad, dtype=torch.int32, device=self.dev)
        res_b = torch.zeros(nbad, dtype=torch.float64, device=self.dev)
        ss.ss_refine_psi(ctx, self.Hd, self.Hu, self.Sd, self.Su, E_b, q, sig_b, inj_b, psi_b, kidx=k_b,
                         tol=self.refine_tol, iters=it_b, resid=res_b)
        self.psi[idx] = psi_b
        self.gc[idx] = gc_b  # the Caroli T of these instances also comes from the FP64 factors
        self.info_o[idx] = info_ob
        self.ir_iters[idx] = it_b
        self.ir_resid[idx] = res_b


def run_spike(args):
    """Step 1 for a small batch (the first --spike-batch instances of the workload) with the plain
    recursion and through 2, 4, 8, 16 partitions merged by SPIKE: wall time per call and Q against the
    plain recursion's."""
    import torch

    import paper_1812_01396_amd as ss

    w, insts, E_np, kidx_np, _ = build_inputs(args.workload)
    nb, s = w["nb"], w["s"]
    dev = torch.device("cuda", 0)

    def t(a, dt=torch.complex128):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)

    hd, hu, sd, su = (t(np.stack([getattr(i, f) for i in insts])) for f in ("Hd", "Hu", "Sd", "Su"))
    nbat = min(args.spike_batch, len(E_np))
    E = t(E_np[:nbat], torch.float64)
    kidx = t(kidx_np[:nbat], torch.int32)
    ctx = ss.Context(0)
    q_ref, _ = ss.ss_precompute_columns(ctx, hd, hu, sd, su, E, kidx=kidx, absorb=w["absorb"])
    q = torch.empty_like(q_ref)
    rows = []
    for p in [1, 2, 4, 8, 16]:
        if p > nb:
            break
        def call():
            if p == 1:
                ss.ss_precompute_columns(ctx, hd, hu, sd, su, E, kidx=kidx, Q=q, absorb=w["absorb"], validate=False)
            else:
                ss.ss_precompute_columns_spike(ctx, hd, hu, sd, su, E, p, kidx=kidx, Q=q, absorb=w["absorb"])
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        err = float(((q - q_ref).reshape(nbat, -1).norm(dim=1) / q_ref.reshape(nbat, -1).norm(dim=1)).max())
        f = nbat * sweep_flops(nb, s) + (nbat * 16.0 * nb * s**3 * np.log2(p) if p > 1 else 0.0)
        rows.append(dict(nparts=p, ms=round(ms, 3), solves_per_s=round(nbat / (ms * 1e-3), 3),
                         tflops=round(f / (ms * 1e-3) / 1e12, 3), q_rel_diff_vs_plain=err))
    ctx.close()
    best = min(rows, key=lambda r: r["ms"])
    out = {"metric": "(E,k) Step-1 solves/sec, small batch", "value": best["solves_per_s"], "unit": "solves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": args.workload + "-spike", "s": s, "nb": nb, "instances": nbat,
                      "absorb": w["absorb"], "best_nparts": best["nparts"]},
           "partitions": rows, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def compare_precisions(workload: str, steps: int = 1, warmup: int = 1, modes=("fp64", "mixed", "mixed-bf16")):
    """One timed step of `workload` in plain FP64 and in the two mixed forms (the block formations and the
    chain with FP32 products, or with BF16-term products on the BF16 matrix cores; FP64 refinement of
    psi, T from the refined psi with the broadening tail), each after `warmup` untimed steps: solves/s and
    T against the stored oracle values, so that every default benchmark line carries the
    plain-FP64-versus-mixed comparison of the same configuration."""
    import gc

    import torch

    res = {}
    for mode in modes:
        print(f"{workload} {mode}: building the pipeline", file=sys.stderr, flush=True)
        pipe = Pipeline(workload, mode=mode)
        for _ in range(warmup):
            pipe.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pipe.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        T = pipe.T.cpu().numpy() if mode == "fp64" else np.stack([pipe.T_psi.cpu().numpy()] * 2, axis=1)
        rec = dict(solves_per_s=round(pipe.n * steps / dt, 3), ms_per_step=round(dt * 1e3 / steps, 1),
                   instances=pipe.n, t_err_all=golden_errors(workload, T))
        if mode != "fp64":
            it = pipe.ir_iters.cpu().numpy()
            rec.update(refine_iters=[int(it.min()), int(it.max())],
                       refine_resid_max=float(pipe.ir_resid.max().item()), fp64_fallback=pipe.fallback)
        res[mode] = rec
        pipe.close()
        for k in list(vars(pipe)):
            setattr(pipe, k, None)
        del pipe
        gc.collect()
        torch.cuda.empty_cache()
    res["config"] = dict(workload=workload, steps=steps, warmup=warmup)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dft512", choices=sorted(WORKLOADS) + ["uneven256", "learned"])
    ap.add_argument("--no-graph", action="store_true", help="uneven256: enqueue eagerly instead of a graph replay")
    ap.add_argument("--no-autotune", action="store_true", help="uneven256: default panel widths and chunks")
    ap.add_argument("--plan-mem-gib", type=float, default=0.0,
                    help="uneven256: chunk work memory (0: the device memory left after the inputs, less 4 GiB)")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "mixed", "mixed-lu", "mixed-bf16"],
                    help="mixed: FP32 products in the block formations and the chain; mixed-lu: also in the LU; "
                         "mixed-bf16: those of mixed from BF16 terms on the BF16 matrix cores")
    ap.add_argument("--absorb", type=float, default=-1.0,
                    help="absorbing boundary of Step 1 (i*absorb*I on the first and last diagonal blocks; 0: the "
                         "closed A = E S - H; negative: the workload's default)")
    ap.add_argument("--chunk", type=int, default=0, help="instances per Q buffer (0: workload default)")
    ap.add_argument("--lu-tile", type=int, default=0, choices=[0, 1],
                    help="tile of the LU's general block products: 0 64 x 64, 1 32 x 64")
    ap.add_argument("--lanes", type=int, default=1,
                    help="split the instances into this many lanes, each with its own context, stream and host "
                         "thread (the refinement's latency-bound tail of one lane overlaps the others' work)")
    ap.add_argument("--refine-tol", type=float, default=1e-10, help="mixed: relative residual the refinement stops at")
    ap.add_argument("--m-inj", type=int, default=0, help="mixed: columns of the injection factor (0: workload's m)")
    ap.add_argument("--roofline-kernel", default="lu_gemm",
                    help="kernel family timed with HIP events for the roofline entry")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (a plain copy of known size, for "
                         "calibrating the FETCH_SIZE and WRITE_SIZE counters)")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure this GPU's FP64/FP32 matrix-core, FP64 vector and copy rates")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra untimed passes that time the recursion (for profiler runs)")
    ap.add_argument("--summarize-trace", default=None, metavar="PATH",
                    help="only print a per-kernel summary of a rocprofv3 kernel trace (*_results.db or "
                         "*kernel_trace.csv) and exit (no GPU needed)")
    ap.add_argument("--trace-steps", type=int, default=1, help="--summarize-trace: steps the trace covers")
    ap.add_argument("--sq-report", nargs="+", default=None, metavar="CSV",
                    help="summarise rocprofv3 --pmc counter CSVs (SQ and GRBM counters) per kernel family and exit")
    ap.add_argument("--traffic-report", nargs=8, default=None,
                    metavar=("FAMILY", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "QUEUE",
                             "ALG_BYTES", "COMMANDS"),
                    help="only print the HBM-traffic summary of a kernel family from rocprofv3 counter CSVs "
                         "(no GPU needed)")
    ap.add_argument("--compare-precisions", action=argparse.BooleanOptionalAction, default=True,
                    help="after the default dft512 line's step, time the s = 1024 workload once in plain FP64 "
                         "and once in mixed precision and add both to the line (precision_comparison)")
    ap.add_argument("--spike-batch", type=int, default=0,
                    help="time Step 1 for this many instances with the plain recursion and through 2-16 SPIKE "
                         "partitions (small batches) and exit")
    ap.add_argument("--cpu-sample", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.trace_steps))
        if not args.summarize_trace.endswith(".db"):
            for name, pat in (("k_lu_gemm", r"k_lu_gemm<"), ("k_dec_update", r"k_dec_update")):
                for q, (n, avg) in trace_queue_stats(args.summarize_trace, pat).items():
                    print(f"# {name} on queue {q}: {n} launches, average {avg:.1f} us")
        return
    if args.sq_report:
        print(sq_report(args.sq_report))
        return
    if args.traffic_report:
        fam, fcsv, wcsv, cfcsv, cwcsv, q, alg, cmds = args.traffic_report
        print(traffic_report(fam, args.workload, fcsv, wcsv, cfcsv, cwcsv, int(q), float(alg), cmds), end="")
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: run with --gpus 1 (the library has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.ceilings:
        import paper_1812_01396_amd as ss
        ctx = ss.Context(0)
        print(json.dumps(dict(ceilings=ctx.measure_ceilings(),
                              datasheet=dict(fp64_mfma_tflops=FP64_PEAK_TFLOPS, fp32_mfma_tflops=FP32_PEAK_TFLOPS,
                                             fp64_valu_tflops=78.6, hbm_gbps=8000.0))))
        ctx.close()
        return
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "launches": 3}))
        return
    if args.spike_batch > 0:
        return run_spike(args)
    if args.workload == "uneven256":
        return run_uneven(args)
    if args.workload == "learned":
        return run_learned(args)
    pipe = Pipeline(args.workload, args.chunk, args.mode, absorb=None if args.absorb < 0 else args.absorb,
                    refine_tol=args.refine_tol, m=args.m_inj, lanes=args.lanes, lu_tile=args.lu_tile)
    w, s, nb, m, nbatch = pipe.w, pipe.w["s"], pipe.w["nb"], pipe.w["m"], pipe.n
    fam = args.roofline_kernel
    timed_ctx = pipe.ctx_s if fam in ("dec_update",) else pipe.ctx

    for _ in range(args.warmup):
        pipe.run()
    torch.cuda.synchronize()
    timed_ctx.kernel_timer(fam)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_launches, k_flops, k_bytes = timed_ctx.kernel_timer_read(with_flops=True)
    timed_ctx.kernel_timer(None)
    # one more (untimed) step with the recursion's kernels bracketed by HIP events: recursion TFLOP/s
    rec_ms, rec_alone_wall, rec_alone_kms = [], None, None
    obs = None
    fam_alone = None
    if not args.no_extra:
        pipe.run(recursion_ms=rec_ms)
        torch.cuda.synchronize()
        rec_alone_wall, rec_alone_kms = pipe.recursion_alone()
        if fam in ("lu_gemm", "form", "chain", "panel", "trsm"):
            # the roofline kernel's launches in Step 1 run by itself: the same family, nothing beside it
            _, a_ms, a_n, a_flops = pipe.recursion_alone(fam, with_flops=True)
            if a_n > 0 and a_flops > 0:
                fam_alone = (a_ms, a_n, a_flops)
        obs = pipe.observables()

    rec_inst = min(pipe.chunk, nbatch) if pipe.lanes > 1 else nbatch
    it_np = pipe.iters.cpu().numpy().astype(np.float64)
    mixed = args.mode != "fp64"
    # the product's T: Caroli (T_LR, T_RL) in fp64 mode; T carried by the refined psi in mixed mode
    T_np = pipe.T.cpu().numpy()
    if mixed:
        T_np = np.stack([pipe.T_psi.cpu().numpy()] * 2, axis=1)
    bad = int((pipe.info_s.cpu() != 0).sum() + (pipe.info_q.cpu() != 0).sum() + (pipe.info_o.cpu() != 0).sum())
    ms_per_step = elapsed * 1e3 / args.steps
    value = nbatch * args.steps / elapsed

    # algorithmic flops of one step
    f_step = nbatch * sweep_flops(nb, s) + dec_flops(s, float(it_np.sum())) + nbatch * obc_flops(nb, s, m)
    fam_flops = {
        "dec_update": args.steps * 32.0 * s**3 * float(it_np.sum()),
        "form": args.steps * nbatch * 2 * (nb - 1) * 8.0 * s**3,
        "chain": args.steps * nbatch * 2 * (nb - 1) * 8.0 * s**3,
        "lu_gemm": k_flops,  # stated per launch by the library (8 m n k per complex product)
    }
    roof = None
    if k_launches > 0 and fam in fam_flops:
        achieved = fam_flops[fam] / (k_ms * 1e-3) / 1e12
        peak = FP32_PEAK_TFLOPS if (mixed and fam in ("form", "chain")) else FP64_PEAK_TFLOPS
        traffic = measured_traffic(fam, args.workload) if not mixed else None
        roof = dict(bound="mfma", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=traffic, kernel=fam,
                    launches=int(k_launches), avg_launch_ms=round(k_ms / k_launches, 4))
        if k_bytes > 0:
            roof["algorithmic_bytes"] = k_bytes / k_launches
        if fam_alone is not None:
            # the same kernel family in Step 1 run by itself after the timed steps (the frac above is
            # inside the step, where the self-energy stream shares the matrix cores)
            a_ms, a_n, a_flops = fam_alone
            a_ach = a_flops / (a_ms * 1e-3) / 1e12
            roof["alone"] = dict(achieved=round(a_ach, 3), frac=round(a_ach / peak, 4), launches=int(a_n),
                                 avg_launch_ms=round(a_ms / a_n, 4), scope="Step 1 by itself")

    cpu = None
    t_err = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        cpu, t_err = cpu_baseline(w, pipe.insts, pipe.E_np, pipe.kidx_np, pipe.inj_np, args.cpu_sample, T_np)

    out = {
        "metric": "(E,k) solves/sec",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": args.workload, "s": s, "nb": nb, "instances": nbatch, "energies": w["n_e"],
                   "k_points": len(w["ks"]), "m_inj": m, "eta": w["eta"], "chunk": pipe.chunk,
                   "precision": args.mode, "absorb": pipe.absorb, "lanes": pipe.lanes},
        "tflops_step": round(f_step / (ms_per_step * 1e-3) / 1e12, 3),
        "frac_fp64_peak_step": round(f_step / (ms_per_step * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
        "decimation_iters": [int(it_np.min()), int(it_np.max()), round(float(it_np.mean()), 2)],
        "nonzero_info": bad,
        # Caroli T_LR - T_RL (fp64 mode; in mixed mode the Caroli pair comes from FP32-product columns and the
        # product's T is the refined psi's)
        "t_lr_minus_t_rl_max": (None if mixed else
                                float(np.abs(pipe.T.cpu().numpy()[:, 0] - pipe.T.cpu().numpy()[:, 1]).max())),
        "refine_iters": ([int(pipe.ir_iters.min()), int(pipe.ir_iters.max())] if mixed else None),
        "refine_resid_max": (float(pipe.ir_resid.max()) if mixed else None),
        "fp64_fallback_per_step": (pipe.fallback / (args.steps + args.warmup) if mixed else None),
        "injection_rank": ([int(pipe.rank.min()), int(pipe.rank.max())] if mixed else None),
        "roofline": roof,
        # the recursion's algorithmic flops / the summed duration of its kernels (form, chain, LU) in one
        # step, measured with HIP events while the self-energies run beside it on the second stream
        "observables": obs,
        "recursion": None if args.no_extra else dict(kernel_ms=round(sum(rec_ms), 2),
                          # with lanes, the timed recursion is lane 0's (pipe.chunk instances)
                          instances_timed=rec_inst,
                          tflops=round(rec_inst * sweep_flops(nb, s) / (sum(rec_ms) * 1e-3) / 1e12, 3),
                          frac_peak=round(rec_inst * sweep_flops(nb, s) / (sum(rec_ms) * 1e-3) / 1e12 /
                                          (FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS), 4),
                          # Step 1 run by itself after the timed steps (nothing beside it on the chip)
                          alone_wall_ms=round(rec_alone_wall, 2), alone_kernel_ms=round(rec_alone_kms, 2),
                          alone_tflops=round(nbatch * sweep_flops(nb, s) / (rec_alone_wall * 1e-3) / 1e12, 3),
                          alone_frac_peak=round(nbatch * sweep_flops(nb, s) / (rec_alone_wall * 1e-3) / 1e12 /
                                                (FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS), 4)),
        "cpu_baseline": cpu,
        "t_err_vs_oracle": t_err,
        # |T - T_oracle| / max(1, T_oracle) over every instance against the stored oracle values
        "t_err_all": golden_errors(args.workload, T_np),
        "device_mem_used_gib": round((torch.cuda.mem_get_info()[1] - torch.cuda.mem_get_info()[0]) / 2**30, 1),
    }
    if args.compare_precisions and args.workload == "dft512" and args.mode == "fp64":
        # release this workload's device memory, then the s = 1024 workload in the three precisions and this
        # workload in the BF16-mixed form
        pipe.close()
        for k in list(vars(pipe)):
            setattr(pipe, k, None)
        del pipe
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        try:
            out["precision_comparison"] = compare_precisions("dft1024")
        except Exception as e:  # reported, never fatal for the headline line
            out["precision_comparison"] = {"error": f"{type(e).__name__}: {e}"}
        try:  # the mixed form of this same workload, against the plain FP64 headline above
            out["mixed_same_workload"] = compare_precisions("dft512", steps=args.steps, modes=("mixed-bf16",))
        except Exception as e:
            out["mixed_same_workload"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
