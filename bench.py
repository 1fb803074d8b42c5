#!/usr/bin/env python3
"""EOFA hot-path benchmark on one MI355X.

One step is one pass of the whole hot path on the 24^3x64, Ls = 24
workload (the shape of the paper's 24ID ensemble, Table 1; synthetic random
SU(3) links, eps = 0.5): both EOFA solves in the Cayley form with even-odd
CGNR to a true residual of 1e-10 (mixed precision: low-precision inner
operator, FP64 reductions and reliable updates), the EOFA action, the
eq. (3.2) force from the two solutions, and a leapfrog momentum/link update
followed by the re-ingest of the new links.  Each step starts from the same
links and momenta (restored and re-ingested inside the timed region), so
every step does the same work and the FP64 reference solves the same
system as the mixed-precision one.

Printed: one JSON line with the sustained operator rate (GFLOP/s counted
with 1320 flops per Wilson hop per 5D site, 72 per bidiagonal 5D op, 144
per inverse 5D op), the roofline of the dominant kernel (the 5D hopping
kernel, measured with HIP events inside the timed region), the FP64-solver
reference time on the same GPU, and the CPU oracle's operator rate on a
bounded sample.

Other modes, each printing its own JSON line instead:
  --dslash      the hopping kernel's rate in all four precisions
  --trajectory  the 24^3x64 leapfrog trajectory, mixed vs FP64 (dH, reversibility)
  --heatbath    the eq. (3.1) heatbath: Lanczos interval, Zolotarev poles, 2 N_p solves
  --hmc         one full trajectory (heatbath, force-gradient MD, energies) by phase;
                --gauge-beta adds the Iwasaki gauge action on an inner time scale;
                --trajectories N runs a chain with M_EOFA's interval reused
  --gauge       the gauge force and action kernels (Iwasaki and Wilson)
  --dense       the EOFA solves on D_EOFA itself against the Cayley form (Table 4)
  --cpu-baselines  the CPU oracle's operator rates and solve times per workload beside the GPU's
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("dslash GFLOP/s & % HBM roofline; EOFA solve time to 1e-10, mixed vs FP64 (1 GPU)")
HBM_PEAK_GBS = 8000.0
FLOPS_DDWF = 1320 + 72 + 72 + 24   # one D_DWF application per 5D site (convention above)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 of the sources that define the hopping kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in ("dslash.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_1611_00298_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def plaquette(ctx, U):
    """Average plaquette Re tr U_P / 3 of the links U, from the Wilson gauge
    action on the GPU: S_W = beta sum_x sum_{mu<nu} (1 - Re tr U_P / 3)."""
    L = ctx.L
    return 1.0 - ctx.gauge_action(U, 1.0, 0.0) / (6.0 * L[0] * L[1] * L[2] * L[3])


def measured_traffic(inner, workload):
    """HBM bytes per launch of the hopping kernel from the committed
    rocprofv3 summary (read and write requests counted by size, see
    profile_summary), or None if there is none or the kernel sources changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"k_hop_{inner}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# kernel-name prefixes of the hopping kernel per inner precision (the last
# template argument, the block-sharing variant, is left open)
HOP_TEMPLATE = {"fp64": "k_hop<0, {}, true, 0, false,", "fp32": "k_hop<1, {}, true, 0, false,",
                "fp16": "k_hop<2, {}, true, 3, false,", "bf16": "k_hop<3, {}, true, 3, false,"}


def profile_summary(args):
    """Summarise rocprofv3 --pmc runs of this benchmark (default mode) per
    launch of the hopping kernel, split into its four forms by position: in
    the CG iteration the hop runs as K1, K2 (not daggered) then K3, K4
    (daggered), so in the dispatch sequence each run of same-direction hop
    launches pairs up as (K1, K2) or (K3, K4).  Read bytes are counted from
    the L2-to-memory read requests by size (128, 64, 32 bytes) and write
    bytes from the write requests (64 or 32 bytes); the elementwise kernel of
    --copy-calibration (2 GiB read, 2 GiB written) checks the counting.
    Prints a text summary for profiles/."""
    import csv
    import glob
    import collections
    import dwf_inputs as din
    pre = din.preset(args.workload)
    Lx, Ly, Lz, Lt = pre["L"]
    Vh = Lx * Ly * Lz * Lt // 2
    n5 = Vh * pre["Ls"]
    sb = {"fp64": 192, "fp32": 96, "fp16": 52, "bf16": 48}[args.inner]
    cb = {"fp64": 16, "fp32": 8, "fp16": 4, "bf16": 4}[args.inner]
    links = 72.0 * cb * Vh
    alg = {"K1": 2 * sb * n5 + links, "K2": 3 * sb * n5 + links, "K3": 2 * sb * n5 + links,
           "K4": 4 * sb * n5 + links}
    hop = {HOP_TEMPLATE[args.inner].format("false"): False, HOP_TEMPLATE[args.inner].format("true"): True}
    disp = collections.defaultdict(dict)   # dispatch id -> counters
    name = {}
    for d in args.profile_summary:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                key = (f, int(r["Dispatch_Id"]))
                disp[key][r["Counter_Name"]] = float(r["Counter_Value"])
                name[key] = r["Kernel_Name"]
        # kernel traces: the duration of each dispatch as a pseudo-counter
        for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                key = (f, int(r["Dispatch_Id"]))
                disp[key]["duration_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                name[key] = r["Kernel_Name"]
    cls = collections.defaultdict(lambda: collections.defaultdict(list))
    calib = collections.defaultdict(list)
    for f in sorted({k[0] for k in disp}):
        keys = sorted(k for k in disp if k[0] == f)
        run, prev = [], None
        for k in keys:
            kn = name[k]
            if "elementwise" in kn:
                calib["all"].append(disp[k])
                continue
            tmpl = next((t for t in hop if t in kn), None)
            if tmpl is None:
                continue
            dag = hop[tmpl]
            if prev is not None and dag != prev:
                run = []
            run.append(k)
            if len(run) == 2:
                for pos, kk in enumerate(run):
                    c = ("K3", "K4")[pos] if dag else ("K1", "K2")[pos]
                    for cn, v in disp[kk].items():
                        cls[c][cn].append(v)
                run = []
            prev = dag
    def rd(c):
        return 128 * c.get("TCC_EA0_RDREQ_128B_sum", 0) + 64 * c.get("TCC_EA0_RDREQ_64B_sum", 0) + \
            32 * c.get("TCC_EA0_RDREQ_32B_sum", 0)
    def wr(c):
        return 64 * c.get("TCC_EA0_WRREQ_64B_sum", 0) + 32 * (c.get("TCC_EA0_WRREQ_sum", 0) -
                                                              c.get("TCC_EA0_WRREQ_64B_sum", 0))
    avg = lambda xs: sum(xs) / len(xs) if xs else float("nan")
    lines = [f"# {HOP_TEMPLATE[args.inner].format('*')} *> (the {args.inner} hopping kernel), bench.py, "
             f"{Lx}x{Ly}x{Lz}x{Lt}, Ls={pre['Ls']}, per launch",
             "# read bytes = 128 TCC_EA0_RDREQ_128B + 64 TCC_EA0_RDREQ_64B + 32 TCC_EA0_RDREQ_32B;",
             "# write bytes = 64 TCC_EA0_WRREQ_64B + 32 (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B)  (no calibration factor)"]
    cal_r = [rd(c) for c in calib["all"] if "TCC_EA0_RDREQ_128B_sum" in c and rd(c) > 1e9]
    cal_w = [wr(c) for c in calib["all"] if "TCC_EA0_WRREQ_sum" in c and wr(c) > 1e9]
    if cal_r or cal_w:
        lines.append("# check on the 2 GiB elementwise kernels of --copy-calibration: read " +
                     ", ".join(f"{v / 2**30:.3f}" for v in cal_r[:6]) + " GiB; written " +
                     ", ".join(f"{v / 2**30:.3f}" for v in cal_w[:6]) + " GiB")
    tot_n = tot_r = tot_w = tot_a = 0.0
    rows = []
    for c in ("K1", "K2", "K3", "K4"):
        cs = cls[c]
        if not cs:
            continue
        n = max(len(v) for v in cs.values())
        m = {cn: avg(v) for cn, v in cs.items()}
        have_rd = "TCC_EA0_RDREQ_128B_sum" in m
        have_wr = "TCC_EA0_WRREQ_sum" in m
        r_, w_ = rd(m), wr(m)
        rows.append((c, n, m, r_ if have_rd else None, w_ if have_wr else None))
        if have_rd and have_wr:
            tot_n += n
            tot_r += n * r_
            tot_w += n * w_
            tot_a += n * alg[c]
    lines.append("kernel_source_sha256: " + kernel_source_hash())
    if tot_n:
        lines += [f"launches: {int(tot_n)}", f"fetch_bytes_per_launch: {tot_r / tot_n:.0f}",
                  f"write_bytes_per_launch: {tot_w / tot_n:.0f}",
                  f"algorithmic_bytes_per_launch: {tot_a / tot_n:.0f}",
                  f"measured_over_algorithmic: {(tot_r + tot_w) / tot_a:.3f}"]
    durs = [(n, m["duration_us"]) for c, n, m, r_, w_ in rows if "duration_us" in m]
    if durs:
        nd = sum(n for n, _ in durs)
        avg_us = sum(n * d for n, d in durs) / nd
        a_avg = sum(n * alg[c] for c, n, m, r_, w_ in rows if "duration_us" in m) / nd
        lines.append(f"trace: {int(nd)} launches, average {avg_us:.1f} us, algorithmic {a_avg / 1e9:.3f} GB "
                     f"per launch: {a_avg / (avg_us * 1e-6) / 1e9:.0f} GB/s = "
                     f"{a_avg / (avg_us * 1e-6) / 8e12:.3f} of 8 TB/s")
    for c, n, m, r_, w_ in rows:
        a_read = alg[c] - sb * n5
        txt = f"{c}: launches {n}, algorithmic {alg[c] / 1e9:.3f} GB (reads {a_read / 1e9:.3f})"
        if "duration_us" in m:
            txt += f", {m['duration_us']:.1f} us ({alg[c] / (m['duration_us'] * 1e-6) / 1e9:.0f} GB/s)"
        if r_ is not None:
            txt += f", read {r_ / 1e9:.3f} GB ({r_ / a_read:.2f}x)"
        if w_ is not None:
            txt += f", written {w_ / 1e9:.3f} GB ({w_ / (sb * n5):.2f}x)"
        w = m.get("SQ_WAVES")
        if w:
            parts = [f"{k.replace('SQ_INSTS_', '')} {m[k] / w:.0f}" for k in
                     ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_LDS",
                      "SQ_INSTS_SALU") if k in m]
            txt += "; instructions per wave: " + ", ".join(parts)
        if "SQ_WAVE_CYCLES" in m and "SQ_WAIT_ANY" in m:
            txt += f"; waves waiting {m['SQ_WAIT_ANY'] / m['SQ_WAVE_CYCLES']:.0%} of their cycles"
            if "SQ_WAIT_INST_ANY" in m:
                txt += f" (on dependencies {m['SQ_WAIT_INST_ANY'] / m['SQ_WAVE_CYCLES']:.0%})"
        if "SQ_LDS_BANK_CONFLICT" in m and "SQ_INSTS_LDS" in m and w:
            txt += f"; LDS bank-conflict cycles per LDS instruction {m['SQ_LDS_BANK_CONFLICT'] / max(m['SQ_INSTS_LDS'], 1):.2f}"
        g = m.get("GRBM_GUI_ACTIVE")
        if g:
            cyc = g / 8.0   # summed over the 8 XCDs
            for k, lab in (("TA_TA_BUSY_sum", "TA busy"), ("TD_TD_BUSY_sum", "TD busy"),
                           ("TD_TC_STALL_sum", "TD stalled on L1"),
                           ("TCP_PENDING_STALL_CYCLES_sum", "L1 stalled on pending L2 data")):
                if k in m:
                    txt += f"; {lab} {m[k] / (256 * cyc):.0%}"
            if "TCP_TCC_READ_REQ_LATENCY_sum" in m and "TCP_TCC_READ_REQ_sum" in m:
                txt += (f"; L2 read latency {m['TCP_TCC_READ_REQ_LATENCY_sum'] / m['TCP_TCC_READ_REQ_sum']:.0f} "
                        f"cycles with {m['TCP_TCC_READ_REQ_LATENCY_sum'] / (256 * cyc):.0f} reads outstanding per CU"
                        f" ({m['TCP_TCC_READ_REQ_sum'] * 128 / 1e9:.2f} GB L1->L2)")
        if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m:
            txt += f"; L2 hit rate {m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.0%}"
        lines.append(txt)
    print("\n".join(lines))
    return 0


def copy_calibration(dev):
    """Known-size references for the FETCH_SIZE / WRITE_SIZE counters: each
    of the three rounds runs a 2 GiB device-to-device copy (the runtime's
    copy kernel) and a 2 GiB elementwise kernel (y = 1 * x, ordinary vector
    loads and stores like the library's kernels); each reads and writes 2 GiB."""
    import torch
    x = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del x, y


def elementwise_reference(dev):
    """Best of 3 timed 2 GiB elementwise kernels (y = 1 * x): the HBM rate
    a plain streaming kernel reaches on this GPU (read + write bytes / time)."""
    import torch
    x = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.mul(x, 1.0, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    return 2 * 2 * 1024**3 / (best * 1e-3) / 1e9


def cpu_baseline(pre, seconds=12.0):
    """The oracle's D_DWF on a slab of the workload's lattice (all of
    Lx, Ly, Lz and Ls, first 4 time slices), repeated for ~`seconds`."""
    import numpy as np
    import dwf_inputs as din
    import oracle
    Lx, Ly, Lz, Lt = pre["L"]
    L = (Lx, Ly, Lz, 4)
    lat = oracle.Lattice(L, pre["Ls"], M5=pre["M5"], alpha=pre["alpha"])
    U = din.random_gauge(L, pre["eps"], pre["seed_gauge"])
    psi = din.gaussian_5d(L, pre["Ls"], 7)
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.ddwf(lat, U, pre["m1"], pre["m1"], psi)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    flops = n * lat.V * lat.Ls * FLOPS_DDWF
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} x oracle D_DWF on a {Lx}x{Ly}x{Lz}x4 slab, Ls={pre['Ls']} "
                      f"({dt:.1f} s, FP64, OpenMP)"}


def cpu_baselines(args):
    """The CPU oracle on this machine's host cores beside the GPU library, per
    workload: the D_DWF and Mhat^dag Mhat rates at 4^4x8 (c1), 16^3x32x16
    (c2) and 24^3x64x24 (c3); the full FP64 EOFA solve of both systems
    (even-odd CGNR in the Cayley form, to 1e-10) at c1, and at c2 its time
    estimated from 20 timed oracle iterations, next to the GPU's FP64 and
    FP16-inner solves of the same systems; and at c3, where a CPU solve
    would take hours, the oracle's recomputation of the GPU solution's true
    residual |v - H chi| / |v|.  Flops: 1488 per 5D site
    for D_DWF and 3024 per odd 5D site for each Mhat.  Prints one JSON line."""
    import numpy as np
    import torch
    import dwf_inputs as din
    import oracle
    from paper_1611_00298_amd import Context
    dev = torch.device("cuda:0")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"metric": "CPU oracle (FP64, OpenMP) beside the GPU: operator rates and EOFA solve times",
           "cores": threads, "workloads": {}}

    def rate(fn, flops, min_s=1.0):
        n, t0 = 0, time.perf_counter()
        while True:
            fn()
            n += 1
            dt = time.perf_counter() - t0
            if dt >= min_s:
                return n * flops / dt / 1e9, dt / n

    for w in ("c1", "c2", "c3"):
        pre = din.preset(w)
        L, Ls, m1, m2 = pre["L"], pre["Ls"], pre["m1"], pre["m2"]
        log(f"cpu baselines: {w} {L} Ls={Ls}")
        lat = oracle.Lattice(L, Ls, M5=pre["M5"], alpha=pre["alpha"])
        U = din.random_gauge(L, pre["eps"], pre["seed_gauge"])
        phi = din.gaussian_4d(L, pre["seed_phi"])
        psi = din.gaussian_5d(L, Ls, 303)
        n5 = lat.V * Ls
        r = {}
        g, sec = rate(lambda: oracle.ddwf(lat, U, m1, m1, psi), n5 * FLOPS_DDWF)
        r["oracle_ddwf"] = {"GFLOPs": g, "seconds": sec}
        odd = (lat.parity_mask() == 1)[None, ..., None, None]
        po = psi * odd
        g, sec = rate(lambda: oracle.schur(lat, U, m1, m2, oracle.schur(lat, U, m1, m2, po), dagger=True),
                      2 * 3024 * n5 / 2)
        r["oracle_mhat_dag_mhat"] = {"GFLOPs": g, "seconds": sec}
        del psi, po
        ctx = Context(L, Ls, torch.from_numpy(U).to(dev), M5=pre["M5"], alpha=pre["alpha"])
        ph = torch.from_numpy(phi).to(dev)
        ctx.eofa_solve(ph, m1, m2, tol=1e-10, inner="fp16", want_mphi=False)   # warm-up
        gpu = {}
        for inner in ("fp64", "fp16"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chiL, chiR, _, S, st = ctx.eofa_solve(ph, m1, m2, tol=1e-10, inner=inner, want_mphi=False)
            torch.cuda.synchronize()
            gpu[inner] = {"seconds": time.perf_counter() - t0, "iters": st["iters"], "S": S,
                          "true_resid": st["true_resid"]}
        r["gpu_solve"] = gpu
        if w == "c1":
            t0 = time.perf_counter()
            cL, cR, its = oracle.eofa_chi(lat, U, m1, m2, phi, tol=1e-10)
            t_orc = time.perf_counter() - t0
            S_orc, _, _ = oracle.action(lat, m1, m2, phi, cL, cR)
            r["oracle_solve"] = {"seconds": t_orc, "iters": [int(v) for v in its], "S": S_orc,
                                 "S_rel_vs_gpu_fp64": abs(S_orc - gpu["fp64"]["S"]) / abs(S_orc),
                                 "gpu_fp64_speedup": t_orc / gpu["fp64"]["seconds"],
                                 "gpu_fp16_speedup": t_orc / gpu["fp16"]["seconds"]}
            log(f"cpu baselines: {w}: oracle solve {t_orc:.1f} s, GPU FP64 {gpu['fp64']['seconds']:.2f} s, "
                f"FP16 {gpu['fp16']['seconds']:.2f} s")
        elif w == "c2":
            # a full CPU solve here takes tens of minutes: time 20 iterations of
            # the oracle's CGNR (the same iteration as the GPU's FP64 solver)
            # and scale by the GPU's FP64 iteration count, stated as an estimate
            om_m, _, _ = oracle.omega_k(lat, m1, m2)
            v = lat.zeros5()
            v[..., 2:, :] = om_m[:, None, None, None, None, None, None] * phi[None, ..., 2:, :]
            b = oracle.g5r5(lat, v)
            t0 = time.perf_counter()
            oracle.solve_ddwf_eo(lat, U, m1, m1, b, fixed=20)
            per_it = (time.perf_counter() - t0) / 20
            n_it = sum(gpu["fp64"]["iters"])
            r["oracle_solve_estimate"] = {"seconds_per_iteration": per_it, "iterations": n_it,
                                          "seconds": per_it * n_it,
                                          "gpu_fp64_speedup": per_it * n_it / gpu["fp64"]["seconds"],
                                          "gpu_fp16_speedup": per_it * n_it / gpu["fp16"]["seconds"],
                                          "how": "20 oracle CGNR iterations timed, times the GPU FP64 "
                                                 "solve's iteration count (both systems)"}
            log(f"cpu baselines: {w}: oracle {per_it:.2f} s per iteration, ~{per_it * n_it:.0f} s for "
                f"{n_it} iterations; GPU FP64 {gpu['fp64']['seconds']:.2f} s, FP16 {gpu['fp16']['seconds']:.2f} s")
            del v, b
        else:
            om_m, _, _ = oracle.omega_k(lat, m1, m2)
            v = lat.zeros5()
            v[..., 2:, :] = om_m[:, None, None, None, None, None, None] * phi[None, ..., 2:, :]
            t0 = time.perf_counter()
            res = float(np.linalg.norm(oracle.H_op(lat, U, m1, m1, chiL.cpu().numpy()) - v) / np.linalg.norm(v))
            r["oracle_residual_check"] = {"seconds": time.perf_counter() - t0, "resid_L": res,
                                          "gpu_resid_L": gpu["fp16"]["true_resid"][0]}
            del v
        ctx.close()
        del ctx, ph
        torch.cuda.empty_cache()
        out["workloads"][w] = r
        log(f"cpu baselines: {w}: D_DWF {r['oracle_ddwf']['GFLOPs']:.1f} GFLOP/s, "
            f"MhatdagMhat {r['oracle_mhat_dag_mhat']['GFLOPs']:.1f} GFLOP/s")
    print(json.dumps(out), flush=True)
    return 0


def dslash(args):
    """Operator rates on the 24^3x64, Ls = 24 workload in every precision: the
    even-odd Schur operator Mhat and Mhat^dag (two hopping-kernel launches
    each, K1/K2 and K3/K4 forms) on a Gaussian half field, 10 applications
    per direction after 2 untimed ones, HIP events on the context stream.
    Prints one JSON line with the hopping kernel's average launch time,
    algorithmic bytes and rate per precision against the 8 TB/s peak."""
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import Context

    pre = din.preset(args.workload)
    if args.lattice:
        pre["L"] = tuple(int(v) for v in args.lattice.split(","))
    if args.ls:
        pre["Ls"] = args.ls
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    log(f"dslash: generating {args.workload} inputs {pre['L']} Ls={pre['Ls']}")
    U = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    psi = t(din.gaussian_5d(pre["L"], pre["Ls"], 303))
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    n4 = pre["L"][0] * pre["L"][1] * pre["L"][2] * pre["L"][3] // 2 * pre["Ls"]
    ref_gbs = elementwise_reference(dev)
    out = {"metric": "dslash GFLOP/s & % HBM roofline per precision (1 GPU)",
           "config": {"workload": f"Moebius DWF even-odd Schur operator {'x'.join(map(str, pre['L']))}, "
                                  f"Ls={pre['Ls']}, alpha={pre['alpha']}, M5={pre['M5']}, m={pre['m1']}",
                      "applications": 20},
           "elementwise_ref_GBs": ref_gbs, "precisions": {}}
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        cls = {"fp64": "hop64", "fp32": "hop32", "fp16": "hop16", "bf16": "hopb16"}[prec]
        for dag in (False, True):
            ctx.dwf_apply(psi, pre["m1"], pre["m1"], dagger=dag, eo=True, prec=prec)
        torch.cuda.synchronize()
        ctx.timing_enable(True)
        for _ in range(10):
            for dag in (False, True):
                ctx.dwf_apply(psi, pre["m1"], pre["m1"], dagger=dag, eo=True, prec=prec)
        q = ctx.timing_query(cls)
        ctx.timing_enable(False)
        avg_ms = q["ms"] / q["count"]
        gbs = q["bytes"] / (q["ms"] * 1e-3) / 1e9
        out["precisions"][prec] = {
            "launches": q["count"], "avg_ms": avg_ms, "avg_bytes": q["bytes"] / q["count"],
            "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "frac_of_elementwise_ref": gbs / ref_gbs,
            "hop_gflops": 1320.0 * n4 / (avg_ms * 1e-3) / 1e9}
        log(f"dslash {prec}: {avg_ms:.4f} ms per hop launch, {gbs:.0f} GB/s algorithmic")
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


# FP64 flops of the gauge kernels (3x3 complex product: 27 complex
# multiplications, 6 flops each, and 18 complex additions, 2 flops each = 198;
# Re tr(a b^dag): 36; a scaled or accumulated matrix: 18 or 36)
GAUGE_FORCE_FLOPS = {"iwasaki": 3 * (22 * 198 + 324) + 198 + 60, "wilson": 3 * (4 * 198 + 108) + 198 + 60}
GAUGE_ACTION_FLOPS = {"iwasaki": 6 * (2 * 198 + 36) + 12 * (4 * 198 + 36), "wilson": 6 * (2 * 198 + 36)}
FP64_PEAK_TFLOPS = 78.6


def gauge_cpu_baseline():
    """The oracle's Iwasaki gauge force and action (numpy, loops as step
    lists) on a 24^3x4 slab of the workload's links, beside the GPU kernels
    on the same slab."""
    import numpy as np
    import torch
    import dwf_inputs as din
    import oracle
    from paper_1611_00298_amd import IWASAKI_C1, Context
    L = (24, 24, 24, 4)
    U = din.random_gauge(L, 0.5, 103)
    t0 = time.perf_counter()
    F = oracle.gauge_force(U, 2.13, IWASAKI_C1)
    t_force = time.perf_counter() - t0
    t0 = time.perf_counter()
    S = oracle.gauge_action(U, 2.13, IWASAKI_C1)
    t_action = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    with Context(L, 2, Ud) as ctx:
        Fg = ctx.gauge_force(Ud, 2.13, IWASAKI_C1).cpu().numpy()
        Sg = ctx.gauge_action(Ud, 2.13, IWASAKI_C1)
    nl = 4 * L[0] * L[1] * L[2] * L[3]
    return {"value": nl / t_force, "unit": "links/s (force)", "cores": 1, "kind": "oracle",
            "sample": "Iwasaki force and action on a 24^3x4 slab (numpy, FP64)",
            "force_s": t_force, "action_s": t_action,
            "gpu_vs_oracle": {"F_maxabs_rel": float(np.abs(Fg - F).max() / np.abs(F).max()),
                              "S_rel": abs(Sg - S) / abs(S)}}


def dense_cpu_baseline():
    """The oracle's direct-path operator H = gamma_5 R_5 D_EOFA (FP64, OpenMP),
    which its non-Cayley solve iterates, applied to a 24^3x4, Ls = 24 slab."""
    import numpy as np
    import dwf_inputs as din
    import oracle
    pre = din.preset("c3")
    L = (24, 24, 24, 4)
    lat = oracle.Lattice(L, pre["Ls"], M5=pre["M5"], alpha=pre["alpha"])
    U = din.random_gauge(L, pre["eps"], 103)
    psi = din.gaussian_5d(L, pre["Ls"], 303)
    oracle.H_op(lat, U, pre["m1"], pre["m2"], psi)   # warm-up
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 10.0:
        psi = oracle.H_op(lat, U, pre["m1"], pre["m2"], psi)
        psi /= np.linalg.norm(psi)
        n += 1
    t = (time.perf_counter() - t0) / n
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    scale = 64 / 4
    return {"value": 1e3 * t * scale, "unit": "ms per full-lattice H application (slab time x 16)",
            "cores": threads, "kind": "oracle",
            "sample": f"{n} applications of H = g5 R5 D_EOFA on a 24^3x4, Ls=24 slab (FP64, OpenMP)"}


def gauge(args):
    """The gauge action of Table 1's ensembles (Iwasaki, c1 = -0.331; Wilson,
    c1 = 0) and its force on the workload's links: 20 force and 5 action
    launches per action after 3 untimed ones, HIP events on the context
    stream.  Prints one JSON line with the average launch time, the
    algorithmic HBM rate (links read once, F written once) and the FP64 rate
    of each kernel."""
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import IWASAKI_C1, Context

    pre = din.preset(args.workload)
    dev = torch.device("cuda:0")
    log(f"gauge: generating {args.workload} links")
    U = torch.from_numpy(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"])).to(dev)
    V = pre["L"][0] * pre["L"][1] * pre["L"][2] * pre["L"][3]
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    F = torch.empty_like(U)
    out = {"metric": "gauge force and action: ms per launch, GB/s and FP64 TFLOP/s (1 GPU)",
           "config": {"workload": f"{'x'.join(map(str, pre['L']))} links, beta = 2.13"}, "actions": {}}
    for name, c1 in (("iwasaki", IWASAKI_C1), ("wilson", 0.0)):
        for _ in range(3):
            ctx.gauge_force(U, 2.13, c1, out=F)
            ctx.gauge_action(U, 2.13, c1)
        torch.cuda.synchronize()
        ctx.timing_enable(True)
        for _ in range(20):
            ctx.gauge_force(U, 2.13, c1, out=F)
        S = 0.0
        for _ in range(5):
            S = ctx.gauge_action(U, 2.13, c1)
        res = {"S": S}
        for kern, units, flops in (("gauge_force", 4 * V, GAUGE_FORCE_FLOPS[name]),
                                   ("gauge_action", V, GAUGE_ACTION_FLOPS[name])):
            q = ctx.timing_query(kern)
            ms = q["ms"] / q["count"]
            res[kern] = {"launches": q["count"], "avg_ms": ms,
                         "achieved_GBs": q["bytes"] / q["count"] / (ms * 1e-3) / 1e9,
                         "flops_per_unit": flops,
                         "tflops": units * flops / (ms * 1e-3) / 1e12,
                         "frac_fp64": units * flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}
            log(f"gauge {name} {kern}: {ms:.3f} ms, {res[kern]['tflops']:.1f} TFLOP/s")
        ctx.timing_enable(False)
        out["actions"][name] = res
    ctx.close()
    if not args.no_cpu_baseline:
        log("gauge: CPU oracle baseline")
        out["cpu_baseline"] = gauge_cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


def dense(args):
    """Table 4's comparison at the solve level: the two EOFA systems on the
    workload solved (a) on D_EOFA itself, whose 5D structure is dense (FP64
    even-odd CGNR), (b) in the Cayley form (FP64), (c) in the Cayley form with
    the mixed-precision solver (args.inner), all to the same true residual
    1e-10 of the same systems.  HIP-event timing of the hopping kernels.
    Prints one JSON line."""
    import numpy as np
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import Context

    pre = din.preset(args.workload)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    log(f"dense: generating {args.workload} inputs")
    U = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    phi = t(din.gaussian_4d(pre["L"], pre["seed_phi"]))
    m1, m2 = pre["m1"], pre["m2"]
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    res, sols = {}, {}
    runs = (("dense_fp64", lambda: ctx.eofa_solve_dense(phi, m1, m2, tol=1e-10, want_mphi=False)),
            ("cayley_fp64", lambda: ctx.eofa_solve(phi, m1, m2, tol=1e-10, inner="fp64", want_mphi=False)),
            ("dense_fp32", lambda: ctx.eofa_solve_dense(phi, m1, m2, tol=1e-10, inner="fp32",
                                                        reliable_delta=args.delta, want_mphi=False)),
            ("cayley_fp32", lambda: ctx.eofa_solve(phi, m1, m2, tol=1e-10, inner="fp32",
                                                   reliable_delta=args.delta, want_mphi=False)),
            ("dense_fp16", lambda: ctx.eofa_solve_dense(phi, m1, m2, tol=1e-10, inner="fp16",
                                                        reliable_delta=args.delta, want_mphi=False)),
            (f"cayley_{args.inner}", lambda: ctx.eofa_solve(phi, m1, m2, tol=1e-10, inner=args.inner,
                                                           reliable_delta=args.delta, want_mphi=False)))
    for name, run in runs:
        torch.cuda.synchronize()
        ctx.timing_enable(True)
        t0 = time.perf_counter()
        chiL, chiR, _, S, st = run()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        cls = "hop_dense" if name.startswith("dense") else "hop"
        q = ctx.timing_query(cls)
        ctx.timing_enable(False)
        sols[name] = (chiL, chiR)
        res[name] = {"seconds": sec, "iters": st["iters"], "true_resid": st["true_resid"], "S": S,
                     "hop_launches": q["count"], "hop_ms_per_launch": q["ms"] / max(q["count"], 1),
                     "hop_GBs": q["bytes"] / max(q["ms"], 1e-9) / 1e6,
                     "hop_frac": q["bytes"] / max(q["ms"], 1e-9) / 1e6 / HBM_PEAK_GBS,
                     "ms_per_iteration": 1e3 * sec / max(1, sum(st["iters"]))}
        log(f"dense: {name}: {sec:.2f} s, iters {st['iters']}, resid {st['true_resid']}")
    d = sols["dense_fp64"]
    for name in res:
        a = sols[name]
        res[name]["chi_rel_diff_vs_dense"] = max(
            float(torch.linalg.vector_norm(a[i] - d[i]) / torch.linalg.vector_norm(d[i])) for i in range(2))
    ctx.close()
    out = {"metric": "EOFA solve: dense D_EOFA vs Cayley form (Table 4 columns), seconds to 1e-10, 1 GPU",
           "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                                  f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}: both systems"},
           "data": "synthetic (random SU(3) links exp(i eps H), Gaussian phi)",
           "solves": res,
           }
    # same inner precision on both sides: dense time / Cayley-form time
    for pr in ("fp64", "fp32", "fp16"):
        if f"dense_{pr}" in res and f"cayley_{pr}" in res:
            out[f"cayley_{pr}_speedup"] = res[f"dense_{pr}"]["seconds"] / res[f"cayley_{pr}"]["seconds"]
    if not args.no_cpu_baseline:
        log("dense: CPU oracle baseline")
        out["cpu_baseline"] = dense_cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


def trajectory(args):
    """The 24^3x64, Ls = 24 trajectory workload (c5): a fermion-only EOFA
    leapfrog trajectory of n_steps x dt from seeded links, pseudofermion and
    momenta.  Mixed precision (inner solver args.inner) forward, then
    backward with flipped momenta (reversibility), and the same trajectory
    with the FP64 solver; reports dH = H_end - H_start for both and the
    distance between their end points.  Prints one JSON line."""
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import Context
    from paper_1611_00298_amd.hmc import hamiltonian, leapfrog

    pre = din.preset("c5")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    log("trajectory: generating c5 inputs")
    U0 = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    phi = t(din.gaussian_4d(pre["L"], pre["seed_phi"]))
    P0 = t(din.gaussian_momenta(pre["L"], pre["seed_mom"]))
    m1, m2, n, dt = pre["m1"], pre["m2"], pre["n_steps"], pre["dt"]
    ctx = Context(pre["L"], pre["Ls"], U0, M5=pre["M5"], alpha=pre["alpha"])
    out = {"metric": "fermion-only EOFA trajectory: dH and reversibility, mixed vs FP64 (1 GPU)",
           "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                                  f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}: {n} leapfrog "
                                  f"steps of dt={dt}, solves to 1e-10", "inner_precision": args.inner},
           "data": "synthetic (random SU(3) links exp(i eps H), Gaussian pseudofermion and momenta)"}
    res = {}
    for label, solver in (("mixed", dict(tol=1e-10, inner=args.inner, reliable_delta=args.delta)),
                          ("fp64", dict(tol=1e-10, inner="fp64"))):
        U, P = U0.clone(), P0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H0, S0, K0, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
        prog = lambda i, st, lab=label: log(f"trajectory {lab}: force {i}: iters {st['iters']} "
                                            f"solve {st['seconds']:.2f}s")
        leapfrog(ctx, U, P, phi, m1, m2, n, dt, progress=prog, **solver)
        H1, S1, K1, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        log(f"trajectory {label}: H0 {H0:.6f} H1 {H1:.6f} dH {H1 - H0:.6e} ({sec:.1f} s)")
        r = {"H0": H0, "dH": H1 - H0, "S0": S0, "S1": S1, "kin0": K0, "kin1": K1, "seconds": sec}
        if label == "mixed":
            Ue, Pe = U.clone(), P.clone()
            P.neg_()
            leapfrog(ctx, U, P, phi, m1, m2, n, dt, progress=prog, **solver)
            Hb, _, _, _ = hamiltonian(ctx, U, P, phi, m1, m2, **solver)
            r["reversibility"] = {"max_abs_dU": float((U - U0).abs().max()),
                                  "max_abs_dP": float((P + P0).abs().max()), "H_back_minus_H0": Hb - H0}
            log(f"trajectory reversed: |dU| {r['reversibility']['max_abs_dU']:.3e} "
                f"|dP| {r['reversibility']['max_abs_dP']:.3e}")
            res["U_mixed"] = Ue
        else:
            r["end_point_vs_mixed"] = {"max_abs_dU": float((U - res.pop("U_mixed")).abs().max())}
        out[label] = r
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


def heatbath(args):
    """The EOFA heatbath of eq. (3.1) on the selected workload (default
    24^3x64, Ls = 24): M_EOFA's spectral interval by Lanczos, Zolotarev's
    rational approximation with the fewest poles reaching a relative error
    of 1e-10 on it, then phi = M_EOFA^(-1/2) eta by 2 N_p Cayley-form
    solves, checked by phi^dag M_EOFA phi = eta^dag eta.  Prints one JSON
    line."""
    import numpy as np
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import Context, rational_inv_sqrt

    pre = din.preset(args.workload)
    dev = torch.device("cuda:0")
    m1, m2 = pre["m1"], pre["m2"]
    log(f"heatbath: generating {args.workload} inputs")
    U = torch.from_numpy(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"])).to(dev)
    eta_h = din.gaussian_4d(pre["L"], pre["seed_phi"])   # P(eta) ~ exp(-eta^dag eta)
    eta = torch.from_numpy(eta_h).to(dev)
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    solver = dict(inner=args.inner, reliable_delta=args.delta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmin, tmax, rmin, rmax, stb = ctx.meofa_bounds(eta, m1, m2, n_iter=args.lanczos, tol=args.lanczos_tol, **solver)
    t_bounds = time.perf_counter() - t0
    log(f"heatbath: Lanczos ({args.lanczos} steps, {t_bounds:.1f} s): theta [{tmin:.6f}, {tmax:.6f}], "
        f"residuals {rmin:.2e}, {rmax:.2e}")
    # Ritz values converge from inside the spectrum: widen by their residuals and 2 %
    lo, hi = 0.98 * max(tmin - rmin, 0.5 * tmin), 1.02 * (tmax + rmax)
    n = 1
    while rational_inv_sqrt(lo, hi, n)[3] > 1e-10:
        n += 1
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, st = ctx.eofa_heatbath(eta, m1, m2, lo=lo, hi=hi, n_poles=n, tol=1e-10, forecast=args.forecast,
                                **solver)
    torch.cuda.synchronize()
    t_hb = time.perf_counter() - t0
    hq = ctx.timing_query("hop")
    ctx.timing_enable(False)
    log(f"heatbath: {n} poles, {2 * n} solves, {t_hb:.1f} s, iterations {st['iters']}")
    _, _, _, S, stc = ctx.eofa_solve(phi, m1, m2, tol=1e-10, want_mphi=False, **solver)
    ee = float(np.vdot(eta_h, eta_h).real)
    ctx.close()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = heatbath_cpu_baseline(solver)
        log(f"heatbath: oracle on {cpu['sample']}: {cpu['value']:.1f} s, GPU on the same: {cpu['gpu_seconds']:.2f} s")
    out = {"metric": "EOFA heatbath (eq. 3.1): time for phi = M_EOFA^-1/2 eta (1 GPU)",
           "value": t_hb, "unit": "s", "higher_is_better": False,
           "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                                  f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}",
                      "inner_precision": args.inner, "tol": 1e-10},
           "data": "synthetic (random SU(3) links exp(i eps H), Gaussian eta)",
           "spectrum": {"lanczos_steps": args.lanczos, "theta": [tmin, tmax], "resid": [rmin, rmax],
                        "seconds": t_bounds, "iters": stb["iters"]},
           "rational": {"interval": [lo, hi], "n_poles": n, "delta": st["delta"]},
           "heatbath": {"seconds": t_hb, "solves": 2 * n, "forecast": args.forecast, "iters": st["iters"],
                        "reliable_updates": st["reliable_updates"], "true_resid": st["true_resid"]},
           "hop": {"launches": hq["count"], "avg_ms": hq["ms"] / max(hq["count"], 1),
                   "achieved_GBs": hq["bytes"] / max(hq["ms"], 1e-30) / 1e6,
                   "peak_GBs": HBM_PEAK_GBS, "frac": hq["bytes"] / max(hq["ms"], 1e-30) / 1e6 / HBM_PEAK_GBS,
                   "time_share": hq["ms"] / 1e3 / t_hb},
           "cpu_baseline": cpu,
           "check": {"S_over_eta2_minus_1": S / ee - 1.0, "bound_2delta": 2 * st["delta"],
                     "solve_iters": stc["iters"]}}
    print(json.dumps(out), flush=True)
    return 0


def heatbath_cpu_baseline(solver):
    """The oracle's heatbath (eq. (3.1) as printed: CGNR on the shifted
    operators, FP64, OpenMP) on the 4^4x8, Ls = 8 case with 4 Zolotarev
    poles on [0.5, 3], beside the GPU heatbath on the same input."""
    import torch
    import dwf_inputs as din
    import oracle
    from paper_1611_00298_amd import Context
    pre = din.preset("c1")
    lat = oracle.Lattice(pre["L"], pre["Ls"], M5=pre["M5"], alpha=pre["alpha"])
    U = din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"])
    eta = din.gaussian_4d(pre["L"], pre["seed_phi"])
    a0, a, b, _ = oracle.zolotarev_inv_sqrt(0.5, 3.0, 4)
    t0 = time.perf_counter()
    ref, _ = oracle.eofa_heatbath(lat, U, pre["m1"], pre["m2"], eta, a0, a, b, tol=1e-10)
    t_cpu = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    with Context(pre["L"], pre["Ls"], torch.from_numpy(U).to(dev), M5=pre["M5"], alpha=pre["alpha"]) as ctx:
        e = torch.from_numpy(eta).to(dev)
        ctx.eofa_heatbath(e, pre["m1"], pre["m2"], coeffs=(a0, a, b), tol=1e-10, **solver)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, _ = ctx.eofa_heatbath(e, pre["m1"], pre["m2"], coeffs=(a0, a, b), tol=1e-10, **solver)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
    import numpy as np
    diff = float(np.linalg.norm(phi.cpu().numpy() - ref) / np.linalg.norm(ref))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": t_cpu, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": "eq. (3.1) heatbath on 4^4x8, Ls=8, 4 poles on [0.5, 3], solves to 1e-10",
            "gpu_seconds": t_gpu, "rel_diff_gpu_vs_oracle": diff}


def hmc(args):
    """One complete EOFA HMC trajectory on the 24^3x64, Ls = 24 trajectory
    workload (fermion-only, or with the Iwasaki gauge action at
    args.gauge_beta > 0 on args.n_gauge inner force-gradient steps per link
    update), timed by phase in the
    rows of Table 4: M_EOFA's
    interval (Lanczos) and the heatbath of eq. (3.1) with chronological
    guesses, the force-gradient QPQPQ integration (args.md_steps steps over
    unit trajectory length, four force evaluations per step), the final
    Hamiltonian, and the Metropolis decision.  Prints one JSON line."""
    import numpy as np
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import IWASAKI_C1, Context, rational_inv_sqrt
    from paper_1611_00298_amd.hmc import force_gradient, hamiltonian

    pre = din.preset("c5")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    m1, m2 = pre["m1"], pre["m2"]
    n, dt = args.md_steps, 1.0 / args.md_steps
    log("hmc: generating c5 inputs")
    U = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    eta_h = din.gaussian_4d(pre["L"], pre["seed_phi"])
    eta = t(eta_h)
    P = t(din.gaussian_momenta(pre["L"], pre["seed_mom"]))
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    solver = dict(tol=1e-10, inner=args.inner, reliable_delta=args.delta)
    gauge = (args.gauge_beta, IWASAKI_C1) if args.gauge_beta > 0 else None
    plaq0 = plaquette(ctx, U)
    sync = torch.cuda.synchronize
    sync()
    t0 = time.perf_counter()
    tmin, tmax, rmin, rmax, _ = ctx.meofa_bounds(eta, m1, m2, n_iter=args.lanczos, tol=args.lanczos_tol, inner=args.inner)
    lo, hi = 0.98 * max(tmin - rmin, 0.5 * tmin), 1.02 * (tmax + rmax)
    n_poles = next(k for k in range(1, 65) if rational_inv_sqrt(lo, hi, k)[3] <= 1e-10)
    sync()
    t_int = time.perf_counter() - t0
    t0 = time.perf_counter()
    phi, hb = ctx.eofa_heatbath(eta, m1, m2, lo=lo, hi=hi, n_poles=n_poles, forecast=args.forecast, **solver)
    sync()
    t_hb = time.perf_counter() - t0
    log(f"hmc: interval [{lo:.4f}, {hi:.3f}] ({t_int:.1f} s), heatbath {n_poles} poles {t_hb:.1f} s")
    t0 = time.perf_counter()
    H0, S0, K0, _ = hamiltonian(ctx, U, P, phi, m1, m2, gauge=gauge, **solver)
    sync()
    t_h0 = time.perf_counter() - t0
    prog = lambda i, st: log(f"hmc: force {i}: iters {st['iters']} solve {st['seconds']:.2f}s")
    t0 = time.perf_counter()
    ctx.chrono(args.chrono)
    fst = force_gradient(ctx, U, P, phi, m1, m2, n, dt, progress=prog, gauge=gauge, n_gauge=args.n_gauge,
                         **solver)
    sync()
    t_md = time.perf_counter() - t0
    t0 = time.perf_counter()
    H1, S1, K1, _ = hamiltonian(ctx, U, P, phi, m1, m2, gauge=gauge, **solver)
    sync()
    t_h1 = time.perf_counter() - t0
    ee = float(np.vdot(eta_h, eta_h).real)
    plaq1 = plaquette(ctx, U)
    ctx.close()
    total = t_int + t_hb + t_h0 + t_md + t_h1
    dH = H1 - H0
    kind = "fermion-only" if gauge is None else "EOFA + Iwasaki gauge"
    out = {"metric": f"{kind} EOFA HMC trajectory: time by phase (Table 4 rows), 1 GPU",
           "value": total, "unit": "s", "higher_is_better": False,
           "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                                  f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}: heatbath + {n} "
                                  f"force-gradient QPQPQ steps, tau = 1, solves to 1e-10",
                      "inner_precision": args.inner,
                      "gauge": None if gauge is None else {"beta": gauge[0], "c1": gauge[1],
                                                           "inner_force_gradient_steps": args.n_gauge}},
           "data": "synthetic (random SU(3) links exp(i eps H), Gaussian eta and momenta)",
           "phases_s": {"interval_lanczos": t_int, "heatbath": t_hb, "initial_H": t_h0,
                        "force_gradient_integration": t_md, "final_H": t_h1},
           "shares": {"heatbath_incl_interval": (t_int + t_hb) / total, "heatbath": t_hb / total,
                      "force_gradient_integration": t_md / total, "energies": (t_h0 + t_h1) / total},
           "heatbath": {"n_poles": n_poles, "interval": [lo, hi], "iters": hb["iters"],
                        "S0_over_eta2_minus_1": S0 / ee - 1.0},
           "md": {"force_evaluations": len(fst), "chrono": args.chrono, "solve_iters_total": [sum(s["iters"][0] for s in fst),
                                                                        sum(s["iters"][1] for s in fst)]},
           "dH": dH, "H0": H0, "S_gauge": [H0 - S0 - K0, H1 - S1 - K1], "plaquette": [plaq0, plaq1],
           "accept_probability": float(min(1.0, np.exp(-dH)))}
    print(json.dumps(out), flush=True)
    return 0


def hmc_chain(args):
    """args.trajectories EOFA HMC trajectories in a chain (run_chain) on the
    24^3x64, Ls = 24 trajectory workload, force-gradient integration as in
    --hmc, with M_EOFA's interval estimated by Lanczos before the first
    trajectory and reused for args.interval_every trajectories (checked
    after every heatbath by phi^dag M phi = eta^dag eta).  Reports the
    Lanczos time amortised over the chain.  Prints one JSON line."""
    import numpy as np
    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import IWASAKI_C1, Context
    from paper_1611_00298_amd.hmc import force_gradient, run_chain

    pre = din.preset("c5")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    m1, m2 = pre["m1"], pre["m2"]
    n, dt = args.md_steps, 1.0 / args.md_steps
    log("hmc chain: generating c5 inputs")
    U = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    gauge = (args.gauge_beta, IWASAKI_C1) if args.gauge_beta > 0 else None

    def draw(rng):
        # per-trajectory seeds for the seeded generators of dwf_inputs
        se, sp = (int(v) for v in rng.integers(1, 2**31, size=2))
        return t(din.gaussian_4d(pre["L"], se)), t(din.gaussian_momenta(pre["L"], sp)), float(rng.random())

    timings = []
    prog = lambda i, st: log(f"hmc chain: force {i}: iters {st['iters']} solve {st['seconds']:.2f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = run_chain(ctx, U, args.trajectories, draw, np.random.Generator(np.random.PCG64(pre["seed_mom"])),
                     m1, m2, n, dt, interval=dict(refresh_every=args.interval_every, n_iter=args.lanczos,
                                                  tol=args.lanczos_tol, guard=1e-6),
                     timings=timings, integrator=force_gradient, progress=prog, chrono=args.chrono,
                     gauge=gauge, n_gauge=args.n_gauge, tol=1e-10, inner=args.inner,
                     reliable_delta=args.delta)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ctx.close()
    t_int = sum(x["interval_s"] for x in timings)
    for i, (r, x) in enumerate(zip(recs, timings)):
        log(f"hmc chain: trajectory {i}: interval {x['interval_s']:.1f} s, trajectory {x['trajectory_s']:.1f} s, "
            f"dH {r['dH']:.4f}, accepted {r['accepted']}")
    out = {"metric": "EOFA HMC chain: time per trajectory with the M_EOFA interval reused (1 GPU)",
           "value": total / len(recs), "unit": "s per trajectory", "higher_is_better": False,
           "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                                  f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}: {len(recs)} "
                                  f"trajectories of {n} force-gradient steps, tau = 1, solves to 1e-10",
                      "inner_precision": args.inner, "interval_every": args.interval_every,
                      "gauge": None if gauge is None else {"beta": gauge[0], "c1": gauge[1]}},
           "data": "synthetic (random SU(3) links exp(i eps H); Gaussian eta and momenta per trajectory)",
           "interval_lanczos_s_total": t_int, "interval_share": t_int / total,
           "interval_s_per_trajectory": t_int / len(recs),
           "trajectories": [{"interval_s": x["interval_s"], "trajectory_s": x["trajectory_s"], "dH": r["dH"],
                             "accepted": r["accepted"], "interval": r["interval"],
                             "heatbath_iters": r["heatbath_iters"], "md_iters": r["md_iters"]}
                            for r, x in zip(recs, timings)]}
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--inner", default="fp16", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--delta", type=float, default=0.3)
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--trajectory", action="store_true",
                    help="instead of the step benchmark: the 24^3x64 fermion-only trajectory workload (c5), "
                         "mixed vs FP64 dH and reversibility")
    ap.add_argument("--heatbath", action="store_true",
                    help="instead of the step benchmark: the EOFA heatbath of eq. (3.1) (Lanczos interval, "
                         "Zolotarev poles, 2 N_p solves) on the selected workload")
    ap.add_argument("--lanczos", type=int, default=12, help="Lanczos steps for the heatbath interval")
    ap.add_argument("--lanczos-tol", type=float, default=1e-5,
                    help="solver tolerance inside the Lanczos steps (the interval needs ~1 %% accuracy)")
    ap.add_argument("--forecast", type=int, default=8,
                    help="heatbath: earlier solutions per side for chronological initial guesses (0: none)")
    ap.add_argument("--hmc", action="store_true",
                    help="instead of the step benchmark: one full EOFA HMC trajectory (heatbath, force-gradient "
                         "integration, energies) on the 24^3x64 trajectory workload, timed by phase")
    ap.add_argument("--md-steps", type=int, default=12, help="hmc: force-gradient steps per unit trajectory")
    ap.add_argument("--trajectories", type=int, default=1,
                    help="hmc: run a chain of this many trajectories with the M_EOFA interval reused")
    ap.add_argument("--interval-every", type=int, default=4,
                    help="hmc chain: trajectories between Lanczos estimates of M_EOFA's interval")
    ap.add_argument("--gauge-beta", type=float, default=0.0,
                    help="hmc: add the Iwasaki gauge action at this beta (0: fermion-only; Table 1's 24ID: 1.633)")
    ap.add_argument("--n-gauge", type=int, default=2,
                    help="hmc: inner force-gradient steps of the gauge dynamics per link update")
    ap.add_argument("--chrono", type=int, default=8,
                    help="hmc: earlier solutions per system for chronological guesses in the MD (0: none)")
    ap.add_argument("--lattice", default=None,
                    help="dslash: lattice extents Lx,Ly,Lz,Lt instead of the workload's (volume sweeps)")
    ap.add_argument("--ls", type=int, default=None, help="dslash: Ls instead of the workload's")
    ap.add_argument("--dense", action="store_true",
                    help="solve on D_EOFA itself (dense 5D blocks) against the Cayley form")
    ap.add_argument("--gauge", action="store_true",
                    help="time the Iwasaki and Wilson gauge force and action kernels")
    ap.add_argument("--dslash", action="store_true",
                    help="instead of the step benchmark: the hopping kernel's rate in all four precisions")
    ap.add_argument("--cpu-baselines", action="store_true",
                    help="the CPU oracle's operator rates and solve times per workload beside the GPU's")
    ap.add_argument("--profile-summary", nargs="+", default=None, metavar="DIR",
                    help="summarise rocprofv3 --pmc output directories of the default mode per hop form "
                         "(K1..K4) for --inner and --workload, and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 3 x 2 GiB device copies first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.profile_summary:
        return profile_summary(args)
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU sharding "
                                   "(4D domain decomposition) is not implemented"}))
        return 2

    if args.trajectory:
        return trajectory(args)
    if args.heatbath:
        return heatbath(args)
    if args.hmc:
        return hmc_chain(args) if args.trajectories > 1 else hmc(args)
    if args.dslash:
        return dslash(args)
    if args.cpu_baselines:
        return cpu_baselines(args)
    if args.gauge:
        return gauge(args)
    if args.dense:
        return dense(args)

    import torch
    import dwf_inputs as din
    from paper_1611_00298_amd import Context

    pre = din.preset(args.workload)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    log(f"bench: generating {args.workload} inputs {pre['L']} Ls={pre['Ls']}")
    U = t(din.random_gauge(pre["L"], pre["eps"], pre["seed_gauge"]))
    phi = t(din.gaussian_4d(pre["L"], pre["seed_phi"]))
    P = t(din.gaussian_momenta(pre["L"], pre.get("seed_mom", 305)))
    m1, m2, tol = pre["m1"], pre["m2"], 1e-10
    ctx = Context(pre["L"], pre["Ls"], U, M5=pre["M5"], alpha=pre["alpha"])
    solver = dict(tol=tol, inner=args.inner, reliable_delta=args.delta)
    plaq = plaquette(ctx, U)

    U0, P0 = U.clone(), P.clone()

    def restart():
        # every step starts from the same configuration: without a gauge
        # action the fermion-only MD would roughen the links step by step
        # and the solves would grow harder, so the steps would not repeat
        U.copy_(U0)
        P.copy_(P0)
        ctx.update_gauge(U)

    last = {}

    def step(record):
        restart()
        chiL, chiR, _, S, st = ctx.eofa_solve(phi, m1, m2, want_mphi=False, **solver)
        F, _, _ = ctx.eofa_force(m1, m2, chiL=chiL, chiR=chiR)
        kin = ctx.md_update(U, P, F, dt_p=args.dt, dt_u=args.dt)
        ctx.update_gauge(U)
        if record is not None:
            record.append(dict(S=S, kin=kin, **st))
            last["chi"] = (chiL, chiR)   # compared with the FP64 solve after the timed region
        return st

    for w in range(args.warmup):
        st = step(None)
        log(f"bench: warmup {w}: iters {st['iters']} reliable {st['reliable_updates']} "
            f"resid {st['true_resid']} {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(recs)
        log(f"bench: step {k}: iters {recs[-1]['iters']} reliable {recs[-1]['reliable_updates']} "
            f"resid {recs[-1]['true_resid']} solve {recs[-1]['seconds']:.3f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ref_gbs = elementwise_reference(dev)
    hop_cls = {"fp64": "hop64", "fp32": "hop32", "fp16": "hop16", "bf16": "hopb16"}[args.inner]
    hq = ctx.timing_query(hop_cls)
    h64 = ctx.timing_query("hop64")
    other = {}
    for cls, label in (("force", "force (eq. 3.2)"), ("md", "md_update"), ("blas", "CG vector kernels")):
        q = ctx.timing_query(cls)
        if q["count"]:
            gbs = q["bytes"] / (q["ms"] * 1e-3) / 1e9
            other[cls] = {"kernel": label, "launches": q["count"], "avg_ms": q["ms"] / q["count"],
                          "avg_bytes": q["bytes"] / q["count"], "achieved_GBs": gbs,
                          "frac": gbs / HBM_PEAK_GBS}
    ctx.timing_enable(False)
    flops = sum(r["flops"] for r in recs)
    solve_s = [r["seconds"] for r in recs]
    avg_ms = hq["ms"] / max(hq["count"], 1)
    avg_bytes = hq["bytes"] / max(hq["count"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9 if hq["count"] else 0.0

    out = {
        "metric": METRIC,
        "value": flops / elapsed / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 (f64 outer)", "fp16": "f32 arith, fp16+norm storage (f64 outer)",
                  "bf16": "f32 arith, bf16 storage (f64 outer)"}[args.inner],
        "data": "synthetic (random SU(3) links exp(i eps H), Gaussian pseudofermion)",
        "config": {"workload": f"EOFA Moebius DWF {'x'.join(map(str, pre['L']))}, Ls={pre['Ls']}, "
                               f"alpha={pre['alpha']}, M5={pre['M5']}, m1={m1}, m2={m2}: two "
                               f"Cayley-form even-odd CG solves to 1e-10 + action + force + MD step",
                   "inner_precision": args.inner, "tol": tol, "parallelism": "none (1 GPU)",
                   "plaquette": plaq},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.inner, args.workload),
                     "elementwise_ref_GBs": ref_gbs, "frac_of_elementwise_ref": achieved / ref_gbs,
                     "kernel": f"k_hop<{args.inner}> (5D hopping + fused 5D ops)",
                     "launches": hq["count"], "avg_ms": avg_ms, "avg_bytes": avg_bytes,
                     "hop_gflops": (1320 * pre["L"][0] * pre["L"][1] * pre["L"][2] * pre["L"][3] // 2
                                    * pre["Ls"]) / (avg_ms * 1e-3) / 1e9 if hq["count"] else 0.0,
                     "fp64_hop_launches": h64["count"],
                     "fp64_hop_GBs": (h64["bytes"] / (h64["ms"] * 1e-3) / 1e9) if h64["count"] else 0.0},
        "other_kernels": other,
        "solve": {"mixed_s": sum(solve_s) / len(solve_s), "iters": recs[-1]["iters"],
                  "reliable_updates": recs[-1]["reliable_updates"],
                  "true_resid": recs[-1]["true_resid"], "inner_used": recs[-1]["inner_used"]},
    }
    if not args.no_fp64_reference:
        log("bench: FP64 reference solve")
        restart()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        chiL64, chiR64, _, S64, st64 = ctx.eofa_solve(phi, m1, m2, want_mphi=False, tol=tol, inner="fp64")
        torch.cuda.synchronize()
        out["solve"]["fp64_s"] = time.perf_counter() - t2
        out["solve"]["fp64_iters"] = st64["iters"]
        out["solve"]["fp64_true_resid"] = st64["true_resid"]
        out["solve"]["speedup_mixed_vs_fp64"] = out["solve"]["fp64_s"] / out["solve"]["mixed_s"]
        # the mixed-precision solution against the FP64 one (same systems, both to the true-residual target)
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        cl, cr = last["chi"]
        out["solve"]["mixed_vs_fp64"] = {"chi_L_rel": rel(cl, chiL64), "chi_R_rel": rel(cr, chiR64),
                                         "S_rel": abs(recs[-1]["S"] - S64) / abs(S64)}
        # the mixed solver's own iteration (recursive z folded into the last
        # hop, Cayley-form directions, scalars read one iteration late,
        # reliable updates) run entirely in FP64: the speed-up over it is
        # that of the reduced-precision arithmetic alone
        log("bench: fused FP64 reference solve")
        restart()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        chiLf, chiRf, _, Sf, stf = ctx.eofa_solve(phi, m1, m2, want_mphi=False, tol=tol, inner="fp64_fused",
                                                  reliable_delta=args.delta)
        torch.cuda.synchronize()
        out["solve"]["fp64_fused_s"] = time.perf_counter() - t3
        out["solve"]["fp64_fused_iters"] = stf["iters"]
        out["solve"]["fp64_fused_true_resid"] = stf["true_resid"]
        out["solve"]["speedup_mixed_vs_fp64_fused"] = out["solve"]["fp64_fused_s"] / out["solve"]["mixed_s"]
        out["solve"]["fp64_fused_vs_fp64"] = {"chi_L_rel": rel(chiLf, chiL64), "chi_R_rel": rel(chiRf, chiR64),
                                              "S_rel": abs(Sf - S64) / abs(S64)}
        del chiL64, chiR64, chiLf, chiRf
    ctx.close()
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(pre)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
