#!/usr/bin/env python3
"""Throughput of the coupling exchange on one MI355X.

One "step" is one call of couple_step(): bin + sort, volume deposition,
restriction with the fused fine-grid lookup and drag, momentum-source deposition,
prolongation and the FP64 conservation sums, for the 10-million-particle packed
bed (box 1x1x2, bulk 128x128x256, fine 512x512x1024; synthetic inputs resident in
HBM before timing).  Prints one JSON line with particle-steps/s, the roofline of
the dominant kernel (timed live with HIP events on the library's stream) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import dataclasses
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, vendor figure
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak, vendor figure
MLP_FLOP_PER_PARTICLE = 2 * (193 * 128 + 128 * 128 + 128 * 128 + 128 * 3)   # 115,712: one forward pass
# a training row: the forward pass, the input gradients of layers 2-4 and the
# weight gradients of all four (297,728)
TRAIN_FLOP_PER_ROW = MLP_FLOP_PER_PARTICLE + 2 * (128 * 128 + 128 * 128 + 128 * 3) + MLP_FLOP_PER_PARTICLE
METRIC = "coupling particle-steps/s, plain vs MLP path at 1e-3 rel err; % HBM peak"


def kernel_alg_bytes(name, n, ncell, nfine, fsz):
    """Algorithmic (compulsory) bytes of one launch of the named kernel.

    restrict_lookup: fine u, v, w read once (3 fsz per fine cell); U written
        (3 fsz per bulk cell); per particle the sorted position and diameter
        read (4 fsz) and the sampled fluid velocity and void fraction written
        (4 fsz).
    restrict: u, v, w, p read, U, P written (the other velocity sources).
    restrict_p: the pressure alone (beside the fused kernel).
    prolong: F_fpi written on the fine grid (3 fsz per fine cell) and read on
        the bulk grid (3 fsz per bulk cell); prolong_eps: the porosity
        (1 + 1); prolong_semi: K and KU (4 + 4).
    """
    if name == "restrict_lookup":
        return 3 * fsz * nfine + 3 * fsz * ncell + n * 8 * fsz
    if name == "restrict":
        return 4 * fsz * nfine + 4 * fsz * ncell
    if name in ("restrict_p", "prolong_eps"):
        return fsz * nfine + fsz * ncell
    if name == "prolong":
        return 3 * fsz * nfine + 3 * fsz * ncell
    if name == "prolong_semi":
        return 4 * fsz * nfine + 4 * fsz * ncell
    return None


def step_alg_bytes(n, ncell, nfine, fsz, sort_passes):
    """Compulsory HBM bytes of one whole step: fine fields read and written once,
    particle inputs read and outputs written once, bulk outputs written and read
    once, plus 16 B per particle per radix pass."""
    fine = 8 * fsz * nfine
    particles = n * (7 * fsz + 4 * fsz + 8)          # pos,d,vel in; drag,beta,cell,perm out
    bulk = ncell * (8 + 11 * fsz * 2)                # count,start; 11 fields written + read
    sort = 16 * n * sort_passes
    return fine + particles + bulk + sort


# Marks of the library's kernel timing -> the kernel names rocprofv3 reports.
PROFILE_NAMES = {
    "restrict_lookup": "cpl::k_restrict_brick<float, 4, 2>",
    "restrict_p": "cpl::k_restrict_planes<float, 2, 3, 4, false>",
    "restrict": "cpl::k_restrict_planes<float, 2, 0, 4, false>",
    "prolong": "cpl::k_prolong<float, 4, 3>",
    "mlp_infer": "cpl::mlp::k_infer",
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_bed128.json")


# The sources each group of profiled kernels is built from: a group's counter
# figures hold only while these hash as they did when the counters were taken.
SOURCE_GROUPS = {
    "step": ["csrc/common.hpp", "csrc/launch.hpp", "csrc/sample.hpp", "csrc/handle.hpp", "csrc/api.hip",
             "csrc/sort.hip", "csrc/deposit.hip", "csrc/stages.hip", "include/couple.h"],
    "mlp": ["csrc/common.hpp", "csrc/launch.hpp", "csrc/sample.hpp", "csrc/mlp.hpp", "csrc/mlp_state.hpp",
            "csrc/mlp.hip", "csrc/mlp_api.hip", "include/couple.h", "include/couple_mlp.h"],
    "boxmap": ["csrc/common.hpp", "csrc/boxmap.hip", "include/couple.h", "include/couple_boxmap.h"],
}


def kernel_group(name):
    return "mlp" if "mlp::" in name else ("boxmap" if "k_boxmap" in name else "step")


def _code_only(text):
    """Source text without comments, trailing blanks and blank lines (none of
    which changes the build)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def source_hashes():
    """Hash per source group (code only) of the files its kernels are built from."""
    import hashlib
    out = {}
    for grp, files in SOURCE_GROUPS.items():
        h = hashlib.sha256()
        for f in files:
            path = os.path.join(ROOT, "paper_1807_11834_amd", f) if f.startswith("csrc/") else os.path.join(ROOT, f)
            h.update(f.encode())
            with open(path, encoding="utf-8") as fh:
                h.update(_code_only(fh.read()).encode())
        out[grp] = h.hexdigest()
    return out


def profiled_traffic(mark):
    """HBM bytes per launch of the kernel behind ``mark`` from the committed
    counter profile, or None when there is none or the sources have changed."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    name = PROFILE_NAMES.get(mark, mark)
    grp = kernel_group(name)
    if prof.get("source_hashes", {}).get(grp) != source_hashes()[grp]:
        return None
    k = prof.get("kernels", {}).get(name)
    return None if k is None else k["traffic_bytes_per_launch"]


def _pmc_means(path):
    """Mean counter value per kernel (KiB per dispatch) from a rocprofv3 csv."""
    import csv
    import glob
    import re
    vals = {}
    for fn in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").strip()
                if "k_boxmap" in k:   # two directions, told apart by their grids
                    k = f"{k}@{r.get('Grid_Size', '')}"
                vals.setdefault(k, []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def traffic_summary(d):
    """JSON summary of the FETCH_SIZE / WRITE_SIZE runs under directory ``d``,
    each counter scaled by what it reads for the 1 GiB copy of --copy-calibration:
    subdirectories fetch, write (the plain path, --no-mlp), fetch_mlp, write_mlp
    (with the surrogate: only its in-step kernels are taken from these, the
    others also ran on the training workload), cal_fetch, cal_write."""
    fetch, write = _pmc_means(os.path.join(d, "fetch")), _pmc_means(os.path.join(d, "write"))
    fm, wm = _pmc_means(os.path.join(d, "fetch_mlp")), _pmc_means(os.path.join(d, "write_mlp"))
    for k in ("cpl::mlp::k_pack", "cpl::mlp::k_infer", "cpl::mlp::k_check"):
        if k in fm and k in wm:
            fetch[k], write[k] = fm[k], wm[k]
    cf, cw = _pmc_means(os.path.join(d, "cal_fetch")), _pmc_means(os.path.join(d, "cal_write"))
    copy = [k for k in cf if "AUnaryFunctor" in k or "MulFunctor" in k]
    if not copy:
        raise SystemExit("no copy kernel in the calibration runs")
    gib_kib = float(1 << 20)
    f_fetch, f_write = gib_kib / cf[copy[0]][0], gib_kib / cw[copy[0]][0]
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if not k.startswith("cpl::"):
            continue
        fk, fn = fetch[k]
        wk, _ = write[k]
        kernels[k] = {"dispatches": fn, "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                      "traffic_bytes_per_launch": int(round((fk * f_fetch + wk * f_write) * 1024))}
    return {
        "workload": "bed128_cic: 10,000,000 particles, bulk 128x128x256, fine 512x512x1024, FP32",
        "source_hashes": source_hashes(),
        "calibration": {"kernel": copy[0], "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                        "fetch_kib": cf[copy[0]][0], "write_kib": cw[copy[0]][0],
                        "fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4)},
        "kernels": kernels,
    }


def trace_summary(csv_path):
    """Markdown table of a rocprofv3 --stats kernel summary (library kernels)."""
    import csv
    import re
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    lines = ["| kernel | calls | avg us | min us | max us | share of traced GPU time |", "|---|---|---|---|---|---|"]
    for r in rows:
        n = re.sub(r"\(.*", "", r["Name"]).replace("void ", "").strip()
        if not n.startswith("cpl::"):
            continue
        lines.append(f"| `{n}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f}% |")
    return "\n".join(lines)


def sort_passes(ncell):
    bits = 1
    while (1 << bits) < ncell:
        bits += 1
    return (bits + 7) // 8


def cpu_baseline(w, frac):
    """Time the FP64 oracle (single-threaded C) on the sub-box x < frac*Lx, y < frac*Ly
    of the workload (full z extent, same fine spacing), one step."""
    import numpy as np

    import oracle
    import workload as W
    g = w.grid
    sub = dataclasses.replace(w, grid=W.Grid((g.box[0] * frac, g.box[1] * frac, g.box[2]),
                                             (int(g.nb[0] * frac), int(g.nb[1] * frac), g.nb[2]), g.ratio))
    pos, d, vel = W.particles(w)
    m = (pos[:, 0] < sub.grid.box[0]) & (pos[:, 1] < sub.grid.box[1])
    pos, d, vel = pos[m], d[m], vel[m]
    fine = W.fine_fields(sub)
    oracle.lib()

    def one_step(threads):
        prev = oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.step(pos, vel, d, fine, sub.grid, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p, eps_min=w.eps_min,
                    cic=True, prec32=True, vel_source="fine")
        dt = time.perf_counter() - t0
        oracle.set_threads(prev)
        return dt

    dt = one_step(1)
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    dt_all = one_step(ncores)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pos.shape[0] / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"one oracle step (FP64, single thread) on the sub-box x<{frac}, y<{frac} of the same "
                       f"workload: {pos.shape[0]} particles, bulk {sub.grid.nb}, fine {sub.grid.nf}; "
                       f"{dt:.1f} s; host {cpu}, {os.cpu_count()} logical CPUs"),
            "all_cores": {"value": pos.shape[0] / dt_all, "cores": ncores, "seconds": round(dt_all, 2),
                          "note": "same sample; OpenMP over the oracle's independent per-particle / per-cell "
                                  "loops, the canonical-order deposition sums and the sort stay serial"}}


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))


def mlp_leg(args, w, cfg, pos, vel, diam, fine, plain_ms, plain_kernels, dev):
    """The learned-surrogate path on the same workload: training pairs from the
    64^3/256^3 Taylor-Green workload (20,000 particles from each of its 100
    advected steps) and from this workload's first step (2,000,000 particles),
    training on the GPU (batch 65,536, Adam lr 1e-3), then the timed step with
    vel_source MLP and the 1 % sampled check with fine fallback at 1e-3."""
    import dataclasses as dc

    import torch

    import paper_1807_11834_amd as cpl
    import workload as W
    from paper_1807_11834_amd import surrogate as S
    t0 = time.perf_counter()
    w1 = W.WORKLOADS["cube64_cic"]
    p1, d1, v1 = W.particles(w1)
    g1 = w1.grid
    cfg1 = cpl.Config(box=g1.box, nb=g1.nb, ratio=g1.ratio, rho_f=w1.rho_f, mu_f=w1.mu_f, rho_p=w1.rho_p,
                      eps_min=w1.eps_min, advect=1, dt=w1.dt, max_particles=p1.shape[0])
    pool = S.PairPool(w1.steps * 20000 + 2_000_000)
    P1, V1, D1 = (torch.from_numpy(a).to(dev) for a in (p1, v1, d1))
    fine1 = W.fine_fields_torch(w1, dev, torch.float32)
    S.collect(pool, cfg1, P1, V1, D1, fine1, steps=w1.steps, per_step=20000, seed=3)
    del P1, V1, D1, fine1
    cfgf = dc.replace(cfg, vel_source=cpl.COUPLE_VEL_FINE, advect=0)
    S.collect(pool, cfgf, pos, vel, diam, fine, steps=1, per_step=2_000_000, seed=4)
    t_pairs = time.perf_counter() - t0
    mlp = cpl.Mlp(65536)
    mlp.set_params(S.he_uniform(0))
    feat, resid = pool.view()
    mlp.fit_norm(feat, resid)
    t0 = time.perf_counter()
    hist = S.train(mlp, feat, resid, steps=args.mlp_steps, batch=65536, seed=3, log_every=max(1, args.mlp_steps // 4),
                   log=lambda m: print("# surrogate " + m, file=sys.stderr, flush=True))
    t_train = time.perf_counter() - t0
    del pool, feat, resid
    torch.cuda.empty_cache()

    n = pos.shape[0]

    def velocities(source, tol=1e30):
        c = cpl.Coupler(dc.replace(cfg, vel_source=source, advect=0, mlp_tol=tol))
        if source == cpl.COUPLE_VEL_MLP:
            cpl.couple_set_mlp(c.h, mlp.m)
        o = c.step(pos, vel, diam, fine, uf=True)
        torch.cuda.synchronize()
        u = o["uf"].clone()
        d = cpl.diag_dict(o["diag"])
        c.close()
        return u, d

    uF, _ = velocities(cpl.COUPLE_VEL_FINE)
    uB, _ = velocities(cpl.COUPLE_VEL_BULK)
    uM, dm = velocities(cpl.COUPLE_VEL_MLP)
    uMF, dmf = velocities(cpl.COUPLE_VEL_MLP, tol=1e-3)
    upflow = torch.tensor([0.0, 0.0, 0.5 if w.fluid == "upflow" else 0.0], device=dev)
    acc = {
        "rel_err_mlp": _rel(uM, uF), "rel_err_mlp_with_fallback": _rel(uMF, uF), "rel_err_bulk": _rel(uB, uF),
        "rel_err_mlp_perturbation": float(torch.linalg.vector_norm((uM - uF).double()) /
                                          torch.linalg.vector_norm((uF - upflow).double())),
        "rel_err_bulk_perturbation": float(torch.linalg.vector_norm((uB - uF).double()) /
                                           torch.linalg.vector_norm((uF - upflow).double())),
        "sampled_rel_err_in_step": float(np.sqrt(dmf["mlp_err2"] / dmf["mlp_ref2"])) if dmf["mlp_ref2"] else None,
        "fallback_fraction": dmf["n_fallback"] / n,
    }
    del uF, uB, uM, uMF

    cm = cpl.Coupler(dc.replace(cfg, vel_source=cpl.COUPLE_VEL_MLP, advect=0, mlp_tol=1e-3))
    cpl.couple_set_mlp(cm.h, mlp.m)
    out = cpl.alloc_outputs(cm.cfg, n, device=dev)
    for k in range(args.warmup):
        cm.step(pos, vel, diam, fine, out=out, step=k)
    stream = torch.cuda.current_stream()
    total, per = timed_steps(lambda k: cm.step(pos, vel, diam, fine, out=out, step=k), args.steps, stream)
    ms = total / args.steps
    dfin = cpl.diag_dict(out["diag"])
    nk = min(args.steps, 20)
    cpl.couple_timing_begin(cm.h, nk)
    for k in range(nk):
        cm.step(pos, vel, diam, fine, out=out, step=k)
    torch.cuda.synchronize()
    stats = cpl.couple_timing_end(cm.h)
    cm.close()
    mlp.close()
    kern = {k: {"launches": l, "avg_ms": t / l} for k, (l, t) in stats.items() if l}
    t_inf = kern["mlp_infer"]["avg_ms"]
    flop = n * MLP_FLOP_PER_PARTICLE
    ach = flop / (t_inf * 1e-3) / 1e12
    vel_mlp = sum(kern[k]["avg_ms"] for k in ("restrict", "mlp_pack", "mlp_infer", "mlp_check") if k in kern)
    vel_plain = plain_kernels.get("restrict_lookup", {}).get("avg_ms")
    return {
        "ms_per_step": ms, "value": n / (ms * 1e-3), "unit": "particle-steps/s", "per_step": step_stats(per),
        "speedup_vs_plain_step": plain_ms / ms,
        "velocity_stage_ms": {"plain (restrict + fine lookup)": vel_plain,
                              "mlp (restrict + pack + infer + check/fallback)": round(vel_mlp, 4)},
        "speedup_vs_plain_velocity_stage": (vel_plain / vel_mlp) if vel_plain else None,
        "accuracy_vs_fine_lookup": acc,
        "last_timed_step": {"sampled_rel_err": float(np.sqrt(dfin["mlp_err2"] / dfin["mlp_ref2"]))
                            if dfin["mlp_ref2"] else None, "fallback_particles": dfin["n_fallback"]},
        "roofline": {"bound": "mfma", "kernel": "mlp_infer", "achieved": round(ach, 1),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / MFMA_BF16_PEAK_TFLOPS, 4),
                     "traffic": profiled_traffic("mlp_infer"), "flop_per_launch": flop, "avg_ms": round(t_inf, 4)},
        "kernels_avg_ms": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "train": {"steps": args.mlp_steps, "batch": 65536, "seconds": round(t_train, 1),
                  "ms_per_step": round(t_train / max(args.mlp_steps, 1) * 1e3, 4),
                  "tflops": round(TRAIN_FLOP_PER_ROW * 65536 * args.mlp_steps / max(t_train, 1e-9) / 1e12, 1),
                  "frac_bf16_peak": round(TRAIN_FLOP_PER_ROW * 65536 * args.mlp_steps / max(t_train, 1e-9) / 1e12
                                          / MFMA_BF16_PEAK_TFLOPS, 4),
                  "pairs_seconds": round(t_pairs, 1), "loss_first_last": [hist[0][1], hist[-1][1]],
                  "pairs": "20,000 per step x 100 advected steps of cube64_cic + 2,000,000 of this workload's "
                           "first step"},
    }


def timed_steps(step_fn, k, stream):
    """Run ``step_fn`` k times on ``stream`` with one HIP event between
    consecutive steps (no per-kernel markers); returns (total ms, per-step ms)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(k):
        step_fn(i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[k]), [ev[i].elapsed_time(ev[i + 1]) for i in range(k)]


def step_stats(per):
    a = np.asarray(per, dtype=np.float64)
    return {"steps": int(a.size), "median_ms": round(float(np.median(a)), 4), "mean_ms": round(float(a.mean()), 4),
            "sd_ms": round(float(a.std(ddof=1)) if a.size > 1 else 0.0, 4), "min_ms": round(float(a.min()), 4),
            "max_ms": round(float(a.max()), 4)}


def advected_leg(args, dev):
    """The 64^3 / 256^3 Taylor-Green cube with 2,000,000 particles advanced by
    its 100 explicit-Euler steps (dt = 1e-4, drag the only force, re-binned every
    step), timed whole from the initial state after a warm-up on a copy."""
    import torch
    import paper_1807_11834_amd as cpl
    import workload as W
    w = W.WORKLOADS["cube64_cic"]
    g = w.grid
    p0, d0, v0 = W.particles(w)
    n = p0.shape[0]
    fine = W.fine_fields_torch(w, dev, torch.float32)
    diam = torch.from_numpy(d0).to(dev)
    cfg = cpl.Config(box=g.box, nb=g.nb, ratio=g.ratio, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p,
                     eps_min=w.eps_min, advect=1, dt=w.dt, max_particles=n)
    c = cpl.Coupler(cfg)
    out = cpl.alloc_outputs(cfg, n, device=dev)
    try:
        pos, vel = torch.from_numpy(p0).to(dev), torch.from_numpy(v0).to(dev)
        for _ in range(max(args.warmup, 1)):
            c.step(pos, vel, diam, fine, out=out)
        pos, vel = torch.from_numpy(p0).to(dev), torch.from_numpy(v0).to(dev)
        stream = torch.cuda.current_stream()
        total, per = timed_steps(lambda i: c.step(pos, vel, diam, fine, out=out, step=i), w.steps, stream)
        dg = cpl.diag_dict(out["diag"])
    finally:
        c.close()
    ms = total / w.steps
    sb = step_alg_bytes(n, g.n_bulk, g.n_fine, 4, sort_passes(g.n_bulk)) + 24 * n   # + advected pos, vel
    print(f"# advected cube: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    del fine, out
    torch.cuda.empty_cache()
    return {"workload": f"{w.name}: {n} particles, bulk {g.nb}, fine {g.nf}, CIC, FP32, {w.steps} explicit-Euler "
                        f"steps of dt = {w.dt} timed whole",
            "ms_per_step": ms, "value": n * w.steps / (total * 1e-3), "unit": "particle-steps/s",
            "per_step": step_stats(per), "step_alg_bytes": sb,
            "step_alg_GBps": round(sb / (ms * 1e-3) / 1e9, 1),
            "step_alg_frac_hbm": round(sb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "n_outside_last_step": dg["n_outside"]}


def _time_variant(args, cfg_v, pos, vel, diam, fine, n, dev, alpha=None):
    """Warm up, then time ``args.steps`` steps of a configuration variant (no
    markers), then up to 20 steps with per-kernel events; returns (ms per step,
    {kernel: avg ms}, diagnostics)."""
    import torch
    import paper_1807_11834_amd as cpl
    c = cpl.Coupler(cfg_v)
    out = cpl.alloc_outputs(cfg_v, n, device=dev)
    try:
        for _ in range(args.warmup):
            c.step(pos, vel, diam, fine, out=out, alpha=alpha)
        stream = torch.cuda.current_stream()
        ms = timed_steps(lambda i: c.step(pos, vel, diam, fine, out=out, alpha=alpha), args.steps, stream)[0] \
            / args.steps
        d = cpl.diag_dict(out["diag"])
        nk = min(args.steps, 20)
        cpl.couple_timing_begin(c.h, nk)
        for _ in range(nk):
            c.step(pos, vel, diam, fine, out=out, alpha=alpha)
        torch.cuda.synchronize()
        stats = cpl.couple_timing_end(c.h)
    finally:
        c.close()
    del out
    torch.cuda.empty_cache()
    return ms, {k: t / l for k, (l, t) in stats.items() if l}, d


def hbm_reference(dev, reps=20):
    """Practical HBM ceiling on this device: the library's streaming reference
    kernels (include/couple_hbmref.h) over 2 GiB buffers -- a read (a scan for
    non-finite values), a write and a copy (read + write bytes) -- the median
    of ``reps`` launches each, with torch's device copy of the same buffer
    beside them."""
    import torch
    import paper_1807_11834_amd as cpl
    nbytes = 2 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def median_ms(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[len(ts) // 2]

    res = {}
    for name, kind, a, b, mult in (("read", cpl.COUPLE_HBMREF_READ, src, flag, 1),
                                   ("write", cpl.COUPLE_HBMREF_WRITE, None, dst, 1),
                                   ("copy", cpl.COUPLE_HBMREF_COPY, src, dst, 2)):
        ms = median_ms(lambda kind=kind, a=a, b=b: cpl.hbmref(kind, a, b, 1.0))
        gbps = mult * nbytes / (ms * 1e-3) / 1e9
        res[name] = {"GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4)}
    ms = median_ms(lambda: dst.copy_(src))
    gbps = 2 * nbytes / (ms * 1e-3) / 1e9
    res["torch_copy"] = {"GBps": round(gbps, 1), "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4)}
    res["note"] = ("2 GiB buffers, median of %d launches; copy and torch_copy count read + write bytes" % reps)
    del src, dst, flag
    torch.cuda.empty_cache()
    return res


def semi_leg(args, cfg, pos, vel, diam, fine, plain_ms, n, g, fsz, dev):
    """The same step with the semi-implicit split on (K, KU deposited and
    prolonged in addition): time per step, the extra kernels and the prolongation
    roofline of K, KU, and the conservation of their sums."""
    ms, kt, d = _time_variant(args, dataclasses.replace(cfg, semi_implicit=1), pos, vel, diam, fine, n, dev)
    kern = {k: v for k, v in kt.items() if k in ("deposit_semi", "deposit_semi_sum", "prolong_semi")}
    ab = kernel_alg_bytes("prolong_semi", n, g.n_bulk, g.n_fine, fsz)
    pr = kern.get("prolong_semi")
    print(f"# semi-implicit split: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return {"ms_per_step": ms, "value": n / (ms * 1e-3), "extra_ms_vs_plain": ms - plain_ms,
            "kernels_avg_ms": {k: round(v, 4) for k, v in kern.items()},
            "prolong_semi_GBps": round(ab / (pr * 1e-3) / 1e9, 1) if pr else None,
            "prolong_semi_frac_hbm": round(ab / (pr * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4) if pr else None,
            "conservation": {"K_b/K_p-1": d["K_b"] / d["K_p"] - 1 if d["K_p"] else 0.0,
                             "K_f/K_b-1": d["K_f"] / d["K_b"] - 1 if d["K_b"] else 0.0}}


def vof_leg(args, w, cfg, pos, vel, diam, fine, plain_ms, n, g, fsz, dev):
    """The same step with the two-fluid drag (water below a tilted free surface
    at z ~ 0.6 L_z, air above: the drag's density and viscosity follow the liquid
    fraction at each particle): time per step, the alpha restriction kernel and
    its roofline."""
    import workload as W
    alpha = W.fine_alpha_torch(w, dev, fine[0].dtype)
    cfg_v = dataclasses.replace(cfg, vof=1, rho_f2=1.2, mu_f2=1.8e-5)
    ms, kt, _ = _time_variant(args, cfg_v, pos, vel, diam, fine, n, dev, alpha=alpha)
    del alpha
    ra = kt.get("restrict_alpha")
    ab = fsz * g.n_fine + fsz * g.n_bulk
    print(f"# two-fluid drag: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return {"ms_per_step": ms, "value": n / (ms * 1e-3), "extra_ms_vs_plain": ms - plain_ms,
            "fluid_2": {"rho": cfg_v.rho_f2, "mu": cfg_v.mu_f2},
            "kernels_avg_ms": {k: round(v, 4) for k, v in kt.items() if k in ("restrict_alpha", "pack_alpha", "drag")},
            "restrict_alpha_GBps": round(ab / (ra * 1e-3) / 1e9, 1) if ra else None,
            "restrict_alpha_frac_hbm": round(ab / (ra * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4) if ra else None}


def precision_leg(args, cfg, pos, vel, diam, fine, plain_ms, n, dev):
    """The same step in the other FP32 precision modes: Kahan-compensated FP32
    per-cell sums and plain FP32 sums (the headline runs FP64-register per-cell
    sums); time per step and the time of the restriction, deposition and
    transfer kernels whose sums the mode changes."""
    import paper_1807_11834_amd as cpl
    res = {}
    keys = ("restrict_p", "restrict_lookup", "deposit_phi", "deposit_phi_sum", "deposit_force", "deposit_force_sum")
    for name, prec in (("fp32_kahan", cpl.COUPLE_FP32_KAHAN), ("fp32_naive", cpl.COUPLE_FP32_NAIVE)):
        ms, kt, _ = _time_variant(args, dataclasses.replace(cfg, precision=prec), pos, vel, diam, fine, n, dev)
        res[name] = {"ms_per_step": ms, "value": n / (ms * 1e-3), "vs_fp64_register_sums": ms / plain_ms,
                     "kernels_avg_ms": {k: round(v, 4) for k, v in kt.items() if k in keys}}
        print(f"# precision {name}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return res


def part_leg(args, cfg, pos, vel, diam, fine, plain_ms, n, dev):
    """The partitioned step (co-located z-slabs with one-layer halos, Sec. 2.2)
    on this workload for K = 2, 4, 8 slabs and both exchange strategies
    (distributed and gather-scatter, Sec. 2.3): time per step against the
    monolithic step, the static communication matrix's bytes per step, and the
    agreement with the monolithic step at full size (cell, perm, count bit for
    bit; the largest deviation of phi and of the prolonged source relative to
    their largest magnitude)."""
    import torch
    import paper_1807_11834_amd as cpl
    ref = cpl.alloc_outputs(cfg, n, device=dev)
    c = cpl.Coupler(cfg)
    try:
        c.step(pos, vel, diam, fine, out=ref)
    finally:
        c.close()
    out = cpl.alloc_outputs(cfg, n, device=dev)
    stream = torch.cuda.current_stream()
    res = {}
    for K in (2, 4, 8):
        p = cpl.Part(cfg, K)
        try:
            comm = p.comm_matrix()
            for name, ex in (("distributed", cpl.COUPLE_EXCHANGE_DISTRIBUTED),
                             ("gather_scatter", cpl.COUPLE_EXCHANGE_GATHER_SCATTER)):
                for _ in range(max(args.warmup, 1)):
                    p.step(pos, vel, diam, fine, out=out, exchange=ex)
                k = min(args.steps, 20)
                total, per = timed_steps(lambda i: p.step(pos, vel, diam, fine, out=out, exchange=ex), k, stream)
                ms = total / k
                same = {key: bool(torch.equal(out[key], ref[key])) for key in ("cell", "perm", "count", "start")}
                dev_phi = float((out["bulk_phi"] - ref["bulk_phi"]).abs().max() / ref["bulk_phi"].abs().max())
                dev_ff = float((out["fine_F"] - ref["fine_F"]).abs().max() / ref["fine_F"].abs().max())
                res[f"K{K}_{name}"] = {"ms_per_step": ms, "value": n / (ms * 1e-3), "per_step": step_stats(per),
                                       "overhead_vs_monolithic": ms / plain_ms - 1.0,
                                       "integers_equal_monolithic": same,
                                       "max_dev_phi": dev_phi, "max_dev_fine_F": dev_ff}
                print(f"# partitioned K={K} {name}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
            res[f"K{K}_comm_bytes_per_step"] = int(comm.sum())
            res[f"K{K}_comm_nonzero_blocks"] = int((comm > 0).sum())
        finally:
            p.close()
    del out, ref
    torch.cuda.empty_cache()
    return res


def boxmap_leg(args, fsz, dev):
    """Transfer through the CSR overlap map between a locally refined grid over
    the bed's box (96 x 96 x 192 base cells, the bottom quarter split 2:1 per
    axis: 4.9M cells) and the bulk grid (128 x 128 x 256): four fields each way.
    Algorithmic bytes per transfer: the map once (8 B column + weight per
    nonzero, 8 B row offset per receiver), the sender fields once and the
    receiver fields written once."""
    import torch
    import paper_1807_11834_amd as cpl
    import workload as W
    box = (1.0, 1.0, 2.0)
    f = W.refined_box_grid_fast(box, (96, 96, 192), (0.0, 1.0, 0.0, 1.0, 0.0, 0.5))
    b = W.box_grid(box, (128, 128, 256))
    prec = cpl.COUPLE_FP64 if fsz == 8 else cpl.COUPLE_FP32_WIDE
    res = {"grids": {"refined_cells": int(f.shape[0]), "bulk_cells": int(b.shape[0])}}
    stream = torch.cuda.current_stream()
    for name, s_, r_ in (("refined_to_bulk", f, b), ("bulk_to_refined", b, f)):
        t0 = time.time()
        m = cpl.BoxMap(s_, r_, precision=prec)
        build_s = time.time() - t0
        try:
            src = torch.rand((4, s_.shape[0]), dtype=m.dtype, device=dev)
            dst = torch.empty((4, r_.shape[0]), dtype=m.dtype, device=dev)
            for _ in range(3):
                m.apply(src, dst)
            k = max(args.steps, 20)
            total, per = timed_steps(lambda i: m.apply(src, dst), k, stream)
            nnz, mr = m.info()
        finally:
            m.close()
        ms = total / k
        ab = nnz * (4 + fsz) + 8 * (r_.shape[0] + 1) + 4 * fsz * (s_.shape[0] + r_.shape[0])
        res[name] = {"ms_per_transfer": ms, "nnz": int(nnz), "longest_row": int(mr), "alg_bytes": int(ab),
                     "GBps": round(ab / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "map_build_s": round(build_s, 2),
                     "traffic": profiled_traffic(f"cpl::k_boxmap<float, 2, 4>@{(r_.shape[0] + 255) // 256 * 256}")}
        print(f"# box map {name}: {ms:.3f} ms per four fields", file=sys.stderr, flush=True)
        del src, dst
    torch.cuda.empty_cache()
    return res


def remap_leg(args, g, fine, fsz, dev):
    """Grid-to-grid transfer between non-nested grids at the bed's size: the four
    fine fields (u, v, w, p; 512 x 512 x 1024 over 1 x 1 x 2) to a 192 x 192 x 384
    grid (ratio 8/3, sender cells straddle receiver faces) and the four coarse
    fields back.  Per direction: average time of one four-field transfer and the
    algorithmic bandwidth (sender fields read once + receiver fields written
    once) against the HBM peak."""
    import torch
    import paper_1807_11834_amd as cpl
    box = g.box
    nc = (192, 192, 384)
    nodes = lambda n: [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]
    prec = cpl.COUPLE_FP64 if fsz == 8 else cpl.COUPLE_FP32_WIDE
    down, up = cpl.Remap(nodes(g.nf), nodes(nc), prec), cpl.Remap(nodes(nc), nodes(g.nf), prec)
    try:
        src = torch.stack(fine)
        coarse = torch.empty((4, nc[2], nc[1], nc[0]), dtype=src.dtype, device=dev)
        back = torch.empty_like(src)
        res = {}
        for name, r, a, b, nsrc, ndst in (("fine_to_nonnested", down, src, coarse, g.n_fine, int(np.prod(nc))),
                                          ("nonnested_to_fine", up, coarse, back, int(np.prod(nc)), g.n_fine)):
            for _ in range(max(args.warmup, 1)):
                r.apply(a, b)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                r.apply(a, b)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            ab = 4 * fsz * (nsrc + ndst)
            res[name] = {"ms_per_4_fields": round(ms, 4), "alg_GBps": round(ab / (ms * 1e-3) / 1e9, 1),
                         "frac_hbm": round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        res["receiver_grid"] = list(nc)
        res["map_nnz_3d"] = down.info()[1]
        del src, coarse, back
    finally:
        down.close()
        up.close()
    torch.cuda.empty_cache()
    print(f"# non-nested transfer: {res}", file=sys.stderr, flush=True)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bed128_cic")
    ap.add_argument("--cpu-frac", type=float, default=0.3125,
                    help="x-y fraction of the oracle sample (40 of the bed's 128 bulk cells per axis)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-presorted", action="store_true", help="skip the spatially sorted input variant")
    ap.add_argument("--vel-source", default="fine", choices=["fine", "bulk"],
                    help="fluid velocity at the particles: fine-grid lookup (default) or bulk trilinear")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-surrogate path")
    ap.add_argument("--no-semi", action="store_true", help="skip the semi-implicit split variant")
    ap.add_argument("--no-vof", action="store_true", help="skip the two-fluid drag variant")
    ap.add_argument("--no-remap", action="store_true", help="skip the non-nested grid transfer")
    ap.add_argument("--no-boxmap", action="store_true", help="skip the transfer through the CSR overlap map")
    ap.add_argument("--no-advected", action="store_true", help="skip the 100-step advected 64^3 cube")
    ap.add_argument("--no-part", action="store_true", help="skip the partitioned (z-slab) step")
    ap.add_argument("--no-precision", action="store_true", help="skip the Kahan and naive FP32 variants")
    ap.add_argument("--traffic-summary", metavar="DIR",
                    help="print the JSON summary of the FETCH_SIZE/WRITE_SIZE runs under DIR and exit")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="print a markdown table of a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy kernel of known size (1 GiB read, 1 GiB written, 3 times): "
                         "the reference that scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--mlp-steps", type=int, default=20000, help="surrogate training steps (batch 65,536)")
    args = ap.parse_args()
    if args.traffic_summary:
        print(json.dumps(traffic_summary(args.traffic_summary), indent=1))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the coupling exchange is built and timed for a single "
              "MI355X (the multi-GPU sharding is a design in DESIGN.md, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"kernel": "elementwise multiply by 1.0 (torch)", "launches": 3,
                                               "bytes_read_per_launch": 1 << 30,
                                               "bytes_written_per_launch": 1 << 30}}), flush=True)
        return

    import paper_1807_11834_amd as cpl
    import workload as W

    dev = torch.device("cuda:0")
    w = W.WORKLOADS[args.workload]
    g = w.grid
    pos_np, d_np, vel_np = W.particles(w)
    n = pos_np.shape[0]
    fp64 = w.precision == "fp64"
    dt = torch.float64 if fp64 else torch.float32
    fsz = 8 if fp64 else 4
    pos = torch.from_numpy(pos_np).to(dev)
    vel = torch.from_numpy(vel_np).to(dev)
    diam = torch.from_numpy(d_np).to(dev)
    fine = W.fine_fields_torch(w, dev, dt)
    del pos_np, vel_np, d_np
    cfg = cpl.Config(box=g.box, nb=g.nb, ratio=g.ratio, rho_f=w.rho_f, mu_f=w.mu_f, rho_p=w.rho_p,
                     eps_min=w.eps_min, deposit=cpl.COUPLE_CIC if w.deposit == "cic" else cpl.COUPLE_NGP,
                     precision=cpl.COUPLE_FP64 if fp64 else cpl.COUPLE_FP32_WIDE,
                     vel_source=cpl.COUPLE_VEL_FINE if args.vel_source == "fine" else cpl.COUPLE_VEL_BULK,
                     advect=0, max_particles=n)
    c = cpl.Coupler(cfg)
    out = cpl.alloc_outputs(cfg, n, device=dev)
    for _ in range(args.warmup):
        c.step(pos, vel, diam, fine, out=out)
    torch.cuda.synchronize()
    print(f"# warmup done: {args.warmup} steps", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    # headline: exactly --steps steps, one event between consecutive steps, no
    # per-kernel markers inside the timed loop
    step_fn = lambda i: c.step(pos, vel, diam, fine, out=out)
    ms_total, per = timed_steps(step_fn, args.steps, stream)
    ms_step = ms_total / args.steps
    value = n * args.steps / (ms_total / 1e3)
    print(f"# timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)
    # the median over at least 100 steps (a second loop when --steps is smaller)
    per100 = per if args.steps >= 100 else timed_steps(step_fn, 100, stream)[1]
    # per-kernel HIP events in a separate loop
    nk = min(args.steps, 20)
    cpl.couple_timing_begin(c.h, nk)
    for _ in range(nk):
        c.step(pos, vel, diam, fine, out=out)
    torch.cuda.synchronize()
    stats = cpl.couple_timing_end(c.h)

    kernels = {k: {"launches": l, "avg_ms": t / l} for k, (l, t) in stats.items() if l}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    ab = kernel_alg_bytes(dom, n, g.n_bulk, g.n_fine, fsz)
    roof = None
    if ab is not None:
        ach = ab / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": profiled_traffic(dom),
                "alg_bytes_per_launch": ab, "avg_ms": round(kernels[dom]["avg_ms"], 4)}
    sb = step_alg_bytes(n, g.n_bulk, g.n_fine, fsz, sort_passes(g.n_bulk))
    hbm = hbm_reference(dev)
    if roof is not None:
        # the dominant kernel reads far more than it writes: its rate against
        # the streaming read's
        roof["frac_of_stream_read"] = round(roof["achieved"] / hbm["read"]["GBps"], 4)
    d = cpl.diag_dict(out["diag"])
    rec = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64 else "f32", "data": "synthetic",
        "config": {"workload": (f"{w.name}: {n} particles, box {g.box}, bulk {g.nb}, fine {g.nf}, "
                                f"{w.deposit.upper()}, {'FP64' if fp64 else 'FP32 data, FP64-register per-cell sums, FP64 global sums'}, "
                                f"{args.vel_source}-grid velocity at the particles"),
                   "n_particles": n, "bulk": list(g.nb), "fine": list(g.nf)},
        "per_step": step_stats(per),
        "median_of_100": step_stats(per100),
        "roofline": roof,
        "step_alg_bytes": sb, "step_alg_GBps": round(sb / (ms_step * 1e-3) / 1e9, 1),
        "step_alg_frac_hbm": round(sb / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "hbm_reference": hbm,
        "kernels_avg_ms": {k: round(v["avg_ms"], 4) for k, v in kernels.items()},
        "conservation": {"V_dep/V_tot-1": d["V_dep"] / d["V_tot"] - 1 if d["V_tot"] else 0.0,
                         "S_b+sumF": [d["S_b"][a] + d["sum_Fp"][a] for a in range(3)]},
    }
    if not args.no_presorted:
        # The same particles stored in the step's canonical (cell, id) order, as a
        # DEM code that keeps its arrays spatially sorted would pass them.
        perm = out["perm"].long()
        pos_s, vel_s, diam_s = pos[perm].contiguous(), vel[perm].contiguous(), diam[perm].contiguous()
        for _ in range(args.warmup):
            c.step(pos_s, vel_s, diam_s, fine, out=out)
        ms_s = timed_steps(lambda i: c.step(pos_s, vel_s, diam_s, fine, out=out), args.steps, stream)[0] / args.steps
        rec["presorted_input"] = {"ms_per_step": ms_s, "value": n / (ms_s * 1e-3),
                                  "note": "same particles passed in the canonical (cell, id) order"}
        del pos_s, vel_s, diam_s
    if not args.no_advected:
        rec["advected_cube64"] = advected_leg(args, dev)
    if not args.no_precision and not fp64:
        rec["precision_modes"] = precision_leg(args, cfg, pos, vel, diam, fine, ms_step, n, dev)
    if not args.no_part:
        rec["partitioned"] = part_leg(args, cfg, pos, vel, diam, fine, ms_step, n, dev)
    if not args.no_semi:
        rec["semi_implicit"] = semi_leg(args, cfg, pos, vel, diam, fine, ms_step, n, g, fsz, dev)
    if not args.no_vof:
        rec["two_fluid_drag"] = vof_leg(args, w, cfg, pos, vel, diam, fine, ms_step, n, g, fsz, dev)
    if not args.no_remap:
        rec["nonnested_transfer"] = remap_leg(args, g, fine, fsz, dev)
    if not args.no_boxmap:
        rec["refined_grid_transfer"] = boxmap_leg(args, fsz, dev)
    if not args.no_mlp:
        print("# surrogate: pairs, training, timing ...", file=sys.stderr, flush=True)
        rec["mlp_path"] = mlp_leg(args, w, cfg, pos, vel, diam, fine, ms_step, kernels, dev)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle sample) ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_frac)
    else:
        rec["cpu_baseline"] = None
    c.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
