"""Throughput of the QS-MHD single-step LBM on one MI355X.

Workload: 128 x 128 x 128 periodic box, pipe of radius 60 along x with 377 wall markers per
plane (48,256 markers), fringe field B0 (1 + tanh((x - 64)/8))/2 along y, Ha = 20, Re = 500,
Rm = 1e-2 (nu = 0.006, eta = 300, 270 magnetic sweeps per fluid step), float32 storage and
arithmetic, seeded synthetic initial state. One step = one fluid step: 270 x (magnetic sweep +
wall correction of b), Lorentz force, fluid predictor, wall correction of u.

value = MLUPS = box cells x fluid steps / wall time / 1e6 (inputs resident in HBM).
roofline = the magnetic sweep kernel (the dominant one): 36 algorithmic bytes per cell
(read u and b, write b*, float32) per launch over its HIP-event-timed average duration, measured
on the 512 x 256 x 256 pipe (1.9 GB of state, far beyond the 256 MB Infinity Cache, so the
sweep streams from HBM); roofline_cache_resident = the same figure on the 128^3 box of `value`,
whose 136 MB state the Infinity Cache holds. Both give the sweep's cells per second
(gcells_per_s): about equal, so the sweep's rate is set by its per-CU chain, not by HBM.
cpu_baseline = the FP64 oracle on this host: the median of 5 fluid steps (270 sweeps each) after
one warm-up step, on a 16-plane slab of the same pipe (1/8 of its cells; the oracle's cost per
cell does not depend on the box length).
batched = the batched form on 64 independent pipes of uneven size and physics (~74 M cells,
~2.3 M markers, tiles autotuned), MLUPS over all their cells (an extra object, not `value`),
next to the same pipes stepped one at a time with the same tiles (sequential_MLUPS).
shard = one GPU's share of the 512 x 256 x 256 pipe under the axial slab decomposition (64- and
128-plane slabs, periodic in x in place of the halo exchange): step rate, sweep time, halo bytes.
accelerated = the accelerated magnetic iteration (alpha = 1/2, 135 sweeps) on the same box, with the
induction residual after a step next to the plain method's (an extra object, not `value`).
precision = float32 against the 16-bit storage forms on the 512 x 256 x 256 pipe at 270 sweeps
per step: the split form (b in float16 hi + lo, float16 copy of u for the sweeps) and the plain
offset forms (all float16; float16 / bfloat16 / float16), each with its per-field error against
the stored FP64 oracle run of the 8 x 32 x 32 pipe after 2000 steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch] [--no-precision]
                       [--no-accel]
HBM traffic of the sweep on the 512 x 256 x 256 pipe (rocprofv3 counters, scaled by a plain copy
of known size), after mkdir -p D1 D2:
  rocprofv3 --pmc FETCH_SIZE -d D1 -o run --output-format csv -- python3 bench.py --hbm-only \
      --hbm-sweeps 4 --calib-copy-mib 1024 > D1/hbm.json
  (the same with WRITE_SIZE into D2), then
  python3 bench.py --traffic-summary D1 D2 --calib-copy-mib 1024
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
SWEEP_BYTES_PER_CELL = 36  # read u (12 B) + b (12 B), write b* (12 B), float32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mag_sweep_pipe512_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2211_09370_amd", "csrc", "mhd_sweep.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def read_traffic(tiles):
    """HBM bytes per sweep launch from committed rocprofv3 counter runs, if the kernel source and
    the launch tiles are those the counters were taken with; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    if kv.get("tiles") != ",".join(str(int(t)) for t in tiles):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _counter_rows(d, counter):
    """(kernel name, value) of every dispatch in the rocprofv3 counter CSVs under directory d."""
    import csv
    import glob

    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def traffic_summary(fetch_dir, write_dir, copy_mib):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the sweep, scaled by what the same
    counters read for a plain copy of copy_mib MiB (the largest torch copy dispatch), written to
    the traffic file together with the hash of the kernel source and the launch tiles (from the
    roofline leg's JSON line, which the fetch run writes to hbm.json in its directory)."""
    leg_file = os.path.join(fetch_dir, "hbm.json")
    if not os.path.exists(leg_file):
        raise SystemExit(f"{leg_file} is missing: the FETCH_SIZE run writes the roofline leg's JSON line "
                         "there (it records the launch tiles the counters belong to)")
    leg = json.load(open(leg_file))["roofline"]
    tiles = ",".join(str(int(t)) for t in leg["tiles"])
    out = {}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _counter_rows(d, counter)
        sweep = [v for k, v in rows if "k_mag_sweep" in k]
        copy = [v for k, v in rows if ("copy" in k.lower() or "elementwise" in k.lower())]
        if not sweep or not copy:
            raise SystemExit(f"no sweep or copy dispatches with {counter} under {d}")
        expect_kib = copy_mib * 1024.0
        scale = expect_kib / max(copy)
        out[tag] = dict(raw_kib=sum(sweep) / len(sweep), n=len(sweep), copy_kib=max(copy), scale=scale)
    fetch_b = out["fetch"]["raw_kib"] * out["fetch"]["scale"] * 1024.0
    write_b = out["write"]["raw_kib"] * out["write"]["scale"] * 1024.0
    import workloads as W

    w = W.large_pipe(Rm=1e-2)
    alg = SWEEP_BYTES_PER_CELL * w.n_cells
    lines = [
        "# HBM-side traffic of the magnetic sweep on the 512 x 256 x 256 pipe (float32), per launch.",
        "# rocprofv3 --pmc FETCH_SIZE / --pmc WRITE_SIZE (KiB per dispatch, averaged over the sweep",
        "# dispatches), each scaled by the ratio of the known size of a plain torch copy to what the",
        "# same counter reads for it. Commands (after mkdir -p D1 D2):",
        f"#   rocprofv3 --pmc FETCH_SIZE -d D1 -o run --output-format csv -- python3 bench.py --hbm-only "
        f"--hbm-sweeps 4 --calib-copy-mib {copy_mib} > D1/hbm.json",
        "#   (the same with --pmc WRITE_SIZE into D2)",
        f"#   python3 bench.py --traffic-summary D1 D2 --calib-copy-mib {copy_mib}",
        f"fetch_kib_raw = {out['fetch']['raw_kib']:.1f}",
        f"fetch_dispatches = {out['fetch']['n']}",
        f"copy_fetch_kib_raw = {out['fetch']['copy_kib']:.1f}",
        f"fetch_scale = {out['fetch']['scale']:.4f}",
        f"write_kib_raw = {out['write']['raw_kib']:.1f}",
        f"write_dispatches = {out['write']['n']}",
        f"copy_write_kib_raw = {out['write']['copy_kib']:.1f}",
        f"write_scale = {out['write']['scale']:.4f}",
        f"algorithmic_bytes_per_launch = {alg}",
        f"hbm_bytes_per_launch = {fetch_b + write_b:.0f}",
        f"traffic_over_algorithmic = {(fetch_b + write_b) / alg:.4f}",
        f"kernel_source_sha256_16 = {kernel_hash()}",
        f"tiles = {tiles}",
    ]
    open(TRAFFIC_FILE, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def hbm_roofline_leg(n_sweeps=None, profile_steps=1):
    """The float32 sweep on the 512 x 256 x 256 pipe (state 1.9 GB, beyond the Infinity Cache):
    default tiles, one warm-up step, then the sweeps of `profile_steps` steps timed by the events
    each launch stamps at kernel start and end. n_sweeps overrides the sweeps per step (counter
    runs use a few; the kernel is the same)."""
    import torch

    import workloads as W
    from paper_2211_09370_amd import MHD_K_MAG_SWEEP, Sim

    w = W.large_pipe(Rm=1e-2)
    n_mag = n_sweeps or w.params.n_mag
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=torch.cuda.Stream())
    sim.set_markers(w.markers)
    sim.set_params(w.params, n_mag=n_mag)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    tiles = list(sim.tiles)
    sim.step(1)
    torch.cuda.synchronize()
    sim.set_profiling(True)
    sim.step(profile_steps)
    n_launch, ms_total = sim.kernel_stats(MHD_K_MAG_SWEEP)
    sim.set_profiling(False)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    avg_s = ms_total / 1e3 / max(n_launch, 1)
    alg_bytes = SWEEP_BYTES_PER_CELL * w.n_cells
    achieved = alg_bytes / avg_s / 1e9
    log(f"bench: 512x256^2 mag_sweep {n_launch} launches, avg {avg_s * 1e6:.2f} us, {achieved:.0f} GB/s")
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": read_traffic(tiles), "kernel": "mag_sweep",
            "workload": w.name, "box": [w.nx, w.ny, w.nz], "tiles": tiles, "launches": n_launch,
            "avg_launch_us": round(avg_s * 1e6, 3), "bytes_per_launch": alg_bytes,
            "gcells_per_s": round(w.n_cells / avg_s / 1e9, 2)}


def shard_leg(steps=3):
    """One GPU's share of the 512 x 256 x 256 pipe under the axial slab decomposition: the float32
    step on a 64-plane (one of eight GPUs) and a 128-plane (one of four) slab of the same pipe,
    periodic in x where the slabs would exchange halos (nothing crosses GPUs here). Reports the
    slab's step rate, its sweep and wall-correction times, and the halo a sweep would send (the two
    x faces of b, three float32 components each)."""
    import torch

    import workloads as W
    from paper_2211_09370_amd import MHD_K_IB, MHD_K_MAG_SWEEP, Sim

    res = []
    for n_gpu, nx in ((8, 64), (4, 128)):
        w = W.pipe_slab(nx)
        stream = torch.cuda.Stream()
        sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=stream)
        sim.set_markers(w.markers)
        sim.set_params(w.params)
        sim.set_field("rho", w.rho)
        sim.set_field("u", w.u)
        sim.set_field("b", w.b)
        sim.step(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        sim.set_profiling(True)
        sim.step(1)
        n_sw, ms_sw = sim.kernel_stats(MHD_K_MAG_SWEEP)
        n_ib, ms_ib = sim.kernel_stats(MHD_K_IB)
        sim.set_profiling(False)
        tiles = list(sim.tiles)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        sweep_us = ms_sw * 1e3 / max(n_sw, 1)
        halo = 2 * w.ny * w.nz * 12
        mlups = w.n_cells * steps / sec / 1e6
        log(f"bench: slab {nx}x256^2 (1 of {n_gpu}): {mlups:.1f} MLUPS, sweep {sweep_us:.2f} us, "
            f"halo {halo / 1e6:.2f} MB per sweep")
        res.append({"gpus": n_gpu, "slab": [w.nx, w.ny, w.nz], "tiles": tiles, "MLUPS": round(mlups, 3),
                    "ms_per_step": round(sec * 1e3 / steps, 4), "sweep_us": round(sweep_us, 3),
                    "sweep_alg_GBs": round(SWEEP_BYTES_PER_CELL * w.n_cells / (sweep_us * 1e-6) / 1e9, 1),
                    "wall_correction_us_per_sweep": round(ms_ib * 1e3 / max(n_sw, 1), 3),
                    "halo_bytes_per_sweep": halo,
                    "whole_pipe_MLUPS_if_halo_hidden": round(mlups * n_gpu, 1)})
    return {"workload": "axial slabs of the 512 x 256 x 256 pipe (R = 120, Ha 30, Re 5000, Rm 1e-2, "
                        "270 sweeps per step), periodic in x in place of the halo exchange",
            "shares": res}


def batched_leg(steps, seq_steps=2):
    """The batched form on 64 seeded pipes: autotuned tiles, graph replay, MLUPS over all cells;
    then the same pipes stepped one at a time as single boxes with the same tiles (graph replay
    too), each timed over seq_steps steps after one warm-up step."""
    import torch

    import workloads as W
    from paper_2211_09370_amd import MHD_K_MAG_SWEEP, Batch

    ps = W.batch_pipes()
    cells = sum(w.n_cells for w in ps)
    sweep_cells = sum(w.n_cells * w.params.n_mag for w in ps)
    markers = sum(w.markers.shape[1] for w in ps)
    B = Batch([(w.nx, w.ny, w.nz, w.markers.shape[1]) for w in ps])
    for p, w in zip(B.pipes, ps):
        p.set_markers(w.markers)
        p.set_params(w.params)
        p.set_field("u", W.batch_fields(w)[1])
    B.tune(3)
    B.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    B.set_profiling(True)
    B.step(1)
    n, ms = B.kernel_stats(MHD_K_MAG_SWEEP)
    B.set_profiling(False)
    tiles = [list(p.tiles) for p in B.pipes]
    B.close()
    del B
    torch.cuda.empty_cache()
    log(f"bench: batched {len(ps)} pipes, {steps} steps in {sec:.3f} s")
    from paper_2211_09370_amd import Sim

    seq = 0.0
    for w, t in zip(ps, tiles):
        s = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=torch.cuda.Stream())
        s.set_markers(w.markers)
        s.set_params(w.params)
        s.set_field("u", W.batch_fields(w)[1])
        s.tiles = t
        s.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(seq_steps)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t0
        s.close()
        del s
    torch.cuda.empty_cache()
    seq_mlups = cells * seq_steps / seq / 1e6
    log(f"bench: the same pipes one at a time: {seq_mlups:.1f} MLUPS")
    return {"workload": f"{len(ps)} pipes, R U[16,64], L in {{32,64,128,256}}, Ha log-U[1,50], "
                        f"Rm log-U[1e-4,1], Re U[50,1000], uniform or fringe field",
            "value": round(cells * steps / sec / 1e6, 3), "unit": "MLUPS", "steps": steps,
            "ms_per_step": round(sec * 1e3 / steps, 3), "cells": cells, "markers": markers,
            "sweep_cells_per_step": sweep_cells, "graph": True, "tiles": "autotuned",
            "sweep_alg_GBs": round(SWEEP_BYTES_PER_CELL * sweep_cells / (ms * 1e-3) / 1e9, 1),
            "sweep_gcell_per_s": round(sweep_cells * steps / sec / 1e9, 3),
            "sequential_MLUPS": round(seq_mlups, 3),
            "sequential_gcell_sweeps_per_s": round(sweep_cells * seq_steps / seq / 1e9, 3),
            "speedup_over_sequential": round(cells * steps / sec / 1e6 / seq_mlups, 4)}


def precision_leg(steps, with_error=True):
    """MLUPS of float32 and of the 16-bit storage forms on the large pipe, and each form's
    per-field error after 2000 steps of the small pipe against the stored oracle run (the split
    form is the accurate one; the plain offset forms are reported with theirs)."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2211_09370_amd import Sim

    w = W.large_pipe(Rm=1e-2)
    B_ind = 1e-2 * w.params.B0  # induced-field scale Rm B0
    forms = {"f32": {}, "f16split": dict(b_storage="f16split", u_scale=W.U0, b_scale=B_ind),
             "f16_f16_f16": dict(rho_storage="f16", u_storage="f16", b_storage="f16", u_scale=W.U0, b_scale=B_ind),
             "f16_bf16_f16": dict(rho_storage="f16", u_storage="bf16", b_storage="f16", u_scale=W.U0,
                                  b_scale=w.params.B0)}
    out = {"workload": w.name, "box": [w.nx, w.ny, w.nz], "n_mag": w.params.n_mag,
           "markers": int(w.markers.shape[1]), "steps": steps, "tiles": "autotuned per form (mhd_tune)"}
    for name, st in forms.items():
        sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=torch.cuda.Stream(), **st)
        sim.set_markers(w.markers)
        sim.set_params(w.params)
        sim.set_field("rho", w.rho)
        sim.set_field("u", w.u)
        sim.set_field("b", w.b)
        sim.tune(5)
        sim.step(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name + "_MLUPS"] = round(w.n_cells * steps / sec / 1e6, 3)
        out[name + "_tiles"] = list(sim.tiles)
        sim.close()
        del sim
        torch.cuda.empty_cache()
        log(f"bench: precision {name} {steps} steps in {sec:.3f} s")
    out["speedup_f16split_over_f32"] = round(out["f16split_MLUPS"] / out["f32_MLUPS"], 4)
    gold = os.path.join(ROOT, "tests", "golden", "oracle_pipe8x32x32_2000steps.npz")
    if with_error and os.path.exists(gold):
        ref = np.load(gold)
        ws = W.small_pipe()
        Rm_B0 = 1e-3 * ws.params.B0
        small = {"f16split": dict(b_storage="f16split", u_scale=W.U0, b_scale=Rm_B0),
                 "f16_f16_f16": dict(rho_storage="f16", u_storage="f16", b_storage="f16", u_scale=W.U0,
                                     b_scale=Rm_B0),
                 "f16_bf16_f16": dict(rho_storage="f16", u_storage="bf16", b_storage="f16", u_scale=W.U0,
                                      b_scale=ws.params.B0)}

        def e(a, r):
            return float(np.abs(a - r).max() / np.abs(r).max())

        rs = max(np.abs(ref["rho"] - 1).max(), math.sqrt(3) * np.abs(ref["u"]).max())
        for name, st in small.items():
            sim = Sim(ws.nx, ws.ny, ws.nz, ws.markers.shape[1], stream=torch.cuda.Stream(), **st)
            sim.set_markers(ws.markers)
            sim.set_params(ws.params)
            sim.set_field("rho", ws.rho)
            sim.set_field("u", ws.u)
            sim.set_field("b", ws.b)
            sim.step(int(ref["steps"]))
            out[name + "_error_vs_oracle"] = {
                "case": "8x32x32 pipe, Ha 5, 2000 steps, max-normalised",
                "u": e(sim.get_field("u"), ref["u"]), "b": e(sim.get_field("b"), ref["b"]),
                "rho": float(np.abs(sim.get_field("rho") - ref["rho"]).max() / rs)}
            sim.close()
            log(f"bench: precision {name} error after {int(ref['steps'])} steps: u {out[name + '_error_vs_oracle']['u']:.2e}")
    return out


def accelerated_leg(w, steps, warmup, res_plain):
    """MLUPS of the accelerated iteration (Sec. 5.8: alpha = 1/2 with half the sweeps, the same
    fixed point and the same error of the slow modes as the plain iteration with all of them) on
    the headline box, with the induction residual after the next step next to the plain run's,
    both after the same number of steps from the same state."""
    import torch

    from paper_2211_09370_amd import Sim

    n_mag = (w.params.n_mag + 1) // 2
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=torch.cuda.Stream())
    sim.set_markers(w.markers)
    sim.set_params(w.params, alpha=0.5, n_mag=n_mag)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    sim.step(1, 1)
    res = sim.budgets()[-1]["res_mag"]
    sim.close()
    log(f"bench: accelerated alpha 1/2, {n_mag} sweeps: {steps} steps in {sec:.3f} s, res_mag {res:.3e} "
        f"(plain {res_plain:.3e})")
    return {"method": "accelerated magnetic iteration, alpha = 1/2 (Sec. 5.8)", "n_mag": n_mag, "steps": steps,
            "value": round(w.n_cells * steps / sec / 1e6, 3), "unit": "MLUPS",
            "res_mag_after_step": res, "res_mag_after_step_plain_270": res_plain}


def transition_study(rms, forms, steps, every):
    """The unsteady large-pipe case across the quasi-static to canonical transition (Sec. 5.7):
    512 x 256 x 256, R = 120, Re = 5000 (tau = 0.5036), Ha = 30, for each Rm (eta = U0 R / Rm,
    n_mag = min(ceil(6 eta), 270)) and storage form, from the Poiseuille profile with a seeded
    divergence-free 5% perturbation, `steps` fluid steps with the energy budgets every `every`
    steps. One JSON line per run: stability (the first step flagged unstable, if any), mass
    drift, the kinetic balance dE_k/dt = P_in + P_p + P_nu + P_L along the run (central
    differences of the records, over max |sum P|), the energy series, and for the 16-bit form
    the per-field error against the float32 run at the end."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2211_09370_amd import Sim, _abi

    for Rm in rms:
        w = W.large_pipe_perturbed(Rm=Rm)
        ref = None
        for form in forms:
            store = {} if form == "f32" else dict(b_storage="f16split", u_scale=W.U0,
                                                  b_scale=Rm * w.params.B0)
            sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=torch.cuda.Stream(), **store)
            sim.set_markers(w.markers)
            sim.set_params(w.params)
            sim.set_field("rho", w.rho)
            sim.set_field("u", w.u)
            sim.set_field("b", w.b)
            sim.record_budget()
            recs, done, unstable_at = [], 0, None
            t0 = time.perf_counter()
            while done < steps:
                sim.step(every, every)
                done += every
                recs += sim.budgets()
                if sim.last_status == _abi.MHD_ERR_UNSTABLE:
                    unstable_at = done
                    break
                if done % (10 * every) == 0 or done == steps:
                    r = recs[-1]
                    log(f"bench: transition Rm {Rm:g} {form}: {done} steps, {time.perf_counter() - t0:.0f} s, "
                        f"E_k {r['E_k']:.4e} E_b {r['E_b']:.3e} u_max {r['u_max']:.4f}")
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            Ek = np.array([r["E_k"] for r in recs])
            P = np.array([r["P_in"] + r["P_p"] + r["P_nu"] + r["P_L"] for r in recs])
            mass = np.array([r["mass"] for r in recs])
            closure = None
            if len(recs) >= 3:
                dEk = (Ek[2:] - Ek[:-2]) / (2 * every)
                closure = float(np.abs(dEk - P[1:-1]).max() / np.abs(P).max())
            out = {"transition": {"workload": w.name, "Rm": Rm, "eta": w.params.eta, "n_mag": w.params.n_mag,
                                  "storage": form, "steps": done, "budget_every": every,
                                  "stable": unstable_at is None, "unstable_by_step": unstable_at,
                                  "ms_per_step": round(sec * 1e3 / max(done, 1), 3),
                                  "MLUPS": round(w.n_cells * done / sec / 1e6, 3),
                                  "mass_drift": float(np.abs(mass - mass[0]).max() / mass[0]),
                                  "kinetic_balance_residual": closure,
                                  "series": {k: [r[k] for r in recs] for k in
                                             ("step", "E_k", "E_m", "E_b", "P_in", "P_p", "P_nu", "P_L",
                                              "M_eta", "M_adv", "D_eta", "u_max", "res_mag")}}}
            if unstable_at is None:
                fields = [sim.get_field(f) for f in ("rho", "u", "b")]
                if form == "f32":
                    ref = fields
                elif ref is not None:
                    e = [float(np.abs(a - r).max() / np.abs(r if i else r - 1.0).max())
                         for i, (a, r) in enumerate(zip(fields, ref))]
                    out["transition"]["error_vs_f32"] = {"rho_minus_1": e[0], "u": e[1], "b": e[2]}
            sim.close()
            del sim
            torch.cuda.empty_cache()
            log(f"bench: transition Rm {Rm:g} {form}: stable {unstable_at is None}, {done} steps in {sec:.0f} s, "
                f"balance {closure}, error {out['transition'].get('error_vs_f32')}")
            print(json.dumps(out), flush=True)


def cpu_baseline(slab=16, reps=5):
    """The oracle on a slab of the headline pipe: the same 128 x 128 cross-section, radius, markers
    per plane, physics and 270 sweeps per step, `slab` planes long (the fringe centred in it),
    one warm-up step, then the median of `reps` timed steps."""
    import statistics

    import oracle
    import workloads as W

    w = W.pipe_workload("pipe16x128x128_R60_fringe_Ha20", 2, slab, 128, 128, 60.0, 500.0, 20.0, 1e-2,
                        bext_kind=W.BEXT_TANH_FRINGE_Y, fringe_x0=slab / 2.0, fringe_w=8.0)
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    o.step(1)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.step(1)
        times.append(time.perf_counter() - t0)
    o.close()
    t = statistics.median(times)
    log(f"bench: oracle steps {', '.join(f'{x:.2f}' for x in times)} s")
    return {"value": w.n_cells / t / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"FP64 oracle on a {w.nx}x{w.ny}x{w.nz} slab of the same pipe ({w.n_cells} cells, "
                       f"{w.markers.shape[1]} markers, {w.params.n_mag} sweeps per step): median of "
                       f"{reps} steps ({t:.2f} s each) after one warm-up step")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-accel", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=3)
    ap.add_argument("--no-precision-error", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--calib-copy-mib", type=int, default=0)
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--hbm-only", action="store_true", help="only the 512 x 256^2 sweep roofline leg")
    ap.add_argument("--hbm-sweeps", type=int, default=0, help="sweeps per step of that leg (0: 270)")
    ap.add_argument("--no-hbm", action="store_true")
    ap.add_argument("--no-shard", action="store_true", help="skip the one-GPU-share slab leg")
    ap.add_argument("--transition", nargs="+", type=float, metavar="RM",
                    help="run the unsteady large-pipe case at these Rm instead of the benchmark")
    ap.add_argument("--transition-forms", nargs="+", default=["f32", "f16split"])
    ap.add_argument("--transition-every", type=int, default=100)
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.calib_copy_mib or 1024)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {args.gpus} requested); "
              "the multi-GPU axial slab design is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2211_09370_amd import MHD_K_MAG_SWEEP, Sim

    torch.cuda.set_device(0)
    if args.calib_copy_mib:  # plain copy of known size, for counter calibration
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
    if args.hbm_only:
        print(json.dumps({"roofline": hbm_roofline_leg(args.hbm_sweeps or None)}), flush=True)
        return
    if args.transition:
        transition_study(args.transition, args.transition_forms, args.steps, args.transition_every)
        return
    w = W.fringe_pipe()
    M = w.markers.shape[1]
    log(f"bench: {w.name} N={w.n_cells} M={M} n_mag={w.params.n_mag}")
    # the solver's own stream: steps replay as captured HIP graphs (the NULL stream cannot be captured)
    stream = torch.cuda.Stream()
    sim = Sim(w.nx, w.ny, w.nz, M, stream=stream)
    sim.set_markers(w.markers)
    sim.set_params(w.params)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)

    sim.step(args.warmup)
    torch.cuda.synchronize()
    log(f"bench: warmup {args.warmup} steps done")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    log(f"bench: timed {args.steps} steps: {gpu_ms:.1f} ms (events), {wall * 1e3:.1f} ms (wall)")
    sec = max(wall, gpu_ms / 1e3)
    mlups = w.n_cells * args.steps / sec / 1e6

    # dominant kernel: event-bracketed launches on the solver's stream
    sim.set_profiling(True)
    sim.step(args.profile_steps)
    n_launch, ms_total = sim.kernel_stats(MHD_K_MAG_SWEEP)
    sim.set_profiling(False)
    avg_s = ms_total / 1e3 / max(n_launch, 1)
    alg_bytes = SWEEP_BYTES_PER_CELL * w.n_cells
    achieved = alg_bytes / avg_s / 1e9
    log(f"bench: mag_sweep {n_launch} launches, avg {avg_s * 1e6:.2f} us, {achieved:.0f} GB/s")

    import numpy as np

    state_ok = bool(np.isfinite(sim.get_field("u")).all())
    accel = None
    if not args.no_accel:
        sim.step(1, 1)  # one recorded step: the induction residual left by 270 plain sweeps
        res_plain = sim.budgets()[-1]["res_mag"]
    sim.close()
    if not args.no_accel:
        accel = accelerated_leg(w, args.steps, args.warmup + args.profile_steps, res_plain)

    hbm = None if args.no_hbm else hbm_roofline_leg(args.hbm_sweeps or None)
    shard = None if args.no_shard else shard_leg()
    batched = None
    if not args.no_batch:
        batched = batched_leg(args.batch_steps)
    precision = None
    if not args.no_precision:
        precision = precision_leg(args.precision_steps, not args.no_precision_error)

    cpu = None
    if not args.no_cpu:
        log("bench: timing the oracle on the host")
        cpu = cpu_baseline()

    out = {
        "metric": "MLUPS (fluid steps x box cells / s) at 270 magnetic sweeps per step",
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "box": [w.nx, w.ny, w.nz], "radius": w.R, "markers": M,
                   "n_mag": w.params.n_mag, "field": "tanh fringe along y", "Ha": 20, "Re": 500,
                   "Rm": 0.01, "storage": "f32", "parallelism": "single GPU"},
        "roofline": hbm,
        "roofline_cache_resident": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                                    "traffic": None, "kernel": "mag_sweep", "workload": w.name,
                                    "note": "136 MB state held by the 256 MB Infinity Cache",
                                    "avg_launch_us": round(avg_s * 1e6, 3), "bytes_per_launch": alg_bytes,
                                    "gcells_per_s": round(w.n_cells / avg_s / 1e9, 2)},
        "sweep_glups": round(w.n_cells * (w.params.n_mag + 1) * args.steps / sec / 1e9, 3),
        "finite": state_ok,
        "accelerated": accel,
        "batched": batched,
        "shard": shard,
        "precision": precision,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
