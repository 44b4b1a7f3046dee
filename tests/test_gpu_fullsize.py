"""Full-size configurations on the GPU, checked at sampled cells against the oracle.

The oracle cannot step a 512 x 256 x 256 box or the 60-million-cell 64-pipe batch, but one step
is local (tests/subbox.py, pinned in tests/test_subbox_cpu.py): at a sampled cell the oracle run
on a small box cut around it gives the whole-box value. The GPU runs the whole box in the
launch configuration the benchmark times (default tiles, graphs for the batch) with two
sweeps per step (the sweep count only repeats the same launches), then the sampled cells are
compared: near and on the wall, on the axis, at tile and box edges, at the periodic seams.
Bars: the float32 bar 1e-5 of each field's maximum; the split form's one-step bar 2e-3.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.subbox import influence_radius, oracle_cell

pytestmark = pytest.mark.gpu

N_MAG = 2


def _sample_cells(w, n, key, margin_x=0):
    g = W.rng_for(key)
    yc, zc, R = int(w.params.yc), int(w.params.zc), w.R
    lo, hi = margin_x, w.nx - 1 - margin_x
    cells = [(lo, yc, zc), (hi, yc, zc), ((lo + hi) // 2, yc, zc), ((lo + hi) // 2, 0, 0),
             (min(hi, max(lo, 127)), min(w.ny - 1, yc + 4), zc)]
    for k in range(n):
        th = g.uniform(0, 2 * math.pi)
        rr = R + g.uniform(-2.5, 2.5) if k % 2 == 0 else g.uniform(0, R)
        cx = int(g.integers(lo, hi + 1))
        cy = int(round(yc + rr * math.cos(th))) % w.ny
        cz = int(round(zc + rr * math.sin(th))) % w.nz
        cells.append((cx, cy, cz))
    return cells


def _compare_cells(label, w, fields, cells, tol, **over):
    rho, u, b = fields
    us, bs = np.abs(u).max(), np.abs(b).max()
    rs = max(np.abs(rho - 1.0).max(), math.sqrt(3.0) * us)
    worst = [0.0, 0.0, 0.0]
    for (cx, cy, cz) in cells:
        r_o, u_o, b_o = oracle_cell(w, (cx, cy, cz), N_MAG, **over)
        worst[0] = max(worst[0], abs(rho[cz, cy, cx] - r_o) / rs)
        worst[1] = max(worst[1], np.abs(u[:, cz, cy, cx] - u_o).max() / us)
        worst[2] = max(worst[2], np.abs(b[:, cz, cy, cx] - b_o).max() / bs)
    print(f"{label}: {len(cells)} cells, err rho-1 {worst[0]:.2e} u {worst[1]:.2e} b {worst[2]:.2e}", flush=True)
    assert max(worst) <= tol, (label, worst)


def _large():
    return W.large_pipe(Rm=1e-2, noise=1e-2, rho_amp=1e-3, b_amp=1e-3)


@pytest.mark.parametrize("form", ["f32", "f16split"])
def test_large_pipe_full_size_sampled_cells(form):
    from paper_2211_09370_amd import Sim

    w = _large()
    print("case large pipe", form, w.nx, w.ny, w.nz, flush=True)
    store = {} if form == "f32" else dict(b_storage="f16split", u_scale=W.U0, b_scale=1e-2 * w.params.B0)
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], **store)
    sim.set_markers(w.markers)
    sim.set_params(w.params, n_mag=N_MAG)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    print("tiles", tuple(sim.tiles), flush=True)
    sim.step(1)
    fields = (sim.get_field("rho"), sim.get_field("u"), sim.get_field("b"))
    sim.close()
    assert all(np.isfinite(f).all() for f in fields)
    cells = _sample_cells(w, 24, key=600)
    _compare_cells(f"large {form}", w, fields, cells, 1e-5 if form == "f32" else 2e-3)


def test_perturbed_large_pipe_three_steps_sampled_cells():
    """The unsteady large-pipe case as specified (Poiseuille profile plus a divergence-free 5%
    perturbation, Re = 5000, tau = 0.5036), three steps of two sweeps in float32 at full size,
    checked at sampled cells against the oracle run for the same three steps on a box cut with
    three steps' influence radius."""
    from paper_2211_09370_amd import Sim

    steps = 3
    w = W.large_pipe_perturbed(Rm=1.0)
    print("case perturbed large pipe", steps, "steps", flush=True)
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1])
    sim.set_markers(w.markers)
    sim.set_params(w.params, n_mag=N_MAG)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    sim.step(steps)
    fields = (sim.get_field("rho"), sim.get_field("u"), sim.get_field("b"))
    sim.close()
    assert all(np.isfinite(f).all() for f in fields)
    cells = _sample_cells(w, 8, key=650)
    rho, u, b = fields
    us, bs = np.abs(u).max(), np.abs(b).max()
    rs = max(np.abs(rho - 1.0).max(), math.sqrt(3.0) * us)
    worst = [0.0, 0.0, 0.0]
    for c in cells:
        r_o, u_o, b_o = oracle_cell(w, c, N_MAG, steps=steps)
        cx, cy, cz = c
        worst[0] = max(worst[0], abs(rho[cz, cy, cx] - r_o) / rs)
        worst[1] = max(worst[1], np.abs(u[:, cz, cy, cx] - u_o).max() / us)
        worst[2] = max(worst[2], np.abs(b[:, cz, cy, cx] - b_o).max() / bs)
    print(f"perturbed large pipe {steps} steps: {len(cells)} cells, err rho-1 {worst[0]:.2e} "
          f"u {worst[1]:.2e} b {worst[2]:.2e}", flush=True)
    assert max(worst) <= 1e-5, worst


def test_batch_64_pipes_full_size_sampled_cells():
    from paper_2211_09370_amd import Batch

    pipes = W.batch_pipes(noise=1e-2)
    print("case batch 64 pipes", sum(w.nx * w.ny * w.nz for w in pipes), "cells", flush=True)
    B = Batch([(w.nx, w.ny, w.nz, w.markers.shape[1]) for w in pipes])
    for p, w in zip(B.pipes, pipes):
        rho, u, b = W.batch_fields(w)
        p.set_markers(w.markers)
        p.set_params(w.params, n_mag=N_MAG)
        p.set_field("rho", rho)
        p.set_field("u", u)
        p.set_field("b", b)
    B.step(1)  # graphs
    r = influence_radius(N_MAG) + 3
    checked = 0
    for i in range(0, len(pipes), 4):  # every fourth pipe: uniform and fringe fields, all lengths
        w = pipes[i]
        w.rho, w.u, w.b = W.batch_fields(w)
        margin = r if w.params.bext_kind == W.BEXT_TANH_FRINGE_Y else 0
        if w.nx - 1 - 2 * margin < 0:
            continue
        p = B.pipes[i]
        fields = (p.get_field("rho"), p.get_field("u"), p.get_field("b"))
        assert all(np.isfinite(f).all() for f in fields)
        _compare_cells(f"batch pipe {i} ({w.nx}x{w.ny}x{w.nz}, kind {w.params.bext_kind})", w, fields,
                       _sample_cells(w, 4, key=700 + i, margin_x=margin), 1e-5)
        checked += 1
    B.close()
    assert checked >= 10


def test_maximum_box_sampled_cells():
    """The largest box the library takes (3 nx ny nz < 2^31): 1024 x 1024 x 680 = 713 M cells, so
    a vector field spans 8.6 GB (the per-component 32-bit offsets stay below 4 GB), 1.93 M
    markers on a radius-300 pipe; one step with one sweep, checked at sampled cells including the
    box's last cell and its first."""
    import time

    from paper_2211_09370_amd import Sim

    nx, ny, nz, R = 1024, 1024, 680, 300.0
    assert 3 * nx * ny * nz < 2 ** 31
    t0 = time.time()
    w = W.pipe_workload("pipe_max", 8, nx, ny, nz, R, 500.0, 20.0, 1e-2, n_mag=1, noise=1e-2)
    cells = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, int(w.params.yc) + 300, int(w.params.zc))]
    cells += _sample_cells(w, 9, key=800)
    ref = [oracle_cell(w, c, 1) for c in cells]  # before the full-size inputs are dropped
    print(f"case maximum box: inputs and {len(cells)} oracle cells in {time.time() - t0:.0f} s", flush=True)
    sim = Sim(nx, ny, nz, w.markers.shape[1])
    sim.set_markers(w.markers)
    sim.set_params(w.params)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    w.rho = w.u = w.b = None
    print(f"maximum box: set up in {time.time() - t0:.0f} s, stepping", flush=True)
    sim.step(1)
    got = {}
    for f in ("rho", "u", "b"):
        a = sim.get_field(f)
        assert np.isfinite(a).all(), f
        got[f] = [a[(..., cz, cy, cx)].copy() for cx, cy, cz in cells]
        got[f + "_max"] = float(np.abs(a - 1.0).max() if f == "rho" else np.abs(a).max())
        del a
    sim.close()
    us, bs = got["u_max"], got["b_max"]
    rs = max(got["rho_max"], math.sqrt(3.0) * us)
    e = [max(abs(float(got["rho"][i]) - ref[i][0]) for i in range(len(cells))) / rs,
         max(np.abs(got["u"][i] - ref[i][1]).max() for i in range(len(cells))) / us,
         max(np.abs(got["b"][i] - ref[i][2]).max() for i in range(len(cells))) / bs]
    print(f"maximum box: {len(cells)} cells, err rho-1 {e[0]:.2e} u {e[1]:.2e} b {e[2]:.2e}, "
          f"{time.time() - t0:.0f} s", flush=True)
    assert max(e) <= 1e-5, e


def test_fringe_pipe_long_run_budget_series():
    """The 128^3 fringe configuration stepped for its full 10,000 steps with the energy budgets
    logged every 100 steps: the state stays finite, the mass (float64 sum of the float32 density) stays
    constant, and the kinetic-energy balance of Sec. 4 holds along the transient, dE_k/dt =
    P_in + P_p + P_nu + P_L with dE_k/dt the central difference of the records (the same balance
    the oracle pins step by step), here over the whole run of the full-size box."""
    import time

    from paper_2211_09370_amd import Sim

    w = W.fringe_pipe()
    steps, every = 10000, 100
    print("case fringe pipe long run", steps, "steps", flush=True)
    t0 = time.time()
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1])
    sim.set_markers(w.markers)
    sim.set_params(w.params)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    sim.record_budget()
    for k in range(steps // 1000):
        sim.step(1000, every)
        print(f"fringe pipe long run: {1000 * (k + 1)} steps, {time.time() - t0:.0f} s", flush=True)
    rec = sim.budgets()
    assert np.isfinite(sim.get_field("u")).all()
    sim.close()
    assert len(rec) == steps // every + 1 and all(r["step"] == every * i for i, r in enumerate(rec))
    mass = np.array([r["mass"] for r in rec])
    assert np.abs(mass - mass[0]).max() <= 1e-7 * mass[0], np.abs(mass - mass[0]).max() / mass[0]
    Ek = np.array([r["E_k"] for r in rec])
    P = np.array([r["P_in"] + r["P_p"] + r["P_nu"] + r["P_L"] for r in rec])
    dEk = (Ek[2:] - Ek[:-2]) / (2 * every)
    resid = np.abs(dEk - P[1:-1]).max() / np.abs(P).max()
    print(f"fringe pipe long run: E_k {Ek[0]:.3e} -> {Ek[-1]:.3e}, max |dE_k/dt - sum P| / max |sum P| "
          f"{resid:.2e}, mass drift {np.abs(mass - mass[0]).max() / mass[0]:.1e}", flush=True)
    assert resid <= 0.05
