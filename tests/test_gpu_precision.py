"""Reduced-precision storage against the FP64 oracle, per field.

Forms (all arithmetic float32; budgets and the flow-rate sum float64):
* offsets, as specified for the precision case of the 8 x 32 x 32 pipe: rho - 1 in float16,
  u in bfloat16 scaled by U0, b in float16 scaled by B0. Every stored value is rounded at every
  write; the magnetic iteration rewrites b 270 times per fluid step and its slowest modes
  contract by only ~1/150 per sweep, so the rounding piles up in b and, through the Lorentz force,
  in u (measured u errors 4.2e-1 and 8.0e-2 after 2000 steps). The 1e-3 velocity target is
  asserted for them as an expected failure (strict: the test fails if a form ever meets it, so
  the claim that it cannot is checked too); their measured errors are reported by the benchmark.
* offsets, all float16, with b scaled by the induced-field scale Rm B0 (b / b_scale ~ 0.1 instead
  of ~1e-4, i.e. out of float16's subnormal range).
* split (f16split): rho and u float32, b = (hi + lo) Rm B0 in two float16 arrays, hi re-quantised
  once per fluid step, the sweeps updating lo; the sweeps read a float16 copy of u. The rounding
  of the iteration is then relative to the change of b within a step. Target: velocity within
  1e-3 (max-normalised) of the oracle after 2000 steps.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from tests.test_gpu_parity import compare, err, oracle_run, random_box

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "oracle_pipe8x32x32_2000steps.npz")


def forms(w):
    Rm_B0 = 1e-3 * w.params.B0
    return {
        "f16/bf16/f16 (b / B0)": dict(rho_storage="f16", u_storage="bf16", b_storage="f16", u_scale=W.U0,
                                     b_scale=w.params.B0),
        "f16/f16/f16 (b / Rm B0)": dict(rho_storage="f16", u_storage="f16", b_storage="f16", u_scale=W.U0,
                                       b_scale=Rm_B0),
        "f32/f32/f16-split (b / Rm B0)": dict(b_storage="f16split", u_scale=W.U0, b_scale=Rm_B0),
    }


TARGET = 1e-3  # velocity error of the 16-bit forms (max-normalised) after 2000 steps
CANNOT_MEET = pytest.mark.xfail(strict=True, reason=(
    "plain 16-bit offsets round b at each of the 270 sweeps of a step and the slowest modes "
    "contract by ~1/150 per sweep: the rounding accumulates about 150-fold (u 4e-1 / 8e-2)"))
NAMES = [pytest.param("f16/bf16/f16 (b / B0)", marks=CANNOT_MEET),
         pytest.param("f16/f16/f16 (b / Rm B0)", marks=CANNOT_MEET),
         "f32/f32/f16-split (b / Rm B0)"]


def run(w, steps, store, **over):
    from paper_2211_09370_amd import Sim

    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], **store)
    sim.set_markers(w.markers)
    sim.set_params(w.params, **over)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    sim.step(steps)
    return sim


def field_errors(sim, rho, u, b):
    rho_scale = max(np.abs(rho - 1.0).max(), math.sqrt(3.0) * np.abs(u).max())
    return (np.abs(sim.get_field("rho") - rho).max() / rho_scale, err(sim.get_field("u"), u),
            err(sim.get_field("b"), b))


_F32 = {}


def f32_reference(w, steps):
    if steps not in _F32:
        s = run(w, steps, {})
        _F32[steps] = (s.get_field("rho"), s.get_field("u"), s.get_field("b"))
        s.close()
    return _F32[steps]


@pytest.mark.parametrize("name", NAMES)
def test_small_pipe_2000_steps_per_field_error(name):
    if not os.path.exists(GOLD):
        pytest.skip("stored oracle run missing (tests/golden/make_oracle_pipe8.py writes it)")
    ref = np.load(GOLD)
    w = W.small_pipe()
    steps = int(ref["steps"])
    print("case", name, flush=True)
    sim = run(w, steps, forms(w)[name])
    e_o = field_errors(sim, ref["rho"], ref["u"], ref["b"])
    e_g = field_errors(sim, *f32_reference(w, steps))
    print(f"{name}: vs oracle rho-1 {e_o[0]:.2e} u {e_o[1]:.2e} b {e_o[2]:.2e} | "
          f"vs GPU f32 rho-1 {e_g[0]:.2e} u {e_g[1]:.2e} b {e_g[2]:.2e}", flush=True)
    assert all(np.isfinite(e_o))
    assert e_o[1] <= TARGET, ("u", e_o[1])
    if "split" in name:
        assert e_o[2] <= TARGET and e_o[0] <= TARGET, e_o


SPLIT = dict(b_storage="f16split", u_scale=0.05, b_scale=0.01)


@pytest.mark.parametrize("shape", [(37, 21, 13), (128, 13, 9), (256, 6, 5)])
def test_split_form_one_step(shape):
    """One step from a random state (b changes by O(b) per sweep there, so the lo rounding is
    O(2^-12 b): bound 2e-3). nx = 128, 256 take the paired sweep."""
    print("case split", shape, flush=True)
    from paper_2211_09370_amd import Sim

    w = random_box(*shape, key=210, n_mag=3)
    sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], **SPLIT)
    sim.set_markers(w.markers)
    sim.set_params(w.params)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)
    # set_field splits b exactly enough that reading it back is the input to float32 rounding
    assert err(sim.get_field("b"), w.b) < 1e-6
    sim.step(1)
    compare(sim, oracle_run(w, 1), tol=2e-3, label=f"split {shape}")


def test_split_form_quarter_fringe_20_steps():
    """From rest, b grows from zero. In this transient lo carries the whole change of b within a
    step, O(b), and the iteration's slowest mode contracts by only ~1/150 per sweep, so the
    float16 rounding of lo (half an ulp, 2^-12 of lo) is carried ~150-fold: up to ~4e-2 of b
    (measured 9e-3). b is therefore held to 2e-2 here; u feels b only through the Lorentz force
    and keeps the 1e-3 velocity target (measured 7e-5). Near steady state lo is small and the
    2000-step run meets 1e-3 in every field."""
    w = W.quarter_fringe_pipe()
    Rm_B0 = 1e-2 * w.params.B0
    print("case split fringe32", flush=True)
    sim = run(w, 20, dict(b_storage="f16split", u_scale=W.U0, b_scale=Rm_B0))
    o = oracle_run(w, 20)
    e_r, e_u, e_b = field_errors(sim, o.rho, o.u, o.b)
    print(f"split fringe32 20 steps err rho-1 {e_r:.2e} u {e_u:.2e} b {e_b:.2e}", flush=True)
    assert e_u <= 1e-3 and e_r <= 1e-3 and e_b <= 2e-2, (e_r, e_u, e_b)


def test_sixteen_bit_forms_with_the_six_magnet_field():
    """The (y, z) table of the six-magnet field staged with 16-bit u and b (every storage form,
    paired sweep), one step of four sweeps against the oracle: the split form within its
    one-step bar, the plain offset forms within loose bounds recorded from measurement."""
    from paper_2211_09370_amd import Sim

    w = W.pipe_workload("six_magnets", 7, 128, 33, 33, 14.0, 50.0, 10.0, 1e-2, bext_kind=W.BEXT_SIX_MAGNETS,
                        n_mag=4, b_amp=1e-4, noise=1e-2)
    o = oracle_run(w, 1)
    Rm_B0 = 1e-2 * w.params.B0
    cases = {"split": (dict(b_storage="f16split", u_scale=W.U0, b_scale=Rm_B0), 2e-3),
             "f16/f16/f16": (dict(rho_storage="f16", u_storage="f16", b_storage="f16", u_scale=W.U0,
                                  b_scale=Rm_B0), 3e-3),  # measured 7.6e-4 (u)
             "f16/bf16/f16": (dict(rho_storage="f16", u_storage="bf16", b_storage="f16", u_scale=W.U0,
                                   b_scale=w.params.B0), 2e-2)}  # measured 6.1e-3 (u)
    for name, (store, bound) in cases.items():
        print("case six magnets", name, flush=True)
        sim = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], **store)
        sim.set_markers(w.markers)
        sim.set_params(w.params)
        sim.set_field("rho", w.rho)
        sim.set_field("u", w.u)
        sim.set_field("b", w.b)
        sim.step(1)
        e = field_errors(sim, o.rho, o.u, o.b)
        print(f"six magnets {name}: err rho-1 {e[0]:.2e} u {e[1]:.2e} b {e[2]:.2e}", flush=True)
        sim.close()
        assert max(e) <= bound, (name, e)
