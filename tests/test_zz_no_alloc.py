"""The allocation-free step (mhd_step_noalloc) against mhd_step, through the C ABI.

mhd_step_noalloc runs the kernels of mhd_step with their scratch in the library's static device
array instead of the solver's workspace, so twin solvers stepped by the two calls must hold the
same fields bit for bit. Two calls in a row on different solvers, the second on a smaller box
(the shared array keeps the first call's contents, which the second must not depend on), with
budget records, the split storage form and flow control; a box whose scratch exceeds the array
is rejected.
"""
import numpy as np
import pytest

import workloads as W
from tests.test_gpu_parity import random_box

pytestmark = pytest.mark.gpu


def _twins(w, **store):
    from paper_2211_09370_amd import Sim

    out = []
    for _ in range(2):
        s = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], **store)
        s.set_markers(w.markers)
        s.set_params(w.params)
        s.set_field("rho", w.rho)
        s.set_field("u", w.u)
        s.set_field("b", w.b)
        out.append(s)
    return out


def _same(a, b, label):
    for f in ("rho", "u", "b"):
        x, y = a.get_field(f), b.get_field(f)
        assert np.array_equal(x, y), (label, f, float(np.abs(x - y).max()))
    assert a.time() == b.time(), label


def test_noalloc_step_matches_step_on_two_calls_in_a_row():
    """Calls in a row on shrinking boxes: 128 x 40 x 36 (paired sweep with x neighbours by wave
    rotation, line tables), 64 x 40 x 36 with flow control (single-cell sweep), 8 x 32 x 32."""
    wide = random_box(128, 40, 36, key=901, n_mag=4, R=14.0)
    big = random_box(64, 40, 36, key=900, n_mag=5, R=14.0)
    big.params.flow_control = 1
    big.params.u_bulk_target = 0.02
    small = W.small_pipe()
    small.params.n_mag = 7
    print("case noalloc: 128x40x36, 64x40x36, then 8x32x32", flush=True)
    for w, steps, every in ((wide, 2, 1), (big, 3, 1), (small, 2, 2)):
        ref, got = _twins(w)
        ref.step(steps, every)
        got.step_noalloc(steps, every)
        _same(ref, got, w.name)
        ra, rb = ref.budgets(), got.budgets()
        assert len(ra) == len(rb) == steps // every
        for x, y in zip(ra, rb):
            assert x == y, (w.name, x, y)
        ref.close()
        got.close()


def test_noalloc_step_in_the_split_form_and_after_plain_steps():
    w = W.quarter_fringe_pipe()
    w.params.n_mag = 6
    store = dict(b_storage="f16split", u_scale=W.U0, b_scale=1e-2 * w.params.B0)
    print("case noalloc: split form 32^3", flush=True)
    ref, got = _twins(w, **store)
    ref.step(2)
    got.step(1)          # graph replay on the workspace scratch, then the static scratch
    got.step_noalloc(1)
    _same(ref, got, "split")
    ref.close()
    got.close()


def test_noalloc_step_rejects_a_box_beyond_the_static_scratch():
    from paper_2211_09370_amd import MhdError, Sim, _abi

    sim = Sim(256, 256, 64, 0)  # 4.2 M cells: 50 MB of Lorentz force alone
    sim.set_params(W.Params(nu=0.1, eta=1.0, n_mag=1))
    with pytest.raises(MhdError) as e:
        sim.step_noalloc(1)
    assert e.value.status == _abi.MHD_ERR_INVALID_ARG
    sim.step(1)  # mhd_step still serves it
    sim.close()
