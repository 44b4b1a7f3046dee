"""Batched form (`mhd_batch_*`): many boxes of different size, marker set, parameters and sweep
count advanced by shared launches (and replayed HIP graphs).

Every box of a batch must evolve bitwise as the same box stepped alone with the same sweep
tiles (the batched kernels run the single-box bodies on per-box arguments), and through that,
or directly, within the float32 bar of the FP64 oracle.
"""
import numpy as np
import pytest

import workloads as W
from tests.test_gpu_parity import compare, oracle_run, random_box

pytestmark = pytest.mark.gpu


def batch_spec():
    """Six boxes: odd / even sweep counts, the paired sweep form (nx = 128, 256), a box without
    wall, flow-rate control, an oscillating force, uniform, fringe and six-magnet fields. Alone,
    the nx = 128 box takes its x neighbours by wave rotation; in the batch the same kernel stages
    halo columns, so the bitwise comparison also checks the two forms against each other."""
    a = random_box(8, 32, 32, key=300, n_mag=7, R=12.0)
    b = random_box(32, 32, 32, key=301, n_mag=4, R=13.0, bext_kind=W.BEXT_UNIFORM_Y)
    c = random_box(128, 20, 20, key=302, n_mag=5, R=7.0)
    c.params.flow_control = 1
    c.params.u_bulk_target = 0.02
    d = random_box(37, 21, 13, key=303, n_mag=3)
    e = random_box(256, 12, 10, key=304, n_mag=1, R=3.5, bext_kind=W.BEXT_UNIFORM_Y)
    e.params.G1 = 1e-5
    e.params.period = 7.0
    f = W.pipe_workload("six_magnets", 305, 16, 33, 33, 14.0, 50.0, 10.0, 1e-2,
                        bext_kind=W.BEXT_SIX_MAGNETS, n_mag=6, b_amp=1e-3)
    return [(a, True), (b, True), (c, True), (d, False), (e, True), (f, True)]


def setup(sim, w, markers):
    if markers:
        sim.set_markers(w.markers)
    sim.set_params(w.params)
    sim.set_field("rho", w.rho)
    sim.set_field("u", w.u)
    sim.set_field("b", w.b)


STORE = {"f32": {}, "f16": dict(rho_storage="f16", u_storage="f16", b_storage="f16",
                                 u_scale=0.05, b_scale=0.01),
         "f16split": dict(b_storage="f16split", u_scale=0.05, b_scale=0.01)}


def make_batch(spec, storage="f32"):
    from paper_2211_09370_amd import Batch

    B = Batch([(w.nx, w.ny, w.nz, w.markers.shape[1] if m else 0) for w, m in spec], **STORE[storage])
    for p, (w, m) in zip(B.pipes, spec):
        setup(p, w, m)
    return B


def make_singles(spec, tiles, storage="f32"):
    from paper_2211_09370_amd import Sim

    out = []
    for (w, m), t in zip(spec, tiles):
        s = Sim(w.nx, w.ny, w.nz, w.markers.shape[1] if m else 0, **STORE[storage])
        setup(s, w, m)
        s.tiles = t
        out.append(s)
    return out


def assert_same(p, s, label):
    for f in ("rho", "u", "b"):
        a, b = p.get_field(f), s.get_field(f)
        assert np.array_equal(a, b), (label, f, float(np.abs(a - b).max()))
    assert p.time() == s.time(), (label, p.time(), s.time())


@pytest.mark.parametrize("storage", ["f32", "f16", "f16split"])
def test_batch_matches_single_boxes_bitwise(storage):
    print("case batch vs single", storage, flush=True)
    spec = batch_spec()
    B = make_batch(spec, storage)
    S = make_singles(spec, [p.tiles for p in B.pipes], storage)
    assert B.pipes[2].tiles[2] == 1 and B.pipes[4].tiles[2] == 1  # paired form in use
    B.step(3)  # graphs
    for s in S:
        s.step(3)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"graph pipe {i}")
    B.set_graph(False)
    B.step(2)  # direct launches
    for s in S:
        s.step(2)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"direct pipe {i}")
    B.close()


def test_batch_pipes_match_oracle():
    print("case batch vs oracle", flush=True)
    spec = batch_spec()
    B = make_batch(spec)
    B.step(3)
    for i, (p, (w, m)) in enumerate(zip(B.pipes, spec)):
        compare(p, oracle_run(w, 3, markers=m), label=f"batch pipe {i}")
    B.close()


def test_batch_budgets_match_single_boxes():
    print("case batch budgets", flush=True)
    spec = batch_spec()
    B = make_batch(spec)
    S = make_singles(spec, [p.tiles for p in B.pipes])
    B.step(4, budget_every=2)
    for s in S:
        s.step(4, 2)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        rb, rs = p.budgets(), s.budgets()
        assert len(rb) == 2 and rb == rs, (i, rb, rs)
    B.close()


def test_batch_tune_keeps_state_and_parity():
    print("case batch tune", flush=True)
    spec = batch_spec()
    B = make_batch(spec)
    before = [[p.get_field(f) for f in ("rho", "u", "b")] for p in B.pipes]
    B.tune(2)
    for p, ref in zip(B.pipes, before):
        for f, r in zip(("rho", "u", "b"), ref):
            assert np.array_equal(p.get_field(f), r)
    tiles = [p.tiles for p in B.pipes]
    print("tuned tiles", tiles, flush=True)
    S = make_singles(spec, tiles)
    B.step(2)
    for s in S:
        s.step(2)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"tuned pipe {i}")
    B.close()


def test_batch_replans_after_parameter_change():
    """Changing a box's sweep count between steps rebuilds the launch plan and the graphs."""
    print("case batch replan", flush=True)
    spec = batch_spec()
    B = make_batch(spec)
    S = make_singles(spec, [p.tiles for p in B.pipes])
    B.step(2)
    for s in S:
        s.step(2)
    for sim in (B.pipes[1], S[1]):
        sim.set_params(spec[1][0].params, n_mag=9)
    B.step(2)
    for s in S:
        s.step(2)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"replanned pipe {i}")
    B.close()


def test_batch_member_rules():
    from paper_2211_09370_amd import MhdError, mhd_destroy, mhd_step, mhd_tune

    spec = batch_spec()[:2]
    B = make_batch(spec)
    for call in (lambda h: mhd_step(h, 1), mhd_destroy, lambda h: mhd_tune(h, 1)):
        with pytest.raises(MhdError) as e:
            call(B.pipes[0]._h)
        assert e.value.status == -5
    B.close()


def test_batch_d3q27_matches_single_boxes_bitwise():
    print("case batch d3q27", flush=True)
    spec = batch_spec()[:3]
    for w, _ in spec:
        w.params.lattice = 27
    B = make_batch(spec)
    S = make_singles(spec, [p.tiles for p in B.pipes])
    B.step(2)
    for s in S:
        s.step(2)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"d3q27 pipe {i}")
    compare(B.pipes[0], oracle_run(spec[0][0], 2), label="batch d3q27 pipe 0")
    B.close()


def test_batch_mixes_fluid_branches_bitwise():
    """Plain, rescaled (gamma) and macroscopic (tau >= 1) boxes advanced by the same launches."""
    print("case batch fluid branches", flush=True)
    spec = batch_spec()[:4]
    spec[0][0].params.gamma = 2.5
    spec[1][0].params.nu = 0.3
    spec[2][0].params.nu = 1.0 / 6.0
    B = make_batch(spec)
    S = make_singles(spec, [p.tiles for p in B.pipes])
    B.step(3)
    for s in S:
        s.step(3)
    for i, (p, s) in enumerate(zip(B.pipes, S)):
        assert_same(p, s, f"branch pipe {i}")
    for i in (0, 1):
        compare(B.pipes[i], oracle_run(spec[i][0], 3, markers=spec[i][1]), label=f"batch branch pipe {i}")
    B.close()


def test_blow_up_in_one_pipe_is_reported_for_that_pipe_only():
    from paper_2211_09370_amd import _abi

    spec = batch_spec()[:2]
    B = make_batch(spec)
    u = spec[1][0].u.copy()
    u[0, 5, 6, 7] = 0.9
    B.pipes[1].set_field("u", u)
    B.step(1)
    B.pipes[0].get_field("u")
    assert B.pipes[0].last_status == _abi.MHD_OK
    B.pipes[1].get_field("u")
    assert B.pipes[1].last_status == _abi.MHD_ERR_UNSTABLE
    B.close()
