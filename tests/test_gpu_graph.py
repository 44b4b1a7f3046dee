"""Graph replay of single-box steps (on a caller stream) against direct launches on the same
inputs: the same fields and budget records bit for bit, across a parameter change, a tile
change and an odd sweep count (the buffer state then alternates between two captured graphs),
in float32 and in the split form."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _sim(w, stream, graph, store):
    from paper_2211_09370_amd import Sim

    s = Sim(w.nx, w.ny, w.nz, w.markers.shape[1], stream=stream, **store)
    s.set_markers(w.markers)
    s.set_params(w.params, n_mag=6)
    s.set_field("rho", w.rho)
    s.set_field("u", w.u)
    s.set_field("b", w.b)
    s.set_graph(graph)
    return s


def _same(a, b, label):
    for f in ("rho", "u", "b"):
        x, y = a.get_field(f), b.get_field(f)
        assert np.isfinite(x).all(), (label, f)
        assert np.array_equal(x, y), (label, f, float(np.abs(x - y).max()))


@pytest.mark.parametrize("store", [{}, dict(b_storage="f16split", u_scale=0.05, b_scale=0.01)],
                         ids=["f32", "split"])
def test_graph_replay_equals_direct_launches(store):
    import torch

    w = W.pipe_workload("graph", 13, 128, 30, 28, 10.0, 50.0, 10.0, 1e-2, bext_kind=W.BEXT_TANH_FRINGE_Y,
                        fringe_x0=64.0, fringe_w=4.0, noise=1e-2, rho_amp=1e-3, b_amp=1e-3)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g, d = _sim(w, st, True, store), _sim(w, st, False, store)
        for s in (g, d):
            s.step(3, 2)
        _same(g, d, "3 steps")
        rg, rd = g.budgets(), d.budgets()
        assert len(rg) == len(rd) == 1 and rg[0] == rd[0]
        for s in (g, d):  # new parameters: captured steps are dropped and taken again
            s.set_params(w.params, n_mag=5, G0=2 * w.params.G0)
            s.step(4)
        _same(g, d, "odd sweep count")
        for s in (g, d):
            s.tiles = (32, 4, 0, 4)
            s.step(2)
        _same(g, d, "new tiles")
        for s in (g, d):
            s.set_time(100, 0.0)
            s.step(1, 1)
        _same(g, d, "after set_time")
        assert g.budgets()[-1]["step"] == d.budgets()[-1]["step"] == 101
        g.close()
        d.close()


def test_two_solvers_on_two_streams_step_independently():
    """Two boxes, each on a stream of its own, stepped in interleaved calls (each replaying its
    own graphs, with profiling switched on and off in between for one of them) end where each
    ends when stepped alone."""
    import torch

    w = W.pipe_workload("graph", 13, 128, 30, 28, 10.0, 50.0, 10.0, 1e-2, bext_kind=W.BEXT_TANH_FRINGE_Y,
                        fringe_x0=64.0, fringe_w=4.0, noise=1e-2, rho_amp=1e-3, b_amp=1e-3)
    w2 = W.small_pipe(noise=1e-2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a, b = _sim(w, s1, True, {}), _sim(w2, s2, True, {})
    for k in range(4):
        a.step(1)
        b.step(1)
        if k == 1:
            a.set_profiling(True)
        if k == 2:
            a.set_profiling(False)
    ra, rb = _sim(w, s1, False, {}), _sim(w2, s2, False, {})
    ra.step(4)
    rb.step(4)
    _same(a, ra, "interleaved box 1")
    _same(b, rb, "interleaved box 2")
    for s in (a, b, ra, rb):
        s.close()
