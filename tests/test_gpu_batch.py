"""Batched realisations: the batch step (graph replay and direct launches)
against the same mocks stepped one by one, bitwise, after every step.

Uneven sizes as in the ensemble workload (48^3/96^3, 64^3/128^3, 96^3/192^3
particles/mesh; a 32^3/64^3 group too), distinct seeds and boxes.  Between
graph replays the test does eager work of its own (state reads, a density)
and synchronises, so every replay is checked against direct launches.
"""

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1507_05329_amd import _lib  # noqa: E402
from paper_1507_05329_amd.inputs import bbks_table, step_edges  # noqa: E402

SPECS = [
    dict(np=48, nmesh=96, box=150.0, seed=101),
    dict(np=32, nmesh=64, box=100.0, seed=102),
    dict(np=64, nmesh=128, box=200.0, seed=103),
    dict(np=48, nmesh=96, box=180.0, seed=104),
    dict(np=96, nmesh=192, box=300.0, seed=105),
    dict(np=64, nmesh=128, box=220.0, seed=106),
    dict(np=32, nmesh=64, box=120.0, seed=107),
    dict(np=96, nmesh=192, box=260.0, seed=108),
]


def state_of(sim):
    st = sim.get_state()
    return st["disp"], st["vres"], st["a_x"], st["a_v"]


def test_batch_groups_and_views():
    from paper_1507_05329_amd.sim import ColaBatch
    say("[gpu] batch groups")
    b = ColaBatch(SPECS)
    try:
        assert len(b) == len(SPECS)
        assert b.ngroups == 4
        for m, sp in zip(b.mocks, SPECS):
            assert (m.np_side, m.nmesh, m.box) == (sp["np"], sp["nmesh"], sp["box"])
    finally:
        b.close()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_step_bitwise_equals_sequential(graph):
    from paper_1507_05329_amd.sim import ColaBatch, ColaSim
    table = bbks_table()
    e = step_edges()
    say(f"[gpu] batch vs sequential, graph={graph}, {len(SPECS)} mocks")
    b = ColaBatch(SPECS, graph=graph)
    seq = [ColaSim(sp["np"], sp["nmesh"], sp["box"]) for sp in SPECS]
    try:
        for m, s, sp in zip(b.mocks, seq, SPECS):
            m.init_2lpt(sp["seed"], *table)
            s.init_2lpt(sp["seed"], *table)
        for i in range(len(e) - 1):
            b.step(e[i], e[i + 1])
            for s in seq:
                s.step(e[i], e[i + 1])
            torch.cuda.synchronize()
            for j, (m, s) in enumerate(zip(b.mocks, seq)):
                dm, vm, axm, avm = state_of(m)
                ds, vs, axs, avs = state_of(s)
                assert axm == axs and avm == avs
                assert torch.equal(dm, ds), f"step {i} mock {j}: displacement differs"
                assert torch.equal(vm, vs), f"step {i} mock {j}: velocity differs"
            # eager work of the program between replays
            rho = b.mocks[i % len(SPECS)].density()
            assert torch.isfinite(rho).all()
            torch.cuda.synchronize()
            say(f"[gpu]   step {i} bitwise equal")
        # outputs through the mock views agree too
        for m, s in zip(b.mocks, seq):
            assert torch.equal(m.density(), s.density())
    finally:
        for s in seq:
            s.close()
        b.close()


def test_batch_graph_and_direct_launches_agree_and_rerun():
    """Two batches on one set of seeds: graph replays vs direct launches, then a
    second initial condition on the same batch replays the same graph again."""
    from paper_1507_05329_amd.sim import ColaBatch
    table = bbks_table()
    e = step_edges()
    say("[gpu] graph vs direct launches")
    g = ColaBatch(SPECS, graph=True)
    d = ColaBatch(SPECS, graph=False)
    try:
        for rep in range(2):
            for bb in (g, d):
                for m, sp in zip(bb.mocks, SPECS):
                    m.init_2lpt(sp["seed"] + 1000 * rep, *table)
                bb.run(e)
            torch.cuda.synchronize()
            for mg, md in zip(g.mocks, d.mocks):
                assert torch.equal(state_of(mg)[0], state_of(md)[0])
            say(f"[gpu]   repetition {rep} equal")
    finally:
        g.close()
        d.close()


def test_batch_step_rejects_mismatched_time():
    from paper_1507_05329_amd.sim import ColaBatch
    table = bbks_table()
    e = step_edges()
    say("[gpu] batch state checks")
    b = ColaBatch(SPECS[:2])
    try:
        with pytest.raises(_lib.ColaError) as ei:
            b.step(e[0], e[1])            # no initial conditions yet
        assert ei.value.code == _lib.COLA_ESTATE
        for m, sp in zip(b.mocks, SPECS[:2]):
            m.init_2lpt(sp["seed"], *table)
        b.mocks[0].step(e[0], e[1])       # one mock ahead of the other
        with pytest.raises(_lib.ColaError) as ei:
            b.step(e[0], e[1])
        assert ei.value.code == _lib.COLA_ESTATE
        b.mocks[1].step(e[0], e[1])
        b.step(e[1], e[2])
        torch.cuda.synchronize()
    finally:
        b.close()
