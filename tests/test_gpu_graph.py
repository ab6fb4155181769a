"""Graph-captured sort cycles of ffpic_step against the same steps launched
one by one.

A context with graphs on runs every whole sort cycle of a step call as a
HIP graph, captured once per host state and replayed afterwards.  The twin
context runs the same steps with graphs off.  Both start from the same
state, so they differ only in the order of the deposit's floating-point
atomic additions: FP64 to 1e-12 relative (fields, particle state), cells and
live counts exactly; FP32-mixed to 2e-5.  The graphs are replayed several
times with synchronising work (diagnostics, particle reads) between the
replays, and every replay is checked.
"""
import numpy as np
import pytest

from paper_2406_14512_amd import ffpic
from paper_2406_14512_amd import workloads as W
from parity_util import rel

pytestmark = pytest.mark.gpu

FIELDS = [ffpic.ER, ffpic.ETH, ffpic.EPH, ffpic.BR, ffpic.BTH, ffpic.BPH]


def twins(w, precision):
    d = w.desc()
    d["precision"] = precision
    out = []
    for graph in (True, False):
        sim = ffpic.Sim(d, capacity=[w.n_per_species] * w.nspec)
        sim.set_graph(graph)
        for s in range(w.nspec):
            sim.load_particles(s, w.particles(s))
        out.append(sim)
    return out


def compare(g, e, tol, nspec):
    for c in FIELDS:
        assert rel(g.field(c), e.field(c)) < tol, c
    for s in range(nspec):
        pg, pe = g.particles(s), e.particles(s)
        assert len(pg["cell"]) == len(pe["cell"])
        assert np.mean(pg["cell"] != pe["cell"]) < 1e-4
        for k in ("ur", "uth", "uph"):
            assert rel(pg[k], pe[k]) < tol, (s, k)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_graph_cycles_match_eager_steps(precision):
    w = W.sheet_1024(n_total=100_000, steps=40)
    w.nr = w.nth = 256
    g, e = twins(w, precision)
    tol = 1e-12 if precision == W.FP64 else 2e-5
    si = int(w.sort_interval)
    for rnd in range(4):
        g.step(si)
        e.step(si)
        g.sync()
        e.sync()
        dg, de = g.diagnostics(ffpic.DIAG_MOMENTS), e.diagnostics(ffpic.DIAG_MOMENTS)
        assert dg["alive"] == de["alive"], rnd
        assert dg["step"] == de["step"] == (rnd + 1) * si
        compare(g, e, tol, w.nspec)
    builds, launches = g.graph_stats()
    assert launches == 4 and 1 <= builds <= 2, (builds, launches)
    assert e.graph_stats() == (0, 0)
    # a step call that is not a whole cycle runs its steps one by one, and
    # the graphs resume afterwards
    g.step(3)
    e.step(3)
    g.step(si - 3 + si)
    e.step(si - 3 + si)
    g.sync()
    e.sync()
    compare(g, e, tol, w.nspec)
    assert g.graph_stats()[1] == launches + 1
    # a setting the launches depend on makes a new graph
    g.set_field_rows(7)
    e.set_field_rows(7)
    g.step(si)
    e.step(si)
    g.sync()
    e.sync()
    compare(g, e, tol, w.nspec)
    assert g.graph_stats()[0] > builds
    g.close()
    e.close()


def test_graph_off_for_per_step_arguments():
    """Surface injection keys its random draws by the step: those cycles are
    launched step by step, and match the oracle-checked eager path."""
    w = W.hybrid_monopole(64)
    d = w.desc()
    sim = ffpic.Sim(d, capacity=[200_000] * w.nspec)
    sim.step(16)
    sim.sync()
    assert sim.graph_stats() == (0, 0)
    sim.close()
