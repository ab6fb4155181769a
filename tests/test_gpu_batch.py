"""Batched magnetospheres and the sort-interval autotuner, through the C ABI.

* A batch step of several independent systems gives what each system gives
  when stepped alone (FP64: 1e-12 relative; FP32-mixed: 1e-5, since only
  the order of the FP32 atomic additions in the deposit differs), and the
  FP64 systems match the oracle.
* Views work as ordinary contexts and are not freed by ffpic_destroy.
* Autotuning leaves the state bit-for-bit as it was, picks one of the timed
  intervals, and a run with the tuned interval still matches the oracle
  (the interval only reorders particles).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2406_14512_amd import ffpic
from paper_2406_14512_amd import workloads as W
from parity_util import rel, rel_grouped  # noqa: F401

pytestmark = pytest.mark.gpu

FIELDS = [(ffpic.ER, oracle.ER), (ffpic.ETH, oracle.ETH), (ffpic.EPH, oracle.EPH),
          (ffpic.BR, oracle.BR), (ffpic.BTH, oracle.BTH), (ffpic.BPH, oracle.BPH)]


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffpic.lib()


def systems():
    a = W.tiny_open_dipole(20000)
    b = W.tiny_dipole(15000)
    b.nr, b.nth = 96, 80
    c = W.sheet_1024(n_total=60000, precision=W.FP32_MIXED)
    c.nr = c.nth = 192
    return [a, b, c]


def descs(ws):
    out = []
    for w in ws:
        d = w.desc()
        d["precision"] = w.precision
        out.append(d)
    return out


@pytest.mark.parametrize("graph", [True, False])
def test_batch_cycles_as_graphs_match_single_contexts(graph):
    """Whole sort cycles of the batch as one graph (every system's launches
    on its own branch), replayed from the state it was captured in, against
    each system stepped alone one step at a time; between the replays the
    views are read (synchronising work), and every replay is checked."""
    ws = systems()
    for w in ws:
        w.sort_interval = 4
    ds = descs(ws)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    batch.set_graph(graph)
    singles = [ffpic.Sim(d, capacity=c) for d, c in zip(ds, caps)]
    for w, v, s in zip(ws, batch.views, singles):
        s.set_graph(False)
        for sp in range(w.nspec):
            p = w.particles(sp)
            v.load_particles(sp, p)
            s.load_particles(sp, p)
    for rnd in range(4):
        batch.step(4)
        batch.sync()
        for s in singles:
            s.step(4)
        for w, d, v, s in zip(ws, ds, batch.views, singles):
            tol = 1e-12 if d["precision"] == W.FP64 else 1e-5
            for g, _ in FIELDS:
                assert rel(v.field(g), s.field(g)) < tol, (rnd, w.name, g)
            dv, ds_ = v.diagnostics(ffpic.DIAG_MOMENTS), s.diagnostics(ffpic.DIAG_MOMENTS)
            assert dv["alive"] == ds_["alive"], (rnd, w.name)
            assert dv["step"] == ds_["step"] == 4 * (rnd + 1)
    builds, launches = batch.graph_stats()
    if graph:
        assert launches == 4 and 1 <= builds <= 2, (builds, launches)
    else:
        assert (builds, launches) == (0, 0)
    # FP64 systems: grouped launches are not used, the graphs hold every
    # system's own launches
    assert batch.grouped_launches() == 0
    batch.close()
    for s in singles:
        s.close()


def test_grouped_batch_graph_matches_single_contexts():
    """Mode 2 (the default for FP32-mixed batches without plasma sources):
    per step, one persistent launch each for the flux functions, masks,
    pushes and field steps of all systems.  Three systems of different grids
    and sort intervals (2 and 4, so that some steps sort only some systems
    and the push launches mix placing and plain pushes), a non-default
    slab height on one of them and the transverse-momentum shell on another
    (its pushes are a kernel instance of their own), against each system
    stepped alone one step at a time; every replay checked, with reads
    between the replays."""
    ws = [W.tiny_open_dipole(20000), W.tiny_dipole(15000),
          W.sheet_1024(n_total=60000, precision=W.FP32_MIXED)]
    ws[1].nr, ws[1].nth = 96, 80
    ws[2].nr = ws[2].nth = 192
    ws[1].shell_r = 4.0
    ds = []
    for w, si in zip(ws, (2, 4, 4)):
        w.sort_interval = si
        d = w.desc()
        d["precision"] = W.FP32_MIXED
        ds.append(d)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    singles = [ffpic.Sim(d, capacity=c) for d, c in zip(ds, caps)]
    for w, v, s in zip(ws, batch.views, singles):
        s.set_graph(False)
        for sp in range(w.nspec):
            p = w.particles(sp)
            v.load_particles(sp, p)
            s.load_particles(sp, p)
    batch.views[2].set_field_rows(7)
    singles[2].set_field_rows(7)
    for rnd in range(5):
        batch.step(4)
        batch.sync()
        for s in singles:
            s.step(4)
        for w, v, s in zip(ws, batch.views, singles):
            for g, _ in FIELDS:
                assert rel(v.field(g), s.field(g)) < 1e-5, (rnd, w.name, g)
            dv, ds_ = v.diagnostics(ffpic.DIAG_MOMENTS), s.diagnostics(ffpic.DIAG_MOMENTS)
            assert dv["alive"] == ds_["alive"], (rnd, w.name)
            assert dv["step"] == ds_["step"] == 4 * (rnd + 1)
            for sp in range(w.nspec):
                pv, ps = v.particles(sp), s.particles(sp)
                assert len(pv["cell"]) == len(ps["cell"])
                assert np.mean(pv["cell"] != ps["cell"]) < 1e-3, (rnd, w.name, sp)
                for k in ("ur", "uth", "uph"):
                    assert rel(pv[k], ps[k]) < 2e-5, (rnd, w.name, sp, k)
    builds, launches = batch.graph_stats()
    assert launches == 5 and 1 <= builds <= 2, (builds, launches)
    assert batch.grouped_launches() == 5
    # mode 1 on the same batch: graphs of every system's own launches
    batch.set_graph(1)
    batch.step(4)
    batch.sync()
    for s in singles:
        s.step(4)
    for w, v, s in zip(ws, batch.views, singles):
        for g, _ in FIELDS:
            assert rel(v.field(g), s.field(g)) < 1e-5, (w.name, g)
    assert batch.grouped_launches() == 5 and batch.graph_stats()[1] == 6
    with pytest.raises(ffpic.FfpicError):
        batch.set_graph(3)
    batch.close()
    for s in singles:
        s.close()


def test_batch_matches_single_contexts_and_oracle():
    ws = systems()
    ds = descs(ws)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    assert len(batch) == 3
    singles = [ffpic.Sim(d, capacity=c) for d, c in zip(ds, caps)]
    for w, v, s in zip(ws, batch.views, singles):
        for sp in range(w.nspec):
            p = w.particles(sp)
            v.load_particles(sp, p)
            s.load_particles(sp, p)
    batch.step(4)
    batch.step(2)
    batch.sync()
    for s in singles:
        s.step(6)
    for w, d, v, s in zip(ws, ds, batch.views, singles):
        tol = 1e-12 if d["precision"] == W.FP64 else 1e-5
        for g, _ in FIELDS:
            assert rel(v.field(g), s.field(g)) < tol, (w.name, g)
        dv, ds_ = v.diagnostics(ffpic.DIAG_MOMENTS), s.diagnostics(ffpic.DIAG_MOMENTS)
        assert dv["alive"] == ds_["alive"]
        assert dv["step"] == ds_["step"] == 6
    # the FP64 systems against the oracle
    for w, d, v in zip(ws, ds, batch.views):
        if d["precision"] != W.FP64:
            continue
        ora = oracle.Oracle(d)
        for sp in range(w.nspec):
            ora.load(sp, w.particles(sp))
        ora.step(6)
        for g, o in FIELDS:
            assert rel(v.field(g), ora.field(o)) < 1e-12, (w.name, g)
    # a view survives ffpic_destroy and close()
    ffpic.lib().ffpic_destroy(batch.views[0]._h)
    assert batch.views[0].n(0) > 0
    for s in singles:
        s.close()
    batch.close()


def snapshot(sim, nspec):
    f = [sim.field(g) for g, _ in FIELDS]
    p = [sim.particles(s) for s in range(nspec)]
    return f, p


def test_autotune_keeps_state_and_semantics(tmp_path, monkeypatch):
    cache = tmp_path / "tuning.txt"
    monkeypatch.setenv("FFPIC_TUNING_CACHE", str(cache))
    w = W.tiny_open_dipole(20000)
    d = w.desc()
    d["precision"] = W.FP64
    d["sort_interval"] = 8
    sim = ffpic.Sim(d, capacity=[w.n_per_species] * w.nspec)
    for sp in range(w.nspec):
        sim.load_particles(sp, w.particles(sp))
    sim.step(3)
    before = snapshot(sim, w.nspec)
    t = sim.autotune(3000.0)
    after = snapshot(sim, w.nspec)
    for a, b in zip(before[0], after[0]):
        assert np.array_equal(a, b)
    for pa, pb in zip(before[1], after[1]):
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k
    assert t["sort_interval"] in t["ms_per_step"]
    assert 8 in t["ms_per_step"] and len(t["ms_per_step"]) >= 1
    assert all(v > 0 for v in t["ms_per_step"].values())
    # the slab rows were tuned after the interval (FP64: no push chunk)
    assert 0 in t["timed"]["field_rows"] and t["field_rows"] in t["timed"]["field_rows"]
    assert t["push_ppt"] == 0 and not t["timed"]["push_ppt"]
    line = cache.read_text().split()
    assert line[:4] == [str(w.nr), str(w.nth), "0", str(w.nspec)]
    assert int(line[5]) == t["sort_interval"] and int(line[6]) == t["field_rows"]
    # stepping on with the tuned interval matches the oracle (which sorts
    # every step): the interval only reorders particles
    sim.step(4)
    ora = oracle.Oracle(d)
    for sp in range(w.nspec):
        ora.load(sp, w.particles(sp))
    ora.step(7)
    for g, o in FIELDS:
        assert rel(sim.field(g), ora.field(o)) < 1e-12, g
    # a descriptor asking for the tuned interval is accepted
    d0 = dict(d, sort_interval=0)
    s0 = ffpic.Sim(d0, capacity=[w.n_per_species] * w.nspec)
    for sp in range(w.nspec):
        s0.load_particles(sp, w.particles(sp))
    s0.step(7)
    for g, o in FIELDS:
        assert rel(s0.field(g), ora.field(o)) < 1e-12, g
    s0.close()
    sim.close()
    with pytest.raises(ffpic.FfpicError):
        ffpic.Sim(d, capacity=[10, 10]).autotune(0.0)


def test_autotune_fp32_tunes_the_push_chunk():
    """FP32-mixed: all three parameters are timed, the state is unchanged,
    and stepping on with the chosen chunk and slab height matches a context
    that keeps the defaults (only the order of atomic additions differs)."""
    w = W.sheet_1024(n_total=60000, precision=W.FP32_MIXED)
    w.nr = w.nth = 192
    d = w.desc()
    d["precision"] = W.FP32_MIXED
    sims = [ffpic.Sim(d, capacity=[w.n_per_species] * w.nspec) for _ in range(2)]
    for sim in sims:
        for sp in range(w.nspec):
            sim.load_particles(sp, w.particles(sp))
        sim.step(3)
    before = snapshot(sims[0], w.nspec)
    t = sims[0].autotune(5000.0)
    after = snapshot(sims[0], w.nspec)
    for a, b in zip(before[0], after[0]):
        assert np.array_equal(a, b)
    assert t["push_ppt"] in (8, 16, 32) and 16 in t["timed"]["push_ppt"]
    assert t["field_rows"] in t["timed"]["field_rows"]
    # both on the tuned interval, one with the defaults for the rest
    sims[1]._chk(ffpic.lib().ffpic_set_field_rows(sims[1]._h, 0))
    for sim in sims:
        sim.step(8)
    for g, _ in FIELDS:
        assert rel(sims[0].field(g), sims[1].field(g)) < 1e-5, g
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("ppt", [8, 32])
def test_push_chunk_setting_single_context(ppt):
    """ffpic_set_push_chunk: a chunk of 8 or 32 particles per thread gives
    what the default 16 gives, over sort cycles whose pushes place the
    sorted order (only the order of the deposit's atomic additions
    differs)."""
    w = W.sheet_1024(n_total=60000, precision=W.FP32_MIXED)
    w.nr = w.nth = 192
    w.sort_interval = 4
    d = w.desc()
    d["precision"] = W.FP32_MIXED
    sims = [ffpic.Sim(d, capacity=[w.n_per_species] * w.nspec) for _ in range(2)]
    for sim in sims:
        for sp in range(w.nspec):
            sim.load_particles(sp, w.particles(sp))
    sims[0].set_push_chunk(ppt)
    with pytest.raises(ffpic.FfpicError):
        sims[1].set_push_chunk(12)
    for rnd in range(4):
        for sim in sims:
            sim.step(4)
            sim.sync()
        for g, _ in FIELDS:
            assert rel(sims[0].field(g), sims[1].field(g)) < 1e-5, (rnd, g)
        a, b = (s.diagnostics(ffpic.DIAG_MOMENTS) for s in sims)
        assert a["alive"] == b["alive"], rnd
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("ppt,gppt", [(8, 0), (32, 0), (8, 16), (16, 32)])
def test_grouped_batch_push_chunk(ppt, gppt):
    """Grouped batch launches with every system's push chunk set to 8, 16 or
    32 particles per thread, and with the batch's grouped chunk overriding
    it (gppt > 0), against the same systems stepped alone with their own
    chunk."""
    ws = [W.sheet_1024(n_total=60000, precision=W.FP32_MIXED) for _ in range(2)]
    ws[0].nr = ws[0].nth = 192
    ws[1].nr, ws[1].nth = 128, 160
    ds = []
    for w in ws:
        w.sort_interval = 4
        d = w.desc()
        d["precision"] = W.FP32_MIXED
        ds.append(d)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    singles = [ffpic.Sim(d, capacity=c) for d, c in zip(ds, caps)]
    for w, v, s in zip(ws, batch.views, singles):
        s.set_graph(False)
        v.set_push_chunk(ppt)
        s.set_push_chunk(ppt)
        for sp in range(w.nspec):
            p = w.particles(sp)
            v.load_particles(sp, p)
            s.load_particles(sp, p)
    batch.set_grouped_chunk(gppt)
    assert batch.graph_settings()[:2] == (2, gppt)
    with pytest.raises(ffpic.FfpicError):
        batch.set_grouped_chunk(12)
    for rnd in range(4):
        batch.step(4)
        batch.sync()
        for s in singles:
            s.step(4)
        for w, v, s in zip(ws, batch.views, singles):
            for g, _ in FIELDS:
                assert rel(v.field(g), s.field(g)) < 1e-5, (rnd, g)
            assert v.diagnostics(ffpic.DIAG_MOMENTS)["alive"] == \
                s.diagnostics(ffpic.DIAG_MOMENTS)["alive"]
    assert batch.grouped_launches() == 4
    batch.close()
    for s in singles:
        s.close()


def test_grouped_batch_more_jobs_than_threads():
    """A grouped push launch with more jobs than a workgroup has threads
    (132 two-species systems: 264 jobs of one kernel instance), so that the
    workgroup's threads need two rounds to find an item's job; systems on
    both sides of job 256 against the same systems stepped alone."""
    n = 132
    ws = []
    for k in range(n):
        w = W.tiny_open_dipole(1500)
        w.nr = w.nth = 32
        w.seed += k
        w.sort_interval = 4
        ws.append(w)
    ds = []
    for w in ws:
        d = w.desc()
        d["precision"] = W.FP32_MIXED
        ds.append(d)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    pick = (0, 1, 127, 128, 130, 131)
    singles = {k: ffpic.Sim(ds[k], capacity=caps[k]) for k in pick}
    for s in singles.values():
        s.set_graph(False)
    for k, (w, v) in enumerate(zip(ws, batch.views)):
        for sp in range(w.nspec):
            p = w.particles(sp)
            v.load_particles(sp, p)
            if k in singles:
                singles[k].load_particles(sp, p)
    for rnd in range(3):
        batch.step(4)
        batch.sync()
        for s in singles.values():
            s.step(4)
        for k, s in singles.items():
            v = batch.views[k]
            for g, _ in FIELDS:
                assert rel(v.field(g), s.field(g)) < 1e-5, (rnd, k, g)
            assert v.diagnostics(ffpic.DIAG_MOMENTS)["alive"] == \
                s.diagnostics(ffpic.DIAG_MOMENTS)["alive"], (rnd, k)
    assert batch.grouped_launches() == 3
    batch.close()
    for s in singles.values():
        s.close()


def test_batch_autotune_chooses_the_graph_mode():
    """ffpic_batch_autotune on an FP32-mixed batch without plasma sources
    also times whole batch cycles with per-system graphs and with grouped
    launches from one checkpoint of every system, keeps the faster mode, and
    leaves every system's state as it was."""
    ws = [W.sheet_1024(n_total=40000, precision=W.FP32_MIXED) for _ in range(3)]
    for w, n in zip(ws, (96, 128, 160)):
        w.nr = w.nth = n
    ds = []
    for w in ws:
        d = w.desc()
        d["precision"] = W.FP32_MIXED
        ds.append(d)
    caps = [[w.n_per_species] * w.nspec for w in ws]
    batch = ffpic.Batch(ds, caps)
    for w, v in zip(ws, batch.views):
        for sp in range(w.nspec):
            v.load_particles(sp, w.particles(sp))
    batch.step(3)
    batch.sync()
    before = [snapshot(v, w.nspec) for w, v in zip(ws, batch.views)]
    batch.autotune(3000.0)
    mode, gppt, ms = batch.graph_settings()
    assert mode in (1, 2) and set(ms) == {1, 2} and all(v > 0 for v in ms.values())
    assert mode == min(ms, key=ms.get)
    assert gppt in (0, 16) and (mode == 2 or gppt == 0)
    assert batch.get_graph() == (mode, ms)
    for (f0, p0), w, v in zip(before, ws, batch.views):
        f1, p1 = snapshot(v, w.nspec)
        for a, b in zip(f0, f1):
            assert np.array_equal(a, b)
        for pa, pb in zip(p0, p1):
            for k in pa:
                assert np.array_equal(pa[k], pb[k]), k
        assert v.diagnostics(ffpic.DIAG_MOMENTS)["step"] == 3
    batch.step(16)
    batch.sync()
    batch.close()
