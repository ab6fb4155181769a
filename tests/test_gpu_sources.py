"""GPU parity of the plasma sources of the dipole (Sect. 5) and the pieces
of the push they change, against the FP64 CPU oracle on the same inputs:
the radiation-reaction ramp, the transverse-momentum shell,
Goldreich-Julian extraction and threshold pair creation.

Bars: cells and counts exact; FP64 particle state to 1e-14 relative and
fields to 1e-12 (L2 per component); FP32-mixed to FP32 rounding for the
placed particles and 2e-5 for fields, normalised by the field group.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2406_14512_amd import ffpic
from paper_2406_14512_amd import workloads as W
from parity_util import rel, rel_grouped  # noqa: F401

pytestmark = pytest.mark.gpu

FIELDS = [(ffpic.ER, oracle.ER, "Er"), (ffpic.ETH, oracle.ETH, "Eth"), (ffpic.EPH, oracle.EPH, "Eph"),
          (ffpic.BR, oracle.BR, "Br"), (ffpic.BTH, oracle.BTH, "Bth"), (ffpic.BPH, oracle.BPH, "Bph")]
FP64_TOL = 1e-12
FP32_TOL = 2e-5
KEYS = ("r", "th", "ur", "uth", "uph")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffpic.lib()


def both(d, precision, cap):
    d = dict(d, precision=precision)
    return ffpic.Sim(d, capacity=[cap] * d["nspec"]), oracle.Oracle(d)


def field_errors(sim, ora):
    return {name: rel(sim.field(g), ora.field(o)) for g, o, name in FIELDS}


def field_errors_grouped(sim, ora):
    """Per-component errors normalised by the field group (E or B)
    rather than by the component itself."""
    return {**rel_grouped([(n, sim.field(g), ora.field(o)) for g, o, n in FIELDS[:3]]),
            **rel_grouped([(n, sim.field(g), ora.field(o)) for g, o, n in FIELDS[3:]])}

def same_particles(sim, ora, nspec, rtol):
    for s in range(nspec):
        g, o = sim.particles(s), ora.particles(s)
        assert len(g["cell"]) == len(o["cell"]), (s, len(g["cell"]), len(o["cell"]))
        assert np.array_equal(g["cell"], o["cell"]), s
        live = o["cell"] >= 0
        for k in KEYS:
            assert np.allclose(g[k][live], o[k][live], rtol=rtol, atol=rtol), (s, k)


def test_shell_push_fp64():
    """Monopole field, E = 0, particles gyrating across B inside the shell
    and free ones outside: one push agrees with the oracle, and inside the
    shell nothing is left of the momentum."""
    d = dict(nr=32, nth=32, rmin=1.0, rmax=10.0, r_lc=3.0, r_abs=9.0, mu=1.0, cfl=0.5,
             omega_b=50.0, rr_coef=0.0, psi_thr=(-W.INF, -W.INF, W.INF, W.INF), ff_enable=0,
             init=W.INIT_MONOPOLE, sort_interval=1, nspec=1, qm=(-1.0,), weight=(1e-6,),
             shell_r=2.0)
    sim, ora = both(d, W.FP64, 1000)
    zero = np.zeros(((d["nr"] + 1), (d["nth"] + 1)))
    for g, o in ((ffpic.ER, oracle.ER), (ffpic.ETH, oracle.ETH), (ffpic.EPH, oracle.EPH)):
        sim.load_fields(g, zero)
        ora.set_field(o, zero)
    rng = np.random.default_rng(21)
    n = 400
    inner = np.arange(n) < n // 2
    p = dict(r=np.where(inner, rng.uniform(1.2, 1.8, n), rng.uniform(3.0, 5.0, n)),
             th=rng.uniform(0.3, 2.8, n), ur=np.where(inner, 0.0, rng.normal(0, 3, n)),
             uth=rng.normal(0, 3, n), uph=rng.normal(0, 3, n))
    sim.load_particles(0, p)
    ora.load(0, p)
    sim.run_phases(ffpic.PHASE_PUSH)
    ora.phases(oracle.PHASE_PUSH)
    same_particles(sim, ora, 1, 1e-14)
    g = sim.particles(0)
    inside = g["r"] < 2.0
    u = np.sqrt(g["ur"] ** 2 + g["uth"] ** 2 + g["uph"] ** 2)
    assert inside.sum() > 100 and np.all(u[inside] < 1e-13)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_shell_and_ramp_steps(precision):
    """The dipole band with radiation reaction on, a ramp whose knots fall
    within the run (factors 0.25 -> 1 -> 0.5) and a shell out to r = 4: ten
    steps against the oracle."""
    w = W.tiny_dipole(20_000, steps=10)
    w.rr_coef = 40.0
    w.shell_r = 4.0
    dt = oracle.timestep(dict(w.desc()))
    w.rr_ramp = ((2 * dt, 0.25), (5 * dt, 1.0), (8 * dt, 0.5))
    sim, ora = both(w.desc(), precision, w.n_per_species)
    for s in range(2):
        p = w.particles(s)
        sim.load_particles(s, p)
        ora.load(s, p)
    sim.step(10)
    ora.step(10)
    sim.sync()
    if precision == W.FP64:
        errs = field_errors(sim, ora)
        assert max(errs.values()) < FP64_TOL, errs
    else:
        errs = field_errors_grouped(sim, ora)
        assert max(errs.values()) < FP32_TOL, errs
    dg = sim.diagnostics(ffpic.DIAG_MOMENTS)
    for s in range(2):
        mo = ora.moments(s)
        assert abs(dg["sum_gamma"][s] - mo[1]) / mo[1] < (1e-12 if precision == W.FP64 else 2e-5)


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_extraction_matches_oracle(precision):
    """An empty sourced dipole: one extraction places the oracle's electrons
    and protons (same cells; FP64 positions bit for bit, FP32 to rounding);
    a second extraction adds nothing."""
    w = W.sourced_dipole(64, precision=precision, n_per_species=0)
    sim, ora = both(w.desc(), precision, 50_000)
    sim.run_phases(ffpic.PHASE_MASK | ffpic.PHASE_EXTRACT)
    ora.phases(oracle.PHASE_MASK | oracle.PHASE_EXTRACT)
    assert ora.n(0) > 20 and ora.n(1) == 0
    for s in (0, 1, 2):
        g, o = sim.particles(s), ora.particles(s)
        assert np.array_equal(g["cell"], o["cell"]), s
        if precision == W.FP64:
            assert np.array_equal(g["th"], o["th"])
            for k in ("r", "uph"):
                assert np.allclose(g[k], o[k], rtol=1e-15, atol=0), k
        else:
            for k in ("r", "th", "uph"):
                assert np.allclose(g[k], o[k], rtol=2e-7, atol=0), k
    n0 = sim.n(0)
    sim.run_phases(ffpic.PHASE_EXTRACT)
    assert sim.n(0) == n0 and sim.n(2) == n0


def _pair_inputs(w, rng):
    out = []
    for gs in ([1.5, 29.9, 30.0 * (1 + 1e-9), 80.0, 500.0] * 40, [10.0, 45.0, 31.0] * 40,
               [100.0, 1000.0] * 10):
        gs = np.asarray(gs)
        n = len(gs)
        u = np.sqrt(gs ** 2 - 1)
        dirs = rng.normal(size=(n, 3))
        dirs /= np.linalg.norm(dirs, axis=1)[:, None]
        out.append(dict(r=rng.uniform(3, 5, n), th=rng.uniform(0.5, 2.6, n), ur=u * dirs[:, 0],
                        uth=u * dirs[:, 1], uph=u * dirs[:, 2]))
    return out


def test_pairs_match_oracle_fp64():
    """Zero fields, leptons around the threshold: three steps of push + pair
    creation; the created pairs are the oracle's, in the oracle's order."""
    w = W.sourced_dipole(32, n_per_species=0)
    d = dict(w.desc(), gj_extract=0.0, shell_r=0.0, rr_coef=0.0, ff_enable=0)
    sim, ora = both(d, W.FP64, 20_000)
    zero = np.zeros((w.nr + 1, w.nth + 1))
    for g, o, _ in FIELDS:
        sim.load_fields(g, zero)
        ora.set_field(o, zero)
    for s, p in enumerate(_pair_inputs(w, np.random.default_rng(8))):
        sim.load_particles(s, p)
        ora.load(s, p)
    for k in range(3):
        sim.run_phases(ffpic.PHASE_PUSH | ffpic.PHASE_PAIRS)
        ora.phases(oracle.PHASE_PUSH | oracle.PHASE_PAIRS)
    assert ora.n(1) > 300
    same_particles(sim, ora, 3, 1e-14)


def test_pair_capacity_error():
    w = W.sourced_dipole(32, n_per_species=0)
    d = dict(w.desc(), gj_extract=0.0, shell_r=0.0, rr_coef=0.0, ff_enable=0)
    sim, _ = both(d, W.FP32_MIXED, 250)
    zero = np.zeros((w.nr + 1, w.nth + 1))
    for g, _, _ in FIELDS:
        sim.load_fields(g, zero)
    for s, p in enumerate(_pair_inputs(w, np.random.default_rng(8))):
        sim.load_particles(s, p)
    n_before = [sim.n(s) for s in range(2)]
    sim.run_phases(ffpic.PHASE_PUSH | ffpic.PHASE_PAIRS)
    with pytest.raises(ffpic.FfpicError) as e:
        sim.sync()
    assert e.value.code == ffpic.ECAPACITY
    assert [sim.n(s) for s in range(2)] == n_before


def test_sourced_dipole_fp64():
    """The sourced dipole (extraction, pair creation, shell, ramp) over 6
    steps: fields to 1e-12, every species' particles to 1e-14, in order."""
    w = W.sourced_dipole(64, n_per_species=2000)
    sim, ora = both(w.desc(), W.FP64, 40_000)
    for s in range(3):
        p = w.particles(s)
        sim.load_particles(s, p)
        ora.load(s, p)
    for k in range(6):
        sim.step(1)
        ora.step(1)
        errs = field_errors(sim, ora)
        assert max(errs.values()) < FP64_TOL, (k + 1, errs)
    assert ora.n(1) > 2000
    same_particles(sim, ora, 3, 1e-12)


def test_sourced_dipole_fp32():
    w = W.sourced_dipole(64, precision=W.FP32_MIXED, n_per_species=2000)
    sim, ora = both(w.desc(), W.FP32_MIXED, 40_000)
    for s in range(3):
        p = w.particles(s)
        sim.load_particles(s, p)
        ora.load(s, p)
    for k in range(5):
        sim.step(1)
        ora.step(1)
        errs = field_errors_grouped(sim, ora)
        assert max(errs.values()) < FP32_TOL, (k + 1, errs)
    dg = sim.diagnostics(ffpic.DIAG_MOMENTS)
    for s in range(3):
        n_o = ora.moments(s)[0]
        assert abs(dg["alive"][s] - n_o) <= 0.01 * n_o + 2, (s, dg["alive"][s], n_o)


def test_sourced_dipole_checkpoint_resumes_fp64():
    """Save after 3 steps, restore into a fresh context and step 3 more: the
    same particles (counts exact, states to 1e-13) and fields (1e-12) as the
    uninterrupted run, extraction and pair draws included."""
    w = W.sourced_dipole(64, n_per_species=2000)
    d = dict(w.desc(), precision=W.FP64)
    a = ffpic.Sim(d, capacity=[40_000] * 3)
    for s in range(3):
        a.load_particles(s, w.particles(s))
    a.step(3)
    blob = a.save()
    a.step(3)
    b = ffpic.Sim(d, capacity=[40_000] * 3)
    b.restore(blob)
    b.step(3)
    for g, _, name in FIELDS:
        assert rel(b.field(g), a.field(g)) < FP64_TOL, name
    for s in range(3):
        pa, pb = a.particles(s), b.particles(s)
        assert len(pa["cell"]) == len(pb["cell"]) and np.array_equal(pa["cell"], pb["cell"]), s
        for k in KEYS:
            assert np.allclose(pa[k], pb[k], rtol=1e-13, atol=1e-13), (s, k)
    assert b.diagnostics(ffpic.DIAG_MOMENTS)["step"] == 6


def test_source_that_would_overflow_a_step_is_rejected():
    """Weights so small that one extraction would add more than 2^30
    particles are refused at creation (the per-cell counts are int32)."""
    w = W.sourced_dipole(64, n_per_species=0)
    d = dict(w.desc(), precision=W.FP64, weight=(1e-30, 1e-30, 1e-30))
    with pytest.raises(ffpic.FfpicError) as e:
        ffpic.Sim(d, capacity=[1000] * 3)
    assert e.value.code == ffpic.EINVAL
