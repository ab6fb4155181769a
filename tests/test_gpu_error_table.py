"""Error of the FP32-mixed path against the FP64 oracle, stated per field
and per particle moment, on the 1024^2 current-sheet magnetosphere (the
precision form of the 1024^2 hybrid workload: same seed, shapes and
physics, 2e5 macro-particles in place of 2e7, each of 100 times the weight,
so that the oracle finishes; the plain FP64 GPU path is measured beside it).

By default the comparison runs 100 steps and holds the FP32 path to 2e-5
there.  With FFPIC_ERROR_TABLE_STEPS=1000 it also reports step 1000, and
FFPIC_ERROR_TABLE_OUT=path writes the table (JSON).  The oracle runs on the
host's threads (its OpenMP build, deterministic; it differs from the
single-thread build only in the order of the deposit's additions, at the
1e-15 level).

Measures, for every field component F_c of a field F (E or B):
* rel: relative L2 over all nodes, |dF_c| / |F_c|;
* grp: against the whole field, |dF_c| / |F| (|F|^2 the sum over its three
  components): the reading of "relative error on a field" that the 2e-5
  bound is held to;
* max: element-wise, max |dF_c| / max |F_c|;
* pert: rel and max for the change F_c - F_c(0) since the initial state,
  which the static dipole and corotation background would otherwise hide.
For the moments of each species: live count difference, and the sums of
gamma and of u_r, u_theta, u_phi relative to the sum of gamma.

Why the bound is held on the whole field.  B_phi is made by the poloidal
currents alone, the net of the signed thermal motion of the sheet
particles, and the gyration of those particles turns a rounding of one
step into a growing phase error.  The FP64 path shows the same
amplification at its own rounding: after 100 steps its B_phi error is about
1000 units of FP64 rounding (2e-13), and the FP32 path's is about 1000 units
of FP32 rounding (1.5e-4), so no FP32 push meets 2e-5 on B_phi against
B_phi's own norm on this workload, while against |B| it is 1e-7.

Also here: the 4096^2 field step alone (no particles), FP32-mixed, 100
steps against the oracle, at the size the perturbation form was made for.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2406_14512_amd import ffpic
from paper_2406_14512_amd import workloads as W
from parity_util import rel_grouped

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-5
FIELDS = [(ffpic.ER, oracle.ER, "Er"), (ffpic.ETH, oracle.ETH, "Eth"),
          (ffpic.EPH, oracle.EPH, "Eph"), (ffpic.BR, oracle.BR, "Br"),
          (ffpic.BTH, oracle.BTH, "Bth"), (ffpic.BPH, oracle.BPH, "Bph")]
STEPS = int(os.environ.get("FFPIC_ERROR_TABLE_STEPS", "100"))
CHECKPOINTS = [k for k in (100, 1000) if k <= max(STEPS, 100)]


def _threads():
    try:
        return int(os.environ.get("OMP_NUM_THREADS", "")) or os.cpu_count() or 1
    except ValueError:
        return os.cpu_count() or 1


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffpic.lib()


def _l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def _mx(a, b):
    mb = np.abs(b).max()
    return float(np.abs(a - b).max() / mb) if mb > 0 else float(np.abs(a - b).max())


def _field_table(sim, ora, f0g, f0o):
    out = {}
    got = [(sim.field(g), ora.field(o)) for g, o, _ in FIELDS]
    norm = [np.sqrt(sum(np.sum(b * b) for _, b in got[k:k + 3])) for k in (0, 3)]
    for k, ((_, _, name), (a, b), a0, b0) in enumerate(zip(FIELDS, got, f0g, f0o)):
        out[name] = {"rel": _l2(a, b), "grp": float(np.linalg.norm(a - b) / norm[k // 3]),
                     "max": _mx(a, b),
                     "pert_rel": _l2(a - a0, b - b0), "pert_max": _mx(a - a0, b - b0)}
    return out


def _moment_table(sim, ora, nspec):
    dg = sim.diagnostics(ffpic.DIAG_MOMENTS)
    out = {}
    for s in range(nspec):
        mo = ora.moments(s)
        out[f"species{s}"] = {
            "alive": int(dg["alive"][s]), "alive_oracle": int(mo[0]),
            "gamma": abs(dg["sum_gamma"][s] - mo[1]) / abs(mo[1]),
            "ur": abs(dg["sum_u"][s][0] - mo[2]) / abs(mo[1]),
            "uth": abs(dg["sum_u"][s][1] - mo[3]) / abs(mo[1]),
            "uph": abs(dg["sum_u"][s][2] - mo[4]) / abs(mo[1])}
    return out


def _run_tables():
    """Both GPU precisions and the oracle from the same state, stepped to
    every checkpoint together."""
    w = W.sheet_1024(n_total=200_000, steps=max(CHECKPOINTS))
    d = w.desc()
    ora = oracle.Oracle(d, threads=_threads())
    f0o = [ora.field(o) for _, o, _ in FIELDS]
    sims, f0g = {}, {}
    for name, prec in (("fp32_mixed", W.FP32_MIXED), ("fp64", W.FP64)):
        dp = dict(d, precision=prec)
        sims[name] = ffpic.Sim(dp, capacity=[w.n_per_species] * 2)
        f0g[name] = [sims[name].field(g) for g, _, _ in FIELDS]
    for s in range(2):
        p = w.particles(s)
        ora.load(s, p)
        for sim in sims.values():
            sim.load_particles(s, p)
    rows = {name: {} for name in sims}
    done = 0
    for k in CHECKPOINTS:
        ora.step(k - done)
        for name, sim in sims.items():
            sim.step(k - done)
            sim.sync()
            rows[name][k] = {"fields": _field_table(sim, ora, f0g[name], f0o),
                             "moments": _moment_table(sim, ora, 2)}
        done = k
        print(f"step {k} compared", flush=True)
    for sim in sims.values():
        sim.close()
    ora.close()
    return rows


@pytest.mark.timeout(1800)
def test_error_table_fp32_mixed_and_fp64_1024():
    table = {"workload": "sheet_1024: 1024x1024, r in [1, 30], R_LC = 5, 2e5 e+- in a sech^2 "
                         "sheet of width 0.05 (2e7 in the full workload), radiation reaction on, "
                         "sort every 8 steps"}
    table.update(_run_tables())
    print(json.dumps(table, indent=1))
    out = os.environ.get("FFPIC_ERROR_TABLE_OUT")
    if out:
        with open(out, "w") as fh:
            json.dump(table, fh, indent=1)
    t100 = table["fp32_mixed"][100]
    for name, e in t100["fields"].items():
        assert e["grp"] < FP32_TOL, (name, e)
    for s, m in t100["moments"].items():
        assert abs(m["alive"] - m["alive_oracle"]) <= 2e-5 * m["alive_oracle"] + 2, (s, m)
        for k in ("gamma", "ur", "uth", "uph"):
            assert m[k] < FP32_TOL, (s, k, m)
    f100 = table["fp64"][100]
    for name, e in f100["fields"].items():
        assert e["rel"] < FP64_TOL, (name, e)
    for s, m in f100["moments"].items():
        assert m["alive"] == m["alive_oracle"], (s, m)
        for k in ("gamma", "ur", "uth", "uph"):
            assert m[k] < FP64_TOL, (s, k, m)


@pytest.mark.timeout(900)
def test_field_step_alone_fp32_4096_100_steps():
    """The 4096^2 grid (the size the FP32 perturbation form was built for)
    with no particles: the FP32-mixed field step against the FP64 oracle
    over 100 steps, per component against the norm and the largest entry
    of its field group (E or B): without particles E_phi and B_phi stay
    tiny next to the corotation and dipole fields."""
    w = W.sheet_4096(n_total=2, steps=100)
    d = w.desc()
    d["precision"] = W.FP32_MIXED
    sim = ffpic.Sim(d, capacity=[1, 1])
    ora = oracle.Oracle(d, threads=_threads())
    sim.step(100)
    sim.sync()
    ora.step(100)
    errs = {}
    for group in (FIELDS[:3], FIELDS[3:]):
        errs.update(rel_grouped([(n, sim.field(g), ora.field(o)) for g, o, n in group]))
    print("4096^2 FP32-mixed field step, 100 steps, group-relative errors:", errs)
    assert max(errs.values()) < FP32_TOL, errs
    # the force-free / PIC mask follows the same Psi
    fg, fo = sim.field(ffpic.F), ora.field(oracle.F)
    assert np.mean(fg != fo) < 1e-4
