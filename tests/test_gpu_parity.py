"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU
oracle on the same seeded inputs.

Tolerances: bit-exact for the particle -> cell index, the sort permutation,
the flux function and the initial fields; 1e-12 relative (L2 over nodes, per
component) for the FP64 path; 2e-5 relative for the FP32-mixed path after
100 steps.
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
# steps of the injected monopole held to FP64_TOL before rounding differences grow
EARLY_STEPS = 3


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffpic.lib()


def pair(w, precision=W.FP64, cap=None):
    d = w.desc()
    d["precision"] = precision
    cap = cap if cap is not None else max(w.n_per_species, 1)
    sim = ffpic.Sim(d, capacity=[cap] * d["nspec"])
    ora = oracle.Oracle(d)
    return sim, ora


def load_both(sim, ora, w, limit=None):
    for s in range(w.nspec):
        p = w.particles(s, limit)
        sim.load_particles(s, p)
        ora.load(s, p)


def field_errors(sim, ora, comps=FIELDS):
    return {name: rel(sim.field(g), ora.field(o)) for g, o, name in comps}


def moment_errors(sim, ora, nspec):
    dg = sim.diagnostics(ffpic.DIAG_MOMENTS)
    out = {}
    for s in range(nspec):
        mo = ora.moments(s)
        out[f"n{s}"] = abs(dg["alive"][s] - mo[0])
        out[f"gamma{s}"] = abs(dg["sum_gamma"][s] - mo[1]) / abs(mo[1])
        for k, nm in enumerate(("ur", "uth", "uph")):
            # sum of gamma bounds the sum of |u_k|: error per unit momentum
            out[f"{nm}{s}"] = abs(dg["sum_u"][s][k] - mo[2 + k]) / abs(mo[1])
    return out


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("grid", [(96, 80), (40, 300)])
@pytest.mark.parametrize("init", [W.INIT_DIPOLE, W.INIT_MONOPOLE, W.INIT_MICHEL,
                                  W.INIT_OPEN_DIPOLE])
def test_initial_fields_and_psi_bit_exact_fp64(init, grid):
    w = W.tiny_open_dipole(10)
    w.nr, w.nth = grid
    w.init = init
    sim, ora = pair(w)
    for g, o, name in FIELDS:
        assert np.array_equal(sim.field(g), ora.field(o)), name
    assert np.array_equal(sim.field(ffpic.PSI), ora.field(oracle.PSI))
    assert np.array_equal(sim.field(ffpic.F), ora.field(oracle.F))


# (40, 300): the flux-function scan runs over two column tiles of 256, the
# second ragged (44 columns), and a last group of 9 rows
PSI_GRIDS = [(96, 80), (40, 300)]


@pytest.mark.parametrize("grid", PSI_GRIDS)
def test_psi_bit_exact_fp64_from_the_same_br(grid):
    w = W.tiny_open_dipole(10)
    w.nr, w.nth = grid
    sim, ora = pair(w)
    ora.set_field(oracle.BR, sim.field(ffpic.BR))   # oracle Psi of the same B_r
    assert np.array_equal(sim.field(ffpic.PSI), ora.field(oracle.PSI))
    assert np.array_equal(sim.field(ffpic.F), ora.field(oracle.F))


@pytest.mark.parametrize("grid", PSI_GRIDS)
def test_psi_bit_exact_fp32_from_rounded_br(grid):
    w = W.tiny_open_dipole(10)
    w.nr, w.nth = grid
    sim, ora = pair(w, W.FP32_MIXED)
    br32 = sim.field(ffpic.BR)
    assert np.array_equal(br32, ora.field(oracle.BR).astype(np.float32).astype(np.float64))
    ora.set_field(oracle.BR, br32)                  # oracle Psi of the same FP32 B_r
    assert np.array_equal(sim.field(ffpic.PSI), ora.field(oracle.PSI))
    assert np.array_equal(sim.field(ffpic.F), ora.field(oracle.F))


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_load_cells_and_sort_permutation_bit_exact(precision):
    w = W.tiny_open_dipole(30_000)
    sim, ora = pair(w, precision)
    sim.record_sort(True)
    load_both(sim, ora, w)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        # the load's sort: slot k holds input particle perm[k], in stable
        # cell order (equal cells keep the input order)
        perm = sim.sort_permutation(s)
        src = w.particles(s)
        assert len(perm) == len(g["cell"])
        assert np.array_equal(g["r"], src["r"][perm].astype(g["r"].dtype)) or \
            np.allclose(g["r"], src["r"][perm], rtol=1e-7, atol=0)
        same = np.diff(g["cell"]) == 0
        assert np.all(np.diff(g["cell"]) >= 0) and np.all(np.diff(perm)[same] > 0)
        assert len(g["cell"]) == len(o["cell"]) > 1000
        assert np.array_equal(g["cell"], o["cell"])
        if precision == W.FP64:
            for k in ("r", "th", "ur", "uth", "uph"):
                assert np.array_equal(g[k], o[k]), k
        else:
            assert np.allclose(g["r"], o["r"], rtol=1e-7, atol=0)
            assert np.allclose(g["uph"], o["uph"].astype(np.float32), rtol=0, atol=0)
        assert np.array_equal(sim.sort_offsets(s), ora.sort_offsets(s))
        assert np.array_equal(sim.diagnostics(ffpic.DIAG_MOMENTS)["removed"][s],
                              ora.removed(s))


def test_push_and_deposit_one_step_fp64():
    w = W.tiny_dipole(50_000)
    sim, ora = pair(w)
    load_both(sim, ora, w)
    sim.run_phases(ffpic.PHASE_PUSH)
    ora.phases(oracle.PHASE_PUSH)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        assert np.array_equal(g["cell"], o["cell"])
        live = o["cell"] >= 0
        for k in ("r", "th", "ur", "uth", "uph"):
            assert np.allclose(g[k][live], o[k][live], rtol=1e-13, atol=1e-13), k
    for gc, oc in ((ffpic.JR, oracle.JR), (ffpic.JTH, oracle.JTH), (ffpic.JPH, oracle.JPH)):
        assert rel(sim.field(gc), ora.field(oc)) < FP64_TOL


@pytest.mark.parametrize("band", [(3.0, 9.0), (1.05, 1.6)])
def test_push_and_deposit_one_step_fp32(band):
    """One FP32-mixed push against the FP64 oracle.  The (3, 9) band puts
    about 2.4 cells in a 64-particle wave (the in-cell deposit takes several
    passes); the band next to the star has about a fifth of the particles
    crossing a cell in the step, more than the workgroup's queue of
    cell-crossing moves holds, so the inline zigzag runs as well."""
    w = W.tiny_dipole(50_000)
    w.sheet_rmin, w.sheet_rmax = band
    sim, ora = pair(w, W.FP32_MIXED)
    load_both(sim, ora, w)
    sim.run_phases(ffpic.PHASE_PUSH)
    ora.phases(oracle.PHASE_PUSH)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        live = o["cell"] >= 0
        # FP32 positions can put a particle within rounding of an edge on the
        # other side of it
        assert np.mean(g["cell"] != o["cell"]) < 1e-3
        same = live & (g["cell"] == o["cell"])
        for k in ("ur", "uth", "uph"):
            assert np.allclose(g[k][same], o[k][same], rtol=1e-5, atol=1e-5 * np.abs(o[k]).max()), k
    for gc, oc in ((ffpic.JR, oracle.JR), (ffpic.JTH, oracle.JTH), (ffpic.JPH, oracle.JPH)):
        e = rel(sim.field(gc), ora.field(oc))
        print("FP32 deposit error", band, gc, e)
        assert e < 2e-5, (gc, e)        # measured 1.4e-7 .. 1.2e-6


@pytest.mark.parametrize("poles", ["north", "both"])
@pytest.mark.parametrize("precision", [W.FP32_MIXED, W.FP64])
def test_push_near_the_axes(poles, precision):
    """Particles within half a cell of the axis, where the gather takes the
    axis ghosts (even components reflected, odd ones with the sign flipped).
    With one pole only, a chunk's cell box is narrow and the FP32 push
    gathers from its LDS patch; with both poles every radial row holds both
    edge columns, the box spans the grid's width and the push gathers from
    HBM."""
    w = W.tiny_dipole(20_000)
    d = w.desc()
    d["precision"] = precision
    g = np.random.Generator(np.random.PCG64(20260))
    n = 20_000
    dth = math.pi / w.nth
    th = g.uniform(0.0, 0.5 * dth, n)
    if poles == "both":
        th[::2] = math.pi - th[::2]
    p = dict(r=g.uniform(2.0, 8.0, n), th=th)
    gam = np.exp(g.uniform(0.0, math.log(10.0), n))
    um = np.sqrt(gam * gam - 1.0)
    mu = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    p["ur"], p["uth"], p["uph"] = um * mu, um * np.sqrt(1 - mu * mu) * np.cos(ph), um * np.sqrt(1 - mu * mu) * np.sin(ph)
    sim = ffpic.Sim(d, capacity=[n, n])
    ora = oracle.Oracle(d)
    for s in range(2):
        sim.load_particles(s, p)
        ora.load(s, p)
    sim.run_phases(ffpic.PHASE_PUSH)
    ora.phases(oracle.PHASE_PUSH)
    rtol = 1e-12 if precision == W.FP64 else 1e-5
    for s in range(2):
        a, o = sim.particles(s), ora.particles(s)
        same = (o["cell"] >= 0) & (a["cell"] == o["cell"])
        assert np.mean(same) > 0.99
        for k in ("ur", "uth", "uph"):
            assert np.allclose(a[k][same], o[k][same], rtol=rtol, atol=rtol * np.abs(o[k]).max()), k
    for gc, oc in ((ffpic.JR, oracle.JR), (ffpic.JTH, oracle.JTH), (ffpic.JPH, oracle.JPH)):
        assert rel(sim.field(gc), ora.field(oc)) < (FP64_TOL if precision == W.FP64 else 2e-5), gc


def test_field_step_fp64():
    w = W.tiny_open_dipole(50_000)
    sim, ora = pair(w)
    load_both(sim, ora, w)
    for ph_g, ph_o in ((ffpic.PHASE_PUSH, oracle.PHASE_PUSH), (ffpic.PHASE_FIELDS, oracle.PHASE_FIELDS)):
        sim.run_phases(ph_g)
        ora.phases(ph_o)
    errs = field_errors(sim, ora)
    assert max(errs.values()) < FP64_TOL, errs


@pytest.mark.parametrize("with_particles", [False, True])
@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_fused_field_step_does_not_depend_on_the_slab_height(precision, with_particles):
    """The fused field step tiles the grid in strips of theta columns and
    slabs of radial rows that read each other's edge rows.  On a grid of
    three strips (the last ragged) with the absorber, the axis rows and
    force-free transition layers, any slab height gives the same fields:
    bit for bit without particles; with particles the deposit's atomic
    additions come in a different order from run to run, so to 1e-13 (FP64)
    or 1e-6 (FP32) element-wise.  Every run matches the oracle."""
    w = W.tiny_open_dipole(4000, steps=5)
    w.nr, w.nth = 61, 600
    psi_pc = w.mu / w.r_lc
    w.psi_thr = (0.85 * psi_pc, 0.9 * psi_pc, 2.3 * psi_pc, 2.4 * psi_pc)
    tol = FP64_TOL if precision == W.FP64 else FP32_TOL
    same = (0.0 if not with_particles else (1e-13 if precision == W.FP64 else 1e-6))
    out = {}
    for rows in (0, 1, 2, 3, 7, 40):
        sim, ora = pair(w, precision)
        sim.set_field_rows(rows)
        if with_particles:
            load_both(sim, ora, w)
        sim.step(5)
        ora.step(5)
        # without particles B_phi and E_phi stay ~1e-9 of the field: in
        # FP32 they are measured against their field group
        errs = field_errors(sim, ora) if precision == W.FP64 or with_particles \
            else field_errors_grouped(sim, ora)
        assert max(errs.values()) < tol, (rows, errs)
        out[rows] = [sim.field(g) for g, _, _ in FIELDS]
    for rows, fields in out.items():
        for k, (a, b) in enumerate(zip(fields, out[0])):
            if same == 0.0:
                assert np.array_equal(a, b), (rows, FIELDS[k][2])
            else:
                assert rel(a, b) <= same, (rows, FIELDS[k][2], rel(a, b))


@pytest.mark.parametrize("factory", [W.tiny_dipole, W.tiny_open_dipole])
def test_full_steps_fp64(factory):
    w = factory(100_000, steps=20)
    sim, ora = pair(w)
    load_both(sim, ora, w)
    sim.step(20)
    ora.step(20)
    sim.sync()
    errs = field_errors(sim, ora)
    assert max(errs.values()) < FP64_TOL, errs
    m = moment_errors(sim, ora, 2)
    for k, v in m.items():
        assert v < (0.5 if k.startswith("n") else FP64_TOL), (k, v)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        assert len(g["cell"]) == len(o["cell"])
        assert np.count_nonzero(g["cell"] != o["cell"]) == 0


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_table1_transition_layers_both_ff_domains(precision):
    """The flux bands of Table 1 on the open dipole: force-free below
    0.85 Psi_pc, linear layer to 0.9 Psi_pc, PIC up to 2.3 Psi_pc, linear
    layer to 2.4 Psi_pc, force-free above (the closed zone near the star).
    Exercises fractional f in the blend, the weighted correction and both
    force-free domains."""
    w = W.tiny_open_dipole(40_000, steps=12)
    psi_pc = w.mu / w.r_lc
    w.psi_thr = (0.85 * psi_pc, 0.9 * psi_pc, 2.3 * psi_pc, 2.4 * psi_pc)
    sim, ora = pair(w, precision)
    f = sim.field(ffpic.F)
    assert np.any((f > 0) & (f < 1)) and np.any(f == 1.0) and np.any(f == 0.0)
    fo = ora.field(oracle.F)
    if precision == W.FP64:
        assert np.array_equal(f, fo)
    else:
        # Psi comes from the FP32 B_r, so f inside the linear layers moves by
        # (relative Psi change ~1e-7) * Psi / (layer width)
        assert np.allclose(f, fo, rtol=0, atol=1e-5)
    load_both(sim, ora, w)
    sim.step(12)
    ora.step(12)
    sim.sync()
    errs = field_errors(sim, ora)
    tol = FP64_TOL if precision == W.FP64 else FP32_TOL
    assert max(errs.values()) < tol, errs
    m = moment_errors(sim, ora, 2)
    for k, v in m.items():
        if k.startswith("n"):
            assert v <= (0 if precision == W.FP64 else 2e-5 * w.n_per_species + 2), (k, v)
        else:
            assert v < tol, (k, v)


def test_michel_monopole_pure_ff_fp64_gpu():
    w = W.michel_monopole(64, pure_ff=True, init=W.INIT_MONOPOLE)
    sim, ora = pair(w, cap=1)
    sim.step(200)
    ora.step(200)
    errs = field_errors(sim, ora)
    assert max(errs.values()) < FP64_TOL, errs
    L = sim.diagnostics(ffpic.DIAG_ENERGY, poynting=True)["L"]
    assert np.allclose(L, ora.poynting(), rtol=1e-10, atol=1e-14)


def small_sheet(n_total=200_000, nr=256):
    w = W.sheet_1024(n_total=n_total, steps=100)
    w.nr = w.nth = nr
    return w


def test_fp32_mixed_vs_fp64_oracle_100_steps():
    w = small_sheet()
    sim, ora = pair(w, W.FP32_MIXED)
    load_both(sim, ora, w)
    sim.step(100)
    ora.step(100)
    sim.sync()
    errs = field_errors(sim, ora)
    print("FP32-mixed field errors after 100 steps:", errs)
    assert max(errs.values()) < FP32_TOL, errs
    m = moment_errors(sim, ora, 2)
    print("FP32-mixed moment errors after 100 steps:", m)
    for k, v in m.items():
        if k.startswith("n"):
            assert v <= 2e-5 * w.n_per_species + 2, (k, v)
        else:
            assert v < FP32_TOL, (k, v)


def test_residual_maps_match_oracle_fp64():
    w = W.tiny_dipole(50_000)
    sim, ora = pair(w)
    load_both(sim, ora, w)
    sim.step(5)
    ora.step(5)
    g, o = sim.field(ffpic.GAUSS), ora.gauss()
    assert rel(g, o) < 1e-10
    g, o = sim.field(ffpic.DIVB), ora.divb()
    # both are roundoff: compare on the scale of the face-flux terms
    scale = np.abs(ora.field(oracle.BR)).max() / (math.exp(ora.dlog) - 1.0)
    assert np.abs(g - o).max() < 1e-13 * scale
    dg = sim.diagnostics(ffpic.DIAG_RESIDUALS)
    assert abs(dg["gauss_max"] - np.abs(ora.gauss()).max()) <= 1e-9 * np.abs(ora.gauss()).max()


def _charge_scale(ora, d):
    """max over interior nodes of |4 pi rho|, rho the oracle's node charge
    over the dual-cell volume"""
    dr3h = ffpic.host_table(d, ffpic.TAB_DR3H)
    dcd = ffpic.host_table(d, ffpic.TAB_DCD)
    vol = dr3h[:, None] * dcd[None, :]
    rho = ora.node_charge() / vol
    return 4.0 * math.pi * np.abs(rho[1:-1]).max()


@pytest.mark.parametrize("factory", [W.tiny_dipole, W.tiny_open_dipole])
def test_gauss_residual_fp32_mixed_in_fp64(factory):
    """The FP32-mixed path forms its Gauss residual in FP64 from the FP64
    background plus the FP32 perturbation, so it resolves the FP32 charge
    conservation error of the deposit rather than the rounding of the
    corotation background.  After 8 steps its map agrees with the oracle's
    (which is roundoff) to 2e-5 of the largest 4 pi rho of the particles."""
    w = factory(50_000, steps=8)
    sim, ora = pair(w, W.FP32_MIXED)
    load_both(sim, ora, w)
    sim.step(8)
    ora.step(8)
    g, o = sim.field(ffpic.GAUSS), ora.gauss()
    scale = _charge_scale(ora, w.desc())
    err = np.abs(g - o).max() / scale
    dg = sim.diagnostics(ffpic.DIAG_RESIDUALS)
    print("FP32-mixed Gauss residual:", factory.__name__, "max |G - G_oracle| / max|4 pi rho| =",
          err, "max |G| / max|4 pi rho| =", np.abs(g).max() / scale,
          "oracle:", np.abs(o).max() / scale)
    assert err < FP32_TOL, err
    assert dg["gauss_max"] == np.abs(g).max()
    # the div B residual of the same run, FP64 background plus perturbation
    db = sim.field(ffpic.DIVB)
    bscale = np.abs(ora.field(oracle.BR)).max() / (math.exp(ora.dlog) - 1.0)
    print("FP32-mixed div B:", np.abs(db).max() / bscale, "oracle:", np.abs(ora.divb()).max() / bscale)
    assert np.abs(db - ora.divb()).max() < 1e-6 * bscale
    assert dg["divb_max"] == np.abs(db).max()


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_save_restore_resumes(precision):
    w = W.tiny_open_dipole(20_000)
    sim, _ = pair(w, precision)
    for s in range(2):
        sim.load_particles(s, w.particles(s))
    sim.step(3)
    blob = sim.save()
    sim.step(4)
    a = {n: sim.field(g) for g, _, n in FIELDS}
    pa = sim.particles(0)
    sim.restore(blob)
    assert sim.diagnostics(0)["step"] == 3
    sim.step(4)
    b = {n: sim.field(g) for g, _, n in FIELDS}
    pb = sim.particles(0)
    tol = 1e-13 if precision == W.FP64 else 1e-6
    for n in a:
        assert rel(b[n], a[n]) < tol, n
    assert np.array_equal(pa["cell"], pb["cell"])


def test_error_paths():
    w = W.tiny_dipole(100)
    sim, _ = pair(w, cap=150)
    p = w.particles(0)
    p["r"][:5] = np.nan
    p["th"][5:8] = -1.0
    sim.load_particles(0, p)
    assert sim.n(0) == 92
    assert sim.diagnostics(0)["removed"][0][0] == 8
    with pytest.raises(ffpic.FfpicError) as e:
        sim.load_particles(0, w.particles(0))          # 92 + 100 > 150 slots
    assert e.value.code == ffpic.ECAPACITY
    assert sim.n(0) == 92


def edge_particles(w, base):
    """Particles on the domain's edges and on grid lines: r at r_min, on a
    node radius and just below the absorber, theta on the axis, on a node
    angle and at the equator; plus a few outside the domain."""
    dlog = math.log(w.rmax / w.rmin) / w.nr
    dth = math.pi / w.nth
    r_edge = [w.rmin, w.rmin * math.exp(3 * dlog), w.r_abs * (1 - 1e-12), 0.5 * (w.r_lc + w.r_abs),
              w.rmin * 0.999, w.r_abs * 1.0001]
    th_edge = [0.0, math.pi, 7 * dth, 0.5 * math.pi, 1e-300, math.pi - 1e-15]
    rr, tt = np.meshgrid(r_edge, th_edge, indexing="ij")
    n = rr.size
    out = {"r": np.concatenate([base["r"], rr.ravel()]),
           "th": np.concatenate([base["th"], tt.ravel()])}
    for k, v in (("ur", 0.3), ("uth", -0.2), ("uph", 0.5)):
        out[k] = np.concatenate([base[k], np.full(n, v)])
    return out


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_ragged_grid_edge_particles_and_empty_species(precision):
    """A grid whose sizes match no tile (97 x 61), particles on the domain's
    edges and grid lines (cells bit-exact in FP64), an empty second species,
    a few steps against the oracle."""
    w = W.tiny_open_dipole(3000, steps=6)
    w.nr, w.nth = 97, 61
    sim, ora = pair(w, precision, cap=w.n_per_species + 64)
    p = edge_particles(w, w.particles(0))
    sim.load_particles(0, p)
    ora.load(0, p)
    g, o = sim.particles(0), ora.particles(0)
    assert len(g["cell"]) == len(o["cell"])
    assert sim.diagnostics(ffpic.DIAG_MOMENTS)["removed"][0] == list(ora.removed(0))
    if precision == W.FP64:
        assert np.array_equal(g["cell"], o["cell"])
    sim.step(6)
    ora.step(6)
    sim.sync()
    assert sim.n(1) == 0
    assert sim.diagnostics(ffpic.DIAG_MOMENTS)["alive"][1] == 0
    errs = field_errors(sim, ora)
    assert max(errs.values()) < (FP64_TOL if precision == W.FP64 else FP32_TOL), errs


def expected_stable_order(cells, kill_cell):
    """Stable order by cell of the live particles not in a kill cell."""
    live = (cells >= 0) & ~kill_cell
    idx = np.nonzero(live)[0]
    return idx[np.argsort(cells[idx], kind="stable")]


def kill_cells(sim, nr, nth):
    f = sim.field(ffpic.F)
    k = (f[:-1, :-1] == 1.0) & (f[1:, :-1] == 1.0) & (f[:-1, 1:] == 1.0) & (f[1:, 1:] == 1.0)
    return k[:nr, :nth].reshape(-1)


@pytest.mark.parametrize("precision", [W.FP32_MIXED, W.FP64])
def test_incremental_sort_is_the_stable_sort(precision):
    """After steps without a sort, the (incremental) re-sort puts every
    particle where a stable sort of the current cells puts it: the exported
    state after the sort is exactly the pre-sort state permuted.  Few
    particles change cell here, so the FP32 sort moves them through its
    compact buffer."""
    check_incremental_sort(small_sheet(60_000, nr=192), precision, moved=(0.0, 0.25))


@pytest.mark.parametrize("precision", [W.FP64, W.FP32_MIXED])
def test_incremental_sort_many_movers(precision):
    """The same with most particles changing cell between sorts (a band next
    to the star, where a fifth of them cross a cell every step): more than
    the FP32 compact buffer holds, so the direct scatter runs."""
    w = W.tiny_dipole(40_000)
    w.sheet_rmin, w.sheet_rmax = 1.05, 1.6
    check_incremental_sort(w, precision, moved=(0.3, 1.0))


def check_incremental_sort(w, precision, moved):
    """moved: bounds on the fraction of slots whose cell changed since the
    previous sort (the FP32 compact buffer holds a quarter of the slots)."""
    d = w.desc()
    d["precision"] = precision
    d["sort_interval"] = 1000           # only the load sorts during the steps
    sim = ffpic.Sim(d, capacity=[w.n_per_species] * 2)
    for s in range(2):
        sim.load_particles(s, w.particles(s))
    prev = [sim.particles(s)["cell"] for s in range(2)]
    sim.record_sort(True)
    for rnd in range(3):
        sim.step(4)
        sim.run_phases(ffpic.PHASE_MASK)
        kc = kill_cells(sim, w.nr, w.nth)
        before = [sim.particles(s) for s in range(2)]
        for s in range(2):
            c0 = before[s]["cell"]
            frac = np.mean(c0[:len(prev[s])] != prev[s][:len(c0)])
            assert moved[0] <= frac <= moved[1], (rnd, s, frac)
        sim.run_phases(ffpic.PHASE_SORT)
        for s in range(2):
            p0 = before[s]
            cells = p0["cell"]
            killed = np.zeros(len(cells), dtype=bool)
            ok = cells >= 0
            killed[ok] = kc[cells[ok]]
            order = expected_stable_order(cells, killed)
            p1 = sim.particles(s)
            assert len(p1["r"]) == len(order), (rnd, s)
            assert np.array_equal(sim.sort_permutation(s), order), (rnd, s)
            for k in ("cell", "r", "th", "ur", "uth", "uph"):
                assert np.array_equal(p1[k], p0[k][order]), (rnd, s, k)
            off = sim.sort_offsets(s)
            assert off[-1] == len(order)
            assert np.array_equal(np.diff(off), np.bincount(p1["cell"], minlength=len(off) - 1))
            prev[s] = p1["cell"]


def test_sort_placed_by_the_push_fp32():
    """FP32: in a step that sorts and pushes, the push writes its particles
    in the sorted order (the sort's separate placement pass is skipped).
    Twin contexts take the same steps, one through ffpic_step (graph cycles
    included) and one with the sort and the rest of each step as separate
    phase calls (the sort then places the particles itself): the particle
    state after every step is bit-identical, the recorded permutation of
    each sort is the stable order of the pre-sort cells, and the fields
    agree exactly.  The particles carry no charge (weight 0), so the
    deposit adds zeros and the order of its atomic additions cannot make
    the twins' fields, and so their particles, differ."""
    w = small_sheet(60_000, nr=192)
    d = w.desc()
    d["precision"] = W.FP32_MIXED
    d["sort_interval"] = 4
    d["weight"] = [0.0, 0.0]
    a = ffpic.Sim(d, capacity=[w.n_per_species] * 2)
    b = ffpic.Sim(d, capacity=[w.n_per_species] * 2)
    for sim in (a, b):
        sim.record_sort(True)
        for s in range(2):
            sim.load_particles(s, w.particles(s))
    rest = (ffpic.PHASE_INJECT | ffpic.PHASE_EXTRACT | ffpic.PHASE_PUSH | ffpic.PHASE_PAIRS |
            ffpic.PHASE_FIELDS)
    for cycle in range(3):
        # b: the cycle's four steps as phase calls, the sort on its own
        b.run_phases(ffpic.PHASE_MASK)
        kc = kill_cells(b, w.nr, w.nth)
        before = [b.particles(s)["cell"] for s in range(2)]
        b.run_phases(ffpic.PHASE_SORT)
        b.run_phases(rest)
        for _ in range(3):
            b.run_phases(ffpic.PHASE_MASK | rest)
        # a: the same four steps as one call (a graph after the first cycle)
        a.step(4)
        a.sync()
        b.sync()
        for s in range(2):
            pa, pb = a.particles(s), b.particles(s)
            for k in ("cell", "r", "th", "ur", "uth", "uph"):
                assert np.array_equal(pa[k], pb[k]), (cycle, s, k)
            c0 = before[s]
            killed = np.zeros(len(c0), dtype=bool)
            ok = c0 >= 0
            killed[ok] = kc[c0[ok]]
            order = expected_stable_order(c0, killed)
            assert np.array_equal(a.sort_permutation(s), order), (cycle, s)
            assert np.array_equal(b.sort_permutation(s), order), (cycle, s)
        for g, _, n in FIELDS:
            assert np.array_equal(a.field(g), b.field(g)), (cycle, n)
    assert a.graph_stats()[1] >= 1
    a.close()
    b.close()


def oracle_ulp_sensitivity(desc, steps):
    """Relative field change of the oracle after `steps` steps when every
    E node is moved by one ulp after the first step: the size of difference
    that rounding alone produces in this configuration."""
    a, b = oracle.Oracle(desc), oracle.Oracle(desc)
    a.step(1)
    b.step(1)
    for c in (oracle.ER, oracle.ETH, oracle.EPH):
        b.set_field(c, np.nextafter(b.field(c), np.inf))
    a.step(steps - 1)
    b.step(steps - 1)
    return max(rel(b.field(o), a.field(o)) for _, o, _ in FIELDS)


def test_injection_matches_oracle_fp64():
    """Surface pair injection of the hybrid monopole.  The injected pairs of
    one phase agree with the oracle's (same Philox draws, same positions) and
    the first steps agree to 1e-12.  Freshly injected pairs are accelerated
    to gamma ~ 100 within a few steps, which amplifies one-ulp differences
    (the device exp and sin against the C library's) by about 1.8x per step:
    after 20 steps the fields are held to ten times the oracle's own change
    under a one-ulp perturbation, and the particle counts exactly."""
    w = W.hybrid_monopole(64)
    sim, ora = pair(w, W.FP64, cap=200_000)
    sim.run_phases(ffpic.PHASE_MASK | ffpic.PHASE_INJECT)
    ora.phases(oracle.PHASE_MASK | oracle.PHASE_INJECT)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        assert len(g["r"]) == len(o["r"]) > 10
        assert np.array_equal(g["cell"], o["cell"])
        assert np.array_equal(g["th"], o["th"])
        for k in ("r", "uph"):
            assert np.allclose(g[k], o[k], rtol=1e-15, atol=0), k
    sim2, ora2 = pair(w, W.FP64, cap=200_000)
    for k in range(EARLY_STEPS):
        sim2.step(1)
        ora2.step(1)
        errs = field_errors(sim2, ora2)
        assert max(errs.values()) < FP64_TOL, (k + 1, errs)
    m = moment_errors(sim2, ora2, 2)
    for k, v in m.items():
        assert v < (0.5 if k.startswith("n") else FP64_TOL), (k, v)
    sim2.step(20 - EARLY_STEPS)
    ora2.step(20 - EARLY_STEPS)
    sim2.sync()
    sens = oracle_ulp_sensitivity(sim2.desc, 20)
    errs = field_errors(sim2, ora2)
    assert max(errs.values()) < 10 * max(sens, FP64_TOL), (errs, sens)
    dg = sim2.diagnostics(ffpic.DIAG_MOMENTS)
    for s in range(2):
        assert dg["alive"][s] == ora2.moments(s)[0]


def field_errors_grouped(sim, ora, elementwise=True):
    """Per-component errors normalised by the field group (E or B)
    rather than by the component itself."""
    return {**rel_grouped([(n, sim.field(g), ora.field(o)) for g, o, n in FIELDS[:3]],
                          elementwise),
            **rel_grouped([(n, sim.field(g), ora.field(o)) for g, o, n in FIELDS[3:]],
                          elementwise)}

def test_injection_fp32_and_capacity_error():
    """FP32-mixed hybrid monopole with injection.  E_r, E_phi, B_theta and
    B_phi start at zero here and are ~1e-5 of the corotation field after a
    step, so errors are measured against the norm of the field group: the
    first 5 steps hold 2e-5 in L2, the first 4 also element-wise.  Later the trajectories' sensitivity (see the
    FP64 test) amplifies FP32 rounding beyond any fixed bar, and 20 steps
    are held to the particle counts only."""
    w = W.hybrid_monopole(64, precision=W.FP32_MIXED)
    sim, ora = pair(w, W.FP32_MIXED, cap=200_000)
    sim.run_phases(ffpic.PHASE_MASK | ffpic.PHASE_INJECT)
    ora.phases(oracle.PHASE_MASK | oracle.PHASE_INJECT)
    for s in range(2):
        g, o = sim.particles(s), ora.particles(s)
        assert np.array_equal(g["cell"], o["cell"])
        for k in ("r", "th"):
            assert np.allclose(g[k], o[k], rtol=2e-7, atol=0), k
        assert np.allclose(g["uph"], o["uph"], rtol=2e-7, atol=0)
    sim, ora = pair(w, W.FP32_MIXED, cap=200_000)
    for k in range(5):
        sim.step(1)
        ora.step(1)
        errs = field_errors_grouped(sim, ora, elementwise=False)
        errs_max = field_errors_grouped(sim, ora)
        print("injected monopole FP32 step", k + 1, "group L2", max(errs.values()),
              "group element-wise", max(errs_max.values()), errs_max)
        assert max(errs.values()) < FP32_TOL, (k + 1, errs)
        # element-wise (the largest error at any node against the group's
        # largest entry): held for 4 steps (measured 1.3e-6 .. 4.3e-6); at
        # step 5 one E_r node next to the injection layer reaches 2.9e-5
        if k < 4:
            assert max(errs_max.values()) < FP32_TOL, (k + 1, errs_max)
    sim.step(15)
    ora.step(15)
    sim.sync()
    dg = sim.diagnostics(ffpic.DIAG_MOMENTS)
    for s in range(2):
        n_o = ora.moments(s)[0]
        assert n_o > 100 and abs(dg["alive"][s] - n_o) <= 0.05 * n_o, (s, dg["alive"][s], n_o)
    # a capacity too small for one step's injection is reported, not overrun
    small, _ = pair(w, W.FP32_MIXED, cap=3)
    small.step(1)
    with pytest.raises(ffpic.FfpicError) as e:
        small.sync()
    assert e.value.code == ffpic.ECAPACITY
    assert small.n(0) == 0
