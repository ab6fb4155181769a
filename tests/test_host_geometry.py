"""The library's host-built geometry tables and initial fields equal the
oracle's bit for bit (CPU only: ffpic_host_table and
ffpic_host_initial_field touch no device).

Both sides build the grid of Sect. 4 (log-spaced r, uniform theta) in FP64
from libm's exp, sin and cos; the face areas, dual volumes and initial
fields are then plain products and differences of those tables.  Equal
tables therefore give equal cells, Psi and initial fields on the GPU, in
both precisions.  Grid (40, 300) is the one where the oracle's sin and cos,
once merged by the compiler into one sincos call, differed in the last bit
(theta_j = 80 pi / 300 and 159 pi / 300).
"""
import numpy as np
import pytest

import oracle
from paper_2406_14512_amd import ffpic
from paper_2406_14512_amd import workloads as W

GRIDS = [(96, 80), (40, 300), (128, 128), (300, 40), (1024, 1024), (257, 513)]
FIELD_GRIDS = [(96, 80), (40, 300), (128, 128), (300, 40), (257, 513)]


def _desc(grid, init=W.INIT_OPEN_DIPOLE, **kw):
    w = W.tiny_open_dipole(10)
    w.nr, w.nth = grid
    w.init = init
    d = w.desc()
    d.update(kw)
    return d


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)
    ffpic.lib()


@pytest.mark.parametrize("grid", GRIDS)
def test_geometry_tables_bit_exact(grid):
    d = _desc(grid)
    o = oracle.Oracle(d)
    t = {k: ffpic.host_table(d, k) for k in range(19)}
    rn, rh, thn, sn, cn, sh, ch = (o.geometry(k) for k in range(7))
    nr, nth = grid
    for got, exp, name in ((t[ffpic.TAB_RN], rn, "r_i"), (t[ffpic.TAB_RH], rh, "r_{i+1/2}"),
                           (t[ffpic.TAB_THN], thn, "theta_j"), (t[ffpic.TAB_SN], sn, "sin theta_j"),
                           (t[ffpic.TAB_CN], cn, "cos theta_j"),
                           (t[ffpic.TAB_SH], sh, "sin theta_{j+1/2}")):
        assert got.shape == exp.shape, name
        bad = np.nonzero(got != exp)[0]
        assert len(bad) == 0, f"{name} differs at {bad[:8]}"
    # derived tables: products and differences of the same entries
    assert np.array_equal(t[ffpic.TAB_RN2], rn * rn)
    assert np.array_equal(t[ffpic.TAB_RH2], rh * rh)
    assert np.array_equal(t[ffpic.TAB_DRN], rn[1:] - rn[:-1])
    assert np.array_equal(t[ffpic.TAB_DCN], cn[:-1] - cn[1:])
    assert np.array_equal(t[ffpic.TAB_DR2N], (rn[1:] * rn[1:] - rn[:-1] * rn[:-1]) * 0.5)
    lo = np.concatenate(([rn[0]], rh))
    hi = np.concatenate((rh, [rn[nr]]))
    assert np.array_equal(t[ffpic.TAB_DR2H], (hi * hi - lo * lo) * 0.5)
    assert np.array_equal(t[ffpic.TAB_DR3H], (hi * hi * hi - lo * lo * lo) / 3.0)
    clo = np.concatenate(([1.0], ch))
    chi = np.concatenate((ch, [-1.0]))
    assert np.array_equal(t[ffpic.TAB_DCD], clo - chi)
    assert t[ffpic.TAB_DCD].shape == (nth + 1,)


@pytest.mark.parametrize("init", [W.INIT_DIPOLE, W.INIT_MONOPOLE, W.INIT_MICHEL,
                                  W.INIT_OPEN_DIPOLE])
@pytest.mark.parametrize("grid", FIELD_GRIDS)
def test_initial_fields_bit_exact(grid, init):
    d = _desc(grid, init)
    o = oracle.Oracle(d)
    for g, c, name in ((ffpic.ER, oracle.ER, "Er"), (ffpic.ETH, oracle.ETH, "Eth"),
                       (ffpic.EPH, oracle.EPH, "Eph"), (ffpic.BR, oracle.BR, "Br"),
                       (ffpic.BTH, oracle.BTH, "Bth"), (ffpic.BPH, oracle.BPH, "Bph")):
        got, exp = ffpic.host_initial_field(d, g), o.field(c)
        bad = np.argwhere(got != exp)
        assert len(bad) == 0, f"{name} differs at {bad[:6].tolist()}"


def test_host_hooks_reject_bad_arguments():
    d = _desc((16, 16))
    with pytest.raises(ffpic.FfpicError):
        ffpic.host_table(d, 19)
    with pytest.raises(ffpic.FfpicError):
        ffpic.host_initial_field(d, ffpic.JR)
    bad = dict(d, nr=1)
    with pytest.raises(ffpic.FfpicError):
        ffpic.host_table(bad, 0)
