"""Closed-form pins of the oracle's particle kinematics and azimuthal deposit.

The push integrates the equation of motion of Sect. 3 (eq. motion) in a
local Cartesian frame at the particle's azimuth, then rotates position and
momentum back into the meridional plane; the deposit of Sect. 3 includes the
azimuthal current J_phi.  The Boris algebra and the Gauss-law pins cannot see
a mistake in those frame changes or in J_phi (Gauss's law holds for any
trajectory, and the rotation does not depend on the basis), so these tests
follow particles in 3-D Cartesian space, written from the definitions of the
spherical unit vectors, and compare with what geometry fixes:

* free streaming in zero fields is the straight line x0 + n dt v, exactly
  (1e-12), also across the equator and past either pole within a cell;
* a uniform E along the rotation axis with B = 0: the discrete Boris map
  adds dt omega_B (q/m) E to u each step, so u_z grows linearly; the field
  comes from the grid by bilinear interpolation, so this holds to
  O(dtheta^2);
* gyration in a uniform B0 z built from nodal Psi = B0 r^2 sin^2(theta) / 2:
  the discrete orbit (u turned by 2 atan(omega dt / 2) per step about z,
  positions summed) to O(Delta^2), second order between two grids;
* the azimuthal E x B drift -E0/B0 in E = E0 varpi-hat, B = B0 z;
* the azimuthal deposit of a move: its node sums total Q v_phi and are
  centred on the move's midpoint in logical coordinates (log r / Delta,
  theta / dtheta); after Ampere, the current density integrated over the
  meridional cross-section is the ring current Q v_phi / varpi (2 pi
  dropped), to O(Delta^2).
"""
import math

import numpy as np
import pytest

from paper_2406_14512_amd import workloads as W

INF = float("inf")


def _desc(n, **kw):
    d = dict(nr=n, nth=n, rmin=1.0, rmax=10.0, r_lc=3.0, r_abs=9.0, mu=1.0, cfl=0.5,
             omega_b=1000.0, rr_coef=0.0, psi_thr=(-INF, -INF, INF, INF), ff_enable=0,
             init=W.INIT_ZERO, precision=0, sort_interval=1, nspec=1, qm=(1.0,),
             weight=(1e-3,))
    d.update(kw)
    return d


# --- spherical geometry, from the definitions of the unit vectors ----------

def _basis(th, ph):
    """r-hat, theta-hat, phi-hat at polar angle th and azimuth ph."""
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    return (np.array([st * cp, st * sp, ct]),
            np.array([ct * cp, ct * sp, -st]),
            np.array([-sp, cp, 0.0]))


def _to_cart(r, th, ur, uth, uph):
    """position and momentum of a meridional-plane state placed at azimuth 0"""
    er, et, ep = _basis(th, 0.0)
    return r * er, ur * er + uth * et + uph * ep


def _to_local(X, U):
    """(r, theta, u_r, u_theta, u_phi) of a Cartesian state at its own azimuth"""
    r = float(np.linalg.norm(X))
    th = math.acos(max(-1.0, min(1.0, X[2] / r)))
    ph = math.atan2(X[1], X[0])
    er, et, ep = _basis(th, ph)
    return np.array([r, th, U @ er, U @ et, U @ ep])


def _load(o, states):
    """Loads the states; the load sorts by cell, so the slot order of the
    given states is kept on the handle for _state()."""
    a = np.array(states, dtype=np.float64)
    p = dict(r=a[:, 0], th=a[:, 1], ur=a[:, 2], uth=a[:, 3], uph=a[:, 4])
    assert o.load(0, p) == len(a)
    got = o.particles(0)
    slot = np.empty(len(a), dtype=np.int64)
    for k in range(len(a)):
        hit = np.nonzero((got["r"] == a[k, 0]) & (got["th"] == a[k, 1]))[0]
        assert len(hit) == 1
        slot[k] = hit[0]
    o.slot_of = slot


def _state(o):
    """state rows in the order the states were given to _load()"""
    p = o.particles(0)
    return np.stack([p["r"], p["th"], p["ur"], p["uth"], p["uph"]], axis=1)[o.slot_of]


def _logical(o, r, th):
    return math.log(r / o.desc["rmin"]) / o.dlog, th / o.dth


# ---------------------------------------------------------------------------
# free streaming: straight lines in 3-D

FREE = [
    (5.0, 1.0, 0.3, -0.5, 0.8),                    # generic
    (4.0, 0.5 * math.pi - 0.05, 0.2, 1.5, 0.4),    # crosses the equator southwards
    (5.5, 0.5 * math.pi + 0.04, -0.3, -1.2, -0.6),  # crosses it northwards
    (5.0, 0.02, 0.1, -2.0, 0.05),                  # passes the north pole inside a cell
    (6.0, math.pi - 0.03, -0.2, 2.0, -0.04),       # passes the south pole inside a cell
    (5.0, 0.5 * math.pi, 0.0, 0.0, 3.0),           # purely azimuthal: drifts outwards
    (3.5, 2.2, 9.0, 1.0, -2.0),                    # fast, mostly radial
]


@pytest.mark.parametrize("n", [32, 48])
def test_free_streaming_is_a_straight_line(oracle_lib, n):
    o = oracle_lib.Oracle(_desc(n))
    _load(o, FREE)
    dt = o.dt
    start = [_to_cart(*s) for s in FREE]
    nsteps = 60
    for k in range(1, nsteps + 1):
        o.phases(oracle_lib.PHASE_PUSH)
        got = _state(o)
        assert got.shape[0] == len(FREE)
        for p, (X0, U) in enumerate(start):
            g = math.sqrt(1.0 + U @ U)
            exp = _to_local(X0 + k * dt * U / g, U)
            scale_u = float(np.linalg.norm(U))
            assert abs(got[p, 0] - exp[0]) <= 1e-12 * exp[0], (k, p, "r")
            assert abs(got[p, 1] - exp[1]) <= 1e-12, (k, p, "theta")
            assert np.all(np.abs(got[p, 2:] - exp[2:]) <= 1e-12 * scale_u), (k, p, "u")
    # the pole-passing particles did come within one cell of the axis
    for p in (3, 4):
        X0, U = start[p]
        g = math.sqrt(1.0 + U @ U)
        w = min(math.hypot(*(X0 + k * dt * U / g)[:2]) for k in range(nsteps + 1))
        assert w < 0.1 * np.linalg.norm(X0) * o.dth


# ---------------------------------------------------------------------------
# uniform E along the rotation axis, B = 0

def _uniform_Ez_error(oracle_lib, n, E0=1e-3, T=2.4):
    o = oracle_lib.Oracle(_desc(n))
    nsteps = int(round(T / o.dt))
    th_n = np.arange(n + 1) * o.dth
    th_h = (np.arange(n + 1) + 0.5) * o.dth
    shape = o.shape
    # E = E0 z: E_r = E0 cos(theta) at (i+1/2, j), E_theta = -E0 sin(theta) at (i, j+1/2)
    o.set_field(oracle_lib.ER, np.broadcast_to(E0 * np.cos(th_n)[None, :], shape))
    o.set_field(oracle_lib.ETH, np.broadcast_to(-E0 * np.sin(th_h)[None, :], shape))
    states = [(5.0, 1.0, 0.2, 0.1, 0.3), (4.0, 2.0, -0.1, 0.3, -0.2)]
    _load(o, states)
    kick = o.dt * o.desc["omega_b"] * o.desc["qm"][0] * E0   # exact Boris kick, B = 0
    X = [_to_cart(*s)[0] for s in states]
    U = [_to_cart(*s)[1] for s in states]
    err_u = err_x = 0.0
    for _ in range(nsteps):
        o.phases(oracle_lib.PHASE_PUSH)
        got = _state(o)
        for p in range(len(states)):
            U[p] = U[p] + np.array([0.0, 0.0, kick])
            X[p] = X[p] + o.dt * U[p] / math.sqrt(1.0 + U[p] @ U[p])
            exp = _to_local(X[p], U[p])
            err_u = max(err_u, float(np.abs(got[p, 2:] - exp[2:]).max()))
            err_x = max(err_x, abs(got[p, 0] - exp[0]), exp[0] * abs(got[p, 1] - exp[1]))
    return err_u / (nsteps * kick), err_x, o.dth


def test_uniform_E_along_axis_accelerates_linearly(oracle_lib):
    e1, x1, dth1 = _uniform_Ez_error(oracle_lib, 32)
    e2, x2, dth2 = _uniform_Ez_error(oracle_lib, 64)
    # bilinear interpolation of cos/sin between samples: error <= dtheta^2 / 8
    assert e1 < dth1 ** 2 and e2 < dth2 ** 2
    assert e1 / e2 > 2.5                      # second order
    assert x2 < x1 and x2 < 1e-3


# ---------------------------------------------------------------------------
# uniform B0 z built from nodal Psi = B0 r^2 sin^2(theta) / 2

def _set_uniform_Bz(o, oracle_lib, B0):
    nr, nth = o.nr, o.nth
    r = o.desc["rmin"] * np.exp(np.arange(nr + 1) * o.dlog)
    th = np.arange(nth + 1) * o.dth
    st, ct = np.sin(th), np.cos(th)
    st[0] = st[-1] = 0.0
    ct[0], ct[-1] = 1.0, -1.0
    psi = 0.5 * B0 * r[:, None] ** 2 * st[None, :] ** 2
    br = np.zeros(o.shape)
    bth = np.zeros(o.shape)
    # magnetic flux through each face divided by its area (per radian of phi)
    face_r = r[:, None] ** 2 * (ct[None, :-1] - ct[None, 1:])
    br[:, :-1] = (psi[:, 1:] - psi[:, :-1]) / face_r
    face_t = st[None, 1:-1] * 0.5 * (r[1:, None] ** 2 - r[:-1, None] ** 2)
    bth[:-1, 1:-1] = -(psi[1:, 1:-1] - psi[:-1, 1:-1]) / face_t
    o.set_field(oracle_lib.BR, br)
    o.set_field(oracle_lib.BTH, bth)


def _gyration_error(oracle_lib, n, periods=1.25):
    d = _desc(n)
    o = oracle_lib.Oracle(d)
    B0, wq = 1e-3, d["omega_b"] * d["qm"][0]
    _set_uniform_Bz(o, oracle_lib, B0)
    start = (5.0, 1.2, 0.1, 0.35, -0.3)
    _load(o, [start])
    X, U = _to_cart(*start)
    gam = math.sqrt(1.0 + U @ U)
    omega = wq * B0 / gam
    alpha = 2.0 * math.atan(0.5 * omega * o.dt)    # discrete rotation per step
    nsteps = int(round(periods * 2.0 * math.pi / alpha))
    rl = math.hypot(U[0], U[1]) / (wq * B0)        # gyration radius
    err_x = err_u = 0.0
    for k in range(1, nsteps + 1):
        o.phases(oracle_lib.PHASE_PUSH)
        got = _state(o)[0]
        a = -alpha * k                             # positive charges turn clockwise about B
        c, s = math.cos(a), math.sin(a)
        Uk = np.array([c * U[0] - s * U[1], s * U[0] + c * U[1], U[2]])
        X = X + o.dt * Uk / gam
        exp = _to_local(X, Uk)
        err_x = max(err_x, abs(got[0] - exp[0]), exp[0] * abs(got[1] - exp[1]))
        err_u = max(err_u, float(np.abs(got[2:] - exp[2:]).max()))
    return err_x / rl, err_u / float(np.linalg.norm(U)), o.dth, nsteps


def test_gyration_in_uniform_Bz_from_nodal_psi(oracle_lib):
    x1, u1, dth1, n1 = _gyration_error(oracle_lib, 32)
    x2, u2, dth2, n2 = _gyration_error(oracle_lib, 64)
    assert n1 > 50 and n2 > n1
    # the field's interpolation error is O(dtheta^2); over a gyration it
    # shifts the phase by about 2 pi times that
    assert x1 < 10 * dth1 ** 2 and u1 < 10 * dth1 ** 2
    assert x1 / x2 > 2.5 and u1 / u2 > 2.5


# ---------------------------------------------------------------------------
# azimuthal E x B drift in E = E0 varpi-hat, B = B0 z

def test_azimuthal_exb_drift(oracle_lib):
    n = 64
    d = _desc(n)
    o = oracle_lib.Oracle(d)
    wq = d["omega_b"] * d["qm"][0]
    B0 = 5.0 / wq                    # omega_B (q/m) B0 = 5
    vd = 0.1                         # E0 / B0
    E0 = vd * B0
    _set_uniform_Bz(o, oracle_lib, B0)
    th_n = np.arange(n + 1) * o.dth
    th_h = (np.arange(n + 1) + 0.5) * o.dth
    # varpi-hat = sin(theta) r-hat + cos(theta) theta-hat
    o.set_field(oracle_lib.ER, np.broadcast_to(E0 * np.sin(th_n)[None, :], o.shape))
    o.set_field(oracle_lib.ETH, np.broadcast_to(E0 * np.cos(th_h)[None, :], o.shape))
    th0, w0 = 0.5 * math.pi - 0.4, 6.0
    r0 = w0 / math.sin(th0)
    # circular orbit at varpi0: wq (E0 + v B0) = -gamma v^2 / varpi0 (v along phi-hat);
    # for varpi0 -> infinity v -> -E0 / B0
    v = -vd
    for _ in range(50):
        g = 1.0 / math.sqrt(1.0 - v * v)
        v = -vd - g * v * v / (wq * B0 * w0)
    assert abs(v + vd) < 1e-2 * vd
    u0 = v / math.sqrt(1.0 - v * v)
    _load(o, [(r0, th0, 0.0, 0.0, u0)])
    z0 = r0 * math.cos(th0)
    T = 10.0
    nsteps = int(T / o.dt)
    vs, dw, dz = [], 0.0, 0.0
    for _ in range(nsteps):
        o.phases(oracle_lib.PHASE_PUSH)
        r, th, ur, uth, uph = _state(o)[0]
        vs.append(uph / math.sqrt(1.0 + ur * ur + uth * uth + uph * uph))
        dw = max(dw, abs(r * math.sin(th) - w0))
        dz = max(dz, abs(r * math.cos(th) - z0))
    vmean = float(np.mean(vs))
    assert abs(vmean - v) < 2e-3 * vd
    assert abs(vmean + vd) < 1e-2 * vd        # the E x B drift speed
    assert dw < 2e-3 * w0 and dz < 2e-3 * w0  # stays on its ring


# ---------------------------------------------------------------------------
# azimuthal deposit

def test_jphi_deposit_total_and_centroid(oracle_lib):
    n = 40
    d = _desc(n, weight=(0.37,))
    o = oracle_lib.Oracle(d)
    rng = np.random.default_rng(20240614)
    m = 60
    states = np.stack([np.exp(rng.uniform(6.0, 30.0, m) * o.dlog),
                       rng.uniform(3.0, n - 4.0, m) * o.dth,
                       rng.normal(size=m), rng.normal(size=m), 2.0 * rng.normal(size=m)], axis=1)
    states[0, 1] = 0.3 * o.dth                 # next to the north pole
    states[1, 1] = math.pi - 0.2 * o.dth       # next to the south pole
    _load(o, states)
    o.phases(oracle_lib.PHASE_PUSH)
    jph = o.field(oracle_lib.JPH)
    I, J = np.meshgrid(np.arange(n + 1.0), np.arange(n + 1.0), indexing="ij")
    Q = d["weight"][0]
    tot = xs = ys = 0.0
    for s in states:
        X0, U = _to_cart(*s)
        g = math.sqrt(1.0 + U @ U)
        X1 = X0 + o.dt * U / g
        v_phi = U[1] / g                       # at azimuth 0, phi-hat = y
        r1 = float(np.linalg.norm(X1))
        th1 = math.atan2(math.hypot(X1[0], X1[1]), X1[2])
        xi0, eta0 = _logical(o, s[0], s[1])
        xi1, eta1 = _logical(o, r1, th1)
        tot += Q * v_phi
        xs += Q * v_phi * 0.5 * (xi0 + xi1)
        ys += Q * v_phi * 0.5 * (eta0 + eta1)
    scale = Q * np.abs(states[:, 2:]).sum()
    assert abs(jph.sum() - tot) < 1e-12 * scale
    assert abs((jph * I).sum() - xs) < 1e-12 * scale * n
    assert abs((jph * J).sum() - ys) < 1e-12 * scale * n


def _ring_current_error(oracle_lib, n):
    d = _desc(n, weight=(0.5,))
    o = oracle_lib.Oracle(d)
    # rings spread over a band of cells, so that where each sits inside its
    # cell averages out
    rng = np.random.default_rng(5)
    m = 200
    states = np.stack([rng.uniform(4.0, 6.0, m), rng.uniform(0.8, 1.4, m),
                       0.05 * rng.normal(size=m), 0.05 * rng.normal(size=m),
                       rng.uniform(0.5, 2.0, m)], axis=1)
    _load(o, states)
    exp = 0.0
    for s in states:
        X0, U = _to_cart(*s)
        g = math.sqrt(1.0 + U @ U)
        X1 = X0 + o.dt * U / g
        xi0, eta0 = _logical(o, s[0], s[1])
        xi1, eta1 = _logical(o, float(np.linalg.norm(X1)),
                             math.atan2(math.hypot(X1[0], X1[1]), X1[2]))
        w_mid = d["rmin"] * math.exp(0.5 * (xi0 + xi1) * o.dlog) * \
            math.sin(0.5 * (eta0 + eta1) * o.dth)
        exp += d["weight"][0] * (U[1] / g) / w_mid   # ring current, 2 pi dropped
    o.phases(oracle_lib.PHASE_PUSH | oracle_lib.PHASE_FIELDS)
    eph = o.field(oracle_lib.EPH)
    # meridional area of the dual cell around each interior node
    r_half = d["rmin"] * np.exp((np.arange(n) + 0.5) * o.dlog)
    area = 0.5 * (r_half[1:] ** 2 - r_half[:-1] ** 2)[:, None] * o.dth
    # from zero fields, Ampere leaves E_phi = -4 pi dt J_phi
    current = -(eph[1:n, 1:n] * area).sum() / (4.0 * math.pi * o.dt)
    return abs(current - exp) / abs(exp), o.dth


def test_jphi_density_integrates_to_ring_current(oracle_lib):
    e1, dth1 = _ring_current_error(oracle_lib, 32)
    e2, dth2 = _ring_current_error(oracle_lib, 64)
    assert e1 < dth1 ** 2 and e2 < dth2 ** 2
    assert e1 / e2 > 3.0
