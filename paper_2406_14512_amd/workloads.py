"""Seeded synthetic magnetosphere workloads.

This module only chooses parameters and draws random particles.  It holds
none of the step's arithmetic (no grid tables, no field formulas, no push),
so both the GPU library and the CPU oracle can be fed from it.

Normalisation (code units): c = 1, stellar radius r_star = 1, magnetic moment
mu = 1, Omega = 1 / R_LC (Sect. 2, light-cylinder radius R_LC = cP/2pi).

* Lorentz coupling omega_B: the polar-cap Lorentz factor of Sect. 2
  (gamma_pc = e Phi_pc / m_e c^2 with Phi_pc = mu Omega^2 / c^2) reads
  gamma_pc = omega_B * mu * Omega^2 in these units, so
  omega_B = gamma_pc * R_LC^2.  We take gamma_pc = 1000.
* Radiation-reaction coefficient K_e: the radiation-limited Lorentz factor of
  Sect. 2 (force balance E ~ gamma_rad^2 B_perp^2 at E = B_perp = B_LC)
  gives K_e = omega_B / (gamma_rad_LC^2 * B_LC), B_LC = mu / R_LC^3.
  We take gamma_rad_LC = 30 when radiation reaction is on.
* Macro-particle weight: the loaded peak density of each species is kappa
  times the Goldreich-Julian charge density at the light cylinder,
  Omega B_LC / 2pi (Sect. 2), with kappa = 10 (the injection multiplicity of
  Sect. 4).  Volumes are per radian of azimuth.

Random numbers come from numpy's PCG64 with explicit seeds
(240614512 + workload index), drawn in fixed-size chunks whose seeds are
derived from (seed, species, chunk) so that any prefix of a large workload
can be regenerated on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Iterator, List, Optional

import numpy as np

SEED_BASE = 240614512
GAMMA_PC = 1000.0
GAMMA_RAD_LC = 30.0
KAPPA = 10.0
CHUNK = 1 << 22  # particles per generator chunk

# init kinds (same numbering as the library and the oracle use)
INIT_ZERO, INIT_DIPOLE, INIT_MONOPOLE, INIT_MICHEL, INIT_OPEN_DIPOLE = 0, 1, 2, 3, 4
FP64, FP32_MIXED = 0, 1
INF = float("inf")


@dataclasses.dataclass
class Workload:
    name: str
    nr: int
    nth: int
    rmin: float
    rmax: float
    r_lc: float
    r_abs: float
    mu: float = 1.0
    cfl: float = 0.5
    omega_b: float = 0.0
    rr_coef: float = 0.0
    psi_thr: tuple = (-INF, -INF, INF, INF)
    ff_enable: int = 0
    init: int = INIT_DIPOLE
    precision: int = FP64
    sort_interval: int = 1
    qm: tuple = (-1.0, 1.0)
    weight: tuple = (0.0, 0.0)
    inject_kappa: float = 0.0   # surface pair injection multiplicity (0 = off)
    rng_seed: int = 0
    # plasma sources of the dipole
    rr_ramp: tuple = ()         # ((t, factor), ...) knots of the radiation-reaction ramp
    shell_r: float = 0.0        # transverse momentum removed below this radius
    gj_extract: float = 0.0     # Goldreich-Julian extraction multiplicity (0 = off)
    gj_species: tuple = (0, 0)  # extracted electron and ion species
    gamma_th: float = 0.0       # pair-creation threshold (0 = off)
    gamma_s: float = 0.0        # Lorentz factor of the created pairs
    pair_species: tuple = (0, 0)  # electron and positron species
    # particle recipe
    n_per_species: int = 0
    kind: str = "none"          # "uniform_band", "sheet", "none"
    band: float = 0.2           # half-width of the uniform band in theta
    sheet_width: float = 0.05   # sech^2 width in theta
    sheet_rmin: float = 0.0
    sheet_rmax: float = 0.0
    drift_beta: float = 0.0
    gamma_max: float = 100.0
    background_frac: float = 0.0
    background_rmin: float = 3.0
    seed: int = SEED_BASE
    steps: int = 1

    @property
    def nspec(self) -> int:
        return len(self.qm)

    def desc(self) -> Dict:
        """Descriptor fields shared by the library and the oracle."""
        return dict(nr=self.nr, nth=self.nth, rmin=self.rmin, rmax=self.rmax,
                    r_lc=self.r_lc, r_abs=self.r_abs, mu=self.mu, cfl=self.cfl,
                    omega_b=self.omega_b, rr_coef=self.rr_coef,
                    psi_thr=tuple(self.psi_thr), ff_enable=self.ff_enable,
                    init=self.init, precision=self.precision,
                    sort_interval=self.sort_interval, nspec=self.nspec,
                    qm=tuple(self.qm), weight=tuple(self.weight),
                    inject_kappa=self.inject_kappa, rng_seed=self.rng_seed,
                    rr_ramp=tuple(tuple(k) for k in self.rr_ramp), shell_r=self.shell_r,
                    gj_extract=self.gj_extract, gj_species=tuple(self.gj_species),
                    gamma_th=self.gamma_th, gamma_s=self.gamma_s,
                    pair_species=tuple(self.pair_species))

    # -- particles ---------------------------------------------------------
    def n_chunks(self) -> int:
        return (self.n_per_species + CHUNK - 1) // CHUNK

    def chunk(self, species: int, index: int) -> Dict[str, np.ndarray]:
        """Chunk `index` of species `species`: dict r, th, ur, uth, uph."""
        n0 = index * CHUNK
        n = min(CHUNK, self.n_per_species - n0)
        if n <= 0:
            z = np.zeros(0)
            return dict(r=z, th=z, ur=z, uth=z, uph=z)
        ss = np.random.SeedSequence(self.seed, spawn_key=(species, index))
        g = np.random.Generator(np.random.PCG64(ss))
        if self.kind == "uniform_band":
            return _uniform_band(g, n, self, species)
        if self.kind == "sheet":
            return _sheet(g, n, self, species)
        raise ValueError(f"workload {self.name} has no particles")

    def particles(self, species: int, limit: Optional[int] = None) -> Dict[str, np.ndarray]:
        """All particles of a species (or the first `limit`), concatenated."""
        n = self.n_per_species if limit is None else min(limit, self.n_per_species)
        parts: List[Dict[str, np.ndarray]] = []
        got = 0
        for c in range(self.n_chunks()):
            if got >= n:
                break
            d = self.chunk(species, c)
            take = min(n - got, len(d["r"]))
            parts.append({k: v[:take] for k, v in d.items()})
            got += take
        if not parts:
            z = np.zeros(0)
            return dict(r=z, th=z, ur=z, uth=z, uph=z)
        return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}

    def iter_chunks(self, species: int) -> Iterator[Dict[str, np.ndarray]]:
        for c in range(self.n_chunks()):
            yield self.chunk(species, c)


def _isotropic(g, n, gamma_max):
    gam = np.exp(g.uniform(0.0, math.log(gamma_max), n))
    umag = np.sqrt(gam * gam - 1.0)
    mu = g.uniform(-1.0, 1.0, n)
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(1.0 - mu * mu)
    return umag * mu, umag * st * np.cos(ph), umag * st * np.sin(ph)


def _uniform_band(g, n, w: Workload, species):
    a3, b3 = w.sheet_rmin ** 3, w.sheet_rmax ** 3
    r = np.cbrt(g.uniform(a3, b3, n))
    s = math.sin(w.band)
    th = np.arccos(g.uniform(-s, s, n))
    ur, uth, uph = _isotropic(g, n, w.gamma_max)
    return dict(r=r, th=th, ur=ur, uth=uth, uph=uph)


def _sheet(g, n, w: Workload, species):
    nb = int(round(n * w.background_frac))
    ns = n - nb
    a3, b3 = w.sheet_rmin ** 3, w.sheet_rmax ** 3
    r = np.cbrt(g.uniform(a3, b3, ns))
    t = min(math.tanh(math.pi / (2.0 * w.sheet_width)), 1.0 - 1e-15)
    th = 0.5 * math.pi + w.sheet_width * np.arctanh(g.uniform(-t, t, ns))
    sign = 1.0 if w.qm[species] > 0 else -1.0
    u_d = w.drift_beta / math.sqrt(1.0 - w.drift_beta ** 2)
    uph = np.full(ns, sign * u_d)
    ur = np.zeros(ns)
    uth = np.zeros(ns)
    if nb:
        # closed-zone background: volume-uniform where sin^2(th) > r / R_LC,
        # at rest, from r = background_rmin out (inside ~3 stellar radii the
        # radiation-reaction rate K B^2 exceeds 1/dt by orders of magnitude,
        # where the explicit radiation-reaction step is unstable)
        rb = np.empty(0)
        tb = np.empty(0)
        while len(rb) < nb:
            m = 2 * (nb - len(rb)) + 64
            rr = np.cbrt(g.uniform(w.background_rmin ** 3, w.r_lc ** 3, m))
            cc = g.uniform(-1.0, 1.0, m)
            ok = (1.0 - cc * cc) > rr / w.r_lc
            rb = np.concatenate([rb, rr[ok]])
            tb = np.concatenate([tb, np.arccos(cc[ok])])
        r = np.concatenate([r, rb[:nb]])
        th = np.concatenate([th, tb[:nb]])
        ur = np.concatenate([ur, np.zeros(nb)])
        uth = np.concatenate([uth, np.zeros(nb)])
        uph = np.concatenate([uph, np.zeros(nb)])
    return dict(r=r, th=th, ur=ur, uth=uth, uph=uph)


def _units(r_lc, rr_on, n_peak):
    omega = 1.0 / r_lc
    b_lc = 1.0 / r_lc ** 3
    omega_b = GAMMA_PC * r_lc ** 2
    rr = omega_b / (GAMMA_RAD_LC ** 2 * b_lc) if rr_on else 0.0
    weight = KAPPA * omega * b_lc / (2.0 * math.pi * n_peak) if n_peak > 0 else 0.0
    return omega_b, rr, weight


# ---------------------------------------------------------------------------
# the workloads

def tiny_dipole(n_per_species: int = 100_000, steps: int = 20) -> Workload:
    """128^2, r in [1,10], R_LC = 3; static dipole + corotation, pure PIC,
    e+- uniform in volume in |theta - pi/2| < 0.2 with r in (3, 9),
    isotropic momenta with gamma log-uniform in [1,100], no radiation
    reaction, 20 steps at CFL 0.5, FP64."""
    r_lc = 3.0
    a, b = r_lc, 3.0 * r_lc
    vol = (b ** 3 - a ** 3) / 3.0 * 2.0 * math.sin(0.2)
    omega_b, _, wgt = _units(r_lc, False, n_per_species / vol)
    return Workload(name="dipole_128", nr=128, nth=128, rmin=1.0, rmax=10.0,
                    r_lc=r_lc, r_abs=3.0 * r_lc, omega_b=omega_b, rr_coef=0.0,
                    init=INIT_DIPOLE, ff_enable=0,
                    weight=(wgt, wgt), n_per_species=n_per_species,
                    kind="uniform_band", band=0.2, sheet_rmin=a, sheet_rmax=b,
                    gamma_max=100.0, seed=SEED_BASE + 1, steps=steps,
                    sort_interval=1)


def tiny_open_dipole(n_per_species: int = 100_000, steps: int = 20) -> Workload:
    """The 128^2 grid with the open-dipole field and a sharp force-free
    domain on open field lines below 0.85 Psi_pc: exercises the mask, the
    particle kill, the force-free current and the E correction."""
    w = tiny_dipole(n_per_species, steps)
    w.name = "open_dipole_128"
    w.init = INIT_OPEN_DIPOLE
    psi_pc = w.mu / w.r_lc
    w.psi_thr = (0.85 * psi_pc, 0.85 * psi_pc, INF, INF)
    w.ff_enable = 1
    return w


def sheet_1024(n_total: int = 20_000_000, steps: int = 1000,
               precision: int = FP64) -> Workload:
    """1024^2, r in [1,30], R_LC = 5; e+- in a sech^2 sheet of width 0.05
    beyond R_LC drifting at +-0.5c in phi; open dipole with the force-free
    domain on open lines below 0.85 Psi_pc; radiation reaction on."""
    r_lc = 5.0
    nps = n_total // 2
    a, b = r_lc, 3.0 * r_lc
    width = 0.05
    n_peak = 3.0 * nps / (2.0 * width * (b ** 3 - a ** 3))
    omega_b, rr, wgt = _units(r_lc, True, n_peak)
    psi_pc = 1.0 / r_lc
    return Workload(name="sheet_1024", nr=1024, nth=1024, rmin=1.0, rmax=30.0,
                    r_lc=r_lc, r_abs=3.0 * r_lc, omega_b=omega_b, rr_coef=rr,
                    psi_thr=(0.85 * psi_pc, 0.85 * psi_pc, INF, INF),
                    ff_enable=1, init=INIT_OPEN_DIPOLE, precision=precision,
                    weight=(wgt, wgt), n_per_species=nps, kind="sheet",
                    sheet_width=width, sheet_rmin=a, sheet_rmax=b,
                    drift_beta=0.5, seed=SEED_BASE + 2, steps=steps,
                    sort_interval=8)


def sheet_4096(n_total: int = 400_000_000, steps: int = 500,
               precision: int = FP32_MIXED) -> Workload:
    """4096^2, r in [1,100], R_LC = 10; 99% of e+- in a sech^2 sheet of width
    0.02 beyond R_LC (drifting at +-0.5c), 1% at rest in the closed zone;
    radiation reaction on; sort every 8 steps."""
    r_lc = 10.0
    nps = n_total // 2
    a, b = r_lc, 3.0 * r_lc
    width = 0.02
    n_peak = 3.0 * (0.99 * nps) / (2.0 * width * (b ** 3 - a ** 3))
    omega_b, rr, wgt = _units(r_lc, True, n_peak)
    psi_pc = 1.0 / r_lc
    return Workload(name="sheet_4096", nr=4096, nth=4096, rmin=1.0, rmax=100.0,
                    r_lc=r_lc, r_abs=3.0 * r_lc, omega_b=omega_b, rr_coef=rr,
                    psi_thr=(0.85 * psi_pc, 0.85 * psi_pc, INF, INF),
                    ff_enable=1, init=INIT_OPEN_DIPOLE, precision=precision,
                    weight=(wgt, wgt), n_per_species=nps, kind="sheet",
                    sheet_width=width, sheet_rmin=a, sheet_rmax=b,
                    drift_beta=0.5, background_frac=0.01,
                    seed=SEED_BASE + 4, steps=steps, sort_interval=8)


def batched_systems(n_systems: int = 64, scale: float = 1.0,
                    steps: int = 200) -> List[Workload]:
    """Independent magnetospheres: grid N^2 with N drawn from
    {256, 512, 768, 1024}, r_max = 6 R_LC, R_LC uniform in [2, 8], particle
    counts log-uniform in [1e6, 1e7] (times `scale`) in sech^2 sheets of
    width 0.05, FP32-mixed."""
    g = np.random.Generator(np.random.PCG64(SEED_BASE + 5))
    out = []
    for k in range(n_systems):
        n = int(g.choice([256, 512, 768, 1024]))
        r_lc = float(g.uniform(2.0, 8.0))
        npart = int(round(math.exp(g.uniform(math.log(1e6), math.log(1e7))) * scale))
        nps = max(npart // 2, 1)
        a, b = r_lc, 3.0 * r_lc
        width = 0.05
        n_peak = 3.0 * nps / (2.0 * width * (b ** 3 - a ** 3))
        omega_b, rr, wgt = _units(r_lc, True, n_peak)
        psi_pc = 1.0 / r_lc
        out.append(Workload(name=f"batch_{k}", nr=n, nth=n, rmin=1.0,
                            rmax=6.0 * r_lc, r_lc=r_lc, r_abs=3.0 * r_lc,
                            omega_b=omega_b, rr_coef=rr,
                            psi_thr=(0.85 * psi_pc, 0.85 * psi_pc, INF, INF),
                            ff_enable=1, init=INIT_OPEN_DIPOLE,
                            precision=FP32_MIXED, weight=(wgt, wgt),
                            n_per_species=nps, kind="sheet", sheet_width=width,
                            sheet_rmin=a, sheet_rmax=b, drift_beta=0.5,
                            seed=SEED_BASE + 5 + 1000 * (k + 1), steps=steps,
                            sort_interval=8))
    return out


def michel_monopole(n: int = 128, pure_ff: bool = True, init: int = INIT_MICHEL,
                    r_lc: float = 5.0) -> Workload:
    """Monopole test of Sect. 4: r in [1, (10/3) R_LC], R_LC = 5, Psi_star = 1,
    absorbing layer from 3 R_LC.  With pure_ff the whole domain is force-free
    (f = 1 everywhere); otherwise the southern hemisphere is force-free and the
    northern one PIC (sharp boundary at Psi = Psi_star)."""
    thr = (INF, INF, INF, INF) if pure_ff else (-INF, -INF, 1.0, 1.0)
    return Workload(name=f"monopole_{n}", nr=n, nth=n, rmin=1.0,
                    rmax=10.0 / 3.0 * r_lc, r_lc=r_lc, r_abs=3.0 * r_lc,
                    mu=1.0, omega_b=GAMMA_PC * r_lc ** 2, psi_thr=thr,
                    ff_enable=1, init=init, n_per_species=0, kind="none",
                    seed=SEED_BASE + 6, steps=1)


def hybrid_monopole(n: int = 128, kappa: float = 10.0, r_lc: float = 5.0,
                    precision: int = FP64) -> Workload:
    """The hybrid monopole of Sect. 4: r in [1, (10/3) R_LC], R_LC = 5, a
    vacuum split-free monopole B = Psi_star / r^2 with corotation, the
    northern hemisphere PIC and the southern one force-free (sharp boundary
    at Psi = Psi_star), e+- pairs injected at the surface of the PIC
    hemisphere with multiplicity kappa_inj.  The macro-particle weight is
    chosen so that about one pair per surface cell is injected per step at
    the equator.

    The sharp cut sits half a cell south of the equator, at
    Psi_star (1 + sin(dtheta / 2)): the equatorial nodes, where the discrete
    flux function equals Psi_star up to rounding, stay on the PIC side by a
    margin of sin(dtheta / 2) instead of being decided by the last bit."""
    rmax = 10.0 / 3.0 * r_lc
    cut = 1.0 * (1.0 + math.sin(0.5 * math.pi / n))
    dr0 = math.log(rmax) / n          # first radial spacing in units of r_star
    dt_est = 0.5 * dr0 / math.sqrt(2.0)
    omega = 1.0 / r_lc
    weight = kappa * omega / (2.0 * n) * dt_est
    return Workload(name=f"hybrid_monopole_{n}", nr=n, nth=n, rmin=1.0, rmax=rmax,
                    r_lc=r_lc, r_abs=3.0 * r_lc, mu=1.0,
                    omega_b=GAMMA_PC * r_lc ** 2, rr_coef=0.0,
                    psi_thr=(-INF, -INF, cut, cut), ff_enable=1, init=INIT_MONOPOLE,
                    precision=precision, sort_interval=8, weight=(weight, weight),
                    inject_kappa=kappa, rng_seed=SEED_BASE + 7, n_per_species=0,
                    kind="none", seed=SEED_BASE + 7, steps=100)


def sourced_dipole(n: int = 64, precision: int = FP64, gamma_th: float = 30.0,
                   gamma_s: float = 5.0, n_per_species: int = 2000) -> Workload:
    """The aligned dipole of Sect. 5 with its plasma sources, scaled down:
    r in [1, 10], R_LC = 3, static dipole + corotation, force-free below
    0.85 Psi_pc and above 2.4 Psi_pc with the linear layers of Table 1;
    species electrons, positrons and protons (m_p = 1836 m_e); electrons and
    protons extracted at the surface to the Goldreich-Julian density every
    step; pairs created by leptons above gamma_th with gamma_s; transverse
    momentum removed within one stellar radius of the surface; the
    radiation-reaction force at 1% for one period, raised to 10% by 1.5
    periods and to its nominal strength at 2 periods.  The macro-particle
    weight puts about two extracted pairs in a surface cell at 45 degrees.
    gamma_pc = 1000 here, so the paper's gamma_th / gamma_pc (about 4e-3)
    would fall below gamma_s = 1.  The run starts from the corotating
    dipole, where E.B = 0 and nothing is accelerated for hundreds of steps;
    a band of energetic particles (every species, isotropic, gamma
    log-uniform in [1, 100], |theta - pi/2| < 0.3, r in (1.5, 3)) is loaded
    so that parents above gamma_th exist from the first step."""
    r_lc = 3.0
    omega_b, rr, _ = _units(r_lc, True, 0.0)
    psi_pc = 1.0 / r_lc
    dlog = math.log(10.0) / n
    dth = math.pi / n
    th = math.pi / 4
    t_45 = (1.0 / r_lc) / (2.0 * math.pi) * abs(math.sin(th + dth) ** 2 - math.sin(th) ** 2) * \
        (math.exp(3.0 * dlog) - 1.0) / 3.0
    w = t_45 / 4.0
    period = 2.0 * math.pi * r_lc
    return Workload(name=f"sourced_dipole_{n}", nr=n, nth=n, rmin=1.0, rmax=10.0,
                    r_lc=r_lc, r_abs=3.0 * r_lc, omega_b=omega_b, rr_coef=rr,
                    psi_thr=(0.85 * psi_pc, 0.9 * psi_pc, 2.3 * psi_pc, 2.4 * psi_pc),
                    ff_enable=1, init=INIT_DIPOLE, precision=precision, sort_interval=4,
                    qm=(-1.0, 1.0, 1.0 / 1836.0), weight=(w, w, w),
                    rng_seed=SEED_BASE + 9,
                    rr_ramp=((0.0, 0.01), (period, 0.01), (1.5 * period, 0.1),
                             (2.0 * period, 1.0)),
                    shell_r=2.0, gj_extract=1.0, gj_species=(0, 2),
                    gamma_th=gamma_th, gamma_s=gamma_s, pair_species=(0, 1),
                    n_per_species=n_per_species, kind="uniform_band", band=0.3,
                    sheet_rmin=1.5, sheet_rmax=3.0, gamma_max=100.0,
                    seed=SEED_BASE + 9, steps=40)
