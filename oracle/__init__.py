"""ctypes wrapper of the plain FP64 CPU oracle (ffpic_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ffpic_oracle.c")
# A test may point this at another build of the oracle (the mutation test
# loads copies with one planted mistake); such a library is used as given.
LIB_OVERRIDE = os.environ.get("FFPIC_ORACLE_LIB", "")
LIB = LIB_OVERRIDE or os.path.join(HERE, "libffpic_oracle.so")
# The same source built with OpenMP: grid loops over rows, particle pushes
# over slot ranges with per-thread deposit rows added in thread order.  With
# one thread it is the single-thread oracle; with more it rounds the
# deposit's sums in another (fixed) order.  Used for timing only: the pins
# and parity tests use the single-thread build.
LIB_OMP = os.path.join(HERE, "libffpic_oracle_omp.so")

# field component numbering of the oracle (ffpic_oracle.h)
ER, ETH, EPH, BR, BTH, BPH, JR, JTH, JPH, PSI, F, B0R, B0TH, B0PH = range(14)
PHASE_MASK, PHASE_KILL, PHASE_SORT, PHASE_PUSH, PHASE_FIELDS, PHASE_INJECT = 1, 2, 4, 8, 16, 32
PHASE_EXTRACT, PHASE_PAIRS = 64, 128


def compile_to(src: str, out: str, openmp: bool = False) -> None:
    """Compile an oracle source file into a shared library with gcc (plain C,
    FP contraction off; with openmp, the OpenMP build)."""
    tmp = out + ".tmp"
    # sin and cos are called as written: with them as builtins GCC merges a
    # sin and a cos of one argument into one sincos call, whose results
    # differ from sin's and cos's in the last bit at some angles (theta_j =
    # 80 pi / 300 and 159 pi / 300, for example)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-fast-math",
                           "-fno-builtin-sin", "-fno-builtin-cos",
                           *(["-fopenmp"] if openmp else []), "-o", tmp, src, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP contraction off)."""
    if LIB_OVERRIDE:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    if force or not os.path.exists(LIB_OMP) or os.path.getmtime(LIB_OMP) < os.path.getmtime(SRC):
        compile_to(SRC, LIB_OMP, openmp=True)
    return LIB


class _Params(C.Structure):
    _fields_ = [("nr", C.c_int), ("nth", C.c_int),
                ("rmin", C.c_double), ("rmax", C.c_double), ("r_lc", C.c_double),
                ("r_abs", C.c_double), ("mu", C.c_double), ("cfl", C.c_double),
                ("omega_b", C.c_double), ("rr_coef", C.c_double),
                ("psi_thr", C.c_double * 4),
                ("ff_enable", C.c_int), ("init", C.c_int),
                ("sort_interval", C.c_int), ("nspec", C.c_int),
                ("qm", C.c_double * 4), ("weight", C.c_double * 4),
                ("inject_kappa", C.c_double), ("rng_seed", C.c_uint64),
                ("rr_ramp_n", C.c_int), ("rr_ramp_t", C.c_double * 4),
                ("rr_ramp_f", C.c_double * 4), ("shell_r", C.c_double),
                ("gj_extract", C.c_double), ("gj_species", C.c_int * 2),
                ("gamma_th", C.c_double), ("gamma_s", C.c_double),
                ("pair_species", C.c_int * 2)]


class _SpecReq(C.Structure):
    _fields_ = [("rmin", C.c_double), ("rmax", C.c_double), ("thmin", C.c_double),
                ("thmax", C.c_double), ("gmin", C.c_double), ("gmax", C.c_double),
                ("numin", C.c_double), ("numax", C.c_double),
                ("ngamma", C.c_int), ("nnu", C.c_int)]


_libs = {}


def lib(path: str = LIB):
    """The oracle library at path (the single-thread build by default)."""
    if path not in _libs:
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.ora_create.restype = P
        L.ora_create.argtypes = [C.POINTER(_Params)]
        L.ora_destroy.argtypes = [P]
        L.ora_info.argtypes = [P, dp]
        L.ora_get_field.argtypes = [P, C.c_int, dp]
        L.ora_geometry.argtypes = [P, C.c_int, dp]
        L.ora_set_field.argtypes = [P, C.c_int, dp]
        L.ora_load_particles.restype = C.c_int64
        L.ora_load_particles.argtypes = [P, C.c_int, C.c_int64, dp, dp, dp, dp, dp]
        L.ora_num_particles.restype = C.c_int64
        L.ora_num_particles.argtypes = [P, C.c_int]
        L.ora_get_particles.restype = C.c_int64
        L.ora_get_particles.argtypes = [P, C.c_int, dp, dp, dp, dp, dp,
                                        np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")]
        L.ora_step.argtypes = [P, C.c_int]
        L.ora_run_phases.argtypes = [P, C.c_int]
        L.ora_step_count.restype = C.c_int64
        L.ora_step_count.argtypes = [P]
        L.ora_set_step.argtypes = [P, C.c_int64]
        L.ora_removed.argtypes = [P, C.c_int, np.ctypeslib.ndpointer(np.int64)]
        L.ora_moments.argtypes = [P, C.c_int, dp]
        L.ora_gauss.argtypes = [P, dp]
        L.ora_divb.argtypes = [P, dp]
        L.ora_node_charge.argtypes = [P, dp]
        L.ora_poynting.argtypes = [P, dp]
        L.ora_sort_offsets.argtypes = [P, C.c_int,
                                       np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")]
        L.ora_boris_rr.argtypes = [dp, dp, dp, C.c_double, C.c_double, C.c_double]
        L.ora_ff_node.argtypes = [dp, dp, dp]
        L.ora_timestep.restype = C.c_double
        L.ora_timestep.argtypes = [C.POINTER(_Params)]
        L.ora_gather.argtypes = [P, C.c_double, C.c_double, dp, dp]
        L.ora_blend.restype = C.c_double
        L.ora_blend.argtypes = [C.c_double, dp]
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.ora_philox4x32.argtypes = [u32p, u32p, u32p]
        L.ora_inject_rate.restype = C.c_double
        L.ora_inject_rate.argtypes = [P, C.c_int]
        L.ora_gj_target.restype = C.c_double
        L.ora_gj_target.argtypes = [P, C.c_int]
        L.ora_spectra.argtypes = [P, C.c_int, C.POINTER(_SpecReq), dp, dp, dp]
        L.ora_synchrotron_F.restype = C.c_double
        L.ora_synchrotron_F.argtypes = [C.c_double]
        L.ora_rr_factor.restype = C.c_double
        L.ora_rr_factor.argtypes = [C.POINTER(_Params), C.c_double]
        L.ora_set_threads.argtypes = [C.c_int]
        L.ora_threads.restype = C.c_int
        _libs[path] = L
    return _libs[path]


def params(desc: dict) -> _Params:
    p = _Params()
    for k in ("nr", "nth", "ff_enable", "init", "sort_interval", "nspec"):
        setattr(p, k, int(desc[k]))
    for k in ("rmin", "rmax", "r_lc", "r_abs", "mu", "cfl", "omega_b", "rr_coef"):
        setattr(p, k, float(desc[k]))
    for k in range(4):
        p.psi_thr[k] = float(desc["psi_thr"][k])
    for k, (q, w) in enumerate(zip(desc["qm"], desc["weight"])):
        p.qm[k] = float(q)
        p.weight[k] = float(w)
    p.inject_kappa = float(desc.get("inject_kappa", 0.0))
    p.rng_seed = int(desc.get("rng_seed", 0))
    ramp = desc.get("rr_ramp", ())
    p.rr_ramp_n = len(ramp)
    for k, (t, f) in enumerate(ramp):
        p.rr_ramp_t[k] = float(t)
        p.rr_ramp_f[k] = float(f)
    p.shell_r = float(desc.get("shell_r", 0.0))
    p.gj_extract = float(desc.get("gj_extract", 0.0))
    p.gamma_th = float(desc.get("gamma_th", 0.0))
    p.gamma_s = float(desc.get("gamma_s", 0.0))
    for k in range(2):
        p.gj_species[k] = int(desc.get("gj_species", (0, 0))[k])
        p.pair_species[k] = int(desc.get("pair_species", (0, 0))[k])
    return p


def philox4x32(ctr, key) -> np.ndarray:
    """Philox4x32-10 output words for a counter (4 words) and key (2 words)."""
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32(np.ascontiguousarray(ctr, dtype=np.uint32),
                         np.ascontiguousarray(key, dtype=np.uint32), out)
    return out


class Oracle:
    """One simulated magnetosphere held by the CPU oracle.  threads=None uses
    the single-thread build; an integer uses the OpenMP build with that many
    threads (for timing)."""

    def __init__(self, desc: dict, threads=None):
        self.desc = dict(desc)
        self.nr, self.nth = int(desc["nr"]), int(desc["nth"])
        self._p = params(desc)
        self._L = lib() if threads is None else lib(LIB_OMP)
        if threads is not None:
            self._L.ora_set_threads(int(threads))
        self._h = self._L.ora_create(C.byref(self._p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        info = np.zeros(4)
        self._L.ora_info(self._h, info)
        self.dt, self.dlog, self.dth, self.omega = (float(x) for x in info)

    def close(self):
        if self._h:
            self._L.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.nr + 1, self.nth + 1)

    def field(self, comp: int) -> np.ndarray:
        out = np.zeros(self.shape)
        self._L.ora_get_field(self._h, comp, out)
        return out

    def geometry(self, which: int) -> np.ndarray:
        """0 r_i, 1 r_{i+1/2}, 2 theta_j, 3 sin theta_j, 4 cos theta_j,
        5 sin theta_{j+1/2}, 6 cos theta_{j+1/2}"""
        n = [self.nr + 1, self.nr, self.nth + 1, self.nth + 1, self.nth + 1,
             self.nth, self.nth][which]
        out = np.zeros(n)
        self._L.ora_geometry(self._h, int(which), out)
        return out

    def set_field(self, comp: int, arr: np.ndarray):
        self._L.ora_set_field(self._h, comp, np.ascontiguousarray(arr, dtype=np.float64))

    def load(self, sp: int, d: dict) -> int:
        a = [np.ascontiguousarray(d[k], dtype=np.float64) for k in ("r", "th", "ur", "uth", "uph")]
        return int(self._L.ora_load_particles(self._h, sp, len(a[0]), *a))

    def n(self, sp: int) -> int:
        return int(self._L.ora_num_particles(self._h, sp))

    def particles(self, sp: int) -> dict:
        n = self.n(sp)
        out = {k: np.zeros(n) for k in ("r", "th", "ur", "uth", "uph")}
        cell = np.zeros(n, dtype=np.int32)
        self._L.ora_get_particles(self._h, sp, out["r"], out["th"], out["ur"],
                                out["uth"], out["uph"], cell)
        out["cell"] = cell
        return out

    def step(self, n: int = 1):
        self._L.ora_step(self._h, int(n))

    def phases(self, mask: int):
        self._L.ora_run_phases(self._h, int(mask))

    def step_count(self) -> int:
        return int(self._L.ora_step_count(self._h))

    def set_step(self, n: int):
        self._L.ora_set_step(self._h, int(n))

    def removed(self, sp: int) -> np.ndarray:
        out = np.zeros(4, dtype=np.int64)
        self._L.ora_removed(self._h, sp, out)
        return out

    def moments(self, sp: int) -> np.ndarray:
        out = np.zeros(5)
        self._L.ora_moments(self._h, sp, out)
        return out

    def gauss(self) -> np.ndarray:
        out = np.zeros(self.shape)
        self._L.ora_gauss(self._h, out)
        return out

    def divb(self) -> np.ndarray:
        out = np.zeros(self.shape)
        self._L.ora_divb(self._h, out)
        return out

    def node_charge(self) -> np.ndarray:
        out = np.zeros(self.shape)
        self._L.ora_node_charge(self._h, out)
        return out

    def poynting(self) -> np.ndarray:
        out = np.zeros(self.nr + 1)
        self._L.ora_poynting(self._h, out)
        return out

    def inject_rate(self, j: int) -> float:
        return float(self._L.ora_inject_rate(self._h, int(j)))

    def spectra(self, sp: int, req: dict) -> dict:
        """gamma histogram dN, radiated power prad and synchrotron SED of one
        species over a region; req keys as in spec_request()."""
        q = spec_request(req)
        dN, sed, prad = np.zeros(q.ngamma), np.zeros(q.nnu), np.zeros(1)
        self._L.ora_spectra(self._h, int(sp), C.byref(q), dN, sed, prad)
        return {"dN": dN, "sed": sed, "prad": float(prad[0])}

    def gj_target(self, j: int) -> float:
        return float(self._L.ora_gj_target(self._h, int(j)))

    def gather(self, r: float, th: float):
        E = np.zeros(3)
        B = np.zeros(3)
        self._L.ora_gather(self._h, float(r), float(th), E, B)
        return E, B

    def sort_offsets(self, sp: int) -> np.ndarray:
        out = np.zeros(self.nr * self.nth + 1, dtype=np.int32)
        self._L.ora_sort_offsets(self._h, sp, out)
        return out


def timestep(desc: dict) -> float:
    p = params(desc)
    return float(lib().ora_timestep(C.byref(p)))


def boris_rr(u, E, B, dt, wq, rr=0.0):
    uu = np.array(u, dtype=np.float64)
    lib().ora_boris_rr(uu, np.asarray(E, dtype=np.float64), np.asarray(B, dtype=np.float64),
                       float(dt), float(wq), float(rr))
    return uu


def spec_request(req: dict) -> _SpecReq:
    q = _SpecReq()
    for k in ("rmin", "rmax", "thmin", "thmax", "gmin", "gmax", "numin", "numax"):
        setattr(q, k, float(req[k]))
    q.ngamma, q.nnu = int(req["ngamma"]), int(req["nnu"])
    return q


def synchrotron_F(x: float) -> float:
    return float(lib().ora_synchrotron_F(float(x)))


def rr_factor(desc: dict, t: float) -> float:
    p = params(desc)
    return float(lib().ora_rr_factor(C.byref(p), float(t)))


def ff_node(E, B):
    out = np.zeros(3)
    lib().ora_ff_node(np.asarray(E, dtype=np.float64), np.asarray(B, dtype=np.float64), out)
    return out


def blend(psi, thr):
    return float(lib().ora_blend(float(psi), np.asarray(thr, dtype=np.float64)))
