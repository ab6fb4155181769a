"""Thin Python binding of the C ABI in include/ffpic.h (argument marshalling
only: every step of the path runs in the HIP kernels of libffpic.so).

Arrays may be numpy arrays (host memory) or torch tensors on the GPU
(device memory, passed by pointer).  There is no CPU fallback: if the
library is not built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffpic.so")

OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_MIXED = 0, 1
INIT_ZERO, INIT_DIPOLE, INIT_MONOPOLE, INIT_MICHEL, INIT_OPEN_DIPOLE = range(5)
(ER, ETH, EPH, BR, BTH, BPH, JR, JTH, JPH, PSI, F, GAUSS, DIVB) = range(13)
PHASE_MASK, PHASE_KILL, PHASE_SORT, PHASE_PUSH, PHASE_FIELDS, PHASE_INJECT = 1, 2, 4, 8, 16, 32
PHASE_EXTRACT, PHASE_PAIRS = 64, 128
DIAG_MOMENTS, DIAG_ENERGY, DIAG_RESIDUALS, DIAG_POYNTING, DIAG_ALL = 1, 2, 4, 8, 15
ERR_NONFINITE, ERR_CFL, ERR_CAPACITY = 1, 2, 4
MAX_SPECIES = 4


class FfpicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ffpic error {code}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nth", C.c_int32),
                ("rmin", C.c_double), ("rmax", C.c_double), ("r_lc", C.c_double),
                ("r_abs", C.c_double), ("mu", C.c_double), ("cfl", C.c_double),
                ("omega_b", C.c_double), ("rr_coef", C.c_double),
                ("psi_thr", C.c_double * 4),
                ("ff_enable", C.c_int32), ("precision", C.c_int32), ("init", C.c_int32),
                ("sort_interval", C.c_int32), ("nspec", C.c_int32), ("pad_", C.c_int32),
                ("capacity", C.c_int64 * MAX_SPECIES),
                ("qm", C.c_double * MAX_SPECIES), ("weight", C.c_double * MAX_SPECIES),
                ("inject_kappa", C.c_double), ("rng_seed", C.c_uint64),
                ("rr_ramp_n", C.c_int32), ("pad2_", C.c_int32),
                ("rr_ramp_t", C.c_double * 4), ("rr_ramp_f", C.c_double * 4),
                ("shell_r", C.c_double), ("gj_extract", C.c_double),
                ("gj_species", C.c_int32 * 2), ("gamma_th", C.c_double),
                ("gamma_s", C.c_double), ("pair_species", C.c_int32 * 2)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("alive", C.c_int64 * MAX_SPECIES),
                ("removed", (C.c_int64 * 4) * MAX_SPECIES),
                ("sum_gamma", C.c_double * MAX_SPECIES),
                ("sum_u", (C.c_double * 3) * MAX_SPECIES),
                ("energy_e", C.c_double), ("energy_b", C.c_double),
                ("gauss_max", C.c_double), ("divb_max", C.c_double),
                ("error_word", C.c_uint32), ("pad_", C.c_uint32)]


SPEC_MAX = 256


class SpectraReq(C.Structure):
    _fields_ = [("rmin", C.c_double), ("rmax", C.c_double), ("thmin", C.c_double),
                ("thmax", C.c_double), ("gmin", C.c_double), ("gmax", C.c_double),
                ("numin", C.c_double), ("numax", C.c_double),
                ("ngamma", C.c_int32), ("nnu", C.c_int32)]


TUNE_MAX = 16


class Tuning(C.Structure):
    _fields_ = [("sort_interval", C.c_int32), ("field_rows", C.c_int32),
                ("push_ppt", C.c_int32), ("ncand", C.c_int32),
                ("cand_kind", C.c_int32 * TUNE_MAX), ("cand", C.c_int32 * TUNE_MAX),
                ("ms_per_step", C.c_double * TUNE_MAX), ("total_ms", C.c_double)]

    KINDS = ("sort_interval", "field_rows", "push_ppt")

    def as_dict(self) -> Dict:
        n = self.ncand
        timed = {k: {} for k in self.KINDS}
        for k in range(n):
            timed[self.KINDS[self.cand_kind[k]]][int(self.cand[k])] = float(self.ms_per_step[k])
        return {"sort_interval": self.sort_interval, "field_rows": self.field_rows,
                "push_ppt": self.push_ppt, "ms_per_step": timed["sort_interval"],
                "timed": timed, "total_ms": float(self.total_ms)}


_lib = None


def lib():
    """Load libffpic.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python paper_2406_14512_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    vp = C.c_void_p
    L.ffpic_create.argtypes = [C.POINTER(Desc), vp, C.POINTER(P)]
    L.ffpic_destroy.argtypes = [P]
    L.ffpic_destroy.restype = None
    L.ffpic_last_error.argtypes = [P]
    L.ffpic_last_error.restype = C.c_char_p
    L.ffpic_info.argtypes = [P, C.POINTER(C.c_double)]
    L.ffpic_load_fields.argtypes = [P, C.c_int, vp, C.c_int]
    L.ffpic_load_particles.argtypes = [P, C.c_int, C.c_int64, vp, vp, vp, vp, vp, C.c_int]
    L.ffpic_step.argtypes = [P, C.c_int32]
    L.ffpic_run_phases.argtypes = [P, C.c_uint32]
    L.ffpic_sync.argtypes = [P]
    L.ffpic_get_field.argtypes = [P, C.c_int, vp, C.c_int]
    L.ffpic_num_particles.argtypes = [P, C.c_int, C.POINTER(C.c_int64)]
    L.ffpic_get_particles.argtypes = [P, C.c_int, vp, vp, vp, vp, vp, vp]
    L.ffpic_get_particles_range.argtypes = [P, C.c_int, C.c_int64, C.POINTER(C.c_int64),
                                            vp, vp, vp, vp, vp, vp]
    L.ffpic_get_sort.argtypes = [P, C.c_int, vp, vp, C.POINTER(C.c_int64)]
    L.ffpic_record_sort.argtypes = [P, C.c_int]
    L.ffpic_set_graph.argtypes = [P, C.c_int]
    L.ffpic_batch_set_graph.argtypes = [P, C.c_int]
    L.ffpic_batch_graph_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ffpic_batch_grouped_launches.argtypes = [P, C.POINTER(C.c_int64)]
    L.ffpic_batch_get_graph.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double)]
    L.ffpic_batch_set_grouped_chunk.argtypes = [P, C.c_int32]
    L.ffpic_graph_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.ffpic_diagnostics.argtypes = [P, C.c_uint32, C.POINTER(Diag), vp]
    L.ffpic_diagnostics_noalloc.argtypes = [P, C.c_uint32, C.POINTER(Diag), vp]
    dptr = C.POINTER(C.c_double)
    L.ffpic_spectra.argtypes = [P, C.c_int, C.POINTER(SpectraReq), dptr, dptr, dptr]
    L.ffpic_save.argtypes = [P, vp, C.POINTER(C.c_size_t)]
    L.ffpic_restore.argtypes = [P, vp, C.c_size_t]
    L.ffpic_set_timing.argtypes = [P, C.c_int]
    L.ffpic_set_field_rows.argtypes = [P, C.c_int32]
    L.ffpic_set_push_chunk.argtypes = [P, C.c_int32]
    L.ffpic_phase_times.argtypes = [P, C.POINTER(C.c_float)]
    L.ffpic_batch_create.argtypes = [C.c_int, C.POINTER(Desc), vp, C.POINTER(P)]
    L.ffpic_batch_view.argtypes = [P, C.c_int, C.POINTER(P)]
    L.ffpic_batch_size.argtypes = [P]
    L.ffpic_batch_step.argtypes = [P, C.c_int32]
    L.ffpic_batch_sync.argtypes = [P]
    L.ffpic_batch_last_error.argtypes = [P]
    L.ffpic_batch_last_error.restype = C.c_char_p
    L.ffpic_batch_destroy.argtypes = [P]
    L.ffpic_host_table.argtypes = [C.POINTER(Desc), C.c_int, vp, C.POINTER(C.c_int64)]
    L.ffpic_host_initial_field.argtypes = [C.POINTER(Desc), C.c_int, vp]
    L.ffpic_autotune.argtypes = [P, C.c_double, C.POINTER(Tuning)]
    L.ffpic_batch_autotune.argtypes = [P, C.c_double, C.POINTER(Tuning)]
    for name in ("ffpic_create", "ffpic_info", "ffpic_load_fields", "ffpic_load_particles",
                 "ffpic_step", "ffpic_run_phases", "ffpic_sync", "ffpic_get_field",
                 "ffpic_num_particles", "ffpic_get_particles", "ffpic_get_sort",
                 "ffpic_diagnostics", "ffpic_save", "ffpic_restore", "ffpic_set_timing",
                 "ffpic_phase_times", "ffpic_get_particles_range", "ffpic_batch_create",
                 "ffpic_batch_view", "ffpic_batch_size", "ffpic_batch_step", "ffpic_batch_sync",
                 "ffpic_batch_destroy", "ffpic_autotune", "ffpic_batch_autotune",
                 "ffpic_spectra", "ffpic_host_table", "ffpic_host_initial_field",
                 "ffpic_diagnostics_noalloc", "ffpic_set_field_rows", "ffpic_record_sort",
                 "ffpic_set_push_chunk",
                 "ffpic_set_graph", "ffpic_graph_stats", "ffpic_batch_set_graph",
                 "ffpic_batch_graph_stats", "ffpic_batch_grouped_launches",
                 "ffpic_batch_get_graph", "ffpic_batch_set_grouped_chunk"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def make_desc(d: Dict, capacity=None) -> Desc:
    s = Desc()
    for k in ("nr", "nth", "ff_enable", "precision", "init", "sort_interval", "nspec"):
        setattr(s, k, int(d[k]))
    for k in ("rmin", "rmax", "r_lc", "r_abs", "mu", "cfl", "omega_b", "rr_coef"):
        setattr(s, k, float(d[k]))
    for k in range(4):
        s.psi_thr[k] = float(d["psi_thr"][k])
    cap = capacity if capacity is not None else d.get("capacity", [0] * int(d["nspec"]))
    for k in range(int(d["nspec"])):
        s.qm[k] = float(d["qm"][k])
        s.weight[k] = float(d["weight"][k])
        s.capacity[k] = int(cap[k])
    s.inject_kappa = float(d.get("inject_kappa", 0.0))
    s.rng_seed = int(d.get("rng_seed", 0))
    ramp = d.get("rr_ramp", ())
    if len(ramp) > 4:
        raise ValueError("at most 4 knots in rr_ramp")
    s.rr_ramp_n = len(ramp)
    for k, (t, f) in enumerate(ramp):
        s.rr_ramp_t[k] = float(t)
        s.rr_ramp_f[k] = float(f)
    s.shell_r = float(d.get("shell_r", 0.0))
    s.gj_extract = float(d.get("gj_extract", 0.0))
    s.gamma_th = float(d.get("gamma_th", 0.0))
    s.gamma_s = float(d.get("gamma_s", 0.0))
    for k in range(2):
        s.gj_species[k] = int(d.get("gj_species", (0, 0))[k])
        s.pair_species[k] = int(d.get("pair_species", (0, 0))[k])
    return s


(TAB_RN, TAB_RH, TAB_RN2, TAB_RH2, TAB_DRN, TAB_DRH, TAB_DR2N, TAB_DR2H, TAB_DR3H, TAB_DR3N,
 TAB_LAMN, TAB_LAMH, TAB_SN, TAB_CN, TAB_SH, TAB_DCN, TAB_DCD, TAB_DTHD, TAB_THN) = range(19)


def host_table(desc: Dict, table: int) -> np.ndarray:
    """FP64 geometry table as ffpic_create builds it on the host (no device)."""
    L = lib()
    d = make_desc(desc, [0] * int(desc["nspec"]))
    n = C.c_int64(0)
    rc = L.ffpic_host_table(C.byref(d), int(table), None, C.byref(n))
    if rc != OK:
        raise FfpicError(rc, "ffpic_host_table rejected its arguments")
    out = np.zeros(n.value)
    L.ffpic_host_table(C.byref(d), int(table), C.c_void_p(out.ctypes.data), C.byref(n))
    return out


def host_initial_field(desc: Dict, comp: int) -> np.ndarray:
    """Initial field component as ffpic_create builds it on the host (no device)."""
    L = lib()
    d = make_desc(desc, [0] * int(desc["nspec"]))
    out = np.zeros((int(desc["nr"]) + 1, int(desc["nth"]) + 1))
    rc = L.ffpic_host_initial_field(C.byref(d), int(comp), C.c_void_p(out.ctypes.data))
    if rc != OK:
        raise FfpicError(rc, "ffpic_host_initial_field rejected its arguments")
    return out


def _ptr(x):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr()), 1 if x.is_cuda else 0
    return C.c_void_p(x.ctypes.data), 0


class Sim:
    """One magnetosphere on the GPU (owns an ffpic_ctx)."""

    def __init__(self, desc: Dict, capacity=None, stream: Optional[int] = None, _view=None):
        L = lib()
        self.desc = dict(desc)
        self.nr, self.nth = int(desc["nr"]), int(desc["nth"])
        self._view = _view is not None
        if _view is not None:
            self._h = _view
        else:
            self._d = make_desc(desc, capacity)
            h = C.c_void_p()
            rc = L.ffpic_create(C.byref(self._d), C.c_void_p(stream or 0), C.byref(h))
            if rc != OK:
                raise FfpicError(rc, "ffpic_create rejected the descriptor or failed to allocate")
            self._h = h
        info = (C.c_double * 4)()
        L.ffpic_info(self._h, info)
        self.dt, self.dlog, self.dth, self.omega = list(info)

    # ---- helpers
    def _chk(self, rc: int):
        if rc != OK:
            msg = lib().ffpic_last_error(self._h)
            raise FfpicError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            if not self._view:       # views belong to their batch
                lib().ffpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.nr + 1, self.nth + 1)

    # ---- API
    def load_fields(self, comp: int, arr):
        a = arr if hasattr(arr, "data_ptr") else np.ascontiguousarray(arr, dtype=np.float64)
        p, dev = _ptr(a)
        self._chk(lib().ffpic_load_fields(self._h, comp, p, dev))

    def load_particles(self, species: int, d: Dict):
        arrs = []
        for k in ("r", "th", "ur", "uth", "uph"):
            x = d[k]
            if not hasattr(x, "data_ptr"):
                x = np.ascontiguousarray(x, dtype=np.float64)
            arrs.append(x)
        ps = [_ptr(x) for x in arrs]
        dev = ps[0][1]
        self._chk(lib().ffpic_load_particles(self._h, species, len(arrs[0]),
                                             *[p for p, _ in ps], dev))

    def step(self, n: int = 1):
        self._chk(lib().ffpic_step(self._h, int(n)))

    def run_phases(self, mask: int):
        self._chk(lib().ffpic_run_phases(self._h, int(mask)))

    def sync(self):
        self._chk(lib().ffpic_sync(self._h))

    def field(self, comp: int) -> np.ndarray:
        out = np.zeros(self.shape)
        self._chk(lib().ffpic_get_field(self._h, comp, C.c_void_p(out.ctypes.data), 0))
        return out

    def n(self, species: int) -> int:
        v = C.c_int64()
        self._chk(lib().ffpic_num_particles(self._h, species, C.byref(v)))
        return int(v.value)

    def particles(self, species: int) -> Dict[str, np.ndarray]:
        n = self.n(species)
        out = {k: np.zeros(n) for k in ("r", "th", "ur", "uth", "uph")}
        cell = np.zeros(n, dtype=np.int32)
        if n:
            self._chk(lib().ffpic_get_particles(
                self._h, species, *[C.c_void_p(out[k].ctypes.data) for k in
                                    ("r", "th", "ur", "uth", "uph")],
                C.c_void_p(cell.ctypes.data)))
        out["cell"] = cell
        return out

    def particles_range(self, species: int, first: int, count: int) -> Dict[str, np.ndarray]:
        """Slots [first, first + count) of a species (clipped to the slots)."""
        n = C.c_int64(count)
        out = {k: np.zeros(max(count, 0)) for k in ("r", "th", "ur", "uth", "uph")}
        cell = np.zeros(max(count, 0), dtype=np.int32)
        self._chk(lib().ffpic_get_particles_range(
            self._h, species, first, C.byref(n),
            *[C.c_void_p(out[k].ctypes.data) for k in ("r", "th", "ur", "uth", "uph")],
            C.c_void_p(cell.ctypes.data)))
        m = n.value
        out = {k: v[:m].copy() for k, v in out.items()}
        out["cell"] = cell[:m].copy()
        return out

    def autotune(self, budget_ms: float) -> Dict:
        """Choose the sort interval by timing (state unchanged afterwards)."""
        t = Tuning()
        self._chk(lib().ffpic_autotune(self._h, float(budget_ms), C.byref(t)))
        return t.as_dict()

    def sort_offsets(self, species: int) -> np.ndarray:
        out = np.zeros(self.nr * self.nth + 1, dtype=np.int32)
        self._chk(lib().ffpic_get_sort(self._h, species, C.c_void_p(out.ctypes.data), None,
                                       None))
        return out

    def set_graph(self, on: bool):
        """Graph capture of whole sort cycles in step() (ffpic_set_graph)."""
        self._chk(lib().ffpic_set_graph(self._h, int(bool(on))))

    def graph_stats(self):
        """(graphs captured, graph launches) so far."""
        b, l = C.c_int64(0), C.c_int64(0)
        self._chk(lib().ffpic_graph_stats(self._h, C.byref(b), C.byref(l)))
        return b.value, l.value

    def record_sort(self, on: bool = True):
        """Record the permutation of the following sorts (ffpic_record_sort)."""
        self._chk(lib().ffpic_record_sort(self._h, int(bool(on))))

    def sort_permutation(self, species: int) -> np.ndarray:
        """perm[k] = slot before the last (recorded) sort of the particle now
        in slot k."""
        off = np.zeros(self.nr * self.nth + 1, dtype=np.int32)
        n = C.c_int64(0)
        L = lib()
        self._chk(L.ffpic_get_sort(self._h, species, C.c_void_p(off.ctypes.data), None,
                                   C.byref(n)))
        perm = np.zeros(max(1, n.value), dtype=np.int32)
        self._chk(L.ffpic_get_sort(self._h, species, C.c_void_p(off.ctypes.data),
                                   C.c_void_p(perm.ctypes.data), C.byref(n)))
        return perm[:n.value].copy()

    def set_field_rows(self, rows: int):
        """Radial rows per workgroup of the fused field step (0 = automatic)."""
        self._chk(lib().ffpic_set_field_rows(self._h, int(rows)))

    def set_push_chunk(self, ppt: int):
        """Particles per thread of the FP32 push's chunks (8, 16 or 32)."""
        self._chk(lib().ffpic_set_push_chunk(self._h, int(ppt)))

    def diagnostics(self, what: int = DIAG_ALL, poynting: bool = False,
                    noalloc: bool = False) -> Dict:
        """ffpic_diagnostics, or with noalloc the allocation-free
        ffpic_diagnostics_noalloc (same results)."""
        d = Diag()
        L = np.zeros(self.nr + 1) if poynting else None
        fn = lib().ffpic_diagnostics_noalloc if noalloc else lib().ffpic_diagnostics
        self._chk(fn(self._h, what | (DIAG_POYNTING if poynting else 0), C.byref(d),
                     C.c_void_p(L.ctypes.data) if L is not None else None))
        ns = int(self.desc["nspec"])
        out = dict(step=d.step, alive=[d.alive[s] for s in range(ns)],
                   removed=[[d.removed[s][k] for k in range(4)] for s in range(ns)],
                   sum_gamma=[d.sum_gamma[s] for s in range(ns)],
                   sum_u=[[d.sum_u[s][k] for k in range(3)] for s in range(ns)],
                   energy_e=d.energy_e, energy_b=d.energy_b, gauss_max=d.gauss_max,
                   divb_max=d.divb_max, error_word=d.error_word)
        if L is not None:
            out["L"] = L
        return out

    def spectra(self, species: int, req: Dict) -> Dict:
        """Gamma histogram dN, radiated power prad and synchrotron SED of one
        species over a region (keys rmin, rmax, thmin, thmax, gmin, gmax,
        numin, numax, ngamma, nnu)."""
        q = SpectraReq()
        for k in ("rmin", "rmax", "thmin", "thmax", "gmin", "gmax", "numin", "numax"):
            setattr(q, k, float(req[k]))
        q.ngamma, q.nnu = int(req["ngamma"]), int(req["nnu"])
        dN, sed, prad = np.zeros(q.ngamma), np.zeros(q.nnu), np.zeros(1)
        dp = dN.ctypes.data_as(C.POINTER(C.c_double))
        self._chk(lib().ffpic_spectra(self._h, int(species), C.byref(q), dp,
                                      sed.ctypes.data_as(C.POINTER(C.c_double)),
                                      prad.ctypes.data_as(C.POINTER(C.c_double))))
        return {"dN": dN, "sed": sed, "prad": float(prad[0])}

    def save(self) -> bytes:
        n = C.c_size_t(0)
        self._chk(lib().ffpic_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._chk(lib().ffpic_save(self._h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._chk(lib().ffpic_restore(self._h, buf, len(blob)))

    def set_timing(self, on: bool):
        self._chk(lib().ffpic_set_timing(self._h, 1 if on else 0))

    def phase_times(self):
        out = (C.c_float * 4)()
        self._chk(lib().ffpic_phase_times(self._h, out))
        return list(out)


class Batch:
    """Independent magnetospheres stepped together (owns an ffpic_batch).
    view(k) gives system k as a Sim that does not own its context."""

    def __init__(self, descs, capacities, stream: Optional[int] = None):
        L = lib()
        n = len(descs)
        arr = (Desc * n)(*[make_desc(d, c) for d, c in zip(descs, capacities)])
        h = C.c_void_p()
        rc = L.ffpic_batch_create(n, arr, C.c_void_p(stream or 0), C.byref(h))
        if rc != OK:
            raise FfpicError(rc, "ffpic_batch_create failed")
        self._h = h
        self.views = []
        for k, d in enumerate(descs):
            v = C.c_void_p()
            self._chk(L.ffpic_batch_view(self._h, k, C.byref(v)))
            self.views.append(Sim(d, _view=v))

    def _chk(self, rc: int):
        if rc != OK:
            msg = lib().ffpic_batch_last_error(self._h)
            raise FfpicError(rc, msg.decode() if msg else "")

    def __len__(self):
        return lib().ffpic_batch_size(self._h)

    def view(self, k: int) -> Sim:
        return self.views[k]

    def step(self, n: int = 1):
        self._chk(lib().ffpic_batch_step(self._h, int(n)))

    def sync(self):
        self._chk(lib().ffpic_batch_sync(self._h))

    GRAPH_OFF, GRAPH_PER_SYSTEM, GRAPH_GROUPED = 0, 1, 2

    def set_graph(self, mode):
        """Graph capture of whole batch cycles (ffpic_batch_set_graph):
        False / 0 off, 1 per-system launches, True / 2 grouped launches
        of all systems where every system allows them (the default)."""
        if isinstance(mode, bool):
            mode = self.GRAPH_GROUPED if mode else self.GRAPH_OFF
        self._chk(lib().ffpic_batch_set_graph(self._h, int(mode)))

    def graph_stats(self):
        """(graphs captured, graph launches) so far."""
        b, l = C.c_int64(0), C.c_int64(0)
        self._chk(lib().ffpic_batch_graph_stats(self._h, C.byref(b), C.byref(l)))
        return b.value, l.value

    def set_grouped_chunk(self, ppt: int):
        """Particles per thread of grouped pushes (8, 16, 32; 0 = each
        system's own setting)."""
        self._chk(lib().ffpic_batch_set_grouped_chunk(self._h, int(ppt)))

    def get_graph(self):
        """(graph mode in use, {mode: ms per batch step} the tuner measured)."""
        return self.graph_settings()[::2]

    def graph_settings(self):
        """(graph mode, grouped push chunk (0 = each system's own),
        {mode: ms per batch step} the tuner measured)."""
        m, g = C.c_int32(0), C.c_int32(0)
        t = (C.c_double * 3)()
        self._chk(lib().ffpic_batch_get_graph(self._h, C.byref(m), C.byref(g), t))
        return m.value, g.value, {k: t[k] for k in range(3) if t[k] > 0}

    def grouped_launches(self):
        """How many graph launches ran grouped launches of all systems."""
        n = C.c_int64(0)
        self._chk(lib().ffpic_batch_grouped_launches(self._h, C.byref(n)))
        return n.value

    def autotune(self, budget_ms: float):
        t = (Tuning * len(self.views))()
        self._chk(lib().ffpic_batch_autotune(self._h, float(budget_ms), t))
        return [x.as_dict() for x in t]

    def close(self):
        if getattr(self, "_h", None):
            for v in self.views:
                v.close()
            lib().ffpic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
