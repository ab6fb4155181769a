"""The C-ABI library loads and exports every entry point include/ffpic.h
declares, and the Python structures match the C layout (checked with gcc).
No compute call is made: these run without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffpic.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ffpic_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_14512_amd import ffpic
    try:
        return ffpic.lib()
    except ImportError:
        from paper_2406_14512_amd import build
        build.build()
        return ffpic.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_header(tmp_path, lib):
    from paper_2406_14512_amd import ffpic
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ffpic.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n",
         sizeof(ffpic_desc), sizeof(ffpic_diag),
         offsetof(ffpic_desc, psi_thr), offsetof(ffpic_desc, capacity),
         offsetof(ffpic_desc, weight), offsetof(ffpic_diag, sum_u),
         offsetof(ffpic_diag, gauss_max), offsetof(ffpic_diag, error_word),
         sizeof(ffpic_tuning), offsetof(ffpic_tuning, ms_per_step),
         offsetof(ffpic_tuning, total_ms), offsetof(ffpic_desc, rr_ramp_f),
         offsetof(ffpic_desc, shell_r), offsetof(ffpic_desc, gj_species),
         offsetof(ffpic_desc, gamma_s), offsetof(ffpic_desc, pair_species),
         sizeof(ffpic_spectra_req), offsetof(ffpic_spectra_req, nnu));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    D, G, T = ffpic.Desc, ffpic.Diag, ffpic.Tuning
    want = [ctypes.sizeof(D), ctypes.sizeof(G), D.psi_thr.offset, D.capacity.offset,
            D.weight.offset, G.sum_u.offset, G.gauss_max.offset, G.error_word.offset,
            ctypes.sizeof(T), T.ms_per_step.offset, T.total_ms.offset, D.rr_ramp_f.offset,
            D.shell_r.offset, D.gj_species.offset, D.gamma_s.offset, D.pair_species.offset,
            ctypes.sizeof(ffpic.SpectraReq), ffpic.SpectraReq.nnu.offset]
    assert got == want


def test_null_and_invalid_arguments_fail_cleanly(lib):
    from paper_2406_14512_amd import ffpic
    from paper_2406_14512_amd import workloads as W
    # descriptor validation happens before any device call
    d = W.tiny_dipole(10).desc()
    bad = dict(d, rmax=0.5)                          # rmax < rmin
    h = ctypes.c_void_p()
    assert lib.ffpic_create(ctypes.byref(ffpic.make_desc(bad, [1, 1])), None,
                            ctypes.byref(h)) == ffpic.EINVAL
    bad = dict(d, psi_thr=(0.3, 0.2, 1.0, 1.0))      # thresholds not ordered
    assert lib.ffpic_create(ctypes.byref(ffpic.make_desc(bad, [1, 1])), None,
                            ctypes.byref(h)) == ffpic.EINVAL
    bad = dict(d, cfl=1.5)
    assert lib.ffpic_create(ctypes.byref(ffpic.make_desc(bad, [1, 1])), None,
                            ctypes.byref(h)) == ffpic.EINVAL
    # plasma sources: species out of range or equal, gamma_s >= gamma_th,
    # ramp knots out of order, negative shell radius
    for kw in (dict(gj_extract=1.0, gj_species=(0, 2)), dict(gj_extract=1.0, gj_species=(1, 1)),
               dict(gamma_th=10.0, gamma_s=10.0, pair_species=(0, 1)),
               dict(gamma_th=10.0, gamma_s=2.0, pair_species=(0, 0)),
               dict(rr_ramp=((2.0, 0.1), (1.0, 1.0))), dict(rr_ramp=((0.0, -1.0),)),
               dict(shell_r=-1.0), dict(inject_kappa=-1.0)):
        assert lib.ffpic_create(ctypes.byref(ffpic.make_desc(dict(d, **kw), [1, 1])), None,
                                ctypes.byref(h)) == ffpic.EINVAL, kw
    assert lib.ffpic_step(None, 1) == ffpic.EINVAL
    assert lib.ffpic_sync(None) == ffpic.EINVAL
    assert lib.ffpic_last_error(None) == b"no context"
    # batch and autotune argument checks (no device call is reached)
    b = ctypes.c_void_p()
    good = ffpic.make_desc(d, [1, 1])
    assert lib.ffpic_batch_create(0, ctypes.byref(good), None, ctypes.byref(b)) == ffpic.EINVAL
    assert lib.ffpic_batch_create(1, None, None, ctypes.byref(b)) == ffpic.EINVAL
    assert lib.ffpic_batch_step(None, 1) == ffpic.EINVAL
    assert lib.ffpic_batch_sync(None) == ffpic.EINVAL
    assert lib.ffpic_batch_view(None, 0, ctypes.byref(b)) == ffpic.EINVAL
    assert lib.ffpic_batch_destroy(None) == ffpic.EINVAL
    assert lib.ffpic_batch_size(None) == 0
    assert lib.ffpic_autotune(None, 100.0, None) == ffpic.EINVAL
    assert lib.ffpic_get_particles_range(None, 0, 0, None, None, None, None, None, None,
                                         None) == ffpic.EINVAL
    q = ffpic.SpectraReq(1.0, 2.0, 0.0, 3.0, 1.0, 10.0, 1.0, 2.0, 4, 4)
    buf = (ctypes.c_double * 8)()
    assert lib.ffpic_spectra(None, 0, ctypes.byref(q), buf, buf, buf) == ffpic.EINVAL
    # graph and tuning settings
    n64 = ctypes.c_int64(0)
    mode = ctypes.c_int32(0)
    assert lib.ffpic_set_push_chunk(None, 16) == ffpic.EINVAL
    assert lib.ffpic_set_field_rows(None, 0) == ffpic.EINVAL
    assert lib.ffpic_set_graph(None, 1) == ffpic.EINVAL
    assert lib.ffpic_batch_set_graph(None, 1) == ffpic.EINVAL
    assert lib.ffpic_batch_get_graph(None, ctypes.byref(mode), None, None) == ffpic.EINVAL
    assert lib.ffpic_batch_set_grouped_chunk(None, 16) == ffpic.EINVAL
    assert lib.ffpic_batch_grouped_launches(None, ctypes.byref(n64)) == ffpic.EINVAL
    assert lib.ffpic_batch_graph_stats(None, ctypes.byref(n64), ctypes.byref(n64)) == ffpic.EINVAL
    assert lib.ffpic_batch_autotune(None, 100.0, None) == ffpic.EINVAL
