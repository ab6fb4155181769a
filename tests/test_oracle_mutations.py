"""The oracle's pins must catch plausible mistakes in the oracle itself.

Each case plants one mistake in a copy of the oracle's source (a wrong sign,
a swapped weight or operand, a wrong rotation), builds it on the CPU and runs
the kinematics and deposit pins against that build in a child process; the
pins must fail.  An unchanged copy built the same way must pass, so a failure
is the planted mistake's and not the harness's.  Every planted text must
occur exactly once in the source, so an edit of the oracle that moves it
shows up here instead of silently testing nothing.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINS = os.path.join(HERE, "test_oracle_kinematics.py")

# (name, original text, mistaken text)
MUTANTS = [
    ("momentum rotated back by +phi' instead of -phi'",
     "double ux = cp * u[0] + sp * u[1], uy = -sp * u[0] + cp * u[1], uz = u[2];",
     "double ux = cp * u[0] - sp * u[1], uy = sp * u[0] + cp * u[1], uz = u[2];"),
    ("sign of J_phi",
     "double qv = Q * vph;",
     "double qv = -Q * vph;"),
    ("J_phi theta weight of one corner",
     "JT(t, 2, i1 + im + 1, j1 + jm) += qv * wx * (1.0 - wy);",
     "JT(t, 2, i1 + im + 1, j1 + jm) += qv * wx * wy;"),
    ("J_phi weights of two theta corners exchanged",
     "JT(t, 2, i1 + im, j1 + jm + 1) += qv * (1.0 - wx) * wy;",
     "JT(t, 2, i1 + im, j1 + jm + 1) += qv * (1.0 - wx) * (1.0 - wy);"),
    ("J_phi at the start of the move instead of its midpoint",
     "double xm = 0.5 * (x1 + x2), ym = 0.5 * (y1 + y2);",
     "double xm = x1, ym = y1;"),
    ("sign of the E_theta term in the local E_z",
     "Es[0] * ct - Es[1] * st};",
     "Es[0] * ct + Es[1] * st};"),
    ("sign of the B_theta term in the local B_x",
     "double B[3] = {Bs[0] * st + Bs[1] * ct,",
     "double B[3] = {Bs[0] * st - Bs[1] * ct,"),
    ("sign of the u_theta term in the local u_z",
     "q->ur[p] * ct - q->uth[p] * st};",
     "q->ur[p] * ct + q->uth[p] * st};"),
    ("sign of u_z in the rotated-back u_theta",
     "q->uth[p] = ux * ct2 - uz * st2;",
     "q->uth[p] = ux * ct2 + uz * st2;"),
    ("sign of the axial displacement",
     "z = r * ct + dt * v[2];",
     "z = r * ct - dt * v[2];"),
    ("polar angle from atan2 with swapped operands",
     "double th2 = atan2(w, z);",
     "double th2 = atan2(z, w);"),
    ("azimuthal displacement dropped from the cylindrical radius",
     "double w = sqrt(x * x + y * y);",
     "double w = sqrt(x * x);"),
    ("J_phi density over the dual face area instead of the dual volume",
     "AT(s, ORA_JPH, i, j) / dvol(s, i, j)",
     "AT(s, ORA_JPH, i, j) / darea_ph(s, i, j)"),
]


def _build_and_run(tmp, tag, text):
    src = os.path.join(tmp, f"oracle_{tag}.c")
    lib = os.path.join(tmp, f"liboracle_{tag}.so")
    with open(src, "w") as f:
        f.write(text)
    oracle.compile_to(src, lib)
    env = dict(os.environ, FFPIC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout[-2000:]


def test_pins_fail_on_planted_mistakes(tmp_path):
    with open(oracle.SRC) as f:
        text = f.read()
    # the oracle's header sits beside its source copies
    with open(os.path.join(os.path.dirname(oracle.SRC), "ffpic_oracle.h")) as f:
        (tmp_path / "ffpic_oracle.h").write_text(f.read())
    jobs = [("unchanged", text)]
    for k, (name, old, new) in enumerate(MUTANTS):
        assert text.count(old) == 1, f"planted text not found exactly once: {name}"
        jobs.append((f"m{k}", text.replace(old, new)))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda a: _build_and_run(str(tmp_path), *a), jobs))
    rc, out = res[0]
    assert rc == 0, f"the unchanged copy failed its pins:\n{out}"
    survivors = [MUTANTS[k][0] for k, (rc, _) in enumerate(res[1:]) if rc == 0]
    errors = [(MUTANTS[k][0], out) for k, (rc, out) in enumerate(res[1:]) if rc not in (0, 1)]
    assert not errors, f"pin runs that did not complete: {errors}"
    assert not survivors, f"mistakes no pin caught: {survivors}"
