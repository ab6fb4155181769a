"""The OpenMP build of the oracle (used to time the CPU baseline on all
cores) computes what the single-thread build computes: bit for bit on one
thread; on four threads the deposit's per-thread rows are added in thread
order, so the result is the same on every run and differs from the
single-thread build only by the order of those additions."""
import numpy as np

import oracle
from paper_2406_14512_amd import workloads as W

COMPS = (oracle.ER, oracle.ETH, oracle.EPH, oracle.BR, oracle.BTH, oracle.BPH)


def _run(w, threads):
    o = oracle.Oracle(w.desc(), threads=threads)
    for s in range(2):
        o.load(s, w.particles(s))
    o.step(5)
    out = [o.field(c) for c in COMPS]
    for s in range(2):
        p = o.particles(s)
        out += [p["r"], p["th"], p["uph"]]
    return out


def test_openmp_build_matches_single_thread(oracle_lib):
    w = W.tiny_open_dipole(20_000, steps=5)
    ser = _run(w, None)
    one = _run(w, 1)
    assert all(np.array_equal(a, b) for a, b in zip(one, ser))
    four = _run(w, 4)
    again = _run(w, 4)
    assert all(np.array_equal(a, b) for a, b in zip(four, again))
    for a, b in zip(four, ser):
        assert a.shape == b.shape
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)
