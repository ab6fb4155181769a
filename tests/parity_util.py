"""Error measures shared by the GPU parity tests."""
import numpy as np


def rel(a, b):
    """Relative error of a against b: the larger of the L2 norm over all
    entries (the reading of "relative error") and the element-wise maximum
    max |a - b| / max |b|, which an error confined to a few nodes (the axis
    rows, the force-free/PIC interface, the absorber's edge) cannot pass
    diluted by the rest of the grid."""
    d = np.asarray(a, dtype=np.float64) - b
    if np.size(d) == 0:
        return 0.0
    nb, mb = np.linalg.norm(b), np.abs(b).max()
    l2 = np.linalg.norm(d) / nb if nb > 0 else np.linalg.norm(d)
    mx = np.abs(d).max() / mb if mb > 0 else np.abs(d).max()
    return float(max(l2, mx))


def rel_grouped(pairs, elementwise=True):
    """Per-component errors normalised by the whole group (E or B): pairs is
    a list of (name, got, ref); each error is ||got - ref|| over the group's
    L2 norm, or (elementwise) the larger of that and max |got - ref| over the
    group's largest entry."""
    ref_l2 = np.sqrt(sum(np.linalg.norm(r) ** 2 for _, _, r in pairs))
    ref_mx = max(np.abs(r).max() for _, _, r in pairs)
    out = {}
    for name, g, r in pairs:
        d = np.asarray(g, dtype=np.float64) - r
        e = np.linalg.norm(d) / ref_l2
        out[name] = float(max(e, np.abs(d).max() / ref_mx) if elementwise else e)
    return out
