"""Element-by-element comparison of a model table with the oracle's.

An element passes when |gpu - oracle| <= tol * max(|oracle|, floor), with the
floor equal to the RMS value of the oracle's table: relative error for every
element at least as large as the table's typical value, and an absolute bound
(tol * RMS) for the elements below it.

Why the floor is the RMS and not smaller: after an epoch, SGD's sensitivity
to rounding makes even a plain sequential FP32 implementation (no
reassociation, same order) differ from the FP64 oracle by up to ~1e-3
relative on elements that sit well below their table's RMS.  Worst table,
one epoch: nfsmall shape 1.1e-3 (C) with a floor of 0.1 x RMS and 1.7e-4 (C)
with a floor of 1 x RMS; ml100k shape 1.8e-4 (W) and 4.1e-5 (W).  Those
elements carry the cancellation residue of much larger terms; no FP32 result
can be held to relative accuracy there.
"""
import numpy as np

FLOOR_OF_RMS = 1.0   # floor = RMS of the oracle's table


def table_errors(g, r, floor_of_rms=FLOOR_OF_RMS):
    """(worst element-wise ratio |g - r| / max(|r|, floor), normwise ratio)."""
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    if r.size == 0:
        return 0.0, 0.0
    d = np.abs(g - r)
    rms = float(np.sqrt(np.mean(r * r)))
    floor = max(floor_of_rms * rms, 1e-12)
    elem = float(np.max(d / np.maximum(np.abs(r), floor)))
    norm = float(d.max() / max(np.abs(r).max(), 1e-3))
    return elem, norm


def compare_tables(pairs, tol, say=print, label=""):
    """pairs: {name: (gpu array, oracle array)}; asserts the element-wise bar.
    Also prints the ratio with a floor of 0.1 x RMS, for information."""
    worst = {}
    tight = {}
    for k, (g, r) in pairs.items():
        worst[k] = table_errors(g, r)
        tight[k] = table_errors(g, r, 0.1)[0]
    say("[cmp] %s element-wise (floor RMS) / normwise: %s; floor 0.1 RMS: %s"
        % (label, {k: "%.2e / %.2e" % v for k, v in worst.items()}, {k: "%.2e" % v for k, v in tight.items()}))
    bad = {k: v for k, v in worst.items() if v[0] > tol}
    assert not bad, bad
    return worst
