"""Error measures shared by the GPU parity tests.

rel_l2: relative L2 norm of the difference over all targets and the three
components.  worst: the largest per-target error norm divided by the RMS of
the per-target reference norm, max_i |out_i - ref_i| / sqrt(mean_i |ref_i|^2):
a single target that is off by a tenth of the typical magnitude gives 0.1
however many targets there are, where its share of the L2 norm shrinks as
1/sqrt(N)."""
import numpy as np


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst(a, b):
    a = np.asarray(a, np.float64).reshape(len(a), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    rms = np.sqrt(np.mean(np.sum(b * b, axis=1)))
    return float(np.max(np.linalg.norm(a - b, axis=1)) / rms)


def check(label, a, b, l2_tol, worst_tol):
    """Prints and asserts both measures; returns (rel_l2, worst)."""
    e, w = rel_l2(a, b), worst(a, b)
    print("%s: rel-L2 %.3e (<= %.0e), worst target %.3e of the rms (<= %.0e)" % (label, e, l2_tol, w, worst_tol),
          flush=True)
    assert e <= l2_tol, (label, e)
    assert w <= worst_tol, (label, w)
    return e, w
