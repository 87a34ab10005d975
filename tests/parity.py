"""Comparison helpers for the GPU-vs-oracle parity tests.

Tolerances (stated once, used by every parity test):

* Field values: the GPU sums float32 terms c_i exp2(Q_i) per voxel, so its
  error scales with A(p) = sum_i |c_i| G_i(p) over the in-support terms, not
  with |Vhat(p)| (signed weights cancel).  Elementwise
  |V_gpu - V_ref| <= 1e-5 A(p) + 1e-12, and norm-wise
  ||V_gpu - V_ref|| / ||V_ref|| <= 1e-5.
* Truncation boundary: a pair whose float64 m^2 lies within BAND of k^2 may
  fall on either side in float32.  The oracle reports those pairs; voxels that
  hold one are checked against the bracket [V_lo, V_hi] instead, and the
  norm-wise bound is taken over the other voxels.
* Gradients: float32 atomics make the summation order vary, so the result is
  one of many correct ones.  Per parameter group (mu, q, l, c) norm-wise
  relative error <= 1e-3, and elementwise |g - g_ref| <= 1e-3 |g_ref| +
  1e-4 max|g_ref(group)|.  Pairs within BAND of the cut may be decided either
  way (as for values); the oracle's boundary slack (the first-order effect of
  flipping each such pair) widens both bounds accordingly.
"""
import numpy as np

BAND = 1e-4
VAL_RTOL = 1e-5
GRAD_RTOL = 1e-3
GROUPS = {"mu": slice(0, 3), "q": slice(3, 7), "l": slice(7, 10), "c": slice(10, 11)}


def check_field(gpu, ref, A, bracket=None, rtol=VAL_RTOL):
    gpu = np.asarray(gpu, dtype=np.float64)
    err = np.abs(gpu - ref)
    tol = rtol * A + 1e-12
    bad = err > tol
    if bracket is not None:
        lo, hi, namb = bracket
        if namb:
            lo_ = np.minimum(lo, hi) - tol
            hi_ = np.maximum(lo, hi) + tol
            inside = (gpu >= lo_) & (gpu <= hi_)
            amb = np.abs(hi - lo) > 0
            bad = np.where(amb, ~inside, bad)
    nbad = int(np.count_nonzero(bad))
    worst = float(np.max(err / (A + 1e-30))) if err.size else 0.0
    assert nbad == 0, f"{nbad} voxels outside tolerance; worst err/A = {worst:.3e}"
    # norm-wise over the voxels that hold no pair near the cut (there the
    # reference is unique); voxels with such a pair were held to the bracket
    keep = np.ones(ref.shape, dtype=bool)
    if bracket is not None and bracket[2]:
        keep = ~(np.abs(bracket[1] - bracket[0]) > 0)
    nref = float(np.linalg.norm(ref[keep]))
    if nref > 0:
        rel = float(np.linalg.norm((gpu - ref)[keep])) / nref
        assert rel <= rtol, f"norm-wise relative error {rel:.3e} over {int(keep.sum())} voxels"
    return worst


def check_grad(gpu, ref, rtol=GRAD_RTOL, slack=None, absolute=None):
    """``slack`` (from ``oracle.field.boundary_slack``): per entry, how far the
    gradient may move because pairs near the cut are decided either way; it is
    added to the elementwise tolerance and its norm to the norm-wise one.
    ``absolute`` (from ``oracle.field.loss_grad_absolute``): the sum of the
    absolute per-pair contributions; when given, the relative tolerance also
    applies to it (for entries that are small differences of large terms,
    e.g. a single primitive's quaternion gradient)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    if slack is None:
        slack = np.zeros_like(ref)
    if absolute is None:
        absolute = np.zeros_like(ref)
    out = {}
    for name, sl in GROUPS.items():
        g, r, s, a = gpu[sl], ref[sl], slack[sl], absolute[sl]
        nr = float(np.linalg.norm(r))
        err = float(np.linalg.norm(g - r))
        assert err <= rtol * (nr + float(np.linalg.norm(a))) + float(np.linalg.norm(s)), \
            f"{name}: norm-wise relative error {err / max(nr, 1e-300):.3e}"
        floor = 0.1 * rtol * float(np.max(np.abs(r))) if r.size else 0.0
        bad = np.abs(g - r) > rtol * (np.abs(r) + a) + floor + s
        assert not np.any(bad), f"{name}: {int(bad.sum())} entries outside tolerance"
        out[name] = err / nr if nr > 0 else err
    return out
