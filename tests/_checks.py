"""Element-by-element comparisons shared by the GPU parity tests.

Every check compares entries one by one.  A whole-vector norm would let a
small-magnitude part of the vector (soft-region entries of a local solve,
stiff-region entries of a displacement) be far off while the norm passes.
"""
import numpy as np


def assert_entrywise(got, ref, tol, scale, what=""):
    """|got_i - ref_i| <= tol * scale_i for every i.

    ``scale`` is a scalar (scaled max-abs: the largest |ref| of the vector,
    or of the part that the entry belongs to) or an array of per-entry
    scales of the same shape as ``ref``.
    """
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    err = np.abs(got - ref)
    bound = tol * np.broadcast_to(np.asarray(scale, dtype=np.float64), ref.shape)
    bad = np.nonzero(~(err <= bound))[0]
    if len(bad):
        i = bad[np.argmax(err[bad] / np.maximum(bound[bad], 1e-300))]
        raise AssertionError(
            f"{what}: {len(bad)} of {len(ref)} entries off; worst at {i}: "
            f"got {got[i]!r} ref {ref[i]!r} |err| {err[i]:.3e} > {bound[i]:.3e}")
    return float(np.max(err / np.maximum(bound, 1e-300))) if len(ref) else 0.0


def max_abs_scaled(got, ref, what=""):
    """Scaled max-abs error max_i |got_i - ref_i| / max_i |ref_i|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    s = float(np.max(np.abs(ref))) if ref.size else 0.0
    return float(np.max(np.abs(got - ref)) / s) if s > 0 else float(np.max(np.abs(got)))


def local_scales(n, parts):
    """Per-entry scale for a sum of local vectors: for every entry the
    largest max-abs over the local vectors that contain it.

    ``parts`` is a list of (indices, local vector) pairs.
    """
    s = np.zeros(n)
    for idx, v in parts:
        m = float(np.max(np.abs(v))) if len(v) else 0.0
        np.maximum.at(s, idx, m)
    return s
