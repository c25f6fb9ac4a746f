"""Element-wise comparison helpers for the parity tests.

A state is compared per column group: the camera rotation (9 entries), the
translation, each of the three intrinsics d1, d2, d3 separately, and the
landmarks.  Within a group the error is the largest absolute difference over
the largest magnitude of the reference, so that a small column (d3 is about
1e-10 in caller units) is measured on its own scale and not hidden by the
focal length or the translation."""

import numpy as np

CAM_GROUPS = {"R": slice(0, 9), "t": slice(9, 12), "d1": slice(12, 13), "d2": slice(13, 14), "d3": slice(14, 15)}


def group_err(a, b) -> float:
    a, b = np.asarray(a, float), np.asarray(b, float)
    scale = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if b.size else 0.0


def state_errs(sg: dict, so: dict, cams_key="cams", lms_key="lms") -> dict:
    """Per-group errors of sg against the reference so (dicts holding camera
    arrays [M, 15] and landmark arrays [N, 3])."""
    out = {g: group_err(sg[cams_key][:, sl], so[cams_key][:, sl]) for g, sl in CAM_GROUPS.items()}
    out["l"] = group_err(sg[lms_key], so[lms_key])
    return out


def assert_state_close(sg: dict, so: dict, tol: float, what="state", **keys):
    errs = state_errs(sg, so, **keys)
    print(f"{what}: " + " ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (what, tol, bad)
    return errs
