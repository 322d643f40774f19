"""The parity bar of the GPU tests: the HIP solver's chi against the FP64
oracle's, element by element.

Two bounds, both stated per comparison and printed with the observed values:

  relative L2   ||chi_gpu - chi_oracle||_2 / ||chi_oracle||_2 <= 1e-4
  per voxel     max |chi_gpu - chi_oracle| <= 1e-4 * max |chi_oracle|

The first is the whole-request tolerance of FP32 arithmetic against the FP64
iteration.  The second keeps an error confined to a few voxels (a partial
tile, a Nyquist line, the padded slice of an odd stack, a strip boundary)
from hiding under the first: in a 256x256 slice with max|chi| ~ 200 ppm it
fails at 0.02 ppm in a single voxel, while FP32 rounding of these iterates
stays near 1e-6 of max|chi|.
"""
import numpy as np

REL_TOL = 1e-4
VOX_TOL = 1e-4


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def errors(got, ref):
    """(relL2, max-abs, max-abs / max|ref|) of got against ref."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mx = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    return rel_l2(got, ref), mx, (mx / scale if scale > 0 else (0.0 if mx == 0.0 else float("inf")))


def check(got, ref, what="", rel_tol=REL_TOL, vox_tol=VOX_TOL):
    """Assert both bounds; returns (relL2, max-abs)."""
    err, mx, frac = errors(got, ref)
    print("  %s relL2 %.3e (bar %.0e)  max-abs %.3e ppm = %.3e of max|ref| (bar %.0e)"
          % (what, err, rel_tol, mx, frac, vox_tol), flush=True)
    assert err <= rel_tol, "%s: relL2 %.3e > %.0e" % (what, err, rel_tol)
    assert frac <= vox_tol, "%s: max-abs %.3e ppm is %.3e of max|ref| > %.0e" % (what, mx, frac, vox_tol)
    return err, mx
