"""Per-candidate semblance tolerances of the GPU parity tests.

Binary32 and bfloat16 windows interpolate in binary32 from exact traveltimes
(relative to the output time), so S agrees with the binary64 oracle on the
same stored samples to within the binary32 accumulation error: 1e-5.

Binary16 windows (one packed dot product per interpolated sample, weights
exact in binary16) round each trace's traveltime to the grid 2^-11 samples
(at most 2^-12 off) and take tau = sqrt(q) in binary32 directly (at most
about 2.5e-4 samples off below 4096 samples).  Each trace's traveltime is
then within 5e-4 samples of the exact one, so to first order S moves by at
most 5e-4 times sum_i |dS/dtau_i|; the tolerance doubles that margin for the
kinks of the linear interpolation at whole samples and adds the binary32
bound.
"""
import numpy as np

TOL_S = 1e-5
TAU_ERR_F16 = 1e-3   # twice the largest traveltime error of the binary16 windows (samples)


def s_tol(store, L, cmp, t, p):
    """Tolerance per candidate for |S_gpu - S_oracle| on the stored traces."""
    if store != "f16":
        return np.full(len(cmp), TOL_S)
    return TOL_S + TAU_ERR_F16 * L.tau_sensitivity(cmp, t, np.asarray(p, dtype=np.float64))
