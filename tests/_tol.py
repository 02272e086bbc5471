"""Per-candidate semblance tolerances of the GPU parity tests.

Binary32 and bfloat16 windows interpolate in binary32 from exact traveltimes
(relative to the output time), so S agrees with the binary64 oracle on the
same stored samples to within the binary32 accumulation error: 1e-5.

Binary16 windows (one packed dot product per interpolated sample, weights
exact in binary16) round each trace's traveltime to the grid 2^(lb-23)
samples, where 2^lb is the smallest power of two at or above
max(4096, nt + 16) (nt + 16: the record and its zero padding), so at most
2^(lb-24) off; and they take tau = sqrt(q) in binary32 directly, with the
square root within one ulp and q within about one ulp, together at most
2 * 2^(lb-24) for tau < 2^lb.  Each trace's traveltime is then within
3 * 2^(lb-24) samples of the exact one (7.3e-4 samples for records of up to
4080 samples, doubling with each doubling of the grid), and to first order S
moves by at most that times sum_i |dS/dtau_i|.  The tolerance takes
1e-3 * 2^(lb-12) per unit of that sum (1.37 times the first-order bound, a
margin for the kinks of the linear interpolation at whole samples) and adds
the binary32 bound.
"""
import numpy as np

TOL_S = 1e-5
PAD = 16             # zero samples stored before and after each record


def tau_err_f16(nt):
    """Traveltime margin (samples) of the binary16 windows for records of nt samples."""
    lb = 12
    while (1 << lb) < nt + PAD:
        lb += 1
    return 1e-3 * 2.0 ** (lb - 12)


def s_tol(store, L, cmp, t, p):
    """Tolerance per candidate for |S_gpu - S_oracle| on the stored traces."""
    if store != "f16":
        return np.full(len(cmp), TOL_S)
    return TOL_S + tau_err_f16(L.nt) * L.tau_sensitivity(cmp, t, np.asarray(p, dtype=np.float64))
