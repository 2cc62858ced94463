"""Error metrics between a reduced-precision run and the FP64 reference.

TEST INFRASTRUCTURE (part of the oracle package).

These are the paper's accuracy metrics (Sec. 4.2, the equations for e_E(t),
e_Omega(t), e_E,max, e_Omega,max and e_Omega,peak): differences of a global
quantity series against the double-precision series, normalised by the
largest absolute value of the double-precision series, in percent.
"""
import numpy as np


def _ref_scale(ref):
    ref = np.asarray(ref, dtype=np.float64)
    return np.max(np.abs(ref))


def e_series(mxp, ref):
    """Per-time-level error |q_mxp(t) - q_dp(t)| / max_t |q_dp(t)| * 100 (e_E(t), e_Omega(t))."""
    mxp = np.asarray(mxp, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(mxp - ref) / _ref_scale(ref) * 100.0


def e_max(mxp, ref):
    """max_i |q_mxp(t_i) - q_dp(t_i)| / max_i |q_dp(t_i)| * 100 (e_E,max and e_Omega,max)."""
    return float(np.max(e_series(mxp, ref)))


def e_peak(mxp, ref):
    """|max_i q_mxp(t_i) - max_i q_dp(t_i)| / max_i |q_dp(t_i)| * 100 (e_Omega,peak)."""
    mxp = np.asarray(mxp, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(abs(np.max(mxp) - np.max(ref)) / _ref_scale(ref) * 100.0)
