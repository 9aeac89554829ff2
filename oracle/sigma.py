"""The five sigma_k nonlinearities of Tab. nonlinearfunctions (Appendix
"Nonlinear function definitions"), evaluated at t = k*x.

``sigma(kind, t)`` returns sigma(t); ``dsigma(kind, t)`` returns
d sigma / d t.  The caller multiplies by k for d/dx.  Piecewise functions
take the derivative of the open piece that holds t, and 0 outside
(a kink at a breakpoint is given the derivative of the piece it belongs to
under the table's inequalities; generators keep tested inputs away from
kinks).
"""
import numpy as np
from scipy.special import erf as _erf, expit as _expit

KINDS = ("sigmoid", "erf", "sin", "linear", "quadratic")
_R2 = np.sqrt(0.5)     # 1/sqrt(2), correctly rounded


def sigma(kind, t):
    t = np.asarray(t, dtype=np.float64)
    if kind == "sigmoid":
        # (1 + exp(-t))^-1
        return _expit(t)
    if kind == "erf":
        # (1 + Erf(t)) / 2
        return 0.5 * (1.0 + _erf(t))
    if kind == "sin":
        # 0 below -pi/2, (1 + sin t)/2 on [-pi/2, pi/2], 1 above
        return np.where(t < -np.pi / 2, 0.0, np.where(t > np.pi / 2, 1.0, 0.5 * (1.0 + np.sin(t))))
    if kind == "linear":
        # max{0, min{1, t + 1/2}}
        return np.maximum(0.0, np.minimum(1.0, t + 0.5))
    if kind == "quadratic":
        # 0 | (1/sqrt2 + t)^2 | 1 - (1/sqrt2 - t)^2 | 1 with breaks at -1/sqrt2, 0, 1/sqrt2
        lo = (_R2 + t) ** 2
        hi = 1.0 - (_R2 - t) ** 2
        return np.where(t < -_R2, 0.0, np.where(t < 0.0, lo, np.where(t <= _R2, hi, 1.0)))
    raise ValueError(f"unknown sigma kind {kind!r}")


def dsigma(kind, t):
    t = np.asarray(t, dtype=np.float64)
    if kind == "sigmoid":
        s = _expit(t)
        return s * (1.0 - s)
    if kind == "erf":
        return np.exp(-t * t) / np.sqrt(np.pi)
    if kind == "sin":
        return np.where((t > -np.pi / 2) & (t < np.pi / 2), 0.5 * np.cos(t), 0.0)
    if kind == "linear":
        return np.where((t > -0.5) & (t < 0.5), 1.0, 0.0)
    if kind == "quadratic":
        return np.where((t > -_R2) & (t < 0.0), 2.0 * (_R2 + t),
                        np.where((t >= 0.0) & (t < _R2), 2.0 * (_R2 - t), 0.0))
    raise ValueError(f"unknown sigma kind {kind!r}")


def support(kind):
    """|t| beyond which sigma is 0 or 1 to below FP64 resolution at eps ~ 12
    (exactly, for the compact kinds)."""
    return {"sigmoid": 40.0, "erf": 6.5, "sin": np.pi / 2, "linear": 0.5, "quadratic": _R2}[kind]
