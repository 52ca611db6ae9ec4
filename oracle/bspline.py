"""Hockney-Eastwood assignment weights W^(p) (Sec. 2.3.2, Eq. w3d).

W^(p) is read as the centered cardinal B-spline M_p of order p (degree p-1,
support [-p/2, p/2]); its Fourier transform is sinc^p, the response used in
Eq. Bk.  It is evaluated here from the truncated-power representation

    M_p(t) = 1/(p-1)! * sum_{j=0..p} (-1)^j C(p, j) (t + p/2 - j)_+^(p-1)

and its d-th derivative replaces the exponent by p-1-d and the factorial by
(p-1-d)!.  The step function used for exponent 0 is right-continuous
((u)_+^0 = 1 for u >= 0), so that each polynomial piece is taken on the
half-open interval [k, k+1) of its argument.
"""
from __future__ import annotations

from math import comb, factorial

import numpy as np


def bspline(t, p: int, d: int = 0) -> np.ndarray:
    """d-th derivative of M_p evaluated at t (float64 array)."""
    if not (1 <= p <= 7):
        raise ValueError("assignment order p must be in 1..7")
    t = np.asarray(t, dtype=np.float64)
    e = p - 1 - d
    if e < 0:
        return np.zeros_like(t)
    out = np.zeros_like(t)
    for j in range(p + 1):
        u = t + 0.5 * p - j
        if e == 0:
            term = (u >= 0.0).astype(np.float64)
        else:
            term = np.where(u > 0.0, u, 0.0) ** e
        out += (-1) ** j * comb(p, j) * term
    return out / factorial(e)
