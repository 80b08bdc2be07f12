"""The FP32 parity convention.

libxfdtd folds the coefficients into per-axis weights in double and rounds
each weight once to the field dtype (documented with xfdtd_get_weights):
  wc = dt (alpha + delta) / d_a, wd = dt delta / d_a, wb = dt beta / d_a,
  wa = dt / d_a.
An FP32 run therefore applies a slightly different linear operator than the
FP64 coefficients describe.  For FP32 parity the oracle runs in FP64 with the
operator the FP32 weights define: spacings d'_a = dt / wa_a and coefficients
c' = w d'_a / dt, from the FP32-rounded initial fields.  Both are computed
here from the rule above, not read back from the library.
"""
from __future__ import annotations

import numpy as np


def effective(coeffs, dt, spacing=(1.0, 1.0, 1.0), dtype=np.float32):
    c = np.asarray(coeffs, dtype=np.float64)
    sp = [float(v) for v in spacing]
    out = np.zeros(12)
    sp2 = []
    for a in range(3):
        s = dt / sp[a]
        r = lambda v: float(dtype(v))
        wc = r(s * (c[4 * a] + c[4 * a + 3]))
        wd = r(s * c[4 * a + 3])
        wb1 = r(s * c[4 * a + 1])
        wb2 = r(s * c[4 * a + 2])
        wa = r(s)
        d2 = dt / wa
        f = d2 / dt
        out[4 * a + 3] = wd * f
        out[4 * a + 0] = wc * f - wd * f
        out[4 * a + 1] = wb1 * f
        out[4 * a + 2] = wb2 * f
        sp2.append(d2)
    return out, tuple(sp2)


def round_fields(fields, dtype=np.float32):
    return [np.asarray(f, dtype=dtype).astype(np.float64) for f in fields]
