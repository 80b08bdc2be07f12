"""Planted mistakes in the oracle must break at least one pin.

Each mutation patches one piece of ``oracle.fdtd`` (on the CPU) with a
plausible slip: a dropped term, a wrong sign or index, a transposed operand.
The pins used are the one-step spectrum against the dispersion relation, the
exact eigenmode, and the App. A wave equations.
"""
import numpy as np
import pytest

from oracle import fdtd as O
from tests import _pins as P

_orig_taps = O.ext_taps
_orig_back = O.back_diff
_orig_A = O._A


def taps_swap_transverse(a):
    # beta_xy applied along z and beta_xz along y
    t = _orig_taps(a)
    if a != 0:
        return t
    out = []
    for slot, sign, off in t:
        if slot in (1, 2):
            slot = 3 - slot
        out.append((slot, sign, off))
    return out


def taps_drop_delta(a):
    return [x for x in _orig_taps(a) if x[0] != 4 * a + 3]


def taps_delta_wrong_offset(a):
    out = []
    for slot, sign, off in _orig_taps(a):
        if slot == 4 * a + 3 and sign < 0:
            off = O.unit(a, -2)
        out.append((slot, sign, off))
    return out


def taps_beta_unshifted(a):
    # the beta pair differences taken without the transverse shift on one side
    out = []
    for slot, sign, off in _orig_taps(a):
        if slot == 4 * a + 1 and sign < 0:
            off = (0, 0, 0)
        out.append((slot, sign, off))
    return out


def back_diff_forward(X, a, d):
    return (O.at(X, O.unit(a, 1)) - X) / d[a]


def A_wrong_cos(theta, coeffs):
    A = _orig_A(theta, coeffs)
    th = np.asarray(theta, dtype=np.float64)
    al, b1, b2, de = O.unpack(coeffs, 0)
    # beta_xy paired with cos(k_x) instead of cos(k_y)
    A[0] = A[0] - 2 * b1 * np.cos(th[..., 1]) + 2 * b1 * np.cos(th[..., 0])
    return A


def faraday_sign_slip(E, B, coeffs, dt, d):
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    return [Bx + dt * (O.ext_diff(Ey, 2, coeffs, d) - O.ext_diff(Ez, 1, coeffs, d)),
            By + dt * (O.ext_diff(Ez, 0, coeffs, d) + O.ext_diff(Ex, 2, coeffs, d)),
            Bz + dt * (O.ext_diff(Ex, 1, coeffs, d) - O.ext_diff(Ey, 0, coeffs, d))]


MUTATIONS = {
    "swap_transverse_beta": ("ext_taps", taps_swap_transverse),
    "drop_delta": ("ext_taps", taps_drop_delta),
    "delta_wrong_offset": ("ext_taps", taps_delta_wrong_offset),
    "beta_unshifted": ("ext_taps", taps_beta_unshifted),
    "ampere_forward_difference": ("back_diff", back_diff_forward),
    "dispersion_wrong_cos": ("_A", A_wrong_cos),
    "faraday_sign": ("faraday", faraday_sign_slip),
}


def _pins_pass():
    ang, mod = P.pin_spectrum((3, 4, 5), seed=11)
    if ang > 1e-10 or mod > 1e-10:
        return False
    if P.pin_plane_wave((8, 8, 8), nsteps=20) > 1e-10:
        return False
    if P.pin_wave_equation((4, 5, 6)) > 1e-8:
        return False
    return True


def test_unmutated_oracle_passes_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(O, attr, fn)
    with np.errstate(all="ignore"):
        try:
            ok = _pins_pass()
        except (ValueError, np.linalg.LinAlgError, FloatingPointError):
            ok = False
    assert not ok, name
