"""FP64 CPU oracle for the extended-Faraday-stencil Yee FDTD scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library.

Everything here follows Blinne et al., "A Systematic Approach to Numerical
Dispersion in Maxwell Solvers" (arXiv:1710.06829), written plainly with numpy in
float64: gather-form stencils with periodic ``np.roll`` indexing, no tiling, no
fusion, no reordering beyond the equations.

Conventions (the readings taken where the paper is silent or ambiguous):
  * periodic boundaries on all three axes; c = 1; vacuum (J = 0);
  * arrays have shape (nz, ny, nx), x fastest; component (i, j, k) sits at the
    staggered site given by the index subscripts of the update equations
    (App. A, eq. update1-6): Ex (i+1/2,j,k), Ey (i,j+1/2,k), Ez (i,j,k+1/2),
    Bx (i,j+1/2,k+1/2), By (i+1/2,j,k+1/2), Bz (i+1/2,j+1/2,k);
  * the state is (E^n, B^{n-1/2}); one step is the Faraday update (B to n+1/2,
    using E^n) followed by the Ampere update (E to n+1, using B^{n+1/2});
  * the 12 coefficients are ordered
    (alpha_x, beta_xy, beta_xz, delta_x, alpha_y, beta_yx, beta_yz, delta_y,
     alpha_z, beta_zx, beta_zy, delta_z),
    beta_ab being the a-derivative's taps shifted along b (Sec. 2, D* eq.).
"""
from __future__ import annotations

import itertools

import numpy as np

AXES = "xyz"
# numpy axis of each spatial axis for arrays shaped (nz, ny, nx)
NP_AXIS = {0: 2, 1: 1, 2: 0}
# transverse axes of each derivative axis, in the order of the coefficient list
TRANSVERSE = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


# ----------------------------------------------------------------------------
# coefficients
# ----------------------------------------------------------------------------
def coeffs_from(beta, delta, alpha=None):
    """Assemble the 12-vector from beta (3x2) and delta (3).

    alpha defaults to the consistency condition eq.(alpha), Sec. 2:
    alpha_a = 1 - 2 beta_ab - 2 beta_ac - 3 delta_a.
    """
    beta = np.asarray(beta, dtype=np.float64).reshape(3, 2)
    delta = np.asarray(delta, dtype=np.float64).reshape(3)
    c = np.zeros(12)
    for a in range(3):
        al = 1.0 - 2.0 * beta[a, 0] - 2.0 * beta[a, 1] - 3.0 * delta[a] \
            if alpha is None else float(np.asarray(alpha)[a])
        c[4 * a:4 * a + 4] = (al, beta[a, 0], beta[a, 1], delta[a])
    return c


def yee_coeffs():
    """The Yee limit: alpha = 1, beta = delta = 0 (Sec. 3, after eq. constraints)."""
    return coeffs_from(np.zeros((3, 2)), np.zeros(3))


def unpack(coeffs, a):
    """(alpha_a, beta_a,t1, beta_a,t2, delta_a) for axis a."""
    c = np.asarray(coeffs, dtype=np.float64)
    return c[4 * a], c[4 * a + 1], c[4 * a + 2], c[4 * a + 3]


# ----------------------------------------------------------------------------
# stencils (Sec. 2)
# ----------------------------------------------------------------------------
def at(X, offset):
    """X[p + offset] for every p, periodic.  offset = (ox, oy, oz) in cells."""
    ox, oy, oz = offset
    return np.roll(X, shift=(-oz, -oy, -ox), axis=(0, 1, 2))


def unit(a, s=1):
    o = [0, 0, 0]
    o[a] = s
    return tuple(o)


def add(*offs):
    return tuple(int(sum(v)) for v in zip(*offs))


def ext_taps(a):
    """Taps of the extended difference D*_a as (coeff_slot, sign, offset).

    Read off the D* definition of Sec. 2, with the half-integer positions of the
    paper mapped to storage indices: a quantity sampled at p +/- 1/2 e_a in the
    paper is X[p + e_a] and X[p] here (the result sits half a cell up along a).
    coeff_slot indexes the 12-vector.
    """
    t1, t2 = TRANSVERSE[a]
    base = 4 * a
    taps = [
        (base + 0, +1.0, unit(a, 1)), (base + 0, -1.0, (0, 0, 0)),        # alpha
        (base + 3, +1.0, unit(a, 2)), (base + 3, -1.0, unit(a, -1)),      # delta
    ]
    for slot, t in ((base + 1, t1), (base + 2, t2)):                      # beta_at
        for s in (+1, -1):
            taps.append((slot, +1.0, add(unit(a, 1), unit(t, s))))
            taps.append((slot, -1.0, unit(t, s)))
    return taps


def ext_diff(X, a, coeffs, d):
    """D*_a X (Sec. 2), result stored at the forward half-cell along a."""
    c = np.asarray(coeffs, dtype=np.float64)
    out = np.zeros_like(X)
    for slot, sign, off in ext_taps(a):
        out += (c[slot] * sign) * at(X, off)
    return out / d[a]


def fwd_diff(X, a, d):
    """Plain two-point difference to the forward half-cell: (X[p+e_a]-X[p])/d_a."""
    return (at(X, unit(a, 1)) - X) / d[a]


def back_diff(X, a, d):
    """Yee difference D_a to the backward half-cell: (X[p]-X[p-e_a])/d_a (Sec. 2)."""
    return (X - at(X, unit(a, -1))) / d[a]


# ----------------------------------------------------------------------------
# the leapfrog step (App. A, eq. update1-6 with J = 0)
# ----------------------------------------------------------------------------
def faraday(E, B, coeffs, dt, d):
    """B^{n+1/2} from B^{n-1/2} and E^n with the extended stencil (update1-3)."""
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    Bx_n = Bx + dt * (ext_diff(Ey, 2, coeffs, d) - ext_diff(Ez, 1, coeffs, d))
    By_n = By + dt * (ext_diff(Ez, 0, coeffs, d) - ext_diff(Ex, 2, coeffs, d))
    Bz_n = Bz + dt * (ext_diff(Ex, 1, coeffs, d) - ext_diff(Ey, 0, coeffs, d))
    return [Bx_n, By_n, Bz_n]


def ampere(E, B, dt, d):
    """E^{n+1} from E^n and B^{n+1/2} with the plain Yee stencil (update4-6)."""
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    Ex_n = Ex + dt * (back_diff(Bz, 1, d) - back_diff(By, 2, d))
    Ey_n = Ey + dt * (back_diff(Bx, 2, d) - back_diff(Bz, 0, d))
    Ez_n = Ez + dt * (back_diff(By, 0, d) - back_diff(Bx, 1, d))
    return [Ex_n, Ey_n, Ez_n]


def ampere_current(E, B, J, dt, d):
    """E^{n+1} with the current term of update4-6, E += c^2 dt (D x B - mu_0 J),
    in units c = mu_0 = 1; J = (Jx, Jy, Jz) at the sites of Ex, Ey, Ez."""
    Ex, Ey, Ez = E
    Bx, By, Bz = B
    Jx, Jy, Jz = J
    Ex_n = Ex + dt * (back_diff(Bz, 1, d) - back_diff(By, 2, d) - Jx)
    Ey_n = Ey + dt * (back_diff(Bx, 2, d) - back_diff(Bz, 0, d) - Jy)
    Ez_n = Ez + dt * (back_diff(By, 0, d) - back_diff(Bx, 1, d) - Jz)
    return [Ex_n, Ey_n, Ez_n]


def step(fields, coeffs, dt, d):
    """One leapfrog step: (E^n, B^{n-1/2}) -> (E^{n+1}, B^{n+1/2})."""
    E, B = list(fields[:3]), list(fields[3:])
    B = faraday(E, B, coeffs, dt, d)
    E = ampere(E, B, dt, d)
    return E + B


def run(fields, n, coeffs, dt, d=(1.0, 1.0, 1.0)):
    """n steps from the six arrays ``fields`` (returns new float64 arrays)."""
    f = [np.array(x, dtype=np.float64, copy=True) for x in fields]
    d = tuple(float(v) for v in d)
    for _ in range(int(n)):
        f = step(f, coeffs, dt, d)
    return f


# ----------------------------------------------------------------------------
# adjoint: literal transposes of the two updates, scatter form
# ----------------------------------------------------------------------------
def scatter(Y, offset):
    """Transpose of ``at(X, offset)``: adds Y[p] into slot p + offset."""
    ox, oy, oz = offset
    return np.roll(Y, shift=(oz, oy, ox), axis=(0, 1, 2))


# (output B component, sign, derivative axis, input E component) per update1-3
FARADAY_TERMS = (
    (0, +1.0, 2, 1), (0, -1.0, 1, 2),
    (1, +1.0, 0, 2), (1, -1.0, 2, 0),
    (2, +1.0, 1, 0), (2, -1.0, 0, 1),
)
# (output E component, sign, derivative axis, input B component) per update4-6
AMPERE_TERMS = (
    (0, +1.0, 1, 2), (0, -1.0, 2, 1),
    (1, +1.0, 2, 0), (1, -1.0, 0, 2),
    (2, +1.0, 0, 1), (2, -1.0, 1, 0),
)


def faraday_T(lamB, coeffs, dt, d):
    """Transpose of the Faraday increment E -> dt*(D* x E) terms: returns the
    three arrays sum_p sum_taps w * lamB_b[p] scattered onto E_c[p+o]."""
    c = np.asarray(coeffs, dtype=np.float64)
    out = [np.zeros_like(lamB[0]) for _ in range(3)]
    for b, sgn, a, e in FARADAY_TERMS:
        for slot, sign, off in ext_taps(a):
            w = dt * sgn * c[slot] * sign / d[a]
            out[e] += w * scatter(lamB[b], off)
    return out


def ampere_T(lamE, dt, d):
    """Transpose of the Ampere increment B -> dt*(D x B) terms."""
    out = [np.zeros_like(lamE[0]) for _ in range(3)]
    for e, sgn, a, b in AMPERE_TERMS:
        w = dt * sgn / d[a]
        out[b] += w * scatter(lamE[e], (0, 0, 0))
        out[b] += -w * scatter(lamE[e], unit(a, -1))
    return out


def faraday_coeff_grad(mu, E, dt, d):
    """d/dcoeff of <mu, Faraday increment(E)> for each of the 12 coefficients.

    The increment is linear in the coefficients, so each partial is the same
    sum with the coefficient replaced by 1 and all other taps dropped.
    """
    g = np.zeros(12)
    for b, sgn, a, e in FARADAY_TERMS:
        for slot, sign, off in ext_taps(a):
            g[slot] += dt * sgn * sign / d[a] * np.sum(mu[b] * at(E[e], off))
    return g


def adjoint_step(lam, E_n, coeffs, dt, d):
    """Reverse one step.

    Forward: B' = B + K(E), E' = E + L(B') with K, L the two increments.
    Given lam = (dLoss/dE', dLoss/dB'), returns (dLoss/dE, dLoss/dB) and the
    coefficient-gradient contribution of this step (E_n is the step's E input).
    """
    lamE, lamB = list(lam[:3]), list(lam[3:])
    LT = ampere_T(lamE, dt, d)
    mu = [lamB[i] + LT[i] for i in range(3)]          # dLoss/dB' in total
    KT = faraday_T(mu, coeffs, dt, d)
    gE = [lamE[i] + KT[i] for i in range(3)]
    g_coef = faraday_coeff_grad(mu, E_n, dt, d)
    return gE + mu, g_coef


def run_with_adjoint(fields, n, coeffs, dt, d, grad_out):
    """Forward n steps, then the exact reverse pass.

    ``grad_out(final_fields) -> six arrays`` gives dLoss/d(final state).
    Returns (final_fields, grad wrt the six initial arrays, grad wrt the 12
    coefficients).  Stores every E^n (plain, no checkpointing).
    """
    d = tuple(float(v) for v in d)
    f = [np.array(x, dtype=np.float64, copy=True) for x in fields]
    Es = []
    for _ in range(int(n)):
        Es.append([x.copy() for x in f[:3]])
        f = step(f, coeffs, dt, d)
    lam = [np.asarray(x, dtype=np.float64) for x in grad_out(f)]
    gc = np.zeros(12)
    for s in reversed(range(int(n))):
        lam, g = adjoint_step(lam, Es[s], coeffs, dt, d)
        gc += g
    return f, lam, gc


# ----------------------------------------------------------------------------
# dispersion relation (Sec. 3) and stability (eq. constraints)
# ----------------------------------------------------------------------------
def _A(theta, coeffs):
    """A_x, A_y, A_z of Sec. 3 for theta_a = k_a * d_a (array (...,3))."""
    th = np.asarray(theta, dtype=np.float64)
    cs = np.cos(th)
    A = []
    for a in range(3):
        al, b1, b2, de = unpack(coeffs, a)
        t1, t2 = TRANSVERSE[a]
        A.append(al + 2.0 * b1 * cs[..., t1] + 2.0 * b2 * cs[..., t2]
                 + de * (1.0 + 2.0 * cs[..., a]))
    return A


def dispersion_rhs(k, coeffs, d=(1.0, 1.0, 1.0)):
    """F(k) = s_x^2 A_x + s_y^2 A_y + s_z^2 A_z (eq. dispersion_relation)."""
    k = np.asarray(k, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    th = k * d
    A = _A(th, coeffs)
    F = 0.0
    for a in range(3):
        s = np.sin(0.5 * th[..., a]) / d[a]
        F = F + s * s * A[a]
    return F


def omega(k, dt, coeffs, d=(1.0, 1.0, 1.0)):
    """Principal-branch frequency: sin(omega dt/2)/dt = sqrt(F) (c = 1).

    NaN where dt^2 F is outside [0, 1] (no real frequency; eq. constraints).
    """
    F = dispersion_rhs(k, coeffs, d)
    x = dt * dt * F
    with np.errstate(invalid="ignore"):
        w = (2.0 / dt) * np.arcsin(np.sqrt(x))
    return np.where((x >= 0.0) & (x <= 1.0), w, np.nan)


def dispersion(k, dt, coeffs, d=(1.0, 1.0, 1.0)):
    """omega, phase velocity omega/|k| and group velocity d omega / d k.

    From eq. dispersion_relation: omega = (2/dt) asin(dt sqrt(F)), so
    d omega/dk_a = 2 dt (dF/dk_a) / sin(omega dt), with
    dF/dk_a = sin(theta_a)/(2 d_a) A_a
              - 2 d_a sin(theta_a) (delta_a s_a^2 + sum_{b != a} beta_ba s_b^2).
    Returns (omega[...], vph[...], vg[..., 3]).
    """
    k = np.asarray(k, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    th = k * d
    A = _A(th, coeffs)
    s2 = [(np.sin(0.5 * th[..., a]) / d[a]) ** 2 for a in range(3)]
    w = omega(k, dt, coeffs, d)
    kn = np.linalg.norm(k, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        vph = w / kn
    c = np.asarray(coeffs, dtype=np.float64)
    vg = np.zeros(k.shape)
    sw = np.sin(w * dt)
    for a in range(3):
        de = c[4 * a + 3]
        cross = 0.0
        for b in range(3):
            if b == a:
                continue
            # beta_ba: the b-derivative's taps shifted along a
            slot = 4 * b + 1 + TRANSVERSE[b].index(a)
            cross = cross + c[slot] * s2[b]
        sa = np.sin(th[..., a])
        dF = sa / (2.0 * d[a]) * A[a] - 2.0 * d[a] * sa * (de * s2[a] + cross)
        with np.errstate(invalid="ignore", divide="ignore"):
            vg[..., a] = 2.0 * dt * dF / sw
    return w, vph, vg


def _quadratic_form(coeffs, d):
    """F as c.u + u^T Q u in u_a = sin^2(theta_a/2) in [0, 1].

    With s_a^2 = u_a/d_a^2 and cos(theta_a) = 1 - 2 u_a, each A_a is affine in u.
    """
    d = np.asarray(d, dtype=np.float64)
    lin = np.zeros(3)
    Q = np.zeros((3, 3))
    for a in range(3):
        al, b1, b2, de = unpack(coeffs, a)
        t1, t2 = TRANSVERSE[a]
        inv = 1.0 / d[a] ** 2
        # A_a = al + de*(1 + 2(1-2u_a)) + 2 b1 (1-2u_t1) + 2 b2 (1-2u_t2)
        lin[a] += inv * (al + 3.0 * de + 2.0 * b1 + 2.0 * b2)
        Q[a, a] += inv * (-4.0 * de)
        Q[a, t1] += 0.5 * inv * (-4.0 * b1)
        Q[t1, a] += 0.5 * inv * (-4.0 * b1)
        Q[a, t2] += 0.5 * inv * (-4.0 * b2)
        Q[t2, a] += 0.5 * inv * (-4.0 * b2)
    return lin, Q


def stability_range(coeffs, d=(1.0, 1.0, 1.0), dims=3):
    """(F_min, F_max) of F over the whole zone 0 <= k_a d_a <= pi.

    ``dims=2`` restricts to k_z = 0 (the paper's 2D setting).

    Exact: F is quadratic in u in the unit cube, so its extrema sit at KKT
    points.  For each of the 27 patterns (each u_a pinned at 0, pinned at 1, or
    free) solve the stationarity equations of the free coordinates and keep the
    feasible solutions.  A face whose restricted Hessian is singular attains its
    extrema on its own boundary (F is constant along a null direction through a
    stationary point), which another pattern enumerates, so such faces are
    skipped.
    """
    lin, Q = _quadratic_form(coeffs, d)

    def F(u):
        return float(lin @ u + u @ Q @ u)

    vals = []
    for pat in itertools.product((0, 1, 2), repeat=3):
        if dims == 2 and pat[2] != 0:
            continue
        free = [a for a in range(3) if pat[a] == 2]
        u = np.array([float(p) if p < 2 else 0.0 for p in pat])
        if free:
            fixed = [a for a in range(3) if pat[a] != 2]
            H = 2.0 * Q[np.ix_(free, free)]
            rhs = -(lin[free] + 2.0 * Q[np.ix_(free, fixed)] @ u[fixed])
            if abs(np.linalg.det(H)) < 1e-14 * max(1.0, np.abs(H).max() ** len(free)):
                continue
            sol = np.linalg.solve(H, rhs)
            if np.any(sol < -1e-12) or np.any(sol > 1.0 + 1e-12):
                continue
            u[free] = np.clip(sol, 0.0, 1.0)
        vals.append(F(u))
    return min(vals), max(vals)


def cfl_dt(coeffs, d=(1.0, 1.0, 1.0), dims=3):
    """Largest stable dt: (dt)^2 F_max = 1 (right inequality of eq. constraints)."""
    _, fmax = stability_range(coeffs, d, dims)
    return 1.0 / np.sqrt(fmax)


# ----------------------------------------------------------------------------
# divergences (eq. divstarb, eq. divE) and the discrete Laplacian (App. A)
# ----------------------------------------------------------------------------
def div_star_B(B, coeffs, d):
    """D* . B at cell centres (eq. divstarb)."""
    return sum(ext_diff(B[a], a, coeffs, d) for a in range(3))


def div_E(E, d):
    """D . E at the nodes (eq. divE): sum_a (E_a[p] - E_a[p-e_a]) / d_a."""
    return sum(back_diff(E[a], a, d) for a in range(3))


def div_B(B, d):
    """Plain Yee divergence of B at cell centres."""
    return sum(fwd_diff(B[a], a, d) for a in range(3))


def laplacian_star(X, coeffs, d):
    """Delta* = D* . D (App. A) applied to one staggered component.

    Along each axis D_a moves the sample half a cell and D*_a moves it back;
    in storage indices that is D*_a of the forward difference, read one cell
    down along a.  The result sits at X's own sites.
    """
    out = np.zeros_like(X)
    for a in range(3):
        out += at(ext_diff(fwd_diff(X, a, d), a, coeffs, d), unit(a, -1))
    return out


# ----------------------------------------------------------------------------
# special inputs: exact eigenmode and the D*-divergence-free projection
# ----------------------------------------------------------------------------
STAGGER = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))


def plane_wave_params(shape, modes, dt, coeffs, d=(1.0, 1.0, 1.0), pol=(0.3, -0.5, 0.8)):
    """Parameters of the exact discrete eigenmode with integer mode numbers
    ``modes`` = (mx, my, mz) on a periodic ``shape`` = (nz, ny, nx) grid.

    Fourier symbols (Sec. 3): D_a -> i K_a, D*_a -> i K_a A_a with
    K_a = 2 sin(theta_a/2)/d_a, and the time difference -> -i W with
    W = 2 sin(omega dt/2)/dt.  Then Ehat is any unit vector with K.Ehat = 0 and
    Bhat = (K* x Ehat)/W, K*_a = K_a A_a, W^2 = K.K* (eq. dispersion_relation).
    Component c of the mode at step n is amp_c cos(k . x_c - omega t_c) at its
    staggered sites x_c (``STAGGER``), with t = n dt for E and (n - 1/2) dt
    for B.  Returns (omega, Ehat, Bhat, k).
    """
    nz, ny, nx = shape
    n = (nx, ny, nz)
    d = np.asarray(d, dtype=np.float64)
    k = np.array([2.0 * np.pi * modes[a] / (n[a] * d[a]) for a in range(3)])
    th = k * d
    A = np.array(_A(th, coeffs), dtype=np.float64)
    K = 2.0 * np.sin(0.5 * th) / d
    Ks = K * A
    w = float(omega(k, dt, coeffs, d))
    W = 2.0 * np.sin(0.5 * w * dt) / dt
    p = np.asarray(pol, dtype=np.float64)
    Kh = K / np.linalg.norm(K)
    Eh = p - (p @ Kh) * Kh
    Eh /= np.linalg.norm(Eh)
    Bh = np.cross(Ks, Eh) / W
    return w, Eh, Bh, k


def plane_wave_sample(shape, params, comp, flat_idx, nsteps, dt, d=(1.0, 1.0, 1.0)):
    """Component ``comp`` (0..5 = Ex..Bz) of the eigenmode ``params`` after
    ``nsteps`` steps at the flat storage indices ``flat_idx`` ((k ny + j) nx + i)."""
    w, Eh, Bh, k = params
    nz, ny, nx = shape
    d = np.asarray(d, dtype=np.float64)
    idx = np.asarray(flat_idx, dtype=np.int64)
    i, j, kk = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    ox, oy, oz = STAGGER[comp]
    phase = k[0] * (i + ox) * d[0] + k[1] * (j + oy) * d[1] + k[2] * (kk + oz) * d[2]
    if comp < 3:
        return Eh[comp] * np.cos(phase - w * nsteps * dt)
    return Bh[comp - 3] * np.cos(phase - w * (nsteps - 0.5) * dt)


def plane_wave(shape, modes, dt, coeffs, d=(1.0, 1.0, 1.0), pol=(0.3, -0.5, 0.8)):
    """Exact discrete eigenmode with integer mode numbers ``modes`` = (mx,my,mz)
    (see ``plane_wave_params``): E sampled at t = 0, B at t = -dt/2, each at
    its staggered sites.  Returns (fields, omega, Ehat, Bhat, k).
    """
    nz, ny, nx = shape
    d = np.asarray(d, dtype=np.float64)
    w, Eh, Bh, k = plane_wave_params(shape, modes, dt, coeffs, d, pol)
    stag = STAGGER
    fields = []
    for c in range(6):
        ox, oy, oz = stag[c]
        x = (np.arange(nx) + ox) * d[0]
        y = (np.arange(ny) + oy) * d[1]
        z = (np.arange(nz) + oz) * d[2]
        phase = k[0] * x[None, None, :] + k[1] * y[None, :, None] + k[2] * z[:, None, None]
        if c < 3:
            fields.append(Eh[c] * np.cos(phase))
        else:
            fields.append(Bh[c - 3] * np.cos(phase + 0.5 * w * dt))
    return fields, w, Eh, Bh, k


def plane_wave_at(shape, modes, dt, coeffs, nsteps, d=(1.0, 1.0, 1.0), pol=(0.3, -0.5, 0.8)):
    """The eigenmode of ``plane_wave`` advanced analytically by nsteps steps."""
    f0, w, Eh, Bh, k = plane_wave(shape, modes, dt, coeffs, d, pol)
    nz, ny, nx = shape
    stag = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))
    t = nsteps * dt
    out = []
    for c in range(6):
        ox, oy, oz = stag[c]
        x = (np.arange(nx) + ox) * d[0]
        y = (np.arange(ny) + oy) * d[1]
        z = (np.arange(nz) + oz) * d[2]
        phase = k[0] * x[None, None, :] + k[1] * y[None, :, None] + k[2] * z[:, None, None]
        if c < 3:
            out.append(Eh[c] * np.cos(phase - w * t))
        else:
            out.append(Bh[c - 3] * np.cos(phase - w * (t - 0.5 * dt)))
    return out


def project_div_star_free(B, coeffs, d=(1.0, 1.0, 1.0)):
    """Remove the part of B that D* . B sees (FFT in index space).

    In index space D*_a has the symbol (e^{i kappa_a} - 1) A_a(kappa) / d_a
    (Sec. 3 with sin(3x/2) = sin(x/2)(1 + 2 cos x)).  With that vector dstar,
    Bhat <- Bhat - conj(dstar) (dstar . Bhat) / |dstar|^2; modes with
    dstar = 0 are left alone.
    """
    d = np.asarray(d, dtype=np.float64)
    nz, ny, nx = B[0].shape
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    kz = 2.0 * np.pi * np.fft.fftfreq(nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    th = np.stack([KX, KY, KZ], axis=-1)
    A = _A(th, coeffs)
    ds = [(np.exp(1j * th[..., a]) - 1.0) * A[a] / d[a] for a in range(3)]
    Bh = [np.fft.fftn(B[a]) for a in range(3)]
    n2 = sum(np.abs(ds[a]) ** 2 for a in range(3))
    dot = sum(ds[a] * Bh[a] for a in range(3))
    safe = n2 > 1e-300
    coef = np.where(safe, dot / np.where(safe, n2, 1.0), 0.0)
    return [np.real(np.fft.ifftn(Bh[a] - np.conj(ds[a]) * coef)) for a in range(3)]


# ----------------------------------------------------------------------------
# dispersion norm f_w (Sec. 4, eq. norm), midpoint rule
# ----------------------------------------------------------------------------
def norm_fw(dt, coeffs, d=(1.0, 1.0, 1.0), n=400, dims=3, weight=None):
    """f_w = (prod d) * integral over [0, pi/d_a] of w(k) (omega(k) - |k|)^2.

    ``dims=2`` integrates k_x, k_y only with k_z = 0 (the paper's 2D tables);
    midpoint rule with n points per axis.  ``weight(k)`` defaults to 1.
    """
    d = np.asarray(d, dtype=np.float64)
    axes = [(np.arange(n) + 0.5) * (np.pi / d[a]) / n for a in range(dims)]
    grids = np.meshgrid(*axes, indexing="ij")
    k = np.zeros(grids[0].shape + (3,))
    for a in range(dims):
        k[..., a] = grids[a]
    w = omega(k, dt, coeffs, d)
    dev = (w - np.linalg.norm(k, axis=-1)) ** 2
    if weight is not None:
        dev = dev * weight(k)
    cell = np.prod([np.pi / d[a] / n for a in range(dims)])
    return float(np.prod(d[:dims]) * np.sum(dev) * cell)
