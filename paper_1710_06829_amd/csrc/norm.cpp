// Dispersion norm f_w (Sec. 4, eq. norm) evaluated on the GPU, and a bounded
// multi-start minimiser of it over an affine family of stencils (Sec. 4 and
// Sec. 5: the paper minimises f_w under the stability constraints of
// eq. constraints inside a search box, from a grid of starting points).
//
// The minimiser is a projected quasi-Newton (BFGS) iteration on the box of
// free parameters with a backtracking line search; a trial point that
// violates the stability constraints is moved back across the (exactly
// computed) stability boundary along the gradient of the margin, so that
// minima on that boundary are reached along it.  The gradient of f_w comes
// from the closed-form derivatives of
// the dispersion relation (computed on the GPU with f_w); a time step tied to
// the stability bound is differentiated through the maximiser of F
// (envelope theorem).

#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/xfdtd.h"
#include "xfdtd_internal.h"

using namespace xfdtd;

namespace {

#define NTRY(expr, what)                                                                             \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return set_error(XFDTD_EHIP, "%s: %s", what, hipGetErrorString(e_));  \
    } while (0)

bool spacing_ok(const xfdtd_grid *g)
{
    return g && g->dx > 0 && g->dy > 0 && g->dz > 0 && isfinite(g->dx) && isfinite(g->dy) && isfinite(g->dz);
}

int check_norm_args(int dims, int64_t n, int weight, double width)
{
    if (dims != 2 && dims != 3) return set_error(XFDTD_EINVAL, "dims must be 2 or 3");
    if (n < 1 || n > (1 << 20)) return set_error(XFDTD_EINVAL, "n must be in [1, 2^20]");
    if ((double)n * n * (dims == 3 ? n : 1) > 4.0e12) return set_error(XFDTD_EINVAL, "n^dims too large");
    if (weight != XFDTD_WEIGHT_UNIT && weight != XFDTD_WEIGHT_AXIS)
        return set_error(XFDTD_EINVAL, "weight must be XFDTD_WEIGHT_UNIT or XFDTD_WEIGHT_AXIS");
    if (weight == XFDTD_WEIGHT_AXIS && !(width > 0 && isfinite(width)))
        return set_error(XFDTD_EINVAL, "width must be finite and > 0");
    return XFDTD_OK;
}

// Device buffers of one norm evaluation (reused by the minimiser).
struct NormDev {
    double *partials = nullptr;  // 14 x nblocks
    double *out = nullptr;       // 15
    unsigned int *bad = nullptr;  // zero between evaluations
    int nblocks = 0;
    hipStream_t s = nullptr;
    ~NormDev()
    {
        if (partials) hipFree(partials);
        if (out) hipFree(out);
        if (bad) hipFree(bad);
    }
    int init(int64_t total, hipStream_t stream)
    {
        s = stream;
        // about 8 samples per thread, 64..1024 workgroups
        const int64_t nb = (total + 2047) / 2048;
        nblocks = (int)(nb < 64 ? 64 : nb > 1024 ? 1024 : nb);
        NTRY(hipMalloc((void **)&partials, sizeof(double) * 14 * (size_t)nblocks), "hipMalloc");
        NTRY(hipMalloc((void **)&out, sizeof(double) * 15), "hipMalloc");
        NTRY(hipMalloc((void **)&bad, sizeof(unsigned int)), "hipMalloc");
        NTRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), s), "hipMemsetAsync");
        return XFDTD_OK;
    }
    // out14: f, df/dc[12], df/ddt.  *nbad: samples with dt^2 F outside (0, 1).
    int eval(const NormArgs &a, double out14[14], unsigned int *nbad)
    {
        double o[15];
        NTRY(launch_norm(a, partials, nblocks, bad, out, s), "norm launch");
        NTRY(hipMemcpyAsync(o, out, sizeof(double) * 15, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        NTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        for (int j = 0; j < 14; ++j) out14[j] = o[j];
        *nbad = (unsigned int)o[14];
        return XFDTD_OK;
    }
};

NormArgs norm_args(const xfdtd_grid *g, double dt, const double *c, int dims, int64_t n, int weight, double width)
{
    NormArgs a;
    for (int i = 0; i < 12; ++i) a.c[i] = c[i];
    a.sp[0] = g->dx;
    a.sp[1] = g->dy;
    a.sp[2] = g->dz;
    a.dt = dt;
    a.width = weight == XFDTD_WEIGHT_AXIS ? width : 1.0;
    a.n = n;
    a.dims = dims;
    a.weight = weight;
    return a;
}

// ---------------------------------------------------------------------------
// minimiser
// ---------------------------------------------------------------------------

struct Eval {
    bool feasible = false;
    double f = INFINITY;
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // df/dz (z: parameters scaled to [0, 1])
    double c[12];
    double dt = 0;
};

struct Problem {
    const xfdtd_grid *g;
    const xfdtd_stencil_problem *p;
    NormDev *dev;
    int m;
    int evals = 0;

    // quantities (12 coefficients, dt) of parameters x, before the alpha rule
    void map(const double *x, double q[13]) const
    {
        for (int r = 0; r < 13; ++r) {
            double v = p->base[r];
            for (int j = 0; j < m; ++j) v += p->map[r * 8 + j] * x[j];
            q[r] = v;
        }
    }

    // coefficients and dt of scaled parameters z (host only)
    void stencil(const double *z, double c[12], double q[13]) const
    {
        double x[8];
        for (int j = 0; j < m; ++j) x[j] = p->lo[j] + z[j] * (p->hi[j] - p->lo[j]);
        map(x, q);
        for (int i = 0; i < 12; ++i) c[i] = q[i];
        if (p->alpha_rule)
            for (int a = 0; a < 3; ++a) c[4 * a] = 1.0 - 2.0 * c[4 * a + 1] - 2.0 * c[4 * a + 2] - 3.0 * c[4 * a + 3];
    }

    // Stability margin (host only, exact over the zone): <= 0 iff F >= 0 and
    // dt^2 F <= 1 everywhere (eq. constraints).
    double margin(const double *z) const
    {
        double c[12], q[13];
        stencil(z, c, q);
        for (int i = 0; i < 12; ++i)
            if (!isfinite(c[i])) return INFINITY;
        const double sp[3] = {g->dx, g->dy, g->dz};
        double flo, fhi;
        f_range(sp, c, &flo, &fhi, p->dims, nullptr);
        if (!(fhi > 0)) return INFINITY;
        // F_min is 0 at k = 0 for every stencil: only a negative F_min counts
        double mg = flo < -1e-12 * fhi ? -flo / fhi : -1.0;
        if (p->dt_mode == 0) {
            if (!(q[12] > 0)) return INFINITY;
            mg = fmax(mg, q[12] * q[12] * fhi - 1.0);
        }
        return mg;
    }

    // Moves an unstable z back across the stability boundary along the
    // margin's gradient (bisection to a margin in [-1e-10, 0)); keeps the
    // progress a step made along the boundary.  False if that fails.
    // Unit outward normal of the stability boundary at z (central differences
    // of the margin); false where the margin is not differentiable there.
    bool normal(const double *z, double *nrm) const
    {
        double nn = 0.0;
        for (int j = 0; j < m; ++j) {
            double zp[8], zm[8];
            for (int i = 0; i < m; ++i) zp[i] = zm[i] = z[i];
            const double h = 1e-7;
            zp[j] = fmin(1.0, z[j] + h);
            zm[j] = fmax(0.0, z[j] - h);
            nrm[j] = (margin(zp) - margin(zm)) / (zp[j] - zm[j]);
            if (!isfinite(nrm[j])) return false;
            nn += nrm[j] * nrm[j];
        }
        if (!(nn > 0)) return false;
        nn = sqrt(nn);
        for (int j = 0; j < m; ++j) nrm[j] /= nn;
        return true;
    }

    bool restore(double *z) const
    {
        const double m0 = margin(z);
        if (m0 <= -1e-12) return true;
        if (!isfinite(m0)) return false;
        double nrm[8];
        if (!normal(z, nrm)) return false;
        auto at = [&](double sft, double *out) {
            for (int j = 0; j < m; ++j) out[j] = fmin(1.0, fmax(0.0, z[j] - sft * nrm[j]));
            return margin(out);
        };
        double zt[8], lo = 0.0, hi = 1e-9;
        while (at(hi, zt) > -1e-12) {
            lo = hi;
            hi *= 2.0;
            if (hi > 1.0) return false;
        }
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (at(mid, zt) > -1e-12)
                lo = mid;
            else
                hi = mid;
        }
        at(hi, zt);
        for (int j = 0; j < m; ++j) z[j] = zt[j];
        return true;
    }

    int evaluate(const double *z, Eval &e)
    {
        double x[8];
        for (int j = 0; j < m; ++j) x[j] = p->lo[j] + z[j] * (p->hi[j] - p->lo[j]);
        double q[13];
        map(x, q);
        for (int i = 0; i < 12; ++i) e.c[i] = q[i];
        if (p->alpha_rule)
            for (int a = 0; a < 3; ++a)
                e.c[4 * a] = 1.0 - 2.0 * e.c[4 * a + 1] - 2.0 * e.c[4 * a + 2] - 3.0 * e.c[4 * a + 3];
        e.feasible = false;
        e.f = INFINITY;
        for (int i = 0; i < 12; ++i)
            if (!isfinite(e.c[i])) return XFDTD_OK;
        const double sp[3] = {g->dx, g->dy, g->dz};
        double flo, fhi, umax[3] = {0, 0, 0};
        f_range(sp, e.c, &flo, &fhi, p->dims, umax);
        if (!(fhi > 0) || flo < -1e-12 * fhi) return XFDTD_OK;  // eq. constraints: 0 <= F
        double dt;
        if (p->dt_mode == 0) {
            dt = q[12];
            if (!(dt > 0) || dt * dt * fhi > 1.0) return XFDTD_OK;  // and dt^2 F <= 1
        } else {
            dt = x[p->dt_param] / sqrt(fhi);
        }
        e.dt = dt;
        double o[14];
        unsigned int nbad = 0;
        int rc = dev->eval(norm_args(g, dt, e.c, p->dims, p->n, p->weight, p->width), o, &nbad);
        if (rc) return rc;
        ++evals;
        if (nbad || !isfinite(o[0])) return XFDTD_OK;  // a sample on the stability boundary
        e.feasible = true;
        e.f = o[0];
        // d f / d c along the time-step dependence (dt_mode 1: dt = x_k F_max^(-1/2))
        double gc[12];
        for (int i = 0; i < 12; ++i) gc[i] = o[1 + i];
        const double gdt = o[13];
        if (p->dt_mode == 1) {
            const double ddt_dfhi = -0.5 * dt / fhi;
            for (int a = 0; a < 3; ++a) {
                const double inv = 1.0 / (sp[a] * sp[a]);
                const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
                const double u = umax[a];
                gc[4 * a] += gdt * ddt_dfhi * u * inv;
                gc[4 * a + 1] += gdt * ddt_dfhi * 2.0 * u * (1.0 - 2.0 * umax[t1]) * inv;
                gc[4 * a + 2] += gdt * ddt_dfhi * 2.0 * u * (1.0 - 2.0 * umax[t2]) * inv;
                gc[4 * a + 3] += gdt * ddt_dfhi * u * (3.0 - 4.0 * u) * inv;
            }
        }
        // alpha rule: alpha_a replaced by 1 - 2 beta_at1 - 2 beta_at2 - 3 delta_a
        if (p->alpha_rule)
            for (int a = 0; a < 3; ++a) {
                const double ga = gc[4 * a];
                gc[4 * a] = 0.0;
                gc[4 * a + 1] -= 2.0 * ga;
                gc[4 * a + 2] -= 2.0 * ga;
                gc[4 * a + 3] -= 3.0 * ga;
            }
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int r = 0; r < 12; ++r) v += p->map[r * 8 + j] * gc[r];
            if (p->dt_mode == 0) v += p->map[12 * 8 + j] * gdt;
            if (p->dt_mode == 1 && j == p->dt_param) v += gdt / sqrt(fhi);
            e.g[j] = v * (p->hi[j] - p->lo[j]);
        }
        return XFDTD_OK;
    }

    // Projected BFGS from z (feasible); best point found in `best`.
    int local(double *z, Eval &cur)
    {
        double H[8][8];
        auto reset = [&]() {
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) H[i][j] = i == j ? 1.0 : 0.0;
        };
        reset();
        for (int it = 0; it < p->max_iter; ++it) {
            bool fixed[8];
            for (int i = 0; i < m; ++i)
                fixed[i] = (z[i] <= 0.0 && cur.g[i] > 0) || (z[i] >= 1.0 && cur.g[i] < 0);
            double d[8], gd = 0.0;
            for (int i = 0; i < m; ++i) {
                d[i] = 0.0;
                if (fixed[i]) continue;
                for (int j = 0; j < m; ++j)
                    if (!fixed[j]) d[i] -= H[i][j] * cur.g[j];
                gd += d[i] * cur.g[i];
            }
            // on the stability boundary with f decreasing outwards: move along
            // the boundary (tangential part of the direction)
            double nrm[8];
            const bool on_boundary = margin(z) > -1e-7 && normal(z, nrm);
            auto tangent = [&](double *v) {
                double vn = 0.0, gn = 0.0;
                for (int i = 0; i < m; ++i) {
                    vn += v[i] * nrm[i];
                    gn += cur.g[i] * nrm[i];
                }
                if (gn < 0 && vn > 0)
                    for (int i = 0; i < m; ++i)
                        if (!fixed[i]) v[i] -= vn * nrm[i];
            };
            if (on_boundary) {
                tangent(d);
                gd = 0.0;
                for (int i = 0; i < m; ++i) gd += d[i] * cur.g[i];
            }
            if (!(gd < 0)) {  // not a descent direction: steepest descent, restart H
                reset();
                gd = 0.0;
                for (int i = 0; i < m; ++i) d[i] = fixed[i] ? 0.0 : -cur.g[i];
                if (on_boundary) tangent(d);
                for (int i = 0; i < m; ++i) gd += d[i] * cur.g[i];
                if (!(gd < 0)) break;  // projected gradient vanishes
            }
            double dmax = 0.0;
            for (int i = 0; i < m; ++i) dmax = fmax(dmax, fabs(d[i]));
            double t = dmax > 0.5 ? 0.5 / dmax : 1.0;
            Eval nxt;
            double zn[8];
            bool ok = false;
            for (int ls = 0; ls < 60; ++ls, t *= 0.5) {
                for (int i = 0; i < m; ++i) zn[i] = fmin(1.0, fmax(0.0, z[i] + t * d[i]));
                if (!restore(zn)) continue;
                double dec = 0.0;
                for (int i = 0; i < m; ++i) dec += cur.g[i] * (zn[i] - z[i]);
                if (!(dec < 0)) continue;
                int rc = evaluate(zn, nxt);
                if (rc) return rc;
                if (nxt.feasible && nxt.f <= cur.f + 1e-4 * dec) {
                    ok = true;
                    break;
                }
            }
            if (!ok) break;
            double s[8], y[8], sy = 0.0, smax = 0.0;
            for (int i = 0; i < m; ++i) {
                s[i] = zn[i] - z[i];
                y[i] = nxt.g[i] - cur.g[i];
                sy += s[i] * y[i];
                smax = fmax(smax, fabs(s[i]));
            }
            const double fprev = cur.f;
            for (int i = 0; i < m; ++i) z[i] = zn[i];
            cur = nxt;
            if (smax < 1e-12 || fabs(fprev - cur.f) <= 1e-15 * fmax(1e-300, fabs(cur.f))) break;
            if (sy > 1e-300) {  // BFGS update of the inverse Hessian
                double Hy[8], yHy = 0.0;
                for (int i = 0; i < m; ++i) {
                    Hy[i] = 0.0;
                    for (int j = 0; j < m; ++j) Hy[i] += H[i][j] * y[j];
                    yHy += y[i] * Hy[i];
                }
                const double r = 1.0 / sy;
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j)
                        H[i][j] += (1.0 + yHy * r) * r * s[i] * s[j] - r * (Hy[i] * s[j] + s[i] * Hy[j]);
            }
        }
        return XFDTD_OK;
    }
};

int check_problem(const xfdtd_stencil_problem *p)
{
    if (!p) return set_error(XFDTD_EINVAL, "null problem");
    if (p->nparam < 1 || p->nparam > 8) return set_error(XFDTD_EINVAL, "nparam must be in [1, 8]");
    int rc = check_norm_args(p->dims, p->n, p->weight, p->width);
    if (rc) return rc;
    for (int r = 0; r < 13; ++r) {
        if (!isfinite(p->base[r])) return set_error(XFDTD_EINVAL, "base must be finite");
        for (int j = 0; j < 8; ++j)
            if (!isfinite(p->map[r * 8 + j])) return set_error(XFDTD_EINVAL, "map must be finite");
    }
    for (int j = 0; j < p->nparam; ++j)
        if (!(isfinite(p->lo[j]) && isfinite(p->hi[j]) && p->lo[j] < p->hi[j]))
            return set_error(XFDTD_EINVAL, "bounds of parameter %d must be finite with lo < hi", j);
    if (p->dt_mode != 0 && p->dt_mode != 1) return set_error(XFDTD_EINVAL, "dt_mode must be 0 or 1");
    if (p->dt_mode == 1) {
        if (p->dt_param < 0 || p->dt_param >= p->nparam) return set_error(XFDTD_EINVAL, "bad dt_param");
        if (!(p->lo[p->dt_param] > 0 && p->hi[p->dt_param] <= 1.0))
            return set_error(XFDTD_EINVAL, "the time-step fraction must have bounds in (0, 1]");
    }
    if (p->starts < 1 || p->starts > 64) return set_error(XFDTD_EINVAL, "starts must be in [1, 64]");
    if (pow((double)p->starts, (double)p->nparam) > 4096.0)
        return set_error(XFDTD_EINVAL, "starts^nparam must be <= 4096");
    if (p->max_iter < 1 || p->max_iter > 100000) return set_error(XFDTD_EINVAL, "max_iter must be in [1, 1e5]");
    return XFDTD_OK;
}

}  // namespace

extern "C" {

int xfdtd_dispersion_norm(const xfdtd_grid *g, double dt, const double coeffs[12], int dims, int64_t n,
                          int weight, double width, double *f, double grad[13], void *stream)
{
    return guarded([&]() -> int {
        if (!spacing_ok(g)) return set_error(XFDTD_EINVAL, "spacings must be finite and > 0");
        if (!coeffs) return set_error(XFDTD_EINVAL, "coeffs is null");
        for (int i = 0; i < 12; ++i)
            if (!isfinite(coeffs[i])) return set_error(XFDTD_EINVAL, "coeffs must be 12 finite values");
        if (!(dt > 0) || !isfinite(dt)) return set_error(XFDTD_EINVAL, "dt must be finite and > 0");
        if (!f) return set_error(XFDTD_EINVAL, "f is null");
        int rc = check_norm_args(dims, n, weight, width);
        if (rc) return rc;
        const int64_t total = dims == 2 ? n * n : n * n * n;
        NormDev dev;
        rc = dev.init(total, (hipStream_t)stream);
        if (rc) return rc;
        double o[14];
        unsigned int nbad = 0;
        rc = dev.eval(norm_args(g, dt, coeffs, dims, n, weight, width), o, &nbad);
        if (rc) return rc;
        if (nbad) {
            *f = NAN;
            return set_error(XFDTD_EUNSTABLE, "%u samples have dt^2 F outside (0, 1): omega undefined", nbad);
        }
        *f = o[0];
        if (grad)
            for (int i = 0; i < 13; ++i) grad[i] = o[1 + i];
        return XFDTD_OK;
    });
}

int xfdtd_optimize_stencil(const xfdtd_grid *g, const xfdtd_stencil_problem *p, double x_out[8],
                           double coeffs_out[12], double *dt_out, double *f_out, int *evals_out, void *stream)
{
    return guarded([&]() -> int {
        if (!spacing_ok(g)) return set_error(XFDTD_EINVAL, "spacings must be finite and > 0");
        int rc = check_problem(p);
        if (rc) return rc;
        if (!x_out || !coeffs_out || !dt_out || !f_out) return set_error(XFDTD_EINVAL, "null output");
        const int m = p->nparam;
        const int64_t total = p->dims == 2 ? p->n * p->n : p->n * p->n * p->n;
        NormDev dev;
        rc = dev.init(total, (hipStream_t)stream);
        if (rc) return rc;
        Problem pr{g, p, &dev, m};
        Eval best;
        double zbest[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int nstart = 1;
        for (int j = 0; j < m; ++j) nstart *= p->starts;
        for (int s = 0; s < nstart; ++s) {
            double z[8];
            int r = s;
            for (int j = 0; j < m; ++j) {
                z[j] = (r % p->starts + 0.5) / p->starts;
                r /= p->starts;
            }
            Eval cur;
            rc = pr.evaluate(z, cur);
            if (rc) return rc;
            if (!cur.feasible) continue;
            rc = pr.local(z, cur);
            if (rc) return rc;
            if (cur.f < best.f) {
                best = cur;
                for (int j = 0; j < m; ++j) zbest[j] = z[j];
            }
        }
        if (evals_out) *evals_out = pr.evals;
        if (!best.feasible) return set_error(XFDTD_EUNSTABLE, "no stable starting point in the search box");
        for (int j = 0; j < m; ++j) x_out[j] = p->lo[j] + zbest[j] * (p->hi[j] - p->lo[j]);
        for (int i = 0; i < 12; ++i) coeffs_out[i] = best.c[i];
        *dt_out = best.dt;
        *f_out = best.f;
        return XFDTD_OK;
    });
}

}  // extern "C"
