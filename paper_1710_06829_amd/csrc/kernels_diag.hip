// Diagnostic kernels of libxfdtd: divergence constraints (Sec. 2.1,
// eq. divstarb and eq. divE) and the dispersion relation with phase and
// group velocity (Sec. 3, Sec. 5).  Memory-bound elementwise work; one
// thread per cell or per wave vector.

#include <math.h>

#include <algorithm>

#include "xfdtd_internal.h"

namespace xfdtd {

namespace {

__device__ __forceinline__ int wrap(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

struct DivCoef {
    double c[12];
    double inv[3];  // 1 / d_a
};

// D*.B at cell centres and D.E at nodes for cell (i, j, k).
template <typename T>
__device__ __forceinline__ void div_at(const Fields<T> &f, Dims d, const DivCoef &cf, int i, int j,
                                       int k, double &dsb, double &de)
{
    int xs[4], ys[4], zs[4];
    for (int o = 0; o < 4; ++o) {
        xs[o] = wrap(i + o - 1, d.nx);
        ys[o] = wrap(j + o - 1, d.ny);
        zs[o] = wrap(k + o - 1, d.nz);
    }
    const int64_t nxy = (int64_t)d.nx * d.ny;
    auto at = [&](const T *X, int ox, int oy, int oz) -> double {
        return (double)X[(int64_t)zs[oz + 1] * nxy + (int64_t)ys[oy + 1] * d.nx + xs[ox + 1]];
    };
    auto g = [&](const T *X, int a, int ox, int oy, int oz) -> double {
        return at(X, ox + (a == 0), oy + (a == 1), oz + (a == 2)) - at(X, ox, oy, oz);
    };
    dsb = 0.0;
    for (int a = 0; a < 3; ++a) {
        const T *X = f.c[3 + a];
        int e[3] = {0, 0, 0}, u[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        e[a] = 1;
        const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
        u[t1] = 1;
        v[t2] = 1;
        const double al = cf.c[4 * a], b1 = cf.c[4 * a + 1], b2 = cf.c[4 * a + 2],
                     de_ = cf.c[4 * a + 3];
        const double s = (al + de_) * g(X, a, 0, 0, 0) +
                         de_ * (g(X, a, e[0], e[1], e[2]) + g(X, a, -e[0], -e[1], -e[2])) +
                         b1 * (g(X, a, u[0], u[1], u[2]) + g(X, a, -u[0], -u[1], -u[2])) +
                         b2 * (g(X, a, v[0], v[1], v[2]) + g(X, a, -v[0], -v[1], -v[2]));
        dsb += s * cf.inv[a];
    }
    de = (at(f.c[0], 0, 0, 0) - at(f.c[0], -1, 0, 0)) * cf.inv[0] +
         (at(f.c[1], 0, 0, 0) - at(f.c[1], 0, -1, 0)) * cf.inv[1] +
         (at(f.c[2], 0, 0, 0) - at(f.c[2], 0, 0, -1)) * cf.inv[2];
}

template <typename T>
__global__ __launch_bounds__(256) void divergence_kernel(Fields<T> f, Dims d, DivCoef cf, T *dsb_out,
                                                         T *de_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.nx) return;
    // y and z loop over the grid (its y and z dimensions are capped)
    for (int k = blockIdx.z; k < d.nz; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < d.ny; j += gridDim.y * blockDim.y) {
            double dsb, de;
            div_at(f, d, cf, i, j, k, dsb, de);
            const int64_t p = ((int64_t)k * d.ny + j) * d.nx + i;
            if (dsb_out) dsb_out[p] = (T)dsb;
            if (de_out) de_out[p] = (T)de;
        }
}

// Per-block partial results: max |D*.B - ref_b|, max |D.E - ref_e|, count of
// non-finite field values.  Grid-stride over all cells.
template <typename T>
__global__ __launch_bounds__(256) void divergence_max_kernel(Fields<T> f, Dims d, DivCoef cf,
                                                             const T *ref_b, const T *ref_e,
                                                             double *partials)
{
    const int64_t n = (int64_t)d.nx * d.ny * d.nz;
    double mb = 0.0, me = 0.0, bad = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % d.nx);
        const int j = (int)((p / d.nx) % d.ny);
        const int k = (int)(p / ((int64_t)d.nx * d.ny));
        double dsb, de;
        div_at(f, d, cf, i, j, k, dsb, de);
        if (ref_b) dsb -= (double)ref_b[p];
        if (ref_e) de -= (double)ref_e[p];
        mb = fmax(mb, fabs(dsb));
        me = fmax(me, fabs(de));
        for (int c = 0; c < 6; ++c)
            if (!isfinite((double)f.c[c][p])) bad += 1.0;
    }
    __shared__ double sm[3][256];
    sm[0][threadIdx.x] = mb;
    sm[1][threadIdx.x] = me;
    sm[2][threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sm[0][threadIdx.x] = fmax(sm[0][threadIdx.x], sm[0][threadIdx.x + s]);
            sm[1][threadIdx.x] = fmax(sm[1][threadIdx.x], sm[1][threadIdx.x + s]);
            sm[2][threadIdx.x] += sm[2][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = sm[0][0];
        partials[3 * blockIdx.x + 1] = sm[1][0];
        partials[3 * blockIdx.x + 2] = sm[2][0];
    }
}

struct DispCoef {
    double c[12];
    double sp[3];
    double dt;
};

// omega, v_ph and v_g at one wave vector (Sec. 3 and Sec. 5), in double.
//   F = sum_a s_a^2 A_a, s_a = sin(k_a d_a / 2)/d_a,
//   A_a = alpha_a + 2 beta_at1 cos(k_t1 d_t1) + 2 beta_at2 cos(k_t2 d_t2)
//         + delta_a (1 + 2 cos(k_a d_a)),
//   omega = (2/dt) asin(dt sqrt(F)) on the principal branch,
//   d omega/d k_a = 2 dt (dF/dk_a) / sin(omega dt).
__device__ __forceinline__ void dispersion_at(const double *kv, int64_t q, const DispCoef &cf, double *omega,
                                              double *vph, double *vg, unsigned int *bad)
{
    double th[3], s2[3], cs[3], sn[3], A[3];
    double kk = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double k = kv[3 * q + a];
        kk += k * k;
        th[a] = k * cf.sp[a];
        const double s = sin(0.5 * th[a]) / cf.sp[a];
        s2[a] = s * s;
        cs[a] = cos(th[a]);
        sn[a] = sin(th[a]);
    }
    // beta_ab sits at slot 4a + 1 + (index of b among a's transverse axes)
    auto beta = [&](int a, int b) -> double {
        const int t1 = (a == 0) ? 1 : 0;
        return cf.c[4 * a + 1 + (b == t1 ? 0 : 1)];
    };
    double F = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
        A[a] = cf.c[4 * a] + 2.0 * cf.c[4 * a + 1] * cs[t1] + 2.0 * cf.c[4 * a + 2] * cs[t2] +
               cf.c[4 * a + 3] * (1.0 + 2.0 * cs[a]);
        F += s2[a] * A[a];
    }
    const double x = cf.dt * cf.dt * F;
    double w;
    if (!(x >= 0.0 && x <= 1.0)) {
        w = NAN;
        atomicAdd(bad, 1u);
    } else {
        w = (2.0 / cf.dt) * asin(sqrt(x));
    }
    omega[q] = w;
    if (vph) vph[q] = w / sqrt(kk);
    if (vg) {
        const double swd = sin(w * cf.dt);
        for (int a = 0; a < 3; ++a) {
            double cross = 0.0;
            for (int b = 0; b < 3; ++b)
                if (b != a) cross += beta(b, a) * s2[b];
            const double dF = sn[a] / (2.0 * cf.sp[a]) * A[a] -
                              2.0 * cf.sp[a] * sn[a] * (cf.c[4 * a + 3] * s2[a] + cross);
            vg[3 * q + a] = 2.0 * cf.dt * dF / swd;
        }
    }
}

// grid-stride over the n wave vectors (the grid is capped in the launcher)
__global__ __launch_bounds__(256) void dispersion_kernel(const double *kv, int64_t n, DispCoef cf,
                                                         double *omega, double *vph, double *vg,
                                                         unsigned int *bad)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dispersion_at(kv, q, cf, omega, vph, vg, bad);
}

// Dispersion norm of Sec. 4 (eq. norm): f_w = prod_a d_a * integral over
// [0, pi/d_a]^dims of w(k) (omega(k) - |k|)^2 (c = 1), by the midpoint rule
// with n points per axis (k_z = 0 when dims = 2), together with its
// derivatives with respect to the 12 coefficients and dt:
//   d omega/dF  = 1 / (sqrt(F) sqrt(1 - dt^2 F))
//   d omega/ddt = -omega/dt + 2 sqrt(F) / (dt sqrt(1 - dt^2 F))
//   dF/d alpha_a = s_a^2, dF/d delta_a = s_a^2 (1 + 2 cos th_a),
//   dF/d beta_at = 2 s_a^2 cos th_t.
// Each thread accumulates its points in FP64; every block writes its 14 sums
// (f, 12 coefficients, dt) to `partials` (j-major: partials[j * nblocks + b]);
// norm_reduce_kernel adds them in a fixed order.  Samples with dt^2 F outside
// (0, 1) are counted in `bad`.
constexpr int NORM_THREADS = 256;

__global__ __launch_bounds__(NORM_THREADS) void norm_kernel(NormArgs a, double *partials, unsigned int *bad)
{
    __shared__ double red[14][NORM_THREADS];
    double acc[14];
    for (int j = 0; j < 14; ++j) acc[j] = 0.0;
    const int64_t n = a.n;
    const int64_t total = a.dims == 2 ? n * n : n * n * n;
    const int64_t stride = (int64_t)gridDim.x * NORM_THREADS;
    unsigned int nbad = 0;
    for (int64_t q = blockIdx.x * (int64_t)NORM_THREADS + threadIdx.x; q < total; q += stride) {
        const int64_t idx[3] = {q % n, (q / n) % n, a.dims == 2 ? 0 : q / (n * n)};
        double s2[3], cs[3], kk = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            if (ax < a.dims) {
                const double th = ((double)idx[ax] + 0.5) * (M_PI / (double)n);  // k_a d_a
                const double k = th / a.sp[ax];
                kk += k * k;
                const double sh = sin(0.5 * th) / a.sp[ax];
                s2[ax] = sh * sh;
                cs[ax] = cos(th);
            } else {
                s2[ax] = 0.0;
                cs[ax] = 1.0;
            }
        }
        double F = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const double A = a.c[4 * ax] + 2.0 * a.c[4 * ax + 1] * cs[t1] + 2.0 * a.c[4 * ax + 2] * cs[t2] +
                             a.c[4 * ax + 3] * (1.0 + 2.0 * cs[ax]);
            F += s2[ax] * A;
        }
        const double x = a.dt * a.dt * F;
        if (!(x > 0.0 && x < 1.0)) {
            ++nbad;
            continue;
        }
        const double sf = sqrt(F), rt = sqrt(1.0 - x);
        const double om = (2.0 / a.dt) * asin(a.dt * sf);
        const double dev = om - sqrt(kk);
        double w = 1.0;
        if (a.weight == 1) {
            double e = 0.0;
            for (int ax = 1; ax < a.dims; ++ax) {
                const double r = ((double)idx[ax] + 0.5) * (M_PI / (double)n) / a.width;
                e += r * r;
            }
            w = exp(-e);
        }
        const double wd = w * dev;
        acc[0] += wd * dev;
        const double g = 2.0 * wd / (sf * rt);  // 2 w dev d omega/dF
        for (int ax = 0; ax < 3; ++ax) {
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            acc[1 + 4 * ax] += g * s2[ax];
            acc[2 + 4 * ax] += g * 2.0 * s2[ax] * cs[t1];
            acc[3 + 4 * ax] += g * 2.0 * s2[ax] * cs[t2];
            acc[4 + 4 * ax] += g * s2[ax] * (1.0 + 2.0 * cs[ax]);
        }
        acc[13] += 2.0 * wd * (-om / a.dt + 2.0 * sf / (a.dt * rt));
    }
    if (nbad) atomicAdd(bad, nbad);
    for (int j = 0; j < 14; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int st = NORM_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < 14; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 14) partials[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// out[j] = scale * sum over blocks of partials[j * nblocks + b] (fixed order)
// for j < 14; out[14] = the count of rejected samples, which is reset to 0
// for the next evaluation.
__global__ __launch_bounds__(NORM_THREADS) void norm_reduce_kernel(const double *partials, int nblocks,
                                                                   double scale, unsigned int *bad,
                                                                   double *out)
{
    __shared__ double red[14][NORM_THREADS];
    for (int j = 0; j < 14; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += NORM_THREADS) v += partials[(int64_t)j * nblocks + b];
        red[j][threadIdx.x] = v;
    }
    __syncthreads();
    for (int st = NORM_THREADS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < 14; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 14) out[threadIdx.x] = scale * red[threadIdx.x][0];
    if (threadIdx.x == 14) {
        out[14] = (double)*bad;
        *bad = 0u;
    }
}

}  // namespace

hipError_t launch_norm(const NormArgs &args, double *partials, int nblocks, unsigned int *bad, double *out,
                       hipStream_t s)
{
    hipLaunchKernelGGL(norm_kernel, dim3(nblocks), dim3(NORM_THREADS), 0, s, args, partials, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double scale = pow(M_PI / (double)args.n, (double)args.dims);  // prod d_a * cell volume
    hipLaunchKernelGGL(norm_reduce_kernel, dim3(1), dim3(NORM_THREADS), 0, s, partials, nblocks, scale, bad,
                       out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divergence(const Fields<T> &f, Dims d, const double coeffs[12], const double sp[3],
                             T *div_star_b, T *div_e, hipStream_t s)
{
    DivCoef cf;
    for (int i = 0; i < 12; ++i) cf.c[i] = coeffs[i];
    for (int a = 0; a < 3; ++a) cf.inv[a] = 1.0 / sp[a];
    dim3 blk(64, 4, 1), grd((d.nx + 63) / 64, (unsigned)std::min((d.ny + 3) / 4, 65535),
                            (unsigned)std::min(d.nz, 65535));
    hipLaunchKernelGGL(divergence_kernel<T>, grd, blk, 0, s, f, d, cf, div_star_b, div_e);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divergence_max(const Fields<T> &f, Dims d, const double coeffs[12],
                                 const double sp[3], const T *ref_b, const T *ref_e,
                                 double *partials, int nblocks, hipStream_t s)
{
    DivCoef cf;
    for (int i = 0; i < 12; ++i) cf.c[i] = coeffs[i];
    for (int a = 0; a < 3; ++a) cf.inv[a] = 1.0 / sp[a];
    hipLaunchKernelGGL(divergence_max_kernel<T>, dim3(nblocks), dim3(256), 0, s, f, d, cf, ref_b,
                       ref_e, partials);
    return hipGetLastError();
}

hipError_t launch_dispersion(const double *k, int64_t n, double dt, const double coeffs[12],
                             const double sp[3], double *omega, double *vph, double *vg,
                             unsigned int *bad, hipStream_t s)
{
    DispCoef cf;
    for (int i = 0; i < 12; ++i) cf.c[i] = coeffs[i];
    for (int a = 0; a < 3; ++a) cf.sp[a] = sp[a];
    cf.dt = dt;
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(dispersion_kernel, dim3((unsigned)nb), dim3(256), 0, s, k, n, cf, omega, vph,
                       vg, bad);
    return hipGetLastError();
}

template hipError_t launch_divergence<float>(const Fields<float> &, Dims, const double *, const double *,
                                             float *, float *, hipStream_t);
template hipError_t launch_divergence<double>(const Fields<double> &, Dims, const double *,
                                              const double *, double *, double *, hipStream_t);
template hipError_t launch_divergence_max<float>(const Fields<float> &, Dims, const double *,
                                                 const double *, const float *, const float *,
                                                 double *, int, hipStream_t);
template hipError_t launch_divergence_max<double>(const Fields<double> &, Dims, const double *,
                                                  const double *, const double *, const double *,
                                                  double *, int, hipStream_t);

}  // namespace xfdtd
