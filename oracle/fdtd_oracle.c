/*
 * Plain FP64 CPU oracle of the extended-Faraday-stencil Yee FDTD step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the benchmark's CPU
 * baseline, never by the library.  It shares no code with the HIP path.
 *
 * Straight gather loops over every cell, periodic indexing through small
 * wrap tables, OpenMP over z-planes, out of place.  The arithmetic follows
 * Blinne et al. (arXiv:1710.06829): the extended difference D* of Sec. 2 in
 * the Faraday update (App. A, eq. update1-3) and the Yee difference in the
 * Ampere update (eq. update4-6), with c = 1 and J = 0.
 *
 * Layout: six arrays Ex,Ey,Ez,Bx,By,Bz of nz*ny*nx doubles, x fastest,
 * index (k*ny + j)*nx + i.  Component sites as in the update equations:
 * Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2) Bx(i,j+1/2,k+1/2) By(i+1/2,j,k+1/2)
 * Bz(i+1/2,j+1/2,k).  Coefficients: alpha_x, beta_xy, beta_xz, delta_x,
 * alpha_y, beta_yx, beta_yz, delta_y, alpha_z, beta_zx, beta_zy, delta_z.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n[3];          /* nx, ny, nz */
    int64_t *wrap[3];      /* wrap[a][i + 2] = (i mod n_a) for i in [-2, n_a + 2) */
} grid_t;

static int64_t at(const grid_t *g, int64_t i, int64_t j, int64_t k)
{
    int64_t ii = g->wrap[0][i + 2], jj = g->wrap[1][j + 2], kk = g->wrap[2][k + 2];
    return (kk * g->n[1] + jj) * g->n[0] + ii;
}

/* X[p + o] with o = (ox, oy, oz) */
static double tap(const grid_t *g, const double *X, int64_t i, int64_t j, int64_t k,
                  int ox, int oy, int oz)
{
    return X[at(g, i + ox, j + oy, k + oz)];
}

/*
 * D*_a X at p (Sec. 2, the D* definition), result at the forward half-cell.
 * e[] is the unit offset along a, t1[]/t2[] along the two transverse axes.
 */
static double ext_diff(const grid_t *g, const double *X, int64_t i, int64_t j, int64_t k,
                       int a, const double *c, const double *d)
{
    static const int T[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    int e[3] = {0, 0, 0}, u[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    e[a] = 1;
    u[T[a][0]] = 1;
    v[T[a][1]] = 1;
    const double alpha = c[4 * a + 0], b1 = c[4 * a + 1], b2 = c[4 * a + 2], delta = c[4 * a + 3];
    double s = 0.0;
    s += alpha * (tap(g, X, i, j, k, e[0], e[1], e[2]) - tap(g, X, i, j, k, 0, 0, 0));
    s += delta * (tap(g, X, i, j, k, 2 * e[0], 2 * e[1], 2 * e[2])
                  - tap(g, X, i, j, k, -e[0], -e[1], -e[2]));
    s += b1 * (tap(g, X, i, j, k, e[0] + u[0], e[1] + u[1], e[2] + u[2])
               - tap(g, X, i, j, k, u[0], u[1], u[2]));
    s += b1 * (tap(g, X, i, j, k, e[0] - u[0], e[1] - u[1], e[2] - u[2])
               - tap(g, X, i, j, k, -u[0], -u[1], -u[2]));
    s += b2 * (tap(g, X, i, j, k, e[0] + v[0], e[1] + v[1], e[2] + v[2])
               - tap(g, X, i, j, k, v[0], v[1], v[2]));
    s += b2 * (tap(g, X, i, j, k, e[0] - v[0], e[1] - v[1], e[2] - v[2])
               - tap(g, X, i, j, k, -v[0], -v[1], -v[2]));
    return s / d[a];
}

/* Yee difference D_a X at p, result at the backward half-cell (Sec. 2). */
static double back_diff(const grid_t *g, const double *X, int64_t i, int64_t j, int64_t k,
                        int a, const double *d)
{
    int e[3] = {0, 0, 0};
    e[a] = 1;
    return (tap(g, X, i, j, k, 0, 0, 0) - tap(g, X, i, j, k, -e[0], -e[1], -e[2])) / d[a];
}

static int grid_init(grid_t *g, int64_t nx, int64_t ny, int64_t nz)
{
    g->n[0] = nx; g->n[1] = ny; g->n[2] = nz;
    for (int a = 0; a < 3; ++a) {
        g->wrap[a] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(g->n[a] + 4));
        if (!g->wrap[a]) return -1;
        for (int64_t i = -2; i < g->n[a] + 2; ++i)
            g->wrap[a][i + 2] = ((i % g->n[a]) + g->n[a]) % g->n[a];
    }
    return 0;
}

static void grid_free(grid_t *g)
{
    for (int a = 0; a < 3; ++a) free(g->wrap[a]);
}

/*
 * n leapfrog steps in place on f[6] (each nz*ny*nx doubles).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_run(int64_t nx, int64_t ny, int64_t nz, const double d[3], double dt,
               const double coeffs[12], double *f[6], int64_t nsteps)
{
    if (nx < 1 || ny < 1 || nz < 1 || nsteps < 0) return -1;
    grid_t g;
    if (grid_init(&g, nx, ny, nz)) return -1;
    const size_t N = (size_t)(nx * ny * nz);
    double *tmp[6];
    for (int c = 0; c < 6; ++c) {
        tmp[c] = (double *)malloc(sizeof(double) * N);
        if (!tmp[c]) return -1;
    }
    double *E[3] = {f[0], f[1], f[2]}, *B[3] = {f[3], f[4], f[5]};
    double *En[3] = {tmp[0], tmp[1], tmp[2]}, *Bn[3] = {tmp[3], tmp[4], tmp[5]};

    for (int64_t s = 0; s < nsteps; ++s) {
        /* Faraday, eq. update1-3: B^{n+1/2} = B^{n-1/2} - dt * (D* x E^n) */
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t p = (k * ny + j) * nx + i;
                    Bn[0][p] = B[0][p] + dt * (ext_diff(&g, E[1], i, j, k, 2, coeffs, d)
                                               - ext_diff(&g, E[2], i, j, k, 1, coeffs, d));
                    Bn[1][p] = B[1][p] + dt * (ext_diff(&g, E[2], i, j, k, 0, coeffs, d)
                                               - ext_diff(&g, E[0], i, j, k, 2, coeffs, d));
                    Bn[2][p] = B[2][p] + dt * (ext_diff(&g, E[0], i, j, k, 1, coeffs, d)
                                               - ext_diff(&g, E[1], i, j, k, 0, coeffs, d));
                }
        /* Ampere, eq. update4-6 (J = 0): E^{n+1} = E^n + dt * (D x B^{n+1/2}) */
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t p = (k * ny + j) * nx + i;
                    En[0][p] = E[0][p] + dt * (back_diff(&g, Bn[2], i, j, k, 1, d)
                                               - back_diff(&g, Bn[1], i, j, k, 2, d));
                    En[1][p] = E[1][p] + dt * (back_diff(&g, Bn[0], i, j, k, 2, d)
                                               - back_diff(&g, Bn[2], i, j, k, 0, d));
                    En[2][p] = E[2][p] + dt * (back_diff(&g, Bn[1], i, j, k, 0, d)
                                               - back_diff(&g, Bn[0], i, j, k, 1, d));
                }
        for (int c = 0; c < 3; ++c) {
            double *t = E[c]; E[c] = En[c]; En[c] = t;
            t = B[c]; B[c] = Bn[c]; Bn[c] = t;
        }
    }
    /* results may sit in the scratch arrays after an odd number of steps */
    for (int c = 0; c < 3; ++c) {
        if (E[c] != f[c]) memcpy(f[c], E[c], sizeof(double) * N);
        if (B[c] != f[3 + c]) memcpy(f[3 + c], B[c], sizeof(double) * N);
    }
    for (int c = 0; c < 6; ++c) free(tmp[c]);
    grid_free(&g);
    return 0;
}

/*
 * Sampled evaluation for large grids: the state after n steps at selected
 * sites is not computable locally, so the oracle offers the one-step map at
 * chosen sites instead: out[m*6 + c] = component c of step(f) at site idx[m].
 */
int oracle_step_at(int64_t nx, int64_t ny, int64_t nz, const double d[3], double dt,
                   const double coeffs[12], const double *const f[6],
                   const int64_t *idx, int64_t m, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || m < 0) return -1;
    grid_t g;
    if (grid_init(&g, nx, ny, nz)) return -1;
    const double *E[3] = {f[0], f[1], f[2]}, *B[3] = {f[3], f[4], f[5]};
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) {
        const int64_t p = idx[q];
        const int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
        /* B^{n+1/2} at p and at the three backward neighbours the Ampere
           update of E at p needs */
        double Bn[4][3];
        const int off[4][3] = {{0, 0, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}};
        for (int r = 0; r < 4; ++r) {
            const int64_t ii = i + off[r][0], jj = j + off[r][1], kk = k + off[r][2];
            const int64_t pp = at(&g, ii, jj, kk);
            Bn[r][0] = B[0][pp] + dt * (ext_diff(&g, E[1], ii, jj, kk, 2, coeffs, d)
                                        - ext_diff(&g, E[2], ii, jj, kk, 1, coeffs, d));
            Bn[r][1] = B[1][pp] + dt * (ext_diff(&g, E[2], ii, jj, kk, 0, coeffs, d)
                                        - ext_diff(&g, E[0], ii, jj, kk, 2, coeffs, d));
            Bn[r][2] = B[2][pp] + dt * (ext_diff(&g, E[0], ii, jj, kk, 1, coeffs, d)
                                        - ext_diff(&g, E[1], ii, jj, kk, 0, coeffs, d));
        }
        /* Bn[1] = p - e_x, Bn[2] = p - e_y, Bn[3] = p - e_z */
        out[q * 6 + 0] = E[0][p] + dt * ((Bn[0][2] - Bn[2][2]) / d[1] - (Bn[0][1] - Bn[3][1]) / d[2]);
        out[q * 6 + 1] = E[1][p] + dt * ((Bn[0][0] - Bn[3][0]) / d[2] - (Bn[0][2] - Bn[1][2]) / d[0]);
        out[q * 6 + 2] = E[2][p] + dt * ((Bn[0][1] - Bn[1][1]) / d[0] - (Bn[0][0] - Bn[2][0]) / d[1]);
        out[q * 6 + 3] = Bn[0][0];
        out[q * 6 + 4] = Bn[0][1];
        out[q * 6 + 5] = Bn[0][2];
    }
    grid_free(&g);
    return 0;
}

int oracle_abi_version(void) { return 1; }
