// Host runtime of libxfdtd: argument checking, coefficient and time-step
// preparation (eq.(alpha), eq. constraints), weight folding, launch
// configuration, and the C entry points declared in include/xfdtd.h.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/xfdtd.h"
#include "xfdtd_internal.h"

using namespace xfdtd;

namespace {

// message of the last failure on this thread (fixed size: never allocates)
thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

int xfdtd::set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

bool xfdtd::log_on()
{
    static const bool on = [] {
        const char *v = getenv("XFDTD_LOG");
        return v && atoi(v) > 0;
    }();
    return on;
}

void xfdtd::xlog(const char *fmt, ...)
{
    if (!log_on()) return;
    char line[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(line, sizeof line, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[xfdtd] %s\n", line);
}

xfdtd::Range::Range(const char *name) noexcept { roctxRangePushA(name); }
xfdtd::Range::~Range() { roctxRangePop(); }

namespace {

std::mutex g_tune_file_mu;

// "<architecture>/<CUs>" of the current device ("" if it cannot be read)
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "";
    }
    std::string arch = p.gcnArchName;
    for (char &c : arch)
        if (c == ' ') c = '_';
    return arch + "/" + std::to_string(p.multiProcessorCount);
}

}  // namespace

bool xfdtd::tune_cache_lookup(const std::string &key, std::vector<int> &vals)
{
    const char *path = getenv("XFDTD_TUNE_CACHE");
    if (!path || !*path) return false;
    const std::string tag = device_tag();
    if (tag.empty()) return false;
    std::lock_guard<std::mutex> lk(g_tune_file_mu);
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[8192];
    while (fgets(line, sizeof line, f)) {
        char *save = nullptr;
        const char *t = strtok_r(line, " \t\n", &save);
        const char *k = t ? strtok_r(nullptr, " \t\n", &save) : nullptr;
        if (!t || !k || tag != t || key != k) continue;
        std::vector<int> v;
        bool ok = true;
        for (const char *w = strtok_r(nullptr, " \t\n", &save); w; w = strtok_r(nullptr, " \t\n", &save)) {
            char *end = nullptr;
            const long x = strtol(w, &end, 10);
            if (!end || *end || x < -1000000 || x > 1000000) {
                ok = false;
                break;
            }
            v.push_back((int)x);
        }
        if (ok && !v.empty()) {
            vals = v;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void xfdtd::tune_cache_store(const std::string &key, const std::vector<int> &vals)
{
    const char *path = getenv("XFDTD_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tag = device_tag();
    if (tag.empty()) return;
    std::string line = tag + " " + key;
    for (int v : vals) line += " " + std::to_string(v);
    line += "\n";
    if (line.size() >= 8000) return;  // longer than a line the lookup reads
    std::lock_guard<std::mutex> lk(g_tune_file_mu);
    FILE *f = fopen(path, "a");
    if (!f) return;
    fputs(line.c_str(), f);
    fclose(f);
}

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return fail(XFDTD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool grid_ok(const xfdtd_grid *g)
{
    if (!g) return false;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if (g->nx > (1 << 30) || g->ny > (1 << 30) || g->nz > (1 << 30)) return false;
    if ((double)g->nx * (double)g->ny * (double)g->nz > 4.0e9) return false;
    // z-planes are addressed with 32-bit byte offsets in the kernels
    if ((double)g->nx * (double)g->ny > (double)(1 << 28)) return false;
    if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0)) return false;
    if (!isfinite(g->dx) || !isfinite(g->dy) || !isfinite(g->dz)) return false;
    return true;
}

bool coeffs_ok(const double *c)
{
    if (!c) return false;
    for (int i = 0; i < 12; ++i)
        if (!isfinite(c[i])) return false;
    return true;
}

// Transverse axes of derivative axis a, in coefficient order.
inline int t1_of(int a) { return a == 0 ? 1 : 0; }
inline int t2_of(int a) { return a == 2 ? 1 : 2; }

// Extremes of F over the zone.  With u_a = sin^2(k_a d_a / 2) in [0, 1] we have
// s_a^2 = u_a / d_a^2 and cos(k_a d_a) = 1 - 2 u_a, so
//   F(u) = sum_a (u_a/d_a^2) (alpha_a + delta_a (3 - 4 u_a) + sum_t 2 beta_at (1 - 2 u_t))
// is a quadratic  lin.u + u^T Q u  on the unit cube.  Its extremes are at
// points where the gradient vanishes within some face of the cube; every face
// is one of 27 patterns (each u_a at 0, at 1, or free).  A face whose Hessian
// is singular reaches its extremes on its own boundary, so it is skipped.
}  // namespace

void xfdtd::f_range(const double sp[3], const double *c, double *out_lo, double *out_hi, int dims,
                    double umax[3])
{
    double lin[3] = {0, 0, 0}, Q[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < 3; ++a) {
        const double inv = 1.0 / (sp[a] * sp[a]);
        const double al = c[4 * a], b1 = c[4 * a + 1], b2 = c[4 * a + 2], de = c[4 * a + 3];
        const int t1 = t1_of(a), t2 = t2_of(a);
        lin[a] += inv * (al + 3.0 * de + 2.0 * b1 + 2.0 * b2);
        Q[a][a] += -4.0 * de * inv;
        // cross term -4 beta_at u_a u_t / d_a^2; S = (Q + Q^T)/2 below
        Q[a][t1] += -4.0 * b1 * inv;
        Q[a][t2] += -4.0 * b2 * inv;
    }
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = (a == b) ? Q[a][a] : 0.5 * (Q[a][b] + Q[b][a]);
    auto F = [&](const double u[3]) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a) {
            v += lin[a] * u[a];
            for (int b = 0; b < 3; ++b) v += u[a] * S[a][b] * u[b];
        }
        return v;
    };
    double lo = INFINITY, hi = -INFINITY;
    for (int pat = 0; pat < 27; ++pat) {
        int st[3] = {pat % 3, (pat / 3) % 3, pat / 9};  // 0: u=0, 1: u=1, 2: free
        if (dims == 2 && st[2] != 0) continue;           // k_z = 0 plane
        double u[3];
        int fr[3], nf = 0;
        for (int a = 0; a < 3; ++a) {
            u[a] = st[a] == 1 ? 1.0 : 0.0;
            if (st[a] == 2) fr[nf++] = a;
        }
        if (nf > 0) {
            // 2 S_ff u_f = -(lin_f + 2 S_fx u_x)
            double M[3][4];
            double scale = 0.0;
            for (int r = 0; r < nf; ++r) {
                double rhs = -lin[fr[r]];
                for (int a = 0; a < 3; ++a)
                    if (st[a] != 2) rhs -= 2.0 * S[fr[r]][a] * u[a];
                for (int q = 0; q < nf; ++q) {
                    M[r][q] = 2.0 * S[fr[r]][fr[q]];
                    scale = fmax(scale, fabs(M[r][q]));
                }
                M[r][nf] = rhs;
            }
            // Gaussian elimination with partial pivoting
            bool singular = scale == 0.0;
            for (int col = 0; col < nf && !singular; ++col) {
                int piv = col;
                for (int r = col + 1; r < nf; ++r)
                    if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
                if (fabs(M[piv][col]) <= 1e-13 * scale) {
                    singular = true;
                    break;
                }
                if (piv != col)
                    for (int q = 0; q <= nf; ++q) {
                        double t = M[col][q];
                        M[col][q] = M[piv][q];
                        M[piv][q] = t;
                    }
                for (int r = 0; r < nf; ++r) {
                    if (r == col) continue;
                    const double f = M[r][col] / M[col][col];
                    for (int q = col; q <= nf; ++q) M[r][q] -= f * M[col][q];
                }
            }
            if (singular) continue;
            bool feasible = true;
            for (int r = 0; r < nf; ++r) {
                double v = M[r][nf] / M[r][r];
                if (v < -1e-12 || v > 1.0 + 1e-12) feasible = false;
                u[fr[r]] = fmin(1.0, fmax(0.0, v));
            }
            if (!feasible) continue;
        }
        const double v = F(u);
        lo = fmin(lo, v);
        if (v > hi) {
            hi = v;
            if (umax)
                for (int q = 0; q < 3; ++q) umax[q] = u[q];
        }
    }
    *out_lo = lo;
    *out_hi = hi;
}

namespace {

int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return n;
}

// Workgroups that run at once: CUs x resident workgroups per CU (one where
// the occupancy is unknown, e.g. without a device).
int64_t fused_slots(int dtype, int tile_x, int tile_y)
{
    const int per = dtype == XFDTD_F32 ? fused_occupancy<float>(tile_x, tile_y)
                                       : fused_occupancy<double>(tile_x, tile_y);
    return (int64_t)device_cus() * (per > 0 ? per : 1);
}

int64_t adjoint_slots(int dtype, int tile_x, int tile_y)
{
    const int per = dtype == XFDTD_F32 ? adjoint_occupancy<float>(tile_x, tile_y)
                                       : adjoint_occupancy<double>(tile_x, tile_y);
    return (int64_t)device_cus() * (per > 0 ? per : 1);
}

// z-chunk length of a z-march launch over (tile_x x tile_y) tiles.  The
// workgroups run in rounds of `slots` (all CUs, each with its resident
// workgroups), a round taking about z + 3 plane iterations (the chunk and its
// 3-plane warm-up), so the chunk minimises rounds x (z + 3) over z >= 4 (or
// the whole depth).  A chunk count just above a multiple of `slots` would
// leave most CUs idle in its last round (the 96^3 adjoint: 264 workgroups of
// 9 planes, 44.8 us per step, against 216 of 11 planes, 28.1 us).  Measured
// on 512x256x256 with 64x16 tiles, one workgroup per CU: 128-plane chunks
// (256 workgroups) beat 2048 chunks of 32 planes by 7 %.
int auto_zchunk(const xfdtd_grid &g, int tile_x, int tile_y, int64_t slots, int warm = 3, int min_z = 4)
{
    const int64_t ntx = (g.nx + tile_x - 1) / tile_x, nty = (g.ny + tile_y - 1) / tile_y;
    const int64_t tiles = ntx * nty, nz = g.nz;
    if (slots < 1) slots = 1;
    // beyond four full rounds of chunks, splitting further only adds warm-up
    const int64_t max_chunks = std::max<int64_t>(1, 4 * slots / tiles + 1);
    int64_t best_z = nz;
    double best = INFINITY;
    for (int64_t c = 1; c <= max_chunks && c <= nz; ++c) {
        const int64_t z = (nz + c - 1) / c;
        if (z < min_z && z < nz) break;
        const int64_t chunks = (nz + z - 1) / z;
        const int64_t rounds = (tiles * chunks + slots - 1) / slots;
        const double cost = (double)rounds * (double)(z + warm);
        if (cost < best) {
            best = cost;
            best_z = z;
        }
    }
    return (int)best_z;
}

int pick_zchunk(const xfdtd_grid &g, int tile_x, int tile_y, int dtype)
{
    const char *env = getenv("XFDTD_ZCHUNK");
    if (env && atoi(env) > 0) return atoi(env);
    // chunks down to one plane: a box too small to fill the CUs with 4-plane
    // chunks gains more from the extra workgroups than the warm-up costs
    // (measured: 32^3 7.7 -> 6.1 us per step, 64^3 10.8 -> 8.3)
    return auto_zchunk(g, tile_x, tile_y, fused_slots(dtype, tile_x, tile_y), 3, 1);
}

// FP64: 8-row tiles (the largest whose LDS fits a CU; measured on
// 512x256x256: 54.8 Gcell/s vs 48.1 with 4 rows, and better on 128^3 too).
// FP32: the 16-row tile (two rows per lane, fewer redundant halo cells per
// output) whenever its z-chunks stay long (>= 64 planes, so the 3-plane
// warm-up is amortised); 8-row tiles otherwise.  Measured on 512x256x256:
// 16 rows 96 Gcell/s vs 8 rows 88; on 128^3 the 8-row tile with 16-plane
// chunks is best.
int pick_tile_y(const xfdtd_grid &g, int tile_x, int dtype)
{
    // a box whose 8-row tiles give fewer workgroups than CUs even in 1-plane
    // chunks takes 4-row tiles (32^3: 6.0 -> 5.5 us per step)
    const int64_t tiles8 = (g.nx + tile_x - 1) / tile_x * ((g.ny + 7) / 8);
    if (tiles8 * g.nz < device_cus()) return 4;
    if (dtype == XFDTD_F64) return 8;
    return pick_zchunk(g, tile_x, 16, dtype) >= 64 ? 16 : 8;
}

// 32-column tiles for narrow boxes (nx <= 96) that they cover with fewer
// loaded columns (tile plus its 4 halo columns) than 64-column tiles: nx = 96
// loads 3 x 36 columns instead of 2 x 68, half of the second 64-wide tile
// being idle.  Measured: 96^3 20 us per step with 32-wide tiles vs 28 us;
// for wider boxes the better width depends on the z-chunking (xfdtd_tune
// times both).
int pick_tile_x(const xfdtd_grid &g)
{
    const int64_t c64 = (g.nx + 63) / 64 * 68, c32 = (g.nx + 31) / 32 * 36;
    return c32 < c64 && g.nx <= 96 ? 32 : 64;
}

// Two-step kernel: workgroups resident per CU, and the default tiling.  Its
// z-march needs 10 warm-up planes per chunk (each stage's 3 plus stage 2's lag
// of 3 and one more plane of E^{n+1}).
int64_t blocked2_slots(int dtype, int tile_x, int tile_y)
{
    const int per = dtype == XFDTD_F32 ? blocked2_occupancy<float>(tile_x, tile_y)
                                       : blocked2_occupancy<double>(tile_x, tile_y);
    return (int64_t)device_cus() * (per > 0 ? per : 1);
}

int blocked2_zchunk(const xfdtd_grid &g, int tile_x, int tile_y, int dtype = XFDTD_F32)
{
    return auto_zchunk(g, tile_x, tile_y, blocked2_slots(dtype, tile_x, tile_y), 10);
}

// 32x16 tiles while their z-chunks stay long (>= 64 planes), 32x8 otherwise
int pick_blocked2_tile_y(const xfdtd_grid &g)
{
    return blocked2_zchunk(g, 32, 16) >= 64 ? 16 : 8;
}

}  // namespace

struct xfdtd_s {
    xfdtd_grid g;
    double dt;
    double coeffs[12];
    int dtype;
    int flags;
    double w[15];  // folded weights as doubles equal to the dtype values
    Weights<float> wf;
    Weights<double> wd;
    void *fields[6];
    void *scratch[6];
    bool bound;
    bool have_scratch;
    hipStream_t stream;
    int tile_x, tile_y, zchunk;  // fused step
    int spp;                     // steps per pass of xfdtd_run: 1 (fused step) or 2 (two-step kernel)
    int btile_x, btile_y, bzchunk;  // two-step kernel
    int atile_x, atile_y, azchunk;  // adjoint step
    int device;
    double *partials;  // device, for reductions
    int npartials;
    double *apartials;  // device, adjoint per-workgroup gradient sums
    int napartials;
    double *grad_acc;   // device, 12 doubles
    hipStream_t aux;    // gradient backward: recompute stream (created on first use)
    int aux_device;
    // Workspaces filled by a forward pass and not yet consumed by a backward
    // pass (which overwrites their E snapshots): start, bytes used, n, seg.
    struct Tape {
        uintptr_t ws, bytes;
        int64_t n, seg;
    };
    std::vector<Tape> tapes;
    // xfdtd_run replays a captured graph of kGraphSteps steps (captured on
    // `cap` once per configuration and bound arrays, key `graph_key`)
    bool use_graph;
    hipStream_t cap;
    hipGraphExec_t gexec;
    std::array<uintptr_t, 20> graph_key;
    // instrumentation: counters, the launches of one replay of the run graph,
    // and the events that time xfdtd_run when timing is on
    struct RunCounts {
        int64_t in_place = 0, fused = 0, two_step = 0;
    };
    xfdtd_stats st{};
    RunCounts graph_counts;
    bool timing = false, t0_set = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int ev_device = -1;
};

namespace {

template <typename T>
Weights<T> fold(const xfdtd_s &h, double out[15])
{
    const double sp[3] = {h.g.dx, h.g.dy, h.g.dz};
    return fold_weights<T>(h.dt, h.coeffs, sp, out);
}

template <typename T>
Fields<T> as_fields(void *const p[6])
{
    Fields<T> f;
    for (int c = 0; c < 6; ++c) f.c[c] = (T *)p[c];
    return f;
}

Dims dims_of(const xfdtd_grid &g) { return Dims{(int)g.nx, (int)g.ny, (int)g.nz}; }

bool ranges_overlap(const void *a, uint64_t na, const void *b, uint64_t nb)
{
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

uint64_t raw_field_bytes(const xfdtd_s *h)
{
    return (uint64_t)h->g.nx * h->g.ny * h->g.nz * (h->dtype == XFDTD_F32 ? 4 : 8);
}

int check_bound(xfdtd_t h)
{
    if (!h) return fail(XFDTD_EINVAL, "null handle");
    if (!h->bound) return fail(XFDTD_ESTATE, "no fields bound (call xfdtd_bind first)");
    return XFDTD_OK;
}

// the folded weights of the handle's dtype
template <typename T>
const Weights<T> &weights_of(const xfdtd_s *h)
{
    return *(const Weights<T> *)(h->dtype == XFDTD_F32 ? (const void *)&h->wf : (const void *)&h->wd);
}

template <typename T>
int run_t(xfdtd_t h, int64_t n, hipStream_t st, xfdtd_s::RunCounts &cnt)
{
    const Dims d = dims_of(h->g);
    const Weights<T> &w = weights_of<T>(h);
    Fields<T> f = as_fields<T>(h->fields);
    if (!h->have_scratch) {
        for (int64_t s = 0; s < n; ++s) {
            HIP_TRY(launch_faraday<T>(f, d, w, st), "faraday launch");
            HIP_TRY(launch_ampere<T>(f, d, w, st), "ampere launch");
            ++cnt.in_place;
        }
        return XFDTD_OK;
    }
    Fields<T> s = as_fields<T>(h->scratch);
    if (h->spp == 2) {
        // Two steps per launch.  Out-of-place launches alternate between the
        // bound fields and the scratch arrays; their count is made even so
        // that the result ends in the bound fields: an odd n starts with one
        // in-place step (even number of two-step launches) or one fused step
        // (odd number); an even n with an odd number of two-step launches
        // does one of them as two fused steps.
        Fields<T> a = f, b = s;
        int64_t pairs = n / 2;
        auto fused = [&]() -> int {
            HIP_TRY(launch_fused<T>(a, b, d, w, h->tile_x, h->tile_y, h->zchunk, st), "fused launch");
            std::swap(a, b);
            ++cnt.fused;
            return XFDTD_OK;
        };
        int rc = XFDTD_OK;
        if ((n & 1) && pairs % 2 == 0) {
            HIP_TRY(launch_faraday<T>(a, d, w, st), "faraday launch");
            HIP_TRY(launch_ampere<T>(a, d, w, st), "ampere launch");
            ++cnt.in_place;
        } else if (n & 1) {
            rc = fused();
        } else if (pairs % 2 == 1) {
            rc = fused();
            if (!rc) rc = fused();
            --pairs;
        }
        if (rc) return rc;
        for (int64_t i = 0; i < pairs; ++i) {
            HIP_TRY(launch_blocked2<T>(a, b, d, w, h->btile_x, h->btile_y, h->bzchunk, st),
                    "two-step launch");
            std::swap(a, b);
            ++cnt.two_step;
        }
        return XFDTD_OK;
    }
    int64_t left = n;
    if (left & 1) {  // odd count: one in-place step keeps the result in `fields`
        HIP_TRY(launch_faraday<T>(f, d, w, st), "faraday launch");
        HIP_TRY(launch_ampere<T>(f, d, w, st), "ampere launch");
        ++cnt.in_place;
        --left;
    }
    for (; left > 0; left -= 2) {
        HIP_TRY(launch_fused<T>(f, s, d, w, h->tile_x, h->tile_y, h->zchunk, st), "fused launch");
        HIP_TRY(launch_fused<T>(s, f, d, w, h->tile_x, h->tile_y, h->zchunk, st), "fused launch");
        cnt.fused += 2;
    }
    return XFDTD_OK;
}

// The two events that time xfdtd_run, on the handle's device.
int ensure_timing_events(xfdtd_s *h)
{
    if (h->t0 && h->t1 && h->ev_device == h->device) return XFDTD_OK;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != h->device) HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    hipError_t e = hipSuccess;
    for (hipEvent_t *ev : {&h->t0, &h->t1}) {
        if (*ev) hipEventDestroy(*ev);
        *ev = nullptr;
        if (e == hipSuccess) e = hipEventCreate(ev);
    }
    if (cur != h->device) hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "creating the timing events");
    h->ev_device = h->device;
    h->t0_set = false;
    return XFDTD_OK;
}

// algorithmic HBM bytes of one step of `values` values per cell
double model_bytes(const xfdtd_s *h, int64_t steps, int values)
{
    const double cells = (double)h->g.nx * (double)h->g.ny * (double)h->g.nz;
    return (double)steps * cells * values * (h->dtype == XFDTD_F32 ? 4.0 : 8.0);
}

}  // namespace

namespace {

// Steps per replay of the captured run graph: a multiple of four, so that the
// graph (like every xfdtd_run call) leaves the result in the bound fields with
// only out-of-place launches whichever kernel runs.
constexpr int64_t kGraphSteps = 32;

std::array<uintptr_t, 20> run_graph_key(const xfdtd_s *h)
{
    std::array<uintptr_t, 20> k{};
    for (int c = 0; c < 6; ++c) {
        k[c] = (uintptr_t)h->fields[c];
        k[6 + c] = (uintptr_t)h->scratch[c];
    }
    k[12] = (uintptr_t)h->spp;
    k[13] = ((uintptr_t)h->tile_x << 16) | (uintptr_t)h->tile_y;
    k[14] = (uintptr_t)h->zchunk;
    k[15] = ((uintptr_t)h->btile_x << 16) | (uintptr_t)h->btile_y;
    k[16] = (uintptr_t)h->bzchunk;
    k[17] = (uintptr_t)h->have_scratch;
    k[18] = (uintptr_t)h->device;
    k[19] = 1;  // a graph is held
    return k;
}

void drop_run_graph(xfdtd_s *h)
{
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    h->graph_key = {};
}

// Captures kGraphSteps steps of xfdtd_run into a graph (on the handle's
// capture stream) unless the cached graph was captured with the same bound
// arrays and launch configuration.
template <typename F>
int ensure_run_graph(xfdtd_s *h, F &&eager)
{
    const std::array<uintptr_t, 20> key = run_graph_key(h);
    if (h->gexec && h->graph_key == key) return XFDTD_OK;
    if (h->gexec) HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");  // a replay may be queued
    drop_run_graph(h);
    if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    xfdtd_s::RunCounts cnt;
    const int rc = eager(kGraphSteps, h->cap, cnt);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap, &graph);
    if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&h->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        h->gexec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    h->graph_key = key;
    h->graph_counts = cnt;
    ++h->st.graph_captures;
    xlog("run graph captured: %lld steps (%lld one-step, %lld two-step launches, %lld in-place steps)",
         (long long)kGraphSteps, (long long)cnt.fused, (long long)cnt.two_step, (long long)cnt.in_place);
    return XFDTD_OK;
}

// Tilings chosen by xfdtd_tune, per (nx, ny, nz, dtype, device): steps per
// pass, then (tile_x, tile_y, zchunk) of the kernel that won.
std::mutex g_tune_mu;
std::map<std::array<int64_t, 5>, std::array<int, 4>> g_tune;

std::array<int64_t, 5> tune_key(const xfdtd_s *h)
{
    return {h->g.nx, h->g.ny, h->g.nz, (int64_t)h->dtype, (int64_t)h->device};
}

// key of a box in the tuning file
std::string tune_file_key(const xfdtd_s *h)
{
    return std::string("single:") + (h->dtype == XFDTD_F32 ? "f32:" : "f64:") + std::to_string(h->g.nx) + "x" +
           std::to_string(h->g.ny) + "x" + std::to_string(h->g.nz);
}

// a stored (steps per pass, tile_x, tile_y, z-chunk) this box can launch
bool valid_tuning(const xfdtd_s *h, const std::vector<int> &c)
{
    if (c.size() != 4 || c[3] < 1 || c[3] > h->g.nz) return false;
    if (c[0] == 2)
        return h->have_scratch && (h->dtype == XFDTD_F32 ? c[1] == 32 && (c[2] == 8 || c[2] == 16)
                                                         : c[1] == 24 && c[2] == 8);
    return c[0] == 1 && (c[1] == 32 || c[1] == 64) &&
           (c[2] == 4 || c[2] == 8 || (c[2] == 16 && h->dtype == XFDTD_F32));
}

// z-chunk lengths worth timing for a kernel whose chunks start with `warm`
// warm-up planes: the cost model's choice, the whole depth and a few splits
std::vector<int> zchunk_candidates(const xfdtd_grid &g, int model)
{
    const int64_t nz = g.nz;
    // a model choice below 4 planes (a small box) adds the other short chunks
    const bool shortz = model < 4;
    const int64_t zs[11] = {model, nz, (nz + 1) / 2, (nz + 3) / 4, (nz + 7) / 8, 16, 32,
                            shortz ? 1 : 0, shortz ? 2 : 0, shortz ? 3 : 0, shortz ? 4 : 0};
    std::vector<int> out;
    for (int64_t z : zs) {
        if (z > nz) z = nz;
        if (z < 1 || (z < 4 && z < nz && !shortz)) continue;
        if (std::find(out.begin(), out.end(), (int)z) == out.end()) out.push_back((int)z);
    }
    return out;
}

// Times each candidate with launches fields -> scratch (the bound state is
// only read) and keeps the fastest per step: one-step tilings and the
// two-step kernel's (two steps per launch).
template <typename T>
int tune_t(xfdtd_t h, double *best_ms)
{
    const Dims d = dims_of(h->g);
    const Weights<T> &w = weights_of<T>(h);
    const Fields<T> f = as_fields<T>(h->fields), s = as_fields<T>(h->scratch);
    std::vector<std::array<int, 4>> cands;  // steps per launch, tile_x, tile_y, zchunk
    auto fits = [&](int tx, int ty, int z) {
        return ((d.nx + tx - 1) / tx) * (int64_t)((d.ny + ty - 1) / ty) * ((h->g.nz + z - 1) / z) <= 0x7fffffff;
    };
    // a box one plane deep: every one-step tiling runs the plane kernel, and
    // the two-step kernel's warm-up makes it several times slower there
    if (h->g.nz == 1) cands.push_back({1, 64, sizeof(T) == 4 ? 16 : 8, 1});
    for (int tx : {64, 32}) {
        if (h->g.nz == 1) break;
        std::vector<int> tys = {sizeof(T) == 4 ? 8 : 4, sizeof(T) == 4 ? 16 : 8};
        // FP32 boxes too small for 4-plane chunks of 8-row tiles: 4-row tiles too
        if (sizeof(T) == 4 && auto_zchunk(h->g, tx, 8, fused_slots(h->dtype, tx, 8), 3, 1) < 4)
            tys.insert(tys.begin(), 4);
        for (int ty : tys)
            for (int z : zchunk_candidates(h->g, auto_zchunk(h->g, tx, ty, fused_slots(h->dtype, tx, ty), 3, 1)))
                if (fits(tx, ty, z)) cands.push_back({1, tx, ty, z});
    }
    if (h->g.nz == 1) {
    } else if (sizeof(T) == 4) {
        for (int ty : {8, 16})
            for (int z : zchunk_candidates(h->g, blocked2_zchunk(h->g, 32, ty)))
                if (fits(32, ty, z)) cands.push_back({2, 32, ty, z});
    } else {
        for (int z : zchunk_candidates(h->g, blocked2_zchunk(h->g, 24, 8, XFDTD_F64)))
            if (fits(24, 8, z)) cands.push_back({2, 24, 8, z});
    }
    // Launches alternate between the scratch arrays and a temporary third
    // state (a copy of the fields), the memory pattern of xfdtd_run, whose
    // every launch reads what the previous one wrote: timing launches that
    // all read the unchanged fields lets a state of about the size of the
    // last-level cache stay there and favours the wrong kernel (128x256x256
    // FP32: the one-step kernel timed at 65.7 us per step ran 90.3 us).
    // Without the temporary (allocation failed) they run fields -> scratch.
    struct Temp {
        void *p = nullptr;
        ~Temp()
        {
            if (p) hipFree(p);
        }
    } temp;
    const size_t esz = sizeof(T), fbytes = ((size_t)h->g.nx * h->g.ny * h->g.nz * esz + 255) / 256 * 256;
    Fields<T> t = s;
    if (hipMalloc(&temp.p, 6 * fbytes) == hipSuccess) {
        for (int c = 0; c < 6; ++c) {
            t.c[c] = (T *)((char *)temp.p + (size_t)c * fbytes);
            HIP_TRY(hipMemcpyAsync(t.c[c], f.c[c], (size_t)h->g.nx * h->g.ny * h->g.nz * esz,
                                   hipMemcpyDeviceToDevice, h->stream),
                    "hipMemcpyAsync");
        }
    } else {
        (void)hipGetLastError();
        temp.p = nullptr;
        t = f;
    }
    // The temporary is freed once the stream has drained (before Temp goes).
    struct Drain {
        hipStream_t s;
        ~Drain() { hipStreamSynchronize(s); }
    } drain{h->stream};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    // Two interleaved passes over the candidates (slow drifts of the clock
    // hit all of them alike); each timing covers about 2 ms of launches and
    // a candidate keeps its faster pass.
    std::vector<double> per(cands.size(), INFINITY);
    std::vector<int> reps(cands.size(), 0);
    for (int pass = 0; pass < 2 && he == hipSuccess; ++pass)
        for (size_t i = 0; i < cands.size() && he == hipSuccess; ++i) {
            const auto &c = cands[i];
            auto timed = [&](int r, float *ms) {
                hipError_t e = hipEventRecord(e0, h->stream);
                for (int q = 0; q < r && e == hipSuccess; ++q) {
                    // without the temporary, every launch reads the fields
                    const bool back = temp.p && (q & 1);
                    const Fields<T> &in = back ? s : t, &out = back ? t : s;
                    e = c[0] == 2 ? launch_blocked2<T>(in, out, d, w, c[1], c[2], c[3], h->stream)
                                  : launch_fused<T>(in, out, d, w, c[1], c[2], c[3], h->stream);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
                return e;
            };
            float ms = 0.f;
            if (reps[i] == 0) {  // warm-up launch, whose time sizes the repetitions
                he = timed(1, &ms);
                reps[i] = (int)std::min(50.0, std::max(3.0, ceil(2.0 / std::max(ms, 1e-3f))));
            }
            if (he == hipSuccess) he = timed(reps[i], &ms);
            if (he == hipSuccess) per[i] = std::min(per[i], (double)ms / reps[i] / c[0]);
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (he != hipSuccess) return hip_fail(he, "tuning launch");
    double best = INFINITY;
    std::array<int, 4> bestc = {h->spp, 0, 0, 0};
    for (size_t i = 0; i < cands.size(); ++i)
        if (per[i] < best) {
            best = per[i];
            bestc = cands[i];
        }
    if (bestc[1] == 0) return fail(XFDTD_EHIP, "no tiling could be timed");
    if (log_on())
        for (size_t i = 0; i < cands.size(); ++i)
            xlog("tune candidate %s %dx%d tiles, z-chunk %d: %.2f us per step", cands[i][0] == 2 ? "two-step" : "one-step",
                 cands[i][1], cands[i][2], cands[i][3], per[i] * 1e3);
    h->spp = bestc[0];
    if (bestc[0] == 2) {
        h->btile_x = bestc[1];
        h->btile_y = bestc[2];
        h->bzchunk = bestc[3];
    } else {
        h->tile_x = bestc[1];
        h->tile_y = bestc[2];
        h->zchunk = bestc[3];
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(h)] = bestc;
    }
    ++h->st.tunes;
    tune_cache_store(tune_file_key(h), {bestc[0], bestc[1], bestc[2], bestc[3]});
    xlog("tune %lldx%lldx%lld %s: %zu candidates, best %s %dx%d tiles, z-chunk %d, %.2f us per step",
         (long long)h->g.nx, (long long)h->g.ny, (long long)h->g.nz, h->dtype == XFDTD_F32 ? "FP32" : "FP64",
         cands.size(), bestc[0] == 2 ? "two-step" : "one-step", bestc[1], bestc[2], bestc[3], best * 1e3);
    if (best_ms) *best_ms = best;
    return XFDTD_OK;
}

}  // namespace

extern "C" {

int xfdtd_abi_version(void) { return 2; }

const char *xfdtd_last_error(void) { return g_err; }

int xfdtd_consistent_alpha(double coeffs[12])
{
    return guarded([&]() -> int {
        if (!coeffs_ok(coeffs)) return fail(XFDTD_EINVAL, "coeffs must be 12 finite values");
        for (int a = 0; a < 3; ++a)
            coeffs[4 * a] = 1.0 - 2.0 * coeffs[4 * a + 1] - 2.0 * coeffs[4 * a + 2] - 3.0 * coeffs[4 * a + 3];
        return XFDTD_OK;
    });
}

int xfdtd_cfl_limit(const xfdtd_grid *g, const double coeffs[12], double *dt_max, double *f_min,
                    double *f_max)
{
    return guarded([&]() -> int {
        if (!grid_ok(g)) return fail(XFDTD_EINVAL, "invalid grid");
        if (!coeffs_ok(coeffs)) return fail(XFDTD_EINVAL, "coeffs must be 12 finite values");
        const double sp[3] = {g->dx, g->dy, g->dz};
        double lo, hi;
        f_range(sp, coeffs, &lo, &hi);
        if (f_min) *f_min = lo;
        if (f_max) *f_max = hi;
        if (!(hi > 0.0)) {
            if (dt_max) *dt_max = INFINITY;
            return fail(XFDTD_EUNSTABLE, "F_max = %g <= 0: no stable positive frequency range", hi);
        }
        if (dt_max) *dt_max = 1.0 / sqrt(hi);
        return XFDTD_OK;
    });
}

int xfdtd_create(const xfdtd_grid *g, double dt, const double coeffs[12], int dtype,
                 int allow_unstable, xfdtd_t *out)
{
    return guarded([&]() -> int {
        if (!out) return fail(XFDTD_EINVAL, "out is null");
        *out = nullptr;
        if (!grid_ok(g)) return fail(XFDTD_EINVAL, "invalid grid (sizes >= 1, spacings > 0)");
        if (!coeffs_ok(coeffs)) return fail(XFDTD_EINVAL, "coeffs must be 12 finite values");
        if (!(dt > 0) || !isfinite(dt)) return fail(XFDTD_EINVAL, "dt must be finite and > 0");
        if (dtype != XFDTD_F32 && dtype != XFDTD_F64) return fail(XFDTD_EINVAL, "dtype must be XFDTD_F32 or XFDTD_F64");
        const double sp[3] = {g->dx, g->dy, g->dz};
        double lo, hi;
        f_range(sp, coeffs, &lo, &hi);
        if (!allow_unstable) {
            const double tol = 1e-12 * fmax(1.0, fabs(hi));
            if (lo < -tol) return fail(XFDTD_EUNSTABLE, "F_min = %.17g < 0: dispersion relation ill-defined", lo);
            if (dt * dt * hi > 1.0 + 1e-12)
                return fail(XFDTD_EUNSTABLE, "dt = %.17g exceeds the stability bound %.17g", dt, 1.0 / sqrt(hi));
        }
        xfdtd_s *h = new (std::nothrow) xfdtd_s();
        if (!h) return fail(XFDTD_EINVAL, "out of host memory");
        h->g = *g;
        h->dt = dt;
        memcpy(h->coeffs, coeffs, sizeof h->coeffs);
        h->dtype = dtype;
        h->flags = 0;
        for (int a = 0; a < 3; ++a) {
            const double al = 1.0 - 2.0 * coeffs[4 * a + 1] - 2.0 * coeffs[4 * a + 2] - 3.0 * coeffs[4 * a + 3];
            if (fabs(al - coeffs[4 * a]) > 1e-12) h->flags |= XFDTD_WARN_ALPHA;
        }
        if (dtype == XFDTD_F32)
            h->wf = fold<float>(*h, h->w);
        else
            h->wd = fold<double>(*h, h->w);
        h->bound = false;
        h->have_scratch = false;
        h->stream = nullptr;
        h->tile_x = pick_tile_x(*g);
        const char *tx = getenv("XFDTD_TILE_X");
        if (tx && (atoi(tx) == 32 || atoi(tx) == 64)) h->tile_x = atoi(tx);
        h->tile_y = pick_tile_y(*g, h->tile_x, dtype);
        const char *ty = getenv("XFDTD_TILE_Y");
        if (ty && (atoi(ty) == 4 || atoi(ty) == 8 || (atoi(ty) == 16 && dtype == XFDTD_F32))) h->tile_y = atoi(ty);
        h->zchunk = pick_zchunk(*g, h->tile_x, h->tile_y, dtype);
        // a box one plane deep runs the plane kernel (64x16 tiles in FP32,
        // 64x8 in FP64) whatever the tiling; report that one
        if (g->nz == 1) {
            h->tile_x = 64;
            h->tile_y = dtype == XFDTD_F32 ? 16 : 8;
            h->zchunk = 1;
        }
    // two-step kernel: 32-column tiles (FP32), 24 x 8 (FP64); the default
    // steps per pass can be overridden with XFDTD_STEPS_PER_PASS (1 or 2)
    h->btile_x = dtype == XFDTD_F32 ? 32 : 24;
    h->btile_y = dtype == XFDTD_F32 ? pick_blocked2_tile_y(*g) : 8;
    h->bzchunk = blocked2_zchunk(*g, h->btile_x, h->btile_y, dtype);
    // Two steps per pass by default for FP32 boxes of at least 2^23 cells and
    // 32 planes; below that the one-step kernel measured as fast or faster
    // (32^3 .. 128^3: its shorter z-march warm-up and smaller halo win while
    // the two-step kernel's halved traffic does not matter; 192^2 x 352 and
    // up: two-step; boxes a few planes deep pay the two-step kernel's 10
    // warm-up planes per chunk: 4096^2 x 1, 9.1 Gcell-updates/s against 73
    // for the plane kernel).  xfdtd_tune decides per box.
    h->spp = dtype == XFDTD_F32 && (double)g->nx * g->ny * g->nz >= (double)(1 << 23) && g->nz >= 32 ? 2 : 1;
    const char *spp = getenv("XFDTD_STEPS_PER_PASS");
    if (spp && (atoi(spp) == 1 || atoi(spp) == 2)) h->spp = atoi(spp);
    const char *bty = getenv("XFDTD_BLK_TILE_Y");
    if (dtype == XFDTD_F32 && bty && (atoi(bty) == 8 || atoi(bty) == 16)) {
        h->btile_y = atoi(bty);
        h->bzchunk = blocked2_zchunk(*g, h->btile_x, h->btile_y);
    }
    const char *bzc = getenv("XFDTD_BLK_ZCHUNK");
    if (bzc && atoi(bzc) > 0) h->bzchunk = atoi(bzc);
        // adjoint: 64x8 tiles for FP32 (64x4 for FP64, whose 64x8 tile does not
        // fit in LDS), its own z-chunk for that tile height
        h->atile_x = pick_tile_x(*g);
        const char *atx = getenv("XFDTD_ADJ_TILE_X");
        if (atx && (atoi(atx) == 32 || atoi(atx) == 64)) h->atile_x = atoi(atx);
        h->atile_y = dtype == XFDTD_F64 && h->atile_x == 64 ? 4 : 8;
        const char *aty = getenv("XFDTD_ADJ_TILE_Y");
        if (aty && (atoi(aty) == 4 || (atoi(aty) == 8 && (dtype == XFDTD_F32 || h->atile_x == 32))))
            h->atile_y = atoi(aty);
        h->azchunk = auto_zchunk(*g, h->atile_x, h->atile_y, adjoint_slots(dtype, h->atile_x, h->atile_y));
        if (getenv("XFDTD_ZCHUNK") && atoi(getenv("XFDTD_ZCHUNK")) > 0) h->azchunk = atoi(getenv("XFDTD_ZCHUNK"));
        const char *azc = getenv("XFDTD_ADJ_ZCHUNK");
        if (azc && atoi(azc) > 0) h->azchunk = atoi(azc);
        h->device = -1;
        h->partials = nullptr;
        h->npartials = 0;
        h->apartials = nullptr;
        h->napartials = 0;
        h->grad_acc = nullptr;
        h->aux = nullptr;
        h->aux_device = -1;
        const char *gr = getenv("XFDTD_GRAPH");
        h->use_graph = !(gr && atoi(gr) == 0);
        h->cap = nullptr;
        h->gexec = nullptr;
        h->graph_key = {};
        xlog("create %lldx%lldx%lld %s: one-step %dx%d tiles, z-chunk %d; two-step %dx%d tiles, z-chunk %d; "
             "%d step%s per pass; adjoint %dx%d tiles, z-chunk %d; run graph %s",
             (long long)g->nx, (long long)g->ny, (long long)g->nz, dtype == XFDTD_F32 ? "FP32" : "FP64", h->tile_x,
             h->tile_y, h->zchunk, h->btile_x, h->btile_y, h->bzchunk, h->spp, h->spp == 2 ? "s" : "", h->atile_x,
             h->atile_y, h->azchunk, h->use_graph ? "on" : "off");
        *out = h;
        return XFDTD_OK;
    });
}

void xfdtd_destroy(xfdtd_t h)
{
    // nothing here allocates or throws
    if (!h) return;
    if (h->partials || h->apartials || h->grad_acc) hipStreamSynchronize(h->stream);
    if (h->aux) {
        hipStreamSynchronize(h->aux);
        hipStreamDestroy(h->aux);
    }
    if (h->partials) hipFree(h->partials);
    if (h->apartials) hipFree(h->apartials);
    if (h->grad_acc) hipFree(h->grad_acc);
    if (h->gexec) {
        hipStreamSynchronize(h->stream);  // a replay may still be queued
        hipGraphExecDestroy(h->gexec);
    }
    if (h->cap) hipStreamDestroy(h->cap);
    if (h->t0) hipEventDestroy(h->t0);
    if (h->t1) hipEventDestroy(h->t1);
    delete h;
}

int xfdtd_flags(xfdtd_t h) { return h ? h->flags : 0; }

int xfdtd_bind(xfdtd_t h, void *const fields[6], void *const scratch[6], void *stream)
{
    return guarded([&]() -> int {
        if (!h) return fail(XFDTD_EINVAL, "null handle");
        if (!fields) return fail(XFDTD_EINVAL, "fields is null");
        const size_t esz = h->dtype == XFDTD_F32 ? 4 : 8;
        const size_t bytes = (size_t)h->g.nx * h->g.ny * h->g.nz * esz;
        void *all[12];
        int nall = 0;
        for (int c = 0; c < 6; ++c) {
            if (!fields[c]) return fail(XFDTD_EINVAL, "fields[%d] is null", c);
            if ((uintptr_t)fields[c] % 16) return fail(XFDTD_EINVAL, "fields[%d] not 16-byte aligned", c);
            all[nall++] = fields[c];
        }
        if (scratch) {
            for (int c = 0; c < 6; ++c) {
                if (!scratch[c]) return fail(XFDTD_EINVAL, "scratch[%d] is null (pass scratch = NULL for none)", c);
                if ((uintptr_t)scratch[c] % 16) return fail(XFDTD_EINVAL, "scratch[%d] not 16-byte aligned", c);
                all[nall++] = scratch[c];
            }
        }
        for (int a = 0; a < nall; ++a)
            for (int b = a + 1; b < nall; ++b) {
                const uintptr_t pa = (uintptr_t)all[a], pb = (uintptr_t)all[b];
                if (pa < pb + bytes && pb < pa + bytes) return fail(XFDTD_EINVAL, "bound arrays %d and %d overlap", a, b);
            }
        if (h->gexec) {  // the cached run graph holds the old arrays: drop it if they change
            bool same = h->stream == (hipStream_t)stream && h->have_scratch == (scratch != nullptr);
            for (int c = 0; c < 6 && same; ++c)
                same = h->fields[c] == fields[c] && h->scratch[c] == (scratch ? scratch[c] : nullptr);
            if (!same) {
                HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
                drop_run_graph(h);
            }
        }
        for (int c = 0; c < 6; ++c) {
            h->fields[c] = fields[c];
            h->scratch[c] = scratch ? scratch[c] : nullptr;
        }
        h->have_scratch = scratch != nullptr;
        h->stream = (hipStream_t)stream;
        h->bound = true;
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        h->device = dev;
        return XFDTD_OK;
    });
}

int xfdtd_step_faraday(xfdtd_t h)
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        const Dims d = dims_of(h->g);
        if (h->dtype == XFDTD_F32)
            HIP_TRY(launch_faraday<float>(as_fields<float>(h->fields), d, h->wf, h->stream), "faraday launch");
        else
            HIP_TRY(launch_faraday<double>(as_fields<double>(h->fields), d, h->wd, h->stream), "faraday launch");
        return XFDTD_OK;
    });
}

int xfdtd_step_ampere(xfdtd_t h)
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        const Dims d = dims_of(h->g);
        if (h->dtype == XFDTD_F32)
            HIP_TRY(launch_ampere<float>(as_fields<float>(h->fields), d, h->wf, h->stream), "ampere launch");
        else
            HIP_TRY(launch_ampere<double>(as_fields<double>(h->fields), d, h->wd, h->stream), "ampere launch");
        return XFDTD_OK;
    });
}

int xfdtd_step_ampere_current(xfdtd_t h, const void *const J[3])
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        if (!J || !J[0] || !J[1] || !J[2]) return fail(XFDTD_EINVAL, "J must be three device arrays");
        const size_t esz = h->dtype == XFDTD_F32 ? 4 : 8;
        for (int c = 0; c < 3; ++c) {
            if ((uintptr_t)J[c] % esz) return fail(XFDTD_EINVAL, "J[%d] is misaligned", c);
            for (int q = 0; q < 3; ++q)  // E is updated in place while J is read
                if (ranges_overlap(J[c], raw_field_bytes(h), h->fields[q], raw_field_bytes(h)))
                    return fail(XFDTD_EINVAL, "J[%d] overlaps the bound E[%d]", c, q);
        }
        const Dims d = dims_of(h->g);
        if (h->dtype == XFDTD_F32) {
            const float *j[3] = {(const float *)J[0], (const float *)J[1], (const float *)J[2]};
            HIP_TRY(launch_ampere<float>(as_fields<float>(h->fields), d, h->wf, h->stream, j, (float)h->dt),
                    "ampere launch");
        } else {
            const double *j[3] = {(const double *)J[0], (const double *)J[1], (const double *)J[2]};
            HIP_TRY(launch_ampere<double>(as_fields<double>(h->fields), d, h->wd, h->stream, j, h->dt),
                    "ampere launch");
        }
        return XFDTD_OK;
    });
}

int xfdtd_run(xfdtd_t h, int64_t n)
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        if (n < 0) return fail(XFDTD_EINVAL, "n must be >= 0");
        Range range("xfdtd_run");
        auto eager = [&](int64_t m, hipStream_t st, xfdtd_s::RunCounts &cnt) {
            return h->dtype == XFDTD_F32 ? run_t<float>(h, m, st, cnt) : run_t<double>(h, m, st, cnt);
        };
        // inside a capture of the caller's stream the launches go straight
        // into the caller's graph
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(h->stream, &cs), "hipStreamIsCapturing");
        const bool capturing = cs != hipStreamCaptureStatusNone;
        const bool timed = h->timing && !capturing && n > 0;
        if (timed) {
            rc = ensure_timing_events(h);
            if (rc) return rc;
            if (!h->t0_set) HIP_TRY(hipEventRecord(h->t0, h->stream), "hipEventRecord");
            h->t0_set = true;
        }
        const int64_t units = h->use_graph && !capturing ? n / kGraphSteps : 0;
        xfdtd_s::RunCounts cnt;
        if (units > 0) {
            rc = ensure_run_graph(h, eager);
            if (rc) return rc;
            for (int64_t u = 0; u < units; ++u) HIP_TRY(hipGraphLaunch(h->gexec, h->stream), "hipGraphLaunch");
            cnt.in_place = units * h->graph_counts.in_place;
            cnt.fused = units * h->graph_counts.fused;
            cnt.two_step = units * h->graph_counts.two_step;
            h->st.graph_replays += units;
        }
        // the remaining steps (all of them without a graph) are launched
        // directly; each part leaves the result in the bound fields, and the
        // steps are the same kernels in the same order either way
        rc = eager(n - units * kGraphSteps, h->stream, cnt);
        if (rc) return rc;
        if (timed) HIP_TRY(hipEventRecord(h->t1, h->stream), "hipEventRecord");
        ++h->st.run_calls;
        h->st.steps += n;
        h->st.in_place_steps += cnt.in_place;
        h->st.fused_launches += cnt.fused;
        h->st.two_step_launches += cnt.two_step;
        h->st.model_bytes += model_bytes(h, n, 12);
        return XFDTD_OK;
    });
}

int xfdtd_run_checked(xfdtd_t h, int64_t n, int64_t every, int64_t *done)
{
    return guarded([&]() -> int {
        if (done) *done = 0;
        int rc = check_bound(h);
        if (rc) return rc;
        if (n < 0 || every < 1) return fail(XFDTD_EINVAL, "need n >= 0 and every >= 1");
        for (int64_t s = 0; s < n;) {
            const int64_t m = std::min(every, n - s);
            rc = xfdtd_run(h, m);
            if (rc) return rc;
            s += m;
            if (done) *done = s;
            double out[3];
            rc = xfdtd_divergence_max(h, nullptr, nullptr, out);
            if (rc == XFDTD_ENONFINITE)
                return fail(XFDTD_ENONFINITE, "%.0f non-finite field values after %lld steps", out[2], (long long)s);
            if (rc) return rc;
        }
        return XFDTD_OK;
    });
}

int xfdtd_get_stats(xfdtd_t h, xfdtd_stats *out)
{
    return guarded([&]() -> int {
        if (!h || !out) return fail(XFDTD_EINVAL, "null argument");
        *out = h->st;
        out->elapsed_ms = -1.0;
        out->gcells_per_s = -1.0;
        if (h->timing && h->t0_set) {
            HIP_TRY(hipEventSynchronize(h->t1), "hipEventSynchronize");
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->t0, h->t1), "hipEventElapsedTime");
            const double cells = (double)h->g.nx * (double)h->g.ny * (double)h->g.nz;
            out->elapsed_ms = ms;
            out->gcells_per_s = ms > 0 ? (double)h->st.steps * cells / ((double)ms * 1e-3) / 1e9 : -1.0;
        }
        return XFDTD_OK;
    });
}

int xfdtd_reset_stats(xfdtd_t h, int timing)
{
    return guarded([&]() -> int {
        if (!h) return fail(XFDTD_EINVAL, "null handle");
        h->st = xfdtd_stats{};
        h->timing = timing != 0;
        h->t0_set = false;
        return XFDTD_OK;
    });
}

int xfdtd_tune(xfdtd_t h, int force, double *best_ms)
{
    return guarded([&]() -> int {
        const int rc = check_bound(h);
        if (rc) return rc;
        if (!h->have_scratch) return fail(XFDTD_ESTATE, "tuning times the fused step: bind scratch arrays");
        Range range("xfdtd_tune");
        if (!force) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(tune_key(h));
            std::vector<int> file;
            if (it == g_tune.end() && tune_cache_lookup(tune_file_key(h), file) && valid_tuning(h, file)) {
                it = g_tune.emplace(tune_key(h), std::array<int, 4>{file[0], file[1], file[2], file[3]}).first;
                xlog("tune %s: taken from the tuning file (%s %dx%d tiles, z-chunk %d)", tune_file_key(h).c_str(),
                     file[0] == 2 ? "two-step" : "one-step", file[1], file[2], file[3]);
            }
            if (it != g_tune.end()) {
                const std::array<int, 4> &c = it->second;
                h->spp = c[0];
                (c[0] == 2 ? h->btile_x : h->tile_x) = c[1];
                (c[0] == 2 ? h->btile_y : h->tile_y) = c[2];
                (c[0] == 2 ? h->bzchunk : h->zchunk) = c[3];
                if (best_ms) *best_ms = -1.0;
                return XFDTD_OK;
            }
        }
        return h->dtype == XFDTD_F32 ? tune_t<float>(h, best_ms) : tune_t<double>(h, best_ms);
    });
}

int xfdtd_launch_config(xfdtd_t h, int *tile_x, int *tile_y, int *zchunk, int *workgroups)
{
    return guarded([&]() -> int {
        if (!h) return fail(XFDTD_EINVAL, "null handle");
        if (tile_x) *tile_x = h->tile_x;
        if (tile_y) *tile_y = h->tile_y;
        if (zchunk) *zchunk = h->zchunk;
        if (workgroups) {
            const int64_t ntx = (h->g.nx + h->tile_x - 1) / h->tile_x, nty = (h->g.ny + h->tile_y - 1) / h->tile_y;
            const int64_t nzc = (h->g.nz + h->zchunk - 1) / h->zchunk;
            *workgroups = (int)(ntx * nty * nzc);
        }
        return XFDTD_OK;
    });
}

int xfdtd_set_steps_per_pass(xfdtd_t h, int steps)
{
    return guarded([&]() -> int {
        if (!h) return fail(XFDTD_EINVAL, "null handle");
        if (steps != 1 && steps != 2) return fail(XFDTD_EINVAL, "steps per pass must be 1 or 2");
        h->spp = steps;
        return XFDTD_OK;
    });
}

int xfdtd_launch_config2(xfdtd_t h, int *steps_per_pass, int *tile_x, int *tile_y, int *zchunk, int *workgroups)
{
    return guarded([&]() -> int {
        if (!h) return fail(XFDTD_EINVAL, "null handle");
        if (steps_per_pass) *steps_per_pass = h->spp;
        if (tile_x) *tile_x = h->btile_x;
        if (tile_y) *tile_y = h->btile_y;
        if (zchunk) *zchunk = h->bzchunk;
        if (workgroups) {
            const int64_t ntx = (h->g.nx + h->btile_x - 1) / h->btile_x;
            const int64_t nty = (h->g.ny + h->btile_y - 1) / h->btile_y;
            *workgroups = (int)(ntx * nty * ((h->g.nz + h->bzchunk - 1) / h->bzchunk));
        }
        return XFDTD_OK;
    });
}

int xfdtd_get_weights(xfdtd_t h, double w[15], int *nw)
{
    return guarded([&]() -> int {
        if (!h || !w) return fail(XFDTD_EINVAL, "null argument");
        memcpy(w, h->w, sizeof h->w);
        if (nw) *nw = 15;
        return XFDTD_OK;
    });
}

int xfdtd_dispersion(const xfdtd_grid *g, double dt, const double coeffs[12], const double *k, int64_t n,
                     double *omega, double *vph, double *vg, void *stream)
{
    return guarded([&]() -> int {
        if (!grid_ok(g)) return fail(XFDTD_EINVAL, "invalid grid");
        if (!coeffs_ok(coeffs)) return fail(XFDTD_EINVAL, "coeffs must be 12 finite values");
        if (!(dt > 0) || !isfinite(dt)) return fail(XFDTD_EINVAL, "dt must be finite and > 0");
        if (n < 0) return fail(XFDTD_EINVAL, "n must be >= 0");
        if (n == 0) return XFDTD_OK;
        if (!k || !omega) return fail(XFDTD_EINVAL, "k and omega must be device pointers");
        if (n > ((int64_t)1 << 38)) return fail(XFDTD_EINVAL, "n too large");
        hipStream_t s = (hipStream_t)stream;
        const double sp[3] = {g->dx, g->dy, g->dz};
        unsigned int *bad = nullptr;
        HIP_TRY(hipMallocAsync((void **)&bad, sizeof(unsigned int), s), "hipMallocAsync");
        HIP_TRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), s), "hipMemsetAsync");
        hipError_t e = launch_dispersion(k, n, dt, coeffs, sp, omega, vph, vg, bad, s);
        unsigned int nbad = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hipFreeAsync(bad, s);
        if (e != hipSuccess) return hip_fail(e, "dispersion");
        if (nbad) return fail(XFDTD_EUNSTABLE, "%u wave vectors have dt^2 F outside [0, 1] (omega = NaN there)", nbad);
        return XFDTD_OK;
    });
}

int xfdtd_divergence(xfdtd_t h, void *div_star_b, void *div_e)
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        const double sp[3] = {h->g.dx, h->g.dy, h->g.dz};
        const Dims d = dims_of(h->g);
        if (h->dtype == XFDTD_F32)
            HIP_TRY(launch_divergence<float>(as_fields<float>(h->fields), d, h->coeffs, sp, (float *)div_star_b,
                                             (float *)div_e, h->stream), "divergence launch");
        else
            HIP_TRY(launch_divergence<double>(as_fields<double>(h->fields), d, h->coeffs, sp, (double *)div_star_b,
                                              (double *)div_e, h->stream), "divergence launch");
        return XFDTD_OK;
    });
}

int xfdtd_divergence_max(xfdtd_t h, const void *ref_b, const void *ref_e, double out[3])
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        if (!out) return fail(XFDTD_EINVAL, "out is null");
        const int nblocks = 1024;
        if (!h->partials) {
            HIP_TRY(hipMalloc((void **)&h->partials, sizeof(double) * 3 * nblocks), "hipMalloc");
            h->npartials = nblocks;
        }
        const double sp[3] = {h->g.dx, h->g.dy, h->g.dz};
        const Dims d = dims_of(h->g);
        if (h->dtype == XFDTD_F32)
            HIP_TRY(launch_divergence_max<float>(as_fields<float>(h->fields), d, h->coeffs, sp, (const float *)ref_b,
                                                 (const float *)ref_e, h->partials, nblocks, h->stream),
                    "divergence_max launch");
        else
            HIP_TRY(launch_divergence_max<double>(as_fields<double>(h->fields), d, h->coeffs, sp,
                                                  (const double *)ref_b, (const double *)ref_e, h->partials,
                                                  nblocks, h->stream),
                    "divergence_max launch");
        double host[3 * 1024];
        HIP_TRY(hipMemcpyAsync(host, h->partials, sizeof(double) * 3 * nblocks, hipMemcpyDeviceToHost, h->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        out[0] = out[1] = out[2] = 0.0;
        for (int b = 0; b < nblocks; ++b) {
            out[0] = fmax(out[0], host[3 * b]);
            out[1] = fmax(out[1], host[3 * b + 1]);
            out[2] += host[3 * b + 2];
        }
        if (out[2] > 0) return fail(XFDTD_ENONFINITE, "%.0f non-finite field values", out[2]);
        return XFDTD_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// adjoint and checkpointed gradient
// ---------------------------------------------------------------------------
namespace {

// the adjoint kernel exists for 4- and 8-row tiles
int adjoint_tile_y(const xfdtd_s *h) { return h->atile_y; }

int ensure_adjoint_buffers(xfdtd_t h)
{
    const int nb = adjoint_blocks(dims_of(h->g), h->atile_x, adjoint_tile_y(h), h->azchunk);
    if (h->napartials < nb) {
        if (h->apartials) {
            HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
            HIP_TRY(hipFree(h->apartials), "hipFree");
            h->apartials = nullptr;
        }
        HIP_TRY(hipMalloc((void **)&h->apartials, sizeof(double) * 12 * (size_t)nb), "hipMalloc");
        h->napartials = nb;
    }
    if (!h->grad_acc) HIP_TRY(hipMalloc((void **)&h->grad_acc, sizeof(double) * 12), "hipMalloc");
    return XFDTD_OK;
}

Scale12 grad_scale(const xfdtd_s *h)
{
    Scale12 sc;
    const double sp[3] = {h->g.dx, h->g.dy, h->g.dz};
    for (int j = 0; j < 12; ++j) sc.s[j] = h->dt / sp[j / 4];
    return sc;
}

// One adjoint launch.  accumulate = 0 overwrites the per-workgroup gradient
// sums, 1 adds to them; reduce != 0 then adds their scaled total to grad.
// partials: the per-workgroup sums (default: the handle's buffer).
template <typename T>
int adjoint_one(xfdtd_t h, const Fields<T> &lin, const Fields<T> &lout, const T *const en[3], double *grad,
                int accumulate, int reduce, double *partials = nullptr)
{
    const Dims d = dims_of(h->g);
    const Weights<T> &w = weights_of<T>(h);
    const int ty = adjoint_tile_y(h);
    if (!partials) partials = h->apartials;
    HIP_TRY(launch_adjoint<T>(lin, lout, en, d, w, h->atile_x, ty, h->azchunk, partials, accumulate, h->stream),
            "adjoint launch");
    if (reduce)
        HIP_TRY(launch_reduce_partials(partials, adjoint_blocks(d, h->atile_x, ty, h->azchunk), grad_scale(h), grad,
                                       h->stream),
                "reduce launch");
    return XFDTD_OK;
}

// Static scratch of the allocation-free adjoint step: the per-workgroup FP64
// gradient sums of one adjoint launch (at most kNoallocBlocks workgroups).
// Each GPU holds its own copy until the process ends; its device address is
// looked up once per device (with that device current) and kept in
// g_scratch_ptr.  In host code the array's name is not a device address.
constexpr int kNoallocBlocks = 16384;
static __device__ __align__(256) double adj_scratch[kNoallocBlocks * 12];
std::mutex g_scratch_mu;
double *g_scratch_ptr[64];

int noalloc_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= 64) return fail(XFDTD_EINVAL, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(adj_scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return XFDTD_OK;
}

// Argument checks shared by the adjoint step entry points (before any device work).
int check_adjoint_args(xfdtd_t h, void *const lam_in[6], void *const lam_out[6], const void *const e_n[3],
                       const double *grad)
{
    if (!h) return fail(XFDTD_EINVAL, "null handle");
    if (!lam_in || !lam_out || !e_n || !grad) return fail(XFDTD_EINVAL, "null argument");
    for (int c = 0; c < 6; ++c)
        if (!lam_in[c] || !lam_out[c]) return fail(XFDTD_EINVAL, "lambda array %d is null", c);
    for (int c = 0; c < 3; ++c)
        if (!e_n[c]) return fail(XFDTD_EINVAL, "e_n[%d] is null", c);
    // every output array must be disjoint from all inputs and the other outputs
    const uint64_t bytes = raw_field_bytes(h);
    auto overlap = [bytes](const void *a, const void *b) { return ranges_overlap(a, bytes, b, bytes); };
    for (int c = 0; c < 6; ++c) {
        for (int q = 0; q < 6; ++q)
            if (overlap(lam_out[c], lam_in[q]) || (q != c && overlap(lam_out[c], lam_out[q])))
                return fail(XFDTD_EINVAL, "lam_out[%d] overlaps another lambda array", c);
        for (int q = 0; q < 3; ++q)
            if (overlap(lam_out[c], e_n[q])) return fail(XFDTD_EINVAL, "lam_out[%d] overlaps e_n[%d]", c, q);
    }
    return check_bound(h);
}

size_t field_bytes(const xfdtd_s *h)
{
    const size_t esz = h->dtype == XFDTD_F32 ? 4 : 8;
    const size_t b = (size_t)h->g.nx * h->g.ny * h->g.nz * esz;
    return (b + 255) / 256 * 256;
}

// Default segment length ceil(sqrt(2 n)): the workspace holds
// 6 ceil(n/seg) + 12 + 6 (seg - 1) field arrays (ws_arrays), within about 6 % of its
// minimum (at sqrt(n)), and the backward pass recomputes about n - 2 seg
// steps, fewer than at sqrt(n).
int64_t default_seg(int64_t n, int64_t seg)
{
    if (seg > 0) return seg;
    int64_t s = (int64_t)ceil(sqrt(2.0 * (double)(n > 0 ? n : 1)));
    return s < 1 ? 1 : s;
}

// Workspace layout, in units of one field array (field_bytes):
//   [0, 6*nck)            checkpoints, state m at step m*seg
//   [6*nck, 6*nck+6)      state A (forward ping-pong, B ping-pong in the last
//                         two segments; backward: B ping-pong of the recompute)
//   [6*nck+6, 6*nck+12)   state B (forward ping-pong; backward: lambda scratch)
//   [6*nck+12, ...)       two sets of (seg-1) E snapshots (3 arrays each):
//                         segment m uses set m & 1, so that the backward pass
//                         recomputes segment m-1 while it reverses segment m
//                         (one set when a single segment covers all n steps)
uint64_t ws_arrays(int64_t n, int64_t seg)
{
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    return (uint64_t)(6 * nck + 12 + (nck > 1 ? 6 : 3) * (seg - 1));
}

// first array of E snapshot i (step s0 + i, i in [1, seg)) of a segment in set `set`
int64_t snap_index(int64_t nck, int64_t seg, int set, int64_t i)
{
    return 6 * nck + 12 + (int64_t)set * 3 * (seg - 1) + 3 * (i - 1);
}

template <typename T>
Fields<T> state_at(char *ws, size_t fb, int64_t first)
{
    Fields<T> f;
    for (int c = 0; c < 6; ++c) f.c[c] = (T *)(ws + (size_t)(first + c) * fb);
    return f;
}

template <typename T>
int grad_forward_t(xfdtd_t h, int64_t n, int64_t seg, char *ws)
{
    const size_t fb = field_bytes(h);
    const Dims d = dims_of(h->g);
    const Weights<T> &w = weights_of<T>(h);
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    const size_t raw = (size_t)h->g.nx * h->g.ny * h->g.nz * (h->dtype == XFDTD_F32 ? 4 : 8);
    Fields<T> fields = as_fields<T>(h->fields);
    Fields<T> ck0 = state_at<T>(ws, fb, 0);
    for (int c = 0; c < 6; ++c)
        HIP_TRY(hipMemcpyAsync(ck0.c[c], fields.c[c], raw, hipMemcpyDeviceToDevice, h->stream), "hipMemcpyAsync");
    Fields<T> A = state_at<T>(ws, fb, 6 * nck), B = state_at<T>(ws, fb, 6 * nck + 6);
    // The E fields of the last two segments go straight to their snapshot
    // sets (both are free during the forward pass), which the backward pass
    // would otherwise recompute; B ping-pongs in state A there.
    const int64_t s0_keep = (nck >= 2 ? nck - 2 : 0) * seg;
    Fields<T> cur = ck0;
    for (int64_t s = 0; s < n; ++s) {
        Fields<T> dst;
        if (s + 1 == n) {
            dst = fields;
        } else if ((s + 1) % seg == 0) {
            dst = state_at<T>(ws, fb, 6 * ((s + 1) / seg));
        } else if (s >= s0_keep) {
            const int64_t m = s / seg, s0 = m * seg;
            const int64_t e = snap_index(nck, seg, (int)(m & 1), s + 1 - s0);
            for (int c = 0; c < 3; ++c) {
                dst.c[c] = (T *)(ws + (size_t)(e + c) * fb);
                dst.c[3 + c] = A.c[3 * ((s - s0) & 1) + c];
            }
        } else {
            dst = (cur.c[0] == A.c[0]) ? B : A;
        }
        HIP_TRY(launch_fused<T>(cur, dst, d, w, h->tile_x, h->tile_y, h->zchunk, h->stream), "fused launch");
        cur = dst;
    }
    return XFDTD_OK;
}

// The recompute stream of the backward pass, on the handle's device.
int ensure_aux_stream(xfdtd_t h)
{
    if (h->aux && h->aux_device == h->device) return XFDTD_OK;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != h->device) HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    hipError_t e = hipSuccess;
    if (h->aux) {
        e = hipStreamSynchronize(h->aux);
        if (e == hipSuccess) e = hipStreamDestroy(h->aux);
        h->aux = nullptr;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
    if (cur != h->device) hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "creating the recompute stream");
    h->aux_device = h->device;
    return XFDTD_OK;
}

// Events of one backward pass (destroyed with it).
struct EventSet {
    std::vector<hipEvent_t> ev;
    ~EventSet()
    {
        for (hipEvent_t e : ev) hipEventDestroy(e);
    }
    hipError_t make(size_t n)
    {
        for (size_t i = 0; i < n; ++i) {
            hipEvent_t e;
            const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (r != hipSuccess) return r;
            ev.push_back(e);
        }
        return hipSuccess;
    }
};

// Backward pass.  The adjoint steps run on the handle's stream, segment by
// segment from the last; segment m - 1 is recomputed from its checkpoint on
// the second stream meanwhile, into the other set of E snapshots (the forward
// pass wrote those of the last two segments).  Events order the two: a
// recompute waits until the adjoint has left the set it overwrites, an
// adjoint segment until its recompute is done.
template <typename T>
int grad_backward_t(xfdtd_t h, int64_t n, int64_t seg, char *ws, void *const lam[6], double grad[12])
{
    int rc = ensure_adjoint_buffers(h);
    if (rc) return rc;
    rc = ensure_aux_stream(h);
    if (rc) return rc;
    const size_t fb = field_bytes(h);
    const Dims d = dims_of(h->g);
    const Weights<T> &w = weights_of<T>(h);
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    const size_t raw = (size_t)h->g.nx * h->g.ny * h->g.nz * (h->dtype == XFDTD_F32 ? 4 : 8);
    hipStream_t mainS = h->stream, aux = h->aux;
    HIP_TRY(hipMemsetAsync(h->grad_acc, 0, sizeof(double) * 12, mainS), "hipMemsetAsync");
    Fields<T> segB = state_at<T>(ws, fb, 6 * nck);   // two B buffers: comps 0..2 and 3..5
    Fields<T> lamS = state_at<T>(ws, fb, 6 * nck + 6);
    Fields<T> lamU = as_fields<T>(lam);
    auto segE = [&](int64_t m, int64_t i) {  // E snapshot of step m*seg + i of segment m, i in [1, seg)
        Fields<T> f;
        const int64_t e = snap_index(nck, seg, (int)(m & 1), i);
        for (int c = 0; c < 3; ++c) f.c[c] = (T *)(ws + (size_t)(e + c) * fb);
        return f;
    };
    // events: [0] start, [1 + (m & 3)] recompute of segment m done,
    // [5 + (m & 3)] adjoint of segment m done.  A stream wait takes the
    // event's latest record when it is issued, and each record below is
    // waited for before its slot is recorded again (a recompute event two
    // segments later, an adjoint event at once), so four slots of each suffice.
    EventSet evs;
    // on every return, the recompute stream has finished before the events go
    struct AuxDrain {
        hipStream_t s;
        ~AuxDrain() { hipStreamSynchronize(s); }
    } drain{aux};
    HIP_TRY(evs.make(9), "hipEventCreate");
    auto ev_rec = [&](int64_t m) { return evs.ev[(size_t)(1 + (m & 3))]; };
    auto ev_adj = [&](int64_t m) { return evs.ev[(size_t)(5 + (m & 3))]; };
    HIP_TRY(hipEventRecord(evs.ev[0], mainS), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(aux, evs.ev[0], 0), "hipStreamWaitEvent");  // checkpoints are written

    // recompute segment m on the second stream, keeping E of every step
    auto recompute = [&](int64_t m) -> int {
        Range range("recompute segment");
        const int64_t s0 = m * seg, s1 = (s0 + seg < n) ? s0 + seg : n;
        if (s1 - s0 > 1) {
            h->st.recomputed_steps += s1 - s0 - 1;
            h->st.model_bytes += model_bytes(h, s1 - s0 - 1, 12);
        }
        Fields<T> in = state_at<T>(ws, fb, 6 * m);
        for (int64_t s = s0; s + 1 < s1; ++s) {
            Fields<T> out;
            Fields<T> e = segE(m, s + 1 - s0);
            for (int c = 0; c < 3; ++c) out.c[c] = e.c[c];
            for (int c = 0; c < 3; ++c) out.c[3 + c] = segB.c[3 * ((s - s0) & 1) + c];
            HIP_TRY(launch_fused<T>(in, out, d, w, h->tile_x, h->tile_y, h->zchunk, aux), "fused launch");
            in = out;
        }
        HIP_TRY(hipEventRecord(ev_rec(m), aux), "hipEventRecord");
        return XFDTD_OK;
    };

    Fields<T> lcur = lamU, lnext = lamS;
    bool first = true;
    for (int64_t m = nck - 1; m >= 0 && n > 0; --m) {
        const int64_t s0 = m * seg, s1 = (s0 + seg < n) ? s0 + seg : n;
        Fields<T> ck = state_at<T>(ws, fb, 6 * m);
        if (m < nck - 2) HIP_TRY(hipStreamWaitEvent(mainS, ev_rec(m), 0), "hipStreamWaitEvent");
        // reverse through the segment
        Range range("adjoint segment");
        for (int64_t s = s1 - 1; s >= s0; --s) {
            const T *en[3];
            if (s == s0) {
                for (int c = 0; c < 3; ++c) en[c] = ck.c[c];
            } else {
                Fields<T> e = segE(m, s - s0);
                for (int c = 0; c < 3; ++c) en[c] = e.c[c];
            }
            // the workgroup sums accumulate over all steps; one reduction at the end
            rc = adjoint_one<T>(h, lcur, lnext, en, h->grad_acc, first ? 0 : 1, 0);
            if (rc) return rc;
            first = false;
            Fields<T> t = lcur;
            lcur = lnext;
            lnext = t;
        }
        HIP_TRY(hipEventRecord(ev_adj(m), mainS), "hipEventRecord");
        if (m >= 2) {  // segment m - 2 reuses this segment's E set
            HIP_TRY(hipStreamWaitEvent(aux, ev_adj(m), 0), "hipStreamWaitEvent");
            rc = recompute(m - 2);
            if (rc) return rc;
        }
    }
    if (!first)
        HIP_TRY(launch_reduce_partials(h->apartials, adjoint_blocks(d, h->atile_x, adjoint_tile_y(h), h->azchunk),
                                       grad_scale(h), h->grad_acc, mainS),
                "reduce launch");
    if (lcur.c[0] != lamU.c[0])
        for (int c = 0; c < 6; ++c)
            HIP_TRY(hipMemcpyAsync(lamU.c[c], lcur.c[c], raw, hipMemcpyDeviceToDevice, mainS), "hipMemcpyAsync");
    HIP_TRY(hipMemcpyAsync(grad, h->grad_acc, sizeof(double) * 12, hipMemcpyDeviceToHost, mainS), "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(mainS), "hipStreamSynchronize");
    HIP_TRY(hipStreamSynchronize(aux), "hipStreamSynchronize");
    return XFDTD_OK;
}

// At most this many workspaces per handle are remembered as holding a
// forward pass; the oldest is forgotten first.
constexpr size_t kMaxTapes = 64;

// Forget every workspace that overlaps [ws, ws + bytes).
void drop_tapes(xfdtd_t h, const void *ws, uint64_t bytes)
{
    const uintptr_t a = (uintptr_t)ws, b = a + bytes;
    std::vector<xfdtd_s::Tape> &t = h->tapes;
    t.erase(std::remove_if(t.begin(), t.end(),
                           [&](const xfdtd_s::Tape &e) { return e.ws < b && a < e.ws + e.bytes; }),
            t.end());
}

int check_ws(xfdtd_t h, int64_t n, int64_t seg, const void *ws, uint64_t ws_bytes)
{
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(XFDTD_EINVAL, "n must be in [0, 2^40]");
    if (seg > ((int64_t)1 << 40)) return fail(XFDTD_EINVAL, "seg must be <= 2^40");
    if ((double)ws_arrays(n, seg) * (double)field_bytes(h) >= 0x1p63)
        return fail(XFDTD_EINVAL, "workspace size exceeds 2^63 bytes");
    if (!ws) return fail(XFDTD_EINVAL, "workspace is null");
    if ((uintptr_t)ws % 256) return fail(XFDTD_EINVAL, "workspace must be 256-byte aligned");
    const uint64_t need = ws_arrays(n, seg) * field_bytes(h);
    if (ws_bytes < need) return fail(XFDTD_EINVAL, "workspace too small: %llu < %llu bytes",
                                     (unsigned long long)ws_bytes, (unsigned long long)need);
    return XFDTD_OK;
}

}  // namespace

extern "C" {

int xfdtd_adjoint_step(xfdtd_t h, void *const lam_in[6], void *const lam_out[6], const void *const e_n[3],
                       double *grad)
{
    return guarded([&]() -> int {
        int rc = check_adjoint_args(h, lam_in, lam_out, e_n, grad);
        if (rc) return rc;
        rc = ensure_adjoint_buffers(h);
        if (rc) return rc;
        if (h->dtype == XFDTD_F32) {
            const float *en[3] = {(const float *)e_n[0], (const float *)e_n[1], (const float *)e_n[2]};
            rc = adjoint_one<float>(h, as_fields<float>(lam_in), as_fields<float>(lam_out), en, grad, 0, 1);
        } else {
            const double *en[3] = {(const double *)e_n[0], (const double *)e_n[1], (const double *)e_n[2]};
            rc = adjoint_one<double>(h, as_fields<double>(lam_in), as_fields<double>(lam_out), en, grad, 0, 1);
        }
        if (rc) return rc;
        ++h->st.adjoint_steps;
        h->st.model_bytes += model_bytes(h, 1, 15);
        return XFDTD_OK;
    });
}

int xfdtd_adjoint_step_noalloc(xfdtd_t h, void *const lam_in[6], void *const lam_out[6], const void *const e_n[3],
                               double *grad)
{
    return guarded([&]() -> int {
        int rc = check_adjoint_args(h, lam_in, lam_out, e_n, grad);
        if (rc) return rc;
        const int nb = adjoint_blocks(dims_of(h->g), h->atile_x, adjoint_tile_y(h), h->azchunk);
        if (nb > kNoallocBlocks)
            return fail(XFDTD_EINVAL,
                        "the adjoint launch of this grid has %d workgroups; the allocation-free step holds "
                        "the sums of at most %d (use xfdtd_adjoint_step)", nb, kNoallocBlocks);
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        if (dev != h->device)
            return fail(XFDTD_EINVAL, "the current device (%d) is not the handle's (%d)", dev, h->device);
        double *ws = nullptr;
        rc = noalloc_scratch(dev, &ws);
        if (rc) return rc;
        // the adjoint kernel overwrites the slot of every workgroup it runs
        // (nothing in the scratch needs to start at zero)
        if (h->dtype == XFDTD_F32) {
            const float *en[3] = {(const float *)e_n[0], (const float *)e_n[1], (const float *)e_n[2]};
            rc = adjoint_one<float>(h, as_fields<float>(lam_in), as_fields<float>(lam_out), en, grad, 0, 1, ws);
        } else {
            const double *en[3] = {(const double *)e_n[0], (const double *)e_n[1], (const double *)e_n[2]};
            rc = adjoint_one<double>(h, as_fields<double>(lam_in), as_fields<double>(lam_out), en, grad, 0, 1, ws);
        }
        if (rc) return rc;
        ++h->st.adjoint_steps;  // counters only: nothing here allocates
        h->st.model_bytes += model_bytes(h, 1, 15);
        return XFDTD_OK;
    });
}

int xfdtd_grad_workspace(xfdtd_t h, int64_t n, int64_t seg, uint64_t *bytes)
{
    return guarded([&]() -> int {
        if (!h || !bytes) return fail(XFDTD_EINVAL, "null argument");
        if (n < 0 || n > ((int64_t)1 << 40)) return fail(XFDTD_EINVAL, "n must be in [0, 2^40]");
        if (seg > ((int64_t)1 << 40)) return fail(XFDTD_EINVAL, "seg must be <= 2^40");
        seg = default_seg(n, seg);
        // 2^40 steps of a 2^35-byte field would overflow 64 bits
        if ((double)ws_arrays(n, seg) * (double)field_bytes(h) >= 0x1p63)
            return fail(XFDTD_EINVAL, "workspace size of n = %lld, seg = %lld exceeds 2^63 bytes", (long long)n,
                        (long long)seg);
        *bytes = ws_arrays(n, seg) * field_bytes(h);
        return XFDTD_OK;
    });
}

int xfdtd_grad_forward(xfdtd_t h, int64_t n, int64_t seg, void *ws, uint64_t ws_bytes)
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        seg = default_seg(n, seg);
        rc = check_ws(h, n, seg, ws, ws_bytes);
        if (rc) return rc;
        const uint64_t wsb = ws_arrays(n, seg) * field_bytes(h);
        for (int c = 0; c < 6; ++c)
            if (ranges_overlap(ws, wsb, h->fields[c], raw_field_bytes(h)))
                return fail(XFDTD_EINVAL, "the workspace overlaps bound field %d", c);
        drop_tapes(h, ws, wsb);
        Range range("xfdtd_grad_forward");
        rc = h->dtype == XFDTD_F32 ? grad_forward_t<float>(h, n, seg, (char *)ws)
                                   : grad_forward_t<double>(h, n, seg, (char *)ws);
        if (rc) return rc;
        h->st.grad_forward_steps += n;
        h->st.model_bytes += model_bytes(h, n, 12);
        xlog("gradient forward pass: %lld steps, segments of %lld (%lld checkpoints)", (long long)n, (long long)seg,
             (long long)(n > 0 ? (n + seg - 1) / seg : 0));
        if (h->tapes.size() >= kMaxTapes) h->tapes.erase(h->tapes.begin());
        h->tapes.push_back({(uintptr_t)ws, (uintptr_t)wsb, n, seg});
        return XFDTD_OK;
    });
}

int xfdtd_grad_backward(xfdtd_t h, int64_t n, int64_t seg, void *ws, uint64_t ws_bytes, void *const lam[6],
                        double grad[12])
{
    return guarded([&]() -> int {
        int rc = check_bound(h);
        if (rc) return rc;
        if (!lam || !grad) return fail(XFDTD_EINVAL, "null argument");
        for (int c = 0; c < 6; ++c)
            if (!lam[c]) return fail(XFDTD_EINVAL, "lam[%d] is null", c);
        seg = default_seg(n, seg);
        rc = check_ws(h, n, seg, ws, ws_bytes);
        if (rc) return rc;
        const uint64_t wsb = ws_arrays(n, seg) * field_bytes(h), fb = raw_field_bytes(h);
        for (int c = 0; c < 6; ++c) {
            if (ranges_overlap(ws, wsb, lam[c], fb)) return fail(XFDTD_EINVAL, "lam[%d] overlaps the workspace", c);
            for (int q = c + 1; q < 6; ++q)
                if (ranges_overlap(lam[c], fb, lam[q], fb)) return fail(XFDTD_EINVAL, "lam[%d] overlaps lam[%d]", c, q);
        }
        auto it = std::find_if(h->tapes.begin(), h->tapes.end(), [&](const xfdtd_s::Tape &e) {
            return e.ws == (uintptr_t)ws && e.n == n && e.seg == seg;
        });
        if (it == h->tapes.end())
            return fail(XFDTD_EINVAL, "the workspace holds no forward pass of n = %lld, seg = %lld on this handle "
                                      "(a backward pass consumes it; run xfdtd_grad_forward again)",
                        (long long)n, (long long)seg);
        h->tapes.erase(it);
        Range range("xfdtd_grad_backward");
        const int64_t before = h->st.recomputed_steps;
        rc = h->dtype == XFDTD_F32 ? grad_backward_t<float>(h, n, seg, (char *)ws, lam, grad)
                                   : grad_backward_t<double>(h, n, seg, (char *)ws, lam, grad);
        if (rc) return rc;
        h->st.adjoint_steps += n;
        h->st.model_bytes += model_bytes(h, n, 15);
        xlog("gradient backward pass: %lld adjoint steps, %lld steps recomputed beside them", (long long)n,
             (long long)(h->st.recomputed_steps - before));
        return XFDTD_OK;
    });
}

}  // extern "C"
