// Batched front end of libxfdtd: many independent periodic boxes of uneven
// sizes, each with its own coefficients and time step, advanced together.
//
// Every step is one launch of the batched fused kernel over a work list of
// (box, tile) items, walked by a persistent grid; the n launches of a run
// are captured once into a HIP graph and replayed.  The launch configuration
// (tile height, z-split, persistent grid size) is chosen by timing a small
// candidate set on the bound data (xfdtd_batch_tune) and cached per set of
// box shapes for the life of the process.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/xfdtd.h"
#include "xfdtd_internal.h"

using namespace xfdtd;

namespace {

#define BTRY(expr, what)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return set_error(XFDTD_EHIP, "%s: %s", what, hipGetErrorString(e_)); \
    } while (0)

struct Config {
    int tile_y = 8, zsplit = 1, grid = 0;
};

std::mutex g_cache_mu;
std::map<std::string, Config> g_cache;

}  // namespace

struct xfdtd_batch_s {
    int64_t m = 0;
    int dtype = XFDTD_F32;
    std::vector<xfdtd_grid> g;
    std::vector<double> dt, coeffs;
    std::vector<void *> f, s;  // m*6 each
    bool bound = false;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    Config cfg;
    bool cfg_set = false;
    void *d_boxes = nullptr;
    int2 *d_items = nullptr;
    int nitems = 0;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_n = -1;
    std::string key;
};

namespace {

int cus()
{
    int dev = 0, n = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 256;
}

void drop_graph(xfdtd_batch_t b)
{
    if (b->gexec) {
        hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->graph_n = -1;
}

template <typename T>
int build_t(xfdtd_batch_t b)
{
    const int ty = b->cfg.tile_y;
    std::vector<BoxDesc<T>> descs((size_t)b->m);
    std::vector<std::pair<double, int64_t>> order;
    for (int64_t i = 0; i < b->m; ++i) {
        const xfdtd_grid &g = b->g[i];
        BoxDesc<T> &d = descs[i];
        for (int c = 0; c < 6; ++c) {
            d.f.c[c] = (T *)b->f[6 * i + c];
            d.s.c[c] = (T *)b->s[6 * i + c];
        }
        d.d = Dims{(int)g.nx, (int)g.ny, (int)g.nz};
        const double sp[3] = {g.dx, g.dy, g.dz};
        d.w = fold_weights<T>(b->dt[i], &b->coeffs[12 * i], sp, nullptr);
        int zc = (int)((g.nz + b->cfg.zsplit - 1) / b->cfg.zsplit);
        if (zc < 4) zc = (int)std::min<int64_t>(4, g.nz);
        d.zchunk = zc;
        d.ntx = (int)((g.nx + 63) / 64);
        d.nty = (int)((g.ny + ty - 1) / ty);
        d.pad = 0;
        order.push_back({-(double)g.nx * g.ny * g.nz, i});
    }
    // largest boxes first: their tiles start in the first rounds
    std::stable_sort(order.begin(), order.end());
    std::vector<int2> items;
    for (auto &o : order) {
        const int64_t i = o.second;
        const BoxDesc<T> &d = descs[i];
        const int nzc = (d.d.nz + d.zchunk - 1) / d.zchunk;
        const int64_t nt = (int64_t)d.ntx * d.nty * nzc;
        for (int64_t t = 0; t < nt; ++t) items.push_back(make_int2((int)i, (int)t));
    }
    if (items.size() > 0x7fffffff) return set_error(XFDTD_EINVAL, "too many work items");
    if (b->d_boxes) hipFree(b->d_boxes);
    if (b->d_items) hipFree(b->d_items);
    b->d_boxes = nullptr;
    b->d_items = nullptr;
    BTRY(hipMalloc(&b->d_boxes, sizeof(BoxDesc<T>) * descs.size()), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_items, sizeof(int2) * std::max<size_t>(1, items.size())), "hipMalloc");
    BTRY(hipMemcpy(b->d_boxes, descs.data(), sizeof(BoxDesc<T>) * descs.size(), hipMemcpyHostToDevice),
         "hipMemcpy");
    if (!items.empty())
        BTRY(hipMemcpy(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice), "hipMemcpy");
    b->nitems = (int)items.size();
    drop_graph(b);
    return XFDTD_OK;
}

int build(xfdtd_batch_t b)
{
    BTRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    return b->dtype == XFDTD_F32 ? build_t<float>(b) : build_t<double>(b);
}

int grid_of(const xfdtd_batch_t b)
{
    const int g = b->cfg.grid;
    return (g <= 0 || g > b->nitems) ? b->nitems : g;
}

int launch_step(xfdtd_batch_t b, int parity, hipStream_t s)
{
    hipError_t e;
    if (b->dtype == XFDTD_F32)
        e = launch_batched<float>((const BoxDesc<float> *)b->d_boxes, b->d_items, b->nitems, parity,
                                  b->cfg.tile_y, grid_of(b), s);
    else
        e = launch_batched<double>((const BoxDesc<double> *)b->d_boxes, b->d_items, b->nitems, parity,
                                   b->cfg.tile_y, grid_of(b), s);
    if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched launch: %s", hipGetErrorString(e));
    return XFDTD_OK;
}

template <typename T>
int unfused_all(xfdtd_batch_t b, hipStream_t s)
{
    for (int64_t i = 0; i < b->m; ++i) {
        const xfdtd_grid &g = b->g[i];
        Fields<T> f;
        for (int c = 0; c < 6; ++c) f.c[c] = (T *)b->f[6 * i + c];
        const Dims d{(int)g.nx, (int)g.ny, (int)g.nz};
        const double sp[3] = {g.dx, g.dy, g.dz};
        const Weights<T> w = fold_weights<T>(b->dt[i], &b->coeffs[12 * i], sp, nullptr);
        hipError_t e = launch_faraday<T>(f, d, w, s);
        if (e == hipSuccess) e = launch_ampere<T>(f, d, w, s);
        if (e != hipSuccess) return set_error(XFDTD_EHIP, "unfused launch: %s", hipGetErrorString(e));
    }
    return XFDTD_OK;
}

std::string shape_key(const xfdtd_batch_t b)
{
    std::string k = b->dtype == XFDTD_F32 ? "f32" : "f64";
    for (auto &g : b->g) k += ":" + std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz);
    return k;
}

}  // namespace

extern "C" {

int xfdtd_batch_create(const xfdtd_grid *grids, const double *dts, const double *coeffs, int64_t m, int dtype,
                       int allow_unstable, xfdtd_batch_t *out)
{
    if (!out) return set_error(XFDTD_EINVAL, "out is null");
    *out = nullptr;
    if (m < 1 || m > (1 << 20)) return set_error(XFDTD_EINVAL, "box count must be in [1, 2^20]");
    if (!grids || !dts || !coeffs) return set_error(XFDTD_EINVAL, "null argument");
    if (dtype != XFDTD_F32 && dtype != XFDTD_F64) return set_error(XFDTD_EINVAL, "bad dtype");
    for (int64_t i = 0; i < m; ++i) {
        const xfdtd_grid &g = grids[i];
        if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > (1 << 30) || g.ny > (1 << 30) || g.nz > (1 << 30) ||
            (double)g.nx * g.ny * g.nz > 4.0e9 || !(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) ||
            !isfinite(g.dx) || !isfinite(g.dy) || !isfinite(g.dz))
            return set_error(XFDTD_EINVAL, "box %lld: invalid grid", (long long)i);
        if (!(dts[i] > 0) || !isfinite(dts[i])) return set_error(XFDTD_EINVAL, "box %lld: bad dt", (long long)i);
        for (int j = 0; j < 12; ++j)
            if (!isfinite(coeffs[12 * i + j])) return set_error(XFDTD_EINVAL, "box %lld: bad coeffs", (long long)i);
        if (!allow_unstable) {
            const double sp[3] = {g.dx, g.dy, g.dz};
            double lo, hi;
            f_range(sp, &coeffs[12 * i], &lo, &hi);
            if (lo < -1e-12 * fmax(1.0, fabs(hi)))
                return set_error(XFDTD_EUNSTABLE, "box %lld: F_min < 0", (long long)i);
            if (dts[i] * dts[i] * hi > 1.0 + 1e-12)
                return set_error(XFDTD_EUNSTABLE, "box %lld: dt exceeds the stability bound", (long long)i);
        }
    }
    xfdtd_batch_s *b = new (std::nothrow) xfdtd_batch_s();
    if (!b) return set_error(XFDTD_EINVAL, "out of host memory");
    b->m = m;
    b->dtype = dtype;
    b->g.assign(grids, grids + m);
    b->dt.assign(dts, dts + m);
    b->coeffs.assign(coeffs, coeffs + 12 * m);
    b->cfg.tile_y = dtype == XFDTD_F64 ? 4 : 8;
    b->key = shape_key(b);
    *out = b;
    return XFDTD_OK;
}

void xfdtd_batch_destroy(xfdtd_batch_t b)
{
    if (!b) return;
    if (b->bound) hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->d_boxes) hipFree(b->d_boxes);
    if (b->d_items) hipFree(b->d_items);
    if (b->capture) hipStreamDestroy(b->capture);
    delete b;
}

int xfdtd_batch_bind(xfdtd_batch_t b, void *const *fields, void *const *scratch, void *stream)
{
    if (!b || !fields || !scratch) return set_error(XFDTD_EINVAL, "null argument");
    const size_t esz = b->dtype == XFDTD_F32 ? 4 : 8;
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int64_t i = 0; i < b->m; ++i) {
        const size_t bytes = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * esz;
        for (int c = 0; c < 6; ++c) {
            for (void *p : {fields[6 * i + c], scratch[6 * i + c]}) {
                if (!p || (uintptr_t)p % 16) return set_error(XFDTD_EINVAL, "box %lld: null or misaligned array", (long long)i);
                spans.push_back({(uintptr_t)p, (uintptr_t)p + bytes});
            }
        }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return set_error(XFDTD_EINVAL, "bound arrays overlap");
    b->f.assign(fields, fields + 6 * b->m);
    b->s.assign(scratch, scratch + 6 * b->m);
    b->stream = (hipStream_t)stream;
    b->bound = true;
    if (!b->capture) BTRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "hipStreamCreate");
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(b->key);
        if (!b->cfg_set && it != g_cache.end()) b->cfg = it->second;
    }
    return build(b);
}

int xfdtd_batch_set_config(xfdtd_batch_t b, int tile_y, int zsplit, int grid)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if ((tile_y != 4 && tile_y != 8 && tile_y != 16) || zsplit < 1 || zsplit > 1024 || grid < 0 ||
        (tile_y == 16 && b->dtype != XFDTD_F32))
        return set_error(XFDTD_EINVAL, "bad configuration");
    b->cfg.tile_y = tile_y;
    b->cfg.zsplit = zsplit;
    b->cfg.grid = grid;
    b->cfg_set = true;
    return b->bound ? build(b) : XFDTD_OK;
}

int xfdtd_batch_get_config(xfdtd_batch_t b, int *tile_y, int *zsplit, int *grid, int *nitems)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (tile_y) *tile_y = b->cfg.tile_y;
    if (zsplit) *zsplit = b->cfg.zsplit;
    if (grid) *grid = b->bound ? grid_of(b) : b->cfg.grid;
    if (nitems) *nitems = b->nitems;
    return XFDTD_OK;
}

int xfdtd_batch_tune(xfdtd_batch_t b, int force, double *best_ms)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
    if (!force) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_cache.find(b->key);
        if (it != g_cache.end()) {
            b->cfg = it->second;
            b->cfg_set = true;
            if (best_ms) *best_ms = -1.0;
            return build(b);
        }
    }
    const int ncu = cus();
    std::vector<Config> cands;
    const int tys[3] = {4, 8, 16};
    for (int ty : tys) {
        if (b->dtype == XFDTD_F64 && ty != 4) continue;
        for (int zs : {1, 2, 4})
            for (int gm : {0, 1, 2}) {
                Config c;
                c.tile_y = ty;
                c.zsplit = zs;
                c.grid = gm == 0 ? 0 : gm * ncu;
                cands.push_back(c);
            }
    }
    hipEvent_t e0, e1;
    BTRY(hipEventCreate(&e0), "hipEventCreate");
    BTRY(hipEventCreate(&e1), "hipEventCreate");
    double best = INFINITY;
    Config bestc = b->cfg;
    int rc = XFDTD_OK;
    for (const Config &c : cands) {
        b->cfg = c;
        rc = build(b);
        if (rc) break;
        // f -> s only: the bound state is not modified by tuning
        rc = launch_step(b, 0, b->stream);
        if (rc) break;
        hipEventRecord(e0, b->stream);
        for (int r = 0; r < 3 && !rc; ++r) rc = launch_step(b, 0, b->stream);
        hipEventRecord(e1, b->stream);
        if (rc) break;
        BTRY(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    b->cfg = bestc;
    b->cfg_set = true;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache[b->key] = bestc;
    }
    if (best_ms) *best_ms = best / 3.0;
    return build(b);
}

int xfdtd_batch_run(xfdtd_batch_t b, int64_t n)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
    if (n < 0) return set_error(XFDTD_EINVAL, "n must be >= 0");
    if (n == 0) return XFDTD_OK;
    if (b->graph_n != n || !b->gexec) {
        drop_graph(b);
        BTRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        int rc = XFDTD_OK;
        int64_t left = n;
        if (left & 1) {  // odd count: one in-place step keeps the result in the state arrays
            rc = b->dtype == XFDTD_F32 ? unfused_all<float>(b, b->capture) : unfused_all<double>(b, b->capture);
            --left;
        }
        for (int64_t s = 0; s < left && !rc; ++s) rc = launch_step(b, (int)(s & 1), b->capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(b->capture, &graph);
        if (rc) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return set_error(XFDTD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            return set_error(XFDTD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        b->graph_n = n;
    }
    BTRY(hipGraphLaunch(b->gexec, b->stream), "hipGraphLaunch");
    return XFDTD_OK;
}

int xfdtd_batch_run_eager(xfdtd_batch_t b, int64_t n)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
    if (n < 0) return set_error(XFDTD_EINVAL, "n must be >= 0");
    int rc = XFDTD_OK;
    int64_t left = n;
    if (left & 1) {
        rc = b->dtype == XFDTD_F32 ? unfused_all<float>(b, b->stream) : unfused_all<double>(b, b->stream);
        --left;
    }
    for (int64_t s = 0; s < left && !rc; ++s) rc = launch_step(b, (int)(s & 1), b->stream);
    return rc;
}

}  // extern "C"
