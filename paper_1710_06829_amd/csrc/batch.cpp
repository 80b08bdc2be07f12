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
#include <array>
#include <map>
#include <queue>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
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

// Launch configuration of a batch; spp = 2 runs the two-step kernel (FP32,
// 32-column tiles, which the one-step kernel also has).
struct Config {
    int tile_x = 64, tile_y = 8, zsplit = 1, grid = 0, spp = 1;
};

// The batched adjoint's tiling as timed by xfdtd_batch_tune: tile width
// (0: nothing timed, the list-scheduling model chooses), tile height, z-split,
// and whether each box's items form one dispatch run (one XCD's L2 then holds
// all of a box's halos) rather than runs of a few tiles.
struct AdjPick {
    int tx = 0, ty = 0, zs = 0, boxrun = 0;
};

std::mutex g_cache_mu;
std::map<std::string, Config> g_cache;
std::map<std::string, AdjPick> g_acache;  // per key, beside g_cache

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
    hipStream_t aux = nullptr;  // recompute stream of the gradient's backward pass
    Config cfg;
    bool cfg_set = false;
    // every box one plane deep: the forward steps run the plane kernel on its
    // own tiles, one step per launch, whatever cfg asks for
    bool plane = false;
    void *d_boxes = nullptr;
    int2 *d_items = nullptr;
    int nitems = 0;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_n = -1;
    std::string key;
    // batched gradient: adjoint work list, per-item gradient sums, per-box
    // item ranges, scales and accumulators
    int2 *d_aitems = nullptr;  // per box contiguous (partial sums follow it)
    int naitems = 0;
    int *d_aorder = nullptr;  // dispatch slots: item numbers, -1 for none
    int naslots = 0;
    std::vector<int> azc;  // adjoint z-chunk per box
    std::vector<int> fzc;  // forward z-chunk per box (of the built work list)
    double *d_apart = nullptr;
    int *d_afirst = nullptr;
    double *d_scale = nullptr, *d_grad = nullptr;
    int atx = 64;  // adjoint tile width, height and z-split, chosen when the work list is built
    int aty = 8, azs = 0;
    int agroup = 1;  // tiles per adjoint work item when every box is one plane deep
    AdjPick apick;  // timed adjoint tiling, used while its tile width is the batch's
    // Workspace lists filled by a forward pass and not yet consumed by a
    // backward pass (which overwrites their E snapshots).
    struct Tape {
        std::vector<uintptr_t> ws;  // per box: start
        uint64_t arrays;            // field arrays per box
        int64_t n, seg;
    };
    std::vector<Tape> tapes;
};

namespace {

int cus()
{
    int dev = 0, n = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 256;
}

// The forward kernels' tile and steps per launch: the plane kernel's for a
// batch of boxes one plane deep, else the configured ones.
int fwd_tx(const xfdtd_batch_s *b) { return b->plane ? plane_tile_x() : b->cfg.tile_x; }
int fwd_ty(const xfdtd_batch_s *b) { return b->plane ? plane_tile_y(b->dtype) : b->cfg.tile_y; }
int fwd_spp(const xfdtd_batch_s *b) { return b->plane ? 1 : b->cfg.spp; }

// z-chunk length of a box under a z-split (at least 4 planes, or the depth)
int64_t box_zchunk(const xfdtd_grid &g, int zsplit)
{
    int64_t zc = (g.nz + zsplit - 1) / zsplit;
    if (zc < 4) zc = std::min<int64_t>(4, g.nz);
    return zc;
}

// Untuned z-split of a batch from a cost model of one step: the work items
// (tiles x z-chunks of every box) cost their chunk plus a 3-plane warm-up in
// plane iterations, run `slots` at a time (CUs x resident workgroups), and
// no item can finish before its own chunk, so a step takes about
// max(total / slots, longest item).  Small batches need the z-split to fill
// the CUs at all: one 96^3 box with z-split 1 gives 24 work items.
int model_zsplit(const xfdtd_batch_s *b, int tile_x, int tile_y)
{
    const int per = b->dtype == XFDTD_F32 ? fused_occupancy<float>(tile_x, tile_y)
                                          : fused_occupancy<double>(tile_x, tile_y);
    const double slots = (double)cus() * (per > 0 ? per : 1);
    int best_s = 1;
    double best = INFINITY;
    for (int zs = 1; zs <= 64; zs *= 2) {
        double total = 0, longest = 0;
        for (const xfdtd_grid &g : b->g) {
            const int64_t zc = box_zchunk(g, zs);
            const double tiles = (double)((g.nx + tile_x - 1) / tile_x) * (double)((g.ny + tile_y - 1) / tile_y);
            total += tiles * (double)((g.nz + zc - 1) / zc) * (double)(zc + 3);
            longest = std::max(longest, (double)(zc + 3));
        }
        const double cost = std::max(std::ceil(total / slots), longest);
        if (cost < best) {
            best = cost;
            best_s = zs;
        }
    }
    return best_s;
}

void drop_graph(xfdtd_batch_t b)
{
    if (b->gexec) {
        hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->graph_n = -1;
}

// Default tile width of a batch: 32 columns only when every box is at most
// 32 cells wide (a 64-wide tile would be at least half idle).  A batch keeps
// enough work items in flight that the 64-wide tiles' lower halo overhead
// wins otherwise (measured: 16 boxes of 96^3, 166 us per step vs 186); the
// tuner times both widths where some box leaves a 64-wide tile part idle.
bool prefer_narrow(const xfdtd_batch_s *b)
{
    for (const xfdtd_grid &g : b->g)
        if (g.nx > 32) return false;
    return true;
}

// Dispatch order of a batch's work items.  Workgroup w of a launch goes to
// XCD w mod 8 and, within an XCD, workgroups start in order as CUs free up,
// so the order decides both the balance between the XCDs (whose L2s are
// separate) and each XCD's schedule.  The items come in runs (consecutive
// tiles of one box and z-chunk, whose halos overlap and are best fetched
// once into one L2); runs go whole, largest first, to the XCD with the least
// work so far, and each XCD's items then go longest first (stable, so a run
// stays together).  Slot 8 j + x of the result holds the j-th item of XCD x,
// or -1 where that XCD's list has ended.
std::vector<int> xcd_schedule(const std::vector<double> &cost, const std::vector<int> &run)
{
    struct Run {
        double cost;
        size_t first, count;
    };
    std::vector<Run> runs;
    for (size_t i = 0; i < cost.size(); ++i) {
        if (i == 0 || run[i] != run[i - 1]) runs.push_back({0.0, i, 0});
        runs.back().cost += cost[i];
        runs.back().count += 1;
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run &a, const Run &c) { return a.cost > c.cost; });
    std::array<double, 8> load{};
    std::array<std::vector<int>, 8> lists;
    for (const Run &r : runs) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += r.cost;
        for (size_t i = r.first; i < r.first + r.count; ++i) lists[x].push_back((int)i);
    }
    size_t len = 0;
    for (auto &l : lists) {
        std::stable_sort(l.begin(), l.end(), [&](int a, int c) { return cost[a] > cost[c]; });
        len = std::max(len, l.size());
    }
    std::vector<int> order(8 * len, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) order[8 * j + x] = lists[x][j];
    return order;
}

// Work items of box descriptor d in tile order (x fastest, then y, then the
// z-chunk), with their costs in plane iterations (chunk length plus the
// kernel's warm-up planes) and run numbers: runs of at most run_len
// consecutive tiles of one z-chunk.
void box_items(int box, int ntx, int nty, int nz, int zchunk, int warm, int run_len, std::vector<int2> &items,
               std::vector<double> &cost, std::vector<int> &run)
{
    const int nzc = (nz + zchunk - 1) / zchunk;
    const int per = ntx * nty;
    for (int c = 0; c < nzc; ++c) {
        const double k = (double)(std::min(zchunk, nz - c * zchunk) + warm);
        for (int t = 0; t < per; ++t) {
            if (t % run_len == 0) run.push_back(run.empty() ? 0 : run.back() + 1);
            else run.push_back(run.back());
            items.push_back(make_int2(box, c * per + t));
            cost.push_back(k);
        }
    }
}

// Adjoint work items of a box one plane deep: groups of `group` of its
// `tiles` tiles (item y = group number), costed by their tile count.
void plane_items(int box, int tiles, int group, int run_len, std::vector<int2> &items, std::vector<double> &cost,
                 std::vector<int> &run)
{
    const int ng = (tiles + group - 1) / group;
    for (int g = 0; g < ng; ++g) {
        if (g % run_len == 0) run.push_back(run.empty() ? 0 : run.back() + 1);
        else run.push_back(run.back());
        items.push_back(make_int2(box, g));
        cost.push_back((double)std::min(group, tiles - g * group));
    }
}

// Run length of a work list: about 1/16 of an XCD's share of the plane
// iterations, in items of the typical cost.
int run_length(double total_cost, double items)
{
    if (items <= 0) return 1;
    const double per_item = total_cost / items;
    return std::max(1, (int)(total_cost / 128.0 / per_item));
}

// Finish time of the dispatch order `order` when each XCD runs `per_xcd`
// workgroups at a time and a workgroup takes the XCD's next slot as soon as
// it is free (items of equal cost take equal time), and how many workgroups
// finish at that time.
std::pair<double, int> simulate_finish(const std::vector<int> &order, const std::vector<double> &cost, int per_xcd)
{
    double worst = 0;
    int at = 0;
    for (int x = 0; x < 8; ++x) {
        std::priority_queue<double, std::vector<double>, std::greater<double>> q;
        for (int i = 0; i < per_xcd; ++i) q.push(0.0);
        for (size_t s = (size_t)x; s < order.size(); s += 8) {
            if (order[s] < 0) continue;
            const double t = q.top();
            q.pop();
            q.push(t + cost[(size_t)order[s]]);
        }
        while (!q.empty()) {
            const double t = q.top();
            q.pop();
            if (t > worst) {
                worst = t;
                at = 1;
            } else if (t == worst) {
                ++at;
            }
        }
    }
    return {worst, at};
}

// Work list of the forward kernels with z-chunks zc[i] per box: items in
// tile order, their costs and the dispatch order.  False if the list is too
// long for 32-bit item numbers.
bool forward_list(const xfdtd_batch_s *b, const std::vector<int> &zc, int warm, std::vector<int2> &all,
                  std::vector<double> &cost, std::vector<int> &order)
{
    const int tx = fwd_tx(b), ty = fwd_ty(b);
    all.clear();
    cost.clear();
    std::vector<int> run;
    double total = 0, count = 0;
    for (size_t i = 0; i < b->g.size(); ++i) {
        const xfdtd_grid &g = b->g[i];
        const double tiles = (double)((g.nx + tx - 1) / tx) * (double)((g.ny + ty - 1) / ty);
        const int64_t nzc = (g.nz + zc[i] - 1) / zc[i];
        total += tiles * ((double)g.nz + (double)nzc * warm);
        count += tiles * (double)nzc;
    }
    if (count > 0x3fffffff) return false;
    const int run_len = run_length(total, count);
    for (size_t i = 0; i < b->g.size(); ++i) {
        const xfdtd_grid &g = b->g[i];
        box_items((int)i, (int)((g.nx + tx - 1) / tx), (int)((g.ny + ty - 1) / ty), (int)g.nz, zc[i], warm, run_len,
                  all, cost, run);
    }
    order = xcd_schedule(cost, run);
    return true;
}

// Per-box z-chunks of z-split 0: starting from whole-depth marches, one box
// at a time gets one more chunk (up to 4) while that shortens the modelled
// finish time of the dispatch order, or keeps it and has fewer workgroups
// finish last.  Splitting a box costs its warm-up planes once more per chunk
// but gives the schedule shorter items to fill in with.
std::vector<int> model_chunks(const xfdtd_batch_s *b, int warm, int per_xcd)
{
    const size_t m = b->g.size();
    std::vector<int> nch(m, 1), zc(m);
    auto zc_of = [&]() {
        for (size_t i = 0; i < m; ++i) zc[i] = (int)box_zchunk(b->g[i], nch[i]);
    };
    zc_of();
    if (m > 256) return zc;  // the search is quadratic in the box count
    std::vector<int2> all;
    std::vector<double> cost;
    std::vector<int> order;
    auto score = [&]() -> std::pair<double, int> {
        zc_of();
        if (!forward_list(b, zc, warm, all, cost, order)) return {INFINITY, 0};
        return simulate_finish(order, cost, per_xcd);
    };
    std::pair<double, int> cur = score();
    for (int it = 0; it < 32; ++it) {
        std::pair<double, int> best = cur;
        size_t arg = m;
        for (size_t i = 0; i < m; ++i) {
            if (nch[i] >= 4 || box_zchunk(b->g[i], nch[i] + 1) == box_zchunk(b->g[i], nch[i])) continue;
            ++nch[i];
            const std::pair<double, int> sc = score();
            --nch[i];
            if (sc < best) {
                best = sc;
                arg = i;
            }
        }
        if (arg == m) break;
        ++nch[arg];
        cur = best;
    }
    zc_of();
    return zc;
}

template <typename T>
int build_t(xfdtd_batch_t b)
{
    const int tx = fwd_tx(b), ty = fwd_ty(b);
    // warm-up planes of a z-chunk: 3 for the one-step march, 10 for two steps,
    // none for the plane kernel
    const int warm = b->plane ? 0 : b->cfg.spp == 2 ? 10 : 3;
    std::vector<int> zc(b->g.size());
    if (b->plane) {
        for (size_t i = 0; i < b->g.size(); ++i) zc[i] = 1;
    } else if (b->cfg.zsplit == 0) {
        const int occ = b->cfg.spp == 2 ? blocked2_occupancy<T>(b->cfg.tile_x, ty)
                                        : fused_occupancy<T>(b->cfg.tile_x, ty);
        zc = model_chunks(b, warm, std::max(1, cus() / 8) * std::max(1, occ));
    } else {
        for (size_t i = 0; i < b->g.size(); ++i) zc[i] = (int)box_zchunk(b->g[i], b->cfg.zsplit);
    }
    b->fzc = zc;
    std::vector<BoxDesc<T>> descs((size_t)b->m);
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
        d.zchunk = zc[(size_t)i];
        d.ntx = (int)((g.nx + tx - 1) / tx);
        d.nty = (int)((g.ny + ty - 1) / ty);
        d.pad = 0;
    }
    std::vector<int2> all;
    std::vector<double> cost;
    std::vector<int> order;
    if (!forward_list(b, zc, warm, all, cost, order)) return set_error(XFDTD_EINVAL, "too many work items");
    std::vector<int2> items;
    for (int j : order) items.push_back(j < 0 ? make_int2(-1, -1) : all[j]);
    xlog("batch of %lld boxes: %s %dx%d tiles, z-split %d, %zu items in %zu slots, grid %d",
         (long long)b->m, b->plane ? "plane" : b->cfg.spp == 2 ? "two-step" : "one-step", tx, ty, b->cfg.zsplit, all.size(),
         order.size(), b->cfg.grid);
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

// descs: the descriptor array to launch with (nullptr: the batch's own)
int launch_step(xfdtd_batch_t b, int parity, hipStream_t s, const void *descs = nullptr)
{
    const void *dd = descs ? descs : b->d_boxes;
    hipError_t e;
    if (b->plane && b->dtype == XFDTD_F32)
        e = launch_batched_plane<float>((const BoxDesc<float> *)dd, b->d_items, b->nitems, parity, grid_of(b), s);
    else if (b->plane)
        e = launch_batched_plane<double>((const BoxDesc<double> *)dd, b->d_items, b->nitems, parity, grid_of(b), s);
    else if (b->dtype == XFDTD_F32)
        e = launch_batched<float>((const BoxDesc<float> *)dd, b->d_items, b->nitems, parity, b->cfg.tile_x,
                                  b->cfg.tile_y, grid_of(b), s);
    else
        e = launch_batched<double>((const BoxDesc<double> *)dd, b->d_items, b->nitems, parity, b->cfg.tile_x,
                                   b->cfg.tile_y, grid_of(b), s);
    if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched launch: %s", hipGetErrorString(e));
    return XFDTD_OK;
}

// One two-step launch (cfg.spp == 2): two steps of every box.
int launch_pair(xfdtd_batch_t b, int parity, hipStream_t s, const void *descs = nullptr)
{
    const void *dd = descs ? descs : b->d_boxes;
    const hipError_t e = launch_batched2<float>((const BoxDesc<float> *)dd, b->d_items, b->nitems, parity,
                                                b->cfg.tile_y, grid_of(b), s);
    if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched two-step launch: %s", hipGetErrorString(e));
    return XFDTD_OK;
}

// The batch's descriptors (as last built) with each box's fields replaced by
// its arrays in `tmp` (6 per box), uploaded to d_out (m descriptors).
template <typename T>
int temp_descs_t(xfdtd_batch_t b, const std::vector<void *> &tmp, void *d_out)
{
    std::vector<BoxDesc<T>> h((size_t)b->m);
    BTRY(hipMemcpy(h.data(), b->d_boxes, sizeof(BoxDesc<T>) * h.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    for (int64_t i = 0; i < b->m; ++i)
        for (int c = 0; c < 6; ++c) h[(size_t)i].f.c[c] = (T *)tmp[(size_t)(6 * i + c)];
    BTRY(hipMemcpy(d_out, h.data(), sizeof(BoxDesc<T>) * h.size(), hipMemcpyHostToDevice), "hipMemcpy");
    return XFDTD_OK;
}

// The launches of n steps on stream s, ending in the state arrays: an odd n
// starts with one in-place unfused step; with the two-step kernel an odd
// number of pairs does one pair as two one-step launches, so that the number
// of out-of-place launches is even.
int launch_steps(xfdtd_batch_t b, int64_t n, hipStream_t s);

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

int launch_steps(xfdtd_batch_t b, int64_t n, hipStream_t s)
{
    int rc = XFDTD_OK;
    int64_t left = n;
    if (left & 1) {  // odd count: one in-place step keeps the result in the state arrays
        rc = b->dtype == XFDTD_F32 ? unfused_all<float>(b, s) : unfused_all<double>(b, s);
        --left;
    }
    if (fwd_spp(b) == 2) {
        int64_t pairs = left / 2;
        if (pairs & 1) {
            for (int p = 0; p < 2 && !rc; ++p) rc = launch_step(b, p, s);
            --pairs;
        }
        for (int64_t q = 0; q < pairs && !rc; ++q) rc = launch_pair(b, (int)(q & 1), s);
        return rc;
    }
    for (int64_t q = 0; q < left && !rc; ++q) rc = launch_step(b, (int)(q & 1), s);
    return rc;
}

std::string shape_key(const xfdtd_batch_t b)
{
    std::string k = b->dtype == XFDTD_F32 ? "f32" : "f64";
    for (auto &g : b->g) k += ":" + std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz);
    return k;
}

// a stored configuration (tile_x, tile_y, zsplit, grid, steps per pass) the
// batch can launch
bool valid_config(const xfdtd_batch_s *b, const std::vector<int> &v, Config &c)
{
    if (v.size() != 5) return false;
    c.tile_x = v[0];
    c.tile_y = v[1];
    c.zsplit = v[2];
    c.grid = v[3];
    c.spp = v[4];
    if ((c.tile_x != 32 && c.tile_x != 64) || (c.tile_y != 4 && c.tile_y != 8 && c.tile_y != 16) || c.zsplit < 0 ||
        c.zsplit > 1024 || c.grid < 0 || (c.tile_y == 16 && b->dtype != XFDTD_F32) || (c.spp != 1 && c.spp != 2))
        return false;
    return c.spp == 1 || (b->dtype == XFDTD_F32 && c.tile_x == 32 && c.tile_y != 4);
}

// Times the batched adjoint's tilings for the bound batch (defined with the
// gradient passes below).
int tune_adjoint(xfdtd_batch_t b, bool lookup);

}  // namespace

extern "C" {

int xfdtd_batch_create(const xfdtd_grid *grids, const double *dts, const double *coeffs, int64_t m, int dtype,
                       int allow_unstable, xfdtd_batch_t *out)
{
    return guarded([&]() -> int {
        if (!out) return set_error(XFDTD_EINVAL, "out is null");
        *out = nullptr;
        if (m < 1 || m > (1 << 20)) return set_error(XFDTD_EINVAL, "box count must be in [1, 2^20]");
        if (!grids || !dts || !coeffs) return set_error(XFDTD_EINVAL, "null argument");
        if (dtype != XFDTD_F32 && dtype != XFDTD_F64) return set_error(XFDTD_EINVAL, "bad dtype");
        for (int64_t i = 0; i < m; ++i) {
            const xfdtd_grid &g = grids[i];
            if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > (1 << 30) || g.ny > (1 << 30) || g.nz > (1 << 30) ||
                (double)g.nx * g.ny * g.nz > 4.0e9 || (double)g.nx * g.ny > (double)(1 << 28) || !(g.dx > 0) ||
                !(g.dy > 0) || !(g.dz > 0) ||
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
        std::unique_ptr<xfdtd_batch_s> hold(new (std::nothrow) xfdtd_batch_s());
        xfdtd_batch_s *b = hold.get();
        if (!b) return set_error(XFDTD_EINVAL, "out of host memory");
        b->m = m;
        b->dtype = dtype;
        b->g.assign(grids, grids + m);
        b->dt.assign(dts, dts + m);
        b->coeffs.assign(coeffs, coeffs + 12 * m);
        b->cfg.tile_x = prefer_narrow(b) ? 32 : 64;
        b->cfg.tile_y = 8;
        b->cfg.zsplit = model_zsplit(b, b->cfg.tile_x, b->cfg.tile_y);
        b->plane = true;
        for (const xfdtd_grid &g : b->g)
            if (g.nz != 1) b->plane = false;
        b->key = shape_key(b);
        *out = hold.release();
        return XFDTD_OK;
    });
}

void xfdtd_batch_destroy(xfdtd_batch_t b)
{
    if (!b) return;
    if (b->bound) hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->d_boxes) hipFree(b->d_boxes);
    if (b->d_items) hipFree(b->d_items);
    for (void *p : {(void *)b->d_aitems, (void *)b->d_aorder, (void *)b->d_apart, (void *)b->d_afirst,
                    (void *)b->d_scale, (void *)b->d_grad})
        if (p) hipFree(p);
    if (b->capture) hipStreamDestroy(b->capture);
    if (b->aux) hipStreamDestroy(b->aux);
    delete b;
}

int xfdtd_batch_bind(xfdtd_batch_t b, void *const *fields, void *const *scratch, void *stream)
{
    return guarded([&]() -> int {
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
        if (!b->aux) BTRY(hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking), "hipStreamCreate");
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            auto it = g_cache.find(b->key);
            if (!b->cfg_set && it != g_cache.end()) b->cfg = it->second;
            auto ia = g_acache.find(b->key);
            if (b->apick.tx == 0 && ia != g_acache.end()) b->apick = ia->second;
        }
        return build(b);
    });
}

int xfdtd_batch_set_config(xfdtd_batch_t b, int tile_x, int tile_y, int zsplit, int grid)
{
    return guarded([&]() -> int {
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if ((tile_x != 32 && tile_x != 64) || (tile_y != 4 && tile_y != 8 && tile_y != 16) || zsplit < 0 ||
            zsplit > 1024 || grid < 0 || (tile_y == 16 && b->dtype != XFDTD_F32))
            return set_error(XFDTD_EINVAL, "bad configuration");
        b->cfg.tile_x = tile_x;
        b->cfg.tile_y = tile_y;
        b->cfg.zsplit = zsplit;
        b->cfg.grid = grid;
        if (b->cfg.spp == 2 && (tile_x != 32 || tile_y == 4)) b->cfg.spp = 1;
        b->cfg_set = true;
        return b->bound ? build(b) : XFDTD_OK;
    });
}

int xfdtd_batch_set_steps_per_pass(xfdtd_batch_t b, int steps)
{
    return guarded([&]() -> int {
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if (steps != 1 && steps != 2) return set_error(XFDTD_EINVAL, "steps per pass must be 1 or 2");
        if (steps == 2 && (b->dtype != XFDTD_F32 || b->cfg.tile_x != 32 || b->cfg.tile_y == 4))
            return set_error(XFDTD_EINVAL, "two steps per pass need FP32 and a 32 x 8 or 32 x 16 tiling");
        if (b->cfg.spp != steps) {
            b->cfg.spp = steps;
            b->cfg_set = true;
            drop_graph(b);
        }
        return XFDTD_OK;
    });
}

int xfdtd_batch_get_steps_per_pass(xfdtd_batch_t b, int *steps)
{
    if (!b || !steps) return set_error(XFDTD_EINVAL, "null argument");
    *steps = fwd_spp(b);
    return XFDTD_OK;
}

int xfdtd_batch_get_adjoint_config(xfdtd_batch_t b, int *tile_x, int *tile_y, int *zsplit, int *nslots)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    const bool built = b->naslots > 0;
    if (tile_x) *tile_x = built ? b->atx : 0;
    if (tile_y) *tile_y = built ? b->aty : 0;
    if (zsplit) *zsplit = built ? b->azs : 0;
    if (nslots) *nslots = b->naslots;
    return XFDTD_OK;
}

int xfdtd_batch_get_config(xfdtd_batch_t b, int *tile_x, int *tile_y, int *zsplit, int *grid, int *nitems)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (tile_x) *tile_x = fwd_tx(b);
    if (tile_y) *tile_y = fwd_ty(b);
    if (zsplit) *zsplit = b->cfg.zsplit;
    if (grid) *grid = b->bound ? grid_of(b) : b->cfg.grid;
    if (nitems) *nitems = b->nitems;
    return XFDTD_OK;
}

int xfdtd_batch_tune(xfdtd_batch_t b, int force, double *best_ms)
{
    return guarded([&]() -> int {
        Range range("xfdtd_batch_tune");
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
        if (!force) {
            bool hit = false;
            {
                std::lock_guard<std::mutex> lk(g_cache_mu);
                auto it = g_cache.find(b->key);
                std::vector<int> file;
                Config fc;
                if (it == g_cache.end() && tune_cache_lookup("batch:" + b->key, file) && valid_config(b, file, fc)) {
                    it = g_cache.emplace(b->key, fc).first;
                    xlog("batch tune: taken from the tuning file (%s %dx%d tiles, z-split %d, grid %d)",
                         fc.spp == 2 ? "two-step" : "one-step", fc.tile_x, fc.tile_y, fc.zsplit, fc.grid);
                }
                if (it != g_cache.end()) {
                    b->cfg = it->second;
                    hit = true;
                }
            }
            if (hit) {  // the cache lock is released: the adjoint's lookup takes it again
                b->cfg_set = true;
                if (best_ms) *best_ms = -1.0;
                const int rc = build(b);
                return rc ? rc : tune_adjoint(b, true);
            }
        }
        const int ncu = cus();
        std::vector<Config> cands;
        const int tys[3] = {4, 8, 16};
        bool narrow = false;  // 32-column candidates where some box leaves 64-wide tiles part idle
        for (const xfdtd_grid &g : b->g)
            if (g.nx % 64 != 0 && g.nx % 64 <= 32) narrow = true;
        // a batch of boxes one plane deep runs the plane kernel whatever the
        // tiling: only its grid is a choice
        if (b->plane)
            for (int gm : {0, 1, 2}) {
                Config c = b->cfg;
                c.spp = 1;
                c.grid = gm == 0 ? 0 : gm * ncu;
                cands.push_back(c);
            }
        for (int tx : {64, 32}) {
            if (b->plane) break;
            if (tx == 32 && !narrow) continue;
            for (int ty : tys) {
                if (b->dtype == XFDTD_F64 && ty == 16) continue;
                const int zm = model_zsplit(b, tx, ty);
                for (int zs : {1, 2, 4, zm}) {
                    if (zs == zm && (zm == 1 || zm == 2 || zm == 4)) continue;  // already a candidate
                    for (int gm : {0, 1, 2}) {
                        Config c;
                        c.tile_x = tx;
                        c.tile_y = ty;
                        c.zsplit = zs;
                        c.grid = gm == 0 ? 0 : gm * ncu;
                        cands.push_back(c);
                    }
                }
            }
        }
        // FP32: the two-step kernel on 32-column tiles, whole-depth or split
        // z-marches (its chunks start with 10 warm-up planes), or per-box
        // chunks from the schedule model (z-split 0)
        if (b->dtype == XFDTD_F32 && !b->plane)
            for (int ty : {8, 16})
                for (int zs : {1, 2, 0})
                    for (int gm : {0, 1}) {
                        Config c;
                        c.tile_x = 32;
                        c.tile_y = ty;
                        c.zsplit = zs;
                        c.grid = gm == 0 ? 0 : gm * ncu;
                        c.spp = 2;
                        cands.push_back(c);
                    }
        hipEvent_t e0, e1;
        BTRY(hipEventCreate(&e0), "hipEventCreate");
        if (hipEventCreate(&e1) != hipSuccess) {
            hipEventDestroy(e0);
            return set_error(XFDTD_EHIP, "hipEventCreate failed");
        }
        // Two interleaved passes over the candidates; each timing covers about
        // 2 ms of steps and a candidate keeps its faster pass.  The launches
        // alternate between the scratch arrays and a temporary copy of the
        // state, as runs alternate between the fields and the scratch arrays
        // (every launch reads what the previous one wrote; launches that all
        // read the unchanged fields can keep a state of about the size of the
        // last-level cache there); without the temporary they run f -> s.  The
        // bound state is not modified.
        struct Temp {
            void *state = nullptr, *descs = nullptr;
            hipStream_t s;
            ~Temp()
            {
                hipStreamSynchronize(s);
                if (state) hipFree(state);
                if (descs) hipFree(descs);
            }
        } temp{nullptr, nullptr, b->stream};
        std::vector<void *> tmp((size_t)(6 * b->m));
        {
            const size_t esz = b->dtype == XFDTD_F32 ? 4 : 8;
            std::vector<size_t> off;
            size_t total = 0;
            for (int64_t i = 0; i < b->m; ++i) {
                const size_t bytes = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * esz;
                for (int c = 0; c < 6; ++c) {
                    off.push_back(total);
                    total += (bytes + 255) / 256 * 256;
                }
            }
            const size_t dsz = b->dtype == XFDTD_F32 ? sizeof(BoxDesc<float>) : sizeof(BoxDesc<double>);
            if (hipMalloc(&temp.state, std::max<size_t>(256, total)) == hipSuccess &&
                hipMalloc(&temp.descs, dsz * (size_t)b->m) == hipSuccess) {
                for (int64_t i = 0; i < b->m; ++i) {
                    const size_t bytes = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * esz;
                    for (int c = 0; c < 6; ++c) {
                        const size_t k = (size_t)(6 * i + c);
                        tmp[k] = (char *)temp.state + off[k];
                        BTRY(hipMemcpyAsync(tmp[k], b->f[k], bytes, hipMemcpyDeviceToDevice, b->stream),
                             "hipMemcpyAsync");
                    }
                }
            } else {
                (void)hipGetLastError();
                if (temp.state) hipFree(temp.state);
                temp.state = nullptr;
            }
        }
        std::vector<double> per(cands.size(), INFINITY);
        std::vector<int> reps(cands.size(), 0);
        const Config prev = b->cfg;
        int rc = XFDTD_OK;
        auto timed = [&](int r, float *ms) {
            int q = hipEventRecord(e0, b->stream) == hipSuccess ? XFDTD_OK : set_error(XFDTD_EHIP, "event record");
            const void *dd = temp.state ? temp.descs : nullptr;
            for (int i = 0; i < r && !q; ++i) {
                const int par = temp.state ? (i & 1) : 0;
                q = fwd_spp(b) == 2 ? launch_pair(b, par, b->stream, dd) : launch_step(b, par, b->stream, dd);
            }
            if (!q && hipEventRecord(e1, b->stream) != hipSuccess) q = set_error(XFDTD_EHIP, "event record");
            if (!q && hipEventSynchronize(e1) != hipSuccess) q = set_error(XFDTD_EHIP, "event synchronize");
            if (!q && hipEventElapsedTime(ms, e0, e1) != hipSuccess) q = set_error(XFDTD_EHIP, "event time");
            return q;
        };
        for (int pass = 0; pass < 2 && !rc; ++pass)
            for (size_t i = 0; i < cands.size() && !rc; ++i) {
                b->cfg = cands[i];
                rc = build(b);
                if (!rc && temp.state)
                    rc = b->dtype == XFDTD_F32 ? temp_descs_t<float>(b, tmp, temp.descs)
                                               : temp_descs_t<double>(b, tmp, temp.descs);
                if (rc) break;
                float ms = 0.f;
                if (reps[i] == 0) {  // warm-up step, whose time sizes the repetitions
                    rc = timed(1, &ms);
                    reps[i] = (int)std::min(50.0, std::max(3.0, ceil(2.0 / std::max(ms, 1e-3f))));
                }
                if (!rc) rc = timed(reps[i], &ms);
                if (!rc) per[i] = std::min(per[i], (double)ms / reps[i] / cands[i].spp);
            }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc) {  // keep the configuration the batch had (its error, if any, is secondary)
            const std::string msg = xfdtd_last_error();
            b->cfg = prev;
            build(b);
            set_error(rc, "%s", msg.c_str());
            return rc;
        }
        if (log_on())
            for (size_t i = 0; i < cands.size(); ++i)
                xlog("batch tune candidate %s %dx%d tiles, z-split %d, grid %d: %.2f us per step",
                     cands[i].spp == 2 ? "two-step" : "one-step", cands[i].tile_x, cands[i].tile_y, cands[i].zsplit,
                     cands[i].grid, per[i] * 1e3);
        double best = INFINITY;
        Config bestc = prev;
        for (size_t i = 0; i < cands.size(); ++i)
            if (per[i] < best) {
                best = per[i];
                bestc = cands[i];
            }
        b->cfg = bestc;
        b->cfg_set = true;
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            g_cache[b->key] = bestc;
        }
        tune_cache_store("batch:" + b->key, {bestc.tile_x, bestc.tile_y, bestc.zsplit, bestc.grid, bestc.spp});
        xlog("batch tune: %zu candidates, best %s %dx%d tiles, z-split %d, grid %d, %.2f us per step", cands.size(),
             bestc.spp == 2 ? "two-step" : "one-step", bestc.tile_x, bestc.tile_y, bestc.zsplit, bestc.grid,
             best * 1e3);
        if (best_ms) *best_ms = best;
        rc = build(b);
        return rc ? rc : tune_adjoint(b, false);
    });
}

int xfdtd_batch_run(xfdtd_batch_t b, int64_t n)
{
    return guarded([&]() -> int {
        Range range("xfdtd_batch_run");
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
        if (n < 0) return set_error(XFDTD_EINVAL, "n must be >= 0");
        if (n == 0) return XFDTD_OK;
        if (b->graph_n != n || !b->gexec) {
            drop_graph(b);
            BTRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            const int rc = launch_steps(b, n, b->capture);
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
    });
}

int xfdtd_batch_run_eager(xfdtd_batch_t b, int64_t n)
{
    return guarded([&]() -> int {
        Range range("xfdtd_batch_run");
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
        if (n < 0) return set_error(XFDTD_EINVAL, "n must be >= 0");
        return launch_steps(b, n, b->stream);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched checkpointed gradient (the single-box schedule of host.cpp, run for
// all boxes at once: one batched launch per step)
// ---------------------------------------------------------------------------
namespace {

size_t box_field_bytes(const xfdtd_batch_s *b, int64_t i)
{
    const size_t esz = b->dtype == XFDTD_F32 ? 4 : 8;
    const size_t by = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * esz;
    return (by + 255) / 256 * 256;
}

int64_t bseg(int64_t n, int64_t seg)
{
    if (seg > 0) return seg;
    int64_t s = (int64_t)ceil(sqrt(2.0 * (double)(n > 0 ? n : 1)));  // as the single-box default
    return s < 1 ? 1 : s;
}

// Per box: nck checkpoints, two scratch states, and E snapshots of one
// segment, in two sets when there are several segments (the backward pass
// recomputes one segment while it reverses through the next).
uint64_t bws_arrays(int64_t n, int64_t seg)
{
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    return (uint64_t)(6 * nck + 12 + (nck > 1 ? 6 : 3) * (seg - 1));
}

template <typename T>
struct BoxWs {  // the workspace of one box, addressed like host.cpp's layout
    char *ws;
    size_t fb;
    int64_t nck;
    Fields<T> state(int64_t first) const
    {
        Fields<T> f;
        for (int c = 0; c < 6; ++c) f.c[c] = (T *)(ws + (size_t)(first + c) * fb);
        return f;
    }
    Fields<T> ck(int64_t m) const { return state(6 * m); }
    Fields<T> A() const { return state(6 * nck); }
    Fields<T> B() const { return state(6 * nck + 6); }
    // E snapshot i (step s0 + i, i in [1, seg)) of a segment, in snapshot set `set`
    T *segE(int set, int64_t seg, int64_t i, int c) const
    {
        return (T *)(ws + (size_t)(6 * nck + 12 + (int64_t)set * 3 * (seg - 1) + 3 * (i - 1) + c) * fb);
    }
};

template <typename T>
BoxDesc<T> fwd_desc(const xfdtd_batch_s *b, int64_t i, const Fields<T> &in, const Fields<T> &out)
{
    const xfdtd_grid &g = b->g[i];
    BoxDesc<T> d;
    d.f = in;
    d.s = out;
    d.d = Dims{(int)g.nx, (int)g.ny, (int)g.nz};
    const double sp[3] = {g.dx, g.dy, g.dz};
    d.w = fold_weights<T>(b->dt[i], &b->coeffs[12 * i], sp, nullptr);
    d.zchunk = b->plane ? 1
                        : b->fzc.size() == b->g.size() ? b->fzc[(size_t)i]
                                                       : (int)box_zchunk(g, std::max(1, b->cfg.zsplit));
    d.ntx = (int)((g.nx + fwd_tx(b) - 1) / fwd_tx(b));
    d.nty = (int)((g.ny + fwd_ty(b) - 1) / fwd_ty(b));
    d.pad = 0;
    return d;
}

// Tile width of the batched adjoint: the forward's, or 32 columns when every
// box is at most 96 cells wide and 32-column tiles load fewer columns in all
// (tile plus its 4 halo columns, summed over the boxes' rows): nx = 96 loads
// 3 x 36 columns instead of 2 x 68.
int pick_adj_tx(const xfdtd_batch_s *b)
{
    if (b->cfg.tile_x == 32) return 32;
    double c64 = 0, c32 = 0;
    for (const xfdtd_grid &g : b->g) {
        if (g.nx > 96) return 64;
        const double rows = (double)g.ny * (double)g.nz;
        c64 += (double)((g.nx + 63) / 64 * 68) * rows;
        c32 += (double)((g.nx + 31) / 32 * 36) * rows;
    }
    return c32 < c64 ? 32 : 64;
}

// The batched adjoint's tile height, chosen with its work list
// (build_adjoint).
int adj_tile(const xfdtd_batch_s *b)
{
    return b->aty;
}

// The default candidate: one the kernel supports (4 or 8; the 64x8 FP64 tile
// does not fit in LDS).
int adj_tile_default(const xfdtd_batch_s *b)
{
    if (b->dtype == XFDTD_F64 && b->atx == 64) return 4;
    return b->cfg.tile_y > 8 ? 8 : b->cfg.tile_y;
}

template <typename T>
AdjDesc<T> adj_desc(const xfdtd_batch_s *b, int64_t i, const Fields<T> &lin, const Fields<T> &lout,
                    T *const en[3])
{
    const BoxDesc<T> f = fwd_desc<T>(b, i, lin, lout);
    AdjDesc<T> a;
    a.lin = lin;
    a.lout = lout;
    for (int c = 0; c < 3; ++c) a.en[c] = en[c];
    a.d = f.d;
    a.w = f.w;
    a.zchunk = b->azc.empty() ? f.zchunk : b->azc[(size_t)i];
    a.ntx = (int)((b->g[i].nx + b->atx - 1) / b->atx);
    a.nty = (int)((b->g[i].ny + adj_tile(b) - 1) / adj_tile(b));
    a.group = b->plane ? b->agroup : 0;
    return a;
}

// Whether the batched adjoint kernel has an atx x ty tile for this dtype
// (FP64 has no 64x8 or 32x12 tile: their planes exceed the LDS).
bool adj_tile_ok(const xfdtd_batch_s *b, int ty)
{
    if (b->atx == 64) return ty == 4 || (ty == 8 && b->dtype == XFDTD_F32);
    return ty == 4 || ty == 8 || (ty == 12 && b->dtype == XFDTD_F32);
}

// Adjoint work list (tile atx x adj_tile): per-box contiguous items, their
// dispatch order, item ranges per box and gradient scales.  The tiling is the
// timed one (apick) when it was timed for this tile width; otherwise the
// adjoint's z-split is its own: the one whose dispatch order finishes first in
// the list-scheduling model (chunks cost their planes plus 4 warm-up
// iterations; CUs x resident workgroups run at once), fewer chunks on ties.
template <typename T>
int build_adjoint(xfdtd_batch_t b)
{
    int aty = adj_tile_default(b);
    const int warm = 4;
    std::vector<int2> items;
    std::vector<double> cost;
    std::vector<int> run, order;
    bool boxrun = false;
    auto make = [&](int zs) {
        items.clear();
        cost.clear();
        run.clear();
        b->azc.assign((size_t)b->m, 1);
        if (b->plane) {  // tiles per work item from the batch's tile count
            int64_t tiles = 0;
            for (int64_t i = 0; i < b->m; ++i)
                tiles += (int64_t)((b->g[i].nx + b->atx - 1) / b->atx) * ((b->g[i].ny + aty - 1) / aty);
            b->agroup = plane_adj_group(tiles);
        }
        double total = 0, count = 0;
        for (int64_t i = 0; i < b->m; ++i) {
            const xfdtd_grid &g = b->g[i];
            const int zc = (int)box_zchunk(g, zs);
            b->azc[(size_t)i] = zc;
            const double tiles = (double)((g.nx + b->atx - 1) / b->atx) * (double)((g.ny + aty - 1) / aty);
            const int nzc = (int)((g.nz + zc - 1) / zc);
            if (b->plane) {  // items of b->agroup tiles, one pass each
                total += tiles;
                count += ceil(tiles / b->agroup);
                continue;
            }
            total += tiles * ((double)g.nz + (double)nzc * warm);
            count += tiles * nzc;
        }
        if (count > 0x3fffffff) return false;
        const int run_len = run_length(total, count);
        for (int64_t i = 0; i < b->m; ++i) {
            const xfdtd_grid &g = b->g[i];
            const size_t r0 = run.size();
            if (b->plane)
                plane_items((int)i, (int)((g.nx + b->atx - 1) / b->atx) * (int)((g.ny + aty - 1) / aty), b->agroup,
                            run_len, items, cost, run);
            else
                box_items((int)i, (int)((g.nx + b->atx - 1) / b->atx), (int)((g.ny + aty - 1) / aty), (int)g.nz,
                          b->azc[(size_t)i], warm, run_len, items, cost, run);
            if (boxrun)
                for (size_t j = r0; j < run.size(); ++j) run[j] = (int)i;
        }
        order = xcd_schedule(cost, run);
        return true;
    };
    // candidate tile heights: the default, and for FP32 32-column tiles the
    // 32x12 tile (9 waves, two per CU: 1.5 loaded positions per cell against
    // 1.69 at 32x8); costs in position-planes (tile positions x planes)
    std::vector<int> tys = {aty};
    if (b->dtype == XFDTD_F32 && b->atx == 32 && aty != 12) tys.push_back(12);
    int best_zs = 1, best_ty = aty;
    double best = INFINITY;
    const AdjPick &pk = b->apick;
    if (pk.tx == b->atx && adj_tile_ok(b, pk.ty) && pk.zs >= 1 && pk.zs <= 1024) {
        tys.clear();
        best_zs = pk.zs;
        best_ty = pk.ty;
        boxrun = pk.boxrun != 0;
    }
    for (int ty : tys) {
        aty = ty;
        const int occ = std::max(1, adjoint_occupancy<T>(b->atx, ty));
        const int per_xcd = std::max(1, cus() / 8) * occ;
        const double positions = (double)(b->atx + 4) * (double)(ty + 4);
        for (int zs : {1, 2, 3, 4, 6, 8, 12, 16}) {
            if (!make(zs)) continue;
            const double t = simulate_finish(order, cost, per_xcd).first * positions;
            if (t < best * (1.0 - 1e-9)) {
                best = t;
                best_zs = zs;
                best_ty = ty;
            }
        }
    }
    aty = best_ty;
    b->aty = best_ty;
    b->azs = best_zs;
    if (!make(best_zs)) return set_error(XFDTD_EINVAL, "too many work items");
    if (tys.empty())
        xlog("batched adjoint: %dx%d tiles, z-split %d, %s runs (timed), %zu items in %zu slots", b->atx, aty,
             best_zs, boxrun ? "whole-box" : "short", items.size(), order.size());
    else
        xlog("batched adjoint: %dx%d tiles, z-split %d (modelled finish %.0f position-planes), %zu items in %zu slots",
             b->atx, aty, best_zs, best, items.size(), order.size());
    if (order.size() > 0x7fffffff) return set_error(XFDTD_EINVAL, "too many work items");
    std::vector<int> first;
    std::vector<double> scale;
    for (int64_t i = 0; i < b->m; ++i) {
        const double sp[3] = {b->g[i].dx, b->g[i].dy, b->g[i].dz};
        for (int j = 0; j < 12; ++j) scale.push_back(b->dt[i] / sp[j / 4]);
    }
    for (size_t j = 0; j < items.size(); ++j)
        while ((int64_t)first.size() <= items[j].x) first.push_back((int)j);
    while ((int64_t)first.size() <= b->m) first.push_back((int)items.size());
    for (void *p : {(void *)b->d_aitems, (void *)b->d_aorder, (void *)b->d_apart, (void *)b->d_afirst,
                    (void *)b->d_scale, (void *)b->d_grad})
        if (p) hipFree(p);
    b->d_aitems = nullptr;
    b->d_aorder = nullptr;
    b->d_apart = nullptr;
    b->d_afirst = nullptr;
    b->d_scale = nullptr;
    b->d_grad = nullptr;
    BTRY(hipMalloc((void **)&b->d_aitems, sizeof(int2) * std::max<size_t>(1, items.size())), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_aorder, sizeof(int) * std::max<size_t>(1, order.size())), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_apart, sizeof(double) * 12 * std::max<size_t>(1, items.size())), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_afirst, sizeof(int) * first.size()), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_scale, sizeof(double) * scale.size()), "hipMalloc");
    BTRY(hipMalloc((void **)&b->d_grad, sizeof(double) * scale.size()), "hipMalloc");
    if (!items.empty())
        BTRY(hipMemcpy(b->d_aitems, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice), "hipMemcpy");
    if (!order.empty())
        BTRY(hipMemcpy(b->d_aorder, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice), "hipMemcpy");
    BTRY(hipMemcpy(b->d_afirst, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice), "hipMemcpy");
    BTRY(hipMemcpy(b->d_scale, scale.data(), sizeof(double) * scale.size(), hipMemcpyHostToDevice), "hipMemcpy");
    b->naitems = (int)items.size();
    b->naslots = (int)order.size();
    return XFDTD_OK;
}

template <typename T>
int upload(std::vector<T> &host, T **dev)
{
    *dev = nullptr;
    if (host.empty()) return XFDTD_OK;
    BTRY(hipMalloc((void **)dev, sizeof(T) * host.size()), "hipMalloc");
    BTRY(hipMemcpy(*dev, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice), "hipMemcpy");
    return XFDTD_OK;
}

template <typename T>
int bgrad_forward_t(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws)
{
    const int64_t m = b->m;
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    // the last two segments write their E snapshots (as in the single-box
    // forward pass)
    const int64_t s0_keep = (nck >= 2 ? nck - 2 : 0) * seg;
    std::vector<BoxWs<T>> W(m);
    std::vector<Fields<T>> cur(m), fields(m);
    for (int64_t i = 0; i < m; ++i) {
        W[i] = BoxWs<T>{(char *)ws[i], box_field_bytes(b, i), nck};
        for (int c = 0; c < 6; ++c) fields[i].c[c] = (T *)b->f[6 * i + c];
        const Fields<T> ck0 = W[i].ck(0);
        const size_t raw = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * sizeof(T);
        for (int c = 0; c < 6; ++c)
            BTRY(hipMemcpyAsync(ck0.c[c], fields[i].c[c], raw, hipMemcpyDeviceToDevice, b->stream), "hipMemcpyAsync");
        cur[i] = ck0;
    }
    // Every box follows the same schedule, so a step's descriptors are fixed
    // by box 0's source and destination arrays; steps with the same ones
    // (the ping-pong, the snapshot slots of a set) share a descriptor array,
    // which keeps the upload at O(m (n/seg + seg)) descriptors.
    std::vector<BoxDesc<T>> descs;
    std::map<std::array<uintptr_t, 4>, int64_t> seen;
    std::vector<int64_t> off((size_t)n);
    std::vector<Fields<T>> dst(m);
    for (int64_t s = 0; s < n; ++s) {
        for (int64_t i = 0; i < m; ++i) {
            const Fields<T> A = W[i].A(), Bs = W[i].B();
            if (s + 1 == n) {
                dst[i] = fields[i];
            } else if ((s + 1) % seg == 0) {
                dst[i] = W[i].ck((s + 1) / seg);
            } else if (s >= s0_keep) {
                const int64_t k = s / seg, s0 = k * seg;
                for (int c = 0; c < 3; ++c) {
                    dst[i].c[c] = W[i].segE((int)(k & 1), seg, s + 1 - s0, c);
                    dst[i].c[3 + c] = A.c[3 * ((s - s0) & 1) + c];
                }
            } else {
                dst[i] = (cur[i].c[0] == A.c[0]) ? Bs : A;
            }
        }
        const std::array<uintptr_t, 4> key = {(uintptr_t)cur[0].c[0], (uintptr_t)cur[0].c[3],
                                              (uintptr_t)dst[0].c[0], (uintptr_t)dst[0].c[3]};
        auto it = seen.find(key);
        if (it == seen.end()) {
            it = seen.emplace(key, (int64_t)descs.size()).first;
            for (int64_t i = 0; i < m; ++i) descs.push_back(fwd_desc<T>(b, i, cur[i], dst[i]));
        }
        off[(size_t)s] = it->second;
        cur = dst;
    }
    BoxDesc<T> *d_descs = nullptr;
    BTRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    int rc = upload(descs, &d_descs);
    if (rc) return rc;
    for (int64_t s = 0; s < n && !rc; ++s) {
        hipError_t e = b->plane ? launch_batched_plane<T>(d_descs + off[(size_t)s], b->d_items, b->nitems, 0,
                                                          grid_of(b), b->stream)
                                : launch_batched<T>(d_descs + off[(size_t)s], b->d_items, b->nitems, 0,
                                                    b->cfg.tile_x, b->cfg.tile_y, grid_of(b), b->stream);
        if (e != hipSuccess) rc = set_error(XFDTD_EHIP, "batched launch: %s", hipGetErrorString(e));
    }
    hipStreamSynchronize(b->stream);
    if (d_descs) hipFree(d_descs);
    return rc;
}

// Batched backward pass, overlapped like the single-box one: the adjoint
// launches run on the bound stream, segment by segment from the last, while
// segment m - 1 is recomputed from its checkpoints on the batch's second
// stream into the other set of E snapshots (the forward pass wrote those of
// the last two segments).  A recompute waits until the
// adjoint has left the set it overwrites, an adjoint segment until its
// recompute is done.
template <typename T>
int bgrad_backward_t(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws, void *const *lam, double *grad)
{
    const int64_t m = b->m;
    b->atx = b->apick.tx ? b->apick.tx : pick_adj_tx(b);
    int rc = build_adjoint<T>(b);
    if (rc) return rc;
    const int64_t nck = n > 0 ? (n + seg - 1) / seg : 1;
    std::vector<BoxWs<T>> W(m);
    std::vector<Fields<T>> lamU(m), lamS(m), lcur(m), lnext(m);
    for (int64_t i = 0; i < m; ++i) {
        W[i] = BoxWs<T>{(char *)ws[i], box_field_bytes(b, i), nck};
        for (int c = 0; c < 6; ++c) lamU[i].c[c] = (T *)lam[6 * i + c];
        lamS[i] = W[i].B();
        lcur[i] = lamU[i];
        lnext[i] = lamS[i];
    }
    // Descriptors, shared between launches with the same arrays (as in the
    // forward pass): recompute launch l of the whole pass uses rdesc[roff[l]],
    // segment k's recompute launches are [rl[k], rl[k + 1]); adjoint launch l
    // uses adesc[aoff[l]], segment k's adjoint launches are [al[k], aend(k)).
    std::vector<BoxDesc<T>> rdesc;
    std::vector<AdjDesc<T>> adesc;
    std::vector<int64_t> roff, aoff, rl(nck + 1, 0), al(nck + 1, 0);
    std::map<std::array<uintptr_t, 4>, int64_t> rseen, aseen;
    for (int64_t k = 0; k < nck && n > 0; ++k) {
        const int64_t s0 = k * seg, s1 = (s0 + seg < n) ? s0 + seg : n;
        rl[k] = (int64_t)roff.size();
        if (k >= nck - 2) continue;  // the forward pass left these segments' snapshots
        std::vector<Fields<T>> in(m), out(m);
        for (int64_t i = 0; i < m; ++i) in[i] = W[i].ck(k);
        for (int64_t s = s0; s + 1 < s1; ++s) {
            for (int64_t i = 0; i < m; ++i) {
                const Fields<T> A = W[i].A();
                for (int c = 0; c < 3; ++c) {
                    out[i].c[c] = W[i].segE((int)(k & 1), seg, s + 1 - s0, c);
                    out[i].c[3 + c] = A.c[3 * ((s - s0) & 1) + c];
                }
            }
            const std::array<uintptr_t, 4> key = {(uintptr_t)in[0].c[0], (uintptr_t)in[0].c[3],
                                                  (uintptr_t)out[0].c[0], (uintptr_t)out[0].c[3]};
            auto it = rseen.find(key);
            if (it == rseen.end()) {
                it = rseen.emplace(key, (int64_t)rdesc.size()).first;
                for (int64_t i = 0; i < m; ++i) rdesc.push_back(fwd_desc<T>(b, i, in[i], out[i]));
            }
            roff.push_back(it->second);
            in = out;
        }
    }
    rl[nck] = (int64_t)roff.size();
    for (int64_t k = nck - 1; k >= 0 && n > 0; --k) {
        const int64_t s0 = k * seg, s1 = (s0 + seg < n) ? s0 + seg : n;
        al[k] = (int64_t)aoff.size();
        for (int64_t s = s1 - 1; s >= s0; --s) {
            const T *e0 = (s == s0) ? W[0].ck(k).c[0] : W[0].segE((int)(k & 1), seg, s - s0, 0);
            const std::array<uintptr_t, 4> key = {(uintptr_t)lcur[0].c[0], (uintptr_t)lnext[0].c[0],
                                                  (uintptr_t)e0, 0};
            auto it = aseen.find(key);
            if (it == aseen.end()) {
                it = aseen.emplace(key, (int64_t)adesc.size()).first;
                for (int64_t i = 0; i < m; ++i) {
                    T *en[3];
                    for (int c = 0; c < 3; ++c)
                        en[c] = (s == s0) ? W[i].ck(k).c[c] : W[i].segE((int)(k & 1), seg, s - s0, c);
                    adesc.push_back(adj_desc<T>(b, i, lcur[i], lnext[i], en));
                }
            }
            aoff.push_back(it->second);
            for (int64_t i = 0; i < m; ++i) std::swap(lcur[i], lnext[i]);
        }
    }
    // segments are reversed from the last, so segment k's adjoint launches end
    // where segment k - 1's begin
    auto aend = [&](int64_t k) { return k > 0 ? al[k - 1] : (int64_t)aoff.size(); };
    BoxDesc<T> *d_r = nullptr;
    AdjDesc<T> *d_a = nullptr;
    struct Free {
        void *p[2];
        ~Free()
        {
            for (void *q : p)
                if (q) hipFree(q);
        }
    };
    BTRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    rc = upload(rdesc, &d_r);
    Free fr{{d_r, nullptr}};
    if (rc) return rc;
    rc = upload(adesc, &d_a);
    fr.p[1] = d_a;
    if (rc) return rc;
    hipStream_t mainS = b->stream, aux = b->aux;
    BTRY(hipMemsetAsync(b->d_grad, 0, sizeof(double) * 12 * m, mainS), "hipMemsetAsync");
    struct Events {
        std::vector<hipEvent_t> ev;
        hipStream_t s[2];
        ~Events()
        {
            // on every return both streams have drained before the events
            // and descriptors go
            for (hipStream_t q : s) hipStreamSynchronize(q);
            for (hipEvent_t e : ev) hipEventDestroy(e);
        }
    } evs{{}, {mainS, aux}};
    // event slots as in the single-box backward pass: [0] start, [1 + (k & 3)]
    // recompute of segment k done, [5 + (k & 3)] adjoint of segment k done
    // (each record is waited for before its slot is recorded again)
    auto ev_rec = [&](int64_t k) { return evs.ev[(size_t)(1 + (k & 3))]; };
    auto ev_adj = [&](int64_t k) { return evs.ev[(size_t)(5 + (k & 3))]; };
    for (int k = 0; k < 9; ++k) {
        hipEvent_t e;
        BTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        evs.ev.push_back(e);
    }
    BTRY(hipEventRecord(evs.ev[0], mainS), "hipEventRecord");
    BTRY(hipStreamWaitEvent(aux, evs.ev[0], 0), "hipStreamWaitEvent");
    auto recompute = [&](int64_t k) -> int {
        for (int64_t l = rl[k]; l < rl[k + 1]; ++l) {
            hipError_t e = b->plane ? launch_batched_plane<T>(d_r + roff[(size_t)l], b->d_items, b->nitems, 0,
                                                              grid_of(b), aux)
                                    : launch_batched<T>(d_r + roff[(size_t)l], b->d_items, b->nitems, 0,
                                                        b->cfg.tile_x, b->cfg.tile_y, grid_of(b), aux);
            if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched gradient launch: %s", hipGetErrorString(e));
        }
        BTRY(hipEventRecord(ev_rec(k), aux), "hipEventRecord");
        return XFDTD_OK;
    };
    // adjoint grid: one workgroup per dispatch slot
    const int ga = b->naslots;
    bool first = true;
    for (int64_t k = nck - 1; k >= 0 && n > 0; --k) {
        if (k < nck - 2) BTRY(hipStreamWaitEvent(mainS, ev_rec(k), 0), "hipStreamWaitEvent");
        for (int64_t l = al[k]; l < aend(k); ++l) {
            hipError_t e = launch_batched_adjoint<T>(d_a + aoff[(size_t)l], b->d_aitems, b->d_aorder, b->naslots,
                                                     b->d_apart, first ? 0 : 1, b->atx, adj_tile(b), ga, mainS,
                                                     b->plane);
            if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched gradient launch: %s", hipGetErrorString(e));
            first = false;
        }
        BTRY(hipEventRecord(ev_adj(k), mainS), "hipEventRecord");
        if (k >= 2) {  // segment k - 2 reuses this segment's E set
            BTRY(hipStreamWaitEvent(aux, ev_adj(k), 0), "hipStreamWaitEvent");
            rc = recompute(k - 2);
            if (rc) return rc;
        }
    }
    if (!first) {
        hipError_t e = launch_reduce_boxes(b->d_apart, b->d_afirst, (int)m, b->d_scale, b->d_grad, mainS);
        if (e != hipSuccess) return set_error(XFDTD_EHIP, "reduce launch: %s", hipGetErrorString(e));
    }
    for (int64_t i = 0; i < m; ++i)
        if (lcur[i].c[0] != lamU[i].c[0]) {
            const size_t raw = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * sizeof(T);
            for (int c = 0; c < 6; ++c)
                BTRY(hipMemcpyAsync(lamU[i].c[c], lcur[i].c[c], raw, hipMemcpyDeviceToDevice, mainS), "hipMemcpyAsync");
        }
    BTRY(hipMemcpyAsync(grad, b->d_grad, sizeof(double) * 12 * m, hipMemcpyDeviceToHost, mainS), "hipMemcpyAsync");
    BTRY(hipStreamSynchronize(mainS), "hipStreamSynchronize");
    BTRY(hipStreamSynchronize(aux), "hipStreamSynchronize");
    return XFDTD_OK;
}

// Timing of the batched adjoint's tilings: the model's choice and, per tile
// height (the default, and 32x12 for FP32 32-column tiles), z-splits 1-4 and
// the model's, each with short runs and with whole-box runs.  The launches
// read the bound state as both lambda and primal E and write only the
// scratch arrays (and the per-item gradient sums, which every backward pass
// overwrites); two interleaved passes of about 2 ms each, a candidate keeping
// its faster.
template <typename T>
int tune_adjoint_t(xfdtd_batch_t b)
{
    const int tx0 = pick_adj_tx(b);
    std::vector<AdjPick> cands;
    // widths: the column-count rule's, and 64 where it chose 32 (the 64-column
    // kernel does more per cell it computes, which can outweigh idle columns)
    for (int tx : {tx0, 64}) {
        if (tx == 64 && tx0 == 64 && !cands.empty()) continue;
        b->atx = tx;
        b->apick = AdjPick{};
        const int rc = build_adjoint<T>(b);  // the model's choice for this width
        if (rc) return rc;
        std::vector<int> tys = {adj_tile_default(b)};
        if (b->dtype == XFDTD_F32 && tx == 32 && tys[0] != 12) tys.push_back(12);
        std::vector<int> zss = {1, 2, 3, 4};
        if (std::find(zss.begin(), zss.end(), b->azs) == zss.end()) zss.push_back(b->azs);
        for (int ty : tys)
            for (int zs : zss)
                for (int run : {0, 1}) cands.push_back(AdjPick{tx, ty, zs, run});
    }
    int rc = XFDTD_OK;
    struct Ev {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Ev()
        {
            for (hipEvent_t x : e)
                if (x) hipEventDestroy(x);
        }
    } ev;
    BTRY(hipEventCreate(&ev.e[0]), "hipEventCreate");
    BTRY(hipEventCreate(&ev.e[1]), "hipEventCreate");
    // the primal E of the timed launches: a copy of the bound E, so that a
    // launch reads as many distinct bytes as in a backward pass (without a
    // copy, E^n is the adjoint input's first three arrays)
    struct TempE {
        void *p = nullptr;
        hipStream_t s;
        ~TempE()
        {
            hipStreamSynchronize(s);
            if (p) hipFree(p);
        }
    } tempE{nullptr, b->stream};
    std::vector<T *> ecopy((size_t)(3 * b->m), nullptr);
    {
        std::vector<size_t> off;
        size_t total = 0;
        for (int64_t i = 0; i < b->m; ++i)
            for (int c = 0; c < 3; ++c) {
                off.push_back(total);
                total += ((size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * sizeof(T) + 255) / 256 * 256;
            }
        if (hipMalloc(&tempE.p, std::max<size_t>(256, total)) == hipSuccess) {
            for (int64_t i = 0; i < b->m; ++i)
                for (int c = 0; c < 3; ++c) {
                    const size_t k = (size_t)(3 * i + c);
                    ecopy[k] = (T *)((char *)tempE.p + off[k]);
                    BTRY(hipMemcpyAsync(ecopy[k], b->f[(size_t)(6 * i + c)],
                                        (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * sizeof(T),
                                        hipMemcpyDeviceToDevice, b->stream),
                         "hipMemcpyAsync");
                }
        } else {
            (void)hipGetLastError();
            tempE.p = nullptr;
            std::fill(ecopy.begin(), ecopy.end(), nullptr);
        }
    }
    std::vector<double> per(cands.size(), INFINITY);
    std::vector<int> reps(cands.size(), 0);
    for (int pass = 0; pass < 2 && !rc; ++pass)
        for (size_t c = 0; c < cands.size() && !rc; ++c) {
            b->apick = cands[c];
            b->atx = cands[c].tx;
            rc = build_adjoint<T>(b);
            if (rc) break;
            std::vector<AdjDesc<T>> descs;
            for (int64_t i = 0; i < b->m; ++i) {
                Fields<T> fin, fout;
                T *en[3];
                for (int k = 0; k < 6; ++k) {
                    fin.c[k] = (T *)b->f[(size_t)(6 * i + k)];
                    fout.c[k] = (T *)b->s[(size_t)(6 * i + k)];
                }
                for (int k = 0; k < 3; ++k) en[k] = ecopy[(size_t)(3 * i + k)] ? ecopy[(size_t)(3 * i + k)] : fin.c[k];
                descs.push_back(adj_desc<T>(b, i, fin, fout, en));
            }
            AdjDesc<T> *d = nullptr;
            rc = upload(descs, &d);
            if (rc) break;
            auto timed = [&](int r, float *ms) -> int {
                BTRY(hipEventRecord(ev.e[0], b->stream), "hipEventRecord");
                for (int i = 0; i < r; ++i) {
                    const hipError_t e = launch_batched_adjoint<T>(d, b->d_aitems, b->d_aorder, b->naslots,
                                                                   b->d_apart, 0, b->atx, adj_tile(b),
                                                                   b->naslots, b->stream, b->plane);
                    if (e != hipSuccess) return set_error(XFDTD_EHIP, "batched adjoint launch: %s", hipGetErrorString(e));
                }
                BTRY(hipEventRecord(ev.e[1], b->stream), "hipEventRecord");
                BTRY(hipEventSynchronize(ev.e[1]), "hipEventSynchronize");
                BTRY(hipEventElapsedTime(ms, ev.e[0], ev.e[1]), "hipEventElapsedTime");
                return XFDTD_OK;
            };
            float ms = 0.f;
            if (reps[c] == 0) {  // warm-up launch, whose time sizes the repetitions
                rc = timed(1, &ms);
                reps[c] = (int)std::min(50.0, std::max(3.0, ceil(2.0 / std::max(ms, 1e-3f))));
            }
            if (!rc) rc = timed(reps[c], &ms);
            if (!rc) per[c] = std::min(per[c], (double)ms / reps[c]);
            hipStreamSynchronize(b->stream);
            hipFree(d);
        }
    if (rc) {
        b->apick = AdjPick{};
        b->atx = tx0;
        return rc;
    }
    size_t best = 0;
    for (size_t c = 0; c < cands.size(); ++c) {
        xlog("batched adjoint tune candidate %dx%d tiles, z-split %d, %s runs: %.2f us per step", cands[c].tx,
             cands[c].ty, cands[c].zs, cands[c].boxrun ? "whole-box" : "short", per[c] * 1e3);
        if (per[c] < per[best]) best = c;
    }
    b->apick = cands[best];
    b->atx = b->apick.tx;
    xlog("batched adjoint tune: %zu candidates, best %dx%d tiles, z-split %d, %s runs, %.2f us per step",
         cands.size(), b->apick.tx, b->apick.ty, b->apick.zs, b->apick.boxrun ? "whole-box" : "short",
         per[best] * 1e3);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_acache[b->key] = b->apick;
    }
    tune_cache_store("batchadj:" + b->key, {b->apick.tx, b->apick.ty, b->apick.zs, b->apick.boxrun});
    return build_adjoint<T>(b);
}

// The adjoint's tiling for xfdtd_batch_tune.  lookup: take a choice of this
// process or of the tuning file for the batch's shapes if there is one (else
// keep the model's), instead of timing.
int tune_adjoint(xfdtd_batch_t b, bool lookup)
{
    if (lookup) {
        b->atx = pick_adj_tx(b);
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_acache.find(b->key);
        std::vector<int> v;
        if (it != g_acache.end()) {
            b->apick = it->second;
        } else if (tune_cache_lookup("batchadj:" + b->key, v) && v.size() == 4 && (v[0] == 32 || v[0] == 64) &&
                   (v[3] == 0 || v[3] == 1) && v[2] >= 1 && v[2] <= 1024) {
            const int tx = b->atx;
            b->atx = v[0];
            if (adj_tile_ok(b, v[1])) {
                b->apick = AdjPick{v[0], v[1], v[2], v[3]};
                g_acache[b->key] = b->apick;
            } else {
                b->atx = tx;
            }
        }
        return XFDTD_OK;
    }
    return b->dtype == XFDTD_F32 ? tune_adjoint_t<float>(b) : tune_adjoint_t<double>(b);
}

// Workspaces: present, aligned, large enough and disjoint from each other.
// Forward (lam == nullptr): also disjoint from the bound arrays, which it
// reads and writes.  Backward: the lambda arrays (it does not touch the bound
// arrays) disjoint from each other and from the workspaces.
int check_bws(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws, const uint64_t *ws_bytes,
              void *const *lam = nullptr)
{
    if (!b) return set_error(XFDTD_EINVAL, "null handle");
    if (!b->bound) return set_error(XFDTD_ESTATE, "bind the batch first");
    if (n < 0 || n > ((int64_t)1 << 40)) return set_error(XFDTD_EINVAL, "n must be in [0, 2^40]");
    if (seg > ((int64_t)1 << 40)) return set_error(XFDTD_EINVAL, "seg must be <= 2^40");
    if (!ws || !ws_bytes) return set_error(XFDTD_EINVAL, "null workspace list");
    for (int64_t i = 0; i < b->m; ++i)
        if ((double)bws_arrays(n, seg) * (double)box_field_bytes(b, i) >= 0x1p63)
            return set_error(XFDTD_EINVAL, "box %lld: workspace size exceeds 2^63 bytes", (long long)i);
    const size_t esz = b->dtype == XFDTD_F32 ? 4 : 8;
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    for (int64_t i = 0; i < b->m; ++i) {
        if (!ws[i] || (uintptr_t)ws[i] % 256)
            return set_error(XFDTD_EINVAL, "box %lld: workspace null or not 256-byte aligned", (long long)i);
        const uint64_t need = bws_arrays(n, seg) * box_field_bytes(b, i);
        if (ws_bytes[i] < need) return set_error(XFDTD_EINVAL, "box %lld: workspace too small", (long long)i);
        spans.push_back({(uintptr_t)ws[i], (uintptr_t)ws[i] + need});
        const size_t bytes = (size_t)b->g[i].nx * b->g[i].ny * b->g[i].nz * esz;
        for (int c = 0; c < 6; ++c) {
            if (lam) {
                spans.push_back({(uintptr_t)lam[6 * i + c], (uintptr_t)lam[6 * i + c] + bytes});
            } else {
                spans.push_back({(uintptr_t)b->f[6 * i + c], (uintptr_t)b->f[6 * i + c] + bytes});
                spans.push_back({(uintptr_t)b->s[6 * i + c], (uintptr_t)b->s[6 * i + c] + bytes});
            }
        }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second)
            return set_error(XFDTD_EINVAL, "workspaces, lambda arrays and bound arrays must not overlap");
    return XFDTD_OK;
}

// At most this many workspace lists per batch are remembered as holding a
// forward pass; the oldest is forgotten first.
constexpr size_t kMaxTapes = 64;

// Forget every remembered workspace list that overlaps one of ws[0..m).
void drop_tapes(xfdtd_batch_t b, void *const *ws, int64_t n, int64_t seg)
{
    std::vector<xfdtd_batch_s::Tape> &t = b->tapes;
    if (t.empty()) return;
    // the new workspaces are disjoint (checked), so sorted by start their ends
    // are sorted too: a span [e0, e1) meets one of them iff the first whose
    // end lies beyond e0 starts before e1
    std::vector<std::pair<uintptr_t, uintptr_t>> span;  // (end, start)
    for (int64_t i = 0; i < b->m; ++i) {
        const uintptr_t a0 = (uintptr_t)ws[i];
        span.push_back({a0 + bws_arrays(n, seg) * box_field_bytes(b, i), a0});
    }
    std::sort(span.begin(), span.end());
    auto hit = [&](const xfdtd_batch_s::Tape &e) {
        for (int64_t j = 0; j < b->m; ++j) {
            const uintptr_t e0 = e.ws[j], e1 = e0 + e.arrays * box_field_bytes(b, j);
            auto it = std::upper_bound(span.begin(), span.end(), std::make_pair(e0, UINTPTR_MAX));
            if (it != span.end() && it->second < e1) return true;
        }
        return false;
    };
    t.erase(std::remove_if(t.begin(), t.end(), hit), t.end());
}

}  // namespace

extern "C" {

int xfdtd_batch_grad_workspace(xfdtd_batch_t b, int64_t n, int64_t seg, uint64_t *bytes)
{
    return guarded([&]() -> int {
        if (!b || !bytes) return set_error(XFDTD_EINVAL, "null argument");
        if (n < 0 || n > ((int64_t)1 << 40)) return set_error(XFDTD_EINVAL, "n must be in [0, 2^40]");
        if (seg > ((int64_t)1 << 40)) return set_error(XFDTD_EINVAL, "seg must be <= 2^40");
        seg = bseg(n, seg);
        for (int64_t i = 0; i < b->m; ++i)
            if ((double)bws_arrays(n, seg) * (double)box_field_bytes(b, i) >= 0x1p63)
                return set_error(XFDTD_EINVAL, "box %lld: workspace size exceeds 2^63 bytes", (long long)i);
        for (int64_t i = 0; i < b->m; ++i) bytes[i] = bws_arrays(n, seg) * box_field_bytes(b, i);
        return XFDTD_OK;
    });
}

int xfdtd_batch_grad_forward(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws, const uint64_t *ws_bytes)
{
    return guarded([&]() -> int {
        Range range("xfdtd_batch_grad_forward");
        seg = bseg(n, seg);
        int rc = check_bws(b, n, seg, ws, ws_bytes);
        if (rc) return rc;
        drop_tapes(b, ws, n, seg);
        rc = b->dtype == XFDTD_F32 ? bgrad_forward_t<float>(b, n, seg, ws) : bgrad_forward_t<double>(b, n, seg, ws);
        if (rc) return rc;
        if (b->tapes.size() >= kMaxTapes) b->tapes.erase(b->tapes.begin());
        xfdtd_batch_s::Tape t{{}, bws_arrays(n, seg), n, seg};
        for (int64_t i = 0; i < b->m; ++i) t.ws.push_back((uintptr_t)ws[i]);
        b->tapes.push_back(std::move(t));
        return XFDTD_OK;
    });
}

int xfdtd_batch_grad_backward(xfdtd_batch_t b, int64_t n, int64_t seg, void *const *ws, const uint64_t *ws_bytes,
                              void *const *lam, double *grad)
{
    return guarded([&]() -> int {
        Range range("xfdtd_batch_grad_backward");
        seg = bseg(n, seg);
        if (!b) return set_error(XFDTD_EINVAL, "null handle");
        if (!lam || !grad) return set_error(XFDTD_EINVAL, "null argument");
        for (int64_t i = 0; i < 6 * b->m; ++i)
            if (!lam[i]) return set_error(XFDTD_EINVAL, "lam[%lld] is null", (long long)i);
        int rc = check_bws(b, n, seg, ws, ws_bytes, lam);
        if (rc) return rc;
        auto it = std::find_if(b->tapes.begin(), b->tapes.end(), [&](const xfdtd_batch_s::Tape &e) {
            if (e.n != n || e.seg != seg) return false;
            for (int64_t i = 0; i < b->m; ++i)
                if (e.ws[i] != (uintptr_t)ws[i]) return false;
            return true;
        });
        if (it == b->tapes.end())
            return set_error(XFDTD_EINVAL, "the workspaces hold no forward pass of n = %lld, seg = %lld on this batch "
                                           "(a backward pass consumes it; run xfdtd_batch_grad_forward again)",
                             (long long)n, (long long)seg);
        b->tapes.erase(it);
        return b->dtype == XFDTD_F32 ? bgrad_backward_t<float>(b, n, seg, ws, lam, grad)
                                     : bgrad_backward_t<double>(b, n, seg, ws, lam, grad);
    });
}

}  // extern "C"
