// Internal declarations shared by the host runtime and the HIP kernels of
// libxfdtd.  Not part of the public interface (include/xfdtd.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <exception>
#include <string>
#include <vector>
#include <new>

#include "../../include/xfdtd.h"

namespace xfdtd {

// Folded weights of one step, in the arithmetic type T.
//   wc[a] = dt (alpha_a + delta_a) / d_a   centre weight of the smoothing star
//   wd[a] = dt delta_a / d_a               along-axis neighbours of the star
//   wb[a][0/1] = dt beta_a,t / d_a         transverse neighbours (t1, t2)
//   wa[a] = dt / d_a                       Yee difference of the Ampere update
// The Faraday increment of a B component is a difference of two "stars"
//   S_a[g](p) = wc g(p) + wd (g(p+e_a) + g(p-e_a)) + sum_t wb_t (g(p+e_t) + g(p-e_t))
// applied to the plain forward difference g(q) = X[q+e_a] - X[q] of an E
// component; this is the extended difference D*_a of Sec. 2 regrouped (the
// delta pair X[p+2e_a] - X[p-e_a] is the sum of three consecutive g).
template <typename T>
struct Weights {
    T wc[3], wd[3], wb[3][2], wa[3];
};

// Pointers of one state (six components) of a box.
template <typename T>
struct Fields {
    T *c[6];  // Ex, Ey, Ez, Bx, By, Bz
};

struct Dims {
    int nx, ny, nz;
};

// Copies a prefetched value into a fresh register at the point where it is
// consumed.  The z-marching kernels keep two alternating sets of prefetch
// registers; without an explicit copy the register allocator may keep a
// consumed value in its prefetch register for the rest of the iteration and
// then move the next load's result at the loop back-edge, which makes the
// wave wait for that load (and the iteration's stores) there.
__device__ __forceinline__ float take(float v)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

__device__ __forceinline__ double take(double v)
{
    double r;
    asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// Launchers (kernels_step.hip).  All return hipSuccess or the launch error.
template <typename T>
hipError_t launch_faraday(const Fields<T> &f, Dims d, const Weights<T> &w, hipStream_t s);
// j (nullable): three device arrays of the current J^{n+1/2}; E -= wj J.
template <typename T>
hipError_t launch_ampere(const Fields<T> &f, Dims d, const Weights<T> &w, hipStream_t s,
                         const T *const *j = nullptr, T wj = T(0));
// One fused step from `in` to `out` (distinct buffers).  tile_x: columns per
// tile (64 or 32), tile_y: rows per tile (4, 8, or 16 in FP32), zchunk:
// planes per workgroup (>= 1).
template <typename T>
hipError_t launch_fused(const Fields<T> &in, const Fields<T> &out, Dims d, const Weights<T> &w, int tile_x,
                        int tile_y, int zchunk, hipStream_t s);

// Two fused steps in one launch from `in` to `out` (distinct buffers): the
// same per-cell arithmetic, one pass over HBM.  FP32; tile_x x tile_y output
// tiles 32x8 or 32x16, zchunk planes per workgroup (>= 1).
// hipErrorInvalidValue for any other tiling or dtype.
template <typename T>
hipError_t launch_blocked2(const Fields<T> &in, const Fields<T> &out, Dims d, const Weights<T> &w, int tile_x,
                           int tile_y, int zchunk, hipStream_t s);
template <typename T>
int blocked2_occupancy(int tile_x, int tile_y);

// Workgroups of the fused step (tile_x x tile_y tiles) resident per CU on
// the current device, from the HIP occupancy calculator; 0 if unknown (no
// device, unsupported tile).
template <typename T>
int fused_occupancy(int tile_x, int tile_y);

// One box of a batch: state f and scratch s (the step alternates between
// them), its grid, weights and tiling (tile_x x tile_y x zchunk, ntx x nty
// tiles per z-chunk).
template <typename T>
struct BoxDesc {
    Fields<T> f, s;
    Dims d;
    Weights<T> w;
    int zchunk, ntx, nty, pad;
};
// Batched fused step over a work list of (box, tile) pairs (device arrays).
// grid: persistent workgroup count (<= 0: one per item).
template <typename T>
hipError_t launch_batched(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int tile_x,
                          int tile_y, int grid, hipStream_t s);

// Batched plane step (every box one plane deep): the boxes' ntx / nty count
// plane tiles (plane_tile_x() x plane_tile_y(dtype) cells).
template <typename T>
hipError_t launch_batched_plane(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int grid,
                                hipStream_t s);
int plane_tile_x();
int plane_tile_y(int dtype);

// Batched two-step launch (FP32): every box advances two steps; the boxes'
// tilings must be 32 x tile_y (tile_y 8 or 16).  hipErrorInvalidValue for
// other tilings or dtypes.
template <typename T>
hipError_t launch_batched2(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int tile_y,
                           int grid, hipStream_t s);

// Adjoint step (kernels_adjoint.hip): lin -> lout (distinct buffers), primal
// E of the step in en[3]; per-workgroup unscaled gradient sums in partials
// (adjoint_blocks(...) x 12 doubles).
struct Scale12 {
    double s[12];
};
// Tiles of tile_x (64 or 32) x tile_y (4, or 8 in FP32) cells.
int adjoint_blocks(Dims d, int tile_x, int tile_y, int zchunk);
// Workgroups of the adjoint step (tile_x x tile_y tiles) resident per CU, or 0.
template <typename T>
int adjoint_occupancy(int tile_x, int tile_y);
// accumulate != 0: add to the per-workgroup slots instead of overwriting.
template <typename T>
hipError_t launch_adjoint(const Fields<T> &lin, const Fields<T> &lout, const T *const en[3], Dims d,
                          const Weights<T> &w, int tile_x, int tile_y, int zchunk, double *partials,
                          int accumulate, hipStream_t s);
// One box of a batched adjoint step: lambda in/out, the step's primal E.
template <typename T>
struct AdjDesc {
    Fields<T> lin, lout;
    const T *en[3];
    Dims d;
    Weights<T> w;
    int zchunk, ntx, nty, group;  // group: tiles per work item of a one-plane box
};
// Most tiles of one plane per workgroup of the adjoint's one-plane pass
// (boxes one plane deep): a workgroup's tiles share one gradient reduction.
constexpr int kPlaneAdjTiles = 16;
// Tiles per workgroup of the one-plane pass over `tiles` tiles in all: as
// many as still leave two workgroups per CU of the current device, 1 to
// kPlaneAdjTiles.
int plane_adj_group(int64_t tiles);
// plane: every box is one plane deep, and work item (b, g) is the tiles
// [g G, (g + 1) G) of box b (fewer at its end), G = boxes[b].group.
template <typename T>
hipError_t launch_batched_adjoint(const AdjDesc<T> *boxes, const int2 *items, const int *order, int nslots,
                                 double *partials, int accumulate, int tile_x, int tile_y, int grid, hipStream_t s,
                                 bool plane = false);
// grad[12b + j] += scale[12b + j] * sum_{i in [first[b], first[b+1])} partials[12i + j]
hipError_t launch_reduce_boxes(const double *partials, const int *first, int nboxes, const double *scale,
                               double *grad, hipStream_t s);
// grad[j] += sc.s[j] * sum over blocks of partials[b*12 + j]; consumes
// partials (above 1024 blocks the sums of 256-block chunks overwrite them).
hipError_t launch_reduce_partials(double *partials, int nblocks, const Scale12 &sc, double *grad, hipStream_t s);

// Diagnostics (kernels_diag.hip).
template <typename T>
hipError_t launch_divergence(const Fields<T> &f, Dims d, const double coeffs[12],
                             const double sp[3], T *div_star_b, T *div_e, hipStream_t s);
template <typename T>
hipError_t launch_divergence_max(const Fields<T> &f, Dims d, const double coeffs[12],
                                 const double sp[3], const T *ref_b, const T *ref_e,
                                 double *partials, int nblocks, hipStream_t s);
hipError_t launch_dispersion(const double *k, int64_t n, double dt, const double coeffs[12],
                             const double sp[3], double *omega, double *vph, double *vg,
                             unsigned int *bad, hipStream_t s);

// Dispersion norm (kernels_diag.hip): f_w and its derivatives with respect to
// the 12 coefficients and dt, out[15] on the device (f, d/dc[12], d/ddt, then
// the number of samples with dt^2 F outside (0, 1)).  `bad` must be 0 on
// entry and is left 0.
struct NormArgs {
    double c[12];
    double sp[3];
    double dt;
    double width;  // weight 1: w = exp(-sum_{t = y, z} (k_t d_t / width)^2)
    int64_t n;     // midpoints per axis
    int dims;      // 2 (k_z = 0) or 3
    int weight;    // 0: w = 1
};
hipError_t launch_norm(const NormArgs &args, double *partials, int nblocks, unsigned int *bad, double *out,
                       hipStream_t s);

// Host helpers shared by the single-box and batched front ends (host.cpp).
// F_min, F_max of the dispersion right-hand side over the whole zone
// (dims = 2: the k_z = 0 plane).  umax (optional) receives
// u_a = sin^2(k_a d_a / 2) at the maximum.
void f_range(const double sp[3], const double *c, double *out_lo, double *out_hi, int dims = 3,
             double umax[3] = nullptr);
// Fold dt*coef/d_a into the star weights, computed in double and rounded
// once to T; out15 receives the T values as doubles (xfdtd_get_weights order).
template <typename T>
Weights<T> fold_weights(double dt, const double *coeffs, const double sp[3], double out15[15])
{
    Weights<T> w;
    for (int a = 0; a < 3; ++a) {
        const double *c = coeffs + 4 * a;
        const double s = dt / sp[a];
        w.wc[a] = (T)(s * (c[0] + c[3]));
        w.wd[a] = (T)(s * c[3]);
        w.wb[a][0] = (T)(s * c[1]);
        w.wb[a][1] = (T)(s * c[2]);
        w.wa[a] = (T)s;
        if (out15) {
            out15[5 * a + 0] = (double)w.wc[a];
            out15[5 * a + 1] = (double)w.wd[a];
            out15[5 * a + 2] = (double)w.wb[a][0];
            out15[5 * a + 3] = (double)w.wb[a][1];
            out15[5 * a + 4] = (double)w.wa[a];
        }
    }
    return w;
}
// Record an error message (thread-local, in a fixed buffer: recording never
// allocates or throws) and return code.
int set_error(int code, const char *fmt, ...);

// Runs the body of a C entry point: a C++ exception (a failed host
// allocation in a std::vector or std::map, a std::system_error from a
// mutex) becomes an error code instead of unwinding into the C caller.
// Instrumentation.  log_on(): XFDTD_LOG=1 in the environment (read once);
// xlog() prints one "[xfdtd] ..." line to stderr when it is set.  Range marks
// a roctx range from construction to destruction (host time of the calls it
// encloses; rocprofv3 --marker-trace records it).
bool log_on();
void xlog(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
struct Range {
    explicit Range(const char *name) noexcept;
    ~Range();
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Persistent tuning results: with XFDTD_TUNE_CACHE=<file> in the environment
// the tuners look a configuration up there when they have none in memory,
// and append the one they time.  A line is "<device> <key> <values...>",
// <device> being the GPU's architecture name and CU count; the last line of
// a key wins.  I/O errors and malformed lines are ignored.
bool tune_cache_lookup(const std::string &key, std::vector<int> &vals);
void tune_cache_store(const std::string &key, const std::vector<int> &vals);

template <typename F>
int guarded(F &&f) noexcept
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return set_error(XFDTD_EINVAL, "out of host memory");
    } catch (const std::exception &e) {
        return set_error(XFDTD_EINVAL, "%s", e.what());
    } catch (...) {
        return set_error(XFDTD_EINVAL, "unexpected C++ exception");
    }
}

}  // namespace xfdtd
