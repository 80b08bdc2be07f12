// Time-step kernels of libxfdtd for gfx950 (CDNA4, wave64).
//
// One step advances (E^n, B^{n-1/2}) to (E^{n+1}, B^{n+1/2}): the Faraday
// update with the extended difference D* (App. A, eq. update1-3; D* from
// Sec. 2) followed by the Yee Ampere update (eq. update4-6; J = 0 except in
// the unfused Ampere kernel, which optionally subtracts dt J).
//
// The extended difference is evaluated as a 7-point "star" of the plain
// forward difference g(q) = X[q+e_a] - X[q] (see Weights in
// xfdtd_internal.h): per B component two stars, each of 7 g values, instead
// of 2 x 12 raw taps.  The regrouping is exact in real arithmetic.
//
//   faraday_kernel / ampere_kernel : one thread per cell (x from the grid,
//       y and z looping over a grid capped at 65535 blocks), in place,
//       periodic indexing; neighbours come through the L1/L2 caches.
//   fused_step_kernel : out of place.  A workgroup owns a TX x TY tile of
//       (x, y) columns (TX = 64 or 32) and marches a chunk of z-planes.  Per
//       plane it stages
//       the next E plane (with a 2-cell halo) in LDS, forms the six g fields
//       on the tile plus a 2/1-cell halo, evaluates B^{n+1/2} on the tile plus
//       a 1-cell halo on the low x and y sides (redundantly with the
//       neighbouring tile), and then E^{n+1} on the tile.  Values a lane needs
//       along z (g at k-1, k, k+1; E at k, k+1, k+2; B^{n+1/2} at k-1) are kept
//       in registers, so z-neighbours never touch LDS.  One barrier per plane
//       (the Ampere update lags one plane).  Each of the 12 field
//       values per cell is read and written once (48 B FP32 / 96 B FP64 per
//       cell-update); halo re-reads of neighbouring tiles add about a fifth
//       to the reads where they miss the XCD's L2.

#include <stdlib.h>

#include <algorithm>

#include <type_traits>

#include "xfdtd_internal.h"

namespace xfdtd {

namespace {

__device__ __forceinline__ int wrap(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

// S_a[g](p) for one g field: centre, along-axis pair, two transverse pairs.
template <typename T>
__device__ __forceinline__ T star(T wc, T wd, T wb0, T wb1, T c, T ap, T am, T t1p, T t1m, T t2p,
                                  T t2m)
{
    return wc * c + wd * (ap + am) + wb0 * (t1p + t1m) + wb1 * (t2p + t2m);
}

// One Ampere component: e + wa1 (b1 - b1m) - wa2 (b2 - b2m)
template <typename T>
__device__ __forceinline__ T ampere_eval(T e, T wa1, T b1, T b1m, T wa2, T b2, T b2m)
{
    return e + (wa1 * (b1 - b1m) - wa2 * (b2 - b2m));
}

template <typename T>
__device__ __forceinline__ void nt_store(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Field pointers in the global address space.  The batched kernels read
// their pointers from a descriptor in memory, so the compiler cannot infer the
// address space and would emit flat accesses, which also count against the
// LDS wait counter and so stall every LDS wait on outstanding field loads.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ void nt_store(gptr<T> p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Element `off` of a z-plane whose base pointer is uniform across the
// workgroup: the byte offset is formed in 32 bits (planes are limited to
// 2^28 cells on the host, < 2^31 bytes in FP64), so a load takes a scalar
// base and a 32-bit per-lane offset and needs no 64-bit address arithmetic
// per lane.  (The compiler emits the non-temporal store below with a 64-bit
// vector address: one 64-bit add per store.)
template <typename T>
__device__ __forceinline__ T ld_plane(gptr<const T> plane, uint32_t off)
{
    return *(gptr<const T>)((gptr<const char>)plane + off * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void st_plane(gptr<T> plane, uint32_t off, T v)
{
    __builtin_nontemporal_store(v, (gptr<T>)((gptr<char>)plane + off * (uint32_t)sizeof(T)));
}

// ---------------------------------------------------------------------------
// unfused Faraday: B += S(D* E) in place
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void faraday_cell(const Fields<T> &f, const Dims &d, const Weights<T> &w, int i, int j,
                                             int k)
{
    // wrapped coordinates for offsets -1..+2
    int xs[4], ys[4], zs[4];
    for (int o = 0; o < 4; ++o) {
        xs[o] = wrap(i + o - 1, d.nx);
        ys[o] = wrap(j + o - 1, d.ny);
        zs[o] = wrap(k + o - 1, d.nz);
    }
    const int64_t nxy = (int64_t)d.nx * d.ny;
    auto at = [&](const T *X, int ox, int oy, int oz) -> T {
        return X[(int64_t)zs[oz + 1] * nxy + (int64_t)ys[oy + 1] * d.nx + xs[ox + 1]];
    };
    // forward difference along axis a of X, at offset (ox, oy, oz)
    auto g = [&](const T *X, int a, int ox, int oy, int oz) -> T {
        return at(X, ox + (a == 0), oy + (a == 1), oz + (a == 2)) - at(X, ox, oy, oz);
    };
    // star S_a of component X at p; transverse axes in coefficient order
    auto S = [&](const T *X, int a) -> T {
        int e[3] = {0, 0, 0}, u[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        e[a] = 1;
        const int t1 = (a == 0) ? 1 : 0, t2 = (a == 2) ? 1 : 2;
        u[t1] = 1;
        v[t2] = 1;
        return star(w.wc[a], w.wd[a], w.wb[a][0], w.wb[a][1], g(X, a, 0, 0, 0),
                    g(X, a, e[0], e[1], e[2]), g(X, a, -e[0], -e[1], -e[2]),
                    g(X, a, u[0], u[1], u[2]), g(X, a, -u[0], -u[1], -u[2]),
                    g(X, a, v[0], v[1], v[2]), g(X, a, -v[0], -v[1], -v[2]));
    };
    const T *Ex = f.c[0], *Ey = f.c[1], *Ez = f.c[2];
    const T bx = S(Ey, 2) - S(Ez, 1);
    const T by = S(Ez, 0) - S(Ex, 2);
    const T bz = S(Ex, 1) - S(Ey, 0);
    const int64_t p = (int64_t)k * nxy + (int64_t)j * d.nx + i;
    f.c[3][p] = f.c[3][p] + bx;
    f.c[4][p] = f.c[4][p] + by;
    f.c[5][p] = f.c[5][p] + bz;
}

// x from the grid's x dimension; y and z loop over the grid (whose y and z
// dimensions are capped at 65535 blocks)
template <typename T>
__global__ __launch_bounds__(256) void faraday_kernel(Fields<T> f, Dims d, Weights<T> w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.nx) return;
    for (int k = blockIdx.z; k < d.nz; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < d.ny; j += gridDim.y * blockDim.y)
            faraday_cell(f, d, w, i, j, k);
}

// ---------------------------------------------------------------------------
// unfused Ampere: E += dt (D x B) in place
// ---------------------------------------------------------------------------
// With a current source (jx non-null; App. A eq. update4-6 in c = mu_0 = 1
// units): E += dt (D x B) - dt J, wj = dt rounded to T.
template <typename T>
__device__ __forceinline__ void ampere_cell(const Fields<T> &f, const Dims &d, const Weights<T> &w,
                                            const T *__restrict__ jx, const T *__restrict__ jy,
                                            const T *__restrict__ jz, T wj, int i, int j, int k)
{
    const int64_t nxy = (int64_t)d.nx * d.ny;
    const int64_t p = (int64_t)k * nxy + (int64_t)j * d.nx + i;
    const int64_t pxm = (int64_t)k * nxy + (int64_t)j * d.nx + wrap(i - 1, d.nx);
    const int64_t pym = (int64_t)k * nxy + (int64_t)wrap(j - 1, d.ny) * d.nx + i;
    const int64_t pzm = (int64_t)wrap(k - 1, d.nz) * nxy + (int64_t)j * d.nx + i;
    const T *Bx = f.c[3], *By = f.c[4], *Bz = f.c[5];
    const T bx = Bx[p], by = By[p], bz = Bz[p];
    if (jx) {
        f.c[0][p] = f.c[0][p] + ((w.wa[1] * (bz - Bz[pym]) - w.wa[2] * (by - By[pzm])) - wj * jx[p]);
        f.c[1][p] = f.c[1][p] + ((w.wa[2] * (bx - Bx[pzm]) - w.wa[0] * (bz - Bz[pxm])) - wj * jy[p]);
        f.c[2][p] = f.c[2][p] + ((w.wa[0] * (by - By[pxm]) - w.wa[1] * (bx - Bx[pym])) - wj * jz[p]);
        return;
    }
    f.c[0][p] = ampere_eval(f.c[0][p], w.wa[1], bz, Bz[pym], w.wa[2], by, By[pzm]);
    f.c[1][p] = ampere_eval(f.c[1][p], w.wa[2], bx, Bx[pzm], w.wa[0], bz, Bz[pxm]);
    f.c[2][p] = ampere_eval(f.c[2][p], w.wa[0], by, By[pxm], w.wa[1], bx, Bx[pym]);
}

template <typename T>
__global__ __launch_bounds__(256) void ampere_kernel(Fields<T> f, Dims d, Weights<T> w, const T *__restrict__ jx,
                                                     const T *__restrict__ jy, const T *__restrict__ jz, T wj)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.nx) return;
    for (int k = blockIdx.z; k < d.nz; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < d.ny; j += gridDim.y * blockDim.y)
            ampere_cell(f, d, w, jx, jy, jz, wj, i, j, k);
}

// ---------------------------------------------------------------------------
// per-position pieces of a step, shared by the one-step and two-step z-marches
// (the same expression trees, so both round every cell's update the same way)
// ---------------------------------------------------------------------------
// The six forward differences g of plane k+1 at a position: z-differences
// from the lane's own E(k+1) (e1) and E(k+2) (e2), x- and y-differences from
// the staged plane E(k+1) (Ex1, Ey1, Ez1: LDS, row pitch PX, own index lg).
template <int PX, typename T>
__device__ __forceinline__ void form_g(T gn[6], const T e1[3], const T e2[3], const T *Ex1, const T *Ey1,
                                       const T *Ez1, int lg)
{
    gn[0] = e2[1] - e1[1];          // g_z[Ey] -> Bx (+S_z)
    gn[1] = Ez1[lg + PX] - e1[2];   // g_y[Ez] -> Bx (-S_y)
    gn[2] = Ez1[lg + 1] - e1[2];    // g_x[Ez] -> By (+S_x)
    gn[3] = e2[0] - e1[0];          // g_z[Ex] -> By (-S_z)
    gn[4] = Ex1[lg + PX] - e1[0];   // g_y[Ex] -> Bz (+S_y)
    gn[5] = Ey1[lg + 1] - e1[1];    // g_x[Ey] -> Bz (-S_x)
}

// Faraday update of a position: bn = bo + (star differences of g(k)); the
// x/y neighbours of g(k) come from G (six LDS planes, row pitch PX, own index
// l), its centre gc and z-neighbours gm = g(k-1), gn = g(k+1) from registers.
template <int PX, int P, typename T>
__device__ __forceinline__ void faraday_stars(T bn[3], const T bo[3], const T gm[6], const T gc[6],
                                              const T gn[6], const T (*G)[P], int l, const Weights<T> &w)
{
    // star argument order: centre, along-axis pair, t1 pair, t2 pair
    const T sz0 = star(w.wc[2], w.wd[2], w.wb[2][0], w.wb[2][1], gc[0], gn[0], gm[0], G[0][l + 1], G[0][l - 1],
                       G[0][l + PX], G[0][l - PX]);
    const T sy1 = star(w.wc[1], w.wd[1], w.wb[1][0], w.wb[1][1], gc[1], G[1][l + PX], G[1][l - PX], G[1][l + 1],
                       G[1][l - 1], gn[1], gm[1]);
    const T sx2 = star(w.wc[0], w.wd[0], w.wb[0][0], w.wb[0][1], gc[2], G[2][l + 1], G[2][l - 1], G[2][l + PX],
                       G[2][l - PX], gn[2], gm[2]);
    const T sz3 = star(w.wc[2], w.wd[2], w.wb[2][0], w.wb[2][1], gc[3], gn[3], gm[3], G[3][l + 1], G[3][l - 1],
                       G[3][l + PX], G[3][l - PX]);
    const T sy4 = star(w.wc[1], w.wd[1], w.wb[1][0], w.wb[1][1], gc[4], G[4][l + PX], G[4][l - PX], G[4][l + 1],
                       G[4][l - 1], gn[4], gm[4]);
    const T sx5 = star(w.wc[0], w.wd[0], w.wb[0][0], w.wb[0][1], gc[5], G[5][l + 1], G[5][l - 1], G[5][l + PX],
                       G[5][l - PX], gn[5], gm[5]);
    bn[0] = bo[0] + (sz0 - sy1);
    bn[1] = bo[1] + (sx2 - sz3);
    bn[2] = bo[2] + (sy4 - sx5);
}

// Ampere update of a position: E^{n+1}(k-1) from E^n(k-1) (ea), B^{n+1/2}(k-1)
// (own value b1, x-1 / y-1 neighbours from Bp: three LDS planes, row pitch
// PX) and the x, y components of B^{n+1/2}(k-2) (b2).
template <int PX, int P, typename T>
__device__ __forceinline__ void ampere3(T en[3], const T ea[3], const T b1[3], const T b2[2], const T (*Bp)[P],
                                        int l, const Weights<T> &w)
{
    en[0] = ampere_eval(ea[0], w.wa[1], b1[2], Bp[2][l - PX], w.wa[2], b1[1], b2[1]);
    en[1] = ampere_eval(ea[1], w.wa[2], b1[0], b2[0], w.wa[0], b1[2], Bp[2][l - 1]);
    en[2] = ampere_eval(ea[2], w.wa[0], b1[1], Bp[1][l - 1], w.wa[1], b1[0], Bp[0][l - PX]);
}

// ---------------------------------------------------------------------------
// fused step, z-march (see the file header)
// ---------------------------------------------------------------------------
// Tiling of the fused step: a workgroup of NW row waves plus one halo wave
// owns a TX x TY tile (TX = 64 or 32 columns).  A row wave holds 64 / TX row
// groups (lane = slot * TX + x); the G = NW * 64 / TX row groups own R rows
// each, y = R*g - 2 .. R*g - 2 + R - 1, so TY = R*G - 4.  The halo wave owns
// the four halo columns x = -2, -1, TXe, TXe+1 over the same row groups.
template <int R_, int NW_, int TX_ = 64>
struct TileCfg {
    static constexpr int R = R_;
    static constexpr int NW = NW_;
    static constexpr int TX = TX_;
    static constexpr int SLOTS = 64 / TX_;
    static constexpr int G = NW_ * SLOTS;
    static constexpr int TY = R_ * G - 4;
    static constexpr int THREADS = 64 * (NW_ + 1);
    static_assert(TX_ == 64 || TX_ == 32, "tile width");
    static_assert(TY > 0, "tile height");
    static_assert(4 * G <= 64, "halo wave must cover 4 columns x G row groups");
};

// LDS of one workgroup of the fused step.  B^{n+1/2} is double-buffered so
// that the Ampere update can lag one plane behind and read the previous
// plane's B after the single barrier per plane.
template <typename T, int TX, int TY>
struct FusedSmem {
    static constexpr int PX = TX + 4;  // row pitch: x in [-2, TX + 2)
    static constexpr int PY = TY + 4;  // rows y in [-2, TY + 2)
    static constexpr int P = PX * PY;
    T Ebuf[2][3][P];  // E(k+1), E(k+2)
    T Gbuf[2][6][P];  // g(k), g(k+1)
    T Bbuf[2][3][P];  // B^{n+1/2}(k-1), B^{n+1/2}(k)
};

// One tile of the fused step: tile number `logical` of a box tiled as
// ntx x nty x (z-chunks), x fastest.  All threads of the workgroup call it.
// One workgroup barrier per plane: iteration k forms g(k+1), B^{n+1/2}(k) and
// E^{n+1}(k-1); everything it reads from LDS was written in iteration k-1.
// Values a position needs along z stay in that lane's registers.
template <typename T, typename C>
__device__ __forceinline__ void fused_tile(const Fields<T> &in, const Fields<T> &out, const Dims &d,
                                           const Weights<T> &w, int zchunk, int ntx, int nty,
                                           int logical, FusedSmem<T, C::TX, C::TY> &sm)
{
    constexpr int R = C::R, NW = C::NW, TX = C::TX, TY = C::TY, G = C::G;
    constexpr int PX = FusedSmem<T, TX, TY>::PX;
    constexpr int P = FusedSmem<T, TX, TY>::P;
    auto &Ebuf = sm.Ebuf;
    auto &Gbuf = sm.Gbuf;
    auto &Bbuf = sm.Bbuf;
    gptr<const T> src[6];
    gptr<T> dst[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        src[c] = (gptr<const T>)in.c[c];
        dst[c] = (gptr<T>)out.c[c];
    }
    const int tx = logical % ntx;
    const int rest = logical / ntx;
    const int ty = rest % nty;
    const int zc = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, k0 = zc * zchunk;
    const int TXe = min(TX, d.nx - x0), TYe = min(TY, d.ny - y0);
    const int KZe = min(zchunk, d.nz - k0);

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int rx = 0, ry0 = 0;
    bool lane_ok;
    if (wave < NW) {
        rx = lane % TX;
        ry0 = R * (wave * C::SLOTS + lane / TX) - 2;
        lane_ok = rx < TXe;
    } else {
        const int sel = lane / G;
        ry0 = R * (lane % G) - 2;
        rx = sel == 0 ? -2 : sel == 1 ? -1 : sel == 2 ? TXe : TXe + 1;
        lane_ok = sel < 4;
    }
    bool isE[R], isG[R], isB[R], isO[R];
    int li[R], col[R], colb[R];
    const uint32_t nxy = (uint32_t)d.nx * (uint32_t)d.ny;  // <= 2^28 (host check)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int ry = ry0 + r;
        const bool valid = lane_ok && ry < TYe + 2;
        isE[r] = valid;                                                  // loads E
        isG[r] = valid && rx < TXe + 1 && ry < TYe + 1;                  // forms g
        isB[r] = valid && rx >= -1 && rx < TXe && ry >= -1 && ry < TYe;  // B^{n+1/2}
        isO[r] = valid && rx >= 0 && rx < TXe && ry >= 0 && ry < TYe;    // outputs
        li[r] = valid ? (ry + 2) * PX + (rx + 2) : 0;
        // idle positions use column 0 so that every lane can load
        // unconditionally (in bounds, value unused)
        col[r] = valid ? wrap(y0 + ry, d.ny) * d.nx + wrap(x0 + rx, d.nx) : 0;
        // B^{n-1/2} is needed only where B^{n+1/2} is formed
        colb[r] = isB[r] ? col[r] : 0;
    }
    const int nz = d.nz;
    auto inc = [nz](int v) { return v + 1 == nz ? 0 : v + 1; };

    // per position: ea = E(k-1), e0 = E(k), e1 = E(k+1); g at k-1, k;
    // b1 = B^{n+1/2}(k-1), b2 = B^{n+1/2}(k-2) (x, y components).  The
    // prefetched E(k+2) and B^{n-1/2}(k) alternate between two register sets
    // (pe, pb): a load issued in one iteration is first waited for in the
    // next, instead of at the loop back-edge together with the stores.
    T ea[R][3], e0[R][3], e1[R][3], pe[2][R][3], pb[2][R][3], gm[R][6], gc[R][6], b1[R][3], b2[R][2];
    int w3 = wrap(k0, nz), w1 = wrap(k0 - 3, nz), wm = wrap(k0 - 4, nz);
    {
        const uint64_t qa = (uint64_t)(uint32_t)wrap(k0 - 2, nz) * nxy, qb = (uint64_t)(uint32_t)wrap(k0 - 1, nz) * nxy;
        const uint64_t qc = (uint64_t)(uint32_t)w1 * nxy;
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                e1[r][c] = ld_plane(src[c] + qa, col[r]);
                pe[0][r][c] = ld_plane(src[c] + qb, col[r]);
                pb[0][r][c] = ld_plane(src[3 + c] + qc, colb[r]);
            }
            if (isE[r]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Ebuf[0][c][li[r]] = e1[r][c];
            }
#pragma unroll
            for (int m = 0; m < 6; ++m) gm[r][m] = gc[r][m] = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) ea[r][c] = e0[r][c] = b1[r][c] = T(0);
            b2[r][0] = b2[r][1] = T(0);
        }
    }
    __syncthreads();

    const int klast = k0 + KZe - 1;
    // One plane iteration; Q = (k - k0 + 3) & 1 is the LDS buffer parity and
    // the prefetch set consumed (set Q^1 is refilled).
    auto plane = [&](auto parity, int k) {
        constexpr int Q = decltype(parity)::value;
        constexpr int eb = Q, gb = Q, bb = Q;
        T e2[R][3], bo[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                e2[r][c] = take(pe[Q][r][c]);
                bo[r][c] = take(pb[Q][r][c]);
            }
        // per-iteration copies of the lane offsets, opaque to the compiler, so
        // that it keeps the addresses in the form scalar plane base + 32-bit
        // lane offset instead of hoisting base + offset out of the loop (which
        // costs a 64-bit vector add per access)
        uint32_t oc[R], ob[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            oc[r] = col[r];
            ob[r] = colb[r];
            asm("" : "+v"(oc[r]), "+v"(ob[r]));
        }
        {
            const uint64_t p3 = (uint64_t)(uint32_t)w3 * nxy;
            w1 = inc(w1);
            const uint64_t p1 = (uint64_t)(uint32_t)w1 * nxy;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pe[Q ^ 1][r][c] = ld_plane(src[c] + p3, oc[r]);
                    pb[Q ^ 1][r][c] = ld_plane(src[3 + c] + p1, ob[r]);
                }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (isE[r]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Ebuf[eb ^ 1][c][li[r]] = e2[r][c];
            }

        // g(k+1) (positions outside the g region read the neighbours of slot
        // 0: in bounds, value unused)
        T gn[R][6];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int lg = isG[r] ? li[r] : 0;
            form_g<PX>(gn[r], e1[r], e2[r], Ebuf[eb][0], Ebuf[eb][1], Ebuf[eb][2], lg);
            if (isG[r]) {
#pragma unroll
                for (int m = 0; m < 6; ++m) Gbuf[gb ^ 1][m][li[r]] = gn[r][m];
            }
        }

        // B^{n+1/2}(k): stars of g(k); z-neighbours from registers
        T bn[R][3];
        const bool doStar = k >= k0 - 1 && k <= klast;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bn[r][0] = bn[r][1] = bn[r][2] = T(0);
            if (isB[r] && doStar) {
                const int l = li[r];
                faraday_stars<PX, P>(bn[r], bo[r], gm[r], gc[r], gn[r], Gbuf[gb], l, w);
#pragma unroll
                for (int c = 0; c < 3; ++c) Bbuf[bb][c][l] = bn[r][c];
            }
        }

        // outputs of plane k-1: E^{n+1}(k-1) from B^{n+1/2}(k-1) (LDS and
        // registers, formed last iteration) and B^{n+1/2}(k-1) itself
        if (k - 1 >= k0 && k - 1 <= klast) {
            const T(*Bp)[P] = Bbuf[bb ^ 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!isO[r]) continue;
                T en[3];
                ampere3<PX, P>(en, ea[r], b1[r], b2[r], Bp, li[r], w);
                const uint64_t pm = (uint64_t)(uint32_t)wm * nxy;
                st_plane(dst[0] + pm, oc[r], en[0]);
                st_plane(dst[1] + pm, oc[r], en[1]);
                st_plane(dst[2] + pm, oc[r], en[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) st_plane(dst[3 + c] + pm, oc[r], b1[r][c]);
            }
        }

        __syncthreads();

#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ea[r][c] = e0[r][c];
                e0[r][c] = e1[r][c];
                e1[r][c] = e2[r][c];
            }
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                gm[r][m] = gc[r][m];
                gc[r][m] = gn[r][m];
            }
            b2[r][0] = b1[r][0];
            b2[r][1] = b1[r][1];
#pragma unroll
            for (int c = 0; c < 3; ++c) b1[r][c] = bn[r][c];
        }
        w3 = inc(w3);
        wm = inc(wm);
    };
    // KZe + 4 iterations (k = k0 - 3 .. klast + 1), two per loop trip; an odd
    // count runs one more iteration (k = klast + 2) whose results are unused,
    // so that the loop has a single exit and the prefetch register sets need
    // no copies at the back-edge
    for (int k = k0 - 3; k <= klast + 1; k += 2) {
        plane(std::integral_constant<int, 0>{}, k);
        plane(std::integral_constant<int, 1>{}, k + 1);
    }
}


// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give each
// XCD a contiguous range of tile numbers so that halo re-reads stay in its L2.
__device__ __forceinline__ int xcd_order(int bid, int nb)
{
    const int q = nb >> 3, r = nb & 7, xcd = bid & 7;
    return xcd * q + min(xcd, r) + (bid >> 3);
}

template <typename T, typename C>
__global__ __launch_bounds__(C::THREADS) void fused_step_kernel(Fields<T> in, Fields<T> out, Dims d,
                                                                Weights<T> w, int zchunk, int ntx, int nty)
{
    __shared__ FusedSmem<T, C::TX, C::TY> sm;
    fused_tile<T, C>(in, out, d, w, zchunk, ntx, nty, xcd_order(blockIdx.x, gridDim.x), sm);
}

// ---------------------------------------------------------------------------
// plane step: boxes one plane deep (nz = 1, the 2D variant of Sec. 2, k_z = 0)
// ---------------------------------------------------------------------------
// A box one plane deep is periodic in z with period one: every z-neighbour of
// a value is the value itself.  The z-march runs four plane iterations (three
// of warm-up) per output plane there; this kernel loads the plane once and
// forms g, B^{n+1/2} and E^{n+1} with the z-march's per-position functions,
// passing each position's own values as its z-neighbours (E(k+1) = E(k),
// g(k-1) = g(k+1) = g(k), B^{n+1/2}(k-2) = B^{n+1/2}(k-1)), so that its
// results are bitwise those of the z-march.  A TX x TY tile spans the
// positions [-2, TX+2) x [-2, TY+2) in row order, R per thread.
template <int TX_, int TY_, int THREADS_>
struct PlaneCfg {
    static constexpr int TX = TX_, TY = TY_, THREADS = THREADS_;
    static constexpr int PX = TX_ + 4, PY = TY_ + 4, P = PX * PY;
    static constexpr int R = (P + THREADS_ - 1) / THREADS_;
};

template <typename T, int P>
struct PlaneSmem {
    T EB[3][P];  // E^n, then B^{n+1/2}
    T G[6][P];   // g of E^n
};

// Tile `logical` (x fastest) of a plane box with ntx tiles per row.
template <typename T, typename C>
__device__ __forceinline__ void plane_tile(const Fields<T> &in, const Fields<T> &out, const Dims &d,
                                           const Weights<T> &w, int ntx, int logical, PlaneSmem<T, C::P> &sm)
{
    constexpr int R = C::R, TX = C::TX, TY = C::TY, PX = C::PX, P = C::P;
    const int x0 = (logical % ntx) * TX, y0 = (logical / ntx) * TY;
    const int TXe = min(TX, d.nx - x0), TYe = min(TY, d.ny - y0);
    gptr<const T> src[6];
    gptr<T> dst[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        src[c] = (gptr<const T>)in.c[c];
        dst[c] = (gptr<T>)out.c[c];
    }
    T e[R][3], bo[R][3], g[R][6], bn[R][3];
    int li[R];
    uint32_t col[R];
    bool isG[R], isB[R], isO[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int sl = (int)threadIdx.x + r * C::THREADS;
        const int rx = sl % PX - 2, ry = sl / PX - 2;
        const bool valid = sl < P && rx < TXe + 2 && ry < TYe + 2;
        isG[r] = valid && rx < TXe + 1 && ry < TYe + 1;                  // forms g
        isB[r] = valid && rx >= -1 && rx < TXe && ry >= -1 && ry < TYe;  // B^{n+1/2}
        isO[r] = valid && rx >= 0 && rx < TXe && ry >= 0 && ry < TYe;    // outputs
        li[r] = valid ? sl : 0;
        // idle positions load column 0 (in bounds, value unused)
        col[r] = valid ? (uint32_t)(wrap(y0 + ry, d.ny) * d.nx + wrap(x0 + rx, d.nx)) : 0u;
        const uint32_t colb = isB[r] ? col[r] : 0u;  // B^{n-1/2} only where B^{n+1/2} is formed
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            e[r][c] = ld_plane(src[c], col[r]);
            bo[r][c] = ld_plane(src[3 + c], colb);
        }
        if (valid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.EB[c][sl] = e[r][c];
        }
    }
    __syncthreads();
    // g of E^n (positions outside the g region read the neighbours of slot 0)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        form_g<PX>(g[r], e[r], e[r], sm.EB[0], sm.EB[1], sm.EB[2], isG[r] ? li[r] : 0);
        if (isG[r]) {
#pragma unroll
            for (int m = 0; m < 6; ++m) sm.G[m][li[r]] = g[r][m];
        }
    }
    __syncthreads();  // E^n is no longer read from LDS
    // B^{n+1/2}: stars of g with g itself as both z-neighbours
#pragma unroll
    for (int r = 0; r < R; ++r) {
        bn[r][0] = bn[r][1] = bn[r][2] = T(0);
        if (isB[r]) {
            faraday_stars<PX, P>(bn[r], bo[r], g[r], g[r], g[r], sm.G, li[r], w);
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.EB[c][li[r]] = bn[r][c];
        }
    }
    __syncthreads();
    // E^{n+1} from B^{n+1/2} (own value also as its z-neighbour); both stored
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!isO[r]) continue;
        const T b2[2] = {bn[r][0], bn[r][1]};
        T en[3];
        ampere3<PX, P>(en, e[r], bn[r], b2, sm.EB, li[r], w);
#pragma unroll
        for (int c = 0; c < 3; ++c) st_plane(dst[c], col[r], en[c]);
#pragma unroll
        for (int c = 0; c < 3; ++c) st_plane(dst[3 + c], col[r], bn[r][c]);
    }
}

template <typename T, typename C>
__global__ __launch_bounds__(C::THREADS) void plane_step_kernel(Fields<T> in, Fields<T> out, Dims d, Weights<T> w,
                                                                int ntx)
{
    __shared__ PlaneSmem<T, C::P> sm;
    plane_tile<T, C>(in, out, d, w, ntx, xcd_order(blockIdx.x, gridDim.x), sm);
}

// Batched plane step (every box of the batch one plane deep): work item i is
// plane tile items[i].y of box items[i].x (box -1: no work), as in
// batched_step_kernel; parity 0: f -> s, 1: s -> f.
template <typename T, typename C>
__global__ __launch_bounds__(C::THREADS) void batched_plane_kernel(const BoxDesc<T> *__restrict__ boxes,
                                                                   const int2 *__restrict__ items, int nitems,
                                                                   int parity)
{
    __shared__ PlaneSmem<T, C::P> sm;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        if (it.x < 0) continue;
        const BoxDesc<T> &b = boxes[it.x];
        plane_tile<T, C>(parity ? b.s : b.f, parity ? b.f : b.s, b.d, b.w, b.ntx, it.y, sm);
        __syncthreads();  // LDS is reused by the next item
    }
}

// Batched step: every box of a batch advances one step.  Work item i is tile
// items[i].y of box items[i].x (box -1: no work); workgroup w takes items w,
// w + gridDim.x, ...  The host orders the list for the XCD each slot lands
// on.  parity 0: f -> s, 1: s -> f.
template <typename T, typename C>
__global__ __launch_bounds__(C::THREADS) void batched_step_kernel(const BoxDesc<T> *__restrict__ boxes,
                                                                  const int2 *__restrict__ items,
                                                                  int nitems, int parity)
{
    __shared__ FusedSmem<T, C::TX, C::TY> sm;
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const int2 it = items[i];
        if (it.x < 0) continue;
        const BoxDesc<T> &b = boxes[it.x];
        const Fields<T> &in = parity ? b.s : b.f;
        const Fields<T> &out = parity ? b.f : b.s;
        fused_tile<T, C>(in, out, b.d, b.w, b.zchunk, b.ntx, b.nty, it.y, sm);
        __syncthreads();  // LDS is reused by the next item
    }
}

// ---------------------------------------------------------------------------
// two steps per pass: the fused z-march applied twice in one sweep
// ---------------------------------------------------------------------------
// (E^n, B^{n-1/2}) -> (E^{n+2}, B^{n+3/2}) with one read and one write of the
// state per two steps (24 B FP32 per cell-update, half of the one-step
// kernel's 48 B).  Stage 1 is the one-step march (iteration k forms g1(k+1),
// B^{n+1/2}(k) and E^{n+1}(k-1)); stage 2 runs the same march on stage 1's
// results three planes behind it (its iteration j = k - 3 forms g2(j+1) from
// the E^{n+1}(k-1) stage 1 has just produced, B^{n+3/2}(j) from the
// B^{n+1/2}(j) stage 1 produced three iterations earlier, and E^{n+2}(j-1)),
// so stage 2 never waits for anything but registers and LDS.
//
// A workgroup owns a TX x TY output tile.  Two chained steps reach four cells
// into the neighbouring tiles (each step two: the extended difference one cell
// below and two above, Ampere one more below), so the workgroup covers the
// (TX + 8) x (TY + 8) positions x, y in [-4, T + 4), one per lane, waves
// aligned with memory rows (blk2_position; LDS index (y + 4) PX + x + 4),
// and evaluates each stage redundantly on the part of the halo the next stage
// needs (regions below).  Every position computes the same per-cell
// expressions as the one-step kernel, so the result is bitwise that of two
// one-step launches.  LDS holds one plane of each staged quantity per stage
// (E, the six g, B).  A plane iteration has two barriers: stage 1 reads its
// planes while stage 2's planes of the previous iteration are written, and
// after the first barrier stage 2 reads while stage 1's new planes are
// written, so every LDS write overlaps the other stage's arithmetic.
template <int TX_, int TY_, int R_, int NW_>
struct Blk2Cfg {
    static constexpr int TX = TX_, TY = TY_, R = R_, NW = NW_;
    static constexpr int PX = TX + 8, PY = TY + 8, P = PX * PY;
    static constexpr int THREADS = 64 * NW;
    static_assert(R * THREADS == P, "one slot per position (every slot writes its own LDS index)");
    static_assert(THREADS <= 1024, "workgroup size");
};

template <typename T, int P>
struct Blk2Smem {
    T E0[3][P];  // stage 1: E^n(k+1)
    T G1[6][P];  // stage 1: g(k) of E^n
    T B1[3][P];  // stage 1: B^{n+1/2}(k-1)
    T E1[3][P];  // stage 2: E^{n+1}(j+1)
    T G2[6][P];  // stage 2: g(j) of E^{n+1}
    T B2[3][P];  // stage 2: B^{n+3/2}(j-1)
};

// Position of slot sl of a two-step tile.  Waves are aligned with memory
// rows.  32-column tiles: the first TX*TY slots are the output cells, two
// 32-column rows per wave (every output row segment is one 128-byte line,
// stored by one instruction); then the 8 halo columns x in [-4, 0) and
// [TX, TX+4) over all TY + 8 rows; then the 8 halo rows y in [-4, 0) and
// [TY, TY+4) over the TX inner columns.  Each part is a whole number of
// waves.  24-column tiles (FP64): the 32 positions of a row, halo included,
// are one half wave, in row order.
template <typename C>
__device__ __forceinline__ void blk2_position(int sl, int &rx, int &ry)
{
    constexpr int TX = C::TX, TY = C::TY, NI = TX * TY, NC = 8 * (TY + 8);
    if constexpr (C::PX == 32) {
        rx = sl % 32 - 4;
        ry = sl / 32 - 4;
        return;
    }
    static_assert(C::PX == 32 || (TX == 32 && NI % 64 == 0 && NC % 64 == 0 && (8 * TX) % 64 == 0),
                  "wave-aligned parts");
    if (sl < NI) {
        rx = sl % TX;
        ry = sl / TX;
    } else if (sl < NI + NC) {
        const int t = sl - NI, c = t % 8;
        rx = c < 4 ? c - 4 : TX + c - 4;
        ry = t / 8 - 4;
    } else {
        const int t = sl - NI - NC, row = t / TX;
        rx = t % TX;
        ry = row < 4 ? row - 4 : TY + row - 4;
    }
}

template <typename T, typename C>
__device__ __forceinline__ void blocked2_tile(const Fields<T> &in, const Fields<T> &out, const Dims &d,
                                              const Weights<T> &w, int zchunk, int ntx, int nty, int logical,
                                              Blk2Smem<T, C::P> &sm)
{
    constexpr int R = C::R, PX = C::PX, P = C::P;
    gptr<const T> src[6];
    gptr<T> dst[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        src[c] = (gptr<const T>)in.c[c];
        dst[c] = (gptr<T>)out.c[c];
    }
    const int tx = logical % ntx;
    const int rest = logical / ntx;
    const int ty = rest % nty;
    const int zc = rest / nty;
    const int x0 = tx * C::TX, y0 = ty * C::TY, k0 = zc * zchunk;
    const int TXe = min(C::TX, d.nx - x0), TYe = min(C::TY, d.ny - y0);
    const int KZe = min(zchunk, d.nz - k0);

    // Regions (tile coordinates; TXe, TYe the tile's extent inside the box):
    //   L1 E^n loaded, staged            [-4, T+4)   G1 g of E^n staged  [-4, T+3)
    //   S1 B^{n+1/2} formed, staged      [-3, T+2)   A1 E^{n+1} formed   [-2, T+2)
    //   G2 g of E^{n+1} staged           [-2, T+1)   S2 B^{n+3/2}        [-1, T)
    //   O  E^{n+2} formed, both stored   [0, T)
    // Each stage reads only inside the region the previous one filled.
    bool inL1[R], inG1[R], inS1[R], inA1[R], inG2[R], inS2[R], inO[R];
    bool inner[R];
    int li[R], col[R], colb[R];
    const uint32_t nxy = (uint32_t)d.nx * (uint32_t)d.ny;  // <= 2^28 (host check)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int sl = (int)threadIdx.x + r * C::THREADS;
        int rx, ry;
        blk2_position<C>(sl, rx, ry);
        const bool v = rx < TXe + 4 && ry < TYe + 4;
        auto in_box = [&](int lo, int hx, int hy) { return v && rx >= lo && ry >= lo && rx < hx && ry < hy; };
        inL1[r] = v;
        inG1[r] = in_box(-4, TXe + 3, TYe + 3);
        inS1[r] = in_box(-3, TXe + 2, TYe + 2);
        inA1[r] = in_box(-2, TXe + 2, TYe + 2);
        inG2[r] = in_box(-2, TXe + 1, TYe + 1);
        inS2[r] = in_box(-1, TXe, TYe);
        inO[r] = in_box(0, TXe, TYe);
        // every slot is a position of the grid (static_assert in Blk2Cfg);
        // positions past the tile's extent (ragged tiles) keep their own LDS
        // slots, which no position of the tile reads
        li[r] = (ry + 4) * PX + (rx + 4);
        // Phase A evaluates every stage at every position without branches
        // (results outside a stage's region are never read), so the
        // neighbour indices of the reads are clamped into the planes: g reads
        // +1 and +PX (slot 0 outside the g regions), the stars and the Ampere
        // update +-1 and +-PX (an interior slot on the outermost ring).
        inner[r] = rx >= -3 && ry >= -3 && rx <= C::TX + 2 && ry <= C::TY + 2;
        // idle positions load column 0 (in bounds, value unused)
        col[r] = v ? wrap(y0 + ry, d.ny) * d.nx + wrap(x0 + rx, d.nx) : 0;
        // B^{n-1/2} is needed only where B^{n+1/2} is formed
        colb[r] = inS1[r] ? col[r] : 0;
    }
    const int nz = d.nz;
    auto inc = [nz](int v) { return v + 1 == nz ? 0 : v + 1; };

    // Values a position keeps along z live in rings of four register slots:
    // the value of plane p sits in slot (p - kbeg) & 3, kbeg = k0 - 5 being
    // the first iteration, and no value is needed more than three planes
    // after the next one arrives.  The loop is unrolled four times, so every
    // slot index is a constant and slots keep their roles at the back-edge
    // (no register moves to rotate queues).
    //   stage 1: E^n at k-1 .. k+2 (E), g1 at k-1 .. k+1 (G), B^{n+1/2} at
    //            k-3 .. k (B); prefetched E^n(k+2) and B^{n-1/2}(k) in two
    //            alternating sets (pe, pb)
    //   stage 2 (plane j = k - 3): E^{n+1} at j-1 .. j+2 (F), g2 at
    //            j-1 .. j+1 (H), B^{n+3/2} at j-2 .. j (Cq)
    T E[4][R][3], G[4][R][6], B[4][R][3], F[4][R][3], H[4][R][6], Cq[4][R][3], pe[2][R][3], pb[2][R][3];
    // first iteration k = k0 - 5: E^n(k0-4) staged and in slot 1, E^n(k0-3)
    // and B^{n-1/2}(k0-5) in the first prefetch set
    int wE = wrap(k0 - 2, nz), wB = wrap(k0 - 5, nz), wm = wrap(k0 - 9, nz);
    {
        const uint64_t qa = (uint64_t)(uint32_t)wrap(k0 - 4, nz) * nxy;
        const uint64_t qb = (uint64_t)(uint32_t)wrap(k0 - 3, nz) * nxy;
        const uint64_t qc = (uint64_t)(uint32_t)wB * nxy;
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int c = 0; c < 3; ++c) E[q][r][c] = B[q][r][c] = F[q][r][c] = Cq[q][r][c] = T(0);
#pragma unroll
                for (int m = 0; m < 6; ++m) G[q][r][m] = H[q][r][m] = T(0);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                E[1][r][c] = ld_plane(src[c] + qa, col[r]);
                pe[0][r][c] = ld_plane(src[c] + qb, col[r]);
                pb[0][r][c] = ld_plane(src[3 + c] + qc, colb[r]);
            }
            if (inL1[r]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) sm.E0[c][li[r]] = E[1][r][c];
            }
        }
    }
    __syncthreads();

    const int klast = k0 + KZe - 1;
    // One plane iteration, i = k - kbeg; I = i & 3 (a constant) picks the ring
    // slots, I & 1 the prefetch set consumed (the other one is refilled).
    auto plane = [&](auto slot, int k) {
        constexpr int I = decltype(slot)::value;
        constexpr int Q = I & 1;
        constexpr int m1 = (I + 3) & 3, s0 = I, p1 = (I + 1) & 3, p2 = (I + 2) & 3;
        // stage 1: E^n(k+2) and B^{n-1/2}(k) arrive
        T bo[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                E[p2][r][c] = pe[Q][r][c];
                bo[r][c] = pb[Q][r][c];
            }
        // lane offsets opaque to the compiler (scalar plane base + 32-bit
        // lane offset per access, as in the one-step kernel)
        uint32_t oc[R], ob[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            oc[r] = col[r];
            ob[r] = colb[r];
            asm("" : "+v"(oc[r]), "+v"(ob[r]));
        }
        {
            const uint64_t pE = (uint64_t)(uint32_t)wE * nxy;
            wB = inc(wB);
            const uint64_t pB = (uint64_t)(uint32_t)wB * nxy;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pe[Q ^ 1][r][c] = ld_plane(src[c] + pE, oc[r]);
                    pb[Q ^ 1][r][c] = ld_plane(src[3 + c] + pB, ob[r]);
                }
        }

        // ---- phase 1: stage 2's planes of the previous iteration go to LDS;
        // stage 1 reads its planes.  Every position writes its own slot of
        // every plane (slots outside a stage's region hold values nothing
        // reads), so the writes need no branches. ----
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int l = li[r];
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.E1[c][l] = F[p2][r][c];  // E^{n+1}(j+1) = (k-2)
#pragma unroll
            for (int m = 0; m < 6; ++m) sm.G2[m][l] = H[p1][r][m];  // g2(j) = (k-3)
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.B2[c][l] = Cq[s0][r][c];  // B^{n+3/2}(j-1) = (k-4)
        }
        // stage 1: g1(k+1), B^{n+1/2}(k), E^{n+1}(k-1)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int ls = inner[r] ? li[r] : PX + 1;
            form_g<PX>(G[p1][r], E[p1][r], E[p2][r], sm.E0[0], sm.E0[1], sm.E0[2], inG1[r] ? li[r] : 0);
            B[s0][r][0] = B[s0][r][1] = B[s0][r][2] = T(0);
            if (inS1[r] && k >= k0 - 3)
                faraday_stars<PX, P>(B[s0][r], bo[r], G[m1][r], G[s0][r], G[p1][r], sm.G1, ls, w);
            ampere3<PX, P>(F[m1][r], E[m1][r], B[m1][r], B[p2][r], sm.B1, ls, w);
        }
        __syncthreads();

        // ---- phase 2: stage 1's planes go to LDS; stage 2 reads its planes ----
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int l = li[r];
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.E0[c][l] = E[p2][r][c];  // E^n(k+2)
#pragma unroll
            for (int m = 0; m < 6; ++m) sm.G1[m][l] = G[p1][r][m];  // g1(k+1)
#pragma unroll
            for (int c = 0; c < 3; ++c) sm.B1[c][l] = B[s0][r][c];  // B^{n+1/2}(k)
        }
        // stage 2, plane j = k - 3: g2(j+1) from E^{n+1}(j+1) (staged, and
        // slot p2) and E^{n+1}(j+2) (slot m1, just formed); B^{n+3/2}(j) from
        // B^{n+1/2}(j) (slot p1); E^{n+2}(j-1) from E^{n+1}(j-1) (slot s0)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int ls = inner[r] ? li[r] : PX + 1;
            form_g<PX>(H[p2][r], F[p2][r], F[m1][r], sm.E1[0], sm.E1[1], sm.E1[2], inG2[r] ? li[r] : 0);
            Cq[p1][r][0] = Cq[p1][r][1] = Cq[p1][r][2] = T(0);
            if (inS2[r] && k >= k0 + 2)
                faraday_stars<PX, P>(Cq[p1][r], B[p1][r], H[s0][r], H[p1][r], H[p2][r], sm.G2, ls, w);
        }
        // outputs of plane j-1 = k-4: E^{n+2}(j-1) and B^{n+3/2}(j-1)
        if (k >= k0 + 4 && k <= klast + 4) {
            const uint64_t pm = (uint64_t)(uint32_t)wm * nxy;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!inO[r]) continue;
                T ex[3];
                ampere3<PX, P>(ex, F[s0][r], Cq[s0][r], Cq[m1][r], sm.B2, li[r], w);
#pragma unroll
                for (int c = 0; c < 3; ++c) st_plane(dst[c] + pm, oc[r], ex[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) st_plane(dst[3 + c] + pm, oc[r], Cq[s0][r][c]);
            }
        }
        __syncthreads();
        wE = inc(wE);
        wm = inc(wm);
    };
    // KZe + 10 iterations (k = k0 - 5 .. klast + 4), four per loop trip;
    // up to three more whose results are unused
    for (int k = k0 - 5; k <= klast + 4; k += 4) {
        plane(std::integral_constant<int, 0>{}, k);
        plane(std::integral_constant<int, 1>{}, k + 1);
        plane(std::integral_constant<int, 2>{}, k + 2);
        plane(std::integral_constant<int, 3>{}, k + 3);
    }
}

template <typename T, typename C>
__global__ __launch_bounds__(C::THREADS) void blocked2_kernel(Fields<T> in, Fields<T> out, Dims d, Weights<T> w,
                                                              int zchunk, int ntx, int nty)
{
    __shared__ Blk2Smem<T, C::P> sm;
    blocked2_tile<T, C>(in, out, d, w, zchunk, ntx, nty, xcd_order(blockIdx.x, gridDim.x), sm);
}

// Batched two-step launch: every box of a batch advances two steps; work item
// i is tile items[i].y of box items[i].x (32-column tiles of the box's
// tiling); a persistent grid walks the list as in batched_step_kernel.
// parity 0: f -> s, 1: s -> f.
// ONE: one workgroup per slot (gridDim.x == nitems), no item loop.  Without
// a loop nothing stays live from one item to the next: the looping variant
// keeps its lane positions across the loop and, at the 128 VGPRs that 15
// waves per workgroup allow, spills some of them into the z-loop.
template <typename T, typename C, bool ONE>
__global__ __launch_bounds__(C::THREADS) void batched_blocked2_kernel(const BoxDesc<T> *__restrict__ boxes,
                                                                      const int2 *__restrict__ items, int nitems,
                                                                      int parity)
{
    __shared__ Blk2Smem<T, C::P> sm;
    if constexpr (ONE) {
        const int2 it = items[blockIdx.x];
        if (it.x < 0) return;
        const BoxDesc<T> &b = boxes[it.x];
        blocked2_tile<T, C>(parity ? b.s : b.f, parity ? b.f : b.s, b.d, b.w, b.zchunk, b.ntx, b.nty, it.y, sm);
    } else {
        for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
            const int2 it = items[i];
            if (it.x < 0) continue;
            const BoxDesc<T> &b = boxes[it.x];
            const Fields<T> &in = parity ? b.s : b.f;
            const Fields<T> &out = parity ? b.f : b.s;
            blocked2_tile<T, C>(in, out, b.d, b.w, b.zchunk, b.ntx, b.nty, it.y, sm);
            __syncthreads();  // LDS is reused by the next item
        }
    }
}

// Two-step tilings (FP32), one position per lane: 32x16 outputs on 40x24
// positions (15 waves), 32x8 on 40x16 (10 waves, for small boxes).  With two
// positions per lane (e.g. 32x24 on 40x32 in 10 waves) the two stages' register
// queues exceed the 168 VGPRs of three waves per SIMD and spill.
using Blk32x16 = Blk2Cfg<32, 16, 1, 15>;
using Blk32x8 = Blk2Cfg<32, 8, 1, 10>;
// FP64: 24x8 outputs on 32x16 positions (8 waves, 98 KB of LDS for the 24
// double planes; a 32-column FP64 tile's planes would exceed the LDS).
using Blk24x8 = Blk2Cfg<24, 8, 1, 8>;

template <typename T, typename F>
hipError_t with_blk2(int tile_x, int tile_y, F &&f)
{
    if constexpr (sizeof(T) == 4) {
        if (tile_x == 32 && tile_y == 16) return f(Blk32x16{});
        if (tile_x == 32 && tile_y == 8) return f(Blk32x8{});
    } else {
        if (tile_x == 24 && tile_y == 8) return f(Blk24x8{});
    }
    return hipErrorInvalidValue;
}

// 64-wide tiles of height 4 and 8 (one row per lane) and 16 (two rows per
// lane); 32-wide tiles (two row groups per wave) of the same heights, for
// boxes whose x extent is 32 modulo 64 or too small to fill the CUs.
using Tile4 = TileCfg<1, 8>;
using Tile8 = TileCfg<1, 12>;
using Tile16 = TileCfg<2, 10>;
using Tile32x4 = TileCfg<1, 4, 32>;
using Tile32x8 = TileCfg<1, 6, 32>;
using Tile32x16 = TileCfg<2, 5, 32>;

// Calls f(C{}) with the tile configuration of (tile_x, tile_y); the two-row
// tiles are FP32 only (FP64 would exceed the LDS of a CU or the registers).
template <typename T, typename F>
hipError_t with_tile(int tile_x, int tile_y, F &&f)
{
    if (tile_x == 64) {
        if (tile_y == 4) return f(Tile4{});
        if (tile_y == 8) return f(Tile8{});
        if constexpr (sizeof(T) == 4)
            if (tile_y == 16) return f(Tile16{});
    } else if (tile_x == 32) {
        if (tile_y == 4) return f(Tile32x4{});
        if (tile_y == 8) return f(Tile32x8{});
        if constexpr (sizeof(T) == 4)
            if (tile_y == 16) return f(Tile32x16{});
    }
    return hipErrorInvalidValue;
}

}  // namespace

// grid of the unfused kernels: x covers nx; y and z are capped at 65535
// blocks (the kernels loop over the rest)
static dim3 unfused_grid(const Dims &d)
{
    return dim3((d.nx + 63) / 64, (unsigned)std::min((d.ny + 3) / 4, 65535), (unsigned)std::min(d.nz, 65535));
}

template <typename T>
hipError_t launch_faraday(const Fields<T> &f, Dims d, const Weights<T> &w, hipStream_t s)
{
    dim3 blk(64, 4, 1), grd = unfused_grid(d);
    hipLaunchKernelGGL(faraday_kernel<T>, grd, blk, 0, s, f, d, w);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ampere(const Fields<T> &f, Dims d, const Weights<T> &w, hipStream_t s, const T *const *j,
                         T wj)
{
    dim3 blk(64, 4, 1), grd = unfused_grid(d);
    hipLaunchKernelGGL(ampere_kernel<T>, grd, blk, 0, s, f, d, w, j ? j[0] : nullptr, j ? j[1] : nullptr,
                       j ? j[2] : nullptr, wj);
    return hipGetLastError();
}

// Plane-kernel tilings: 64x16 outputs in FP32 (1360 positions, 3 per thread
// of 512, 49 KB of LDS), 64x8 in FP64 (816 positions, one per thread of
// 1024, 59 KB).  Measured at 4096^2 against 256 threads with 6 and 4
// positions each: 82.4 against 73.5 Gcell-updates/s (FP32), 44.3 against
// 37.7 (FP64); 128- and 32-column and 32-row tiles were slower.
template <typename T>
using PlaneTile = std::conditional_t<sizeof(T) == 4, PlaneCfg<64, 16, 512>, PlaneCfg<64, 8, 1024>>;

template <typename T>
hipError_t launch_plane(const Fields<T> &in, const Fields<T> &out, Dims d, const Weights<T> &w, hipStream_t s)
{
    using C = PlaneTile<T>;
    const int ntx = (d.nx + C::TX - 1) / C::TX, nty = (d.ny + C::TY - 1) / C::TY;
    const int64_t nb = (int64_t)ntx * nty;
    if (d.nz != 1 || nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((plane_step_kernel<T, C>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, in, out, d, w, ntx);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batched_plane(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int grid,
                                hipStream_t s)
{
    using C = PlaneTile<T>;
    if (nitems <= 0) return hipSuccess;
    if (grid <= 0 || grid > nitems) grid = nitems;
    hipLaunchKernelGGL((batched_plane_kernel<T, C>), dim3(grid), dim3(C::THREADS), 0, s, boxes, items, nitems,
                       parity);
    return hipGetLastError();
}

int plane_tile_x() { return 64; }
int plane_tile_y(int dtype) { return dtype == XFDTD_F32 ? PlaneTile<float>::TY : PlaneTile<double>::TY; }

// Boxes one plane deep run the plane kernel whatever the tiling asked for.
template <typename T>
hipError_t launch_fused(const Fields<T> &in, const Fields<T> &out, Dims d, const Weights<T> &w, int tile_x,
                        int tile_y, int zchunk, hipStream_t s)
{
    if (d.nz == 1) return launch_plane<T>(in, out, d, w, s);
    if (tile_x != 64 && tile_x != 32) return hipErrorInvalidValue;
    const int ntx = (d.nx + tile_x - 1) / tile_x;
    const int nty = (d.ny + tile_y - 1) / tile_y;
    const int nzc = (d.nz + zchunk - 1) / zchunk;
    const int64_t nb = (int64_t)ntx * nty * nzc;
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    return with_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        hipLaunchKernelGGL((fused_step_kernel<T, C>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, in, out, d, w,
                           zchunk, ntx, nty);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_blocked2(const Fields<T> &in, const Fields<T> &out, Dims d, const Weights<T> &w, int tile_x,
                           int tile_y, int zchunk, hipStream_t s)
{
    if (tile_x <= 0 || tile_y <= 0 || zchunk <= 0) return hipErrorInvalidValue;
    const int ntx = (d.nx + tile_x - 1) / tile_x;
    const int nty = (d.ny + tile_y - 1) / tile_y;
    const int nzc = (d.nz + zchunk - 1) / zchunk;
    const int64_t nb = (int64_t)ntx * nty * nzc;
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    return with_blk2<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        hipLaunchKernelGGL((blocked2_kernel<T, C>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, in, out, d, w,
                           zchunk, ntx, nty);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_batched2(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int tile_y,
                           int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (grid <= 0 || grid > nitems) grid = nitems;
    return with_blk2<T>(32, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        if (grid == nitems)
            hipLaunchKernelGGL((batched_blocked2_kernel<T, C, true>), dim3(grid), dim3(C::THREADS), 0, s, boxes,
                               items, nitems, parity);
        else
            hipLaunchKernelGGL((batched_blocked2_kernel<T, C, false>), dim3(grid), dim3(C::THREADS), 0, s, boxes,
                               items, nitems, parity);
        return hipGetLastError();
    });
}

template <typename T>
int blocked2_occupancy(int tile_x, int tile_y)
{
    int n = 0;
    const hipError_t e = with_blk2<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, blocked2_kernel<T, C>, C::THREADS, 0);
    });
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

template <typename T>
hipError_t launch_batched(const BoxDesc<T> *boxes, const int2 *items, int nitems, int parity, int tile_x,
                          int tile_y, int grid, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (grid <= 0 || grid > nitems) grid = nitems;
    return with_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        hipLaunchKernelGGL((batched_step_kernel<T, C>), dim3(grid), dim3(C::THREADS), 0, s, boxes, items, nitems,
                           parity);
        return hipGetLastError();
    });
}

template <typename T>
int fused_occupancy(int tile_x, int tile_y)
{
    int n = 0;
    const hipError_t e = with_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fused_step_kernel<T, C>, C::THREADS, 0);
    });
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

template hipError_t launch_batched2<float>(const BoxDesc<float> *, const int2 *, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_batched2<double>(const BoxDesc<double> *, const int2 *, int, int, int, int,
                                            hipStream_t);
template int blocked2_occupancy<float>(int, int);
template int blocked2_occupancy<double>(int, int);
template hipError_t launch_blocked2<float>(const Fields<float> &, const Fields<float> &, Dims,
                                           const Weights<float> &, int, int, int, hipStream_t);
template hipError_t launch_blocked2<double>(const Fields<double> &, const Fields<double> &, Dims,
                                            const Weights<double> &, int, int, int, hipStream_t);
template int fused_occupancy<float>(int, int);
template int fused_occupancy<double>(int, int);
template hipError_t launch_batched<float>(const BoxDesc<float> *, const int2 *, int, int, int, int, int,
                                          hipStream_t);
template hipError_t launch_batched<double>(const BoxDesc<double> *, const int2 *, int, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_batched_plane<float>(const BoxDesc<float> *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_batched_plane<double>(const BoxDesc<double> *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_faraday<float>(const Fields<float> &, Dims, const Weights<float> &, hipStream_t);
template hipError_t launch_faraday<double>(const Fields<double> &, Dims, const Weights<double> &, hipStream_t);
template hipError_t launch_ampere<float>(const Fields<float> &, Dims, const Weights<float> &, hipStream_t,
                                         const float *const *, float);
template hipError_t launch_ampere<double>(const Fields<double> &, Dims, const Weights<double> &, hipStream_t,
                                          const double *const *, double);
template hipError_t launch_fused<float>(const Fields<float> &, const Fields<float> &, Dims,
                                        const Weights<float> &, int, int, int, hipStream_t);
template hipError_t launch_fused<double>(const Fields<double> &, const Fields<double> &, Dims,
                                         const Weights<double> &, int, int, int, hipStream_t);

}  // namespace xfdtd
