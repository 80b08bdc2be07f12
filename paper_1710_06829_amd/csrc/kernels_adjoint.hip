// Adjoint (reverse-mode) step of the extended-stencil leapfrog, gfx950.
//
// Forward step (App. A, eq. update1-6): B' = B + K E,  E' = E + L B', with K
// the Faraday increment (the extended difference D* of Sec. 2 in the star
// form of xfdtd_internal.h) and L the Yee Ampere increment.  Given the
// gradients (lE', lB') of a loss with respect to (E', B'), one reverse step is
//   mu  = lB' + L^T lE'          L^T: forward differences of lE'
//   lE  = lE' + K^T mu           K^T: backward differences of the stars of mu
//   lB  = mu
// and the coefficient gradient of the step is <mu, (dK/dcoeff) E> with E the
// step's primal input.  With g = forward difference of a primal E component,
//   d/d alpha_a : sum_q g(q) mu(q)
//   d/d delta_a : sum_q g(q) (mu(q) + mu(q+e_a) + mu(q-e_a))
//   d/d beta_at : sum_q g(q) (mu(q+e_t) + mu(q-e_t))
// (times dt/d_a and the term's sign); the neighbour sums of mu are exactly
// those the stars use, so the gradient costs a few FMAs per cell.
//
// The kernel mirrors fused_step_kernel: a workgroup owns a TX x TY tile
// (TX = 64 or 32), marches a chunk of z-planes, stages lE', mu, the stars of
// mu and the primal E (whose x+1 / y+1 neighbours the gradient needs) in LDS
// for x/y neighbours and keeps z-neighbours in registers.  HBM traffic per
// cell: read lE', lB', E (9 values), write lE, lB (6 values).
// Per-workgroup gradient sums (unscaled, FP64) go to `partials`.

#include <type_traits>

#include "xfdtd_internal.h"

namespace xfdtd {

namespace {

__device__ __forceinline__ int wrapa(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

// Global-address-space pointers: the batched kernel reads its pointers from a
// descriptor in memory, where the compiler would otherwise emit flat accesses
// (which also hold up every LDS wait until outstanding loads return).
template <typename T>
using gptr_a = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ void nt_store_a(gptr_a<T> p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Plane accesses with a uniform base and a 32-bit lane offset (planes are
// limited to 2^32 bytes on the host): scalar base + vector offset addressing.
template <typename T>
__device__ __forceinline__ T ld_plane_a(gptr_a<const T> plane, uint32_t off)
{
    return *(gptr_a<const T>)((gptr_a<const char>)plane + off * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void st_plane_a(gptr_a<T> plane, uint32_t off, T v)
{
    __builtin_nontemporal_store(v, (gptr_a<T>)((gptr_a<char>)plane + off * (uint32_t)sizeof(T)));
}

// Tiling of the adjoint step: a TX x TY tile (TX = 64 or 32 columns) with
// one row per lane; a row wave holds 64 / TX rows (lane = slot * TX + x) of
// the TY + 4 rows y = -2 .. TY + 1, and one more wave the four halo columns
// x = -2, -1, TXe, TXe + 1 over those rows.
template <int TX_, int TY_>
struct AdjCfg {
    static constexpr int TX = TX_;
    static constexpr int TY = TY_;
    static constexpr int SLOTS = 64 / TX_;
    static constexpr int ROWW = (TY_ + 4) / SLOTS;  // row waves
    static constexpr int WAVES = ROWW + 1;
    static constexpr int THREADS = 64 * WAVES;
    static_assert(TX_ == 64 || TX_ == 32, "tile width");
    static_assert((TY_ + 4) % SLOTS == 0, "rows per row wave");
    static_assert(4 * (TY_ + 4) <= 64, "halo wave must cover 4 columns x TY + 4 rows");
    // waves per SIMD the compiler must leave room for: two 9-wave workgroups
    // of the 32x12 tile per CU need five
    static constexpr int MIN_WAVES = (TX_ == 32 && TY_ == 12) ? 5 : 1;
};

// gradient slots: the 12-coefficient order (alpha, beta_t1, beta_t2, delta per axis)
// One workgroup barrier per plane: iteration k forms mu(k+1) and the stars of
// plane k, and outputs plane k-1 (whose stars' neighbours were written in
// iteration k-1).  accumulate != 0 adds this step's sums to `partials`
// (each workgroup owns its 12 slots), else overwrites them.
template <typename T, typename C>
struct AdjSmem {
    static constexpr int PX = C::TX + 4;
    static constexpr int PY = C::TY + 4;
    static constexpr int P = PX * PY;
    T LEbuf[2][3][P];  // lE'(k+1), lE'(k+2)
    T Mbuf[2][3][P];   // mu(k), mu(k+1)
    T Sbuf[2][6][P];   // stars of mu at planes k-1, k
    T Ebuf[2][3][P];   // primal E(k), E(k+1)
    double red[12][C::WAVES];
};

// Shared storage of the one-plane pass: one plane each of lE', mu, the six
// stars and the primal E (15 planes, half of AdjSmem's double buffers) and the
// reduction slots, so that two workgroups share a CU.
template <typename T, typename C>
struct PlaneAdjStore {
    T planes[15][AdjSmem<T, C>::P];
    double red[12][C::WAVES];
};

// Per-position pieces of the reverse step, shared by the z-march and the
// one-plane pass (which passes a position's own values as its z-neighbours).
//
// mu = lB' + L^T lE' at a position: l1 = lE'(k+1) and l2 = lE'(k+2) of the
// position, Lx, Ly, Lz the LDS planes of lE'(k+1), lg its index there (slot 0
// outside the mu region: in bounds, value unused).
template <int PX, typename T>
__device__ __forceinline__ void adj_mu(T mu[3], const T bo[3], const T l1[3], const T l2[3], const T *Lx,
                                       const T *Ly, const T *Lz, int lg, const Weights<T> &w)
{
    const T fzy = l2[1] - l1[1], fzx = l2[0] - l1[0];
    const T fyz = Lz[lg + PX] - l1[2], fyx = Lx[lg + PX] - l1[0];
    const T fxz = Lz[lg + 1] - l1[2], fxy = Ly[lg + 1] - l1[1];
    mu[0] = bo[0] + (w.wa[1] * fyz - w.wa[2] * fzy);
    mu[1] = bo[1] + (w.wa[2] * fzx - w.wa[0] * fxz);
    mu[2] = bo[2] + (w.wa[0] * fxy - w.wa[1] * fyx);
}

// The six stars of mu at a position from its centre mc and its neighbour
// sums along x (px), y (py) and z (pz).
template <typename T>
__device__ __forceinline__ void adj_stars(T s[6], const T mc[3], const T px[3], const T py[3], const T pz[3],
                                          const Weights<T> &w)
{
    s[0] = w.wc[2] * mc[0] + w.wd[2] * pz[0] + w.wb[2][0] * px[0] + w.wb[2][1] * py[0];  // S_z mu_x
    s[1] = w.wc[1] * mc[0] + w.wd[1] * py[0] + w.wb[1][0] * px[0] + w.wb[1][1] * pz[0];  // S_y mu_x
    s[2] = w.wc[0] * mc[1] + w.wd[0] * px[1] + w.wb[0][0] * py[1] + w.wb[0][1] * pz[1];  // S_x mu_y
    s[3] = w.wc[2] * mc[1] + w.wd[2] * pz[1] + w.wb[2][0] * px[1] + w.wb[2][1] * py[1];  // S_z mu_y
    s[4] = w.wc[1] * mc[2] + w.wd[1] * py[2] + w.wb[1][0] * px[2] + w.wb[1][1] * pz[2];  // S_y mu_z
    s[5] = w.wc[0] * mc[2] + w.wd[0] * px[2] + w.wb[0][0] * py[2] + w.wb[0][1] * pz[2];  // S_x mu_z
}

// The coefficient-gradient sums of an output position at plane k: forward
// differences of the primal E(k) (n0; n1 = E(k+1); x+1 / y+1 neighbours from
// the LDS planes Ex, Ey, Ez at index li) against mu and its neighbour sums.
template <int PX, typename T>
__device__ __forceinline__ void adj_grad(double acc[12], const T n0[3], const T n1[3], const T *Ex, const T *Ey,
                                         const T *Ez, int li, const T mc[3], const T px[3], const T py[3],
                                         const T pz[3])
{
    const T gzEy = n1[1] - n0[1], gzEx = n1[0] - n0[0];
    const T gxEz = Ez[li + 1] - n0[2], gxEy = Ey[li + 1] - n0[1];
    const T gyEz = Ez[li + PX] - n0[2], gyEx = Ex[li + PX] - n0[0];
    // axis x (slots 0..3): +g_x[Ez] with mu_y, -g_x[Ey] with mu_z
    acc[0] += (double)(gxEz * mc[1] - gxEy * mc[2]);
    acc[1] += (double)(gxEz * py[1] - gxEy * py[2]);
    acc[2] += (double)(gxEz * pz[1] - gxEy * pz[2]);
    acc[3] += (double)(gxEz * px[1] - gxEy * px[2]);
    // axis y (slots 4..7): -g_y[Ez] with mu_x, +g_y[Ex] with mu_z
    acc[4] += (double)(gyEx * mc[2] - gyEz * mc[0]);
    acc[5] += (double)(gyEx * px[2] - gyEz * px[0]);
    acc[6] += (double)(gyEx * pz[2] - gyEz * pz[0]);
    acc[7] += (double)(gyEx * py[2] - gyEz * py[0]);
    // axis z (slots 8..11): +g_z[Ey] with mu_x, -g_z[Ex] with mu_y
    acc[8] += (double)(gzEy * mc[0] - gzEx * mc[1]);
    acc[9] += (double)(gzEy * px[0] - gzEx * px[1]);
    acc[10] += (double)(gzEy * py[0] - gzEx * py[1]);
    acc[11] += (double)(gzEy * pz[0] - gzEx * pz[1]);
}

// lE = lE' + backward differences of the stars at an output position of plane
// k-1: la = lE'(k-1); stars 3 and 0 at k-1 (s3a, s0a) and k-2 (s3b, s0b)
// from registers, stars 1, 2, 4, 5 of plane k-1 from the LDS planes Sp.
template <int PX, int P, typename T>
__device__ __forceinline__ void adj_out(T le[3], const T la[3], T s3a, T s3b, T s0a, T s0b, const T (*Sp)[P], int li)
{
    le[0] = la[0] + ((s3a - s3b) - (Sp[4][li] - Sp[4][li - PX]));
    le[1] = la[1] + ((Sp[5][li] - Sp[5][li - 1]) - (s0a - s0b));
    le[2] = la[2] + ((Sp[1][li] - Sp[1][li - PX]) - (Sp[2][li] - Sp[2][li - 1]));
}

// Sum of v over the wave's 64 lanes, complete in lane 63 (fixed order, in
// registers through DPP lane moves): inclusive scans within each row of 16
// lanes (shifts by 1, 2, 4, 8; lanes shifted in from outside the row add
// zero), then rows 1 and 3 add the last lane of rows 0 and 2 (row broadcast
// of lane 15), then rows 2 and 3 add lane 31 (row broadcast of lane 31).
__device__ __forceinline__ double wave_sum_lane63(double v)
{
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0.0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return v;
}

// The workgroup's 12 gradient sums (FP64, fixed order) into slot: written,
// or added to when accumulate != 0.
template <typename C>
__device__ __forceinline__ void adj_reduce(double acc[12], double (&red)[12][C::WAVES], double *__restrict__ slot,
                                           int accumulate, int wave, int lane)
{
    // delta_a: the centre term (that of alpha_a) plus the along-axis
    // neighbours, which are all the delta slots accumulate per plane
    acc[3] += acc[0];
    acc[7] += acc[4];
    acc[11] += acc[8];
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        const double v = wave_sum_lane63(acc[j]);
        if (lane == 63) red[j][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        double v = 0.0;
        for (int wv = 0; wv < C::WAVES; ++wv) v += red[threadIdx.x][wv];
        slot[threadIdx.x] = accumulate ? slot[threadIdx.x] + v : v;
    }
}

// One tile (number `logical`) of the adjoint step.  slot: this tile's 12
// gradient sums (written, or added to when accumulate != 0).  PLANE: the box
// is one plane deep (nz = 1, periodic in z with period one), and one pass
// with every z-neighbour the position's own value replaces the z-march's five
// iterations (three of warm-up and one past the plane): the same values, the
// same per-position functions, bitwise the z-march's adjoint fields; its
// gradient products are added to the lane's plane_acc, which the caller
// reduces (for several tiles at once: a tile of one plane is too little work
// to carry a workgroup reduction of its own).
template <typename T, typename C, bool PLANE = false>
__device__ __forceinline__ void adjoint_tile(const Fields<T> &lin, const Fields<T> &lout,
                                             const T *__restrict__ en_x, const T *__restrict__ en_y,
                                             const T *__restrict__ en_z, const Dims &d, const Weights<T> &w,
                                             int zchunk, int ntx, int nty, int logical, AdjSmem<T, C> &sm,
                                             double *__restrict__ slot, int accumulate, double *plane_acc = nullptr)
{
    constexpr int TX = C::TX, TY = C::TY;
    constexpr int PX = AdjSmem<T, C>::PX;
    constexpr int PY = AdjSmem<T, C>::PY;
    constexpr int P = AdjSmem<T, C>::P;
    auto &LEbuf = sm.LEbuf;
    auto &Mbuf = sm.Mbuf;
    auto &Sbuf = sm.Sbuf;
    auto &Ebuf = sm.Ebuf;
    auto &red = sm.red;
    const int tx = logical % ntx;
    const int rest = logical / ntx;
    const int ty = rest % nty;
    const int zc = rest / nty;
    const int x0 = tx * TX, y0 = ty * TY, k0 = zc * zchunk;
    const int TXe = min(TX, d.nx - x0), TYe = min(TY, d.ny - y0);
    const int KZe = min(zchunk, d.nz - k0);

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int rx = 0, ry = 0;
    bool valid;
    if (wave < C::ROWW) {
        ry = wave * C::SLOTS + lane / TX - 2;
        rx = lane % TX;
        valid = rx < TXe && ry < TYe + 2;
    } else {
        const int sel = lane / PY;
        ry = lane % PY - 2;
        rx = sel == 0 ? -2 : sel == 1 ? -1 : sel == 2 ? TXe : TXe + 1;
        valid = sel < 4 && ry < TYe + 2;
    }
    const bool isE = valid;                                                   // loads lE'
    const bool isG = valid && rx < TXe + 1 && ry < TYe + 1;                   // forms mu
    const bool isB = valid && rx >= -1 && rx < TXe && ry >= -1 && ry < TYe;   // stars
    const bool isO = valid && rx >= 0 && rx < TXe && ry >= 0 && ry < TYe;     // outputs

    const int li = valid ? (ry + 2) * PX + (rx + 2) : 0;
    const uint32_t nxy = (uint32_t)d.nx * (uint32_t)d.ny;  // <= 2^28 (host check)
    const int gyc = valid ? wrapa(y0 + ry, d.ny) : 0, gxc = valid ? wrapa(x0 + rx, d.nx) : 0;
    const int col = gyc * d.nx + gxc;
    // lB' is needed only where mu is formed, the primal E only at the output
    // cells and their x+1 / y+1 neighbours; other lanes load column 0
    const int colb = isG ? col : 0;
    const int coln = (valid && rx >= 0 && rx <= TXe && ry >= 0 && ry <= TYe) ? col : 0;
    const int nz = d.nz;
    auto inc = [nz](int v) { return v + 1 == nz ? 0 : v + 1; };
    gptr_a<const T> en[3] = {(gptr_a<const T>)en_x, (gptr_a<const T>)en_y, (gptr_a<const T>)en_z};
    gptr_a<const T> src[6];
    gptr_a<T> dst[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        src[c] = (gptr_a<const T>)lin.c[c];
        dst[c] = (gptr_a<T>)lout.c[c];
    }

    if constexpr (PLANE) {
        // sm is the kernel's PlaneAdjStore: planes 0-2 lE', 3-5 mu, 6-11 the
        // stars, 12-14 the primal E
        PlaneAdjStore<T, C> &st = reinterpret_cast<PlaneAdjStore<T, C> &>(sm);
        T(*PL)[P] = st.planes;
        T(*LEp)[P] = PL, (*Mp)[P] = PL + 3, (*Sq)[P] = PL + 6, (*Ep)[P] = PL + 12;
        double *acc = plane_acc;
        T le[3], bo[3], e0[3], mu[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            le[c] = src[c][col];
            bo[c] = src[3 + c][colb];
            e0[c] = en[c][coln];
        }
        if (isE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                LEp[c][li] = le[c];
                Ep[c][li] = e0[c];
            }
        }
        __syncthreads();
        adj_mu<PX>(mu, bo, le, le, LEp[0], LEp[1], LEp[2], isG ? li : 0, w);
        if (isG) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Mp[c][li] = mu[c];
        }
        __syncthreads();
        T s[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        if (isB) {
            T px[3], py[3], pz[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T *M = Mp[c];
                px[c] = M[li + 1] + M[li - 1];
                py[c] = M[li + PX] + M[li - PX];
                pz[c] = mu[c] + mu[c];
            }
            adj_stars(s, mu, px, py, pz, w);
#pragma unroll
            for (int m = 0; m < 6; ++m) Sq[m][li] = s[m];
            if (isO) adj_grad<PX>(acc, e0, e0, Ep[0], Ep[1], Ep[2], li, mu, px, py, pz);
        }
        __syncthreads();
        if (isO) {
            T lo[3];
            adj_out<PX, P>(lo, le, s[3], s[3], s[0], s[0], Sq, li);
            const uint32_t oc = col;
#pragma unroll
            for (int c = 0; c < 3; ++c) st_plane_a(dst[c], oc, lo[c]);
#pragma unroll
            for (int c = 0; c < 3; ++c) st_plane_a(dst[3 + c], oc, mu[c]);
        }
        return;
    }

    // Values a lane keeps along z live in rings of four register slots: the
    // value of plane p sits in slot (p - kbeg) & 3, kbeg = k0 - 3 being the
    // first iteration; the loop is unrolled four times so that every slot
    // index is a constant and slots keep their roles from one loop trip to
    // the next (no register moves to rotate queues).
    //   LE: lE' at k-1 .. k+2;  MU: mu at k-1 .. k+1;  EN: primal E at k, k+1
    //   (staged in LDS for the x+1 and y+1 neighbours the gradient needs);
    //   S0, S3: stars 0 and 3 of mu at k-2 .. k.
    // Prefetched values (lE'(k+2), lB'(k+1), E(k+1)) alternate between two
    // register sets, so a load issued in one iteration is first waited for in
    // the next.
    T LE[4][3], MU[4][3], EN[4][3], S0[4], S3[4];
    T pe[2][3], pb[2][3], pn[2][3];
    double acc[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[j] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int c = 0; c < 3; ++c) LE[q][c] = MU[q][c] = EN[q][c] = T(0);
        S0[q] = S3[q] = T(0);
    }

    // plane trackers (k starts at k0 - 3): w3 = k+3 (lE' prefetch),
    // wb = k+1 -> k+2 (lB' prefetch), wn = k+1 -> k+2 (primal E prefetch),
    // wm = k-1 (outputs)
    int w3 = wrapa(k0, nz), wb = wrapa(k0 - 2, nz), wn = wrapa(k0 - 2, nz), wm = wrapa(k0 - 4, nz);
    {
        const uint64_t pa = (uint64_t)(uint32_t)wrapa(k0 - 2, nz) * nxy, pq = (uint64_t)(uint32_t)wrapa(k0 - 1, nz) * nxy;
        const uint64_t pm = (uint64_t)(uint32_t)wrapa(k0 - 3, nz) * nxy;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            LE[1][c] = src[c][pa + col];    // lE'(kbeg + 1)
            pe[0][c] = src[c][pq + col];    // lE'(kbeg + 2)
            pb[0][c] = src[3 + c][pa + colb];
            pn[0][c] = en[c][pa + coln];
            EN[0][c] = en[c][pm + coln];    // E(kbeg)
        }
        if (isE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                LEbuf[0][c][li] = LE[1][c];
                Ebuf[0][c][li] = EN[0][c];
            }
        }
    }
    __syncthreads();

    const int klast = k0 + KZe - 1;
    // One plane iteration, i = k - kbeg; I = i & 3 picks the ring slots,
    // B = I & 1 the LDS buffers and the prefetch set consumed (set B^1 is
    // refilled).
    auto plane = [&](auto slot, int k) {
        constexpr int I = decltype(slot)::value;
        constexpr int B = I & 1;
        constexpr int eb = B, mb = B, sb = B;
        constexpr int m1 = (I + 3) & 3, s0 = I, p1 = (I + 1) & 3, p2 = (I + 2) & 3;
        T bo[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            LE[p2][c] = pe[B][c];  // lE'(k+2)
            bo[c] = pb[B][c];      // lB'(k+1)
            EN[p1][c] = pn[B][c];  // E(k+1)
        }
        // per-iteration copies of the lane offsets, opaque to the compiler, so
        // that addresses stay scalar plane base + 32-bit lane offset (no
        // per-lane 64-bit adds hoisted out of the loop)
        uint32_t oc = col, ob = colb, on = coln;
        asm("" : "+v"(oc), "+v"(ob), "+v"(on));
        {
            const uint64_t p3 = (uint64_t)(uint32_t)w3 * nxy;
            wb = inc(wb);
            wn = inc(wn);
            const uint64_t pq = (uint64_t)(uint32_t)wb * nxy, pn2 = (uint64_t)(uint32_t)wn * nxy;  // k+2: own E
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pe[B ^ 1][c] = ld_plane_a(src[c] + p3, oc);
                pb[B ^ 1][c] = ld_plane_a(src[3 + c] + pq, ob);
                pn[B ^ 1][c] = ld_plane_a(en[c] + pn2, on);
            }
        }
        if (isE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                LEbuf[eb ^ 1][c][li] = LE[p2][c];
                Ebuf[eb ^ 1][c][li] = EN[p1][c];
            }
        }

        // mu(k+1) = lB'(k+1) + L^T lE' (lanes outside the mu region read the
        // neighbours of slot 0: in bounds, value unused)
        adj_mu<PX>(MU[p1], bo, LE[p1], LE[p2], LEbuf[eb][0], LEbuf[eb][1], LEbuf[eb][2], isG ? li : 0, w);
        if (isG) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Mbuf[mb ^ 1][c][li] = MU[p1][c];
        }

        // stars of mu at plane k
        const T *mn = MU[p1], *mc = MU[s0], *mm = MU[m1];
        T s[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
        T px[3] = {T(0), T(0), T(0)}, py[3] = {T(0), T(0), T(0)}, pz[3] = {T(0), T(0), T(0)};
        if (isB && k >= k0 - 1 && k <= klast) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T *M = Mbuf[mb][c];
                px[c] = M[li + 1] + M[li - 1];
                py[c] = M[li + PX] + M[li - PX];
                pz[c] = mn[c] + mm[c];
            }
            adj_stars(s, mc, px, py, pz, w);
#pragma unroll
            for (int m = 0; m < 6; ++m) Sbuf[sb][m][li] = s[m];
            if (isO && k >= k0)  // coefficient gradient at plane k
                adj_grad<PX>(acc, EN[s0], EN[p1], Ebuf[eb][0], Ebuf[eb][1], Ebuf[eb][2], li, mc, px, py, pz);
        }
        S0[s0] = s[0];
        S3[s0] = s[3];

        // outputs of plane k-1: lE = lE' + backward differences of its stars
        // (stars 0 and 3 of planes k-1 and k-2 from registers)
        if (isO && k - 1 >= k0) {
            const T(*Sp)[P] = Sbuf[sb ^ 1];
            const uint64_t po = (uint64_t)(uint32_t)wm * nxy;
            T le[3];
            adj_out<PX, P>(le, LE[m1], S3[m1], S3[p2], S0[m1], S0[p2], Sp, li);
            st_plane_a(dst[0] + po, oc, le[0]);
            st_plane_a(dst[1] + po, oc, le[1]);
            st_plane_a(dst[2] + po, oc, le[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) st_plane_a(dst[3 + c] + po, oc, mm[c]);
        }
        __syncthreads();
        w3 = inc(w3);
        wm = inc(wm);
    };
    // KZe + 4 iterations (k = k0 - 3 .. klast + 1), four per loop trip; the
    // loop leaves after exactly that many (an extra iteration would write the
    // outputs of a plane beyond the chunk)
    for (int k = k0 - 3;; k += 4) {
        plane(std::integral_constant<int, 0>{}, k);
        if (k + 1 > klast + 1) break;
        plane(std::integral_constant<int, 1>{}, k + 1);
        if (k + 2 > klast + 1) break;
        plane(std::integral_constant<int, 2>{}, k + 2);
        if (k + 3 > klast + 1) break;
        plane(std::integral_constant<int, 3>{}, k + 3);
        if (k + 4 > klast + 1) break;
    }

    // workgroup reduction of the 12 gradient sums (FP64)
    adj_reduce<C>(acc, red, slot, accumulate, wave, lane);
}

// Shared storage of a workgroup: the z-march's, or the one-plane pass's.
template <typename T, typename C, bool PLANE>
using AdjStore = std::conditional_t<PLANE, PlaneAdjStore<T, C>, AdjSmem<T, C>>;
// waves per SIMD to leave room for: two 13-wave workgroups of the one-plane
// pass share a CU
template <typename C, bool PLANE>
constexpr int adj_min_waves() { return PLANE ? 7 : C::MIN_WAVES; }

template <typename T, typename C, bool PLANE = false>
__global__ __launch_bounds__(C::THREADS, (adj_min_waves<C, PLANE>())) void adjoint_step_kernel(
    Fields<T> lin, Fields<T> lout, const T *__restrict__ en_x, const T *__restrict__ en_y,
    const T *__restrict__ en_z, Dims d, Weights<T> w, int zchunk, int ntx, int nty,
    double *__restrict__ partials, int accumulate)
{
    __shared__ AdjStore<T, C, PLANE> store;
    AdjSmem<T, C> &sm = reinterpret_cast<AdjSmem<T, C> &>(store);
    if constexpr (PLANE) {
        // consecutive tiles, as many per workgroup as the grid leaves; one
        // reduction into the first one's slot, the others' slots hold zero
        const int ntiles = ntx * nty;
        const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
        const int t0 = (int)blockIdx.x * per, t1 = min(t0 + per, ntiles);
        if (t0 >= ntiles) return;  // the whole workgroup, before any barrier
        double acc[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) acc[j] = 0.0;
        for (int t = t0; t < t1; ++t) {
            adjoint_tile<T, C, true>(lin, lout, en_x, en_y, en_z, d, w, zchunk, ntx, nty, t, sm, nullptr, 0, acc);
            __syncthreads();  // LDS is reused by the next tile
        }
        adj_reduce<C>(acc, store.red, partials + (int64_t)t0 * 12, accumulate, threadIdx.x >> 6, threadIdx.x & 63);
        if (!accumulate && threadIdx.x < 12)
            for (int t = t0 + 1; t < t1; ++t) partials[(int64_t)t * 12 + threadIdx.x] = 0.0;
        return;
    }
    const int nb = gridDim.x, bid = blockIdx.x;
    const int q = nb >> 3, r = nb & 7, xcd = bid & 7;
    const int logical = xcd * q + min(xcd, r) + (bid >> 3);
    adjoint_tile<T, C, PLANE>(lin, lout, en_x, en_y, en_z, d, w, zchunk, ntx, nty, logical, sm,
                              partials + (int64_t)blockIdx.x * 12, accumulate);
}

// Batched adjoint step: work item j is tile items[j].y of box items[j].x
// (each box's items contiguous); its 12 gradient sums live at partials[12 j]
// (the item list is fixed for a batch, so the sums accumulate per item across
// steps).  Workgroup w takes the slots w, w + gridDim.x, ... of `order`, which
// holds item numbers in the host's dispatch order (-1: no work).
// ONE: one workgroup per slot (gridDim.x == nslots), no slot loop: nothing
// stays live from one item to the next (the looping variant of the 32x12 tile
// spills at the register budget of five waves per SIMD).  PLANE: every box is
// one plane deep (the one-plane pass of adjoint_tile).
template <typename T, typename C, bool ONE, bool PLANE = false>
__global__ __launch_bounds__(C::THREADS, (adj_min_waves<C, PLANE>())) void batched_adjoint_kernel(const AdjDesc<T> *__restrict__ boxes,
                                                                     const int2 *__restrict__ items,
                                                                     const int *__restrict__ order, int nslots,
                                                                     double *__restrict__ partials,
                                                                     int accumulate)
{
    __shared__ AdjStore<T, C, PLANE> store;
    AdjSmem<T, C> &sm = reinterpret_cast<AdjSmem<T, C> &>(store);
    if constexpr (ONE) {
        const int j = order[blockIdx.x];
        if (j < 0) return;
        const int2 it = items[j];
        const AdjDesc<T> &b = boxes[it.x];
        if constexpr (PLANE) {  // it.y: a group of b.group tiles
            double acc[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) acc[q] = 0.0;
            const int t0 = it.y * b.group, t1 = min(t0 + b.group, b.ntx * b.nty);
            for (int t = t0; t < t1; ++t) {
                adjoint_tile<T, C, true>(b.lin, b.lout, b.en[0], b.en[1], b.en[2], b.d, b.w, b.zchunk, b.ntx, b.nty,
                                         t, sm, nullptr, 0, acc);
                __syncthreads();  // LDS is reused by the next tile
            }
            adj_reduce<C>(acc, store.red, partials + (int64_t)j * 12, accumulate, threadIdx.x >> 6,
                          threadIdx.x & 63);
        } else {
            adjoint_tile<T, C>(b.lin, b.lout, b.en[0], b.en[1], b.en[2], b.d, b.w, b.zchunk, b.ntx, b.nty, it.y,
                               sm, partials + (int64_t)j * 12, accumulate);
        }
        return;
    }
    for (int i = blockIdx.x; i < nslots; i += gridDim.x) {
        const int j = order[i];
        if (j < 0) continue;
        const int2 it = items[j];
        const AdjDesc<T> &b = boxes[it.x];
        adjoint_tile<T, C, PLANE>(b.lin, b.lout, b.en[0], b.en[1], b.en[2], b.d, b.w, b.zchunk, b.ntx, b.nty, it.y,
                                  sm, partials + (int64_t)j * 12, accumulate);
        __syncthreads();
    }
}

// Sums of the 12-value slots i0, i0 + stride, ... (count of them) of
// partials by a 256-thread workgroup, fixed order: thread t adds slots
// number t, t + 256, ... in turn (all 12 values of a slot loaded together),
// then a tree over the threads; slot value j's total ends in sm[j][0].
__device__ __forceinline__ void sum_slots(const double *partials, int i0, int count, int stride,
                                          double (&sm)[12][256])
{
    double v[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) v[j] = 0.0;
    for (int m = (int)threadIdx.x; m < count; m += 256) {
        const double *p = partials + ((int64_t)i0 + (int64_t)m * stride) * 12;
#pragma unroll
        for (int j = 0; j < 12; ++j) v[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j < 12; ++j) sm[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < 12; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + st];
        __syncthreads();
    }
}

// grad[12 b + j] += scale[12 b + j] * sum of partials over box b's items
// [first[b], first[b+1]); one block per box, fixed order.
__global__ __launch_bounds__(256) void reduce_boxes_kernel(const double *__restrict__ partials,
                                                           const int *__restrict__ first,
                                                           const double *__restrict__ scale,
                                                           double *__restrict__ grad)
{
    __shared__ double sm[12][256];
    const int b = blockIdx.x;
    sum_slots(partials, first[b], first[b + 1] - first[b], 1, sm);
    if (threadIdx.x < 12) grad[12 * b + threadIdx.x] += scale[12 * b + threadIdx.x] * sm[threadIdx.x][0];
}

// First stage of a long reduction: workgroup k sums the slots [256 k,
// 256 k + 256) and writes the sums into slot 256 k, in place.
__global__ __launch_bounds__(256) void reduce_chunks_kernel(double *partials, int nblocks)
{
    __shared__ double sm[12][256];
    const int i0 = (int)blockIdx.x * 256;
    sum_slots(partials, i0, min(256, nblocks - i0), 1, sm);  // ends with a barrier: slot i0 has been read
    if (threadIdx.x < 12) partials[(int64_t)i0 * 12 + threadIdx.x] = sm[threadIdx.x][0];
}

// grad[j] += scale[j] * sum over the slots 0, stride, ... (nslots of them)
// of partials[slot][j], one block, fixed order.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *__restrict__ partials,
                                                              int nslots, int stride, Scale12 sc,
                                                              double *__restrict__ grad)
{
    __shared__ double sm[12][256];
    sum_slots(partials, 0, nslots, stride, sm);
    if (threadIdx.x < 12) grad[threadIdx.x] += sc.s[threadIdx.x] * sm[threadIdx.x][0];
}

// Calls f(C{}) with the adjoint tile configuration of (tile_x, tile_y); the
// 64x8 tile is FP32 only (in FP64 it would exceed the 160 KiB of LDS), and so
// is the 32x12 tile (8 row waves and the halo wave; two workgroups per CU).
template <typename T, typename F>
hipError_t with_adj_tile(int tile_x, int tile_y, F &&f)
{
    if (tile_x == 64) {
        if (tile_y == 4) return f(AdjCfg<64, 4>{});
        if constexpr (sizeof(T) == 4)
            if (tile_y == 8) return f(AdjCfg<64, 8>{});
    } else if (tile_x == 32) {
        if (tile_y == 4) return f(AdjCfg<32, 4>{});
        if (tile_y == 8) return f(AdjCfg<32, 8>{});
        if constexpr (sizeof(T) == 4)
            if (tile_y == 12) return f(AdjCfg<32, 12>{});
    }
    return hipErrorInvalidValue;
}

}  // namespace

int adjoint_blocks(Dims d, int tile_x, int tile_y, int zchunk)
{
    const int ntx = (d.nx + tile_x - 1) / tile_x;
    const int nty = (d.ny + tile_y - 1) / tile_y;
    const int nzc = (d.nz + zchunk - 1) / zchunk;
    return ntx * nty * nzc;
}

template <typename T>
hipError_t launch_adjoint(const Fields<T> &lin, const Fields<T> &lout, const T *const en[3], Dims d,
                          const Weights<T> &w, int tile_x, int tile_y, int zchunk, double *partials,
                          int accumulate, hipStream_t s)
{
    if (tile_x != 64 && tile_x != 32) return hipErrorInvalidValue;
    const int ntx = (d.nx + tile_x - 1) / tile_x;
    const int nty = (d.ny + tile_y - 1) / tile_y;
    const int nb = adjoint_blocks(d, tile_x, tile_y, zchunk);
    return with_adj_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        if (d.nz == 1) {  // one plane: the one-plane pass, several tiles per workgroup (same partial slots)
            const int g = plane_adj_group(nb);
            hipLaunchKernelGGL((adjoint_step_kernel<T, C, true>), dim3((nb + g - 1) / g), dim3(C::THREADS), 0, s,
                               lin, lout, en[0], en[1], en[2], d, w, zchunk, ntx, nty, partials, accumulate);
        }
        else
            hipLaunchKernelGGL((adjoint_step_kernel<T, C>), dim3(nb), dim3(C::THREADS), 0, s, lin, lout, en[0],
                               en[1], en[2], d, w, zchunk, ntx, nty, partials, accumulate);
        return hipGetLastError();
    });
}

int plane_adj_group(int64_t tiles)
{
    static int ncu[64];  // per device, looked up once
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        dev = -1;
    }
    int n = dev >= 0 ? __atomic_load_n(&ncu[dev], __ATOMIC_RELAXED) : 0;
    if (n <= 0) {
        if (dev < 0 || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0) {
            (void)hipGetLastError();
            n = 256;
        } else {
            __atomic_store_n(&ncu[dev], n, __ATOMIC_RELAXED);
        }
    }
    const int64_t g = tiles / (2 * (int64_t)n);
    return (int)(g < 1 ? 1 : g > kPlaneAdjTiles ? kPlaneAdjTiles : g);
}

template <typename T>
int adjoint_occupancy(int tile_x, int tile_y)
{
    int n = 0;
    const hipError_t e = with_adj_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, adjoint_step_kernel<T, C>, C::THREADS, 0);
    });
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

template int adjoint_occupancy<float>(int, int);
template int adjoint_occupancy<double>(int, int);

hipError_t launch_reduce_partials(double *partials, int nblocks, const Scale12 &sc, double *grad, hipStream_t s)
{
    if (nblocks > 1024) {  // chunks of 256 slots first (one workgroup each), then their sums
        const int nch = (nblocks + 255) / 256;
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3(nch), dim3(256), 0, s, partials, nblocks);
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partials, nch, 256, sc, grad);
    } else {
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, 1, sc, grad);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batched_adjoint(const AdjDesc<T> *boxes, const int2 *items, const int *order, int nslots,
                                 double *partials, int accumulate, int tile_x, int tile_y, int grid, hipStream_t s,
                                 bool plane)
{
    if (nslots <= 0) return hipSuccess;
    if (grid <= 0 || grid > nslots) grid = nslots;
    return with_adj_tile<T>(tile_x, tile_y, [&](auto cfg) {
        using C = decltype(cfg);
        if (plane)  // every box one plane deep: one workgroup per slot
            hipLaunchKernelGGL((batched_adjoint_kernel<T, C, true, true>), dim3(nslots), dim3(C::THREADS), 0, s,
                               boxes, items, order, nslots, partials, accumulate);
        else if (grid == nslots)
            hipLaunchKernelGGL((batched_adjoint_kernel<T, C, true>), dim3(grid), dim3(C::THREADS), 0, s, boxes,
                               items, order, nslots, partials, accumulate);
        else
            hipLaunchKernelGGL((batched_adjoint_kernel<T, C, false>), dim3(grid), dim3(C::THREADS), 0, s, boxes,
                               items, order, nslots, partials, accumulate);
        return hipGetLastError();
    });
}

hipError_t launch_reduce_boxes(const double *partials, const int *first, int nboxes, const double *scale,
                               double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_boxes_kernel, dim3(nboxes), dim3(256), 0, s, partials, first, scale, grad);
    return hipGetLastError();
}

template hipError_t launch_batched_adjoint<float>(const AdjDesc<float> *, const int2 *, const int *, int, double *,
                                                  int, int, int, int, hipStream_t, bool);
template hipError_t launch_batched_adjoint<double>(const AdjDesc<double> *, const int2 *, const int *, int,
                                                   double *, int, int, int, int, hipStream_t, bool);
template hipError_t launch_adjoint<float>(const Fields<float> &, const Fields<float> &, const float *const[3],
                                          Dims, const Weights<float> &, int, int, int, double *, int, hipStream_t);
template hipError_t launch_adjoint<double>(const Fields<double> &, const Fields<double> &,
                                           const double *const[3], Dims, const Weights<double> &, int, int, int,
                                           double *, int, hipStream_t);

}  // namespace xfdtd
