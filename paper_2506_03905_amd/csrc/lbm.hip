// lbm.hip -- gfx950 kernels and C ABI of the LBM-RANS hot path.
//
// One time step (Ponsin & Lozano, arXiv 2506.03905) is two launches:
//   k_step  fused streaming (single-buffer AA pattern) + wall links
//           (halfway bounce-back eq. 31 with the wall velocity of eq. 35,
//           Bouzidi's or Yu's interpolated rules eq. 36-37, or the
//           regularized reconstruction eq. 19/23/26-28 with the gradient of
//           eq. 27-28 or of Cai-Degrigny, eq. 29-30) + plate edges +
//           moments (eq. 4-5) + BGK/Guo or central-moment (eq. 7) collision
//           with tau from nu + nu_t (eq. 8, 10) + the Spalart-Allmaras
//           update (eq. 11-14);
//   k_wall  the per-wall-cell FP64 Newton solve for u_tau at the reference
//           node F (Sec. 3.1, eq. 20-22), the slip velocity (eq. 35) and the
//           SA Dirichlet value nu_tilde_B = nu kappa y_B+ (Sec. 2.2).
// A residual reduction (mass, momentum, velocity change, mean u_tau) runs
// every K steps in FP64 with a fixed summation order.  The serving pool runs
// the same cell update for many lattices at once: small ones in a persistent
// kernel with the time loop inside (k_serve), large ones in shared launches
// per phase (k_mstep, k_mwall, k_mreduce).
//
// AA pattern: after an even step (and after initialisation) slot A[opp(i)][x]
// holds the post-collision f*_i(x); an odd step pulls from neighbours and
// pushes to neighbours, leaving A[i][x + c_i] = f*_i(x).  Each slot is read and
// written by one thread only, so one buffer suffices.  Populations that leave
// the domain through a wall or an open boundary are parked in the cell's own
// free slot A[opp(i)][x]; populations that cross a symmetry plane are pushed
// to their mirrored destination.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_device.hpp"

using namespace lbmd;

// Staging memory of lbm_moments_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never uses this name as an
// address: the device address of each GPU's copy comes from
// hipGetSymbolAddress (scratch_on below) and is what kernels and copies get.
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int BLK = 256;  // threads per block of the per-cell kernels (128 and 512 measured slower)
#ifndef LBM_XSTAGE
#define LBM_XSTAGE 1
#endif
#ifndef LBM_ROWMAP
#define LBM_ROWMAP 1
#endif
constexpr int NRED = 8;        // reduction slots
constexpr int RED_BLOCKS = 2048;
constexpr int MID_BLOCKS = 256;  // blocks of the middle pass of a reduction
constexpr int RES_STICKY = 2 * NRED;  // result[RES_STICKY]: 1 once any reduction saw a bad cell

// ---------------------------------------------------------------------------
// Thread -> cell mapping.
// Channel: flat cell index; the hardware places block b on XCD b % 8, so the
// logical block order is remapped to give each XCD one contiguous range of
// rows (neighbouring rows of the SA stencil then share an L2).
// Plate: one row per group of blocks, blocks aligned to the right end of the
// row so that columns nx-2 and nx-1 share a block (outlet exchange in LDS).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t xcd_block(uint32_t b, uint32_t nb)
{
    uint32_t nb8 = nb & ~7u;
    if (b >= nb8) return b;
    return (int64_t)(b & 7u) * (nb8 >> 3) + (b >> 3);
}

template <typename T> __device__ __forceinline__ T clamp0(T v) { return v > (T)0 ? v : (T)0; }

// ---------------------------------------------------------------------------
// Per-cell context: coordinates, neighbour offsets (periodic in x for the
// channel and in z), wall index.
// ---------------------------------------------------------------------------
struct Cell {
    int x, y, z;
    int64_t cell, wi;
    int64_t oxm, oxp, ozm, ozp, sy, sz;
    int64_t pb;  // index of population 0 of this cell in the row-interleaved layout
    bool bottom, top;
};

// Population storage is row-interleaved: each row of nx cells (fixed y, z)
// holds its Q populations as Q consecutive runs of nx values,
//   index(q, x, row) = (row * Q + q) * nx + x,   row = y + ny z,
// so one row's populations form one contiguous block of HBM.
template <int Q> __device__ __forceinline__ int64_t pidx(int nx, int q, int x, int64_t row)
{
    return (row * Q + q) * (int64_t)nx + x;
}

// INT: the cell's row is known to hold neither a wall cell nor a symmetry
// plane (an interior row of the channel's row mapping), so every boundary
// test below folds away at compile time.
template <int Q, bool PLATE, bool INT = false>
__device__ __forceinline__ Cell make_cell(const KP &P, int x, int y, int z, bool active)
{
    Cell C;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    C.x = x;
    C.y = y;
    C.z = z;
    C.sy = nx;
    C.sz = (int64_t)nx * ny;
    C.cell = (int64_t)x + (int64_t)nx * (y + (int64_t)ny * z);
    C.pb = pidx<Q>(nx, 0, x, y + (int64_t)ny * z);
    C.oxm = (x == 0) ? (PLATE ? 0 : nx - 1) : -1;
    C.oxp = (x == nx - 1) ? (PLATE ? 0 : -(int64_t)(nx - 1)) : 1;
    C.ozm = (z == 0) ? (int64_t)(nz - 1) * C.sz : -C.sz;
    C.ozp = (z == nz - 1) ? -(int64_t)(nz - 1) * C.sz : C.sz;
    C.bottom = !INT && y == 0;
    C.top = !INT && y == ny - 1;
    C.wi = (active && !INT) ? wall_index(P, x, y, z) : -1;
    return C;
}

// offset from the cell to the cell x + c
__device__ __forceinline__ int64_t off(const Cell &C, int ccx, int ccy, int ccz)
{
    return (ccx > 0 ? C.oxp : (ccx < 0 ? C.oxm : 0)) + (int64_t)ccy * C.sy + (ccz > 0 ? C.ozp : (ccz < 0 ? C.ozm : 0));
}

// offset, in the population layout, from slot (q, x) to slot (q, x + c)
template <int Q> __device__ __forceinline__ int64_t poff(const Cell &C, int ccx, int ccy, int ccz)
{
    return (ccx > 0 ? C.oxp : (ccx < 0 ? C.oxm : 0)) +
           (int64_t)Q * ((int64_t)ccy * C.sy + (ccz > 0 ? C.ozp : (ccz < 0 ? C.ozm : 0)));
}

// Staged odd-step pushes (XS): on the channel's row mapping a block covers BLK
// consecutive columns of one row; the x-shifted pushes that land inside the
// block are staged in LDS at their destination column and written after one
// barrier as whole aligned runs.  A push shifted by one column straight to
// HBM leaves every cache line of its run written in two parts by two waves,
// which costs HBM write efficiency; staged, only the block's two edge
// columns are written alone.  Directions with c_x != 0 own one LDS row each.
template <int Q> __host__ __device__ constexpr int nxdirs()
{
    int n = 0;
    for (int i = 0; i < Q; ++i) n += cx<Q>(i) != 0;
    return n;
}
template <int Q> __host__ __device__ constexpr int xslot(int i)
{
    int n = 0;
    for (int k = 0; k < i; ++k) n += cx<Q>(k) != 0;
    return n;
}

// ---------------------------------------------------------------------------
// gather: the incoming populations of one cell (deviations f - w rho0) with
// the wall links (eq. 31) and symmetry planes resolved; the open-boundary
// unknowns of the plate are left at 0 for plate_edges.
// ---------------------------------------------------------------------------
// FOLD: the storage shift is left on the values (the collision works on the
// stored values, see finish).
template <int Q, typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool IBB = false, bool FOLD = false>
__device__ __forceinline__ void gather(const KP &P, const Cell &C, T *f)
{
    using SS = Stor<S>;
    const int nx = P.nx;
    const int x = C.x;
    const bool bottom = C.bottom, top = C.top;
    const int64_t pb = C.pb, wi = C.wi;
    const S *__restrict__ A = (const S *)P.pops;
    T rho_w = 0, uwv[3] = {0, 0, 0};
    if (!HRFD && wi >= 0) {
        rho_w = (T)P.wrho[wi];
        uwv[0] = (T)P.uw[wi];
        uwv[1] = (T)P.uw[P.nwall + wi];
        uwv[2] = (T)P.uw[2 * P.nwall + wi];
    }
    const bool active = true;
    const CellK<T> &K = ck<T>(P);
    // ---- gather the incoming populations (deviations f - w rho0) ----------
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ccx = cx<Q>(i), ccy = cy<Q>(i), ccz = cz<Q>(i);
        constexpr int io = opp<Q>(i), im = opp<Q>(mir<Q>(i));
        const bool ycross = (ccy > 0 && bottom) || (ccy < 0 && top);
        const bool wall = ycross && (top ? (P.flow == FLOW_CHANNEL) : bottom_is_wall(P, x, -ccx));
        // the slot holds population i (interior), opp(i) (wall) or mir(i)
        // (symmetry); the index is selected, not branched on, so that every
        // load is issued unconditionally (an open-boundary unknown reads a
        // slot of its own row and is discarded)
        int64_t idx = pb + i * nx;
        if (ODD)
            idx = !ycross ? pb + io * nx + poff<Q>(C, -ccx, -ccy, -ccz)
                          : (wall ? pb + i * nx : pb + im * nx + poff<Q>(C, -ccx, 0, -ccz));
        f[i] = SS::ld(ld_pop(&A[idx]));
    });
    // storage shift of the population the slot held (uniform branch)
    if (!FOLD && P.shifted)
        sfor<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int ccx = cx<Q>(i), ccy = cy<Q>(i);
            const bool ycross = (ccy > 0 && bottom) || (ccy < 0 && top);
            const bool wall = ycross && (top ? (P.flow == FLOW_CHANNEL) : bottom_is_wall(P, x, -ccx));
            f[i] += !ycross ? K.soff[i] : (wall ? K.soff[opp<Q>(i)] : K.soff[mir<Q>(i)]);
        });
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ccx = cx<Q>(i), ccy = cy<Q>(i), ccz = cz<Q>(i);
        const bool xopen = PLATE && ((ccx > 0 && x == 0) || (ccx < 0 && x == nx - 1));
        const bool ycross = (ccy > 0 && bottom) || (ccy < 0 && top);
        const bool wall = ycross && (top ? (P.flow == FLOW_CHANNEL) : bottom_is_wall(P, x, -ccx));
        T v = f[i];
        // eq. 31: f_i = f*_opp(i) + 2 w_i rho_w (c_i . u_w) / cs2 (halfway links;
        // interpolated links keep f*_opp(i) here and are finished by ibb_links)
        if (!HRFD && wall && wi >= 0 && (!IBB || P.bb_interp == IBB_HALFWAY))
            v += (T)(6.0 * wgt<Q>(i)) * rho_w * ((T)ccx * uwv[0] + (T)ccy * uwv[1] + (T)ccz * uwv[2]);
        f[i] = (active && !xopen) ? v : (T)0;
    });
}

// Interpolated bounce-back (eq. 36 Bouzidi, eq. 37 Yu) at a wall cell, the
// wall at q = d_w from B along every wall link.  On entry f[r] of a wall link r
// holds f*_k(B) (k = opp(r), the population that left B towards the wall) and
// f[k] holds f_k(B, t+1) = f*_k(F), arrived from F = B - c_k; ibuf keeps B's
// post-collision populations of the previous step, f*_r(B) = f_r(F, t+1).
// On the plate the outlet column is treated after the outlet copy and the
// others before it; a reflection whose halfway source lies outside the
// lattice stays an open-boundary unknown.
template <int Q, typename T, bool PLATE>
__device__ __forceinline__ void ibb_links(const KP &P, const Cell &C, T *f)
{
    const int64_t wi = C.wi;
    if (P.bb_interp == IBB_HALFWAY || wi < 0) return;
    const T q = (T)P.wall_dist;
    const T rho_w = (T)P.wrho[wi];
    const T uwv[3] = {(T)P.uw[wi], (T)P.uw[P.nwall + wi], (T)P.uw[2 * P.nwall + wi]};
    const double *fr_prev = P.ibuf + wi * Q;
    const int side = C.bottom ? -1 : 1;  // wall below / above the cell
    const bool bouzidi = P.bb_interp == IBB_BOUZIDI;
    sfor<Q>([&](auto ic) {
        constexpr int r = decltype(ic)::value;  // leaves the wall
        constexpr int k = opp<Q>(r);
        constexpr int crx = cx<Q>(r), cry = cy<Q>(r), crz = cz<Q>(r);
        if (cry != -side) return;
        if (!(side < 0 ? bottom_is_wall(P, C.x, -crx) : P.flow == FLOW_CHANNEL)) return;
        if (PLATE && (C.x - crx < 0 || C.x - crx >= P.nx)) return;
        // eq. 31's moving-wall term, 2 w rho_w (c_r . u_w) / cs2
        const T m = (T)(6.0 * wgt<Q>(r)) * rho_w * ((T)crx * uwv[0] + (T)cry * uwv[1] + (T)crz * uwv[2]);
        const T fkB = f[r], fkF = f[k], frB = (T)fr_prev[r];
        T v;
        if (bouzidi) {
            if (q < (T)0.5)
                v = (T)2 * q * fkB + ((T)1 - (T)2 * q) * fkF + m;
            else
                v = fkB / ((T)2 * q) + ((T)2 * q - (T)1) / ((T)2 * q) * frB + m / ((T)2 * q);
        } else {
            const T frW = q * fkB + ((T)1 - q) * fkF + m;  // at the wall point
            v = frW + q / ((T)1 + q) * (frB - frW);
        }
        f[r] = v;
    });
}

// Zou-He inlet (D2Q9, west face, u = (U, 0)): the known weights sum to 1 in
// deviation form.
template <typename T> __device__ __forceinline__ void zou_he(const KP &P, T *f)
{
    const T U = (T)P.u_inlet, r0 = (T)P.rho0;
    T s = f[0] + f[3] + f[4] + (T)2 * (f[2] + f[6] + f[8]);
    T rho = (r0 + s) / ((T)1 - U);
    f[1] = f[2] + (T)(2.0 / 3.0) * rho * U;
    f[5] = f[6] - (T)0.5 * (f[3] - f[4]) + (T)(1.0 / 6.0) * rho * U;
    f[7] = f[8] + (T)0.5 * (f[3] - f[4]) + (T)(1.0 / 6.0) * rho * U;
}

// ---------------------------------------------------------------------------
// Spalart-Allmaras update of one cell (eq. 10-14) from nu_tilde^n and
// u^{n-1} (ping-pong index rd); wall cells get their value from k_wall.
// ---------------------------------------------------------------------------
template <int Q, typename T, bool PLATE>
__device__ __forceinline__ void sa_cell(const KP &P, const Cell &C, int rd, T nt0)
{
    constexpr int D = Lat<Q>::D;
    if (!P.sa_on) return;
    const int ny = P.ny;
    const int64_t N = P.ncell;
    const int x = C.x, y = C.y;
    const int64_t cell = C.cell, wi = C.wi, sy = C.sy;
    const int64_t oxm = C.oxm, oxp = C.oxp, ozm = C.ozm, ozp = C.ozp;
    const T *__restrict__ u_rd = (const T *)P.u[rd];
    const T *__restrict__ nt_rd = (const T *)P.nt[rd];
    T *__restrict__ nt_wr = (T *)P.nt[rd ^ 1];
    const bool dirichlet = (wi >= 0) || (PLATE && x == 0);
    if (dirichlet) {
        if (wi < 0) nt_wr[cell] = nt0;  // plate inlet keeps its value; walls: k_wall
        return;
    }
    T ntm[3], ntp[3], g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    // x neighbours (plate outlet: zero-gradient copy)
    {
        const int64_t cm = cell + oxm, cp = cell + oxp;  // plate: oxp = 0 at the outlet
        ntm[0] = nt_rd[cm];
        ntp[0] = nt_rd[cp];
        g[1][0] = (u_rd[N + cp] - u_rd[N + cm]) * (T)0.5;
        if (D == 3) g[2][0] = (u_rd[2 * N + cp] - u_rd[2 * N + cm]) * (T)0.5;
    }
    // y neighbours (plate symmetry planes: mirror image, same tangential velocity)
    {
        const int64_t cm = C.bottom ? cell : cell - sy, cp = C.top ? cell : cell + sy;
        ntm[1] = nt_rd[cm];
        ntp[1] = nt_rd[cp];
        g[0][1] = (u_rd[cp] - u_rd[cm]) * (T)0.5;
        if (D == 3) g[2][1] = (u_rd[2 * N + cp] - u_rd[2 * N + cm]) * (T)0.5;
    }
    if (D == 3) {
        const int64_t cm = cell + ozm, cp = cell + ozp;
        ntm[2] = nt_rd[cm];
        ntp[2] = nt_rd[cp];
        g[0][2] = (u_rd[cp] - u_rd[cm]) * (T)0.5;
        g[1][2] = (u_rd[N + cp] - u_rd[N + cm]) * (T)0.5;
    }
    T u0[3] = {u_rd[cell], u_rd[N + cell], D == 3 ? u_rd[2 * N + cell] : (T)0};
    const T d = wall_dist<T>(P, x, y);
    const T rhs = sa_rhs<D, T>(P, nt0, ntm, ntp, u0, g, d);
    nt_wr[cell] = clamp0(nt0 + rhs);
}

// ---------------------------------------------------------------------------
// FP64 reductions.  Slots: 0 sum(rho - rho0), 1-3 sum(rho u), 4 sum |u -
// u_snap|^2, 5 sum |u|^2, 6 count of cells with a non-finite value or rho <= 0,
// 7 sum of u_tau over the wall cells.  Sums run in a fixed tree order.
// ---------------------------------------------------------------------------
template <int NT> __device__ __forceinline__ void block_sum(double (*sh)[NT], double *v, int nv)
{
    const int t = threadIdx.x;
    for (int k = 0; k < nv; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < nv; ++k) sh[k][t] += sh[k][t + s];
        __syncthreads();
    }
}

// One cell's share of slots 0-6, taken inside the step from the density and
// velocity it has just computed (the snapshot u_snap is refreshed on the way).
struct RedAcc {
    double v[7];
};

// BGK collision with Guo forcing of one cell (see finish).  SH: f holds the
// stored values f - soff of the storage shift, and the relaxation targets
// f_eq - soff, so that f* - soff is what is left in f.
template <int Q, typename T, bool SH>
__device__ __forceinline__ void bgk_collide(const CellK<T> &K, T *f, T drho, T rho, T ux, T uy, T uz, T jx, T jy,
                                            T jz, T omega)
{
    constexpr int D = Lat<Q>::D;
    const T Fx = K.fx, Fy = K.fy, Fz = K.fz;
    // BGK with Guo forcing, f* = f - omega (f - f_eq) + S with
    //   f_eq_i = w_i (drho + rho (3 cu + 9/2 cu^2 - 3/2 u.u))      (deviation form)
    //   S_i    = (1 - omega/2) w_i (3 (c_i.F - u.F) + 9 cu (c_i.F)),  cu = c_i.u
    // taken per pair (i, opp(i)): the parts even in c_i are shared by the
    // pair, the odd parts change sign.  The relaxation acts on f - f_eq:
    // written as (1 - omega) f + omega f_eq, the rounding of 1 - omega
    // (omega near 2) leaves (1 - omega) + omega != 1 in the momentum sum, a
    // bias of ulp(1) * rho u per step that the FP32 path accumulated to
    // 1e-4 of u within 1000 steps (the body force is ~1e-8 per step).
    const T uu = ux * ux + uy * uy + uz * uz;
    const T fpref = (T)1 - (T)0.5 * omega;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    // r = rho u - (j + F/2): the first moment the equilibrium carries minus
    // the one eq. 5 gives it, exact to the rounding of a small number.  The
    // half-force shift is a few ulp of j in FP32, so the rounding of u is
    // the same at every step and would bias the momentum input by up to a
    // tenth of the body force per step; the source removes omega r.
    const T rx = fma(rho, ux, -jx) - (T)0.5 * Fx, ry = fma(rho, uy, -jy) - (T)0.5 * Fy;
    const T rz = D == 3 ? fma(rho, uz, -jz) - (T)0.5 * Fz : (T)0;
    // odd part of the source per unit weight: 3 c_i . G, G = (1 - omega/2) F - omega r
    const T Gx = (T)3 * (fpref * Fx - omega * rx), Gy = (T)3 * (fpref * Fy - omega * ry);
    const T Gz = (T)3 * (fpref * Fz - omega * rz);
    // per unit weight: the c-independent parts of f_eq and of S
    const T e0 = drho - (T)1.5 * rho * uu;
    const T s0 = (T)-3 * fpref * uF;
    const T r45 = (T)4.5 * rho, r3 = (T)3 * rho;
    const T f9 = (T)9 * fpref;
    {
        const T w0 = (T)wgt<Q>(0);
        const T e = SH ? w0 * e0 - K.sfe[0] : w0 * e0;
        f[0] = (f[0] - omega * (f[0] - e)) + w0 * s0;
    }
    sfor<(Q - 1) / 2>([&](auto kc) {
        constexpr int i = 2 * decltype(kc)::value + 1, io = opp<Q>(i);
        static_assert(io == i + 1, "pairs (2k+1, 2k+2)");
        const T w = (T)wgt<Q>(i);
        const T cu = (T)cx<Q>(i) * ux + (T)cy<Q>(i) * uy + (T)cz<Q>(i) * uz;
        T E = w * (e0 + r45 * (cu * cu)), O = (w * r3) * cu;   // f_eq = E +- O
        if constexpr (SH) {
            E -= K.sfe[decltype(kc)::value + 1];
            O -= K.sfo[decltype(kc)::value + 1];
        }
        const T Se = w * s0 + (f9 * K.cf[i]) * cu;                     // S = Se +- So
        const T So = w * ((T)cx<Q>(i) * Gx + (T)cy<Q>(i) * Gy + (T)cz<Q>(i) * Gz);
        const T ti = f[i] - (E + O), tio = f[io] - (E - O);
        f[i] = (f[i] - omega * ti) + (Se + So);
        f[io] = (f[io] - omega * tio) + (Se - So);
    });
}

// ---------------------------------------------------------------------------
// finish: HRFD reconstruction (wall cells), moments, collision, AA store,
// velocity, wall density and the Spalart-Allmaras update of one cell.
// rd: ping-pong index of u^{n-1} / nu_tilde^n; results go to rd ^ 1.
// ---------------------------------------------------------------------------
template <int Q, typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool CMC, bool XS = false, bool IBB = false,
          bool RED = false, bool INT = false>
__device__ __forceinline__ T finish(const KP &P, const Cell &C, int rd, T *f, S *lds = nullptr, RedAcc *ra = nullptr)
{
    constexpr int D = Lat<Q>::D;
    using SS = Stor<S>;
    const int nx = P.nx;
    const int64_t N = P.ncell;
    const int x = C.x, y = C.y, z = C.z;
    const bool bottom = C.bottom, top = C.top;
    const int64_t cell = C.cell, wi = C.wi, sy = C.sy;
    S *__restrict__ A = (S *)P.pops;
    const T *__restrict__ u_rd = (const T *)P.u[rd];
    T *__restrict__ u_wr = (T *)P.u[rd ^ 1];
    const T *__restrict__ nt_rd = (const T *)P.nt[rd];
    const CellK<T> &K = ck<T>(P);
    const T nt0 = P.sa_on ? nt_rd[cell] : (T)0;

    // ---- HRFD: regularized reconstruction at the wall cells (D2Q9) --------
    if (HRFD && wi >= 0) {
        const int side = bottom ? -1 : 1;  // outward normal n = (0, side)
        T spar = f[0] + f[1] + f[2];
        T sperp = side < 0 ? (f[4] + f[6] + f[7]) : (f[3] + f[5] + f[8]);
        const T rhoB = (T)P.rho0 + spar + (T)2 * sperp;  // eq. 23 with u_B . n = 0
        const T tx = (T)P.tdir[wi];
        const T ubwf = (T)P.ubwf[wi];
        const T uBx = ubwf * tx;
        const int64_t F = cell - side * sy, FF = cell - 2 * side * sy;
        const T uFt = u_rd[F] * tx, uFFt = u_rd[FF] * tx;  // t = (tx, 0)
        const T gfd = ((T)-3 * ubwf + (T)4 * uFt - uFFt) * (T)0.5;            // eq. 28
        const T G = (T)P.beta * (T)P.gan[wi] + ((T)1 - (T)P.beta) * gfd;     // eq. 27
        // tangential derivative of the wall-function u_x along the wall
        int64_t wl = -1, wr = -1;
        if (P.flow == FLOW_CHANNEL) {
            const int xl = x == 0 ? nx - 1 : x - 1, xr = x == nx - 1 ? 0 : x + 1;
            wl = wall_index(P, xl, y, z);
            wr = wall_index(P, xr, y, z);
        } else {
            wl = x - 1 >= P.plate_start ? wi - 1 : -1;
            wr = x + 1 < nx ? wi + 1 : -1;
        }
        T dudx = 0;
        if (wl >= 0 && wr >= 0)
            dudx = ((T)(P.ubwf[wr] * P.tdir[wr]) - (T)(P.ubwf[wl] * P.tdir[wl])) * (T)0.5;
        else if (wr >= 0)
            dudx = (T)(P.ubwf[wr] * P.tdir[wr]) - uBx;
        else if (wl >= 0)
            dudx = uBx - (T)(P.ubwf[wl] * P.tdir[wl]);
        // S_xy = G t_x n'_y / 2 with the inward normal n' = (0, -side)
        const T Sxy = (T)0.5 * G * tx * (T)(-side);
        const T Sxx = dudx, Syy = -dudx;
        const T nutB = P.sa_on ? nut_of<T>(P, nt0) : (T)0;
        const T tauB = (T)0.5 + (T)3 * ((T)P.nu + nutB);
        const T uu = uBx * uBx;
        sfor<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const T ccx = (T)cx<Q>(i), ccy = (T)cy<Q>(i);
            const T cu = ccx * uBx;
            const T w = (T)wgt<Q>(i);
            const T feqd = w * ((rhoB - (T)P.rho0) + rhoB * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu));
            const T QS = (ccx * ccx - (T)(1.0 / 3.0)) * Sxx + (ccy * ccy - (T)(1.0 / 3.0)) * Syy + (T)2 * ccx * ccy * Sxy;
            f[i] = feqd - w * rhoB * tauB * (T)3 * QS;  // eq. 26, deviation form
        });
    }

    // ---- moments (eq. 4-5) ------------------------------------------------
    T drho = 0, jx = 0, jy = 0, jz = 0;
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        drho += f[i];
        if constexpr (cx<Q>(i) > 0) jx += f[i];
        if constexpr (cx<Q>(i) < 0) jx -= f[i];
        if constexpr (cy<Q>(i) > 0) jy += f[i];
        if constexpr (cy<Q>(i) < 0) jy -= f[i];
        if constexpr (cz<Q>(i) > 0) jz += f[i];
        if constexpr (cz<Q>(i) < 0) jz -= f[i];
    });
    // FOLD (interior rows, BGK, 16-bit storage): f holds the stored values
    // f - soff; the moments add the offsets' sums, and the collision relaxes
    // the stored values towards f_eq - soff, which leaves f* - soff to be
    // stored.  It saves two additions per population where the instruction
    // issue bounds the step; FP32 and FP64 keep the plain order of operations.
    constexpr bool FOLD = INT && !CMC && sizeof(S) == 2;
    if (FOLD && P.shifted) {
        drho += K.ssum;
        jx += K.sj[0];
        jy += K.sj[1];
        jz += K.sj[2];
    }
    const T rho = K.rho0 + drho;
    const T Fx = K.fx, Fy = K.fy, Fz = K.fz;
    const T inv = Num<T>::rcp(rho);
    const T ux = (jx + (T)0.5 * Fx) * inv, uy = (jy + (T)0.5 * Fy) * inv, uz = D == 3 ? (jz + (T)0.5 * Fz) * inv : (T)0;

    // ---- collision with tau_eff = 1/2 + (nu + nu_t)/cs2 -------------------------
    const T nut = P.sa_on ? nut_of<T>(P, nt0) : (T)0;
    const T omega = Num<T>::rcp((T)0.5 + (T)3 * (K.nu + nut));
    if constexpr (CMC) {
        // central-moment operator, eq. 7
        const T uvec[3] = {ux, uy, uz}, Fv[3] = {Fx, Fy, Fz};
        cm_collide<Q, T>(f, drho, rho, uvec, Fv, omega);
    } else {
        bgk_collide<Q, T, FOLD>(K, f, drho, rho, ux, uy, uz, jx, jy, jz, omega);
    }
    // post-collision populations of a wall cell for its interpolated links
    if (IBB && P.bb_interp != IBB_HALFWAY && wi >= 0)
        sfor<Q>([&](auto ic) { P.ibuf[wi * Q + decltype(ic)::value] = (double)f[decltype(ic)::value]; });
    // ---- store (AA pattern) ---------------------------------------------------
    // Odd step: the store addresses are recomputed here from the cell's base
    // and offsets, hidden from the compiler by an empty asm, instead of being
    // kept from the gather (19 live 64-bit addresses across the collision):
    // fewer VGPRs, more waves per SIMD.  (On the even step the store slots are
    // the gather's own and the occupancy is already higher.)
    Cell Cs = C;
    if (ODD) asm volatile("" : "+v"(Cs.pb), "+v"(Cs.oxm), "+v"(Cs.oxp), "+v"(Cs.ozm), "+v"(Cs.ozp));
    const int64_t pbs = Cs.pb;
    // staged pushes: the block's columns [x - tid, x - tid + xs_lim) lie in the
    // row, so a push to block column t stays in the row iff 0 <= t < xs_lim
    const int xs_lim = XS ? min(BLK, nx - (x - (int)threadIdx.x)) : 0;
    if (!FOLD && P.shifted) sfor<Q>([&](auto ic) { f[decltype(ic)::value] -= K.soff[decltype(ic)::value]; });
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ccxi = cx<Q>(i), ccyi = cy<Q>(i), cczi = cz<Q>(i);
        constexpr int io = opp<Q>(i), im = mir<Q>(i);
        const T fp = f[i];
        // even step: own slot opp(i); odd step: the neighbour's slot i, or the
        // own free slot opp(i) for a population leaving through a wall or an
        // open boundary, or the mirrored destination across a symmetry plane
        // (index selected, store unconditional)
        int64_t idx = pbs + io * nx;
        if (ODD) {
            const bool xopen = PLATE && ((ccxi > 0 && x == nx - 1) || (ccxi < 0 && x == 0));
            const bool ycross = (ccyi < 0 && bottom) || (ccyi > 0 && top);
            const bool wall = top ? (P.flow == FLOW_CHANNEL) : bottom_is_wall(P, x, ccxi);
            if (!xopen)
                idx = !ycross ? pbs + i * nx + poff<Q>(Cs, ccxi, ccyi, cczi)
                              : (wall ? pbs + io * nx : pbs + im * nx + poff<Q>(Cs, ccxi, 0, cczi));
            if constexpr (XS && ccxi != 0) {
                const int t = (int)threadIdx.x + ccxi;
                if (!ycross && (unsigned)t < (unsigned)xs_lim) {
                    lds[xslot<Q>(i) * BLK + t] = SS::st(fp);
                    return;
                }
                // a push across the block's edge writes one value of a line
                // the neighbouring block fills: an ordinary (not streaming)
                // store lets L2 merge the two parts (measured 2 % faster)
                if (!ycross) {
                    A[idx] = SS::st(fp);
                    return;
                }
            }
        }
        st_pop(&A[idx], SS::st(fp));
    });
    u_wr[cell] = ux;
    u_wr[N + cell] = uy;
    if (D == 3) u_wr[2 * N + cell] = uz;
    if (wi >= 0) P.wrho[wi] = (double)rho;
    if constexpr (RED) {
        T *__restrict__ us = (T *)P.usnap;
        const T uv[3] = {ux, uy, uz};
        const double rhod = (double)rho;
        double du2 = 0.0, uu = 0.0;
        bool bad = !(rhod > 0.0) || !isfinite(rhod);
        ra->v[0] = (double)drho;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double ua = (double)uv[a], d = ua - (double)us[a * N + cell];
            us[a * N + cell] = uv[a];
            ra->v[1 + a] = rhod * ua;
            uu += ua * ua;
            du2 += d * d;
            bad = bad || !isfinite(ua);
        }
        ra->v[4] = du2;
        ra->v[5] = uu;
        ra->v[6] = bad ? 1.0 : 0.0;
    }

    // ---- Spalart-Allmaras update from nu_tilde^n and u^{n-1} -------------------
    // (the staged odd step runs it after its staged stores: cell_update)
    if (!XS) sa_cell<Q, T, PLATE>(P, C, rd, nt0);
    return nt0;
}

// ---------------------------------------------------------------------------
// cell_update: one fused LBM-RANS step of the cell (x, y, z) by one thread of
// a BLK-thread block.  Plate blocks must be aligned to the right end of a row
// (columns nx-2 and nx-1 in one block) for the outlet exchange through LDS.
// ---------------------------------------------------------------------------
// IBB: interpolated bounce-back links may be present (else the halfway rule
// is compiled in alone, keeping the common kernels lean).
template <int Q, typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool CMC, bool XS = false, bool IBB = false,
          bool RED = false, bool INT = false>
__device__ __forceinline__ void cell_update(const KP &P, int rd, int x, int y, int z, bool active, RedAcc *ra = nullptr)
{
    const int nx = P.nx;
    const int tid = threadIdx.x;
    const Cell C = make_cell<Q, PLATE, INT>(P, x, y, z, active);
    if constexpr (XS) {
        // a block covers columns [x - tid, x - tid + BLK) of one row.  The
        // FP32 D3Q19 odd step runs fastest at four blocks per CU (fewer
        // neighbour-row streams in flight: 0.8 % faster at 512x256x256 and
        // 1.5 % at 768x384x384 than at five, while three are slower); its
        // staging array is sized so that LDS holds the CU at four.
        constexpr int lds_rows = (Q == 19 && sizeof(S) == 4) ? 2 : 1;
        __shared__ S lds[nxdirs<Q>() * BLK * lds_rows];
        T f[Q];
        T nt0 = 0;
        if (active) {
            gather<Q, S, T, ODD, PLATE, HRFD, IBB, INT && !CMC && sizeof(S) == 2>(P, C, f);
            if constexpr (IBB && !HRFD) ibb_links<Q, T, false>(P, C, f);
            nt0 = finish<Q, S, T, ODD, PLATE, HRFD, CMC, true, IBB, false, INT>(P, C, rd, f, lds);
        }
        __syncthreads();
        S *__restrict__ A = (S *)P.pops;
        const int xs_lim = min(BLK, nx - (x - tid));  // the block's columns in the row
        sfor<Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int ccx = cx<Q>(i), ccy = cy<Q>(i), ccz = cz<Q>(i);
            if constexpr (ccx != 0) {
                const bool ycross = (ccy < 0 && C.bottom) || (ccy > 0 && C.top);
                const int src = tid - ccx;  // thread that staged column x
                if (active && !ycross && (unsigned)src < (unsigned)xs_lim)
                    st_pop(&A[C.pb + i * nx + poff<Q>(C, 0, ccy, ccz)], lds[xslot<Q>(i) * BLK + tid]);
            }
        });
        // the SA update after the staged stores: they leave the block sooner
        // (odd step 2 % faster than with the update before the barrier)
        if (active) sa_cell<Q, T, PLATE>(P, C, rd, nt0);
        return;
    }
    T f[Q];
    if (active) gather<Q, S, T, ODD, PLATE, HRFD, IBB, INT && !CMC && sizeof(S) == 2>(P, C, f);
    if constexpr (IBB && !HRFD)
        if (active && (!PLATE || x != nx - 1)) ibb_links<Q, T, PLATE>(P, C, f);
    if (PLATE) {
        // outlet: unknown populations copied from column nx-2 (through LDS)
        __shared__ T xch[3][BLK];
        if (active && x == nx - 2) {
            xch[0][tid] = f[2];
            xch[1][tid] = f[6];
            xch[2][tid] = f[8];
        }
        __syncthreads();
        if (active && x == nx - 1) {
            f[2] = xch[0][tid - 1];
            f[6] = xch[1][tid - 1];
            f[8] = xch[2][tid - 1];
            if constexpr (IBB && !HRFD) ibb_links<Q, T, PLATE>(P, C, f);
        }
        if (active && x == 0) zou_he(P, f);
    }
    if (!active) return;
    finish<Q, S, T, ODD, PLATE, HRFD, CMC, false, IBB, RED, INT>(P, C, rd, f, nullptr, ra);
}

// plate mapping: rows aligned to the right end, nseg blocks per row
__device__ __forceinline__ void plate_block(int nx, int64_t b, int tid, int &x, int &y)
{
    const int nseg = (nx + BLK - 1) / BLK;
    const int row = (int)(b / nseg), seg = (int)(b - (int64_t)row * nseg);
    x = nx - (nseg - seg) * BLK + tid;
    y = row;
}

// ---------------------------------------------------------------------------
// k_step: one fused LBM-RANS step, one thread per cell.  RED (even channel
// steps that end a reduction interval): each block also writes its FP64
// partial sums of slots 0-6 to P.partials[blockIdx.x].
// ---------------------------------------------------------------------------
// One cell update of k_step; XS: the staged odd step of the row mapping;
// INT: the block's row is interior (known per block).
template <int Q, typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool CMC, bool IBB, bool RED, bool XS,
          bool INT>
__device__ __forceinline__ void step_cell(const KP &P, int rd, int x, int y, int z, bool active)
{
    if constexpr (RED) {
        RedAcc ra = {};
        cell_update<Q, S, T, ODD, PLATE, HRFD, CMC, false, IBB, true, INT>(P, rd, x, y, z, active, &ra);
        __shared__ double sh[7][BLK];
        block_sum<BLK>(sh, ra.v, 7);
        if (threadIdx.x == 0)
            for (int k = 0; k < 7; ++k) P.partials[(int64_t)blockIdx.x * NRED + k] = sh[k][0];
    } else {
        cell_update<Q, S, T, ODD, PLATE, HRFD, CMC, XS, IBB, false, INT>(P, rd, x, y, z, active);
    }
}

// With 16-bit storage the step is limited by instruction issue more than by
// HBM, and five waves per SIMD (at most 96 VGPRs) beat four; FP32 and FP64
// keep the compiler's register allocation (five waves cost FP32 4 %).
template <int Q, typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool CMC, bool IBB, bool RED = false>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 2 ? 5 : 1, 8)))
k_step(KP P, int rd)
{
    static_assert(!RED || (!ODD && !PLATE), "the fused reduction is built for even channel steps");
    constexpr bool XS = ODD && !PLATE && LBM_XSTAGE;
    const int nx = P.nx, ny = P.ny;
    const int64_t N = P.ncell;
    const int tid = threadIdx.x;
    int x, y, z;
    bool active;
    if (!PLATE && P.rowmap) {
        // XCD k (hardware block b -> XCD b % 8) owns the rows y in
        // [k ny/8, (k+1) ny/8) for every z, walked z-major: the z+-1 and y+-1
        // neighbours of the SA stencil are then a few rows apart in one L2.
        // A block covers BLK consecutive columns of one row, so whether the
        // row is a wall row is known per block.
        const uint32_t b = blockIdx.x, xcd = b & 7u, l = b >> 3;
        const uint32_t nseg = (uint32_t)((nx + BLK - 1) / BLK), rows = (uint32_t)ny >> 3;
        const uint32_t seg = l % nseg, r = l / nseg;
        y = (int)(xcd * rows + r % rows);
        z = (int)(r / rows);
        x = (int)(seg * BLK) + tid;
        active = x < nx;
        if (y != 0 && y != ny - 1)
            step_cell<Q, S, T, ODD, PLATE, HRFD, CMC, IBB, RED, XS, true>(P, rd, x, y, z, active);
        else
            step_cell<Q, S, T, ODD, PLATE, HRFD, CMC, IBB, RED, XS, false>(P, rd, x, y, z, active);
        return;
    }
    if (!PLATE) {
        const int64_t cell = xcd_block(blockIdx.x, gridDim.x) * BLK + tid;
        active = cell < N;
        const int64_t r = cell / nx;
        x = (int)(cell - r * nx);
        y = (int)(r % ny);
        z = (int)(r / ny);
    } else {
        // rows aligned to the right end so that columns nx-2 and nx-1 share a block
        plate_block(nx, blockIdx.x, tid, x, y);
        z = 0;
        active = x >= 0;
    }
    // (the staged store needs the row mapping)
    step_cell<Q, S, T, ODD, PLATE, HRFD, CMC, IBB, RED, false, false>(P, rd, x, y, z, active);
}

// ---------------------------------------------------------------------------
// k_wall: wall function at every wall cell from u^n (buffer wr); writes the
// Dirichlet nu_tilde_B into nu_tilde buffer wr.
// ---------------------------------------------------------------------------
template <int D, typename T> __device__ __forceinline__ void wall_cell(const KP &P, int64_t w, int wr)
{
    const int nx = P.nx, ny = P.ny;
    const int64_t N = P.ncell, sy = nx;
    int x, z, side;
    if (P.flow == FLOW_CHANNEL) {
        const int64_t per = (int64_t)nx * P.nz;
        side = w < per ? -1 : 1;
        const int64_t r = w < per ? w : w - per;
        x = (int)(r % nx);
        z = (int)(r / nx);
    } else {
        side = -1;
        x = P.plate_start + (int)w;
        z = 0;
    }
    const int yrow = side < 0 ? 0 : ny - 1;
    const int64_t B = x + (int64_t)nx * (yrow + (int64_t)ny * z);
    const int64_t F = B - side * sy;
    const T *u = (const T *)P.u[wr];
    const double uFx = (double)u[F], uFz = D == 3 ? (double)u[2 * N + F] : 0.0;
    const double uBx = (double)u[B], uBz = D == 3 ? (double)u[2 * N + B] : 0.0;
    const double ut = sqrt(uFx * uFx + uFz * uFz);
    double tx = 1.0, tz = 0.0;
    if (ut > 0.0) {
        tx = uFx / ut;
        tz = uFz / ut;
    }
    // B and F sit d_w and 1 + d_w from the wall (Sec. 3.1; d_w = 1/2 halfway)
    const double yB = P.wall_dist, yF = 1.0 + P.wall_dist;
    const double utau = solve_utau(P, ut, yF, P.utau[w]);
    const double yBp = yB * utau / P.nu;
    double uw[3] = {0.0, 0.0, 0.0};
    if (P.scheme == WALL_FIXED) {
        const double *s = side < 0 ? P.wall_u_bottom : P.wall_u_top;
        uw[0] = s[0];
        uw[1] = s[1];
        uw[2] = s[2];
    } else if (P.scheme == WALL_SLIP) {
        // eq. 35 with nu_t|B = nu kappa y_B+ and Delta_w = y_B
        const double s = utau * utau * yB / (P.nu * (1.0 + P.kappa * yBp));
        uw[0] = uBx - s * tx;
        uw[2] = uBz - s * tz;
    } else {
        P.ubwf[w] = utau * uplus(P, yBp);
        if (P.scheme == WALL_CD) {
            // eq. 29 with Delta = 1: third-order one-sided difference of the law
            const double dp = utau / P.nu;
            P.gan[w] = utau * ((-11.0 / 6.0) * uplus(P, yBp) + 3.0 * uplus(P, yBp + dp) -
                               1.5 * uplus(P, yBp + 2.0 * dp) + (1.0 / 3.0) * uplus(P, yBp + 3.0 * dp));
        } else {
            P.gan[w] = utau * utau / P.nu * duplus(P, yBp);
        }
    }
    P.utau[w] = utau;
    P.tdir[w] = tx;
    P.tdir[P.nwall + w] = 0.0;
    P.tdir[2 * P.nwall + w] = tz;
    P.uw[w] = uw[0];
    P.uw[P.nwall + w] = uw[1];
    P.uw[2 * P.nwall + w] = uw[2];
    if (P.sa_on) ((T *)P.nt[wr])[B] = (T)(P.nu * P.kappa * yBp);
}

template <int D, typename T> __global__ void __launch_bounds__(BLK) k_wall(KP P, int wr)
{
    const int64_t w = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (w < P.nwall) wall_cell<D, T>(P, w, wr);
}

// ---------------------------------------------------------------------------
// Canonical post-collision population f*_i(x) (deviation) of the last step.
// odd_state: the last step was odd (pushed layout).
// ---------------------------------------------------------------------------
template <int Q, int i, typename S, typename T>
__device__ __forceinline__ T canon_raw(const KP &P, const S *A, int x, int y, int z, int64_t cell, bool odd_state);

// population i of the last step as a deviation f_i - w_i rho0
template <int Q, int i, typename S, typename T>
__device__ __forceinline__ T canon_f(const KP &P, const S *A, int x, int y, int z, int64_t cell, bool odd_state)
{
    T v = canon_raw<Q, i, S, T>(P, A, x, y, z, cell, odd_state);
    if (P.shifted) v += ck<T>(P).soff[i];
    return v;
}

template <int Q, int i, typename S, typename T>
__device__ __forceinline__ T canon_raw(const KP &P, const S *A, int x, int y, int z, int64_t cell, bool odd_state)
{
    using SS = Stor<S>;
    constexpr int io = opp<Q>(i), im = mir<Q>(i);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int64_t row = y + (int64_t)ny * z;
    if (!odd_state) return SS::ld(A[pidx<Q>(nx, io, x, row)]);
    constexpr int ccx = cx<Q>(i), ccy = cy<Q>(i), ccz = cz<Q>(i);
    const bool plate = P.flow == FLOW_PLATE;
    const bool xopen = plate && ((ccx > 0 && x == nx - 1) || (ccx < 0 && x == 0));
    const bool ycross = (ccy < 0 && y == 0) || (ccy > 0 && y == ny - 1);
    if (xopen) return SS::ld(A[pidx<Q>(nx, io, x, row)]);
    int xd = x + ccx, zd = z + ccz;
    if (!plate) xd = (xd + nx) % nx;
    zd = (zd + nz) % nz;
    if (!ycross) return SS::ld(A[pidx<Q>(nx, i, xd, y + ccy + (int64_t)ny * zd)]);
    const bool wall = (y == ny - 1 && ccy > 0) ? (P.flow == FLOW_CHANNEL) : bottom_is_wall(P, x, ccx);
    if (wall) return SS::ld(A[pidx<Q>(nx, io, x, row)]);
    return SS::ld(A[pidx<Q>(nx, im, xd, y + (int64_t)ny * zd)]);
}

template <int Q, typename S, typename T> __global__ void __launch_bounds__(BLK) k_export_f(KP P, bool odd_state, double *out)
{
    const int64_t cell = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (cell >= P.ncell) return;
    const int64_t r = cell / P.nx;
    const int x = (int)(cell - r * P.nx), y = (int)(r % P.ny), z = (int)(r / P.ny);
    const S *A = (const S *)P.pops;
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        out[i * P.ncell + cell] = (double)canon_f<Q, i, S, T>(P, A, x, y, z, cell, odd_state) + wgt<Q>(i) * P.rho0;
    });
}

// rho (eq. 4, summed in double), u (the stored eq. 5 velocity) and nu_t
// (eq. 10) of the last step, converted to the output type O.
template <int Q, typename S, typename T, typename O>
__global__ void __launch_bounds__(BLK) k_export_moments(KP P, bool odd_state, int cur, O *rho, O *u, O *nut)
{
    constexpr int D = Lat<Q>::D;
    const int64_t cell = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (cell >= P.ncell) return;
    const int64_t N = P.ncell;
    if (rho) {
        const int64_t r = cell / P.nx;
        const int x = (int)(cell - r * P.nx), y = (int)(r % P.ny), z = (int)(r / P.ny);
        const S *A = (const S *)P.pops;
        double s = 0.0;
        sfor<Q>([&](auto ic) { s += (double)canon_f<Q, decltype(ic)::value, S, T>(P, A, x, y, z, cell, odd_state); });
        rho[cell] = (O)(P.rho0 + s);
    }
    if (u) {
        const T *uc = (const T *)P.u[cur];
        for (int a = 0; a < D; ++a) u[a * N + cell] = (O)uc[a * N + cell];
    }
    if (nut) {
        const T nt = ((const T *)P.nt[cur])[cell];
        nut[cell] = P.sa_on ? (O)nut_of<T>(P, nt) : (O)0;
    }
}

template <typename T> __global__ void __launch_bounds__(BLK) k_export_nt(KP P, int cur, double *out)
{
    const int64_t cell = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (cell >= P.ncell) return;
    out[cell] = (double)((const T *)P.nt[cur])[cell];
}

// ---------------------------------------------------------------------------
// Initialisation: f*_i = f_eq(rho0, u0) in the even layout, u^0 = u0,
// nu_tilde = ratio * nu.  u0: device doubles (D*ncell) or NULL (uniform).
// ---------------------------------------------------------------------------
template <int Q, typename S, typename T>
__global__ void __launch_bounds__(BLK) k_init(KP P, const double *u0, double ux0, double uy0, double uz0, double ntinit)
{
    constexpr int D = Lat<Q>::D;
    using SS = Stor<S>;
    const int64_t cell = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (cell >= P.ncell) return;
    const int64_t N = P.ncell;
    double u[3] = {ux0, uy0, D == 3 ? uz0 : 0.0};
    if (u0)
        for (int a = 0; a < D; ++a) u[a] = u0[a * N + cell];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    S *A = (S *)P.pops;
    const int64_t row = cell / P.nx;
    const int x = (int)(cell - row * P.nx);
    // the wall cells' previous post-collision populations (interpolated links)
    const int64_t wi = P.bb_interp != IBB_HALFWAY ? wall_index(P, x, (int)(row % P.ny), (int)(row / P.ny)) : -1;
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const double cu = cx<Q>(i) * u[0] + cy<Q>(i) * u[1] + cz<Q>(i) * u[2];
        const double fd = wgt<Q>(i) * P.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        A[pidx<Q>(P.nx, opp<Q>(i), x, row)] = SS::st((T)fd - ck<T>(P).soff[i]);
        if (wi >= 0) P.ibuf[wi * Q + i] = fd;
    });
    T *u_0 = (T *)P.u[0], *us = (T *)P.usnap;
    for (int a = 0; a < D; ++a) {
        u_0[a * N + cell] = (T)u[a];
        us[a * N + cell] = (T)u[a];
    }
    ((T *)P.nt[0])[cell] = (T)ntinit;
    ((T *)P.nt[1])[cell] = (T)ntinit;
    if (cell == 0) P.result[RES_STICKY] = 0.0;
}

__global__ void k_init_wall(KP P)
{
    const int64_t w = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (w >= P.nwall) return;
    P.utau[w] = 0.0;
    P.wrho[w] = P.rho0;
    P.ubwf[w] = 0.0;
    P.gan[w] = 0.0;
    for (int a = 0; a < 3; ++a) {
        P.tdir[a * P.nwall + w] = a == 0 ? 1.0 : 0.0;
        P.uw[a * P.nwall + w] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Reduction: per-block FP64 partials in a fixed tree order, then one block.
// slots: 0 sum(rho - rho0), 1-3 sum(rho u), 4 sum |u - usnap|^2, 5 sum |u|^2,
// 6 bad-value count.
// ---------------------------------------------------------------------------

// Block b of nb: FP64 partial sums (slots 0-7) over its share of the cells,
// written to P.partials[b]; the velocity snapshot is refreshed on the way.
template <int Q, typename S, typename T> __device__ __forceinline__ void reduce_part(const KP &P, bool odd_state, int cur, int b, int nb)
{
    constexpr int D = Lat<Q>::D;
    __shared__ double sh[8][BLK];
    const int64_t N = P.ncell;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const S *A = (const S *)P.pops;
    const T *uc = (const T *)P.u[cur];
    T *us = (T *)P.usnap;
    for (int64_t cell = (int64_t)b * BLK + threadIdx.x; cell < N; cell += (int64_t)nb * BLK) {
        const int64_t r = cell / P.nx;
        const int x = (int)(cell - r * P.nx), y = (int)(r % P.ny), z = (int)(r / P.ny);
        double drho = 0.0;
        sfor<Q>([&](auto ic) { drho += (double)canon_f<Q, decltype(ic)::value, S, T>(P, A, x, y, z, cell, odd_state); });
        const double rho = P.rho0 + drho;
        double uu = 0.0, du = 0.0;
        bool bad = !(rho > 0.0) || !isfinite(rho);
        for (int a = 0; a < D; ++a) {
            const double ua = (double)uc[a * N + cell];
            const double d = ua - (double)us[a * N + cell];
            us[a * N + cell] = uc[a * N + cell];
            acc[1 + a] += rho * ua;
            uu += ua * ua;
            du += d * d;
            bad = bad || !isfinite(ua);
        }
        acc[0] += drho;
        acc[4] += du;
        acc[5] += uu;
        acc[6] += bad ? 1.0 : 0.0;
    }
    // slot 7: this block's share of the wall cells' u_tau
    for (int64_t w = (int64_t)b * BLK + threadIdx.x; w < P.nwall; w += (int64_t)nb * BLK)
        acc[7] += P.utau[w];
    block_sum<BLK>(sh, acc, 8);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) P.partials[b * NRED + k] = sh[k][0];
}

template <int Q, typename S, typename T> __global__ void __launch_bounds__(BLK) k_reduce(KP P, bool odd_state, int cur)
{
    reduce_part<Q, S, T>(P, odd_state, cur, blockIdx.x, gridDim.x);
}

// Middle pass of a lattice's reduction: block b of MID_BLOCKS sums its fixed
// slice of the nrows partial rows (slots 0-6, written by k_reduce or by a
// fused k_step) and of the wall cells' u_tau (slot 7) into P.mid[b].
__global__ void __launch_bounds__(BLK) k_reduce_mid(KP P, int64_t nrows)
{
    __shared__ double sh[8][BLK];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t b = blockIdx.x;
    const int64_t rper = (nrows + MID_BLOCKS - 1) / MID_BLOCKS, wper = (P.nwall + MID_BLOCKS - 1) / MID_BLOCKS;
    const int64_t r1 = std::min(nrows, (b + 1) * rper), w1 = std::min(P.nwall, (b + 1) * wper);
    for (int64_t r = b * rper + threadIdx.x; r < r1; r += BLK)
        for (int k = 0; k < 7; ++k) acc[k] += P.partials[r * NRED + k];
    for (int64_t w = b * wper + threadIdx.x; w < w1; w += BLK) acc[7] += P.utau[w];
    block_sum<BLK>(sh, acc, 8);
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) P.mid[b * NRED + k] = sh[k][0];
}

// Last pass: the MID_BLOCKS rows of P.mid into result slot `slot`; the sticky
// divergence flag P.result[RES_STICKY] is raised when this reduction saw a
// bad cell.
__global__ void __launch_bounds__(BLK) k_reduce_final(KP P, int slot)
{
    __shared__ double sh[8][BLK];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < MID_BLOCKS; b += BLK)
        for (int k = 0; k < 8; ++k) acc[k] += P.mid[b * NRED + k];
    block_sum<BLK>(sh, acc, 8);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 8; ++k) P.result[slot * NRED + k] = sh[k][0];
        const bool bad = sh[6][0] > 0.0 || !isfinite(sh[4][0]) || !isfinite(sh[5][0]);
        if (bad) P.result[RES_STICKY] = 1.0;
    }
}

// ---------------------------------------------------------------------------
// Serving.  Small D2Q9 lattices: a persistent kernel, one workgroup per
// lattice, loops over time steps with barriers between the phases of a step
// (fused cell update, wall function, periodic residual).  Large lattices: each
// phase of a step is one launch over every resident lattice of a kind, a
// table mapping each block to (slot, block of that slot).  Both stop a
// lattice on convergence, divergence or its step cap, on the device, with
// the same cell update code as k_step.
// ---------------------------------------------------------------------------
constexpr int SBLK = 512;
constexpr int SERVE_MAX_NY = 256;  // plate rows held in the outlet exchange buffer
constexpr int MRED = 128;          // reduction blocks per large lattice

enum { SLOT_IDLE = 0, SLOT_RUNNING = 1, SLOT_CONVERGED = 2, SLOT_CAPPED = 3, SLOT_DIVERGED = 4 };

struct SlotDesc {
    KP kp;
    int64_t step;       // steps done (large lattices: at the start of the chunk)
    int64_t max_steps;  // step cap
    int64_t snap_step;  // step of the previous residual snapshot
    int64_t stop_step;  // step at which the lattice stopped
    double tol, residual, mean_utau;
    double tol_utau;         // Delta u_tau / u_tau criterion (0: off)
    double prev_mean_utau;   // mean u_tau at the previous reduction (0: none yet)
    double d_utau_rel;       // its relative change over the last interval (-1: none yet)
    int status, reduce_every, variant, conv_by;  // conv_by: 1 residual, 2 u_tau
};

// residual r = ||u - u_snap|| / (K ||u||), mean u_tau and the stop decision
// from the FP64 sums {du^2, u^2, non-finite count, sum u_tau}; thread 0 only.
// A lattice converges at a reduction step when r < tol, or when the mean
// friction velocity changed by less than tol_utau (relative) since the
// previous reduction (the criterion of Sec. 4.1.1, over the reduction
// interval); conv_by records which.
__device__ __forceinline__ void slot_verdict(SlotDesc &SD, int64_t nwall, int64_t step, double du2, double uu,
                                             double bad, double sutau, bool red_now)
{
    const double K = (double)(step - SD.snap_step);
    const double r = uu > 0.0 ? sqrt(du2) / (K * sqrt(uu)) : 0.0;
    const double mu = nwall > 0 ? sutau / (double)nwall : 0.0;
    const double prev = SD.prev_mean_utau;
    SD.d_utau_rel = prev > 0.0 ? fabs(mu - prev) / prev : -1.0;
    SD.prev_mean_utau = mu;
    SD.residual = r;
    SD.mean_utau = mu;
    SD.snap_step = step;
    if (bad > 0.0 || !isfinite(r) || !isfinite(mu)) {
        SD.status = SLOT_DIVERGED;
    } else if (red_now && r < SD.tol) {
        SD.status = SLOT_CONVERGED;
        SD.conv_by = 1;
    } else if (red_now && SD.tol_utau > 0.0 && SD.d_utau_rel >= 0.0 && SD.d_utau_rel < SD.tol_utau) {
        SD.status = SLOT_CONVERGED;
        SD.conv_by = 2;
    } else if (step >= SD.max_steps) {
        SD.status = SLOT_CAPPED;
    }
    if (SD.status != SLOT_RUNNING) SD.stop_step = step;
}

template <typename S, typename T, bool ODD, bool PLATE, bool HRFD, bool CMC>
__device__ __forceinline__ void serve_cells(const KP &P, int rd, T (*xch)[SERVE_MAX_NY])
{
    const int nx = P.nx;
    const int64_t N = P.ncell;
    if (PLATE) {
        // outlet: the incoming populations of column nx-2 before anyone writes
        for (int y = threadIdx.x; y < P.ny; y += SBLK) {
            const Cell Cn = make_cell<9, true>(P, nx - 2, y, 0, true);
            T g[9];
            gather<9, S, T, ODD, true, HRFD, !HRFD>(P, Cn, g);
            if (!HRFD) ibb_links<9, T, true>(P, Cn, g);
            xch[0][y] = g[2];
            xch[1][y] = g[6];
            xch[2][y] = g[8];
        }
        __syncthreads();
    }
    for (int64_t cell = threadIdx.x; cell < N; cell += SBLK) {
        const int y = (int)(cell / nx), x = (int)(cell - (int64_t)y * nx);
        const Cell C = make_cell<9, PLATE>(P, x, y, 0, true);
        T f[9];
        gather<9, S, T, ODD, PLATE, HRFD, !HRFD>(P, C, f);
        if (!HRFD && (!PLATE || x != nx - 1)) ibb_links<9, T, PLATE>(P, C, f);
        if (PLATE) {
            if (x == nx - 1) {
                f[2] = xch[0][y];
                f[6] = xch[1][y];
                f[8] = xch[2][y];
                if (!HRFD) ibb_links<9, T, PLATE>(P, C, f);
            }
            if (x == 0) zou_he(P, f);
        }
        finish<9, S, T, ODD, PLATE, HRFD, CMC, false, !HRFD>(P, C, rd, f);
    }
}

// P: the lattice's parameters copied to LDS (the descriptor itself is
// written by the kernel, so reading it from global memory would reload every
// field after every store)
template <typename S, typename T, bool PLATE, bool HRFD, bool CMC>
__device__ void serve_loop(SlotDesc &SD, const KP &P, int chunk)
{
    __shared__ T xch[3][SERVE_MAX_NY];
    __shared__ double red[4][SBLK];
    __shared__ int stop;
    int64_t step = SD.step;
    const int64_t N = P.ncell, max_steps = SD.max_steps;
    const int reduce_every = SD.reduce_every;
    if (threadIdx.x == 0) stop = 0;
    __syncthreads();
    for (int s = 0; s < chunk; ++s) {
        const int rd = (int)(step & 1);
        if ((step + 1) & 1)
            serve_cells<S, T, true, PLATE, HRFD, CMC>(P, rd, xch);
        else
            serve_cells<S, T, false, PLATE, HRFD, CMC>(P, rd, xch);
        __syncthreads();
        for (int64_t w = threadIdx.x; w < P.nwall; w += SBLK) wall_cell<2, T>(P, w, rd ^ 1);
        __syncthreads();
        ++step;
        const bool red_now = reduce_every > 0 && step % reduce_every == 0;
        if (red_now || step >= max_steps) {
            const T *uc = (const T *)P.u[step & 1];
            T *us = (T *)P.usnap;
            double acc[4] = {0, 0, 0, 0};
            for (int64_t cell = threadIdx.x; cell < N; cell += SBLK) {
                for (int a = 0; a < 2; ++a) {
                    const double ua = (double)uc[a * N + cell], d = ua - (double)us[a * N + cell];
                    us[a * N + cell] = uc[a * N + cell];
                    acc[0] += d * d;
                    acc[1] += ua * ua;
                    acc[2] += isfinite(ua) ? 0.0 : 1.0;
                }
            }
            for (int64_t w = threadIdx.x; w < P.nwall; w += SBLK) acc[3] += P.utau[w];
            block_sum<SBLK>(red, acc, 4);
            if (threadIdx.x == 0) {
                slot_verdict(SD, P.nwall, step, red[0][0], red[1][0], red[2][0], red[3][0], red_now);
                stop = SD.status != SLOT_RUNNING;
            }
            __syncthreads();
            if (stop) break;
        }
    }
    if (threadIdx.x == 0) SD.step = step;
}

// one workgroup per listed small lattice of one kind (storage, collision,
// flow, wall treatment)
template <typename S, typename T, bool CMC, bool PLATE, bool HRFD>
__global__ void __launch_bounds__(SBLK) k_serve(SlotDesc *slots, const int *list, int chunk)
{
    static_assert(sizeof(KP) % 8 == 0 && sizeof(KP) / 8 <= SBLK, "KP copy");
    __shared__ KP sP;
    SlotDesc &SD = slots[list[blockIdx.x]];
    if (SD.status != SLOT_RUNNING) return;
    if (threadIdx.x < sizeof(KP) / 8) ((int64_t *)&sP)[threadIdx.x] = ((const int64_t *)&SD.kp)[threadIdx.x];
    __syncthreads();
    serve_loop<S, T, PLATE, HRFD, CMC>(SD, sP, chunk);
}

// ---- large lattices: one launch per phase over all lattices of a kind -----
// tab[b] = (slot, block of that slot); s = step within the chunk.
__device__ __forceinline__ bool mslot(const SlotDesc *slots, int slot, int s, int64_t &step)
{
    const SlotDesc &SD = slots[slot];
    step = SD.step + s;
    return SD.status == SLOT_RUNNING && step < SD.max_steps;
}

template <int Q, typename S, typename T, bool ODD, bool CMC>
__device__ __forceinline__ void mstep_body(const KP &P, int rd, int64_t lb)
{
    const int tid = threadIdx.x;
    if (P.flow == FLOW_PLATE) {
        if constexpr (Q == 9) {
            int x, y;
            plate_block(P.nx, lb, tid, x, y);
            if (P.scheme >= WALL_HRFD)
                cell_update<Q, S, T, ODD, true, true, CMC, false, false>(P, rd, x, y, 0, x >= 0);
            else
                cell_update<Q, S, T, ODD, true, false, CMC, false, true>(P, rd, x, y, 0, x >= 0);
        }
        return;
    }
    const int64_t cell = lb * BLK + tid;
    const bool active = cell < P.ncell;
    const int64_t r = active ? cell / P.nx : 0;
    const int x = active ? (int)(cell - r * P.nx) : 0, y = (int)(r % P.ny), z = (int)(r / P.ny);
    if constexpr (Q == 9) {
        if (P.scheme >= WALL_HRFD) {
            cell_update<Q, S, T, ODD, false, true, CMC, false, false>(P, rd, x, y, z, active);
            return;
        }
    }
    cell_update<Q, S, T, ODD, false, false, CMC, false, true>(P, rd, x, y, z, active);
}

template <int Q, typename S, typename T, bool CMC>
__global__ void __launch_bounds__(BLK) k_mstep(const SlotDesc *__restrict__ slots, const int2 *__restrict__ tab, int s)
{
    const int2 e = tab[blockIdx.x];
    int64_t step;
    if (!mslot(slots, e.x, s, step)) return;
    const KP &P = slots[e.x].kp;
    const int rd = (int)(step & 1);
    if ((step + 1) & 1)
        mstep_body<Q, S, T, true, CMC>(P, rd, e.y);
    else
        mstep_body<Q, S, T, false, CMC>(P, rd, e.y);
}

template <int D, typename T> __global__ void __launch_bounds__(BLK) k_mwall(const SlotDesc *__restrict__ slots, const int2 *__restrict__ tab, int s)
{
    const int2 e = tab[blockIdx.x];
    int64_t step;
    if (!mslot(slots, e.x, s, step)) return;
    const KP &P = slots[e.x].kp;
    const int64_t w = (int64_t)e.y * BLK + threadIdx.x;
    if (w < P.nwall) wall_cell<D, T>(P, w, (int)(step & 1) ^ 1);
}

// residual due after step `step` (the cap included)?
__device__ __forceinline__ bool mdue(const SlotDesc &SD, int64_t after, bool &red_now)
{
    red_now = SD.reduce_every > 0 && after % SD.reduce_every == 0;
    return red_now || after >= SD.max_steps;
}

template <int Q, typename S, typename T> __global__ void __launch_bounds__(BLK) k_mreduce(const SlotDesc *__restrict__ slots, const int *__restrict__ list, int s)
{
    const int slot = list[blockIdx.x / MRED], b = blockIdx.x % MRED;
    int64_t step;
    if (!mslot(slots, slot, s, step)) return;
    bool red_now;
    if (!mdue(slots[slot], step + 1, red_now)) return;
    const int cur = (int)((step + 1) & 1);
    reduce_part<Q, S, T>(slots[slot].kp, cur != 0, cur, b, MRED);
}

__global__ void __launch_bounds__(BLK) k_mreduce_final(SlotDesc *slots, const int *list, int s)
{
    const int slot = list[blockIdx.x];
    int64_t step;
    if (!mslot(slots, slot, s, step)) return;
    SlotDesc &SD = slots[slot];
    bool red_now;
    if (!mdue(SD, step + 1, red_now)) return;
    __shared__ double sh[8][BLK];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < MRED; b += BLK)
        for (int k = 0; k < 8; ++k) acc[k] += SD.kp.partials[b * NRED + k];
    block_sum<BLK>(sh, acc, 8);
    // slots: 4 = sum du^2, 5 = sum u^2, 6 = bad cells, 7 = sum u_tau
    if (threadIdx.x == 0) slot_verdict(SD, SD.kp.nwall, step + 1, sh[4][0], sh[5][0], sh[6][0], sh[7][0], red_now);
}

// end of a chunk: steps done by every listed lattice
__global__ void k_mfinish(SlotDesc *slots, const int *list, int n, int chunk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    SlotDesc &SD = slots[list[i]];
    if (SD.status == SLOT_RUNNING) {
        SD.step += chunk;
        if (SD.step > SD.max_steps) SD.step = SD.max_steps;
    } else {
        SD.step = SD.stop_step;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(LBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

int storage_bytes(int precision)
{
    switch (precision) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16: return 2;
    case LBM_BF16: return 2;
    default: return -1;
    }
}

struct Layout {
    int64_t pops, u0, u1, nt0, nt1, usnap, utau, tdir, uw, wrho, ubwf, gan, partials, result, mid, ibuf, total;
};

int64_t nwall_of(int flow, int nx, int nz, int plate_start)
{
    if (flow == LBM_FLOW_CHANNEL) return 2LL * nx * nz;
    int x0 = plate_start < 0 ? 0 : plate_start;
    return nx > x0 ? (int64_t)(nx - x0) : 0;
}

bool make_layout(int Q, int nx, int ny, int nz, const lbm_params_t *p, Layout *L)
{
    const int sb = storage_bytes(p->precision);
    if (sb < 0) return false;
    const int tb = p->precision == LBM_F64 ? 8 : 4;
    const int D = Q == 9 ? 2 : 3;
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t nw = nwall_of(p->flow, nx, nz, p->plate_start);
    int64_t o = 0;
    L->pops = o; o = align256(o + (int64_t)Q * N * sb);
    L->u0 = o; o = align256(o + (int64_t)D * N * tb);
    L->u1 = o; o = align256(o + (int64_t)D * N * tb);
    L->nt0 = o; o = align256(o + N * tb);
    L->nt1 = o; o = align256(o + N * tb);
    L->usnap = o; o = align256(o + (int64_t)D * N * tb);
    L->utau = o; o = align256(o + (nw + 1) * 8);
    L->tdir = o; o = align256(o + 3 * (nw + 1) * 8);
    L->uw = o; o = align256(o + 3 * (nw + 1) * 8);
    L->wrho = o; o = align256(o + (nw + 1) * 8);
    L->ubwf = o; o = align256(o + (nw + 1) * 8);
    L->gan = o; o = align256(o + (nw + 1) * 8);
    // one partial-sum row per block of the standalone reduction or of the step
    // (fused reduction): the larger of the row-mapped and flat grids
    const int64_t step_blocks = std::max((int64_t)ny * nz * ((nx + BLK - 1) / BLK), (N + BLK - 1) / BLK);
    L->partials = o; o = align256(o + std::max((int64_t)RED_BLOCKS, step_blocks) * NRED * 8);
    L->result = o; o = align256(o + 32 * 8);
    L->mid = o; o = align256(o + (int64_t)MID_BLOCKS * NRED * 8);
    L->ibuf = o; o = align256(o + (p->bb_interp != LBM_IBB_HALFWAY ? (int64_t)Q * nw * 8 : 0));
    L->total = o;
    return true;
}

}  // namespace

struct lbm {
    int Q, D, nx, ny, nz;
    lbm_params_t p;
    KP kp;
    Layout L;
    char *base;
    int64_t bytes;
    hipStream_t stream;
    int device;                 // the GPU holding the caller's buffer
    int64_t step;
    int64_t last_reduce_step;   // step of the last reduction (-1: none)
    int64_t prev_reduce_step;
    int reduce_count;
    bool diverged;
    bool timing;
    int timing_every;         // time 2 consecutive steps in every timing_every (1: all)
    bool chain_open;          // the last launch on the stream was followed by an event
    // non-blocking divergence check: the sticky flag of the reductions is
    // copied to pinned host memory after each periodic reduction
    double *flag_host;
    hipEvent_t flag_ev;
    bool flag_pending;
    // One chain of events on the stream; the interval that ends at event k
    // belongs to ev_kind[k] (a k_step or k_wall launch, or nothing timed).
    // One event per launch keeps the instrumentation light.
    std::vector<hipEvent_t> ev;
    std::vector<char> ev_kind;
    size_t n_ev;
    double acc_step_ms, acc_wall_ms;
    int64_t acc_step_n, acc_wall_n;
};

namespace {

template <int Q, typename S, typename T> struct Impl {
    static constexpr int D = Lat<Q>::D;
    // red: the even channel step that ends a reduction interval (fused reduction)
    template <bool PLATE, bool HRFD, bool IBB> static void (*pick(bool odd, bool cm, bool red))(KP, int)
    {
        if constexpr (!PLATE) {
            if (red && !odd)
                return cm ? k_step<Q, S, T, false, PLATE, HRFD, true, IBB, true> : k_step<Q, S, T, false, PLATE, HRFD, false, IBB, true>;
        }
        if (cm) return odd ? k_step<Q, S, T, true, PLATE, HRFD, true, IBB> : k_step<Q, S, T, false, PLATE, HRFD, true, IBB>;
        return odd ? k_step<Q, S, T, true, PLATE, HRFD, false, IBB> : k_step<Q, S, T, false, PLATE, HRFD, false, IBB>;
    }
    template <bool PLATE> static void (*pick_bb(bool odd, bool cm, bool ibb, bool red))(KP, int)
    {
        return ibb ? pick<PLATE, false, true>(odd, cm, red) : pick<PLATE, false, false>(odd, cm, red);
    }
    // launches one step; *nblocks (if given) receives the grid size
    static int step(lbm *h, bool odd, int rd, bool red, int64_t *nblocks)
    {
        const KP &P = h->kp;
        const bool plate = h->p.flow == LBM_FLOW_PLATE;
        const bool hrfd = h->p.scheme >= LBM_WALL_HRFD;
        dim3 grid;
        if (plate || P.rowmap)
            grid = dim3((unsigned)((int64_t)h->ny * h->nz * ((h->nx + BLK - 1) / BLK)));
        else
            grid = dim3((unsigned)((P.ncell + BLK - 1) / BLK));
        const bool cm = h->p.collision == LBM_COLL_CM;
        const bool ibb = h->p.bb_interp != LBM_IBB_HALFWAY;
        red = red && !plate && !odd;
        void (*kern)(KP, int) = nullptr;
        if constexpr (Q == 9) {
            if (plate) {
                if (hrfd) kern = pick<true, true, false>(odd, cm, false);
                else kern = pick_bb<true>(odd, cm, ibb, false);
            } else {
                if (hrfd) kern = pick<false, true, false>(odd, cm, red);
                else kern = pick_bb<false>(odd, cm, ibb, red);
            }
        } else {
            kern = pick_bb<false>(odd, cm, ibb, red);
        }
        if (nblocks) *nblocks = grid.x;
        hipLaunchKernelGGL(kern, grid, dim3(BLK), 0, h->stream, P, rd);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int wall(lbm *h, int wr)
    {
        if (h->kp.nwall == 0) return LBM_OK;
        dim3 grid((unsigned)((h->kp.nwall + BLK - 1) / BLK));
        hipLaunchKernelGGL((k_wall<D, T>), grid, dim3(BLK), 0, h->stream, h->kp, wr);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int init(lbm *h, const double *u0dev)
    {
        dim3 grid((unsigned)((h->kp.ncell + BLK - 1) / BLK));
        const double ntinit = h->p.sa_on ? h->p.nut_init_ratio * h->p.nu : 0.0;
        const double *ui = h->p.u_init;
        hipLaunchKernelGGL((k_init<Q, S, T>), grid, dim3(BLK), 0, h->stream, h->kp, u0dev, ui[0], ui[1], ui[2], ntinit);
        HIPCHK(hipGetLastError());
        if (h->kp.nwall > 0) {
            dim3 gw((unsigned)((h->kp.nwall + BLK - 1) / BLK));
            hipLaunchKernelGGL(k_init_wall, gw, dim3(BLK), 0, h->stream, h->kp);
            HIPCHK(hipGetLastError());
        }
        return wall(h, 0);
    }
    // fused_nb > 0: the step just launched wrote fused_nb partial rows
    static int reduce(lbm *h, bool odd_state, int cur, int slot, int64_t fused_nb)
    {
        int64_t nb = fused_nb;
        if (nb <= 0) {
            nb = std::min((h->kp.ncell + BLK - 1) / BLK, (int64_t)RED_BLOCKS);
            hipLaunchKernelGGL((k_reduce<Q, S, T>), dim3((unsigned)nb), dim3(BLK), 0, h->stream, h->kp, odd_state, cur);
            HIPCHK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_reduce_mid, dim3(MID_BLOCKS), dim3(BLK), 0, h->stream, h->kp, nb);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(BLK), 0, h->stream, h->kp, slot);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int moments(lbm *h, bool odd_state, int cur, void *rho, void *u, void *nut, int dtype)
    {
        dim3 grid((unsigned)((h->kp.ncell + BLK - 1) / BLK));
        if (dtype == LBM_OUT_F32)
            hipLaunchKernelGGL((k_export_moments<Q, S, T, float>), grid, dim3(BLK), 0, h->stream, h->kp, odd_state, cur,
                               (float *)rho, (float *)u, (float *)nut);
        else
            hipLaunchKernelGGL((k_export_moments<Q, S, T, double>), grid, dim3(BLK), 0, h->stream, h->kp, odd_state, cur,
                               (double *)rho, (double *)u, (double *)nut);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int nt(lbm *h, int cur, double *out)
    {
        dim3 grid((unsigned)((h->kp.ncell + BLK - 1) / BLK));
        hipLaunchKernelGGL((k_export_nt<T>), grid, dim3(BLK), 0, h->stream, h->kp, cur, out);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int pops(lbm *h, bool odd_state, double *out)
    {
        dim3 grid((unsigned)((h->kp.ncell + BLK - 1) / BLK));
        hipLaunchKernelGGL((k_export_f<Q, S, T>), grid, dim3(BLK), 0, h->stream, h->kp, odd_state, out);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
};

#define LBM_DISPATCH(h, fn, ...)                                                                 \
    ((h)->Q == 9 ? ((h)->p.precision == LBM_F64   ? Impl<9, double, double>::fn(__VA_ARGS__)    \
                    : (h)->p.precision == LBM_F32 ? Impl<9, float, float>::fn(__VA_ARGS__)      \
                    : (h)->p.precision == LBM_F16 ? Impl<9, _Float16, float>::fn(__VA_ARGS__)   \
                                                  : Impl<9, bf16s, float>::fn(__VA_ARGS__))     \
                 : ((h)->p.precision == LBM_F64   ? Impl<19, double, double>::fn(__VA_ARGS__)   \
                    : (h)->p.precision == LBM_F32 ? Impl<19, float, float>::fn(__VA_ARGS__)     \
                    : (h)->p.precision == LBM_F16 ? Impl<19, _Float16, float>::fn(__VA_ARGS__)  \
                                                  : Impl<19, bf16s, float>::fn(__VA_ARGS__)))

int check_params(int lattice, int nx, int ny, int nz, const lbm_params_t *p)
{
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->size != (int32_t)sizeof(lbm_params_t) || p->version != LBM_PARAMS_VERSION)
        return fail(LBM_EINVAL, "params size/version mismatch (use lbm_params_default)");
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return fail(LBM_EINVAL, "unknown lattice %d", lattice);
    if (nx < 1 || ny < 4 || nz < 1) return fail(LBM_EINVAL, "bad dimensions %d x %d x %d", nx, ny, nz);
    if (lattice == LBM_D2Q9 && nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
    if (storage_bytes(p->precision) < 0) return fail(LBM_EINVAL, "unknown precision %d", p->precision);
    if (p->flow != LBM_FLOW_CHANNEL && p->flow != LBM_FLOW_PLATE) return fail(LBM_EINVAL, "unknown flow %d", p->flow);
    if (p->flow == LBM_FLOW_PLATE && (lattice != LBM_D2Q9 || nx < 4))
        return fail(LBM_EINVAL, "the plate needs D2Q9 and nx >= 4");
    if (p->scheme < LBM_WALL_FIXED_BB || p->scheme > LBM_WALL_CAI_DEGRIGNY) return fail(LBM_EINVAL, "unknown wall scheme");
    if (p->scheme >= LBM_WALL_HRFD && lattice != LBM_D2Q9) return fail(LBM_EINVAL, "HRFD is D2Q9 only");
    if (p->law != LBM_LAW_REICHARDT && p->law != LBM_LAW_SA) return fail(LBM_EINVAL, "unknown wall law");
    if (!(p->nu > 0.0)) return fail(LBM_EINVAL, "nu must be > 0 (tau_eff > 1/2)");
    if (!(p->rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 must be > 0");
    if (p->reduce_every < 0) return fail(LBM_EINVAL, "reduce_every must be >= 0");
    if (p->collision != LBM_COLL_BGK && p->collision != LBM_COLL_CM) return fail(LBM_EINVAL, "unknown collision %d", p->collision);
    if (p->bb_interp < LBM_IBB_HALFWAY || p->bb_interp > LBM_IBB_YU) return fail(LBM_EINVAL, "unknown bb_interp %d", p->bb_interp);
    if (p->bb_interp != LBM_IBB_HALFWAY && p->scheme >= LBM_WALL_HRFD)
        return fail(LBM_EINVAL, "interpolated links apply to the bounce-back schemes only");
    if (p->bb_interp == LBM_IBB_HALFWAY ? p->wall_dist != 0.5 : !(p->wall_dist > 0.0 && p->wall_dist <= 1.0))
        return fail(LBM_EINVAL, "wall_dist must be 1/2 for halfway walls and in (0, 1] otherwise");
    if ((int64_t)nx * ny * nz > (int64_t)1 << 40) return fail(LBM_EINVAL, "lattice too large");
    return LBM_OK;
}

// the cell-update constants from the double-precision parameters
template <typename T> void fill_cellk(const KP &k, int Q, CellK<T> &c)
{
    memset(&c, 0, sizeof c);
    c.nu = (T)k.nu;
    c.rho0 = (T)k.rho0;
    c.fx = (T)k.fx;
    c.fy = (T)k.fy;
    c.fz = (T)k.fz;
    c.cv1_3 = (T)(k.cv1 * k.cv1 * k.cv1);
    c.kappa2 = (T)(k.kappa * k.kappa);
    c.cb1 = (T)k.cb1;
    c.cw1 = (T)k.cw1;
    c.cw2 = (T)k.cw2;
    const double c3 = k.cw3 * k.cw3 * k.cw3;
    c.cw3_6 = (T)(c3 * c3);
    c.rlim = (T)k.rlim;
    c.cb2 = (T)k.cb2;
    c.inv_sigma = (T)(1.0 / k.sigma);
    c.wall_dist = (T)k.wall_dist;
    for (int i = 0; i < Q; ++i) {
        const int *cv = Q == 9 ? Lat<9>::c[i] : Lat<19>::c[i];
        const double w = Q == 9 ? wgt<9>(i) : wgt<19>(i);
        c.cf[i] = (T)(w * (cv[0] * k.fx + cv[1] * k.fy + cv[2] * k.fz));
        if (k.shift_u != 0.0)
            c.soff[i] = (T)(Q == 9 ? shift_off<9, double>(i, k.rho0, k.shift_u) : shift_off<19, double>(i, k.rho0, k.shift_u));
    }
    // the same offsets as the collision on stored values uses them (from the
    // rounded soff, so that both forms see the same numbers)
    double ssum = 0, sj[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        const int *cv = Q == 9 ? Lat<9>::c[i] : Lat<19>::c[i];
        ssum += (double)c.soff[i];
        for (int a = 0; a < 3; ++a) sj[a] += cv[a] * (double)c.soff[i];
    }
    c.ssum = (T)ssum;
    for (int a = 0; a < 3; ++a) c.sj[a] = (T)sj[a];
    c.sfe[0] = c.soff[0];
    for (int kp = 1; 2 * kp < Q; ++kp) {
        c.sfe[kp] = (T)(0.5 * ((double)c.soff[2 * kp - 1] + (double)c.soff[2 * kp]));
        c.sfo[kp] = (T)(0.5 * ((double)c.soff[2 * kp - 1] - (double)c.soff[2 * kp]));
    }
}

void fill_kp(lbm *h)
{
    KP &k = h->kp;
    const lbm_params_t &p = h->p;
    memset(&k, 0, sizeof k);
    k.nx = h->nx;
    k.ny = h->ny;
    k.nz = h->nz;
    k.flow = p.flow;
    k.ncell = (int64_t)h->nx * h->ny * h->nz;
    k.scheme = p.scheme;
    k.law = p.law;
    k.sa_on = p.sa_on;
    k.plate_start = p.plate_start < 0 ? 0 : p.plate_start;
    k.nwall = nwall_of(p.flow, h->nx, h->nz, p.plate_start);
    k.nu = p.nu;
    k.rho0 = p.rho0;
    k.fx = p.force[0];
    k.fy = p.force[1];
    k.fz = h->D == 3 ? p.force[2] : 0.0;
    k.u_inlet = p.u_inlet;
    k.kappa = p.kappa;
    k.B = p.B;
    k.beta = p.scheme == LBM_WALL_CAI_DEGRIGNY ? 1.0 : p.beta;  // eq. 30
    k.reC = p.B - log(p.kappa) / p.kappa;
    k.cb1 = p.cb1;
    k.cb2 = p.cb2;
    k.sigma = p.sigma;
    k.cw1 = p.cb1 / (p.kappa * p.kappa) + (1.0 + p.cb2) / p.sigma;  // definition after eq. 14
    k.cw2 = p.cw2;
    k.cw3 = p.cw3;
    k.cv1 = p.cv1;
    k.rlim = p.rlim;
    k.shift_u = p.store_shift_u;
    k.shifted = p.store_shift_u != 0.0;
    // row-slab XCD mapping for wide channels (see k_step); flat mapping otherwise
    k.rowmap = (LBM_ROWMAP && p.flow == LBM_FLOW_CHANNEL && h->nx >= BLK / 2 && h->ny % 8 == 0) ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        k.wall_u_bottom[a] = p.wall_u_bottom[a];
        k.wall_u_top[a] = p.wall_u_top[a];
    }
    const Layout &L = h->L;
    char *b = h->base;
    k.pops = b + L.pops;
    k.u[0] = b + L.u0;
    k.u[1] = b + L.u1;
    k.nt[0] = b + L.nt0;
    k.nt[1] = b + L.nt1;
    k.usnap = b + L.usnap;
    k.utau = (double *)(b + L.utau);
    k.tdir = (double *)(b + L.tdir);
    k.uw = (double *)(b + L.uw);
    k.wrho = (double *)(b + L.wrho);
    k.ubwf = (double *)(b + L.ubwf);
    k.gan = (double *)(b + L.gan);
    k.partials = (double *)(b + L.partials);
    k.ibuf = (double *)(b + L.ibuf);
    k.bb_interp = p.bb_interp;
    k.wall_dist = p.wall_dist;
    k.result = (double *)(b + L.result);
    k.mid = (double *)(b + L.mid);
    fill_cellk(k, h->Q, k.kd);
    fill_cellk(k, h->Q, k.kf);
}

int run_init(lbm *h, const double *u0dev)
{
    h->step = 0;
    h->last_reduce_step = -1;
    h->prev_reduce_step = 0;
    h->reduce_count = 0;
    h->diverged = false;
    h->flag_pending = false;  // the device-side sticky flag is cleared by the init kernel
    return LBM_DISPATCH(h, init, h, u0dev);
}

// mark the end of an interval of the given kind on the handle's stream
enum : char { EV_NONE = 0, EV_STEP = 1, EV_WALL = 2 };

int record(lbm *h, char kind)
{
    if (h->n_ev >= h->ev.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        h->ev.push_back(e);
        h->ev_kind.push_back(EV_NONE);
    }
    HIPCHK(hipEventRecord(h->ev[h->n_ev], h->stream));
    h->ev_kind[h->n_ev] = kind;
    ++h->n_ev;
    return LBM_OK;
}

int flush_timing(lbm *h)
{
    if (h->n_ev == 0) return LBM_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (size_t k = 1; k < h->n_ev; ++k) {
        if (h->ev_kind[k] == EV_NONE) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev[k - 1], h->ev[k]));
        if (h->ev_kind[k] == EV_STEP) {
            h->acc_step_ms += ms;
            h->acc_step_n++;
        } else {
            h->acc_wall_ms += ms;
            h->acc_wall_n++;
        }
    }
    h->n_ev = 0;
    return LBM_OK;
}

// Device bytes of the requested moment fields in the output type.
int64_t moments_bytes(const lbm *h, const void *rho, const void *u, const void *nut, int dtype)
{
    const int64_t e = dtype == LBM_OUT_F32 ? 4 : 8;
    return e * h->kp.ncell * ((rho ? 1 : 0) + (u ? h->D : 0) + (nut ? 1 : 0));
}

// Moments to host buffers through device staging at `stage` (at least
// moments_bytes bytes): export kernel, copies, one synchronization.
int moments_via(lbm *h, char *stage, void *rho, void *u, void *nut, int dtype)
{
    const int64_t N = h->kp.ncell, e = dtype == LBM_OUT_F32 ? 4 : 8;
    const bool odd_state = (h->step & 1) != 0;
    const int cur = (int)(h->step & 1);
    char *p = stage;
    char *drho = rho ? p : nullptr;
    p += rho ? N * e : 0;
    char *du = u ? p : nullptr;
    p += u ? h->D * N * e : 0;
    char *dn = nut ? p : nullptr;
    int rc = LBM_DISPATCH(h, moments, h, odd_state, cur, drho, du, dn, dtype);
    hipError_t er = hipSuccess;
    if (!rc && rho) er = hipMemcpyAsync(rho, drho, N * e, hipMemcpyDeviceToHost, h->stream);
    if (!rc && er == hipSuccess && u) er = hipMemcpyAsync(u, du, h->D * N * e, hipMemcpyDeviceToHost, h->stream);
    if (!rc && er == hipSuccess && nut) er = hipMemcpyAsync(nut, dn, N * e, hipMemcpyDeviceToHost, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    if (rc) return rc;
    if (er != hipSuccess || e2 != hipSuccess)
        return fail(LBM_EHIP, "moment copy failed: %s", hipGetErrorString(er != hipSuccess ? er : e2));
    return LBM_OK;
}

// The GPU that holds a device pointer (the current device if the runtime
// cannot tell).
int buffer_device(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) == hipSuccess && a.device >= 0) return a.device;
    (void)hipGetLastError();
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

// Makes `dev` the current device for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device address of `scratch` on GPU `dev`, looked up once per device with
// that device current and kept.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES] = {};

int scratch_on(int dev, char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        DeviceGuard g(dev);
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return fail(LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = (char *)ptr;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

// Reads the divergence flag copied after an earlier reduction if that copy
// has completed (never waits).
int poll_flag(lbm *h)
{
    if (!h->flag_pending) return LBM_OK;
    const hipError_t e = hipEventQuery(h->flag_ev);
    if (e == hipErrorNotReady) return LBM_OK;
    if (e != hipSuccess) return fail(LBM_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
    h->flag_pending = false;
    if (*h->flag_host != 0.0) h->diverged = true;
    return LBM_OK;
}

// Queues the copy of the sticky divergence flag to pinned host memory.
int push_flag(lbm *h)
{
    if (!h->flag_host) {
        HIPCHK(hipHostMalloc((void **)&h->flag_host, sizeof(double), hipHostMallocDefault));
        *h->flag_host = 0.0;
        HIPCHK(hipEventCreateWithFlags(&h->flag_ev, hipEventDisableTiming));
    }
    HIPCHK(hipMemcpyAsync(h->flag_host, h->kp.result + RES_STICKY, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipEventRecord(h->flag_ev, h->stream));
    h->flag_pending = true;
    return LBM_OK;
}

int do_reduce(lbm *h, int64_t fused_nb = 0)
{
    const bool odd_state = (h->step & 1) != 0;
    const int cur = (int)(h->step & 1);
    const int slot = h->reduce_count & 1;
    int rc = LBM_DISPATCH(h, reduce, h, odd_state, cur, slot, fused_nb);
    if (rc) return rc;
    h->prev_reduce_step = h->last_reduce_step < 0 ? 0 : h->last_reduce_step;
    h->last_reduce_step = h->step;
    h->reduce_count++;
    return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_params_default(lbm_params_t *p)
{
    memset(p, 0, sizeof *p);
    p->size = (int32_t)sizeof(lbm_params_t);
    p->version = LBM_PARAMS_VERSION;
    p->precision = LBM_F32;
    p->flow = LBM_FLOW_CHANNEL;
    p->scheme = LBM_WALL_SLIP_BB;
    p->law = LBM_LAW_REICHARDT;
    p->sa_on = 1;
    p->plate_start = 0;
    p->reduce_every = 100;
    p->nu = 1e-3;
    p->rho0 = 1.0;
    p->u_ref = 1.0;
    p->nut_init_ratio = 3.0;
    p->kappa = 0.41;
    p->B = 5.2;
    p->beta = 0.28;
    p->cb1 = 0.1355;
    p->cb2 = 0.622;
    p->sigma = 2.0 / 3.0;
    p->cw2 = 0.3;
    p->cw3 = 2.0;
    p->cv1 = 7.1;
    p->rlim = 10.0;
    p->bb_interp = LBM_IBB_HALFWAY;
    p->wall_dist = 0.5;
}

int64_t lbm_footprint(lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p)
{
    int rc = check_params(lattice, nx, ny, nz, p);
    if (rc) return rc;
    Layout L;
    if (!make_layout((int)lattice, nx, ny, nz, p, &L)) return fail(LBM_EINVAL, "bad precision");
    return L.total;
}

int lbm_create(lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p, void *dev_buf,
               int64_t buf_bytes, void *stream, lbm_t **out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(lattice, nx, ny, nz, p);
    if (rc) return rc;
    Layout L;
    make_layout((int)lattice, nx, ny, nz, p, &L);
    if (!dev_buf || buf_bytes < L.total)
        return fail(LBM_EINVAL, "device buffer too small: %lld < %lld bytes", (long long)buf_bytes, (long long)L.total);
    if (((uintptr_t)dev_buf & 255u) != 0) return fail(LBM_EINVAL, "device buffer must be 256-byte aligned");
    lbm *h = new (std::nothrow) lbm();
    if (!h) return fail(LBM_ENOMEM, "host allocation failed");
    h->Q = (int)lattice;
    h->D = lattice == LBM_D2Q9 ? 2 : 3;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->p = *p;
    h->L = L;
    h->base = (char *)dev_buf;
    h->bytes = buf_bytes;
    h->stream = (hipStream_t)stream;
    h->device = buffer_device(dev_buf);
    h->timing = false;
    h->timing_every = 1;
    h->chain_open = false;
    h->flag_host = nullptr;
    h->flag_ev = nullptr;
    h->flag_pending = false;
    h->n_ev = 0;
    h->acc_step_ms = h->acc_wall_ms = 0.0;
    h->acc_step_n = h->acc_wall_n = 0;
    fill_kp(h);
    rc = run_init(h, nullptr);
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return LBM_OK;
}

int lbm_set_velocity(lbm_t *h, const double *u, int on_device)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!u) return fail(LBM_EINVAL, "u is NULL");
    const size_t bytes = (size_t)h->D * h->kp.ncell * sizeof(double);
    const double *dev = u;
    double *tmp = nullptr;
    if (!on_device) {
        HIPCHK(hipMalloc((void **)&tmp, bytes));
        hipError_t e = hipMemcpyAsync(tmp, u, bytes, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return fail(LBM_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
        }
        dev = tmp;
    }
    int rc = run_init(h, dev);
    if (tmp) {
        hipError_t e = hipStreamSynchronize(h->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return fail(LBM_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    return rc;
}

int lbm_set_wall_bc(lbm_t *h, lbm_wall_scheme_t scheme, double beta)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (scheme < LBM_WALL_FIXED_BB || scheme > LBM_WALL_CAI_DEGRIGNY) return fail(LBM_EINVAL, "unknown wall scheme");
    if (scheme >= LBM_WALL_HRFD && h->Q != 9) return fail(LBM_EINVAL, "HRFD is D2Q9 only");
    if (scheme >= LBM_WALL_HRFD && h->p.bb_interp != LBM_IBB_HALFWAY)
        return fail(LBM_EINVAL, "interpolated links apply to the bounce-back schemes only");
    h->p.scheme = scheme;
    h->p.beta = beta;
    h->kp.scheme = scheme;
    h->kp.beta = scheme == LBM_WALL_CAI_DEGRIGNY ? 1.0 : beta;  // eq. 30
    // refresh the wall state for the new scheme from the current velocity
    return LBM_DISPATCH(h, wall, h, (int)(h->step & 1));
}

int lbm_step(lbm_t *h, int64_t n)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    int rc = poll_flag(h);
    if (rc) return rc;
    if (h->diverged) return fail(LBM_EDIVERGED, "the solution diverged at or before step %lld", (long long)h->last_reduce_step);
    // host time before the call is not counted: the first timed step opens a
    // new chain of events
    h->chain_open = false;
    for (int64_t s = 0; s < n; ++s) {
        const int64_t next = h->step + 1;
        const bool odd = (next & 1) != 0;
        const int rd = (int)(h->step & 1);
        const bool red = h->p.reduce_every > 0 && next % h->p.reduce_every == 0;
        const bool timed = h->timing && (h->timing_every <= 1 || h->step % h->timing_every < 2);
        if (timed && !h->chain_open && (rc = record(h, EV_NONE))) return rc;
        int64_t nb = 0;
        rc = LBM_DISPATCH(h, step, h, odd, rd, red, &nb);
        if (rc) return rc;
        // the channel's even steps carry the reduction's first pass
        const bool fused = red && !odd && h->p.flow == LBM_FLOW_CHANNEL;
        if (timed && (rc = record(h, EV_STEP))) return rc;
        rc = LBM_DISPATCH(h, wall, h, rd ^ 1);
        if (rc) return rc;
        if (timed && (rc = record(h, EV_WALL))) return rc;
        h->chain_open = timed;
        h->step = next;
        if (red) {
            rc = do_reduce(h, fused ? nb : 0);
            if (rc) return rc;
            if ((rc = poll_flag(h))) return rc;  // an earlier reduction's flag, if already back
            if ((rc = push_flag(h))) return rc;
            if (h->chain_open && (rc = record(h, EV_NONE))) return rc;
        }
        if (h->timing && h->n_ev >= 8192) {
            rc = flush_timing(h);
            if (rc) return rc;
            h->chain_open = false;
        }
        if (h->diverged) return fail(LBM_EDIVERGED, "the solution diverged before step %lld", (long long)h->step);
    }
    return LBM_OK;
}

int lbm_moments(lbm_t *h, void *rho, void *u, void *nu_t, int dtype, int where)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (dtype != LBM_OUT_F64 && dtype != LBM_OUT_F32) return fail(LBM_EINVAL, "unknown output dtype %d", dtype);
    if (where != LBM_ON_HOST && where != LBM_ON_DEVICE) return fail(LBM_EINVAL, "unknown location %d", where);
    const bool odd_state = (h->step & 1) != 0;
    const int cur = (int)(h->step & 1);
    if (where == LBM_ON_DEVICE) return LBM_DISPATCH(h, moments, h, odd_state, cur, rho, u, nu_t, dtype);
    const int64_t bytes = moments_bytes(h, rho, u, nu_t, dtype);
    char *tmp = nullptr;
    if (bytes > 0) HIPCHK(hipMalloc((void **)&tmp, bytes));
    int rc = moments_via(h, tmp, rho, u, nu_t, dtype);
    (void)hipFree(tmp);
    return rc;
}

int lbm_nu_tilde(lbm_t *h, double *nt, int on_device)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!nt) return fail(LBM_EINVAL, "nt is NULL");
    const int64_t N = h->kp.ncell;
    const int cur = (int)(h->step & 1);
    if (on_device) return LBM_DISPATCH(h, nt, h, cur, nt);
    double *tmp = nullptr;
    HIPCHK(hipMalloc((void **)&tmp, N * sizeof(double)));
    int rc = LBM_DISPATCH(h, nt, h, cur, tmp);
    hipError_t e = rc ? hipSuccess : hipMemcpyAsync(nt, tmp, N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (rc) return rc;
    if (e != hipSuccess || e2 != hipSuccess) return fail(LBM_EHIP, "nu_tilde copy failed");
    return LBM_OK;
}

int lbm_populations(lbm_t *h, double *f_host)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!f_host) return fail(LBM_EINVAL, "f is NULL");
    const size_t nb = (size_t)h->Q * h->kp.ncell * sizeof(double);
    double *tmp = nullptr;
    HIPCHK(hipMalloc((void **)&tmp, nb));
    int rc = LBM_DISPATCH(h, pops, h, (h->step & 1) != 0, tmp);
    hipError_t e = rc ? hipSuccess : hipMemcpyAsync(f_host, tmp, nb, hipMemcpyDeviceToHost, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (rc) return rc;
    if (e != hipSuccess || e2 != hipSuccess) return fail(LBM_EHIP, "population copy failed");
    return LBM_OK;
}

int lbm_wall(lbm_t *h, double *u_tau, double *cf, double *t, double *u_w, int64_t n)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    const int64_t nw = h->kp.nwall;
    if (n < nw) return fail(LBM_EINVAL, "wall buffers hold %lld < %lld entries", (long long)n, (long long)nw);
    if (nw == 0) return LBM_OK;
    std::vector<double> ut(nw), td(3 * nw), uw(3 * nw);
    HIPCHK(hipMemcpyAsync(ut.data(), h->kp.utau, nw * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(td.data(), h->kp.tdir, 3 * nw * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(uw.data(), h->kp.uw, 3 * nw * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int64_t w = 0; w < nw; ++w) {
        if (u_tau) u_tau[w] = ut[w];
        if (cf) cf[w] = 2.0 * (ut[w] / h->p.u_ref) * (ut[w] / h->p.u_ref);
        for (int a = 0; a < 3; ++a) {
            if (t) t[3 * w + a] = td[a * nw + w];
            if (u_w) u_w[3 * w + a] = uw[a * nw + w];
        }
    }
    return LBM_OK;
}

int64_t lbm_ncell(const lbm_t *h) { return h ? h->kp.ncell : -1; }
int64_t lbm_nwall(const lbm_t *h) { return h ? h->kp.nwall : -1; }
int64_t lbm_steps(const lbm_t *h) { return h ? h->step : -1; }

int lbm_residual(lbm_t *h, lbm_residual_t *out)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    if (h->last_reduce_step != h->step) {
        int rc = do_reduce(h);
        if (rc) return rc;
    }
    double r[2 * NRED];
    HIPCHK(hipMemcpyAsync(r, h->kp.result, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const int cur = (h->reduce_count - 1) & 1, prv = cur ^ 1;
    const double *c = r + cur * NRED, *q = r + prv * NRED;
    memset(out, 0, sizeof *out);
    out->step = h->step;
    out->steps_since_previous = h->last_reduce_step - h->prev_reduce_step;
    out->mass = (double)h->kp.ncell * h->p.rho0 + c[0];
    for (int a = 0; a < 3; ++a) out->momentum[a] = c[1 + a];
    const double K = out->steps_since_previous > 0 ? (double)out->steps_since_previous : 1.0;
    out->l2_du_rel = c[5] > 0.0 ? sqrt(c[4]) / (K * sqrt(c[5])) : 0.0;
    const double nw = h->kp.nwall > 0 ? (double)h->kp.nwall : 1.0;
    out->mean_u_tau = c[7] / nw;
    const double prev = q[7] / nw;
    out->d_u_tau_rel = (h->reduce_count >= 2 && prev > 0.0) ? fabs(out->mean_u_tau - prev) / prev : -1.0;
    out->nan_flag = c[6] > 0.0 || !isfinite(c[4]) || !isfinite(c[5]) ? 1.0 : 0.0;
    if (out->nan_flag != 0.0) {
        h->diverged = true;
        return fail(LBM_EDIVERGED, "divergence detected at step %lld", (long long)h->step);
    }
    return LBM_OK;
}

int lbm_set_timing(lbm_t *h, int on)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (on < 0) return fail(LBM_EINVAL, "timing period must be >= 0");
    int rc = flush_timing(h);
    if (rc) return rc;
    h->timing = on != 0;
    h->timing_every = on > 1 ? on : 1;
    h->acc_step_ms = h->acc_wall_ms = 0.0;
    h->acc_step_n = h->acc_wall_n = 0;
    return LBM_OK;
}

int lbm_get_timing(lbm_t *h, lbm_timing_t *out)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    int rc = flush_timing(h);
    if (rc) return rc;
    out->step_launches = h->acc_step_n;
    out->step_ms = h->acc_step_ms;
    out->wall_launches = h->acc_wall_n;
    out->wall_ms = h->acc_wall_ms;
    return LBM_OK;
}

int64_t lbm_checkpoint_bytes(const lbm_t *h)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    return 64 + h->L.total;
}

int lbm_save(lbm_t *h, void *host, int64_t bytes)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!host || bytes < 64 + h->L.total) return fail(LBM_EINVAL, "checkpoint buffer too small");
    int64_t hdr[8] = {0x4c424d434b505431LL, h->Q, h->nx, h->ny, h->nz, h->step, h->L.total, h->p.precision};
    memcpy(host, hdr, sizeof hdr);
    HIPCHK(hipMemcpyAsync((char *)host + 64, h->base, h->L.total, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_load(lbm_t *h, const void *host, int64_t bytes)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (!host || bytes < 64 + h->L.total) return fail(LBM_EINVAL, "checkpoint buffer too small");
    int64_t hdr[8];
    memcpy(hdr, host, sizeof hdr);
    if (hdr[0] != 0x4c424d434b505431LL || hdr[1] != h->Q || hdr[2] != h->nx || hdr[3] != h->ny || hdr[4] != h->nz ||
        hdr[6] != h->L.total || hdr[7] != h->p.precision)
        return fail(LBM_EINVAL, "checkpoint does not match this lattice");
    HIPCHK(hipMemcpyAsync(h->base, (const char *)host + 64, h->L.total, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->step = hdr[5];
    h->last_reduce_step = -1;
    h->prev_reduce_step = h->step;
    h->reduce_count = 0;
    h->diverged = false;
    h->flag_pending = false;  // a copy queued before the load is stale
    return LBM_OK;
}

int lbm_destroy(lbm_t *h)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->flag_ev) (void)hipEventDestroy(h->flag_ev);
    if (h->flag_host) (void)hipHostFree(h->flag_host);
    delete h;
    return LBM_OK;
}

int lbm_moments_noalloc(lbm_t *h, void *rho, void *u, void *nu_t, int dtype, int where)
{
    if (!h) return fail(LBM_ESTATE, "NULL handle");
    if (dtype != LBM_OUT_F64 && dtype != LBM_OUT_F32) return fail(LBM_EINVAL, "unknown output dtype %d", dtype);
    if (where != LBM_ON_HOST && where != LBM_ON_DEVICE) return fail(LBM_EINVAL, "unknown location %d", where);
    DeviceGuard g(h->device);
    if (where == LBM_ON_DEVICE) return lbm_moments(h, rho, u, nu_t, dtype, where);  // allocates nothing
    const int64_t bytes = moments_bytes(h, rho, u, nu_t, dtype);
    if (bytes > LBM_NOALLOC_SCRATCH_BYTES)
        return fail(LBM_EINVAL, "lbm_moments_noalloc: the requested fields need %lld bytes of staging, more than the %lld of its scratch; use lbm_moments",
                    (long long)bytes, (long long)LBM_NOALLOC_SCRATCH_BYTES);
    if (bytes == 0) return LBM_OK;
    char *ptr = nullptr;
    int rc = scratch_on(h->device, &ptr);
    if (rc) return rc;
    return moments_via(h, ptr, rho, u, nu_t, dtype);
}

const char *lbm_last_error(void) { return g_err; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving pool: one caller-owned device buffer, a slot table, first-fit
// allocation by footprint.  Small D2Q9 lattices run in the persistent
// k_serve launch (stream A); larger ones run the regular kernels on stream B,
// so the two overlap on the device.
// ---------------------------------------------------------------------------
namespace {

// D2Q9 lattices up to SERVE_SMALL_CELLS cells (channels up to
// SERVE_SMALL_CHANNEL) run in the persistent launch, where a step of a lattice
// takes a few microseconds whatever else is resident; larger ones go to the
// multi-lattice launches, whose step time grows with the total resident work.
constexpr int64_t SERVE_SMALL_CELLS = 4 * SBLK, SERVE_SMALL_CHANNEL = 8 * SBLK;

struct PoolSlot {
    bool used = false, small = false, releasing = false;
    lbm *h = nullptr;
    int64_t off = 0, bytes = 0;
    int status = SLOT_IDLE;
    int key = 0;  // launch kind: see slot_key
    double residual = 0.0, mean_utau = 0.0, d_utau_rel = -1.0;
    int conv_by = 0;
    int64_t steps = 0, max_steps = 0, reduce_every = 100;
    int64_t step_blocks = 0, wall_blocks = 0;
};

// small: precision x collision x flow x wall treatment (32 kinds);
// large: lattice x precision x collision (16 kinds)
int slot_key(const lbm *h, bool small)
{
    const int v = h->p.precision * 2 + (h->p.collision == LBM_COLL_CM ? 1 : 0);
    if (small) return v * 4 + (h->p.flow == LBM_FLOW_PLATE ? 2 : 0) + (h->p.scheme >= LBM_WALL_HRFD ? 1 : 0);
    return (h->Q == 19 ? 8 : 0) + v;
}
constexpr int NKEY = 16, NSKEY = 32;

struct PoolGroup {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool in_flight = false;
    SlotDesc *mirror = nullptr;    // pinned: descriptors copied back at the end of a chunk
    int *hlist = nullptr;          // pinned staging of the slot lists
    int64_t *hpref = nullptr;      // pinned staging of the block prefix sums (large group)
    std::vector<int> chunk_slots;  // slots running when the chunk was launched
};

}  // namespace

struct lbm_pool {
    char *base;
    int64_t bytes, data_off;
    int max_slots;
    bool own_sA;
    SlotDesc *dslots;       // device descriptors
    SlotDesc *hstage;       // pinned staging of descriptor uploads
    int *dlist;             // device slot lists: [0, M) small group, [M, 3M) large group
    int64_t *dpref;         // device block prefix sums (2 (M + 1))
    int2 *dtab;             // device block tables: cells [0, tab_cap), walls [tab_cap, 2 tab_cap)
    int64_t tab_cap, tab_used_step, tab_used_wall;
    PoolGroup g[2];         // 0: persistent small-lattice launches, 1: large lattices
    std::vector<PoolSlot> slots;
    std::map<int64_t, int64_t> freel;  // offset -> size
};

namespace {

int64_t pool_alloc(lbm_pool *pl, int64_t bytes)
{
    bytes = align256(bytes);
    for (auto it = pl->freel.begin(); it != pl->freel.end(); ++it) {
        if (it->second >= bytes) {
            const int64_t off = it->first, rest = it->second - bytes;
            pl->freel.erase(it);
            if (rest > 0) pl->freel[off + bytes] = rest;
            return off;
        }
    }
    return -1;
}

void pool_free(lbm_pool *pl, int64_t off, int64_t bytes)
{
    bytes = align256(bytes);
    auto it = pl->freel.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != pl->freel.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        pl->freel.erase(nx);
    }
    if (it != pl->freel.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            pl->freel.erase(it);
        }
    }
}

// ---- launches -------------------------------------------------------------
template <typename S, typename T, bool CMC> int launch_serve(lbm_pool *pl, int fw, const int *dlist, int n, int chunk)
{
    hipStream_t st = pl->g[0].stream;
    SlotDesc *d = pl->dslots;
    switch (fw) {
    case 0: hipLaunchKernelGGL((k_serve<S, T, CMC, false, false>), dim3(n), dim3(SBLK), 0, st, d, dlist, chunk); break;
    case 1: hipLaunchKernelGGL((k_serve<S, T, CMC, false, true>), dim3(n), dim3(SBLK), 0, st, d, dlist, chunk); break;
    case 2: hipLaunchKernelGGL((k_serve<S, T, CMC, true, false>), dim3(n), dim3(SBLK), 0, st, d, dlist, chunk); break;
    default: hipLaunchKernelGGL((k_serve<S, T, CMC, true, true>), dim3(n), dim3(SBLK), 0, st, d, dlist, chunk); break;
    }
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

int serve_key(lbm_pool *pl, int key, const int *dlist, int n, int chunk)
{
    const int fw = key & 3, v = key >> 2;
    const bool cm = v & 1;
    switch (v / 2) {
    case LBM_F64: return cm ? launch_serve<double, double, true>(pl, fw, dlist, n, chunk) : launch_serve<double, double, false>(pl, fw, dlist, n, chunk);
    case LBM_F32: return cm ? launch_serve<float, float, true>(pl, fw, dlist, n, chunk) : launch_serve<float, float, false>(pl, fw, dlist, n, chunk);
    case LBM_F16: return cm ? launch_serve<_Float16, float, true>(pl, fw, dlist, n, chunk) : launch_serve<_Float16, float, false>(pl, fw, dlist, n, chunk);
    default: return cm ? launch_serve<bf16s, float, true>(pl, fw, dlist, n, chunk) : launch_serve<bf16s, float, false>(pl, fw, dlist, n, chunk);
    }
}

struct MLaunch {
    int64_t step_off, step_n, wall_off, wall_n;
    const int *list;
    int nlist;
    int s;
};

template <int Q, typename S, typename T, bool CMC> struct MKind {
    static int step(lbm_pool *pl, const MLaunch &m)
    {
        hipStream_t st = pl->g[1].stream;
        if (m.step_n > 0) hipLaunchKernelGGL((k_mstep<Q, S, T, CMC>), dim3((unsigned)m.step_n), dim3(BLK), 0, st, pl->dslots, pl->dtab + m.step_off, m.s);
        if (m.wall_n > 0) hipLaunchKernelGGL((k_mwall<Lat<Q>::D, T>), dim3((unsigned)m.wall_n), dim3(BLK), 0, st, pl->dslots, pl->dtab + pl->tab_cap + m.wall_off, m.s);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
    static int reduce(lbm_pool *pl, const MLaunch &m)
    {
        hipStream_t st = pl->g[1].stream;
        hipLaunchKernelGGL((k_mreduce<Q, S, T>), dim3((unsigned)(m.nlist * MRED)), dim3(BLK), 0, st, pl->dslots, m.list, m.s);
        hipLaunchKernelGGL(k_mreduce_final, dim3((unsigned)m.nlist), dim3(BLK), 0, st, pl->dslots, m.list, m.s);
        HIPCHK(hipGetLastError());
        return LBM_OK;
    }
};

template <int Q> int mdispatch(lbm_pool *pl, int v, const MLaunch &m, bool red)
{
    const bool cm = v & 1;
#define LBM_MK(S_, T_)                                                                       \
    return cm ? (red ? MKind<Q, S_, T_, true>::reduce(pl, m) : MKind<Q, S_, T_, true>::step(pl, m)) \
              : (red ? MKind<Q, S_, T_, false>::reduce(pl, m) : MKind<Q, S_, T_, false>::step(pl, m))
    switch (v / 2) {
    case LBM_F64: LBM_MK(double, double);
    case LBM_F32: LBM_MK(float, float);
    case LBM_F16: LBM_MK(_Float16, float);
    default: LBM_MK(bf16s, float);
    }
#undef LBM_MK
}

int mlaunch(lbm_pool *pl, int key, const MLaunch &m, bool red)
{
    return key >= 8 ? mdispatch<19>(pl, key - 8, m, red) : mdispatch<9>(pl, key, m, red);
}

__global__ void k_mtab(int2 *tab, const int64_t *pref, const int *slots, int n)
{
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i >= pref[n]) return;
    int lo = 0, hi = n - 1;  // largest k with pref[k] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (pref[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    tab[i] = make_int2(slots[lo], (int)(i - pref[lo]));
}

// ---- group bookkeeping -------------------------------------------------------
void finish_release(lbm_pool *pl, int i)
{
    PoolSlot &S = pl->slots[i];
    if (!S.small) {
        pl->tab_used_step -= S.step_blocks;
        pl->tab_used_wall -= S.wall_blocks;
    }
    lbm_destroy(S.h);
    pool_free(pl, S.off, S.bytes);
    S = PoolSlot{};
}

void harvest(lbm_pool *pl, int gi)
{
    PoolGroup &G = pl->g[gi];
    for (int i : G.chunk_slots) {
        PoolSlot &S = pl->slots[i];
        if (!S.used) continue;
        const SlotDesc &d = G.mirror[i];
        S.status = d.status;
        S.residual = d.residual;
        S.mean_utau = d.mean_utau;
        S.d_utau_rel = d.d_utau_rel;
        S.conv_by = d.conv_by;
        S.steps = d.step;
        S.h->step = d.step;
        S.h->last_reduce_step = -1;
    }
    G.in_flight = false;
    for (int i = 0; i < pl->max_slots; ++i) {
        PoolSlot &S = pl->slots[i];
        if (S.used && S.releasing && (S.small ? 0 : 1) == gi) finish_release(pl, i);
    }
}

int launch_small(lbm_pool *pl, int chunk)
{
    PoolGroup &G = pl->g[0];
    G.chunk_slots.clear();
    int start[NSKEY], cnt[NSKEY], n = 0;
    for (int k = 0; k < NSKEY; ++k) {
        start[k] = n;
        for (int i = 0; i < pl->max_slots; ++i) {
            const PoolSlot &S = pl->slots[i];
            if (S.used && !S.releasing && S.small && S.status == SLOT_RUNNING && S.key == k) {
                G.hlist[n++] = i;
                G.chunk_slots.push_back(i);
            }
        }
        cnt[k] = n - start[k];
    }
    if (n == 0) return LBM_OK;
    HIPCHK(hipMemcpyAsync(pl->dlist, G.hlist, sizeof(int) * n, hipMemcpyHostToDevice, G.stream));
    for (int k = 0; k < NSKEY; ++k)
        if (cnt[k]) {
            int rc = serve_key(pl, k, pl->dlist + start[k], cnt[k], chunk);
            if (rc) return rc;
        }
    HIPCHK(hipMemcpyAsync(G.mirror, pl->dslots, sizeof(SlotDesc) * pl->max_slots, hipMemcpyDeviceToHost, G.stream));
    HIPCHK(hipEventRecord(G.done, G.stream));
    G.in_flight = true;
    return LBM_OK;
}

int launch_large(lbm_pool *pl, int chunk)
{
    PoolGroup &G = pl->g[1];
    const int M = pl->max_slots;
    G.chunk_slots.clear();
    int lstart[NKEY], lcnt[NKEY], n = 0;
    int64_t soff[NKEY], scnt[NKEY], woff[NKEY], wcnt[NKEY];
    int64_t *ps = G.hpref, *pw = G.hpref + (M + 1);
    ps[0] = pw[0] = 0;
    for (int k = 0; k < NKEY; ++k) {
        lstart[k] = n;
        soff[k] = ps[n];
        woff[k] = pw[n];
        for (int i = 0; i < M; ++i) {
            const PoolSlot &S = pl->slots[i];
            if (S.used && !S.releasing && !S.small && S.status == SLOT_RUNNING && S.key == k) {
                G.hlist[n] = i;
                ps[n + 1] = ps[n] + S.step_blocks;
                pw[n + 1] = pw[n] + S.wall_blocks;
                ++n;
                G.chunk_slots.push_back(i);
            }
        }
        lcnt[k] = n - lstart[k];
        scnt[k] = ps[n] - soff[k];
        wcnt[k] = pw[n] - woff[k];
    }
    if (n == 0) return LBM_OK;
    int *dl = pl->dlist + M;
    int64_t *dps = pl->dpref, *dpw = pl->dpref + (M + 1);
    HIPCHK(hipMemcpyAsync(dl, G.hlist, sizeof(int) * n, hipMemcpyHostToDevice, G.stream));
    HIPCHK(hipMemcpyAsync(dps, ps, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, G.stream));
    HIPCHK(hipMemcpyAsync(dpw, pw, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, G.stream));
    if (ps[n] > 0)
        hipLaunchKernelGGL(k_mtab, dim3((unsigned)((ps[n] + BLK - 1) / BLK)), dim3(BLK), 0, G.stream, pl->dtab, dps, dl, n);
    if (pw[n] > 0)
        hipLaunchKernelGGL(k_mtab, dim3((unsigned)((pw[n] + BLK - 1) / BLK)), dim3(BLK), 0, G.stream, pl->dtab + pl->tab_cap, dpw, dl, n);
    HIPCHK(hipGetLastError());
    for (int s = 0; s < chunk; ++s) {
        bool due = false;
        for (int i : G.chunk_slots) {
            const PoolSlot &S = pl->slots[i];
            const int64_t after = S.steps + s + 1;
            if (after <= S.max_steps && (after % S.reduce_every == 0 || after == S.max_steps)) due = true;
        }
        for (int k = 0; k < NKEY; ++k) {
            if (!lcnt[k]) continue;
            const MLaunch m{soff[k], scnt[k], woff[k], wcnt[k], dl + lstart[k], lcnt[k], s};
            int rc = mlaunch(pl, k, m, false);
            if (rc) return rc;
        }
        if (!due) continue;
        for (int k = 0; k < NKEY; ++k) {
            if (!lcnt[k]) continue;
            const MLaunch m{soff[k], scnt[k], woff[k], wcnt[k], dl + lstart[k], lcnt[k], s};
            int rc = mlaunch(pl, k, m, true);
            if (rc) return rc;
        }
    }
    hipLaunchKernelGGL(k_mfinish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, G.stream, pl->dslots, dl, n, chunk);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(G.mirror, pl->dslots, sizeof(SlotDesc) * M, hipMemcpyDeviceToHost, G.stream));
    HIPCHK(hipEventRecord(G.done, G.stream));
    G.in_flight = true;
    return LBM_OK;
}

int launch_group(lbm_pool *pl, int gi, int chunk) { return gi == 0 ? launch_small(pl, chunk) : launch_large(pl, chunk); }

int wait_group(lbm_pool *pl, int gi)
{
    PoolGroup &G = pl->g[gi];
    if (!G.in_flight) return LBM_OK;
    HIPCHK(hipEventSynchronize(G.done));
    harvest(pl, gi);
    return LBM_OK;
}

void pool_teardown(lbm_pool *pl)
{
    for (auto &G : pl->g) {
        if (G.stream) (void)hipStreamSynchronize(G.stream);
        if (G.done) (void)hipEventDestroy(G.done);
        if (G.mirror) (void)hipHostFree(G.mirror);
        if (G.hlist) (void)hipHostFree(G.hlist);
        if (G.hpref) (void)hipHostFree(G.hpref);
    }
    for (auto &S : pl->slots)
        if (S.used && S.h) lbm_destroy(S.h);
    if (pl->hstage) (void)hipHostFree(pl->hstage);
    if (pl->g[1].stream) (void)hipStreamDestroy(pl->g[1].stream);
    delete pl;
}

}  // namespace

extern "C" {

int lbm_pool_create(void *dev_buf, int64_t bytes, int max_slots, void *stream, lbm_pool_t **out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65536) return fail(LBM_EINVAL, "max_slots must be in [1, 65536]");
    if (!dev_buf || ((uintptr_t)dev_buf & 255u)) return fail(LBM_EINVAL, "pool buffer must be non-NULL and 256-byte aligned");
    const int64_t M = max_slots;
    // block tables: at most two blocks per 256 cells, and no cell takes fewer
    // than 32 bytes of the buffer
    const int64_t tab_cap = bytes / (32 * 128) + 4 * M;
    const int64_t desc = align256(M * (int64_t)sizeof(SlotDesc));
    const int64_t lists = align256(3 * M * (int64_t)sizeof(int));
    const int64_t prefs = align256(2 * (M + 1) * (int64_t)sizeof(int64_t));
    const int64_t tabs = align256(2 * tab_cap * (int64_t)sizeof(int2));
    const int64_t data_off = desc + lists + prefs + tabs;
    if (bytes < data_off + 4096) return fail(LBM_EINVAL, "pool buffer too small");
    lbm_pool *pl = new (std::nothrow) lbm_pool();
    if (!pl) return fail(LBM_ENOMEM, "host allocation failed");
    pl->base = (char *)dev_buf;
    pl->bytes = bytes;
    pl->max_slots = max_slots;
    pl->dslots = (SlotDesc *)pl->base;
    pl->dlist = (int *)(pl->base + desc);
    pl->dpref = (int64_t *)(pl->base + desc + lists);
    pl->dtab = (int2 *)(pl->base + desc + lists + prefs);
    pl->tab_cap = tab_cap;
    pl->tab_used_step = pl->tab_used_wall = 0;
    pl->data_off = data_off;
    pl->slots.assign(max_slots, PoolSlot{});
    pl->g[0].stream = (hipStream_t)stream;
    hipError_t e = hipStreamCreateWithFlags(&pl->g[1].stream, hipStreamNonBlocking);
    for (int gi = 0; gi < 2 && e == hipSuccess; ++gi) {
        PoolGroup &G = pl->g[gi];
        e = hipEventCreateWithFlags(&G.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.mirror, sizeof(SlotDesc) * M, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.hlist, sizeof(int) * M, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&G.hpref, sizeof(int64_t) * 2 * (M + 1), hipHostMallocDefault);
    }
    if (e == hipSuccess) e = hipHostMalloc((void **)&pl->hstage, sizeof(SlotDesc) * M, hipHostMallocDefault);
    if (e != hipSuccess) {
        pool_teardown(pl);
        return fail(LBM_EHIP, "pool set-up: %s", hipGetErrorString(e));
    }
    pl->freel[data_off] = bytes - data_off;
    *out = pl;
    return LBM_OK;
}

int64_t lbm_pool_free_bytes(const lbm_pool_t *pl)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    int64_t best = 0;
    for (auto &kv : pl->freel) best = kv.second > best ? kv.second : best;
    return best;
}

int lbm_pool_admit(lbm_pool_t *pl, lbm_lattice_t lattice, int nx, int ny, int nz, const lbm_params_t *p,
                   const double *u0_host, double tol, double tol_utau, int64_t max_steps, int *slot)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    if (!slot) return fail(LBM_EINVAL, "slot is NULL");
    *slot = -1;
    int64_t need = lbm_footprint(lattice, nx, ny, nz, p);
    if (need < 0) return (int)need;
    if (!(tol >= 0.0) || !(tol_utau >= 0.0) || max_steps < 1)
        return fail(LBM_EINVAL, "tol and tol_utau must be >= 0 and max_steps >= 1");
    int idx = -1;
    for (int i = 0; i < pl->max_slots; ++i)
        if (!pl->slots[i].used) {
            idx = i;
            break;
        }
    if (idx < 0) return fail(LBM_ENOMEM, "no free slot");
    const int64_t cells2 = (int64_t)nx * ny;
    const bool small = lattice == LBM_D2Q9 &&
                       (cells2 <= SERVE_SMALL_CELLS || (p->flow == LBM_FLOW_CHANNEL && cells2 <= SERVE_SMALL_CHANNEL)) &&
                       (p->flow == LBM_FLOW_CHANNEL || ny <= SERVE_MAX_NY);
    const int64_t off = pool_alloc(pl, need);
    if (off < 0) return fail(LBM_ENOMEM, "no free block of %lld bytes", (long long)need);
    PoolGroup &G = pl->g[small ? 0 : 1];
    lbm *h = nullptr;
    int rc = lbm_create(lattice, nx, ny, nz, p, pl->base + off, align256(need), G.stream, &h);
    if (!rc && u0_host) rc = lbm_set_velocity(h, u0_host, 0);
    int64_t sb = 0, wb = 0;
    if (!rc && !small) {
        // blocks of this lattice in the multi-lattice launches (k_mstep, k_mwall)
        sb = p->flow == LBM_FLOW_PLATE ? (int64_t)ny * ((nx + BLK - 1) / BLK) : (h->kp.ncell + BLK - 1) / BLK;
        wb = (h->kp.nwall + BLK - 1) / BLK;
        if (pl->tab_used_step + sb > pl->tab_cap || pl->tab_used_wall + wb > pl->tab_cap || sb > INT32_MAX)
            rc = fail(LBM_ENOMEM, "pool block table full");
    }
    if (rc) {
        if (h) lbm_destroy(h);
        pool_free(pl, off, need);
        return rc;
    }
    PoolSlot &S = pl->slots[idx];
    S = PoolSlot{};
    S.used = true;
    S.small = small;
    S.h = h;
    S.off = off;
    S.bytes = need;
    S.status = SLOT_RUNNING;
    S.key = slot_key(h, small);
    S.max_steps = max_steps;
    S.reduce_every = h->p.reduce_every > 0 ? h->p.reduce_every : 100;
    S.step_blocks = sb;
    S.wall_blocks = wb;
    if (!small) {
        pl->tab_used_step += sb;
        pl->tab_used_wall += wb;
    }
    SlotDesc &d = pl->hstage[idx];
    d = SlotDesc{};
    d.kp = h->kp;
    d.step = 0;
    d.snap_step = 0;
    d.stop_step = 0;
    d.max_steps = max_steps;
    d.tol = tol;
    d.tol_utau = tol_utau;
    d.prev_mean_utau = 0.0;
    d.d_utau_rel = -1.0;
    d.conv_by = 0;
    d.status = SLOT_RUNNING;
    d.reduce_every = (int)S.reduce_every;
    d.variant = S.key;
    HIPCHK(hipMemcpyAsync(pl->dslots + idx, &d, sizeof d, hipMemcpyHostToDevice, G.stream));
    *slot = idx;
    return LBM_OK;
}

int lbm_pool_pump(lbm_pool_t *pl, int64_t steps, int *in_flight)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    if (steps < 1 || steps > (1 << 30)) return fail(LBM_EINVAL, "steps must be in [1, 2^30]");
    for (int gi = 0; gi < 2; ++gi) {
        PoolGroup &G = pl->g[gi];
        if (G.in_flight) {
            const hipError_t e = hipEventQuery(G.done);
            if (e == hipSuccess)
                harvest(pl, gi);
            else if (e != hipErrorNotReady)
                return fail(LBM_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
        }
        if (!G.in_flight) {
            int rc = launch_group(pl, gi, (int)steps);
            if (rc) return rc;
        }
    }
    if (in_flight) *in_flight = (pl->g[0].in_flight ? 1 : 0) + (pl->g[1].in_flight ? 1 : 0);
    return LBM_OK;
}

int lbm_pool_step(lbm_pool_t *pl, int64_t steps)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    if (steps < 1 || steps > (1 << 30)) return fail(LBM_EINVAL, "steps must be in [1, 2^30]");
    for (int gi = 0; gi < 2; ++gi) {
        int rc = wait_group(pl, gi);
        if (rc) return rc;
    }
    for (int gi = 0; gi < 2; ++gi) {
        int rc = launch_group(pl, gi, (int)steps);
        if (rc) return rc;
    }
    for (int gi = 0; gi < 2; ++gi) {
        int rc = wait_group(pl, gi);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_pool_poll(lbm_pool_t *pl, int slot, lbm_pool_status_t *out)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    if (slot < 0 || slot >= pl->max_slots || !pl->slots[slot].used || pl->slots[slot].releasing)
        return fail(LBM_EINVAL, "bad slot %d", slot);
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const PoolSlot &S = pl->slots[slot];
    out->status = S.status;
    out->batched = S.small ? 1 : 0;
    out->steps = S.steps;
    out->residual = S.residual;
    out->mean_u_tau = S.mean_utau;
    out->d_u_tau_rel = S.d_utau_rel;
    out->converged_by = S.conv_by;
    out->footprint = S.bytes;
    return LBM_OK;
}

lbm_t *lbm_pool_lattice(lbm_pool_t *pl, int slot)
{
    if (!pl || slot < 0 || slot >= pl->max_slots || !pl->slots[slot].used || pl->slots[slot].releasing) {
        fail(LBM_EINVAL, "bad slot %d", slot);
        return nullptr;
    }
    return pl->slots[slot].h;
}

int lbm_pool_release(lbm_pool_t *pl, int slot)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    if (slot < 0 || slot >= pl->max_slots || !pl->slots[slot].used || pl->slots[slot].releasing)
        return fail(LBM_EINVAL, "bad slot %d", slot);
    PoolSlot &S = pl->slots[slot];
    PoolGroup &G = pl->g[S.small ? 0 : 1];
    if (G.in_flight) {
        // the group's chunk in flight may still touch the slot: free it when
        // that chunk is harvested
        S.releasing = true;
        return LBM_OK;
    }
    HIPCHK(hipStreamSynchronize(G.stream));  // the slot's own set-up work
    finish_release(pl, slot);
    return LBM_OK;
}

int lbm_pool_destroy(lbm_pool_t *pl)
{
    if (!pl) return fail(LBM_ESTATE, "NULL pool");
    pool_teardown(pl);
    return LBM_OK;
}

}  // extern "C"
