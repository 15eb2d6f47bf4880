// lbm_device.hpp -- device-side building blocks of the gfx950 LBM-RANS library.
//
// Lattices, storage conversions, the wall laws with their FP64 Newton solve,
// the Spalart-Allmaras right-hand side and the boundary classification shared
// by the step, export and reduction kernels.
//
// Method: Ponsin & Lozano, arXiv 2506.03905 (Sec. 2-3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace lbmd {

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1, so
// that every lattice constant below folds into an immediate.
template <typename F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F> __host__ __device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Lattices.  Order: rest, then opposite pairs (2k-1, 2k).  D2Q9 is the paper's
// lattice (Sec. 2.1); D3Q19 is its three-dimensional counterpart.
// ---------------------------------------------------------------------------
template <int Q> struct Lat;

template <> struct Lat<9> {
    static constexpr int D = 2;
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
};
template <> struct Lat<19> {
    static constexpr int D = 3;
    static constexpr int c[19][3] = {
        {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
        {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
};

template <int Q> __host__ __device__ constexpr int cx(int i) { return Lat<Q>::c[i][0]; }
template <int Q> __host__ __device__ constexpr int cy(int i) { return Lat<Q>::c[i][1]; }
template <int Q> __host__ __device__ constexpr int cz(int i) { return Lat<Q>::c[i][2]; }
template <int Q> __host__ __device__ constexpr double wgt(int i)
{
    return Q == 9 ? (i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0))
                  : (i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0));
}
template <int Q> __host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// specular partner: same tangential components, wall-normal (y) component flipped
template <int Q> __host__ __device__ constexpr int mir(int i)
{
    int r = -1;
    for (int k = 0; k < Q; ++k)
        if (cx<Q>(k) == cx<Q>(i) && cy<Q>(k) == -cy<Q>(i) && cz<Q>(k) == cz<Q>(i)) r = k;
    return r;
}

// ---------------------------------------------------------------------------
// Storage types.  Populations are stored as deviations f_i - w_i rho0.
// ---------------------------------------------------------------------------
struct bf16s {
    uint16_t b;
};

template <typename S> struct Stor;
template <> struct Stor<double> {
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <> struct Stor<float> {
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <> struct Stor<_Float16> {
    __device__ static float ld(_Float16 v) { return static_cast<float>(v); }
    __device__ static _Float16 st(float v) { return static_cast<_Float16>(v); }
};
template <> struct Stor<bf16s> {
    __device__ static float ld(bf16s v) { return __uint_as_float(static_cast<uint32_t>(v.b) << 16); }
    // round to nearest even, NaN kept a NaN: one hardware conversion on gfx950
    __device__ static bf16s st(float v) { return bf16s{__builtin_bit_cast(uint16_t, static_cast<__bf16>(v))}; }
};

// Storage offset of population i: f_eq_i(rho0, (U, 0, 0)) - w_i rho0.  The
// stored value of population i is (f_i - w_i rho0) - shift_off<Q>(i, ...).
template <int Q, typename T> __host__ __device__ __forceinline__ T shift_off(int i, T rho0, T U)
{
    const T cu = (T)cx<Q>(i) * U;
    return (T)wgt<Q>(i) * rho0 * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * U * U);
}

// Population loads/stores.  With LBM_NT_POPS the streamed populations use
// non-temporal accesses, leaving L2 to the re-read stencil fields.
#ifndef LBM_NT_POPS
#define LBM_NT_POPS 1
#endif
#ifndef LBM_NT_LD
#define LBM_NT_LD LBM_NT_POPS
#endif
#ifndef LBM_NT_ST
#define LBM_NT_ST LBM_NT_POPS
#endif
template <typename S> __device__ __forceinline__ S ld_pop(const S *p)
{
#if LBM_NT_LD
    if constexpr (std::is_same<S, bf16s>::value) {
        bf16s r;
        r.b = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p));
        return r;
    } else {
        return __builtin_nontemporal_load(p);
    }
#else
    return *p;
#endif
}
template <typename S> __device__ __forceinline__ void st_pop(S *p, S v)
{
#if LBM_NT_ST
    if constexpr (std::is_same<S, bf16s>::value)
        __builtin_nontemporal_store(v.b, reinterpret_cast<uint16_t *>(p));
    else
        __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// ---------------------------------------------------------------------------
// Constants of the cell update, computed once on the host in double precision
// and kept in the compute type, so that the update converts nothing per cell.
// ---------------------------------------------------------------------------
template <typename T> struct CellK {
    T nu, rho0, fx, fy, fz;                           // viscosity, reference density, body force
    T cv1_3, kappa2, cb1, cw1, cw2, cw3_6, rlim, cb2; // SA constants (eq. 10-14): cv1^3, kappa^2, cw3^6
    T inv_sigma, wall_dist;
    T cf[19];    // w_i (c_i . F), the direction's share of the Guo forcing term
    T soff[19];  // storage offset of population i (zero without the storage shift)
    // the storage offsets split for the collision on stored values: sfe[0] =
    // soff[0], and for the pair k = (2k-1, 2k) the even and odd parts
    // sfe[k] = (soff[2k-1] + soff[2k]) / 2, sfo[k] = (soff[2k-1] - soff[2k]) / 2;
    // ssum = sum of soff, sj = sum of c_i soff (zero without the shift)
    T sfe[10], sfo[10];
    T ssum, sj[3];
};

// ---------------------------------------------------------------------------
// Kernel parameters (by value).
// ---------------------------------------------------------------------------
struct KP {
    int nx, ny, nz, flow;
    int64_t ncell;
    int scheme, law, sa_on, plate_start;
    int rowmap, pad_;
    int64_t nwall;
    double nu, rho0, fx, fy, fz, u_inlet;
    double kappa, B, beta;
    double reC;          // Reichardt constant C = B - ln(kappa)/kappa
    double cb1, cb2, sigma, cw1, cw2, cw3, cv1, rlim;
    double wall_u_bottom[3], wall_u_top[3];
    double shift_u;      // storage shift: stored = f - f_eq(rho0, (shift_u, 0, 0))
    void *pops;          // Q * ncell storage
    void *u[2];          // D * ncell compute type, ping-pong
    void *nt[2];         // ncell compute type, ping-pong
    void *usnap;         // D * ncell compute type (residual snapshot)
    double *utau;        // nwall
    double *tdir;        // 3 * nwall (SoA)
    double *uw;          // 3 * nwall (SoA)
    double *wrho;        // nwall: density of the wall cell at the last step
    double *ubwf;        // nwall: wall-function speed at B, u_tau u+(y_B+)
    double *gan;         // nwall: analytic wall-normal gradient (u_tau^2/nu) du+/dy+ at B
    double *partials;    // reduction partials
    double *result;      // reduction result slots
    double *mid;         // reduction middle-pass rows
    double *ibuf;        // Q * nwall: post-collision populations of the wall cells (interpolated links)
    double wall_dist;    // distance of the first node from the wall (1/2: halfway)
    int bb_interp;       // IBB_HALFWAY / IBB_BOUZIDI / IBB_YU
    int shifted;         // storage shift on (shift_u != 0)
    CellK<double> kd;    // cell-update constants, FP64 path
    CellK<float> kf;     // the same in FP32 (FP32, FP16 and BF16 storage)
};

template <typename T> __host__ __device__ __forceinline__ const CellK<T> &ck(const KP &P);
template <> __host__ __device__ __forceinline__ const CellK<double> &ck<double>(const KP &P) { return P.kd; }
template <> __host__ __device__ __forceinline__ const CellK<float> &ck<float>(const KP &P) { return P.kf; }

constexpr int FLOW_CHANNEL = 0, FLOW_PLATE = 1;
constexpr int WALL_FIXED = 0, WALL_SLIP = 1, WALL_HRFD = 2, WALL_CD = 3;
constexpr int IBB_HALFWAY = 0, IBB_BOUZIDI = 1, IBB_YU = 2;
constexpr int LAW_REICHARDT = 0, LAW_SA = 1;

// wall index of a boundary cell (or -1)
__device__ __forceinline__ int64_t wall_index(const KP &P, int x, int y, int z)
{
    if (P.flow == FLOW_CHANNEL) {
        if (y == 0) return x + (int64_t)P.nx * z;
        if (y == P.ny - 1) return (int64_t)P.nx * P.nz + x + (int64_t)P.nx * z;
        return -1;
    }
    if (y == 0 && x >= P.plate_start) return x - P.plate_start;
    return -1;
}

// Does a population leaving cell x through the bottom face, with x-velocity
// component cx_out, hit the plate?  It crosses y = 0 at X = x + 1/2 + cx_out/2
// (cell-edge coordinates); the plate covers X >= plate_start, the leading-edge
// point included.  For a population arriving at x through the bottom face
// with x-velocity cx_in, the emitting link is the one with cx_out = -cx_in
// (bounce-back) or the mirrored one of the neighbour, both giving the same X.
// A link leaving cell x of the bottom row with x-velocity cx_out crosses the
// bottom at X = x + 1/2 + cx_out/2: a wall on the plate (X >= plate_start, the
// leading-edge point included), a symmetry plane upstream.  The halfway
// crossing point is used for every wall distance, so that a link and its
// specular image agree and the AA streaming stays a bijection.
__device__ __forceinline__ bool bottom_is_wall(const KP &P, int x, int cx_out)
{
    if (P.flow == FLOW_CHANNEL) return true;
    return 2 * x + 1 + cx_out >= 2 * P.plate_start;
}

// Reciprocal, division, square root and x^(1/6) of the cell update.  With
// FP64 storage they stay correctly rounded (element-wise parity with the
// oracle); the FP32 path uses the hardware approximations (about 1 ulp, far
// inside its tolerance), which cut the instruction count of the update.
template <typename T> struct Num {
    static __device__ __forceinline__ T rcp(T x) { return (T)1 / x; }
    static __device__ __forceinline__ T div(T a, T b) { return a / b; }
    static __device__ __forceinline__ T sqrt_(T x) { return sqrt(x); }
    static __device__ __forceinline__ T root6(T x) { return sqrt(cbrt(x)); }
};
template <> struct Num<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float root6(float x)
    {
        return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 6.0f));
    }
};

// ---------------------------------------------------------------------------
// Wall laws (double).
// ---------------------------------------------------------------------------
// SA-consistent law, eq. 16, with atan2 for arctan(b/(y+a)) and B-bar read
// as 5.0333908790505579 so that u+(0) = 0.
__device__ __forceinline__ double uplus_sa(double y)
{
    const double Bb = 5.0333908790505579, a1 = 8.148221580024245, a2 = -6.9287093849022945;
    const double b1 = 7.4600876082527945, b2 = 7.468145790401841;
    const double c1 = 2.5496773539754747, c2 = 1.3301651588535228, c3 = 3.599459109332379,
                 c4 = 3.639753186868684494;
    double p1 = y + a1, p2 = y + a2;
    return Bb + c1 * log(p1 * p1 + b1 * b1) - c2 * log(p2 * p2 + b2 * b2) - c3 * atan2(b1, p1) -
           c4 * atan2(b2, p2);
}
// eq. 15
__device__ __forceinline__ double duplus_sa(double y)
{
    const double cv13 = 7.1 * 7.1 * 7.1;
    double k = 0.41 * y, k3 = k * k * k;
    return (cv13 + k3) / (cv13 + (1.0 + k) * k3);
}
// Reichardt's law with C = B - ln(kappa)/kappa (log-law intercept B)
__device__ __forceinline__ double uplus_re(double y, double kappa, double C)
{
    return log1p(kappa * y) / kappa + C * (1.0 - exp(-y * (1.0 / 11.0)) - y * (1.0 / 11.0) * exp(-y * (1.0 / 3.0)));
}
__device__ __forceinline__ double duplus_re(double y, double kappa, double C)
{
    double e3 = exp(-y * (1.0 / 3.0));
    return 1.0 / (1.0 + kappa * y) + C * (exp(-y * (1.0 / 11.0)) * (1.0 / 11.0) - e3 * (1.0 / 11.0) + y * (1.0 / 33.0) * e3);
}
__device__ __forceinline__ double uplus(const KP &P, double y)
{
    return P.law == LAW_SA ? uplus_sa(y) : uplus_re(y, P.kappa, P.reC);
}
__device__ __forceinline__ double duplus(const KP &P, double y)
{
    return P.law == LAW_SA ? duplus_sa(y) : duplus_re(y, P.kappa, P.reC);
}
// u+ and du+/dy+ together (shared exponentials for Reichardt's law)
__device__ __forceinline__ void uplus_both(const KP &P, double y, double &u, double &du)
{
    if (P.law == LAW_SA) {
        u = uplus_sa(y);
        du = duplus_sa(y);
        return;
    }
    const double k = P.kappa, C = P.reC;
    // e^{-y/11} = a^3 and e^{-y/3} = a^11 with a = e^{-y/33}: one exponential
    const double a = exp(-y * (1.0 / 33.0)), a2 = a * a, a3 = a2 * a, a8 = (a2 * a2) * (a2 * a2);
    const double e11 = a3, e3 = a8 * a3;
    u = log1p(k * y) / k + C * (1.0 - e11 - y * (1.0 / 11.0) * e3);
    du = 1.0 / (1.0 + k * y) + C * ((e11 - e3) * (1.0 / 11.0) + y * (1.0 / 33.0) * e3);
}

// Friction velocity from u_t = u_tau u+(y u_tau / nu) (Sec. 3.1): Newton in
// FP64 from a warm start, safeguarded by a bracket of the unique root (G is
// increasing).  Quadratic convergence: the error left after a correction of
// relative size d is about c d^2 with c = |G'' u / 2 G'| of order one, so a
// correction below 1e-7 of u_tau leaves an error near 1e-14 and ends the
// iteration (a warm start from the previous step usually needs one step).
__device__ __forceinline__ double solve_utau(const KP &P, double ut, double y, double warm)
{
    if (!(ut > 0.0)) return 0.0;
    const double nu = P.nu;
    double u = warm > 0.0 ? warm : sqrt(nu * ut / y);
    double lo = 0.0, hi = 1.0e300;
    for (int it = 0; it < 100; ++it) {
        const double yp = y * u / nu;
        double up, dup;
        uplus_both(P, yp, up, dup);
        const double g = u * up - ut;
        if (g == 0.0) return u;
        if (g < 0.0)
            lo = u;
        else
            hi = u;
        double un = u - g / (up + yp * dup);
        const bool inside = un > lo && un < hi;
        if (!inside) un = hi < 1.0e299 ? 0.5 * (lo + hi) : 2.0 * u;
        if (inside && fabs(un - u) <= 1.0e-7 * un) return un;
        u = un;
    }
    return u;
}

// ---------------------------------------------------------------------------
// Spalart-Allmaras right-hand side (eq. 10-14) at one node.  ntm/ntp: minus /
// plus neighbours per axis; g[c][a] = d u_c / d x_a by central differences.
// ---------------------------------------------------------------------------
template <int D, typename T>
__device__ __forceinline__ T sa_rhs(const KP &P, T nt0, const T *ntm, const T *ntp, const T *u0,
                                    const T (*g)[3], T d)
{
    const CellK<T> &K = ck<T>(P);
    const T nu = K.nu;
    T conv = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) conv += u0[a] > (T)0 ? u0[a] * (nt0 - ntm[a]) : u0[a] * (ntp[a] - nt0);
    T S;
    if (D == 2) {
        S = fabs(g[1][0] - g[0][1]);
    } else {
        T wx = g[2][1] - g[1][2], wy = g[0][2] - g[2][0], wz = g[1][0] - g[0][1];
        S = Num<T>::sqrt_(wx * wx + wy * wy + wz * wz);
    }
    using N = Num<T>;
    T chi = N::div(nt0, nu), chi3 = chi * chi * chi;
    T fv1 = N::div(chi3, chi3 + K.cv1_3);
    T fv2 = (T)1 - N::div(chi, (T)1 + chi * fv1);
    T kd2 = K.kappa2 * d * d;
    T St = S + N::div(nt0, kd2) * fv2;
    T Pr, r;
    if (St > (T)0) {
        Pr = K.cb1 * St * nt0;
        r = N::div(nt0, St * kd2);
        r = r > K.rlim ? K.rlim : r;
    } else {
        Pr = 0;
        r = K.rlim;
    }
    T r2 = r * r;
    T gg = r + K.cw2 * (r2 * r2 * r2 - r);
    T g2 = gg * gg, g6 = g2 * g2 * g2;
    const T c6 = K.cw3_6;
    T ratio = N::div((T)1 + c6, g6 + c6);
    T fw = gg * N::root6(ratio);
    const T ntd = N::div(nt0, d);
    T Ds = K.cw1 * fw * ntd * ntd;
    T diff = 0, grad2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        diff += (nu + (T)0.5 * (ntp[a] + nt0)) * (ntp[a] - nt0) - (nu + (T)0.5 * (nt0 + ntm[a])) * (nt0 - ntm[a]);
        T ga = (T)0.5 * (ntp[a] - ntm[a]);
        grad2 += ga * ga;
    }
    return -conv + Pr - Ds + (diff + K.cb2 * grad2) * K.inv_sigma;
}

// ---------------------------------------------------------------------------
// Central-moment collision (eq. 7, Sec. 2.1) in closed form, deviation form.
// Post-collision central moments: rho; F/2 (first order); rho cs2 delta +
// (1 - omega) dev(k) (second order: deviatoric part relaxed with omega, trace
// to equilibrium); cs2 F_b / 2 for (2 e_a + e_b); rho cs2^2 for (2 e_a + 2 e_b).
// They are shifted back to raw moments with u and mapped to populations with
// the inverse of the (constant) raw-moment matrix of the lattice:
//   rest      f0 = m0 - sum_a m_aa + sum_{a<b} m_aabb
//   face +-a  f  = ((m_aa - sum_b m_aabb) +- (m_a - sum_b m_abb)) / 2
//   edge ab   f  = (m_aabb + s m_abb + t m_aab + s t m_ab) / 4, (s, t) = (c_a, c_b)
// f: deviations f - w rho0 on entry, post-collision deviations on exit.
// ---------------------------------------------------------------------------
template <int Q, typename T>
__host__ __device__ __forceinline__ void cm_collide(T *f, T drho, T rho, const T *u, const T *F, T omega)
{
    constexpr int D = Lat<Q>::D;
    const T c2 = (T)(1.0 / 3.0), c4 = (T)(1.0 / 9.0);
    // raw second moments of the deviations
    T P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int c[3] = {cx<Q>(i), cy<Q>(i), cz<Q>(i)};
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                if (c[a] * c[b] != 0) P[a][b] += (T)(c[a] * c[b]) * f[i];
    });
    // central second moments without the isotropic rho0 cs2 part:
    // k_ab = Pi_ab - rho u_a u_b + (u_a F_b + u_b F_a)/2
    T k[3][3];
    T tr = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            k[a][b] = P[a][b] - rho * u[a] * u[b] + (T)0.5 * (u[a] * F[b] + u[b] * F[a]);
            if (a == b) tr += k[a][a];
        }
    const T rel = (T)1 - omega;
    // post-collision central moments: K2 = second order (without rho cs2 on the
    // diagonal, added below), k1 = first order
    T K2[3][3], k1[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        k1[a] = (T)0.5 * F[a];
#pragma unroll
        for (int b = a; b < D; ++b) K2[a][b] = rel * (a == b ? k[a][a] - tr / (T)D : k[a][b]);
    }
    // raw moments of the post-collision deviations (rho0 parts removed):
    //   m0 = drho; m_a = rho u_a + F_a/2
    //   m_aa  = drho cs2 + K2_aa + 2 u_a k1_a + rho u_a^2
    //   m_ab  = K2_ab + u_a k1_b + u_b k1_a + rho u_a u_b
    //   m_aab = cs2 F_b/2 + u_b Kaa + 2 u_a K2_ab + 2 u_a u_b k1_a + u_a^2 k1_b + rho u_a^2 u_b
    //   m_aabb = drho cs2^2 + 2 u_b K_aab + u_b^2 Kaa + 2 u_a K_abb + 4 u_a u_b K2_ab
    //            + 2 u_a u_b^2 k1_a + u_a^2 Kbb + 2 u_a^2 u_b k1_b + rho u_a^2 u_b^2
    //   with Kaa = rho cs2 + K2_aa the full post-collision central moment.
    T ma[3], maa[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ma[a] = rho * u[a] + k1[a];
        maa[a] = drho * c2 + K2[a][a] + (T)2 * u[a] * k1[a] + rho * u[a] * u[a];
    }
    T mab[3][3], maab[3][3], maabb[3][3];  // [a][b] with a != b; maab[a][b] = m_{a a b}
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            if (a == b) continue;
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            const T Kab = K2[lo][hi];
            const T Kaa = rho * c2 + K2[a][a];
            mab[a][b] = Kab + u[a] * k1[b] + u[b] * k1[a] + rho * u[a] * u[b];
            maab[a][b] = c2 * (T)0.5 * F[b] + u[b] * Kaa + (T)2 * u[a] * Kab + (T)2 * u[a] * u[b] * k1[a] +
                         u[a] * u[a] * k1[b] + rho * u[a] * u[a] * u[b];
        }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) {
            const T Kab = K2[a][b];
            const T Kaa = rho * c2 + K2[a][a], Kbb = rho * c2 + K2[b][b];
            const T Kaab = c2 * (T)0.5 * F[b], Kabb = c2 * (T)0.5 * F[a];
            const T v = drho * c4 + (T)2 * u[b] * Kaab + u[b] * u[b] * Kaa + (T)2 * u[a] * Kabb +
                        (T)4 * u[a] * u[b] * Kab + (T)2 * u[a] * u[b] * u[b] * k1[a] + u[a] * u[a] * Kbb +
                        (T)2 * u[a] * u[a] * u[b] * k1[b] + rho * u[a] * u[a] * u[b] * u[b];
            // the rho0 cs2^2 part of the deviation moment: Kaa u_b^2 etc. carry rho cs2,
            // rho = rho0 + drho, so only drho enters the constant term above
            maabb[a][b] = maabb[b][a] = v;
        }
    // populations
    sfor<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int c[3] = {cx<Q>(i), cy<Q>(i), cz<Q>(i)};
        constexpr int nnz = (c[0] != 0) + (c[1] != 0) + (c[2] != 0);
        if constexpr (nnz == 0) {
            T v = drho;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                v -= maa[a];
#pragma unroll
                for (int b = a + 1; b < D; ++b) v += maabb[a][b];
            }
            f[i] = v;
        } else if constexpr (nnz == 1) {
            constexpr int a = c[0] != 0 ? 0 : (c[1] != 0 ? 1 : 2);
            T even = maa[a], odd = ma[a];
#pragma unroll
            for (int b = 0; b < D; ++b) {
                if (b == a) continue;
                even -= maabb[a][b];
                odd -= maab[b][a];  // m_{a b b}
            }
            f[i] = (T)0.5 * (even + (T)c[a] * odd);
        } else {
            constexpr int a = c[0] != 0 ? 0 : 1;
            constexpr int b = c[2] != 0 ? 2 : 1;
            constexpr int s = c[a], t = c[b];
            f[i] = (T)0.25 * (maabb[a][b] + (T)s * maab[b][a] + (T)t * maab[a][b] + (T)(s * t) * mab[a][b]);
        }
    });
}

template <typename T> __device__ __forceinline__ T nut_of(const KP &P, T nt)
{
    const CellK<T> &K = ck<T>(P);
    T chi = Num<T>::div(nt, K.nu), chi3 = chi * chi * chi;
    return Num<T>::div(nt * chi3, chi3 + K.cv1_3);
}

// distance to the closest wall of a cell centre (Sec. 2.2)
// Distance to the closest wall: node y lies y + d_w above the bottom wall, the
// channel's top wall d_w above node ny - 1; the plate's leading-edge point
// sits at x = plate_start on the wall plane (node x at x + 1/2).
template <typename T> __device__ __forceinline__ T wall_dist(const KP &P, int x, int y)
{
    const T dw = ck<T>(P).wall_dist;
    T yc = (T)y + dw;
    if (P.flow == FLOW_CHANNEL) {
        T yt = (T)(P.ny - 1 - y) + dw;
        return yc < yt ? yc : yt;
    }
    T dx = (T)P.plate_start - ((T)x + (T)0.5);
    if (dx <= (T)0) return yc;
    return sqrt(dx * dx + yc * yc);
}

}  // namespace lbmd
