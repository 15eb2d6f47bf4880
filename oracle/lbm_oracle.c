/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the LBM-RANS hot path.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg of the
 * benchmark).  It shares no code with the HIP library.
 *
 * Method: Ponsin & Lozano, arXiv 2506.03905.  One time step follows the
 * paper's order -- collision with nu_eff from the previous step (Sec. 2.1,
 * eq. 2, 7-8 and Sec. 3.1 around eq. 26), streaming (eq. 3), wall treatment
 * (eq. 31/35 or eq. 19/23/26-28), moments (eq. 4-5), the wall-function solve
 * for u_tau (Sec. 3.1, eq. 20-22) and the Spalart-Allmaras update
 * (Sec. 2.2, eq. 10-14).  Where the paper leaves a choice open the reading is
 * stated next to the code.  Readings in force:
 *   - collision is BGK (the paper's base model, Sec. 2.1) with the
 *     second-order equilibrium and Guo forcing weighted by (1 - omega/2),
 *     the BGK form of the (I - Lambda/2) R source of eq. 7, or the
 *     central-moment operator of eq. 7 itself (orc_collide_cm: T built from
 *     the definition of the central moments, T f* = k* solved by Gaussian
 *     elimination);
 *   - the velocity is the half-force-shifted first moment (eq. 5);
 *   - rho_w in eq. 31 is the post-collision density of the boundary cell;
 *   - the u_tau reference node F is the second node off the wall (Sec. 3.1),
 *     y_F = 1.5, y_B = 0.5 in lattice units, for both wall schemes;
 *   - SA: forward Euler with dt = 1, one update per LBM step, vorticity by
 *     central differences of the previous step's velocity, first-order upwind
 *     convection, conservative diffusion with face value nu + mean(nu_tilde),
 *     c_b2 term by central differences, no trip term, production switched
 *     off and r = r_lim when S_tilde <= 0, nu_tilde clipped at 0;
 *   - eq. 35 uses nu_t|B = nu kappa y_B+ and Delta_w = y_B, with the LBM
 *     velocity at B from the previous step.
 * Pins: every routine is checked against closed forms, invariants or the
 * paper's tables on the CPU, and a set of planted single-line mistakes must
 * each fail one of those checks.  The coupled step as a whole has no closed
 * form; its parity rests on those pieces.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads: the per-cell loops are shared out by rows (OpenMP) on lattices of
 * at least ORC_PAR_MIN cells.  Every cell's arithmetic is the same whatever
 * thread runs it, and no loop sums across cells, so any thread count gives
 * bitwise the same result. */
#define ORC_PAR_MIN 16384
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define CS2 (1.0 / 3.0)

/* ---------------------------------------------------------------------- */
/* Lattices: D2Q9 (the paper's, Sec. 2.1) and D3Q19.  Order: rest, then    */
/* opposite pairs (2k-1, 2k).                                              */
/* ---------------------------------------------------------------------- */
static const int D2Q9_C[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const int D3Q19_C[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

int orc_lattice(int q, int *c, double *w, int *opp)
{
    const int(*cc)[3];
    if (q == 9)
        cc = D2Q9_C;
    else if (q == 19)
        cc = D3Q19_C;
    else
        return -1;
    for (int i = 0; i < q; ++i) {
        int s = abs(cc[i][0]) + abs(cc[i][1]) + abs(cc[i][2]);
        for (int a = 0; a < 3; ++a) c[3 * i + a] = cc[i][a];
        if (q == 9)
            w[i] = s == 0 ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else
            w[i] = s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    for (int i = 0; i < q; ++i) {
        opp[i] = -1;
        for (int j = 0; j < q; ++j)
            if (cc[j][0] == -cc[i][0] && cc[j][1] == -cc[i][1] && cc[j][2] == -cc[i][2]) opp[i] = j;
    }
    return 0;
}

/* second-order equilibrium, c_s^2 = 1/3 */
void orc_feq(int q, double rho, const double *u, double *feq)
{
    int c[19 * 3], opp[19];
    double w[19];
    orc_lattice(q, c, w, opp);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < q; ++i) {
        double cu = c[3 * i] * u[0] + c[3 * i + 1] * u[1] + c[3 * i + 2] * u[2];
        feq[i] = w[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Moments (eq. 4-5) and BGK collision with Guo forcing (eq. 2; omega = 1/tau
 * from eq. 8).  The forcing population is (1 - omega/2) w_i [ (c_i - u)/cs2 +
 * (c_i.u) c_i / cs2^2 ] . F. */
void orc_collide(int q, const double *f, double tau, const double *force, double *fpost,
                 double *rho_out, double *u_out)
{
    int c[19 * 3], opp[19];
    double w[19], feq[19];
    orc_lattice(q, c, w, opp);
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) m[a] += f[i] * c[3 * i + a];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * force[a]) / rho;
    orc_feq(q, rho, u, feq);
    double omega = 1.0 / tau;
    for (int i = 0; i < q; ++i) {
        double cu = c[3 * i] * u[0] + c[3 * i + 1] * u[1] + c[3 * i + 2] * u[2];
        double src = 0.0;
        for (int a = 0; a < 3; ++a) src += ((c[3 * i + a] - u[a]) / CS2 + cu * c[3 * i + a] / (CS2 * CS2)) * force[a];
        src *= (1.0 - 0.5 * omega) * w[i];
        fpost[i] = f[i] - omega * (f[i] - feq[i]) + src;
    }
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

/* Central-moment collision, eq. 7 (Sec. 2.1): k = T f with
 * T_ji = prod_a (c_ia - u_a)^{p_ja}; k* = (I - Lambda) k + Lambda k_eq +
 * (I - Lambda/2) R; f* = T^{-1} k*.  Lambda relaxes the deviatoric second-order
 * central moments with omega and every other moment with 1 (for D2Q9 this is
 * Lambda = diag[1,1,1,1,omega,omega,1,1,1] in the basis of eq. 7; D3Q19 uses the
 * same rule on its 19 central moments).  k_eq are the central moments of the
 * Maxwellian (fourth-order Hermite equilibrium): rho, 0, rho cs2 delta, 0,
 * rho cs2^2; R are those of the forcing term: F in first order, cs2 F_b for
 * the moment (2 e_a + e_b), zero otherwise.  f* is found by Gaussian
 * elimination, T being u-dependent. */
static const int CM_B9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {2, 0, 0}, {0, 2, 0},
                                {1, 1, 0}, {2, 1, 0}, {1, 2, 0}, {2, 2, 0}};
static const int CM_B19[19][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
                                  {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1},
                                  {1, 0, 2}, {0, 1, 2}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}};

static double ipow(double b, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= b;
    return r;
}

/* solves A x = b in place (n <= 19), partial pivoting; returns 0 on success */
static int gauss_solve(int n, double A[19][19], double *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double m = A[r][c] / A[c][c];
            if (m == 0.0) continue;
            for (int k = c; k < n; ++k) A[r][k] -= m * A[c][k];
            b[r] -= m * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r][k] * b[k];
        b[r] = s / A[r][r];
    }
    return 0;
}

void orc_collide_cm(int q, const double *f, double tau, const double *force, double *fpost,
                    double *rho_out, double *u_out)
{
    int c[19 * 3], opp[19];
    double w[19];
    orc_lattice(q, c, w, opp);
    const int D = q == 9 ? 2 : 3;
    const int(*P)[3] = q == 9 ? CM_B9 : CM_B19;
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) m[a] += f[i] * c[3 * i + a];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * force[a]) / rho;
    double T[19][19], k[19], ks[19];
    for (int j = 0; j < q; ++j) {
        k[j] = 0.0;
        for (int i = 0; i < q; ++i) {
            T[j][i] = 1.0;
            for (int a = 0; a < 3; ++a) T[j][i] *= ipow(c[3 * i + a] - u[a], P[j][a]);
            k[j] += T[j][i] * f[i];
        }
    }
    double omega = 1.0 / tau;
    double tr = 0.0; /* trace of the second-order central moments */
    for (int j = 0; j < q; ++j)
        if (P[j][0] + P[j][1] + P[j][2] == 2)
            for (int a = 0; a < D; ++a)
                if (P[j][a] == 2) tr += k[j];
    for (int j = 0; j < q; ++j) {
        int ord = P[j][0] + P[j][1] + P[j][2];
        if (ord == 0) {
            ks[j] = rho;
        } else if (ord == 1) {
            int a = P[j][0] ? 0 : (P[j][1] ? 1 : 2);
            ks[j] = 0.5 * force[a]; /* (1 - 1) k + 1 * 0 + (1 - 1/2) F_a */
        } else if (ord == 2) {
            int diag = P[j][0] == 2 || P[j][1] == 2 || P[j][2] == 2;
            if (diag)
                ks[j] = rho * CS2 + (1.0 - omega) * (k[j] - tr / D);
            else
                ks[j] = (1.0 - omega) * k[j];
        } else if (ord == 3) {
            /* moment (2 e_a + e_b): forcing central moment cs2 F_b, relaxed with 1 */
            int b = P[j][0] == 1 ? 0 : (P[j][1] == 1 ? 1 : 2);
            ks[j] = 0.5 * CS2 * force[b];
        } else {
            ks[j] = rho * CS2 * CS2;
        }
    }
    for (int j = 0; j < q; ++j) fpost[j] = ks[j];
    gauss_solve(q, T, fpost);
    if (rho_out) *rho_out = rho;
    if (u_out)
        for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

/* ---------------------------------------------------------------------- */
/* Wall laws.                                                              */
/* ---------------------------------------------------------------------- */
/* SA-consistent law, eq. 16.  Readings: arctan(b/(y+a)) is taken as
 * atan2(b, y+a) (the branch that keeps u+ continuous where y+a2 = 0) and the
 * printed B-bar is read as 5.0333908790505579 (one dropped digit), which
 * makes u+(0) = 0 as the derivation requires. */
static const double SA_BBAR = 5.0333908790505579;
static const double SA_A1 = 8.148221580024245, SA_A2 = -6.9287093849022945;
static const double SA_B1 = 7.4600876082527945, SA_B2 = 7.468145790401841;
static const double SA_C1 = 2.5496773539754747, SA_C2 = 1.3301651588535228;
static const double SA_C3 = 3.599459109332379, SA_C4 = 3.639753186868684494;

double orc_uplus(int law, double yp, double kappa, double B)
{
    if (law == ORC_SA_LAW) {
        return SA_BBAR + SA_C1 * log((yp + SA_A1) * (yp + SA_A1) + SA_B1 * SA_B1) -
               SA_C2 * log((yp + SA_A2) * (yp + SA_A2) + SA_B2 * SA_B2) - SA_C3 * atan2(SA_B1, yp + SA_A1) -
               SA_C4 * atan2(SA_B2, yp + SA_A2);
    }
    /* Reichardt: ln(1 + kappa y+)/kappa + C (1 - e^{-y+/11} - (y+/11) e^{-y+/3});
     * C chosen so the log-law intercept is B: C = B - ln(kappa)/kappa. */
    double C = B - log(kappa) / kappa;
    return log(1.0 + kappa * yp) / kappa + C * (1.0 - exp(-yp / 11.0) - (yp / 11.0) * exp(-yp / 3.0));
}

double orc_duplus(int law, double yp, double kappa, double B)
{
    if (law == ORC_SA_LAW) {
        /* eq. 15, written for the SA constants kappa = 0.41, c_v1 = 7.1 */
        double cv1 = 7.1, ky = 0.41 * yp;
        (void)kappa;
        return (cv1 * cv1 * cv1 + ky * ky * ky) / (cv1 * cv1 * cv1 + (1.0 + ky) * ky * ky * ky);
    }
    double C = B - log(kappa) / kappa;
    return 1.0 / (1.0 + kappa * yp) +
           C * (exp(-yp / 11.0) / 11.0 - exp(-yp / 3.0) / 11.0 + (yp / 33.0) * exp(-yp / 3.0));
}

/* The friction velocity solves u_t = u_tau u+(y u_tau / nu) (Sec. 3.1, the
 * wall law at node F).  G(u_tau) is strictly increasing, so the root is
 * unique; the oracle finds it by plain bisection down to adjacent doubles. */
double orc_solve_utau(int law, double ut, double y, double nu, double kappa, double B)
{
    if (!(ut > 0.0)) return 0.0;
    double lo = 0.0, hi = ut > sqrt(nu * ut / y) ? ut : sqrt(nu * ut / y);
    while (hi * orc_uplus(law, y * hi / nu, kappa, B) - ut < 0.0) hi *= 2.0;
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (mid * orc_uplus(law, y * mid / nu, kappa, B) - ut < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    double glo = fabs(lo * orc_uplus(law, y * lo / nu, kappa, B) - ut);
    double ghi = fabs(hi * orc_uplus(law, y * hi / nu, kappa, B) - ut);
    return glo < ghi ? lo : hi;
}

/* ---------------------------------------------------------------------- */
/* Spalart-Allmaras (Sec. 2.2).                                            */
/* ---------------------------------------------------------------------- */
double orc_nut(const orc_params *p, double nt)
{
    /* eq. 10 */
    double chi = nt / p->nu, chi3 = chi * chi * chi, cv13 = p->cv1 * p->cv1 * p->cv1;
    return nt * chi3 / (chi3 + cv13);
}

/* Right-hand side of eq. 11 at one node, discretized as described after
 * eq. 14.  ntm/ntp: nu_tilde at the minus/plus neighbour along each axis;
 * um/up: velocity at those neighbours, [axis*3 + component]; u0 the velocity
 * at the node; d the wall distance. */
double orc_sa_rhs(const orc_params *p, int D, double nt0, const double *ntm, const double *ntp,
                  const double *u0, const double *um, const double *up, double d)
{
    double nu = p->nu, k = p->kappa;
    double cw1 = p->cb1 / (k * k) + (1.0 + p->cb2) / p->sigma; /* constants after eq. 14 */
    /* convection: first-order upwind */
    double conv = 0.0;
    for (int a = 0; a < D; ++a) {
        double ua = u0[a];
        if (ua > 0.0)
            conv += ua * (nt0 - ntm[a]);
        else
            conv += ua * (ntp[a] - nt0);
    }
    /* vorticity magnitude from central differences: g[c][a] = d u_c / d x_a */
    double g[3][3] = {{0}};
    for (int a = 0; a < D; ++a)
        for (int c = 0; c < 3; ++c) g[c][a] = 0.5 * (up[3 * a + c] - um[3 * a + c]);
    double S;
    if (D == 2) {
        S = fabs(g[1][0] - g[0][1]);
    } else {
        double wx = g[2][1] - g[1][2], wy = g[0][2] - g[2][0], wz = g[1][0] - g[0][1];
        S = sqrt(wx * wx + wy * wy + wz * wz);
    }
    /* eq. 10, 13 */
    double chi = nt0 / nu, chi3 = chi * chi * chi, cv13 = p->cv1 * p->cv1 * p->cv1;
    double fv1 = chi3 / (chi3 + cv13);
    double fv2 = 1.0 - chi / (1.0 + chi * fv1);
    double St = S + nt0 / (k * k * d * d) * fv2;
    /* eq. 12, 14 */
    double P, r;
    if (St > 0.0) {
        P = p->cb1 * St * nt0;
        r = nt0 / (St * k * k * d * d);
        if (r > p->rlim) r = p->rlim;
    } else {
        P = 0.0;
        r = p->rlim;
    }
    double g6 = 0.0, gg = r + p->cw2 * (pow(r, 6.0) - r);
    g6 = pow(gg, 6.0);
    double cw36 = pow(p->cw3, 6.0);
    double fw = gg * pow((1.0 + cw36) / (g6 + cw36), 1.0 / 6.0);
    double Dst = cw1 * fw * (nt0 / d) * (nt0 / d);
    /* diffusion, conservative form, and the c_b2 gradient-squared term */
    double diff = 0.0, grad2 = 0.0;
    for (int a = 0; a < D; ++a) {
        diff += (nu + 0.5 * (ntp[a] + nt0)) * (ntp[a] - nt0) - (nu + 0.5 * (nt0 + ntm[a])) * (nt0 - ntm[a]);
        double ga = 0.5 * (ntp[a] - ntm[a]);
        grad2 += ga * ga;
    }
    return -conv + P - Dst + (diff + p->cb2 * grad2) / p->sigma;
}

/* ---------------------------------------------------------------------- */
/* Boundary building blocks.                                               */
/* ---------------------------------------------------------------------- */
/* Zou-He velocity inlet on a west face, u = (U, 0) (D2Q9, no body force):
 * density from the known populations, then the three unknown ones (c_x > 0)
 * from the non-equilibrium bounce-back closure. */
void orc_zou_he_west(double *f, double U)
{
    double rho = (f[0] + f[3] + f[4] + 2.0 * (f[2] + f[6] + f[8])) / (1.0 - U);
    f[1] = f[2] + (2.0 / 3.0) * rho * U;
    f[5] = f[6] - 0.5 * (f[3] - f[4]) + (1.0 / 6.0) * rho * U;
    f[7] = f[8] + 0.5 * (f[3] - f[4]) + (1.0 / 6.0) * rho * U;
}

/* eq. 19 with eq. 17 and eq. 26: f_i = f_eq(rho, u) - w_i rho tau / cs2 Q_i:S */
void orc_regularized(int q, double rho, const double *u, const double *S, double tau, double *f)
{
    int c[19 * 3], opp[19];
    double w[19], feq[19];
    orc_lattice(q, c, w, opp);
    orc_feq(q, rho, u, feq);
    for (int i = 0; i < q; ++i) {
        double QS = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                QS += ((double)c[3 * i + a] * c[3 * i + b] - (a == b ? CS2 : 0.0)) * S[3 * a + b];
        f[i] = feq[i] - w[i] * rho * tau / CS2 * QS;
    }
}

/* ---------------------------------------------------------------------- */
/* The lattice.                                                            */
/* ---------------------------------------------------------------------- */
struct orc {
    orc_params p;
    int D;
    int64_t ncell, nwall, steps;
    int c[19 * 3], opp[19];
    double w[19];
    double *fpost, *fnew;       /* q*ncell */
    double *u_prev, *u_cur;     /* 3*ncell (z component zero in 2-D) */
    double *rho;                /* ncell: density of the last step */
    double *nt, *nt_next;       /* ncell */
    int64_t *wall_of;           /* ncell -> wall index or -1 */
    int64_t *wB, *wF, *wFF;     /* nwall */
    int *wside;                 /* -1: wall below (n = -y), +1: wall above */
    double *utau, *tdir, *uw;   /* nwall, 3*nwall, 3*nwall */
};

static int64_t cidx(const orc *o, int x, int y, int z) { return x + (int64_t)o->p.nx * (y + (int64_t)o->p.ny * z); }
static int wrapi(int a, int n) { return ((a % n) + n) % n; }

/* wall distance (Sec. 2.2: distance to the closest wall).  Node y lies
 * y + d_w above the bottom wall (d_w = wall_dist, 1/2 for halfway walls); the
 * channel's top wall lies d_w above node ny - 1; the plate's leading-edge
 * point is at x = plate_start on the wall plane (node x at x + 1/2). */
static double wall_distance(const orc *o, int x, int y)
{
    const double dw = o->p.wall_dist;
    double yc = y + dw;
    if (o->p.flow == ORC_CHANNEL) {
        double yt = (o->p.ny - 1 - y) + dw;
        return yc < yt ? yc : yt;
    }
    double xc = x + 0.5, dx = o->p.plate_start - xc;
    if (dx <= 0.0) return yc;
    return sqrt(dx * dx + yc * yc);
}

/* Dirichlet nodes of the SA field: wall cells and the plate's inlet column */
static int sa_dirichlet(const orc *o, int64_t cell, int x)
{
    if (o->wall_of[cell] >= 0) return 1;
    if (o->p.flow == ORC_PLATE && x == 0) return 1;
    return 0;
}

/* Wall function at every wall cell from the current velocity u_cur:
 * Newton-free (bisection) solve for u_tau at F, slip velocity eq. 35 and the
 * SA Dirichlet value nu_tilde_B = nu kappa y_B+ (Sec. 2.2). */
static void wall_function(orc *o, double *nt_out)
{
    const orc_params *p = &o->p;
    const double yB = p->wall_dist, yF = 1.0 + p->wall_dist; /* Sec. 3.1: B and F */
#pragma omp parallel for schedule(static) if (o->nwall >= ORC_PAR_MIN / 16)
    for (int64_t w = 0; w < o->nwall; ++w) {
        double n[3] = {0.0, (double)o->wside[w], 0.0};
        double uF[3], uB[3];
        for (int a = 0; a < 3; ++a) {
            uF[a] = o->u_cur[3 * o->wF[w] + a];
            uB[a] = o->u_cur[3 * o->wB[w] + a];
        }
        double uFn = uF[0] * n[0] + uF[1] * n[1] + uF[2] * n[2];
        double uBn = uB[0] * n[0] + uB[1] * n[1] + uB[2] * n[2];
        double uFt[3], uBt[3];
        for (int a = 0; a < 3; ++a) {
            uFt[a] = uF[a] - uFn * n[a];
            uBt[a] = uB[a] - uBn * n[a];
        }
        double ut = sqrt(uFt[0] * uFt[0] + uFt[1] * uFt[1] + uFt[2] * uFt[2]);
        double t[3] = {1.0, 0.0, 0.0};
        if (ut > 0.0)
            for (int a = 0; a < 3; ++a) t[a] = uFt[a] / ut;
        double ut_ = orc_solve_utau(p->law, ut, yF, p->nu, p->kappa, p->B);
        double yBp = yB * ut_ / p->nu;
        o->utau[w] = ut_;
        for (int a = 0; a < 3; ++a) o->tdir[3 * w + a] = t[a];
        if (p->scheme == ORC_BB_FIXED) {
            const double *uwall = o->wside[w] < 0 ? p->wall_u_bottom : p->wall_u_top;
            for (int a = 0; a < 3; ++a) o->uw[3 * w + a] = uwall[a];
        } else if (p->scheme == ORC_BB_SLIP) {
            /* eq. 35: u_w = u_B - u_tau^2 Delta_w / (nu + nu_t|B) */
            double s = ut_ * ut_ * yB / (p->nu * (1.0 + p->kappa * yBp));
            for (int a = 0; a < 3; ++a) o->uw[3 * w + a] = uBt[a] - s * t[a];
        } else {
            for (int a = 0; a < 3; ++a) o->uw[3 * w + a] = 0.0;
        }
        if (p->sa_on && nt_out) nt_out[o->wB[w]] = p->nu * p->kappa * yBp;
    }
}

orc *orc_create(const orc_params *p, const double *u0)
{
    if (!(p->q == 9 || p->q == 19)) return NULL;
    if (p->q == 9 && p->nz != 1) return NULL;
    if (p->nx < 1 || p->ny < 4 || p->nz < 1) return NULL;
    if (p->flow == ORC_PLATE && (p->q != 9 || p->nx < 4)) return NULL;
    if ((p->scheme == ORC_HRFD || p->scheme == ORC_CAI_DEGRIGNY) && p->q != 9) return NULL;
    /* interpolated links are bounce-back rules; any other wall sits halfway */
    if (p->bb_interp < ORC_IBB_HALFWAY || p->bb_interp > ORC_IBB_YU) return NULL;
    if (p->bb_interp != ORC_IBB_HALFWAY && p->scheme != ORC_BB_FIXED && p->scheme != ORC_BB_SLIP) return NULL;
    if (p->bb_interp == ORC_IBB_HALFWAY ? p->wall_dist != 0.5 : !(p->wall_dist > 0.0 && p->wall_dist <= 1.0)) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->p = *p;
    o->D = p->q == 9 ? 2 : 3;
    o->ncell = (int64_t)p->nx * p->ny * p->nz;
    orc_lattice(p->q, o->c, o->w, o->opp);
    int64_t N = o->ncell, Q = p->q;
    o->fpost = (double *)calloc(Q * N, sizeof(double));
    o->fnew = (double *)calloc(Q * N, sizeof(double));
    o->u_prev = (double *)calloc(3 * N, sizeof(double));
    o->u_cur = (double *)calloc(3 * N, sizeof(double));
    o->rho = (double *)calloc(N, sizeof(double));
    o->nt = (double *)calloc(N, sizeof(double));
    o->nt_next = (double *)calloc(N, sizeof(double));
    o->wall_of = (int64_t *)malloc(N * sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) o->wall_of[i] = -1;

    /* wall cells: the bottom row (all x for the channel, x >= plate_start for
     * the plate), then the top row for the channel; z-major, x fastest */
    int64_t nw = 0;
    int x0 = p->flow == ORC_PLATE ? p->plate_start : 0;
    if (x0 < 0) x0 = 0;
    int nrow = p->nx - x0 > 0 ? p->nx - x0 : 0;
    nw = (int64_t)nrow * p->nz * (p->flow == ORC_CHANNEL ? 2 : 1);
    o->nwall = nw;
    o->wB = (int64_t *)malloc((nw + 1) * sizeof(int64_t));
    o->wF = (int64_t *)malloc((nw + 1) * sizeof(int64_t));
    o->wFF = (int64_t *)malloc((nw + 1) * sizeof(int64_t));
    o->wside = (int *)malloc((nw + 1) * sizeof(int));
    o->utau = (double *)calloc(nw + 1, sizeof(double));
    o->tdir = (double *)calloc(3 * (nw + 1), sizeof(double));
    o->uw = (double *)calloc(3 * (nw + 1), sizeof(double));
    int64_t w = 0;
    for (int side = -1; side <= 1; side += 2) {
        if (side == 1 && p->flow != ORC_CHANNEL) break;
        for (int z = 0; z < p->nz; ++z)
            for (int x = x0; x < p->nx; ++x) {
                int yB = side < 0 ? 0 : p->ny - 1, st = side < 0 ? 1 : -1;
                o->wB[w] = cidx(o, x, yB, z);
                o->wF[w] = cidx(o, x, yB + st, z);
                o->wFF[w] = cidx(o, x, yB + 2 * st, z);
                o->wside[w] = side;
                o->wall_of[o->wB[w]] = w;
                ++w;
            }
    }

    /* initial state: f* = f_eq(rho0, u0), nu_tilde = ratio * nu, then the wall
     * function once from u0 */
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = cidx(o, x, y, z);
                double u[3] = {0.0, 0.0, 0.0}, feq[19];
                for (int a = 0; a < o->D; ++a) u[a] = u0 ? u0[a * N + i] : 0.0;
                orc_feq(Q, p->rho0, u, feq);
                for (int k = 0; k < Q; ++k) o->fpost[k * N + i] = feq[k];
                for (int a = 0; a < 3; ++a) o->u_cur[3 * i + a] = u[a];
                o->rho[i] = p->rho0;
                o->nt[i] = p->sa_on ? p->nut_init_ratio * p->nu : 0.0;
            }
    wall_function(o, o->nt);
    memcpy(o->u_prev, o->u_cur, 3 * N * sizeof(double));
    return o;
}

void orc_destroy(orc *o)
{
    if (!o) return;
    free(o->fpost); free(o->fnew); free(o->u_prev); free(o->u_cur); free(o->rho);
    free(o->nt); free(o->nt_next); free(o->wall_of); free(o->wB); free(o->wF); free(o->wFF);
    free(o->wside); free(o->utau); free(o->tdir); free(o->uw);
    free(o);
}

/* Does a population that reaches cell (x, y) through the wall-normal face
 * side (-1 bottom, +1 top) with x-velocity cx reflect off a wall (1) or a
 * symmetry plane (0)?  Channel: walls.  Plate: the top is a symmetry plane;
 * at the bottom the crossing point X = x + 1/2 - cx/2 decides: on the plate
 * (X >= plate_start, the leading-edge point included) it is a wall.  The
 * halfway crossing point is used whatever the wall distance: a link and its
 * specular image then always agree, so streaming stays a bijection. */
static int crossing_is_wall(const orc *o, int x, int side, int cx)
{
    if (o->p.flow == ORC_CHANNEL) return 1;
    if (side > 0) return 0;
    return 2 * x + 1 - cx >= 2 * o->p.plate_start;
}

/* Interpolated bounce-back at the wall cells (eq. 36, eq. 37) with the wall
 * at q = wall_dist from B along every wall-crossing link (a flat wall).  For
 * the link k into the wall and its reflection r = opp(k): f*_k(B) leaves B
 * towards the wall, f_k(B, t+1) = f*_k(F) arrived at B from F = B - c_k, and
 * f*_r(B) is B's own population leaving the wall one step earlier, which is
 * f_r(F, t+1).  rho_w = rho_B; the moving-wall term is eq. 31's.
 * Plate: the outlet column is treated after the outlet copy (outlet = 1),
 * the other columns before it (outlet = 0), so that the copy carries the
 * interpolated values of column nx - 2; a reflection whose halfway source
 * lies outside the lattice stays an open-boundary unknown. */
static void interpolated_bounce_back(orc *o, int outlet)
{
    const orc_params *p = &o->p;
    const int Q = p->q;
    const int64_t N = o->ncell;
    const double q = p->wall_dist;
#pragma omp parallel for schedule(static) if (o->nwall >= ORC_PAR_MIN / 16)
    for (int64_t w = 0; w < o->nwall; ++w) {
        const int64_t cell = o->wB[w];
        const int side = o->wside[w];
        const int x = (int)(cell % p->nx);
        if (p->flow == ORC_PLATE && (x == p->nx - 1) != (outlet != 0)) continue;
        double rho_w = 0.0;
        for (int k = 0; k < Q; ++k) rho_w += o->fpost[k * N + cell];
        for (int k = 0; k < Q; ++k) {
            const int *ck = &o->c[3 * k];
            if (ck[1] != side) continue; /* k points into the wall */
            const int r = o->opp[k];
            if (!crossing_is_wall(o, x, side, o->c[3 * r])) continue;
            const int sx = x - o->c[3 * r];
            if (p->flow == ORC_PLATE && (sx < 0 || sx >= p->nx)) continue;
            const double cu = ck[0] * o->uw[3 * w] + ck[1] * o->uw[3 * w + 1] + ck[2] * o->uw[3 * w + 2];
            const double corr = 2.0 * o->w[k] * rho_w * cu / CS2;
            const double fkB = o->fpost[k * N + cell], fkF = o->fnew[k * N + cell];
            const double frB = o->fpost[r * N + cell];
            double fr;
            if (p->bb_interp == ORC_IBB_BOUZIDI) {
                if (q < 0.5)
                    fr = 2.0 * q * fkB + (1.0 - 2.0 * q) * fkF - corr;
                else
                    fr = fkB / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * frB - corr / (2.0 * q);
            } else {
                /* linear interpolation to the wall point, reflection there,
                 * linear interpolation back to B through F (Yu) */
                const double frW = q * fkB + (1.0 - q) * fkF - corr;
                fr = frW + q / (1.0 + q) * (frB - frW);
            }
            o->fnew[r * N + cell] = fr;
        }
    }
}

static void stream(orc *o)
{
    const orc_params *p = &o->p;
    const int Q = p->q, nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = o->ncell;
#pragma omp parallel for collapse(2) schedule(static) if (o->ncell >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t cell = cidx(o, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    const int *ci = &o->c[3 * i];
                    int sx = x - ci[0], sy = y - ci[1], sz = wrapi(z - ci[2], nz);
                    if (p->flow == ORC_CHANNEL) sx = wrapi(sx, nx);
                    int xin = sx >= 0 && sx < nx, yin = sy >= 0 && sy < ny;
                    double val;
                    if (xin && yin) {
                        /* eq. 3, pull form */
                        val = o->fpost[i * N + cidx(o, sx, sy, sz)];
                    } else if (!xin) {
                        val = NAN; /* open-boundary unknown, filled below */
                    } else {
                        int side = sy < 0 ? -1 : 1;
                        if (crossing_is_wall(o, x, side, ci[0])) {
                            /* eq. 31: f_ibar(x_b, t+1) = f*_i(x_b, t) - 2 w_i rho_w c_i.u_w / cs2,
                             * i = opp of the incoming direction (it points into the wall) */
                            int io = o->opp[i];
                            double rho_w = 0.0, uw[3] = {0.0, 0.0, 0.0};
                            for (int k = 0; k < Q; ++k) rho_w += o->fpost[k * N + cell];
                            int64_t wi = o->wall_of[cell];
                            if (wi >= 0)
                                for (int a = 0; a < 3; ++a) uw[a] = o->uw[3 * wi + a];
                            const int *co = &o->c[3 * io];
                            double cu = co[0] * uw[0] + co[1] * uw[1] + co[2] * uw[2];
                            val = o->fpost[io * N + cell] - 2.0 * o->w[io] * rho_w * cu / CS2;
                        } else {
                            /* symmetry: specular reflection (normal velocity flipped) */
                            int m = -1;
                            for (int k = 0; k < Q; ++k)
                                if (o->c[3 * k] == ci[0] && o->c[3 * k + 1] == -ci[1] && o->c[3 * k + 2] == ci[2]) m = k;
                            val = o->fpost[m * N + cidx(o, sx, y, sz)];
                        }
                    }
                    o->fnew[i * N + cell] = val;
                }
            }
    const int interp = p->bb_interp != ORC_IBB_HALFWAY;
    if (interp) interpolated_bounce_back(o, 0);
    if (p->flow == ORC_PLATE) {
        /* outlet: the unknown populations are copied from the streamed
         * populations of the column x = nx - 2 */
#pragma omp parallel for schedule(static) if (o->ncell >= ORC_PAR_MIN)
        for (int y = 0; y < ny; ++y) {
            int64_t c1 = cidx(o, nx - 1, y, 0), c2 = cidx(o, nx - 2, y, 0);
            for (int i = 0; i < Q; ++i)
                if (o->c[3 * i] < 0) o->fnew[i * N + c1] = o->fnew[i * N + c2];
        }
        /* inlet: Zou-He with u = (u_inlet, 0) */
#pragma omp parallel for schedule(static) if (o->ncell >= ORC_PAR_MIN)
        for (int y = 0; y < ny; ++y) {
            int64_t c0 = cidx(o, 0, y, 0);
            double f[9];
            for (int i = 0; i < 9; ++i) f[i] = o->fnew[i * N + c0];
            orc_zou_he_west(f, p->u_inlet);
            for (int i = 0; i < 9; ++i) o->fnew[i * N + c0] = f[i];
        }
        if (interp) interpolated_bounce_back(o, 1);
    }
}

/* One HRFD reconstruction at a wall cell of a 2-D lattice (Sec. 3.1).
 * f: streamed populations at B on entry, reconstructed ones on exit.
 * side: -1 wall below (n = -y), +1 wall above; t: unit tangential direction;
 * uF_t, uFF_t: previous-step velocity at F and FF projected on t; dudx: the
 * tangential derivative of u_x along the wall; ntB: nu_tilde at B. */
void orc_hrfd_cell(const orc_params *p, double *f, int side, const double *t, double utau,
                   double uF_t, double uFF_t, double dudx, double ntB)
{
    const int Q = p->q;
    const double yB = 0.5;
    int c[19 * 3], opp[19];
    double w[19];
    orc_lattice(Q, c, w, opp);
    double n[3] = {0.0, (double)side, 0.0}, ni[3] = {0.0, (double)-side, 0.0};
    /* eq. 23-25 with u_B . n = 0 (the wall-function velocity is tangential) */
    double fpar = 0.0, fperp = 0.0;
    for (int i = 0; i < Q; ++i) {
        double cn = c[3 * i] * n[0] + c[3 * i + 1] * n[1] + c[3 * i + 2] * n[2];
        if (cn == 0.0) fpar += f[i];
        if (cn > 0.0) fperp += f[i];
    }
    double rhoB = fpar + 2.0 * fperp;
    /* u_B = u_tau u+(y_B+) t (Sec. 3.1) */
    double yBp = yB * utau / p->nu;
    double ubwf = utau * orc_uplus(p->law, yBp, p->kappa, p->B);
    double uB[3];
    for (int a = 0; a < 3; ++a) uB[a] = ubwf * t[a];
    /* eq. 27-28: blended gradient of the tangential velocity along the inward
     * normal; the analytic part is (u_tau^2/nu) du+/dy+ (eq. 15 for the SA law),
     * the FD part uses the wall-function u_B and the flow at F, FF */
    double g_an = utau * utau / p->nu * orc_duplus(p->law, yBp, p->kappa, p->B);
    double g_fd = (-3.0 * ubwf + 4.0 * uF_t - uFF_t) / 2.0;
    double G = p->beta * g_an + (1.0 - p->beta) * g_fd;
    /* Sec. 3.1.2: the Cai-Degrigny variant takes eq. 27 with beta = 1 and the
     * third-order difference of the law (eq. 29) in place of its derivative
     * (eq. 30); the flow at F and FF does not enter */
    if (p->scheme == ORC_CAI_DEGRIGNY)
        G = orc_cai_degrigny_grad(p->law, utau, p->nu, yB, 1.0, p->kappa, p->B);
    /* S_ab = (d_a u_b + d_b u_a)/2 with d_{n'} u = t G, d_x u_x = dudx,
     * v_B = 0 along the wall (so d_x u_y = 0) and S_yy = -S_xx */
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[3 * a + b] = 0.5 * G * (t[a] * ni[b] + t[b] * ni[a]);
    S[0] += dudx;
    S[4] -= dudx;
    /* tau_eff from nu + nu_t(B) (text after eq. 26) */
    double tau = 0.5 + (p->nu + (p->sa_on ? orc_nut(p, ntB) : 0.0)) / CS2;
    orc_regularized(Q, rhoB, uB, S, tau, f);
}

/* HRFD (or Cai-Degrigny) over every wall cell (Sec. 3.1, eq. 19, 23, 26-30).  Wall state
 * (u_tau, t) and the velocities at F, FF are those of the previous step;
 * nu_tilde_B is the Dirichlet value set by the previous step. */
static void hrfd(orc *o)
{
    const orc_params *p = &o->p;
    const int Q = p->q;
    const int64_t N = o->ncell;
    const double yB = 0.5;
    double *ubx = (double *)malloc((o->nwall + 1) * sizeof(double));
#pragma omp parallel for schedule(static) if (o->nwall >= ORC_PAR_MIN / 16)
    for (int64_t w = 0; w < o->nwall; ++w)
        ubx[w] = o->utau[w] * orc_uplus(p->law, yB * o->utau[w] / p->nu, p->kappa, p->B) * o->tdir[3 * w];
#pragma omp parallel for schedule(static) if (o->nwall >= ORC_PAR_MIN / 16)
    for (int64_t w = 0; w < o->nwall; ++w) {
        int64_t cell = o->wB[w];
        const double *t = &o->tdir[3 * w];
        double uFt = 0.0, uFFt = 0.0;
        for (int a = 0; a < 3; ++a) {
            uFt += o->u_prev[3 * o->wF[w] + a] * t[a];
            uFFt += o->u_prev[3 * o->wFF[w] + a] * t[a];
        }
        /* d u_x / dx of the wall-function velocity along the wall: central
         * between neighbouring wall cells, one-sided at the ends of the plate */
        int x = (int)(cell % p->nx);
        int64_t wl, wr;
        if (p->flow == ORC_CHANNEL) {
            wl = o->wall_of[cell - x + wrapi(x - 1, p->nx)];
            wr = o->wall_of[cell - x + wrapi(x + 1, p->nx)];
        } else {
            wl = x - 1 >= p->plate_start ? o->wall_of[cell - 1] : -1;
            wr = x + 1 < p->nx ? o->wall_of[cell + 1] : -1;
        }
        double dudx;
        if (wl >= 0 && wr >= 0)
            dudx = (ubx[wr] - ubx[wl]) / 2.0;
        else if (wr >= 0)
            dudx = ubx[wr] - ubx[w];
        else if (wl >= 0)
            dudx = ubx[w] - ubx[wl];
        else
            dudx = 0.0;
        double f[19];
        for (int i = 0; i < Q; ++i) f[i] = o->fnew[i * N + cell];
        orc_hrfd_cell(p, f, o->wside[w], t, o->utau[w], uFt, uFFt, dudx, o->nt[cell]);
        for (int i = 0; i < Q; ++i) o->fnew[i * N + cell] = f[i];
    }
    free(ubx);
}

static void collide_and_sa(orc *o)
{
    const orc_params *p = &o->p;
    const int Q = p->q, D = o->D, nx = p->nx, ny = p->ny, nz = p->nz;
    const int64_t N = o->ncell;
#pragma omp parallel for collapse(2) schedule(static) if (o->ncell >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t cell = cidx(o, x, y, z);
                double f[19], fp[19], rho, u[3];
                for (int i = 0; i < Q; ++i) f[i] = o->fnew[i * N + cell];
                /* nu_eff = nu + nu_t from the current nu_tilde (Sec. 2.1, after eq. 9) */
                double nut = p->sa_on ? orc_nut(p, o->nt[cell]) : 0.0;
                double tau = 0.5 + (p->nu + nut) / CS2;
                if (p->collision == ORC_CM)
                    orc_collide_cm(Q, f, tau, p->force, fp, &rho, u);
                else
                    orc_collide(Q, f, tau, p->force, fp, &rho, u);
                for (int i = 0; i < Q; ++i) o->fpost[i * N + cell] = fp[i];
                for (int a = 0; a < 3; ++a) o->u_cur[3 * cell + a] = u[a];
                o->rho[cell] = rho;
            }
    if (!p->sa_on) {
        memcpy(o->nt_next, o->nt, N * sizeof(double));
        return;
    }
    /* SA update from nu_tilde^n and the previous step's velocity */
#pragma omp parallel for collapse(2) schedule(static) if (o->ncell >= ORC_PAR_MIN)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t cell = cidx(o, x, y, z);
                if (sa_dirichlet(o, cell, x)) {
                    o->nt_next[cell] = o->nt[cell];
                    continue;
                }
                double ntm[3] = {0}, ntp[3] = {0}, um[9] = {0}, up[9] = {0}, u0[3];
                for (int a = 0; a < 3; ++a) u0[a] = o->u_prev[3 * cell + a];
                for (int a = 0; a < D; ++a) {
                    for (int sgn = -1; sgn <= 1; sgn += 2) {
                        int q3[3] = {x, y, z};
                        q3[a] += sgn;
                        int dims[3] = {nx, ny, nz};
                        double ntv, uv[3];
                        int mirror = 0; /* 0 inside, 1 zero-gradient copy, 2 symmetry mirror */
                        if (a == 2 || (a == 0 && p->flow == ORC_CHANNEL)) {
                            q3[a] = wrapi(q3[a], dims[a]);
                        } else if (q3[a] < 0 || q3[a] >= dims[a]) {
                            mirror = (a == 1) ? 2 : 1;
                            q3[a] -= sgn;
                        }
                        int64_t nb = cidx(o, q3[0], q3[1], q3[2]);
                        ntv = o->nt[nb];
                        for (int c = 0; c < 3; ++c) uv[c] = o->u_prev[3 * nb + c];
                        if (mirror == 2) uv[1] = -uv[1];
                        if (sgn < 0) {
                            ntm[a] = ntv;
                            for (int c = 0; c < 3; ++c) um[3 * a + c] = uv[c];
                        } else {
                            ntp[a] = ntv;
                            for (int c = 0; c < 3; ++c) up[3 * a + c] = uv[c];
                        }
                    }
                }
                double d = wall_distance(o, x, y);
                double v = o->nt[cell] + orc_sa_rhs(p, D, o->nt[cell], ntm, ntp, u0, um, up, d);
                o->nt_next[cell] = v > 0.0 ? v : 0.0;
            }
}

void orc_step(orc *o, int64_t n)
{
    for (int64_t s = 0; s < n; ++s) {
        stream(o);
        if (o->p.scheme == ORC_HRFD || o->p.scheme == ORC_CAI_DEGRIGNY) hrfd(o);
        collide_and_sa(o);
        wall_function(o, o->nt_next);
        double *t = o->nt; o->nt = o->nt_next; o->nt_next = t;
        double *uu = o->u_prev; o->u_prev = o->u_cur; o->u_cur = uu;
        o->steps++;
    }
}

int64_t orc_ncell(const orc *o) { return o->ncell; }
int64_t orc_nwall(const orc *o) { return o->nwall; }
int64_t orc_steps(const orc *o) { return o->steps; }

void orc_get_u(const orc *o, double *out)
{
    for (int a = 0; a < o->D; ++a)
        for (int64_t i = 0; i < o->ncell; ++i) out[a * o->ncell + i] = o->u_prev[3 * i + a];
}
void orc_get_rho(const orc *o, double *out)
{
    for (int64_t i = 0; i < o->ncell; ++i) {
        double s = 0.0;
        for (int k = 0; k < o->p.q; ++k) s += o->fpost[k * o->ncell + i];
        out[i] = s;
    }
}
void orc_get_nt(const orc *o, double *out) { memcpy(out, o->nt, o->ncell * sizeof(double)); }
void orc_get_nut(const orc *o, double *out)
{
    for (int64_t i = 0; i < o->ncell; ++i) out[i] = o->p.sa_on ? orc_nut(&o->p, o->nt[i]) : 0.0;
}
void orc_get_f(const orc *o, double *out) { memcpy(out, o->fpost, o->p.q * o->ncell * sizeof(double)); }
void orc_get_wall(const orc *o, double *utau, double *uw, double *tdir, int64_t *cell)
{
    for (int64_t w = 0; w < o->nwall; ++w) {
        if (utau) utau[w] = o->utau[w];
        for (int a = 0; a < 3; ++a) {
            if (uw) uw[3 * w + a] = o->uw[3 * w + a];
            if (tdir) tdir[3 * w + a] = o->tdir[3 * w + a];
        }
        if (cell) cell[w] = o->wB[w];
    }
}
void orc_totals(const orc *o, double *out4)
{
    double m = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < o->ncell; ++i) {
        m += o->rho[i];
        for (int a = 0; a < 3; ++a) j[a] += o->rho[i] * o->u_prev[3 * i + a];
    }
    out4[0] = m;
    for (int a = 0; a < 3; ++a) out4[1 + a] = j[a];
}

/* eq. 29: third-order one-sided difference of the wall function at y_B with
 * spacing delta (Cai-Degrigny), in physical units of velocity / length. */
double orc_cai_degrigny_grad(int law, double utau, double nu, double yB, double delta, double kappa,
                             double B)
{
    double yp = yB * utau / nu, dp = delta * utau / nu;
    return utau / delta *
           (-11.0 / 6.0 * orc_uplus(law, yp, kappa, B) + 3.0 * orc_uplus(law, yp + dp, kappa, B) -
            1.5 * orc_uplus(law, yp + 2.0 * dp, kappa, B) + 1.0 / 3.0 * orc_uplus(law, yp + 3.0 * dp, kappa, B));
}
