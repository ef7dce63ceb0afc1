/*
 * oracle.c -- plain CPU reference of the two-belt Shan-Chen lattice Boltzmann
 * method (Chibbaro, Falcucci, Chen, Shan, Chiatti, Succi, "Lattice Boltzmann
 * models for non-ideal fluids with arrested phase-separation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path loads, links or
 * calls this library: it is used by the test suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no source with the HIP
 * library (no header, no table, no helper).
 *
 * It is written to be checked by eye against the paper, not to be fast:
 * every step is a separate full-lattice pass in the order the paper states
 * it, on plain row-major arrays, with the 24-link sum written as a loop over
 * the link table.  Floating point is `real` = double; compiling with
 * -DORACLE_F32 gives a single-precision twin (float arithmetic, expf) that is
 * used only to size the tolerance of single-precision results; its global
 * sums are still accumulated in double.
 *
 * Array layout: site (x, y) of an nx-by-ny periodic lattice has index
 * s = y*nx + x; populations are f[i*N + s] with N = nx*ny, i = 0..8.
 *
 * Readings taken where the paper is silent or garbled (each is argued in the
 * design notes):
 *   - force sign: F = -psi(x) sum_k K_k psi(x + c_k) c_k, negative G attracts
 *     (section II force formula with its minus sign; section III statement
 *     that positive G is repulsive; critical point G = -4);
 *   - force coupling into eq. (1): Shan-Chen velocity shift, the equilibrium
 *     is evaluated at u_eq = (j + tau F) / rho and F_i = 0;
 *   - first-belt energy includes the rest link with weight
 *     G1 w_0 + G2 p_s0, p_s0 = 1 - sum of the 24 link weights = 247/420
 *     (normalisation eq. weights_1); second-belt energy runs over its 16
 *     links only.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_F32
typedef float real;
#define REAL_EXP expf
#define REAL_SQRT sqrtf
#else
typedef double real;
#define REAL_EXP exp
#define REAL_SQRT sqrt
#endif

/* ---------------------------------------------------------------------------
 * Lattice tables.
 *
 * D2Q9 speeds and weights (section II equilibrium, section IV "nine-speed
 * 2DQ9 model"): rest, the four axis speeds, the four diagonals; c_s^2 = 1/3.
 * ------------------------------------------------------------------------ */
static const int Q_CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int Q_CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double Q_W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* The 24 interaction links of the two-belt lattice (section III, the
 * two-belt figure and Table 1): belt 1 = the 8 moving D2Q9 speeds
 * (|c|^2 = 1, 2); belt 2 = the 16 links with |c|^2 = 4, 5, 8, i.e. the 5x5
 * block without its inner 3x3.  Order: belt 1 in D2Q9 order, then belt 2
 * grouped by |c|^2, counter-clockwise from +x inside each group. */
static const int L_CX[24] = {1, 0, -1, 0,  1, -1, -1, 1,
                             2, 0, -2, 0,
                             2, 1, -1, -2, -2, -1, 1, 2,
                             2, -2, -2, 2};
static const int L_CY[24] = {0, 1, 0, -1, 1, 1, -1, -1,
                             0, 2, 0, -2,
                             1, 2, 2, 1, -1, -2, -2, -1,
                             2, 2, -2, -2};

/* Table 1 weights p(|c|^2). */
static double link_p(int c2)
{
    switch (c2) {
    case 1: return 4.0 / 63.0;
    case 2: return 4.0 / 135.0;
    case 4: return 1.0 / 180.0;
    case 5: return 2.0 / 945.0;
    case 8: return 1.0 / 15120.0;
    default: return 0.0;
    }
}

/* D2Q9 weight of a first-belt link, looked up by its |c|^2. */
static double link_w(int c2)
{
    if (c2 == 1) return 1.0 / 9.0;
    if (c2 == 2) return 1.0 / 36.0;
    return 0.0;
}

/* Rest weight of the first belt for the G2 coupling: eq. (weights_1) makes
 * p_s0 + (sum of the 24 link weights) = 1, which gives 247/420. */
static const double P_S0 = 247.0 / 420.0;

/* Coupling of link k in eq. (FORCE): first-belt links carry G1 w + G2 p_s,
 * second-belt links carry G2 p_m. */
static void link_couplings(double G1, double G2, double K[24])
{
    for (int k = 0; k < 24; ++k) {
        int c2 = L_CX[k] * L_CX[k] + L_CY[k] * L_CY[k];
        if (k < 8)
            K[k] = G1 * link_w(c2) + G2 * link_p(c2);
        else
            K[k] = G2 * link_p(c2);
    }
}

/* Periodic wrap of a lattice coordinate (offsets are at most 2 sites). */
static int64_t wrap(int64_t a, int64_t n)
{
    while (a < 0) a += n;
    while (a >= n) a -= n;
    return a;
}

/* Pairwise sum, used for every global sum so that the oracle's own rounding
 * stays far below the tolerances it is used to check. */
static double pairwise_sum(const double* a, int64_t n)
{
    if (n <= 16) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i];
        return s;
    }
    int64_t h = n / 2;
    return pairwise_sum(a, h) + pairwise_sum(a + h, n - h);
}

/* ---------------------------------------------------------------------------
 * Exported tables (so the tests can check them against Table 1 exactly).
 * ------------------------------------------------------------------------ */
void orc_d2q9(int8_t cx[9], int8_t cy[9], double w[9])
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = (int8_t)Q_CX[i];
        cy[i] = (int8_t)Q_CY[i];
        w[i] = Q_W[i];
    }
}

/* K[k]: force/energy coupling of link k; KE[0]: rest coupling of the energy
 * (G1 w_0 + G2 p_s0), KE[1 + k] = K[k]. */
void orc_tables(int8_t cx[24], int8_t cy[24], double K[24], double KE[25],
                double G1, double G2)
{
    link_couplings(G1, G2, K);
    for (int k = 0; k < 24; ++k) {
        cx[k] = (int8_t)L_CX[k];
        cy[k] = (int8_t)L_CY[k];
        KE[1 + k] = K[k];
    }
    KE[0] = G1 * Q_W[0] + G2 * P_S0;
}

int orc_real_bytes(void) { return (int)sizeof(real); }

/* Threads the OpenMP loops of this library use (for timing reports). */
int orc_threads(void) { return omp_get_max_threads(); }

/* Set that number (single-thread timings). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ---------------------------------------------------------------------------
 * Section II: equilibrium, moments, pseudopotential.
 * ------------------------------------------------------------------------ */

/* Second-order equilibrium, section II:
 * f_i^eq = w_i rho (1 + c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u^2/(2 c_s^2)). */
static real feq(int i, real rho, real ux, real uy)
{
    const real cs2 = (real)CS2;
    real cu = (real)Q_CX[i] * ux + (real)Q_CY[i] * uy;
    real uu = ux * ux + uy * uy;
    return (real)Q_W[i] * rho *
           ((real)1 + cu / cs2 + cu * cu / ((real)2 * cs2 * cs2) - uu / ((real)2 * cs2));
}

/* Populations at equilibrium with a given density and velocity (u may be
 * NULL for a fluid at rest): the initial state of section IV. */
void orc_init(int64_t nx, int64_t ny, const double* rho, const double* ux,
              const double* uy, real* f)
{
    int64_t N = nx * ny;
    for (int64_t s = 0; s < N; ++s) {
        real u = ux ? (real)ux[s] : (real)0;
        real v = uy ? (real)uy[s] : (real)0;
        for (int i = 0; i < 9; ++i) f[i * N + s] = feq(i, (real)rho[s], u, v);
    }
}

/* rho = sum_i f_i, j = rho u = sum_i c_i f_i (section II). */
void orc_moments(int64_t nx, int64_t ny, const real* f, real* rho, real* jx,
                 real* jy)
{
    int64_t N = nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        real r = 0, a = 0, b = 0;
        for (int i = 0; i < 9; ++i) {
            real fi = f[i * N + s];
            r += fi;
            a += (real)Q_CX[i] * fi;
            b += (real)Q_CY[i] * fi;
        }
        rho[s] = r;
        jx[s] = a;
        jy[s] = b;
    }
}

/* psi = sqrt(rho0) (1 - exp(-rho/rho0)), section II and section III. */
void orc_psi(int64_t n, double rho0, const real* rho, real* psi)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s)
        psi[s] = REAL_SQRT((real)rho0) * ((real)1 - REAL_EXP(-rho[s] / (real)rho0));
}

/* ---------------------------------------------------------------------------
 * Section III: two-belt pseudopotential force, eq. (FORCE) with the sign of
 * the section II force formula:
 *   F(x) = -psi(x) sum_{k=1}^{24} K_k psi(x + c_k) c_k.
 * ------------------------------------------------------------------------ */
void orc_force(int64_t nx, int64_t ny, double G1, double G2, const real* psi,
               real* Fx, real* Fy)
{
    double K[24];
    link_couplings(G1, G2, K);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < ny; ++y) {
        for (int64_t x = 0; x < nx; ++x) {
            real sx = 0, sy = 0;
            for (int k = 0; k < 24; ++k) {
                int64_t xn = wrap(x + L_CX[k], nx);
                int64_t yn = wrap(y + L_CY[k], ny);
                real v = (real)K[k] * psi[yn * nx + xn];
                sx += v * (real)L_CX[k];
                sy += v * (real)L_CY[k];
            }
            Fx[y * nx + x] = -psi[y * nx + x] * sx;
            Fy[y * nx + x] = -psi[y * nx + x] * sy;
        }
    }
}

/* ---------------------------------------------------------------------------
 * eq. (1), right-hand side: BGK relaxation towards the equilibrium taken at
 * the force-shifted velocity u_eq = (j + tau F)/rho:
 *   f*_i = f_i - (f_i - f_i^eq(rho, u_eq)) / tau.
 * ------------------------------------------------------------------------ */
void orc_collide(int64_t nx, int64_t ny, double tau, const real* f,
                 const real* Fx, const real* Fy, real* fpost)
{
    int64_t N = nx * ny;
    const real t = (real)tau;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        real rho = 0, jx = 0, jy = 0;
        for (int i = 0; i < 9; ++i) {
            real fi = f[i * N + s];
            rho += fi;
            jx += (real)Q_CX[i] * fi;
            jy += (real)Q_CY[i] * fi;
        }
        real ux = (jx + t * Fx[s]) / rho;
        real uy = (jy + t * Fy[s]) / rho;
        for (int i = 0; i < 9; ++i) {
            real fi = f[i * N + s];
            fpost[i * N + s] = fi - (fi - feq(i, rho, ux, uy)) / t;
        }
    }
}

/* eq. (1), left-hand side: free streaming, f_i(x + c_i, t+1) = f*_i(x, t). */
void orc_stream(int64_t nx, int64_t ny, const real* fpost, real* fnext)
{
    int64_t N = nx * ny;
    for (int i = 0; i < 9; ++i) {
#pragma omp parallel for schedule(static)
        for (int64_t y = 0; y < ny; ++y) {
            int64_t yd = wrap(y + Q_CY[i], ny);
            for (int64_t x = 0; x < nx; ++x) {
                int64_t xd = wrap(x + Q_CX[i], nx);
                fnext[i * N + yd * nx + xd] = fpost[i * N + y * nx + x];
            }
        }
    }
}

/* One or more full time steps of eq. (1), in place on f (pre-collision
 * populations at t -> at t + nsteps): moments, psi, force, collision,
 * streaming. */
int orc_step(int64_t nx, int64_t ny, double tau, double rho0, double G1,
             double G2, real* f, int64_t nsteps)
{
    int64_t N = nx * ny;
    real* rho = (real*)malloc(sizeof(real) * N);
    real* jx = (real*)malloc(sizeof(real) * N);
    real* jy = (real*)malloc(sizeof(real) * N);
    real* psi = (real*)malloc(sizeof(real) * N);
    real* Fx = (real*)malloc(sizeof(real) * N);
    real* Fy = (real*)malloc(sizeof(real) * N);
    real* fpost = (real*)malloc(sizeof(real) * 9 * N);
    if (!rho || !jx || !jy || !psi || !Fx || !Fy || !fpost) {
        free(rho); free(jx); free(jy); free(psi); free(Fx); free(Fy); free(fpost);
        return -1;
    }
    for (int64_t n = 0; n < nsteps; ++n) {
        orc_moments(nx, ny, f, rho, jx, jy);
        orc_psi(N, rho0, rho, psi);
        orc_force(nx, ny, G1, G2, psi, Fx, Fy);
        orc_collide(nx, ny, tau, f, Fx, Fy, fpost);
        orc_stream(nx, ny, fpost, f);
    }
    free(rho); free(jx); free(jy); free(psi); free(Fx); free(Fy); free(fpost);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Section V: pseudo-potential energy of the state f (pre-collision, time t).
 *   E_s = 1/2 sum_x psi(x) sum_{i=0}^{8} (G1 w_i + G2 p_si) psi(x + c_i)
 *   E_m = 1/2 sum_x psi(x) sum_{i=1}^{16} G2 p_mi psi(x + c_mi)
 *   E_bulk = (G1 + G2)/2 sum_x psi^2            (eq. Ebulk)
 * out = {M = sum rho, E_s, E_m, sum psi^2, E_bulk}.
 * ------------------------------------------------------------------------ */
int orc_observables(int64_t nx, int64_t ny, double rho0, double G1, double G2,
                    const real* f, double out[5])
{
    int64_t N = nx * ny;
    double K[24];
    link_couplings(G1, G2, K);
    double KE0 = G1 * Q_W[0] + G2 * P_S0;
    real* rho = (real*)malloc(sizeof(real) * N);
    real* jx = (real*)malloc(sizeof(real) * N);
    real* jy = (real*)malloc(sizeof(real) * N);
    real* psi = (real*)malloc(sizeof(real) * N);
    double* a = (double*)malloc(sizeof(double) * N);
    if (!rho || !jx || !jy || !psi || !a) {
        free(rho); free(jx); free(jy); free(psi); free(a);
        return -1;
    }
    orc_moments(nx, ny, f, rho, jx, jy);
    orc_psi(N, rho0, rho, psi);

    for (int64_t s = 0; s < N; ++s) a[s] = (double)rho[s];
    out[0] = pairwise_sum(a, N);

    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            double p = (double)psi[y * nx + x];
            double acc = KE0 * p;
            for (int k = 0; k < 8; ++k)
                acc += K[k] * (double)psi[wrap(y + L_CY[k], ny) * nx + wrap(x + L_CX[k], nx)];
            a[y * nx + x] = 0.5 * p * acc;
        }
    out[1] = pairwise_sum(a, N);

    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            double p = (double)psi[y * nx + x];
            double acc = 0.0;
            for (int k = 8; k < 24; ++k)
                acc += K[k] * (double)psi[wrap(y + L_CY[k], ny) * nx + wrap(x + L_CX[k], nx)];
            a[y * nx + x] = 0.5 * p * acc;
        }
    out[2] = pairwise_sum(a, N);

    for (int64_t s = 0; s < N; ++s) a[s] = (double)psi[s] * (double)psi[s];
    out[3] = pairwise_sum(a, N);
    out[4] = 0.5 * (G1 + G2) * out[3];

    free(rho); free(jx); free(jy); free(psi); free(a);
    return 0;
}

/* A run with an energy trace: the state is logged at every t in
 * [0, nsteps] with t % log_every == 0 (pre-collision state at t), one row
 * {t, M, E_s, E_m, sum psi^2, E_bulk} per log point.  Returns the number of
 * rows written, or -1 if cap is too small or memory runs out. */
int64_t orc_run(int64_t nx, int64_t ny, double tau, double rho0, double G1,
                double G2, real* f, int64_t nsteps, int64_t log_every,
                double* trace, int64_t cap)
{
    int64_t rows = 0;
    for (int64_t t = 0; t <= nsteps; ++t) {
        if (log_every > 0 && t % log_every == 0) {
            if (rows >= cap) return -1;
            double o[5];
            if (orc_observables(nx, ny, rho0, G1, G2, f, o)) return -1;
            trace[rows * 6 + 0] = (double)t;
            for (int c = 0; c < 5; ++c) trace[rows * 6 + 1 + c] = o[c];
            ++rows;
        }
        if (t < nsteps && orc_step(nx, ny, tau, rho0, G1, G2, f, 1)) return -1;
    }
    return rows;
}
