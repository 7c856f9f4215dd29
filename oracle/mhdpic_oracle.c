/*
 * Reference oracle for the cosmic-ray particle step of the MHD-PIC method
 * (Bai, Caprioli, Sironi & Spitkovsky 2015, "Magnetohydrodynamic-Particle-in-Cell
 * Method for Coupling Cosmic Rays with a Thermal Plasma").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded,
 * binary64 CPU implementation of what the GPU library computes.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may build,
 * load or call it.  It shares no code, header, table or constant with the
 * GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 * Contraction must stay off: every multiply and add below is rounded on its
 * own, and fma() is used only where it is written out.
 *
 * What is computed, in the paper's order:
 *   - particle kinematics: v = gamma*u, gamma = sqrt(C^2+v^2)/C,
 *     E_k = v^2/(gamma+1)                                   (Sec. 2.2, eq. parEk)
 *   - CR charge and current carried by a particle: n = (q/mc) m,
 *     J = (q/mc) m u                                        (App. A.1, eq. nJCR)
 *   - gas ion charge n_g = (q/mc)_g rho                     (App. A.1, eq. ng)
 *   - E0 = -v_g x B; R = n_CR/(n_g+n_CR);
 *     F_CR = (1-R)(n_CR E0 + J_CR x B); E = E0 - F_CR/n_g   (Sec. 2.1, eqs. emf0,
 *                                                           defR, lorentz2, emfcr2)
 *   - TSC (quadratic spline) interpolation and deposit      (Sec. 3)
 *   - drift-kick-rotate-kick-drift relativistic Boris push,
 *     with the parallel electric field removed at the particle (App. A.2)
 *   - predictor deposit of n_CR, J_CR at x^(n); corrector deposit of
 *     -dM = -m(v^(n+1)-v^(n)) and -dE_k = -m(E_k^(n+1)-E_k^(n)) at x^(n+1/2)
 *                                                           (App. A.3)
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes):
 *   - the rotation vector is b = (h/2) B / gamma with h = (q/mc) dt, the
 *     standard Boris half-angle form (the printed b = h B / gamma would turn
 *     the velocity twice as far per step as the gyration it integrates);
 *   - the parallel-field removal is E <- E - ((E.B)/B^2) B, skipped when B = 0;
 *   - TSC weights about the nearest cell centre, offset d in [-1/2, 1/2):
 *     w(-1) = (1/2 - d)^2 / 2, w(0) = 3/4 - d^2, w(+1) = (1/2 + d)^2 / 2;
 *   - a position is held as an integer cell index plus the offset d from
 *     that cell's centre in cell units; a drift adds u*dt/(2 dx) to d;
 *   - deposits are amounts (not densities) held as 64-bit integers in units
 *     of 2^-frac_bits: each stencil cell k other than the centre receives
 *     round-half-even(W_k * V) of the exact product, and the centre receives
 *     round-half-even(V) minus the others, so the integers sum to the
 *     particle's rounded total exactly;
 *   - the n_CR, J_CR arrays are refreshed every step at the particle
 *     positions x^(n+1) (the predictor input of the next step); the -dM,
 *     -dE_k arrays accumulate over steps until the caller reads and clears them;
 *   - faces (Sec. 5: a conducting wall, an inflow boundary) are periodic,
 *     reflecting or absorbing per axis and side.  A particle that crosses a
 *     reflecting face during a half drift is mirrored back (offset negated,
 *     that axis's four-velocity and three-velocity negated); one that crosses
 *     an absorbing face leaves the box: crossed in the first half drift it
 *     deposits nothing, in the second it has deposited -dM, -dE_k but
 *     deposits no n_CR, J_CR.  At a non-periodic face a stencil cell beyond
 *     the box is its mirror image inside (cell -1-k is cell k, cell n+k is
 *     cell n-1-k): gathers read the mirror cell's field and deposits land on
 *     it, so every amount stays in the box;
 *   - particles can be added (each deposits its n_CR, J_CR at once) and
 *     removed (its n_CR, J_CR at its current position is taken back).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mhdpic_oracle.h"

#define SQ(a) ((a) * (a))

/* ------------------------------------------------------------------------ */
/* Exact round-half-even of a real product                                  */
/* ------------------------------------------------------------------------ */

/* Returns round-half-to-even of the exact real product a*b as a 64-bit
 * integer.  Each operand is split into an integer significand and a power of
 * two (frexp is exact); the significands are multiplied exactly in 128-bit
 * integer arithmetic and the result is shifted right with round-half-even.
 * Caller guarantees |a*b| < 2^62. */
int64_t oracle_rne_product(double a, double b) {
    if (a == 0.0 || b == 0.0) return 0;
    int ea, eb;
    double fa = frexp(a, &ea); /* a = fa * 2^ea, 1/2 <= |fa| < 1 */
    double fbm = frexp(b, &eb);
    int64_t ma = (int64_t)ldexp(fa, 53); /* |ma| < 2^53, exact */
    int64_t mb = (int64_t)ldexp(fbm, 53);
    int e = ea + eb - 106;               /* a*b = ma*mb*2^e */
    __int128 p = (__int128)ma * (__int128)mb;
    int neg = p < 0;
    unsigned __int128 q = (unsigned __int128)(neg ? -p : p);
    unsigned __int128 r;
    if (e >= 0) {
        r = q << e;
    } else {
        int s = -e;
        if (s > 120) return 0; /* |a*b| < 2^-14: rounds to zero */
        unsigned __int128 ip = q >> s;
        unsigned __int128 rem = q - (ip << s);
        unsigned __int128 half = ((unsigned __int128)1) << (s - 1);
        if (rem > half || (rem == half && (ip & 1))) ip += 1;
        r = ip;
    }
    int64_t out = (int64_t)r;
    return neg ? -out : out;
}

int64_t oracle_quantize(double W, double V) { return oracle_rne_product(W, V); }

/* ------------------------------------------------------------------------ */
/* Kinematics (Sec. 2.2)                                                    */
/* ------------------------------------------------------------------------ */

static double dot3(const double a[3], const double b[3]) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* Lorentz factor, three-velocity and kinetic energy per unit mass of a
 * particle with four-velocity (spatial part) v:
 *   gamma = sqrt(C^2 + v^2) / C,  u = v / gamma,  E_k = v^2 / (gamma + 1).
 * gamma is formed as sqrt(C^2+v^2) * (1/C) and 1/gamma as C / sqrt(C^2+v^2). */
void oracle_lorentz(const double v[3], double C, double* gamma, double u[3], double* ek) {
    double C2 = C * C;
    double iC = 1.0 / C;
    double s = dot3(v, v);
    double r = sqrt(C2 + s);
    double g = r * iC;
    double ig = C / r;
    for (int d = 0; d < 3; ++d) u[d] = v[d] * ig;
    *gamma = g;
    *ek = s / (g + 1.0);
}

/* ------------------------------------------------------------------------ */
/* Boris push (App. A.2)                                                    */
/* ------------------------------------------------------------------------ */

/* Removes the component of E along B at the particle: E <- E - ((E.B)/B^2) B.
 * Left unchanged where B = 0. */
void oracle_clean_E(double E[3], const double B[3]) {
    double eb = dot3(E, B);
    double bb = dot3(B, B);
    if (bb > 0.0) {
        double f = eb / bb;
        for (int d = 0; d < 3; ++d) E[d] = E[d] - f * B[d];
    }
}

/* Kick - rotate - kick of the relativistic Boris scheme with fixed fields.
 * hq = (q/mc) dt / 2 (half of h).  v0 = v + hq E;
 * t = (hq / gamma(v0)) B;  p = v0 + v0 x t;  v1 = v0 + (2/(1+t^2)) p x t;
 * v' = v1 + hq E. */
void oracle_boris_kick_rotate_kick(const double v[3], const double E[3], const double B[3],
                                   double hq, double C, double vout[3]) {
    double he[3], w[3], t[3], p[3], q[3], r[3];
    for (int d = 0; d < 3; ++d) he[d] = hq * E[d];
    for (int d = 0; d < 3; ++d) w[d] = v[d] + he[d];
    double C2 = C * C;
    double sw = dot3(w, w);
    double rw = sqrt(C2 + sw);
    double f = hq * (C / rw); /* (h/2) / gamma */
    for (int d = 0; d < 3; ++d) t[d] = f * B[d];
    p[0] = w[0] + (w[1] * t[2] - w[2] * t[1]);
    p[1] = w[1] + (w[2] * t[0] - w[0] * t[2]);
    p[2] = w[2] + (w[0] * t[1] - w[1] * t[0]);
    double tt = dot3(t, t);
    double c2 = 2.0 / (1.0 + tt);
    for (int d = 0; d < 3; ++d) q[d] = c2 * p[d];
    r[0] = w[0] + (q[1] * t[2] - q[2] * t[1]);
    r[1] = w[1] + (q[2] * t[0] - q[0] * t[2]);
    r[2] = w[2] + (q[0] * t[1] - q[1] * t[0]);
    for (int d = 0; d < 3; ++d) vout[d] = r[d] + he[d];
}

/* ------------------------------------------------------------------------ */
/* TSC shape function (Sec. 3)                                              */
/* ------------------------------------------------------------------------ */

/* Quadratic-spline weights of the cells at offsets -1, 0, +1 from the cell
 * whose centre is nearest, for a particle at offset d (cell units). */
void oracle_tsc_weights(double d, double w[3]) {
    double a = 0.5 - d;
    double b = 0.5 + d;
    w[0] = 0.5 * (a * a);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (b * b);
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                             */
/* ------------------------------------------------------------------------ */

static int64_t n_cells(const oracle_box* bx) {
    return (int64_t)bx->n[0] * bx->n[1] * (bx->ndim == 3 ? bx->n[2] : 1);
}

static int wrap_index(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static int periodic_axis(const oracle_box* bx, int d) {
    return bx->bc[d][0] == ORACLE_PERIODIC;
}

/* Cell index along axis d for an index that may lie one or two cells beyond
 * the box: wrapped on a periodic axis, mirrored at a non-periodic face. */
static int map_index(const oracle_box* bx, int d, int i) {
    int n = bx->n[d];
    if (periodic_axis(bx, d)) return wrap_index(i, n);
    if (i < 0) return -1 - i;
    if (i >= n) return 2 * n - 1 - i;
    return i;
}

static int64_t cell_linear(const oracle_box* bx, const int c[3]) {
    int64_t z = bx->ndim == 3 ? c[2] : 0;
    return (z * bx->n[1] + c[1]) * bx->n[0] + c[0];
}

/* Stencil of a particle: the 3^ndim cells around the nearest cell centre and
 * their weights, ordered z outer, y, x inner, offsets -1, 0, +1.  Weight of
 * cell (a,b,c) is (wx[a]*wy[b])*wz[c] in 3D and wx[a]*wy[b] in 2D. */
typedef struct {
    int nk, centre;
    int64_t cell[27];
    double W[27];
} stencil;

static void make_stencil(const oracle_box* bx, const int i[3], const double dl[3], stencil* st) {
    double w[3][3];
    for (int d = 0; d < bx->ndim; ++d) oracle_tsc_weights(dl[d], w[d]);
    int k = 0;
    int zlo = bx->ndim == 3 ? -1 : 0, zhi = bx->ndim == 3 ? 1 : 0;
    for (int oz = zlo; oz <= zhi; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int c[3];
                c[0] = map_index(bx, 0, i[0] + ox);
                c[1] = map_index(bx, 1, i[1] + oy);
                c[2] = bx->ndim == 3 ? map_index(bx, 2, i[2] + oz) : 0;
                st->cell[k] = cell_linear(bx, c);
                double wxy = w[0][ox + 1] * w[1][oy + 1];
                st->W[k] = bx->ndim == 3 ? wxy * w[2][oz + 1] : wxy;
                if (ox == 0 && oy == 0 && oz == 0) st->centre = k;
                ++k;
            }
    st->nk = k;
}

/* Adds sign times the amount V (already in quanta, i.e. multiplied by
 * 2^frac_bits) to the stencil cells of D: each cell receives its rounded
 * share, so taking a deposit back (sign -1) removes exactly the integers it
 * added.  Integers wrap modulo 2^64 (unsigned arithmetic).  Returns
 * ORACLE_ERANGE if |V| >= 2^51. */
static int deposit_signed(int64_t* D, const stencil* st, double V, int sign) {
    if (!(fabs(V) < 2251799813685248.0)) return ORACLE_ERANGE; /* 2^51 */
    int64_t total = oracle_rne_product(V, 1.0);
    uint64_t rest = 0;
    for (int k = 0; k < st->nk; ++k) {
        if (k == st->centre) continue;
        int64_t q = oracle_rne_product(st->W[k], V);
        uint64_t a = sign > 0 ? (uint64_t)q : (uint64_t)0 - (uint64_t)q;
        D[st->cell[k]] = (int64_t)((uint64_t)D[st->cell[k]] + a);
        rest += (uint64_t)q;
    }
    uint64_t qc = (uint64_t)total - rest;
    uint64_t a = sign > 0 ? qc : (uint64_t)0 - qc;
    D[st->cell[st->centre]] = (int64_t)((uint64_t)D[st->cell[st->centre]] + a);
    return ORACLE_OK;
}

static int deposit_amount(int64_t* D, const stencil* st, double V) {
    return deposit_signed(D, st, V, 1);
}

/* Moves a particle by u*hdx cells along each axis and renormalises the
 * offset into [-1/2, 1/2).  A cell index that leaves the box wraps on a
 * periodic axis; at a reflecting face the position is mirrored about the
 * face (cell -1 at offset d becomes cell 0 at offset -d; cell n becomes cell
 * n-1) and the axis's components of v and u change sign.  A position exactly
 * on the upper face mirrors onto itself; it is kept inside at the largest
 * offset below 1/2.  Returns 1 if the particle crossed an absorbing face (the
 * remaining axes are then not moved), else 0. */
static int drift(const oracle_box* bx, int i[3], double dl[3], double u[3], double v[3],
                 const double hdx[3]) {
    for (int d = 0; d < bx->ndim; ++d) {
        int n = bx->n[d];
        dl[d] = dl[d] + u[d] * hdx[d];
        while (dl[d] >= 0.5) { dl[d] = dl[d] - 1.0; i[d] += 1; }
        while (dl[d] < -0.5) { dl[d] = dl[d] + 1.0; i[d] -= 1; }
        if (i[d] >= 0 && i[d] < n) continue;
        if (periodic_axis(bx, d)) {
            i[d] = wrap_index(i[d], n);
            continue;
        }
        int side = i[d] < 0 ? 0 : 1;
        if (bx->bc[d][side] == ORACLE_ABSORB) return 1;
        /* reflect.  A half drift moves less than one cell, so i is -1 or n.
         * From cell 0 the offset in cell -1 is above -1/2 (strictly, and exactly
         * so in binary64), so its negation stays below 1/2; at the upper face
         * the offset in cell n can be exactly -1/2 (the position on the face). */
        dl[d] = -dl[d];
        if (side == 0) {
            i[d] = 0;
        } else {
            i[d] = n - 1;
            if (dl[d] >= 0.5) dl[d] = nextafter(0.5, 0.0);
        }
        v[d] = -v[d];
        u[d] = -u[d];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cell-centred field preparation (Sec. 2.1; App. A.3 predictor)            */
/* ------------------------------------------------------------------------ */

int oracle_fieldprep(const oracle_box* bx, const double* B, const double* vg, const double* rho,
                     const int64_t* D, double* E) {
    int64_t nc = n_cells(bx);
    double iS = ldexp(1.0, -bx->frac_bits);
    double dV = bx->dx[0] * bx->dx[1];
    if (bx->ndim == 3) dV = dV * bx->dx[2];
    for (int64_t c = 0; c < nc; ++c) {
        double b[3] = {B[c], B[nc + c], B[2 * nc + c]};
        double g[3] = {vg[c], vg[nc + c], vg[2 * nc + c]};
        double e0[3];
        e0[0] = -(g[1] * b[2] - g[2] * b[1]);
        e0[1] = -(g[2] * b[0] - g[0] * b[2]);
        e0[2] = -(g[0] * b[1] - g[1] * b[0]);
        double e[3] = {e0[0], e0[1], e0[2]};
        if (bx->hall) {
            double n = ((double)D[c] * iS) / dV;
            double J[3];
            for (int d = 0; d < 3; ++d) J[d] = ((double)D[(1 + d) * nc + c] * iS) / dV;
            double ng = bx->qomc_gas * rho[c];
            double R = n / (ng + n);
            double jxb[3];
            jxb[0] = J[1] * b[2] - J[2] * b[1];
            jxb[1] = J[2] * b[0] - J[0] * b[2];
            jxb[2] = J[0] * b[1] - J[1] * b[0];
            for (int d = 0; d < 3; ++d) {
                double F = (1.0 - R) * (n * e0[d] + jxb[d]);
                e[d] = e0[d] - F / ng;
            }
        }
        for (int d = 0; d < 3; ++d) E[d * nc + c] = e[d];
    }
    return ORACLE_OK;
}

/* Cell-centred feedback of the predictor step (App. A.3: computed at cell
 * centres from n_CR, J_CR deposited at the particles' positions, R from the gas
 * density, E0 and B).  Per cell, in code units (c = 1, no 4 pi):
 *   out[0..2]  -F_CR, F_CR = (1-R)(n_CR E0 + J_CR x B)       (Sec. 2.2, eq. lorentz2)
 *   out[3]     -(1-R) J_CR . E0                               (eq. engeq, first equality)
 *   out[4..6]  (E - E0) x B, E the field of eq. emfcr2       (eq. engeq, energy flux)
 *   out[7..9]  Lambda = R (u_CR - v_g) / v_A, u_CR = J_CR/n_CR,
 *              v_A = |B|/sqrt(rho); zero where n_CR = 0 or B = 0   (eq. lambda)
 * Without the Hall term R is taken as 0 in out[0..6] (the particles then feel
 * E = E0); Lambda always uses R = n_CR/(n_g + n_CR). */
int oracle_feedback(const oracle_box* bx, const double* B, const double* vg, const double* rho,
                    const int64_t* D, double* out) {
    int64_t nc = n_cells(bx);
    double iS = ldexp(1.0, -bx->frac_bits);
    double dV = bx->dx[0] * bx->dx[1];
    if (bx->ndim == 3) dV = dV * bx->dx[2];
    for (int64_t c = 0; c < nc; ++c) {
        double b[3] = {B[c], B[nc + c], B[2 * nc + c]};
        double g[3] = {vg[c], vg[nc + c], vg[2 * nc + c]};
        double e0[3];
        e0[0] = -(g[1] * b[2] - g[2] * b[1]);
        e0[1] = -(g[2] * b[0] - g[0] * b[2]);
        e0[2] = -(g[0] * b[1] - g[1] * b[0]);
        double n = ((double)D[c] * iS) / dV;
        double J[3];
        for (int d = 0; d < 3; ++d) J[d] = ((double)D[(1 + d) * nc + c] * iS) / dV;
        double ng = bx->qomc_gas * rho[c];
        double RL = n / (ng + n);
        double R = bx->hall ? RL : 0.0;
        double jxb[3];
        jxb[0] = J[1] * b[2] - J[2] * b[1];
        jxb[1] = J[2] * b[0] - J[0] * b[2];
        jxb[2] = J[0] * b[1] - J[1] * b[0];
        double e[3];
        for (int d = 0; d < 3; ++d) {
            double F = (1.0 - R) * (n * e0[d] + jxb[d]);
            out[d * nc + c] = -F;
            e[d] = bx->hall ? e0[d] - F / ng : e0[d];
        }
        double je0 = (J[0] * e0[0] + J[1] * e0[1]) + J[2] * e0[2];
        out[3 * nc + c] = -((1.0 - R) * je0);
        double de[3] = {e[0] - e0[0], e[1] - e0[1], e[2] - e0[2]};
        out[4 * nc + c] = de[1] * b[2] - de[2] * b[1];
        out[5 * nc + c] = de[2] * b[0] - de[0] * b[2];
        out[6 * nc + c] = de[0] * b[1] - de[1] * b[0];
        double bb = (b[0] * b[0] + b[1] * b[1]) + b[2] * b[2];
        for (int d = 0; d < 3; ++d) out[(7 + d) * nc + c] = 0.0;
        if (n != 0.0 && bb > 0.0) {
            double vA = sqrt(bb / rho[c]);
            for (int d = 0; d < 3; ++d) out[(7 + d) * nc + c] = (RL * (J[d] / n - g[d])) / vA;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Initialisation                                                           */
/* ------------------------------------------------------------------------ */

static int check_box(const oracle_box* bx) {
    if (bx->ndim != 2 && bx->ndim != 3) return ORACLE_EINVAL;
    for (int d = 0; d < bx->ndim; ++d) {
        if (bx->n[d] < 1) return ORACLE_EINVAL;
        if (!(bx->dx[d] > 0.0)) return ORACLE_EINVAL;
        for (int side = 0; side < 2; ++side)
            if (bx->bc[d][side] < ORACLE_PERIODIC || bx->bc[d][side] > ORACLE_ABSORB) return ORACLE_EINVAL;
        if ((bx->bc[d][0] == ORACLE_PERIODIC) != (bx->bc[d][1] == ORACLE_PERIODIC)) return ORACLE_EINVAL;
        /* a mirrored position must land inside: at least two cells */
        if (bx->bc[d][0] != ORACLE_PERIODIC && bx->n[d] < 2) return ORACLE_EINVAL;
    }
    if (bx->ndim == 2 && bx->n[2] != 1) return ORACLE_EINVAL;
    if (!(bx->C > 0.0)) return ORACLE_EINVAL;
    if (bx->frac_bits < 0 || bx->frac_bits > 60) return ORACLE_EINVAL;
    if (bx->max_move_cells < 1 || bx->max_move_cells > 2) return ORACLE_EINVAL;
    if (bx->hall && !(bx->qomc_gas != 0.0)) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* Deposits n_CR = (q/mc) m and J_CR = (q/mc) m u at the particle's current
 * position into D[0..3] (App. A.1, eq. nJCR). */
static int deposit_charge_current(const oracle_box* bx, int64_t* D, int64_t nc, const int i[3],
                                  const double dl[3], double qm, double m, const double u[3],
                                  double S) {
    stencil st;
    make_stencil(bx, i, dl, &st);
    double qmm = qm * m;
    int rc = deposit_amount(D, &st, qmm * S);
    for (int d = 0; d < 3 && rc == ORACLE_OK; ++d)
        rc = deposit_amount(D + (1 + d) * nc, &st, (qmm * u[d]) * S);
    return rc;
}

/* Converts particles first .. first+N_new-1 of P from global positions x,
 * four-velocities v (arrays [3][N_new]) and m, qm, and deposits their n_CR,
 * J_CR into D[0..3].  On a non-periodic axis a position must lie inside the
 * box (ORACLE_ERANGE otherwise). */
int oracle_add(const oracle_box* bx, oracle_particles* P, int64_t first, const double* x,
               const double* v, const double* m, const double* qm, int64_t* D) {
    int rc = check_box(bx);
    if (rc) return rc;
    int64_t N = P->N, nc = n_cells(bx);
    int64_t Nn = N - first;
    double S = ldexp(1.0, bx->frac_bits);
    for (int64_t k = 0; k < Nn; ++k) {
        int64_t j = first + k;
        int i[3] = {0, 0, 0};
        double dl[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < bx->ndim; ++d) {
            double s = (x[d * Nn + k] - bx->x0[d]) / bx->dx[d];
            double fl = floor(s);
            if (!isfinite(s)) return ORACLE_ENONFINITE;
            /* the cell count along the box from x0 must fit a 32-bit int */
            if (!(fl >= -2147483648.0 && fl < 2147483648.0)) return ORACLE_ERANGE;
            if (!periodic_axis(bx, d) && !(fl >= 0.0 && fl < (double)bx->n[d])) return ORACLE_ERANGE;
            dl[d] = (s - fl) - 0.5;
            i[d] = wrap_index((int)(int64_t)fl, bx->n[d]);
        }
        double vj[3] = {v[k], v[Nn + k], v[2 * Nn + k]};
        if (!isfinite(vj[0]) || !isfinite(vj[1]) || !isfinite(vj[2])) return ORACLE_ENONFINITE;
        for (int d = 0; d < 3; ++d) {
            P->cell[d * N + j] = i[d];
            P->delta[d * N + j] = dl[d];
            P->v[d * N + j] = vj[d];
        }
        P->m[j] = m[k];
        P->qm[j] = qm[k];
        if (P->alive) P->alive[j] = 1;
        double g, u[3], ek;
        oracle_lorentz(vj, bx->C, &g, u, &ek);
        rc = deposit_charge_current(bx, D, nc, i, dl, qm[k], m[k], u, S);
        if (rc) return rc;
    }
    return ORACLE_OK;
}

int oracle_init(const oracle_box* bx, oracle_particles* P, const double* x, const double* v,
                const double* m, const double* qm, int64_t* D) {
    int rc = check_box(bx);
    if (rc) return rc;
    memset(D, 0, sizeof(int64_t) * 8 * (size_t)n_cells(bx));
    return oracle_add(bx, P, 0, x, v, m, qm, D);
}

/* Removes particle j: takes its n_CR, J_CR deposit at its current position
 * back out of D[0..3] and marks it gone (P->alive must be given). */
int oracle_remove(const oracle_box* bx, oracle_particles* P, int64_t j, int64_t* D) {
    int rc = check_box(bx);
    if (rc) return rc;
    if (!P->alive || j < 0 || j >= P->N || !P->alive[j]) return ORACLE_EINVAL;
    int64_t N = P->N, nc = n_cells(bx);
    int i[3];
    double dl[3], v[3];
    for (int d = 0; d < 3; ++d) {
        i[d] = P->cell[d * N + j];
        dl[d] = P->delta[d * N + j];
        v[d] = P->v[d * N + j];
    }
    double g, u[3], ek;
    oracle_lorentz(v, bx->C, &g, u, &ek);
    stencil st;
    make_stencil(bx, i, dl, &st);
    double S = ldexp(1.0, bx->frac_bits);
    double qmm = P->qm[j] * P->m[j];
    rc = deposit_signed(D, &st, qmm * S, -1);
    for (int d = 0; d < 3 && rc == ORACLE_OK; ++d)
        rc = deposit_signed(D + (1 + d) * nc, &st, (qmm * u[d]) * S, -1);
    if (rc) return rc;
    P->alive[j] = 0;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* One particle step and the step loop (App. A.2, A.3)                      */
/* ------------------------------------------------------------------------ */

int oracle_check_dt(const oracle_box* bx, double dt) {
    if (!isfinite(dt)) return ORACLE_EINVAL;
    /* |u| < C, so a half drift moves at most C*|dt|/(2 dx) cells; the move
     * limit (App. A.4) allows max_move_cells per full step. */
    for (int d = 0; d < bx->ndim; ++d) {
        double cells = bx->C * fabs(dt) / bx->dx[d];
        if (!(cells <= bx->max_move_cells * (1.0 - 1e-12))) return ORACLE_ERANGE;
    }
    return ORACLE_OK;
}

/* One MHD step of the particles: E is prepared once from the n_CR, J_CR in
 * D[0..3] (Sec. 2.1), then every particle takes n_sub steps of dt/n_sub with
 * that E and the caller's B (App. A, "Timestepping and Code Performance":
 * particle sub-cycling with the fields of the half MHD step).  The corrector
 * feedback -dM, -dE_k of every sub-step accumulates in D[4..7]; n_CR, J_CR are
 * deposited at the particles' final positions only, as the next MHD step's
 * predictor input, and copied into D[0..3] at the end. */
int oracle_step_sub(const oracle_box* bx, oracle_particles* P, const double* B, const double* vg,
                    const double* rho, double dt, int n_steps, int n_sub, int64_t* D,
                    int64_t* nJ_next, double* E) {
    int rc = check_box(bx);
    if (rc) return rc;
    if (n_sub < 1) return ORACLE_EINVAL;
    double dts = dt / (double)n_sub;
    rc = oracle_check_dt(bx, dts);
    if (rc) return rc;
    int64_t N = P->N, nc = n_cells(bx);
    double S = ldexp(1.0, bx->frac_bits);
    double C = bx->C;
    double hdt = 0.5 * dts;
    double hdx[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < bx->ndim; ++d) hdx[d] = hdt / bx->dx[d];

    for (int step = 0; step < n_steps; ++step) {
        /* Predictor: cell-centred E from the current n_CR, J_CR (Sec. 2.1). */
        oracle_fieldprep(bx, B, vg, rho, D, E);
        memset(nJ_next, 0, sizeof(int64_t) * 4 * (size_t)nc);
        for (int sub = 0; sub < n_sub; ++sub) {
            const int last = sub == n_sub - 1;
            for (int64_t j = 0; j < N; ++j) {
                if (P->alive && !P->alive[j]) continue;
                int i[3];
                double dl[3], v[3];
                for (int d = 0; d < 3; ++d) {
                    i[d] = P->cell[d * N + j];
                    dl[d] = P->delta[d * N + j];
                    v[d] = P->v[d * N + j];
                }
                double m = P->m[j], qm = P->qm[j];

                double g0, u0[3], ek0;
                oracle_lorentz(v, C, &g0, u0, &ek0);

                /* drift to x^(n+1/2); through an absorbing face: gone, no deposits */
                if (drift(bx, i, dl, u0, v, hdx)) {
                    if (!P->alive) return ORACLE_EINVAL;
                    P->alive[j] = 0;
                    continue;
                }

                /* TSC interpolation of E and B at x^(n+1/2) */
                stencil sh;
                make_stencil(bx, i, dl, &sh);
                double Ep[3] = {0.0, 0.0, 0.0}, Bp[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < sh.nk; ++k)
                    for (int d = 0; d < 3; ++d) {
                        Ep[d] = fma(sh.W[k], E[d * nc + sh.cell[k]], Ep[d]);
                        Bp[d] = fma(sh.W[k], B[d * nc + sh.cell[k]], Bp[d]);
                    }
                oracle_clean_E(Ep, Bp);

                /* kick - rotate - kick */
                double hq = qm * hdt;
                double vn[3];
                oracle_boris_kick_rotate_kick(v, Ep, Bp, hq, C, vn);
                if (!isfinite(vn[0]) || !isfinite(vn[1]) || !isfinite(vn[2])) return ORACLE_ENONFINITE;

                double g1, u1[3], ek1;
                oracle_lorentz(vn, C, &g1, u1, &ek1);

                /* corrector feedback at x^(n+1/2): -dM, -dE_k */
                for (int d = 0; d < 3; ++d) {
                    rc = deposit_amount(D + (4 + d) * nc, &sh, (-(m * (vn[d] - v[d]))) * S);
                    if (rc) return rc;
                }
                rc = deposit_amount(D + 7 * nc, &sh, (-(m * (ek1 - ek0))) * S);
                if (rc) return rc;

                /* drift to x^(n+1); through an absorbing face: gone after the
                 * corrector deposit, before the predictor one */
                if (drift(bx, i, dl, u1, vn, hdx)) {
                    if (!P->alive) return ORACLE_EINVAL;
                    P->alive[j] = 0;
                    continue;
                }

                /* n_CR, J_CR at the end of the MHD step for the next predictor */
                if (last) {
                    rc = deposit_charge_current(bx, nJ_next, nc, i, dl, qm, m, u1, S);
                    if (rc) return rc;
                }

                for (int d = 0; d < 3; ++d) {
                    P->cell[d * N + j] = i[d];
                    P->delta[d * N + j] = dl[d];
                    P->v[d * N + j] = vn[d];
                }
            }
        }
        memcpy(D, nJ_next, sizeof(int64_t) * 4 * (size_t)nc);
    }
    return ORACLE_OK;
}

/* n_steps steps of one particle step each (App. A.3). */
int oracle_step(const oracle_box* bx, oracle_particles* P, const double* B, const double* vg,
                const double* rho, double dt, int n_steps, int64_t* D, int64_t* nJ_next,
                double* E) {
    return oracle_step_sub(bx, P, B, vg, rho, dt, n_steps, 1, D, nJ_next, E);
}

/* Global positions x = x0 + dx * ((i + 1/2) + d). */
int oracle_positions(const oracle_box* bx, const oracle_particles* P, double* x) {
    int64_t N = P->N;
    for (int64_t j = 0; j < N; ++j)
        for (int d = 0; d < 3; ++d) {
            if (d < bx->ndim)
                x[d * N + j] = bx->x0[d] +
                               bx->dx[d] * (((double)P->cell[d * N + j] + 0.5) + P->delta[d * N + j]);
            else
                x[d * N + j] = 0.0;
        }
    return ORACLE_OK;
}
