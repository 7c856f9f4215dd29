/*
 * Reference oracle for the MHD-PIC cosmic-ray particle step.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.
 *
 * All pointers are host pointers.  Arrays are structure-of-arrays with the
 * component index outermost: a [3][N] array holds x-components of all
 * particles, then y, then z.  Grid arrays are [comp][nz][ny][nx], x fastest.
 */
#ifndef MHDPIC_ORACLE_H
#define MHDPIC_ORACLE_H
#include <stdint.h>

/* Particle boundary of one face of a box (Sec. 5: a conducting wall at x = 0
 * and an inflow boundary at x = L_x; periodic otherwise). */
enum { ORACLE_PERIODIC = 0, ORACLE_REFLECT = 1, ORACLE_ABSORB = 2 };

enum {
    ORACLE_OK = 0,
    ORACLE_EINVAL = -1,
    ORACLE_ERANGE = -4,
    ORACLE_ENONFINITE = -5
};

typedef struct {
    int32_t ndim;           /* 2 or 3 */
    int32_t n[3];           /* cells per dimension; n[2] = 1 in 2D */
    double dx[3];           /* cell size */
    double x0[3];           /* lower corner of the box */
    double C;               /* reduced particle speed of light */
    double qomc_gas;        /* (q/mc)_g of the gas ions: n_g = qomc_gas * rho */
    int32_t hall;           /* 1: E = E0 - F_CR/n_g; 0: E = E0 */
    int32_t frac_bits;      /* deposits in units of 2^-frac_bits */
    int32_t max_move_cells; /* a particle moves at most this many cells per step */
    int32_t bc[3][2];       /* per axis, low and high face: ORACLE_PERIODIC (both faces or
                               neither), ORACLE_REFLECT or ORACLE_ABSORB */
} oracle_box;

typedef struct {
    int64_t N;
    int32_t* cell; /* [3][N] cell index per dimension (z = 0 in 2D) */
    double* delta; /* [3][N] offset from the cell centre, cell units (z = 0 in 2D) */
    double* v;     /* [3][N] spatial four-velocity gamma*u */
    double* m;     /* [N] CR mass carried by the particle */
    double* qm;    /* [N] (q/mc) of the particle */
    int32_t* alive; /* [N] 1 while the particle is in the box, 0 once it left through an
                       absorbing face or was removed; NULL: every particle stays */
} oracle_particles;

int64_t oracle_rne_product(double a, double b);
int64_t oracle_quantize(double W, double V);
void oracle_lorentz(const double v[3], double C, double* gamma, double u[3], double* ek);
void oracle_clean_E(double E[3], const double B[3]);
void oracle_boris_kick_rotate_kick(const double v[3], const double E[3], const double B[3],
                                   double hq, double C, double vout[3]);
void oracle_tsc_weights(double d, double w[3]);
int oracle_fieldprep(const oracle_box* bx, const double* B, const double* vg, const double* rho,
                     const int64_t* D, double* E);
int oracle_feedback(const oracle_box* bx, const double* B, const double* vg, const double* rho,
                    const int64_t* D, double* out);
int oracle_init(const oracle_box* bx, oracle_particles* P, const double* x, const double* v,
                const double* m, const double* qm, int64_t* D);
int oracle_add(const oracle_box* bx, oracle_particles* P, int64_t first, const double* x,
               const double* v, const double* m, const double* qm, int64_t* D);
int oracle_remove(const oracle_box* bx, oracle_particles* P, int64_t j, int64_t* D);
int oracle_check_dt(const oracle_box* bx, double dt);
int oracle_step(const oracle_box* bx, oracle_particles* P, const double* B, const double* vg,
                const double* rho, double dt, int n_steps, int64_t* D, int64_t* nJ_next,
                double* E);
int oracle_step_sub(const oracle_box* bx, oracle_particles* P, const double* B, const double* vg,
                    const double* rho, double dt, int n_steps, int n_sub, int64_t* D,
                    int64_t* nJ_next, double* E);
int oracle_positions(const oracle_box* bx, const oracle_particles* P, double* x);

#endif
