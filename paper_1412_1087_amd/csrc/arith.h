// Per-particle arithmetic of the CR step, binary64.  Every operation is
// rounded on its own (the library is built with contraction off); fma is used
// only where written.  The sequence is the canonical one of the design notes,
// so results are bit-identical to any other implementation of that sequence.
#pragma once
#include "common.h"

namespace mhdpic {

__device__ __forceinline__ double dot3(double a0, double a1, double a2, double b0, double b1,
                                       double b2) {
    return (a0 * b0 + a1 * b1) + a2 * b2;
}

// Kinematics of a particle with spatial four-velocity v (Sec. 2.2):
// gamma = sqrt(C^2+v^2)*(1/C), u = v*(C/sqrt(C^2+v^2)), E_k = v^2/(gamma+1).
struct Kin {
    double u[3];
    double ek;
};

__device__ __forceinline__ Kin lorentz(const double v[3], double C, double C2, double iC) {
    Kin k;
    double s = dot3(v[0], v[1], v[2], v[0], v[1], v[2]);
    double r = __builtin_sqrt(C2 + s);
    double g = r * iC;
    double ig = C / r;
    k.u[0] = v[0] * ig;
    k.u[1] = v[1] * ig;
    k.u[2] = v[2] * ig;
    k.ek = s / (g + 1.0);
    return k;
}

// Drift by u*hdx cells and renormalise the offset to [-1/2, 1/2).  The move
// limit guarantees |u*hdx| < 1, so a single correction suffices.  Returns the
// cell shift (-1, 0, +1); the caller wraps the index.
__device__ __forceinline__ int drift1(double& d, double u, double hdx) {
    d = d + u * hdx;
    if (d >= 0.5) {
        d = d - 1.0;
        return 1;
    }
    if (d < -0.5) {
        d = d + 1.0;
        return -1;
    }
    return 0;
}

__device__ __forceinline__ int wrap_shift(int i, int s, int n) {
    int r = i + s;
    if (r < 0) r += n;
    if (r >= n) r -= n;
    return r;
}

// TSC (quadratic spline) weights of the cells at offsets -1, 0, +1 (Sec. 3).
__device__ __forceinline__ void tsc(double d, double w[3]) {
    double a = 0.5 - d;
    double b = 0.5 + d;
    w[0] = 0.5 * (a * a);
    w[1] = 0.75 - d * d;
    w[2] = 0.5 * (b * b);
}

// Kick - rotate - kick with fixed fields (App. A.2); hq = (q/mc) dt / 2.
__device__ __forceinline__ void boris(const double v[3], const double E[3], const double B[3],
                                      double hq, double C, double C2, double vn[3]) {
    double he0 = hq * E[0], he1 = hq * E[1], he2 = hq * E[2];
    double w0 = v[0] + he0, w1 = v[1] + he1, w2 = v[2] + he2;
    double sw = dot3(w0, w1, w2, w0, w1, w2);
    double rw = __builtin_sqrt(C2 + sw);
    double f = hq * (C / rw);
    double t0 = f * B[0], t1 = f * B[1], t2 = f * B[2];
    double p0 = w0 + (w1 * t2 - w2 * t1);
    double p1 = w1 + (w2 * t0 - w0 * t2);
    double p2 = w2 + (w0 * t1 - w1 * t0);
    double tt = dot3(t0, t1, t2, t0, t1, t2);
    double c2 = 2.0 / (1.0 + tt);
    double q0 = c2 * p0, q1 = c2 * p1, q2 = c2 * p2;
    double r0 = w0 + (q1 * t2 - q2 * t1);
    double r1 = w1 + (q2 * t0 - q0 * t2);
    double r2 = w2 + (q0 * t1 - q1 * t0);
    vn[0] = r0 + he0;
    vn[1] = r1 + he1;
    vn[2] = r2 + he2;
}

// E <- E - ((E.B)/B^2) B where B != 0 (App. A.2).
__device__ __forceinline__ void clean_parallel(double E[3], const double B[3]) {
    double eb = dot3(E[0], E[1], E[2], B[0], B[1], B[2]);
    double bb = dot3(B[0], B[1], B[2], B[0], B[1], B[2]);
    if (bb > 0.0) {
        double f = eb / bb;
        E[0] = E[0] - f * B[0];
        E[1] = E[1] - f * B[1];
        E[2] = E[2] - f * B[2];
    }
}

// round-half-even(W*V) of the exact product for |W*V| < 2^51, as an int64:
// fma rounds W*V + 1.5*2^52 once, to an integer held in the mantissa.
__device__ __forceinline__ int64_t quant(double W, double V) {
    double q = __builtin_fma(W, V, kMagic);
    uint64_t b = (uint64_t)__double_as_longlong(q);
    return (int64_t)(b - ((uint64_t)kMagicHi << 32));
}

// round-half-even(V) for |V| < 2^51.
__device__ __forceinline__ int64_t quant1(double V) {
    double q = V + kMagic;
    uint64_t b = (uint64_t)__double_as_longlong(q);
    return (int64_t)(b - ((uint64_t)kMagicHi << 32));
}

}  // namespace mhdpic
