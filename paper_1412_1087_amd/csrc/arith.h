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

namespace mhdpic {

// ---------------------------------------------------------------------------
// Precision form: binary32 offsets, velocities, fields and weights; the
// Lorentz factor, u (rounded to binary32 afterwards) and E_k in binary64.
// ---------------------------------------------------------------------------

struct Kin32 {
    float u[3];
    double g;  // Lorentz factor
};

__device__ __forceinline__ Kin32 lorentz32(const float v[3], double C, double C2, double iC) {
    Kin32 k;
    double v0 = v[0], v1 = v[1], v2 = v[2];
    double s = dot3(v0, v1, v2, v0, v1, v2);
    double r = __builtin_sqrt(C2 + s);
    k.g = r * iC;
    double ig = C / r;
    k.u[0] = (float)(v0 * ig);
    k.u[1] = (float)(v1 * ig);
    k.u[2] = (float)(v2 * ig);
    return k;
}

__device__ __forceinline__ int drift1f(float& d, float u, float hdx) {
    d = d + u * hdx;
    if (d >= 0.5f) {
        d = d - 1.0f;
        return 1;
    }
    if (d < -0.5f) {
        d = d + 1.0f;
        return -1;
    }
    return 0;
}

__device__ __forceinline__ void tscf(float d, float w[3]) {
    float a = 0.5f - d;
    float b = 0.5f + d;
    w[0] = 0.5f * (a * a);
    w[1] = 0.75f - d * d;
    w[2] = 0.5f * (b * b);
}

// Policies used by the kernels that exist in both precisions.  Besides the
// working precision they fix how the corrector's momentum and energy changes
// (App. A.3) are formed: `Inc` carries what the push hands to `corrector`.
struct F64Pol {
    using R = double;
    using Part = PartF64;
    struct K {
        double u[3];
        double ek;
    };
    struct Inc {};
    __device__ static __forceinline__ K kin(const double v[3], double C, double C2, double iC) {
        Kin k = lorentz(v, C, C2, iC);
        return K{{k.u[0], k.u[1], k.u[2]}, k.ek};
    }
    __device__ static __forceinline__ double hdx(double h) { return h; }
    __device__ static __forceinline__ int drift(double& d, double u, double h) { return drift1(d, u, h); }
    __device__ static __forceinline__ void weights(double d, double w[3]) { tsc(d, w); }
    __device__ static __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    __device__ static __forceinline__ void clean(double E[3], const double B[3]) { clean_parallel(E, B); }
    __device__ static __forceinline__ void push(const double v[3], const double E[3], const double B[3],
                                                double hq, double C, double C2, double vn[3], Inc&) {
        boris(v, E, B, hq, C, C2, vn);
    }
    // the canonical sequence: differences of the stored states, E_k from
    // v^2/(gamma+1) at both ends (Sec. 2.2, eq. parEk)
    __device__ static __forceinline__ void corrector(const double v[3], const double vn[3],
                                                     const K& k0, const K& k1, const Inc&,
                                                     double dv[3], double& dek) {
        dv[0] = vn[0] - v[0];
        dv[1] = vn[1] - v[1];
        dv[2] = vn[2] - v[2];
        dek = k1.ek - k0.ek;
    }
};

struct F32Pol {
    using R = float;
    using Part = PartF32;
    using K = Kin32;
    // Binary64 changes of the kick-rotate-kick, from its own terms (see push)
    struct Inc {
        double dv[3];  // v' - v = x + 2 he, x the rotation's change q x t
        double num;    // |v'|^2 - |v|^2 = 2 he . (2 w + x)
    };
    __device__ static __forceinline__ K kin(const float v[3], double C, double C2, double iC) {
        return lorentz32(v, C, C2, iC);
    }
    __device__ static __forceinline__ float hdx(double h) { return (float)h; }
    __device__ static __forceinline__ int drift(float& d, float u, float h) { return drift1f(d, u, h); }
    __device__ static __forceinline__ void weights(float d, float w[3]) { tscf(d, w); }
    __device__ static __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    __device__ static __forceinline__ void clean(float E[3], const float B[3]) {
        float eb = (E[0] * B[0] + E[1] * B[1]) + E[2] * B[2];
        float bb = (B[0] * B[0] + B[1] * B[1]) + B[2] * B[2];
        if (bb > 0.0f) {
            float f = eb / bb;
            E[0] = E[0] - f * B[0];
            E[1] = E[1] - f * B[1];
            E[2] = E[2] - f * B[2];
        }
    }
    // binary32 kick and rotation; 1/gamma of v0 in binary64.  The stored
    // v' is rounded to binary32, so v' - v and E_k(v') - E_k(v) of the stored
    // states would carry that rounding, about 1e-7 |v| and 1e-7 |v|^2, however
    // small the change itself.  The changes are therefore also formed in
    // binary64 from the step's own terms: v' - v = x + 2 he exactly, with x
    // = q x t the rotation's change (a product of binary32 numbers, exact in
    // binary64, minus another), and, because the rotation keeps |w + x| = |w|,
    // |v'|^2 - |v|^2 = 2 he . (2 w + x).
    __device__ static __forceinline__ void push(const float v[3], const float E[3], const float B[3],
                                                double hqd, double C, double C2, float vn[3],
                                                Inc& inc) {
        const float hq = (float)hqd;
        float he0 = hq * E[0], he1 = hq * E[1], he2 = hq * E[2];
        float w0 = v[0] + he0, w1 = v[1] + he1, w2 = v[2] + he2;
        double wd0 = w0, wd1 = w1, wd2 = w2;
        double rw = __builtin_sqrt(C2 + dot3(wd0, wd1, wd2, wd0, wd1, wd2));
        float fr = (float)(hqd * (C / rw));
        float t0 = fr * B[0], t1 = fr * B[1], t2 = fr * B[2];
        float p0 = w0 + (w1 * t2 - w2 * t1);
        float p1 = w1 + (w2 * t0 - w0 * t2);
        float p2 = w2 + (w0 * t1 - w1 * t0);
        float tt = (t0 * t0 + t1 * t1) + t2 * t2;
        float c2 = 2.0f / (1.0f + tt);
        float q0 = c2 * p0, q1 = c2 * p1, q2 = c2 * p2;
        vn[0] = (w0 + (q1 * t2 - q2 * t1)) + he0;
        vn[1] = (w1 + (q2 * t0 - q0 * t2)) + he1;
        vn[2] = (w2 + (q0 * t1 - q1 * t0)) + he2;
        const double x0 = (double)q1 * (double)t2 - (double)q2 * (double)t1;
        const double x1 = (double)q2 * (double)t0 - (double)q0 * (double)t2;
        const double x2 = (double)q0 * (double)t1 - (double)q1 * (double)t0;
        const double h0 = he0, h1 = he1, h2 = he2;
        inc.dv[0] = x0 + 2.0 * h0;
        inc.dv[1] = x1 + 2.0 * h1;
        inc.dv[2] = x2 + 2.0 * h2;
        inc.num = 2.0 * dot3(h0, h1, h2, 2.0 * wd0 + x0, 2.0 * wd1 + x1, 2.0 * wd2 + x2);
    }
    // E_k(v') - E_k(v) = (|v'|^2 - |v|^2) / (gamma' + gamma)  (Sec. 2.2, eq. parEk)
    __device__ static __forceinline__ void corrector(const float*, const float*, const K& k0,
                                                     const K& k1, const Inc& inc, double dv[3],
                                                     double& dek) {
        dv[0] = inc.dv[0];
        dv[1] = inc.dv[1];
        dv[2] = inc.dv[2];
        dek = inc.num / (k1.g + k0.g);
    }
};

}  // namespace mhdpic
