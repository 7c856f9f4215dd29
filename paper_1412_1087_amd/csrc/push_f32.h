// Precision form of the fused gather + push + deposit.
//
// Offsets, velocities, fields, TSC weights, the gather and the Boris rotation
// run in binary32.  Binary64 is kept where cancellation or the fixed point
// needs it: the Lorentz factors (and so u and E_k), the rotation's 1/gamma,
// the feedback amounts -m dv, -m dE_k, (q/mc) m u, and the quantisation of
// every contribution (fma of the binary32 weight with the binary64 amount).
// Deposits are the same exact int64 fixed point as the binary64 form.
#pragma once
#include "kernels.h"
#include "push_f64.h"

namespace mhdpic {

struct PushArgs32 {
    PartF32 P;
    uint32_t* key;
    uint32_t* count;
    const float* EB;  // [cells][6]
    int64_t* Dcorr;
    int64_t* nJ;
    const BoxDev* boxes;
    const WorkItem* items;
    const uint32_t* n_items;
    uint32_t* err;
    int64_t NC;
};

template <int NDIM, int TX, int TY, int TZ>
struct Tiling32 {
    static constexpr int FX = TX + 2, FY = TY + 2, FZ = NDIM == 3 ? TZ + 2 : 1;
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = NDIM == 3 ? TZ + 4 : 1;
    static constexpr int NF = FX * FY * FZ;
    static constexpr int NP = PX * PY * PZ;
    static constexpr size_t lds_bytes() { return (size_t)NF * 4 * 8 + (size_t)NP * 4 * 8 + (size_t)NF * 6 * 4; }
};

struct Kin32 {
    float u[3];
    double ek;
};

// gamma in binary64 from binary32 four-velocity; u rounded to binary32.
__device__ __forceinline__ Kin32 lorentz32(const float v[3], double C, double C2, double iC) {
    Kin32 k;
    double v0 = v[0], v1 = v[1], v2 = v[2];
    double s = dot3(v0, v1, v2, v0, v1, v2);
    double r = __builtin_sqrt(C2 + s);
    double g = r * iC;
    double ig = C / r;
    k.u[0] = (float)(v0 * ig);
    k.u[1] = (float)(v1 * ig);
    k.u[2] = (float)(v2 * ig);
    k.ek = s / (g + 1.0);
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

template <int NDIM, int SX, int SY>
__device__ __forceinline__ void lds_deposit4f(unsigned long long* box, int base, const float wx[3],
                                              const float wy[3], const float wz[3],
                                              const double V[4]) {
    int64_t acc[4] = {0, 0, 0, 0};
    int64_t tot[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) tot[c] = quant1(V[c]);
    unsigned long long* p0 = box + 4 * base;
    constexpr int ZN = NDIM == 3 ? 3 : 1;
#pragma unroll
    for (int oz = 0; oz < ZN; ++oz) {
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const bool centre = ox == 1 && oy == 1 && (NDIM == 2 || oz == 1);
                if (centre) continue;
                float wxy = wx[ox] * wy[oy];
                double W = (double)(NDIM == 3 ? wxy * wz[oz] : wxy);
                unsigned long long* p = p0 + 4 * ((oz * SY + oy) * SX + ox);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    int64_t q = quant(W, V[c]);
                    acc[c] += q;
                    atomicAdd(p + c, (unsigned long long)q);
                }
            }
        }
    }
    constexpr int CZ = NDIM == 3 ? 1 : 0;
    unsigned long long* pc = p0 + 4 * ((CZ * SY + 1) * SX + 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) atomicAdd(pc + c, (unsigned long long)(tot[c] - acc[c]));
}

// Deposit over a stencil into global memory (initialisation only).
template <int NDIM>
__device__ __forceinline__ void deposit_global_f(int64_t* dst, const BoxDev& bx, const int i[3],
                                                 const float wx[3], const float wy[3],
                                                 const float wz[3], double V) {
    int64_t tot = quant1(V);
    int64_t acc = 0;
    const int zlo = NDIM == 3 ? 0 : 1, zhi = NDIM == 3 ? 2 : 1;
    int64_t centre = 0;
    for (int oz = zlo; oz <= zhi; ++oz)
        for (int oy = 0; oy < 3; ++oy)
            for (int ox = 0; ox < 3; ++ox) {
                int cx = pmod(i[0] + ox - 1, bx.n[0]);
                int cy = pmod(i[1] + oy - 1, bx.n[1]);
                int cz = NDIM == 3 ? pmod(i[2] + oz - 1, bx.n[2]) : 0;
                int64_t g = bx.cell_off + ((int64_t)cz * bx.n[1] + cy) * bx.n[0] + cx;
                if (ox == 1 && oy == 1 && oz == 1) {
                    centre = g;
                    continue;
                }
                float wxy = wx[ox] * wy[oy];
                double W = (double)(NDIM == 3 ? wxy * wz[oz] : wxy);
                int64_t q = quant(W, V);
                acc += q;
                atomicAdd((unsigned long long*)&dst[g], (unsigned long long)q);
            }
    atomicAdd((unsigned long long*)&dst[centre], (unsigned long long)(tot - acc));
}

template <int NDIM>
__global__ void k_deposit_nJ_global_f32(PartF32 P, int64_t* __restrict__ nJ, int64_t NC,
                                        const BoxDev* __restrict__ boxes,
                                        const int64_t* __restrict__ part_off, int nb, int64_t N,
                                        uint32_t* err) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const BoxDev& bx = boxes[find_box(part_off, nb, j)];
    int i[3];
    unpack_cell<NDIM>(P.cell[j], i[0], i[1], i[2]);
    float wx[3], wy[3], wz[3] = {0.0f, 1.0f, 0.0f};
    tscf(P.d[0][j], wx);
    tscf(P.d[1][j], wy);
    if (NDIM == 3) tscf(P.d[2][j], wz);
    float v[3] = {P.v[0][j], P.v[1][j], P.v[2][j]};
    Kin32 k = lorentz32(v, bx.C, bx.C2, bx.iC);
    double qmm = (double)P.qm[j] * (double)P.m[j];
    double V[4] = {qmm * bx.S, (qmm * (double)k.u[0]) * bx.S, (qmm * (double)k.u[1]) * bx.S,
                   (qmm * (double)k.u[2]) * bx.S};
    for (int c = 0; c < 4; ++c) {
        if (!(fabs(V[c]) < kMaxAmount)) {
            latch(err, ERRBIT_RANGE);
            continue;
        }
        deposit_global_f<NDIM>(nJ + c * NC, bx, i, wx, wy, wz, V[c]);
    }
}

// Key = tile of x^(n+1/2) with the binary32 drift of the precision form.
template <int NDIM>
__global__ void k_rekey_f32(PartF32 P, uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                            const BoxDev* __restrict__ boxes, const int64_t* __restrict__ part_off,
                            int nb, int64_t N, int3 T) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = j < N;
    uint32_t k = 0;
    if (act) {
        const BoxDev& bx = boxes[find_box(part_off, nb, j)];
        int i[3];
        unpack_cell<NDIM>(P.cell[j], i[0], i[1], i[2]);
        float v[3] = {P.v[0][j], P.v[1][j], P.v[2][j]};
        Kin32 kn = lorentz32(v, bx.C, bx.C2, bx.iC);
        for (int d = 0; d < NDIM; ++d) {
            float dl = P.d[d][j];
            int s = drift1f(dl, kn.u[d], (float)bx.hdx[d]);
            i[d] = wrap_shift(i[d], s, bx.n[d]);
        }
        k = tile_of<NDIM>(bx, T, i[0], i[1], i[2]);
        key[j] = k;
    }
    wave_claim(count, k, act);
}

template <int NDIM, int TX, int TY, int TZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_push_f32(PushArgs32 a) {
    using TL = Tiling32<NDIM, TX, TY, TZ>;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* Dc = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* Dp = Dc + (size_t)TL::NF * 4;
    float* F = reinterpret_cast<float*>(Dp + (size_t)TL::NP * 4);

    const uint32_t nitems = *a.n_items;
    const uint32_t per_xcd = (nitems + 7u) / 8u;
    const uint32_t bid = blockIdx.x;
    const uint32_t slot = bid >> 3;
    if (slot >= per_xcd) return;
    const uint32_t item = (bid & 7u) * per_xcd + slot;
    if (item >= nitems) return;
    const WorkItem w = a.items[item];
    const BoxDev& bx = a.boxes[w.box];

    const int lt = w.tile - bx.tile_off;
    const int ntx = bx.nt[0], nty = bx.nt[1];
    const int tx = lt % ntx, ty = (lt / ntx) % nty, tz = NDIM == 3 ? lt / (ntx * nty) : 0;
    const int ox = tx * TX, oy = ty * TY, oz = tz * TZ;
    const int sx = min(TX, bx.n[0] - ox), sy = min(TY, bx.n[1] - oy);
    const int sz = NDIM == 3 ? min(TZ, bx.n[2] - oz) : 1;
    const int fz_used = NDIM == 3 ? sz + 2 : 1;
    const int pz_used = NDIM == 3 ? sz + 4 : 1;

    for (int c = threadIdx.x; c < TL::NF; c += BLOCK) {
        int lx = c % TL::FX, ly = (c / TL::FX) % TL::FY, lz = c / (TL::FX * TL::FY);
        float* f = F + 6 * c;
        if (lx < sx + 2 && ly < sy + 2 && lz < fz_used) {
            int64_t g = global_cell<NDIM>(bx, ox + lx - 1, oy + ly - 1, NDIM == 3 ? oz + lz - 1 : 0);
            const float* s = a.EB + 6 * g;
#pragma unroll
            for (int q = 0; q < 6; ++q) f[q] = s[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Dc[4 * c + q] = 0ull;
    }
    for (int c = threadIdx.x; c < TL::NP * 4; c += BLOCK) Dp[c] = 0ull;
    __syncthreads();

    const double C = bx.C, C2 = bx.C2, iC = bx.iC, S = bx.S, hdt = bx.hdt;
    const float hdx0 = (float)bx.hdx[0], hdx1 = (float)bx.hdx[1], hdx2 = (float)bx.hdx[2];
    const int3 T = make_int3(TX, TY, TZ);
    uint32_t errbits = 0;

    for (int base = w.begin; base < w.end; base += BLOCK) {
        const int j = base + (int)threadIdx.x;
        const bool act = j < w.end;
        uint32_t nkey = 0;
        if (act) {
            int i[3];
            unpack_cell<NDIM>(a.P.cell[j], i[0], i[1], i[2]);
            float dl[3] = {a.P.d[0][j], a.P.d[1][j], NDIM == 3 ? a.P.d[2][j] : 0.0f};
            float v[3] = {a.P.v[0][j], a.P.v[1][j], a.P.v[2][j]};
            const double m = (double)a.P.m[j], qm = (double)a.P.qm[j];

            Kin32 k0 = lorentz32(v, C, C2, iC);
            int s0 = drift1f(dl[0], k0.u[0], hdx0);
            int s1 = drift1f(dl[1], k0.u[1], hdx1);
            int s2 = NDIM == 3 ? drift1f(dl[2], k0.u[2], hdx2) : 0;
            i[0] = wrap_shift(i[0], s0, bx.n[0]);
            i[1] = wrap_shift(i[1], s1, bx.n[1]);
            if (NDIM == 3) i[2] = wrap_shift(i[2], s2, bx.n[2]);
            int lx = i[0] - ox, ly = i[1] - oy, lz = NDIM == 3 ? i[2] - oz : 0;
            bool inside = lx >= 0 && lx < sx && ly >= 0 && ly < sy && lz >= 0 && lz < sz;
            if (!inside) {
                errbits |= ERRBIT_STATE;
                lx = min(max(lx, 0), sx - 1);
                ly = min(max(ly, 0), sy - 1);
                lz = NDIM == 3 ? min(max(lz, 0), sz - 1) : 0;
            }

            float wx[3], wy[3], wz[3] = {0.0f, 1.0f, 0.0f};
            tscf(dl[0], wx);
            tscf(dl[1], wy);
            if (NDIM == 3) tscf(dl[2], wz);
            const int fbase = (lz * TL::FY + ly) * TL::FX + lx;
            float E[3] = {0.0f, 0.0f, 0.0f}, Bp[3] = {0.0f, 0.0f, 0.0f};
            constexpr int ZN = NDIM == 3 ? 3 : 1;
#pragma unroll
            for (int oz2 = 0; oz2 < ZN; ++oz2) {
#pragma unroll
                for (int oy2 = 0; oy2 < 3; ++oy2) {
#pragma unroll
                    for (int ox2 = 0; ox2 < 3; ++ox2) {
                        float wxy = wx[ox2] * wy[oy2];
                        float W = NDIM == 3 ? wxy * wz[oz2] : wxy;
                        const float* f = F + 6 * (fbase + (oz2 * TL::FY + oy2) * TL::FX + ox2);
                        E[0] = __builtin_fmaf(W, f[0], E[0]);
                        E[1] = __builtin_fmaf(W, f[1], E[1]);
                        E[2] = __builtin_fmaf(W, f[2], E[2]);
                        Bp[0] = __builtin_fmaf(W, f[3], Bp[0]);
                        Bp[1] = __builtin_fmaf(W, f[4], Bp[1]);
                        Bp[2] = __builtin_fmaf(W, f[5], Bp[2]);
                    }
                }
            }
            {
                float eb = (E[0] * Bp[0] + E[1] * Bp[1]) + E[2] * Bp[2];
                float bb = (Bp[0] * Bp[0] + Bp[1] * Bp[1]) + Bp[2] * Bp[2];
                if (bb > 0.0f) {
                    float f = eb / bb;
                    E[0] = E[0] - f * Bp[0];
                    E[1] = E[1] - f * Bp[1];
                    E[2] = E[2] - f * Bp[2];
                }
            }

            // kick - rotate - kick: binary32 except 1/gamma of v0
            const double hqd = qm * hdt;
            const float hq = (float)hqd;
            float he0 = hq * E[0], he1 = hq * E[1], he2 = hq * E[2];
            float w0 = v[0] + he0, w1 = v[1] + he1, w2 = v[2] + he2;
            double wd0 = w0, wd1 = w1, wd2 = w2;
            double rw = __builtin_sqrt(C2 + dot3(wd0, wd1, wd2, wd0, wd1, wd2));
            float fr = (float)(hqd * (C / rw));
            float t0 = fr * Bp[0], t1 = fr * Bp[1], t2 = fr * Bp[2];
            float p0 = w0 + (w1 * t2 - w2 * t1);
            float p1 = w1 + (w2 * t0 - w0 * t2);
            float p2 = w2 + (w0 * t1 - w1 * t0);
            float tt = (t0 * t0 + t1 * t1) + t2 * t2;
            float c2 = 2.0f / (1.0f + tt);
            float q0 = c2 * p0, q1 = c2 * p1, q2 = c2 * p2;
            float vn[3];
            vn[0] = (w0 + (q1 * t2 - q2 * t1)) + he0;
            vn[1] = (w1 + (q2 * t0 - q0 * t2)) + he1;
            vn[2] = (w2 + (q0 * t1 - q1 * t0)) + he2;
            if (!isfinite(vn[0]) || !isfinite(vn[1]) || !isfinite(vn[2])) errbits |= ERRBIT_NONFINITE;
            Kin32 k1 = lorentz32(vn, C, C2, iC);

            double Vc[4];
            Vc[0] = (-(m * ((double)vn[0] - (double)v[0]))) * S;
            Vc[1] = (-(m * ((double)vn[1] - (double)v[1]))) * S;
            Vc[2] = (-(m * ((double)vn[2] - (double)v[2]))) * S;
            Vc[3] = (-(m * (k1.ek - k0.ek))) * S;
            bool okc = fabs(Vc[0]) < kMaxAmount && fabs(Vc[1]) < kMaxAmount &&
                       fabs(Vc[2]) < kMaxAmount && fabs(Vc[3]) < kMaxAmount;
            if (okc) lds_deposit4f<NDIM, TL::FX, TL::FY>(Dc, fbase, wx, wy, wz, Vc);
            else errbits |= ERRBIT_RANGE;

            int t0s = drift1f(dl[0], k1.u[0], hdx0);
            int t1s = drift1f(dl[1], k1.u[1], hdx1);
            int t2s = NDIM == 3 ? drift1f(dl[2], k1.u[2], hdx2) : 0;
            i[0] = wrap_shift(i[0], t0s, bx.n[0]);
            i[1] = wrap_shift(i[1], t1s, bx.n[1]);
            if (NDIM == 3) i[2] = wrap_shift(i[2], t2s, bx.n[2]);
            const int pbase = NDIM == 3
                                  ? ((lz + t2s + 1) * TL::PY + (ly + t1s + 1)) * TL::PX + (lx + t0s + 1)
                                  : (ly + t1s + 1) * TL::PX + (lx + t0s + 1);
            tscf(dl[0], wx);
            tscf(dl[1], wy);
            if (NDIM == 3) tscf(dl[2], wz);
            const double qmm = qm * m;
            double Vp[4];
            Vp[0] = qmm * S;
            Vp[1] = (qmm * (double)k1.u[0]) * S;
            Vp[2] = (qmm * (double)k1.u[1]) * S;
            Vp[3] = (qmm * (double)k1.u[2]) * S;
            bool okp = fabs(Vp[0]) < kMaxAmount && fabs(Vp[1]) < kMaxAmount &&
                       fabs(Vp[2]) < kMaxAmount && fabs(Vp[3]) < kMaxAmount;
            if (okp) lds_deposit4f<NDIM, TL::PX, TL::PY>(Dp, pbase, wx, wy, wz, Vp);
            else errbits |= ERRBIT_RANGE;

            a.P.cell[j] = pack_cell<NDIM>(i[0], i[1], i[2]);
            a.P.d[0][j] = dl[0];
            a.P.d[1][j] = dl[1];
            if (NDIM == 3) a.P.d[2][j] = dl[2];
            a.P.v[0][j] = vn[0];
            a.P.v[1][j] = vn[1];
            a.P.v[2][j] = vn[2];

            int ni[3] = {i[0], i[1], i[2]};
            float e0 = dl[0], e1 = dl[1], e2 = dl[2];
            ni[0] = wrap_shift(ni[0], drift1f(e0, k1.u[0], hdx0), bx.n[0]);
            ni[1] = wrap_shift(ni[1], drift1f(e1, k1.u[1], hdx1), bx.n[1]);
            if (NDIM == 3) ni[2] = wrap_shift(ni[2], drift1f(e2, k1.u[2], hdx2), bx.n[2]);
            nkey = tile_of<NDIM>(bx, T, ni[0], ni[1], ni[2]);
            a.key[j] = nkey;
        }
        wave_claim(a.count, nkey, act);
    }
    if (errbits) latch(a.err, errbits);
    __syncthreads();

    const int64_t NC = a.NC;
    for (int c = threadIdx.x; c < TL::NF; c += BLOCK) {
        int lx = c % TL::FX, ly = (c / TL::FX) % TL::FY, lz = c / (TL::FX * TL::FY);
        if (!(lx < sx + 2 && ly < sy + 2 && lz < fz_used)) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx - 1, oy + ly - 1, NDIM == 3 ? oz + lz - 1 : 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dc[4 * c + q];
            if (val) atomicAdd((unsigned long long*)&a.Dcorr[q * NC + g], val);
        }
    }
    for (int c = threadIdx.x; c < TL::NP; c += BLOCK) {
        int lx = c % TL::PX, ly = (c / TL::PX) % TL::PY, lz = c / (TL::PX * TL::PY);
        if (!(lx < sx + 4 && ly < sy + 4 && lz < pz_used)) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx - 2, oy + ly - 2, NDIM == 3 ? oz + lz - 2 : 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dp[4 * c + q];
            if (val) atomicAdd((unsigned long long*)&a.nJ[q * NC + g], val);
        }
    }
}

}  // namespace mhdpic
