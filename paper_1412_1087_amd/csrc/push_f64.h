// Fused gather + Boris push + deposit, binary64 form.
//
// One work item = up to P particles whose half-step cell x^(n+1/2) lies in one
// tile of TX x TY (x TZ) cells.  The block stages in LDS:
//   F  : E and B of the tile plus one ghost layer, [cell][6] doubles;
//   Dc : -dM, -dE_k of the same cells, [cell][4] int64 (corrector, at x^(n+1/2));
//   Dp : n_CR, J_CR of the tile plus two ghost layers, [cell][4] int64
//        (at x^(n+1), one more cell of reach after the second half drift).
// Each particle's 3^NDIM-cell contributions go to LDS with 64-bit integer
// atomics; the block then adds the non-zero LDS cells to the global arrays
// with 64-bit atomics.  Integer sums make the result independent of the order
// in which particles, waves and blocks run.
#pragma once
#include "kernels.h"

namespace mhdpic {

struct PushArgs {
    PartF64 P;                 // tile-sorted particles, updated in place
    uint32_t* key;             // out: tile of the next half-step cell
    uint32_t* count;           // out: particles per next tile (pre-zeroed)
    const double* EB;          // [cells][6]
    int64_t* Dcorr;            // [4][cells] accumulated -dM, -dE_k
    int64_t* nJ;               // [4][cells] n_CR, J_CR at x^(n+1) (pre-zeroed)
    const BoxDev* boxes;
    const WorkItem* items;
    const uint32_t* n_items;
    uint32_t* err;
    int64_t NC;
};

template <int NDIM, int TX, int TY, int TZ>
struct Tiling {
    static constexpr int FX = TX + 2, FY = TY + 2, FZ = NDIM == 3 ? TZ + 2 : 1;
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = NDIM == 3 ? TZ + 4 : 1;
    static constexpr int NF = FX * FY * FZ;
    static constexpr int NP = PX * PY * PZ;
    static constexpr size_t lds_bytes() { return (size_t)NF * 6 * 8 + (size_t)NF * 4 * 8 + (size_t)NP * 4 * 8; }
};

template <int NDIM>
__device__ __forceinline__ int64_t global_cell(const BoxDev& bx, int x, int y, int z) {
    x = pmod(x, bx.n[0]);
    y = pmod(y, bx.n[1]);
    z = NDIM == 3 ? pmod(z, bx.n[2]) : 0;
    return bx.cell_off + ((int64_t)z * bx.n[1] + y) * bx.n[0] + x;
}

// Adds 4 channel amounts V[0..3] of one particle to an LDS box [cell][4]
// whose (-1,-1,-1) stencil corner is at cell index `base`.
template <int NDIM, int SX, int SY>
__device__ __forceinline__ void lds_deposit4(unsigned long long* box, int base, const double wx[3],
                                             const double wy[3], const double wz[3],
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
                double wxy = wx[ox] * wy[oy];
                double W = NDIM == 3 ? wxy * wz[oz] : wxy;
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

template <int NDIM, int TX, int TY, int TZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_push_f64(PushArgs a) {
    using TL = Tiling<NDIM, TX, TY, TZ>;
    extern __shared__ __align__(16) unsigned char smem[];
    double* F = reinterpret_cast<double*>(smem);
    unsigned long long* Dc = reinterpret_cast<unsigned long long*>(smem + (size_t)TL::NF * 48);
    unsigned long long* Dp = Dc + (size_t)TL::NF * 4;

    // XCD-aware mapping: consecutive (spatially adjacent) items go to the
    // same XCD, whose L2 then holds their fields and deposits.
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

    // stage fields of the tile + 1 ghost layer, zero the deposit boxes
    for (int c = threadIdx.x; c < TL::NF; c += BLOCK) {
        int lx = c % TL::FX, ly = (c / TL::FX) % TL::FY, lz = c / (TL::FX * TL::FY);
        double* f = F + 6 * c;
        if (lx < sx + 2 && ly < sy + 2 && lz < fz_used) {
            int64_t g = global_cell<NDIM>(bx, ox + lx - 1, oy + ly - 1, NDIM == 3 ? oz + lz - 1 : 0);
            const double* s = a.EB + 6 * g;
#pragma unroll
            for (int q = 0; q < 6; ++q) f[q] = s[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Dc[4 * c + q] = 0ull;
    }
    for (int c = threadIdx.x; c < TL::NP * 4; c += BLOCK) Dp[c] = 0ull;
    __syncthreads();

    const double C = bx.C, C2 = bx.C2, iC = bx.iC, S = bx.S, hdt = bx.hdt;
    const double hdx0 = bx.hdx[0], hdx1 = bx.hdx[1], hdx2 = bx.hdx[2];
    const int3 T = make_int3(TX, TY, TZ);
    uint32_t errbits = 0;

    for (int base = w.begin; base < w.end; base += BLOCK) {
        const int j = base + (int)threadIdx.x;
        const bool act = j < w.end;
        uint32_t nkey = 0;
        if (act) {
            int i[3];
            unpack_cell<NDIM>(a.P.cell[j], i[0], i[1], i[2]);
            double dl[3] = {a.P.d[0][j], a.P.d[1][j], NDIM == 3 ? a.P.d[2][j] : 0.0};
            double v[3] = {a.P.v[0][j], a.P.v[1][j], a.P.v[2][j]};
            const double m = a.P.m[j], qm = a.P.qm[j];

            Kin k0 = lorentz(v, C, C2, iC);
            // drift to x^(n+1/2)
            int s0 = drift1(dl[0], k0.u[0], hdx0);
            int s1 = drift1(dl[1], k0.u[1], hdx1);
            int s2 = NDIM == 3 ? drift1(dl[2], k0.u[2], hdx2) : 0;
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

            // TSC gather of E, B at x^(n+1/2)
            double wx[3], wy[3], wz[3] = {0.0, 1.0, 0.0};
            tsc(dl[0], wx);
            tsc(dl[1], wy);
            if (NDIM == 3) tsc(dl[2], wz);
            const int fbase = (lz * TL::FY + ly) * TL::FX + lx;
            double E[3] = {0.0, 0.0, 0.0}, Bp[3] = {0.0, 0.0, 0.0};
            constexpr int ZN = NDIM == 3 ? 3 : 1;
#pragma unroll
            for (int oz2 = 0; oz2 < ZN; ++oz2) {
#pragma unroll
                for (int oy2 = 0; oy2 < 3; ++oy2) {
#pragma unroll
                    for (int ox2 = 0; ox2 < 3; ++ox2) {
                        double wxy = wx[ox2] * wy[oy2];
                        double W = NDIM == 3 ? wxy * wz[oz2] : wxy;
                        const double* f = F + 6 * (fbase + (oz2 * TL::FY + oy2) * TL::FX + ox2);
                        E[0] = __builtin_fma(W, f[0], E[0]);
                        E[1] = __builtin_fma(W, f[1], E[1]);
                        E[2] = __builtin_fma(W, f[2], E[2]);
                        Bp[0] = __builtin_fma(W, f[3], Bp[0]);
                        Bp[1] = __builtin_fma(W, f[4], Bp[1]);
                        Bp[2] = __builtin_fma(W, f[5], Bp[2]);
                    }
                }
            }
            clean_parallel(E, Bp);

            // kick - rotate - kick
            const double hq = qm * hdt;
            double vn[3];
            boris(v, E, Bp, hq, C, C2, vn);
            if (!isfinite(vn[0]) || !isfinite(vn[1]) || !isfinite(vn[2])) errbits |= ERRBIT_NONFINITE;
            Kin k1 = lorentz(vn, C, C2, iC);

            // corrector feedback at x^(n+1/2): -dM, -dE_k (App. A.3)
            double Vc[4];
            Vc[0] = (-(m * (vn[0] - v[0]))) * S;
            Vc[1] = (-(m * (vn[1] - v[1]))) * S;
            Vc[2] = (-(m * (vn[2] - v[2]))) * S;
            Vc[3] = (-(m * (k1.ek - k0.ek))) * S;
            bool okc = fabs(Vc[0]) < kMaxAmount && fabs(Vc[1]) < kMaxAmount &&
                       fabs(Vc[2]) < kMaxAmount && fabs(Vc[3]) < kMaxAmount;
            if (okc) lds_deposit4<NDIM, TL::FX, TL::FY>(Dc, fbase, wx, wy, wz, Vc);
            else errbits |= ERRBIT_RANGE;

            // drift to x^(n+1)
            int t0 = drift1(dl[0], k1.u[0], hdx0);
            int t1 = drift1(dl[1], k1.u[1], hdx1);
            int t2 = NDIM == 3 ? drift1(dl[2], k1.u[2], hdx2) : 0;
            i[0] = wrap_shift(i[0], t0, bx.n[0]);
            i[1] = wrap_shift(i[1], t1, bx.n[1]);
            if (NDIM == 3) i[2] = wrap_shift(i[2], t2, bx.n[2]);
            // (-1,-1,-1) corner in the Dp box, whose origin is the tile origin - 2
            const int pbase = NDIM == 3
                                  ? ((lz + t2 + 1) * TL::PY + (ly + t1 + 1)) * TL::PX + (lx + t0 + 1)
                                  : (ly + t1 + 1) * TL::PX + (lx + t0 + 1);

            // n_CR, J_CR at x^(n+1) (predictor input of the next step)
            tsc(dl[0], wx);
            tsc(dl[1], wy);
            if (NDIM == 3) tsc(dl[2], wz);
            const double qmm = qm * m;
            double Vp[4];
            Vp[0] = qmm * S;
            Vp[1] = (qmm * k1.u[0]) * S;
            Vp[2] = (qmm * k1.u[1]) * S;
            Vp[3] = (qmm * k1.u[2]) * S;
            bool okp = fabs(Vp[0]) < kMaxAmount && fabs(Vp[1]) < kMaxAmount &&
                       fabs(Vp[2]) < kMaxAmount && fabs(Vp[3]) < kMaxAmount;
            if (okp) lds_deposit4<NDIM, TL::PX, TL::PY>(Dp, pbase, wx, wy, wz, Vp);
            else errbits |= ERRBIT_RANGE;

            // store x^(n+1), v^(n+1)
            a.P.cell[j] = pack_cell<NDIM>(i[0], i[1], i[2]);
            a.P.d[0][j] = dl[0];
            a.P.d[1][j] = dl[1];
            if (NDIM == 3) a.P.d[2][j] = dl[2];
            a.P.v[0][j] = vn[0];
            a.P.v[1][j] = vn[1];
            a.P.v[2][j] = vn[2];

            // tile of the next half-step cell (same operations as the next step)
            int ni[3] = {i[0], i[1], i[2]};
            double e0 = dl[0], e1 = dl[1], e2 = dl[2];
            ni[0] = wrap_shift(ni[0], drift1(e0, k1.u[0], hdx0), bx.n[0]);
            ni[1] = wrap_shift(ni[1], drift1(e1, k1.u[1], hdx1), bx.n[1]);
            if (NDIM == 3) ni[2] = wrap_shift(ni[2], drift1(e2, k1.u[2], hdx2), bx.n[2]);
            nkey = tile_of<NDIM>(bx, T, ni[0], ni[1], ni[2]);
            a.key[j] = nkey;
        }
        wave_claim(a.count, nkey, act);
    }
    if (errbits) latch(a.err, errbits);
    __syncthreads();

    // flush the LDS boxes into the global arrays
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
