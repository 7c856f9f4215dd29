// Fused gather + Boris push + deposit (App. A.2, A.3), both precision forms.
//
// One work item = up to P particles whose half-step cell x^(n+1/2) lies in one
// tile of TX x TY (x TZ) cells.  The block stages three LDS boxes on one index
// geometry, the tile plus two ghost layers (strides PX = TX+4, PY = TY+4):
//   F  : E and B of the tile plus one ghost layer, [6][cells];
//   Dc : -dM, -dE_k at x^(n+1/2), same cells as F, [4][cells] int64;
//   Dp : n_CR, J_CR at x^(n+1), all cells, [4][cells] int64.
// F and Dc skip the outermost plane (rows in 2D) on each side, which they
// never touch.  Because the three boxes share strides, a particle's cell has
// the same LDS bank in all of them; the binning orders particles so that 16
// consecutive lanes have distinct bank residues.
//
// Each particle's 3^NDIM contributions per channel go to LDS with 64-bit
// integer atomics; the block then adds the non-zero LDS cells to the global
// arrays with 64-bit atomics.  Integer sums make the result independent of the
// order in which particles, waves and blocks run.
#pragma once
#include "kernels.h"

namespace mhdpic {

template <class Pol>
struct PushArgsT {
    typename Pol::Part P;        // tile-sorted particles, updated in place
    uint16_t* code;              // out: code word (pack_code)
    uint32_t* cnt;               // out: [item][code] particle counts
    const typename Pol::R* EB;   // [cells][6] E and B
    int64_t* Dcorr;              // [4][cells] accumulated -dM, -dE_k
    int64_t* nJ;                 // [4][cells] n_CR, J_CR at x^(n+1) (pre-zeroed)
    const BoxDev* boxes;
    const WorkItem* items;
    const uint32_t* n_items;
    uint32_t* err;
    int64_t NC;
    int32_t do_pred;             // 0: skip n_CR, J_CR (a sub-step before the last)
};

template <class Pol, int NDIM, int TX, int TY, int TZ>
struct Geo {
    using R = typename Pol::R;
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = NDIM == 3 ? TZ + 4 : 1;
    static constexpr int NP = PX * PY * PZ;
    static constexpr int FOFF = NDIM == 3 ? PX * PY : PX;  // skipped leading plane/row
    static constexpr int NFF = NP - 2 * FOFF;
    static constexpr int CORNER = NDIM == 3 ? PX * PY + PX + 1 : PX + 1;
    static constexpr size_t lds_bytes() {
        return (size_t)NFF * 4 * 8 + (size_t)NP * 4 * 8 + (size_t)NFF * 6 * sizeof(R);
    }
    // index of tile-local cell (lx, ly, lz), each in [-2, extent + 2)
    __device__ static __forceinline__ int index(int lx, int ly, int lz) {
        return NDIM == 3 ? ((lz + 2) * PY + (ly + 2)) * PX + (lx + 2) : (ly + 2) * PX + (lx + 2);
    }
    __device__ static __forceinline__ void coords(int p, int& lx, int& ly, int& lz) {
        lx = p % PX - 2;
        ly = (p / PX) % PY - 2;
        lz = NDIM == 3 ? p / (PX * PY) - 2 : 0;
    }
};

// Adds 4 channel amounts V[0..3] of one particle to an LDS box [4][NB] whose
// (-1,-1,-1) stencil corner is at index `base`; weights in the working
// precision, quantised against the binary64 amounts.
template <class Pol, int NDIM, int SX, int SY, int NB>
__device__ __forceinline__ void lds_deposit4(unsigned long long* box, int base,
                                             const typename Pol::R wx[3],
                                             const typename Pol::R wy[3],
                                             const typename Pol::R wz[3], const double V[4]) {
    using R = typename Pol::R;
    int64_t acc[4] = {0, 0, 0, 0};
    int64_t tot[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) tot[c] = quant1(V[c]);
    unsigned long long* p0 = box + base;
    constexpr int ZN = NDIM == 3 ? 3 : 1;
#pragma unroll 1
    for (int oz = 0; oz < ZN; ++oz) {
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const bool centre = ox == 1 && oy == 1 && (NDIM == 2 || oz == 1);
                if (centre) continue;
                R wxy = wx[ox] * wy[oy];
                double W = (double)(NDIM == 3 ? wxy * wz[oz] : wxy);
                unsigned long long* p = p0 + (oz * SY + oy) * SX + ox;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    int64_t q = quant(W, V[c]);
                    // keep q opaque: otherwise the compiler sums the raw fma
                    // bits and keeps a second copy of every q for the atomic
                    asm("" : "+v"(q));
                    acc[c] += q;
                    atomicAdd(p + c * NB, (unsigned long long)q);
                }
            }
        }
    }
    constexpr int CZ = NDIM == 3 ? 1 : 0;
    unsigned long long* pc = p0 + (CZ * SY + 1) * SX + 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) atomicAdd(pc + c * NB, (unsigned long long)(tot[c] - acc[c]));
}

// One particle's stored state (in 2D the third offset reads as 0).
template <int NDIM, typename R>
struct PartRec {
    uint32_t cell = 0;
    R d[3] = {R(0), R(0), R(0)}, v[3] = {R(0), R(0), R(0)};
    R m = R(0), qm = R(0);
    template <typename PS>
    __device__ __forceinline__ void load(const PS& P, int j) {
        cell = P.cell[j];
        d[0] = P.d[0][j];
        d[1] = P.d[1][j];
        d[2] = NDIM == 3 ? P.d[2][j] : R(0);
        v[0] = P.v[0][j];
        v[1] = P.v[1][j];
        v[2] = P.v[2][j];
        m = P.m[j];
        qm = P.qm[j];
    }
};

template <class Pol, int NDIM, int TX, int TY, int TZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_push(PushArgsT<Pol> a) {
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    using R = typename Pol::R;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* Dc = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* Dp = Dc + (size_t)G::NFF * 4;
    R* F = reinterpret_cast<R*>(Dp + (size_t)G::NP * 4);
    constexpr int K = Codes<NDIM>::K;
    __shared__ uint32_t s_cnt[K];

    uint32_t item;
    if (!item_of_block(a.n_items, item)) return;
    for (int c = threadIdx.x; c < K; c += BLOCK) s_cnt[c] = 0;
    const WorkItem w = a.items[item];
    const BoxDev bx = a.boxes[w.box];  // a copy: kept in registers across the stores
    int tx, ty, tz;
    tile_coords<NDIM>(bx, w.tile, tx, ty, tz);
    const int ox = tile_origin(bx, 0, tx, TX), oy = tile_origin(bx, 1, ty, TY);
    const int oz = NDIM == 3 ? tile_origin(bx, 2, tz, TZ) : 0;
    const int sx = tile_extent(bx, 0, tx, TX), sy = tile_extent(bx, 1, ty, TY);
    const int sz = NDIM == 3 ? tile_extent(bx, 2, tz, TZ) : 1;

    // stage E, B of the tile + 1 ghost layer; zero the deposit boxes
    for (int c = threadIdx.x; c < G::NFF; c += BLOCK) {
        int lx, ly, lz;
        G::coords(c + G::FOFF, lx, ly, lz);
        bool in = lx >= -1 && lx <= sx && ly >= -1 && ly <= sy && (NDIM == 2 || (lz >= -1 && lz <= sz));
        if (in) {
            int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
            const R* s = a.EB + 6 * g;
#pragma unroll
            for (int q = 0; q < 6; ++q) F[q * G::NFF + c] = s[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Dc[q * G::NFF + c] = 0ull;
    }
    const bool do_pred = a.do_pred != 0;
    if (do_pred)
        for (int c = threadIdx.x; c < G::NP * 4; c += BLOCK) Dp[c] = 0ull;
    __syncthreads();

    const double C = bx.C, C2 = bx.C2, iC = bx.iC, S = bx.S, hdt = bx.hdt;
    const R hx = Pol::hdx(bx.hdx[0]), hy = Pol::hdx(bx.hdx[1]), hz = Pol::hdx(bx.hdx[2]);
    const int3 T = make_int3(TX, TY, TZ);
    uint32_t errbits = 0;

    // In 3D the next particle is loaded while this one is pushed: binary64
    // runs two waves per SIMD (LDS-limited), so registers are free, and the
    // binary32 kernel still fits the 128 registers of four waves per SIMD.
    // In 2D the registers are not there.
    constexpr bool kPrefetch = NDIM == 3;
    PartRec<NDIM, R> nxt;
    if (kPrefetch && w.begin + (int)threadIdx.x < w.end) nxt.load(a.P, w.begin + (int)threadIdx.x);
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += BLOCK) {
        PartRec<NDIM, R> cur;
        if (kPrefetch) {
            cur = nxt;
            if (j + BLOCK < w.end) nxt.load(a.P, j + BLOCK);
        } else {
            cur.load(a.P, j);
        }
        int i[3];
        unpack_cell<NDIM>(cur.cell, i[0], i[1], i[2]);
        R dl[3] = {cur.d[0], cur.d[1], cur.d[2]};
        R v[3] = {cur.v[0], cur.v[1], cur.v[2]};
        const double m = (double)cur.m, qm = (double)cur.qm;

        typename Pol::K k0 = Pol::kin(v, C, C2, iC);
        // drift to x^(n+1/2)
        int s0 = Pol::drift(dl[0], k0.u[0], hx);
        int s1 = Pol::drift(dl[1], k0.u[1], hy);
        int s2 = NDIM == 3 ? Pol::drift(dl[2], k0.u[2], hz) : 0;
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
        const int corner = G::index(lx, ly, lz) - G::CORNER;  // (-1,-1,-1) neighbour
        const int fbase = corner - G::FOFF;

        // TSC gather of E, B at x^(n+1/2)
        R wx[3], wy[3], wz[3] = {R(0), R(1), R(0)};
        Pol::weights(dl[0], wx);
        Pol::weights(dl[1], wy);
        if (NDIM == 3) Pol::weights(dl[2], wz);
        R E[3] = {R(0), R(0), R(0)}, Bp[3] = {R(0), R(0), R(0)};
        constexpr int ZN = NDIM == 3 ? 3 : 1;
#pragma unroll 1
        for (int oz2 = 0; oz2 < ZN; ++oz2) {
            // all 9 x 6 values of the plane first, so the reads overlap
            R fv[9][6];
            const R* fp = F + fbase + oz2 * G::PY * G::PX;
#pragma unroll
            for (int c9 = 0; c9 < 9; ++c9)
#pragma unroll
                for (int q = 0; q < 6; ++q) fv[c9][q] = fp[(c9 / 3) * G::PX + c9 % 3 + q * G::NFF];
#pragma unroll
            for (int oy2 = 0; oy2 < 3; ++oy2) {
#pragma unroll
                for (int ox2 = 0; ox2 < 3; ++ox2) {
                    R wxy = wx[ox2] * wy[oy2];
                    R W = NDIM == 3 ? wxy * wz[oz2] : wxy;
                    const R* f = fv[oy2 * 3 + ox2];
                    E[0] = Pol::fma(W, f[0], E[0]);
                    E[1] = Pol::fma(W, f[1], E[1]);
                    E[2] = Pol::fma(W, f[2], E[2]);
                    Bp[0] = Pol::fma(W, f[3], Bp[0]);
                    Bp[1] = Pol::fma(W, f[4], Bp[1]);
                    Bp[2] = Pol::fma(W, f[5], Bp[2]);
                }
            }
        }
        Pol::clean(E, Bp);

        // kick - rotate - kick
        R vn[3];
        Pol::push(v, E, Bp, qm * hdt, C, C2, vn);
        if (!isfinite(vn[0]) || !isfinite(vn[1]) || !isfinite(vn[2])) errbits |= ERRBIT_NONFINITE;
        typename Pol::K k1 = Pol::kin(vn, C, C2, iC);

        // corrector feedback at x^(n+1/2): -dM, -dE_k (App. A.3)
        double Vc[4];
        Vc[0] = (-(m * ((double)vn[0] - (double)v[0]))) * S;
        Vc[1] = (-(m * ((double)vn[1] - (double)v[1]))) * S;
        Vc[2] = (-(m * ((double)vn[2] - (double)v[2]))) * S;
        Vc[3] = (-(m * (k1.ek - k0.ek))) * S;
        bool okc = fabs(Vc[0]) < kMaxAmount && fabs(Vc[1]) < kMaxAmount &&
                   fabs(Vc[2]) < kMaxAmount && fabs(Vc[3]) < kMaxAmount;
        if (okc) lds_deposit4<Pol, NDIM, G::PX, G::PY, G::NFF>(Dc, fbase, wx, wy, wz, Vc);
        else errbits |= ERRBIT_RANGE;

        // drift to x^(n+1)
        int t0 = Pol::drift(dl[0], k1.u[0], hx);
        int t1 = Pol::drift(dl[1], k1.u[1], hy);
        int t2 = NDIM == 3 ? Pol::drift(dl[2], k1.u[2], hz) : 0;
        i[0] = wrap_shift(i[0], t0, bx.n[0]);
        i[1] = wrap_shift(i[1], t1, bx.n[1]);
        if (NDIM == 3) i[2] = wrap_shift(i[2], t2, bx.n[2]);
        const int pbase = corner + (NDIM == 3 ? (t2 * G::PY + t1) * G::PX + t0 : t1 * G::PX + t0);

        // n_CR, J_CR at x^(n+1): the predictor input of the next step (at
        // the last sub-step of a sub-cycled step only)
        if (do_pred) {
            Pol::weights(dl[0], wx);
            Pol::weights(dl[1], wy);
            if (NDIM == 3) Pol::weights(dl[2], wz);
            const double qmm = qm * m;
            double Vp[4];
            Vp[0] = qmm * S;
            Vp[1] = (qmm * (double)k1.u[0]) * S;
            Vp[2] = (qmm * (double)k1.u[1]) * S;
            Vp[3] = (qmm * (double)k1.u[2]) * S;
            bool okp = fabs(Vp[0]) < kMaxAmount && fabs(Vp[1]) < kMaxAmount &&
                       fabs(Vp[2]) < kMaxAmount && fabs(Vp[3]) < kMaxAmount;
            if (okp) lds_deposit4<Pol, NDIM, G::PX, G::PY, G::NP>(Dp, pbase, wx, wy, wz, Vp);
            else errbits |= ERRBIT_RANGE;
        }

        // store x^(n+1), v^(n+1)
        a.P.cell[j] = pack_cell<NDIM>(i[0], i[1], i[2]);
        a.P.d[0][j] = dl[0];
        a.P.d[1][j] = dl[1];
        if (NDIM == 3) a.P.d[2][j] = dl[2];
        a.P.v[0][j] = vn[0];
        a.P.v[1][j] = vn[1];
        a.P.v[2][j] = vn[2];

        // tile and bank residue of the next half-step cell (the operations of
        // the next step's first drift)
        int ni[3] = {i[0], i[1], i[2]};
        R e0 = dl[0], e1 = dl[1], e2 = dl[2];
        ni[0] = wrap_shift(ni[0], Pol::drift(e0, k1.u[0], hx), bx.n[0]);
        ni[1] = wrap_shift(ni[1], Pol::drift(e1, k1.u[1], hy), bx.n[1]);
        if (NDIM == 3) ni[2] = wrap_shift(ni[2], Pol::drift(e2, k1.u[2], hz), bx.n[2]);
        int res;
        const int k = move_code<NDIM>(bx, T, tx, ty, tz, ni, errbits, res);
        // predicted shift of the next predictor deposit (velocity as now)
        const int p0 = Pol::drift(e0, k1.u[0], hx), p1 = Pol::drift(e1, k1.u[1], hy);
        const int p2 = NDIM == 3 ? Pol::drift(e2, k1.u[2], hz) : 0;
        a.code[j] = pack_code(k, res, shift_class<NDIM>(p0, p1, p2));
        // most particles stay in the tile: one LDS atomic per wave for them
        const uint64_t stays = __ballot(k == Codes<NDIM>::STAY);
        if (k != Codes<NDIM>::STAY) atomicAdd(&s_cnt[k], 1u);
        else if (lane_id() == __ffsll((unsigned long long)stays) - 1)
            atomicAdd(&s_cnt[k], (uint32_t)__popcll(stays));
    }
    if (errbits) latch(a.err, errbits);
    __syncthreads();
    for (int c = threadIdx.x; c < K; c += BLOCK) a.cnt[(size_t)item * K + c] = s_cnt[c];

    // flush the LDS boxes into the global arrays
    const int64_t NC = a.NC;
    for (int c = threadIdx.x; c < G::NFF; c += BLOCK) {
        int lx, ly, lz;
        G::coords(c + G::FOFF, lx, ly, lz);
        bool in = lx >= -1 && lx <= sx && ly >= -1 && ly <= sy && (NDIM == 2 || (lz >= -1 && lz <= sz));
        if (!in) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dc[q * G::NFF + c];
            if (val) atomicAdd((unsigned long long*)&a.Dcorr[q * NC + g], val);
        }
    }
    for (int c = threadIdx.x; c < (do_pred ? G::NP : 0); c += BLOCK) {
        int lx, ly, lz;
        G::coords(c, lx, ly, lz);
        bool in = lx < sx + 2 && ly < sy + 2 && (NDIM == 2 || lz < sz + 2);
        if (!in) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dp[q * G::NP + c];
            if (val) atomicAdd((unsigned long long*)&a.nJ[q * NC + g], val);
        }
    }
}

// n_CR = (q/mc) m and J_CR = (q/mc) m u at the current positions (App. A.1),
// once at initialisation, on the tile-sorted particles of the first work
// list: the same LDS box and deposit as the push's predictor, then a flush
// with 64-bit global atomics.  The integers equal those of a particle-by-
// particle deposit.
template <class Pol, int NDIM, int TX, int TY, int TZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_deposit_nJ_tiled(typename Pol::Part P, int64_t* __restrict__ nJ, int64_t NC,
                   const BoxDev* __restrict__ boxes, const WorkItem* __restrict__ items,
                   const uint32_t* __restrict__ n_items, uint32_t* err) {
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    using R = typename Pol::R;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* Dp = reinterpret_cast<unsigned long long*>(smem);
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    const BoxDev& bx = boxes[w.box];
    int tx, ty, tz;
    tile_coords<NDIM>(bx, w.tile, tx, ty, tz);
    const int ox = tile_origin(bx, 0, tx, TX), oy = tile_origin(bx, 1, ty, TY);
    const int oz = NDIM == 3 ? tile_origin(bx, 2, tz, TZ) : 0;
    const int sx = tile_extent(bx, 0, tx, TX), sy = tile_extent(bx, 1, ty, TY);
    const int sz = NDIM == 3 ? tile_extent(bx, 2, tz, TZ) : 1;
    for (int c = threadIdx.x; c < G::NP * 4; c += BLOCK) Dp[c] = 0ull;
    __syncthreads();
    uint32_t errbits = 0;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += BLOCK) {
        int i[3];
        unpack_cell<NDIM>(P.cell[j], i[0], i[1], i[2]);
        int lx = i[0] - ox, ly = i[1] - oy, lz = NDIM == 3 ? i[2] - oz : 0;
        if (!(lx >= 0 && lx < sx && ly >= 0 && ly < sy && lz >= 0 && lz < sz)) {
            errbits |= ERRBIT_STATE;
            lx = min(max(lx, 0), sx - 1);
            ly = min(max(ly, 0), sy - 1);
            lz = NDIM == 3 ? min(max(lz, 0), sz - 1) : 0;
        }
        const int corner = G::index(lx, ly, lz) - G::CORNER;
        R wx[3], wy[3], wz[3] = {R(0), R(1), R(0)};
        Pol::weights(P.d[0][j], wx);
        Pol::weights(P.d[1][j], wy);
        if (NDIM == 3) Pol::weights(P.d[2][j], wz);
        R v[3] = {P.v[0][j], P.v[1][j], P.v[2][j]};
        typename Pol::K k = Pol::kin(v, bx.C, bx.C2, bx.iC);
        const double qmm = (double)P.qm[j] * (double)P.m[j];
        double V[4];
        V[0] = qmm * bx.S;
        V[1] = (qmm * (double)k.u[0]) * bx.S;
        V[2] = (qmm * (double)k.u[1]) * bx.S;
        V[3] = (qmm * (double)k.u[2]) * bx.S;
        const bool ok = fabs(V[0]) < kMaxAmount && fabs(V[1]) < kMaxAmount &&
                        fabs(V[2]) < kMaxAmount && fabs(V[3]) < kMaxAmount;
        if (ok) lds_deposit4<Pol, NDIM, G::PX, G::PY, G::NP>(Dp, corner, wx, wy, wz, V);
        else errbits |= ERRBIT_RANGE;
    }
    if (errbits) latch(err, errbits);
    __syncthreads();
    for (int c = threadIdx.x; c < G::NP; c += BLOCK) {
        int lx, ly, lz;
        G::coords(c, lx, ly, lz);
        bool in = lx < sx + 2 && ly < sy + 2 && (NDIM == 2 || lz < sz + 2);
        if (!in) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dp[q * G::NP + c];
            if (val) atomicAdd((unsigned long long*)&nJ[q * NC + g], val);
        }
    }
}

}  // namespace mhdpic
