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
    typename Pol::Part P;        // out: tile-sorted particles (the ids already there)
    int64_t src_delta;           // bytes from each array of P to the same array of the
                                 // buffer the particles are read from (0: in place)
    const uint32_t* map;         // slot j of P -> slot of its particle in that buffer;
                                 // NULL: slot j itself
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
    int32_t grp;                 // launch group of this launch's boxes, -1: all boxes
};

template <class Pol, int NDIM, int TX, int TY, int TZ>
struct Geo {
    using R = typename Pol::R;
    // boxes of (T + 4) cells per axis, rows and planes padded (lds_strides)
    static constexpr LdsStrides ST = lds_strides(TX, TY, TZ, NDIM);
    static constexpr int SX = ST.sx, SP = NDIM == 3 ? ST.sp : 0;  // row, plane strides
    static constexpr int NP = NDIM == 3 ? SP * (TZ + 4) : SX * (TY + 4);
    static constexpr int FOFF = NDIM == 3 ? SP : SX;  // skipped leading plane/row
    static constexpr int NFF = NP - 2 * FOFF;
    static constexpr int CORNER = NDIM == 3 ? SP + SX + 1 : SX + 1;
    // field words per cell: binary64 E, B interleaved (48 B, three 16-byte
    // units); binary32 E and B in two planes of 16-byte cells (xyz + a pad)
    static constexpr int FW = sizeof(R) == 8 ? 6 : 8;
    static constexpr size_t lds_bytes() {
        return (size_t)NFF * 4 * 8 + (size_t)NP * 4 * 8 + (size_t)NFF * FW * sizeof(R) + (size_t)NP * 4;
    }
    // index of tile-local cell (lx, ly, lz), each in [-2, extent + 2)
    __device__ static __forceinline__ int index(int lx, int ly, int lz) {
        return (NDIM == 3 ? (lz + 2) * SP : 0) + (ly + 2) * SX + (lx + 2);
    }
    // padding cells come out beyond the box (lx >= TX + 2 or ly >= TY + 2)
    __device__ static __forceinline__ void coords(int p, int& lx, int& ly, int& lz) {
        int r = p;
        lz = 0;
        if constexpr (NDIM == 3) {
            r = p % SP;
            lz = p / SP - 2;
        }
        lx = r % SX - 2;
        ly = r / SX - 2;
    }
};

// Adds 4 channel amounts V[0..3] of one particle to an LDS box [4][NB] whose
// (-1,-1,-1) stencil corner is at index `base`; weights in the working
// precision, quantised against the binary64 amounts.
//
// A stencil cell k other than the centre is sent the bit pattern of
// fma(W_k, V, 1.5*2^52), which is 1.5*2^52 with round-half-even(W_k V) added
// to its low bits, as an integer: the pattern P of 1.5*2^52 plus the rounded
// product.  The centre is sent round(V) minus the sum of those patterns, that
// is its own amount minus (K-1) P, for K stencil cells.  A cell of the box
// thus holds its amount plus P times (the particles whose stencil covers it
// minus K times those centred on it); the flush removes that from counts of
// particles per centre cell (kept in `ncnt`, see flush_fix).  This saves the
// subtraction of P from every contribution.
template <class Pol, int NDIM, int SX, int SP, int NB>
__device__ __forceinline__ void lds_deposit4(unsigned long long* box, int base,
                                             const typename Pol::R wx[3],
                                             const typename Pol::R wy[3],
                                             const typename Pol::R wz[3], const double V[4]) {
    using R = typename Pol::R;
    uint64_t acc[4] = {0, 0, 0, 0};
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
                unsigned long long* p = p0 + oz * SP + oy * SX + ox;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint64_t r = (uint64_t)__double_as_longlong(__builtin_fma(W, V[c], kMagic));
                    acc[c] += r;
                    atomicAdd(p + c * NB, (unsigned long long)r);
                }
            }
        }
    }
    constexpr int CZ = NDIM == 3 ? 1 : 0;
    unsigned long long* pc = p0 + CZ * SP + SX + 1;
#pragma unroll
    for (int c = 0; c < 4; ++c) atomicAdd(pc + c * NB, (unsigned long long)((uint64_t)quant1(V[c]) - acc[c]));
}

// Pattern excess of an LDS cell at tile-local (lx, ly, lz): P times (the
// particles whose stencil covers it minus K times those centred on it), from
// the centre counts of the box (ncnt: corrector counts in the low 16 bits,
// predictor counts in the high 16 bits; shift selects one).  Counts are only
// ever nonzero on cells [-1, s] per axis (centres lie in the tile or, for the
// predictor, one cell beyond it), so only those neighbours are read.  Products
// are modulo 2^64 like the sums they correct; only a count modulo 2^16
// matters, because P is a multiple of 2^48.
template <int NDIM, int SX, int SP>
__device__ __forceinline__ uint64_t flush_fix(const uint32_t* ncnt, int lx, int ly, int lz, int sx,
                                              int sy, int sz, int shift) {
    constexpr int K = NDIM == 3 ? 27 : 9;
    uint32_t cover = 0, own = 0;
    const int zlo = NDIM == 3 ? -1 : 0, zhi = NDIM == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
        const int z = lz + dz;
        if (NDIM == 3 && (z < -1 || z > sz)) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = ly + dy;
            if (y < -1 || y > sy) continue;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = lx + dx;
                if (x < -1 || x > sx) continue;
                const int idx = (NDIM == 3 ? (z + 2) * SP : 0) + (y + 2) * SX + (x + 2);
                const uint32_t n = (ncnt[idx] >> shift) & 0xFFFFu;
                cover += n;
                if (dx == 0 && dy == 0 && dz == 0) own = n;
            }
        }
    }
    return (uint64_t)(cover - (uint32_t)K * own) * ((uint64_t)kMagicHi << 32);
}

// E, B of LDS field cell c (field-region index).  A 128-bit LDS read of a
// wave is served 16 lanes at a time, as a 64-bit atomic is, while a 64-bit
// read is served 32 lanes at a time; with 16-byte cell units the gather's
// reads see the same bank pattern as the deposit atomics, for which the
// binning spreads 16 consecutive lanes over distinct cells modulo 16.
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int NFF>
__device__ __forceinline__ void field_cell(const double* F, int c, double f[6]) {
    const f64x2* p = reinterpret_cast<const f64x2*>(F + 6 * c);
    const f64x2 a = p[0], b = p[1], d = p[2];
    f[0] = a.x;
    f[1] = a.y;
    f[2] = b.x;
    f[3] = b.y;
    f[4] = d.x;
    f[5] = d.y;
}
template <int NFF>
__device__ __forceinline__ void field_cell(const float* F, int c, float f[6]) {
    const f32x4 e = reinterpret_cast<const f32x4*>(F)[c];
    const f32x4 b = reinterpret_cast<const f32x4*>(F + 4 * NFF)[c];
    f[0] = e.x;
    f[1] = e.y;
    f[2] = e.z;
    f[3] = b.x;
    f[4] = b.y;
    f[5] = b.z;
}
__device__ __forceinline__ void field_store(double* F, int NFF, int c, const double* s) {
    for (int q = 0; q < 6; ++q) F[6 * c + q] = s[q];
}
__device__ __forceinline__ void field_store(float* F, int NFF, int c, const float* s) {
    for (int q = 0; q < 3; ++q) {
        F[4 * c + q] = s[q];
        F[4 * NFF + 4 * c + q] = s[3 + q];
    }
}

// Array p of another particle buffer of the same layout, delta bytes away
// (the two buffers of a context share one layout, so one offset serves every
// array and the kernel holds one set of array addresses).
template <typename T>
__device__ __forceinline__ const T* other_buffer(const T* p, int64_t delta) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + delta);
}

// One particle's stored state (in 2D the third offset reads as 0), read from
// slot j of the buffer delta bytes away from P.
template <int NDIM, typename R>
struct PartRec {
    uint32_t cell = 0;
    R d[3] = {R(0), R(0), R(0)}, v[3] = {R(0), R(0), R(0)};
    R m = R(0), qm = R(0);
    template <typename PS>
    __device__ __forceinline__ void load(const PS& P, int64_t delta, int j) {
        cell = other_buffer(P.cell, delta)[j];
        d[0] = other_buffer(P.d[0], delta)[j];
        d[1] = other_buffer(P.d[1], delta)[j];
        d[2] = NDIM == 3 ? other_buffer(P.d[2], delta)[j] : R(0);
        v[0] = other_buffer(P.v[0], delta)[j];
        v[1] = other_buffer(P.v[1], delta)[j];
        v[2] = other_buffer(P.v[2], delta)[j];
        m = other_buffer(P.m, delta)[j];
        qm = other_buffer(P.qm, delta)[j];
    }
};

// Launch shape of the push per precision and dimension: threads per block,
// the waves per SIMD the register budget must allow (4: at most 128 VGPRs),
// whether the next particle's state is loaded during the current push, and
// whether the gather reads a stencil row (3 cells) or a plane (9 cells) of
// fields into registers before its multiply-adds.
template <class Pol, int NDIM>
struct PushShape {
    static constexpr int BLOCK = 512;
    static constexpr int WAVES = 4;
    static constexpr bool PREFETCH = NDIM == 3 && std::is_same<typename Pol::R, float>::value;
    static constexpr bool ROWS = NDIM == 3 && std::is_same<typename Pol::R, double>::value;
};

template <class Pol, int NDIM, int TX, int TY, int TZ, int BLOCK>
__global__ void __launch_bounds__(BLOCK, (PushShape<Pol, NDIM>::WAVES)) k_push(PushArgsT<Pol> a) {
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    using R = typename Pol::R;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* Dc = reinterpret_cast<unsigned long long*>(smem);
    unsigned long long* Dp = Dc + (size_t)G::NFF * 4;
    R* F = reinterpret_cast<R*>(Dp + (size_t)G::NP * 4);
    uint32_t* ncnt = reinterpret_cast<uint32_t*>(F + (size_t)G::NFF * G::FW);  // [NP] centre counts
    constexpr int K = Codes<NDIM>::K;
    __shared__ uint32_t s_cnt[K];

    uint32_t item;
    if (!item_of_block(a.n_items, item)) return;
    for (int c = threadIdx.x; c < K; c += BLOCK) s_cnt[c] = 0;
    const WorkItem w = a.items[item];
    const BoxDev bx = a.boxes[w.box];  // a copy: kept in registers across the stores
    if (a.grp >= 0 && bx.grp != a.grp) return;  // a box of another tile shape
    // the slot that holds the particle of slot jd (the binning's map, if it
    // left one); each one is read an iteration ahead of its particle, the
    // first before the fields are staged
    auto src_of = [&](int jd) { return a.map ? (int)a.map[jd] : jd; };
    const int j0 = w.begin + (int)threadIdx.x;
    int src = j0 < w.end ? src_of(j0) : 0;
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
            field_store(F, G::NFF, c, a.EB + 6 * g);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Dc[q * G::NFF + c] = 0ull;
    }
    const bool do_pred = a.do_pred != 0;
    if (do_pred)
        for (int c = threadIdx.x; c < G::NP * 4; c += BLOCK) Dp[c] = 0ull;
    for (int c = threadIdx.x; c < G::NP; c += BLOCK) ncnt[c] = 0u;
    __syncthreads();

    const double C = bx.C, C2 = bx.C2, iC = bx.iC, S = bx.S, hdt = bx.hdt;
    const R hx = Pol::hdx(bx.hdx[0]), hy = Pol::hdx(bx.hdx[1]), hz = Pol::hdx(bx.hdx[2]);
    const int3 T = make_int3(TX, TY, TZ);
    uint32_t errbits = 0;

    // the binary32 3D kernel loads the next particle while it pushes this one
    // and still fits the 128 registers of four waves per SIMD; the others
    // have no registers to spare for it
    constexpr bool kPrefetch = PushShape<Pol, NDIM>::PREFETCH;
    PartRec<NDIM, R> nxt;
    if (kPrefetch && j0 < w.end) {
        nxt.load(a.P, a.src_delta, src);
        if (j0 + BLOCK < w.end) src = src_of(j0 + BLOCK);
    }
    for (int j = j0; j < w.end; j += BLOCK) {
        // the offset is re-read each iteration, so the read addresses are
        // formed where they are used instead of being held in (spilled)
        // scalar registers for the whole loop
        int64_t delta = a.src_delta;
        asm volatile("" : "+s"(delta));
        PartRec<NDIM, R> cur;
        if (kPrefetch) {
            cur = nxt;
            if (j + BLOCK < w.end) {
                nxt.load(a.P, delta, src);
                if (j + 2 * BLOCK < w.end) src = src_of(j + 2 * BLOCK);
            }
        } else {
            cur.load(a.P, delta, src);
            if (j + BLOCK < w.end) src = src_of(j + BLOCK);
        }
        int i[3];
        unpack_cell<NDIM>(cur.cell, i[0], i[1], i[2]);
        R dl[3] = {cur.d[0], cur.d[1], cur.d[2]};
        R v[3] = {cur.v[0], cur.v[1], cur.v[2]};
        const double m = (double)cur.m, qm = (double)cur.qm;

        typename Pol::K k0 = Pol::kin(v, C, C2, iC);
        // drift to x^(n+1/2) (a reflecting face mirrors the particle and its
        // velocity; the binning has already dropped the particles this drift
        // takes through an absorbing face)
        const int s0 = half_drift<Pol>(bx, 0, i[0], dl[0], v[0], k0.u[0], hx);
        const int s1 = half_drift<Pol>(bx, 1, i[1], dl[1], v[1], k0.u[1], hy);
        const int s2 = NDIM == 3 ? half_drift<Pol>(bx, 2, i[2], dl[2], v[2], k0.u[2], hz) : 0;
        int lx = i[0] - ox, ly = i[1] - oy, lz = NDIM == 3 ? i[2] - oz : 0;
        bool inside = lx >= 0 && lx < sx && ly >= 0 && ly < sy && lz >= 0 && lz < sz &&
                      s0 != kGone && s1 != kGone && s2 != kGone;
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
        if (PushShape<Pol, NDIM>::ROWS) {
            // stencil rows (z outer, then y) of 18 values each, unrolled, so
            // that a row's reads overlap the previous row's multiply-adds as
            // far as the register budget allows (1.9 % off the push against a
            // rolled loop)
#pragma unroll
            for (int r = 0; r < 3 * ZN; ++r) {
                const int oz2 = r / 3, oy2 = r - 3 * (r / 3);
                const int fc = fbase + oz2 * G::SP + oy2 * G::SX;
                R fv[3][6];
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) field_cell<G::NFF>(F, fc + c3, fv[c3]);
                const R wyo = oy2 == 0 ? wy[0] : (oy2 == 1 ? wy[1] : wy[2]);
                const R wzo = oz2 == 0 ? wz[0] : (oz2 == 1 ? wz[1] : wz[2]);
#pragma unroll
                for (int ox2 = 0; ox2 < 3; ++ox2) {
                    R wxy = wx[ox2] * wyo;
                    R W = NDIM == 3 ? wxy * wzo : wxy;
                    const R* f = fv[ox2];
                    E[0] = Pol::fma(W, f[0], E[0]);
                    E[1] = Pol::fma(W, f[1], E[1]);
                    E[2] = Pol::fma(W, f[2], E[2]);
                    Bp[0] = Pol::fma(W, f[3], Bp[0]);
                    Bp[1] = Pol::fma(W, f[4], Bp[1]);
                    Bp[2] = Pol::fma(W, f[5], Bp[2]);
                }
            }
        } else
#pragma unroll
        for (int oz2 = 0; oz2 < ZN; ++oz2) {
            // all 9 x 6 values of the plane first, so the reads overlap (and,
            // unrolled, the next plane's reads the current plane's sums)
            R fv[9][6];
            const int fc = fbase + oz2 * G::SP;
#pragma unroll
            for (int c9 = 0; c9 < 9; ++c9) field_cell<G::NFF>(F, fc + (c9 / 3) * G::SX + c9 % 3, fv[c9]);
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
        typename Pol::Inc inc;
        Pol::push(v, E, Bp, qm * hdt, C, C2, vn, inc);
        if (!isfinite(vn[0]) || !isfinite(vn[1]) || !isfinite(vn[2])) errbits |= ERRBIT_NONFINITE;
        typename Pol::K k1 = Pol::kin(vn, C, C2, iC);

        // corrector feedback at x^(n+1/2): -dM, -dE_k (App. A.3)
        double dv[3], dek;
        Pol::corrector(v, vn, k0, k1, inc, dv, dek);
        double Vc[4];
        Vc[0] = (-(m * dv[0])) * S;
        Vc[1] = (-(m * dv[1])) * S;
        Vc[2] = (-(m * dv[2])) * S;
        Vc[3] = (-(m * dek)) * S;
        bool okc = fabs(Vc[0]) < kMaxAmount && fabs(Vc[1]) < kMaxAmount &&
                   fabs(Vc[2]) < kMaxAmount && fabs(Vc[3]) < kMaxAmount;
        if (okc) {
            lds_deposit4<Pol, NDIM, G::SX, G::SP, G::NFF>(Dc, fbase, wx, wy, wz, Vc);
            atomicAdd(&ncnt[corner + G::CORNER], 1u);
        } else {
            errbits |= ERRBIT_RANGE;
        }

        // drift to x^(n+1); through an absorbing face the particle leaves
        // after its corrector deposit and before its predictor one
        int t0 = half_drift<Pol>(bx, 0, i[0], dl[0], vn[0], k1.u[0], hx);
        int t1 = t0 == kGone ? 0 : half_drift<Pol>(bx, 1, i[1], dl[1], vn[1], k1.u[1], hy);
        int t2 = NDIM == 3 && t0 != kGone && t1 != kGone
                     ? half_drift<Pol>(bx, 2, i[2], dl[2], vn[2], k1.u[2], hz) : 0;
        const bool gone = t0 == kGone || t1 == kGone || t2 == kGone;
        if (gone) t0 = t1 = t2 = 0;
        const int pbase = corner + (NDIM == 3 ? t2 * G::SP : 0) + t1 * G::SX + t0;

        // n_CR, J_CR at x^(n+1): the predictor input of the next step (at
        // the last sub-step of a sub-cycled step only)
        if (do_pred && !gone) {
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
            if (okp) {
                lds_deposit4<Pol, NDIM, G::SX, G::SP, G::NP>(Dp, pbase, wx, wy, wz, Vp);
                atomicAdd(&ncnt[pbase + G::CORNER], 1u << 16);
            } else {
                errbits |= ERRBIT_RANGE;
            }
        }

        // store x^(n+1), v^(n+1) and the particle's constants at its slot (a
        // particle that left keeps only its mark)
        a.P.cell[j] = gone ? kDeadCell : pack_cell<NDIM>(i[0], i[1], i[2]);
        a.P.d[0][j] = dl[0];
        a.P.d[1][j] = dl[1];
        if (NDIM == 3) a.P.d[2][j] = dl[2];
        a.P.v[0][j] = vn[0];
        a.P.v[1][j] = vn[1];
        a.P.v[2][j] = vn[2];
        if (a.map) {
            a.P.m[j] = cur.m;
            a.P.qm[j] = cur.qm;
        }

        // tile and bank residue of the next half-step cell (the operations of
        // the next step's first drift), or the gone code if that drift takes
        // the particle through an absorbing face
        const int k = next_code<Pol, NDIM>(bx, T, tx, ty, tz, i, dl, vn, k1.u, hx, hy, hz, gone,
                                            errbits, a.code[j]);
        // most particles stay in the tile: one LDS atomic per wave for them
        const uint64_t stays = __ballot(k == Codes<NDIM>::STAY);
        if (k != Codes<NDIM>::STAY && k != Codes<NDIM>::GONE) atomicAdd(&s_cnt[k], 1u);
        else if (k == Codes<NDIM>::STAY && lane_id() == __ffsll((unsigned long long)stays) - 1)
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
        const uint64_t fix = flush_fix<NDIM, G::SX, G::SP>(ncnt, lx, ly, lz, sx, sy, sz, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dc[q * G::NFF + c] - fix;
            if (val) atomicAdd((unsigned long long*)&a.Dcorr[q * NC + g], val);
        }
    }
    for (int c = threadIdx.x; c < (do_pred ? G::NP : 0); c += BLOCK) {
        int lx, ly, lz;
        G::coords(c, lx, ly, lz);
        bool in = lx < sx + 2 && ly < sy + 2 && (NDIM == 2 || lz < sz + 2);
        if (!in) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
        const uint64_t fix = flush_fix<NDIM, G::SX, G::SP>(ncnt, lx, ly, lz, sx, sy, sz, 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dp[q * G::NP + c] - fix;
            if (val) atomicAdd((unsigned long long*)&a.nJ[q * NC + g], val);
        }
    }
}

// Tile-local index l (cell minus tile origin) of a tile of extent s in a box
// of n cells, within one cell of the tile ([-1, s]), taking a periodic wrap
// into account; kFar if it is farther.
constexpr int kFar = -1000000;
__device__ __forceinline__ int near_tile(int l, int s, int n, bool periodic) {
    if (periodic) {
        if (l < -1) l += n;
        else if (l > s) l -= n;
    }
    return (l >= -1 && l <= s) ? l : kFar;
}

// n_CR = (q/mc) m and J_CR = (q/mc) m u at the current positions (App. A.1),
// added to nJ for the particles of a work list (all particles at
// initialisation, the new ones after an injection): the same LDS box and
// deposit as the push's predictor, then a flush with 64-bit global atomics.
// The integers equal those of a particle-by-particle deposit.  With REMOVE,
// only the particles whose tag is below t_cut with t_now at least twice the
// tag (Sec. 5) are taken: their amounts are deposited negated, which takes
// back exactly the integers they added (round-half-even is odd), and they are
// marked as gone.
template <class Pol, int NDIM, int TX, int TY, int TZ, int BLOCK, bool REMOVE>
__global__ void __launch_bounds__(BLOCK)
k_deposit_nJ_tiled(typename Pol::Part P, int64_t* __restrict__ nJ, int64_t NC,
                   const BoxDev* __restrict__ boxes, const WorkItem* __restrict__ items,
                   const uint32_t* __restrict__ n_items, uint32_t* err, double t_cut, double t_now,
                   int grp) {
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    using R = typename Pol::R;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* Dp = reinterpret_cast<unsigned long long*>(smem);
    uint32_t* ncnt = reinterpret_cast<uint32_t*>(Dp + (size_t)G::NP * 4);  // [NP] centre counts
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    const BoxDev& bx = boxes[w.box];
    if (grp >= 0 && bx.grp != grp) return;  // a box of another tile shape
    int tx, ty, tz;
    tile_coords<NDIM>(bx, w.tile, tx, ty, tz);
    const int ox = tile_origin(bx, 0, tx, TX), oy = tile_origin(bx, 1, ty, TY);
    const int oz = NDIM == 3 ? tile_origin(bx, 2, tz, TZ) : 0;
    const int sx = tile_extent(bx, 0, tx, TX), sy = tile_extent(bx, 1, ty, TY);
    const int sz = NDIM == 3 ? tile_extent(bx, 2, tz, TZ) : 1;
    for (int c = threadIdx.x; c < G::NP * 4; c += BLOCK) Dp[c] = 0ull;
    for (int c = threadIdx.x; c < G::NP; c += BLOCK) ncnt[c] = 0u;
    __syncthreads();
    uint32_t errbits = 0;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += BLOCK) {
        const uint32_t cell = P.cell[j];
        if (cell == kDeadCell) continue;
        if (REMOVE) {
            const double t = P.tag[j];
            if (!(t < t_cut && 2.0 * t <= t_now)) continue;
        }
        int i[3];
        unpack_cell<NDIM>(cell, i[0], i[1], i[2]);
        // the particle's cell relative to the tile: inside it after a sort by
        // the current cell, or (after a step: the work list groups by the
        // last half-step cell) up to one cell beyond it, across a periodic
        // wrap of the box, as the push's own x^(n+1) deposit allows
        const int lx = near_tile(i[0] - ox, sx, bx.n[0], bx.face[0][0] == FACE_PERIODIC);
        const int ly = near_tile(i[1] - oy, sy, bx.n[1], bx.face[1][0] == FACE_PERIODIC);
        const int lz = NDIM == 3 ? near_tile(i[2] - oz, sz, bx.n[2], bx.face[2][0] == FACE_PERIODIC) : 0;
        if (lx == kFar || ly == kFar || lz == kFar) {
            errbits |= ERRBIT_STATE;
            continue;
        }
        if (REMOVE) P.cell[j] = kDeadCell;
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
        if (REMOVE)
            for (int c = 0; c < 4; ++c) V[c] = -V[c];
        const bool ok = fabs(V[0]) < kMaxAmount && fabs(V[1]) < kMaxAmount &&
                        fabs(V[2]) < kMaxAmount && fabs(V[3]) < kMaxAmount;
        if (ok) {
            lds_deposit4<Pol, NDIM, G::SX, G::SP, G::NP>(Dp, corner, wx, wy, wz, V);
            atomicAdd(&ncnt[corner + G::CORNER], 1u);
        } else {
            errbits |= ERRBIT_RANGE;
        }
    }
    if (errbits) latch(err, errbits);
    __syncthreads();
    for (int c = threadIdx.x; c < G::NP; c += BLOCK) {
        int lx, ly, lz;
        G::coords(c, lx, ly, lz);
        bool in = lx < sx + 2 && ly < sy + 2 && (NDIM == 2 || lz < sz + 2);
        if (!in) continue;
        int64_t g = global_cell<NDIM>(bx, ox + lx, oy + ly, oz + lz);
        const uint64_t fix = flush_fix<NDIM, G::SX, G::SP>(ncnt, lx, ly, lz, sx, sy, sz, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned long long val = Dp[q * G::NP + c] - fix;
            if (val) atomicAdd((unsigned long long*)&nJ[q * NC + g], val);
        }
    }
}

}  // namespace mhdpic
