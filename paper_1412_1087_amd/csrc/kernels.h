// HIP kernels of the MHD-PIC cosmic-ray particle step (binary64 form and
// shared bookkeeping).  gfx950: wave64, 160 KB LDS per CU, 8 XCDs.
#pragma once
#include "arith.h"
#include "common.h"

namespace mhdpic {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ void latch(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

// Box that owns global index g, given ascending offsets off[0..nb] (off[nb] = total).
__device__ __forceinline__ int find_box(const int64_t* off, int nb, int64_t g) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Every lane of the wave must call this (no divergence at the call site).
// Returns, for active lanes, a distinct slot obtained from counters[key]; one
// atomic per distinct key in the wave.
__device__ __forceinline__ uint32_t wave_claim(uint32_t* counters, uint32_t key, bool active) {
    uint64_t pending = __ballot(active);
    uint32_t slot = 0;
    const int lane = lane_id();
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        uint32_t k = __shfl(key, leader);
        uint64_t grp = __ballot(active && key == k) & pending;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&counters[k], (uint32_t)__popcll(grp));
        base = __shfl(base, leader);
        if ((grp >> lane) & 1ull) slot = base + (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
        pending &= ~grp;
    }
    return slot;
}

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// fills and copies
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = val;
}

__global__ void k_fill_i64(int64_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

__global__ void k_copy_i64(int64_t* __restrict__ dst, const int64_t* __restrict__ src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// initialisation: global positions -> (cell, offset); n_CR, J_CR deposit
// ---------------------------------------------------------------------------

template <int NDIM, typename PS, typename T>
__global__ void k_init_convert(PS P, const double* __restrict__ x, const double* __restrict__ v,
                               const double* __restrict__ m, const double* __restrict__ qm,
                               const BoxDev* __restrict__ boxes, const int64_t* __restrict__ part_off,
                               int nb, int64_t N, uint32_t* err) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    int b = find_box(part_off, nb, j);
    const BoxDev& bx = boxes[b];
    int ic[3] = {0, 0, 0};
    bool bad = false, far = false;
    for (int d = 0; d < NDIM; ++d) {
        double s = (x[d * N + j] - bx.x0[d]) / bx.dx[d];
        double fl = floor(s);
        if (!isfinite(s)) bad = true;
        // the cell count from x0 must fit a 32-bit int
        else if (!(fl >= -2147483648.0 && fl < 2147483648.0)) far = true;
        double off = (s - fl) - 0.5;
        ic[d] = (bad || far) ? 0 : pmod((int)(long long)fl, bx.n[d]);
        T o = (T)off;
        if (o >= (T)0.5) {  // binary32 rounding can reach the upper edge
            o = o - (T)1;
            ic[d] = wrap_shift(ic[d], 1, bx.n[d]);
        }
        P.d[d][j] = o;
    }
    for (int d = 0; d < 3; ++d) {
        double vd = v[d * N + j];
        if (!isfinite(vd)) bad = true;
        P.v[d][j] = (T)vd;
    }
    if (!isfinite(m[j]) || !isfinite(qm[j])) bad = true;
    if (bad) latch(err, ERRBIT_NONFINITE);
    if (far) latch(err, ERRBIT_RANGE);
    P.cell[j] = pack_cell<NDIM>(ic[0], ic[1], ic[2]);
    P.m[j] = m[j];
    P.qm[j] = qm[j];
    P.pid[j] = (int32_t)j;
}

// ---------------------------------------------------------------------------
// binning by tile of the half-step cell x^(n+1/2)
// ---------------------------------------------------------------------------

// Global index of cell (x, y, z) of a periodic box; coordinates may lie
// outside [0, n) and are wrapped.
template <int NDIM>
__device__ __forceinline__ int64_t global_cell(const BoxDev& bx, int x, int y, int z) {
    x = pmod(x, bx.n[0]);
    y = pmod(y, bx.n[1]);
    z = NDIM == 3 ? pmod(z, bx.n[2]) : 0;
    return bx.cell_off + ((int64_t)z * bx.n[1] + y) * bx.n[0] + x;
}

// Tiles along a dimension start at multiples of T, except that when n % T == 1
// the last tile starts at n - 2: every tile is at least two cells wide, so a
// step (at most two cells) never crosses a whole tile.
__device__ __forceinline__ int tile_index(const BoxDev& bx, int d, int i, int T) {
    return (bx.small_last[d] && i >= bx.n[d] - 2) ? bx.nt[d] - 1 : i / T;
}

__device__ __forceinline__ int tile_origin(const BoxDev& bx, int d, int t, int T) {
    return (bx.small_last[d] && t == bx.nt[d] - 1) ? bx.n[d] - 2 : t * T;
}

__device__ __forceinline__ int tile_extent(const BoxDev& bx, int d, int t, int T) {
    int end = t == bx.nt[d] - 1 ? bx.n[d] : tile_origin(bx, d, t + 1, T);
    return end - tile_origin(bx, d, t, T);
}

template <int NDIM>
__device__ __forceinline__ uint32_t tile_of(const BoxDev& bx, const int3 T, int ix, int iy,
                                            int iz) {
    int tx = tile_index(bx, 0, ix, T.x), ty = tile_index(bx, 1, iy, T.y);
    int tz = NDIM == 3 ? tile_index(bx, 2, iz, T.z) : 0;
    return (uint32_t)(bx.tile_off + (tz * bx.nt[1] + ty) * bx.nt[0] + tx);
}

// Exclusive scan of tile counts and the work list: each tile's particles are
// split into items of at most P particles.  One block of 1024 threads.
__global__ void __launch_bounds__(1024)
k_scan(const uint32_t* __restrict__ count, uint32_t* __restrict__ start,
       uint32_t* __restrict__ cursor, const int32_t* __restrict__ tile_box,
       WorkItem* __restrict__ items, uint32_t* __restrict__ item_first,
       uint32_t* __restrict__ n_items, int NT, int P) {
    __shared__ uint32_t s_a[1024], s_b[1024];
    const int t = threadIdx.x;
    const int per = (NT + 1023) / 1024;
    const int t0 = min(t * per, NT), t1 = min(t0 + per, NT);
    uint32_t sum = 0, nit = 0;
    for (int i = t0; i < t1; ++i) {
        uint32_t c = count[i];
        sum += c;
        nit += (c + P - 1) / P;
    }
    s_a[t] = sum;
    s_b[t] = nit;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t a = t >= off ? s_a[t - off] : 0u;
        uint32_t b = t >= off ? s_b[t - off] : 0u;
        __syncthreads();
        s_a[t] += a;
        s_b[t] += b;
        __syncthreads();
    }
    uint32_t off = s_a[t] - sum;
    uint32_t io = s_b[t] - nit;
    for (int i = t0; i < t1; ++i) {
        uint32_t c = count[i];
        start[i] = off;
        cursor[i] = off;
        item_first[i] = io;
        for (uint32_t k = 0; k < c; k += (uint32_t)P) {
            WorkItem w;
            w.tile = i;
            w.begin = (int32_t)(off + k);
            w.end = (int32_t)(off + min(k + (uint32_t)P, c));
            w.box = tile_box[i];
            items[io++] = w;
        }
        off += c;
    }
    if (t == 1023) {
        start[NT] = s_a[1023];
        item_first[NT] = s_b[1023];
        *n_items = s_b[1023];
    }
}

// Moves every particle to its slot in the tile-sorted order.
template <int NDIM, typename PS>
__global__ void k_scatter(PS A, PS Bo, const uint32_t* __restrict__ key,
                          uint32_t* __restrict__ cursor, int64_t N) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = j < N;
    uint32_t k = act ? key[j] : 0u;
    uint32_t s = wave_claim(cursor, k, act);
    if (!act) return;
    Bo.cell[s] = A.cell[j];
    for (int d = 0; d < NDIM; ++d) Bo.d[d][s] = A.d[d][j];
    for (int d = 0; d < 3; ++d) Bo.v[d][s] = A.v[d][j];
    Bo.m[s] = A.m[j];
    Bo.qm[s] = A.qm[j];
    Bo.pid[s] = A.pid[j];
}

// ---------------------------------------------------------------------------
// direction codes of tile-to-tile moves
// ---------------------------------------------------------------------------

template <int NDIM>
struct Codes {
    static constexpr int K = NDIM == 3 ? 27 : 9;
    static constexpr int STAY = NDIM == 3 ? 13 : 4;
};

// Per-dimension code of a move from tile coordinate a to b on a ring of n
// tiles: 1 = same, 2 = next, 0 = previous; -1 if farther.
__device__ __forceinline__ int dir_code(int a, int b, int n) {
    int d = b - a;
    d += d < 0 ? n : 0;
    return d == 0 ? 1 : (d == 1 ? 2 : (d == n - 1 ? 0 : -1));  // selects, no branches
}

template <int NDIM>
__device__ __forceinline__ void tile_coords(const BoxDev& bx, int tile, int& tx, int& ty, int& tz) {
    int lt = tile - bx.tile_off;
    tx = lt % bx.nt[0];
    ty = (lt / bx.nt[0]) % bx.nt[1];
    tz = NDIM == 3 ? lt / (bx.nt[0] * bx.nt[1]) : 0;
}

// Bank residues: 64-bit LDS words of equal residue (index mod kResidues)
// share a bank pair; the binning orders particles so that 16 consecutive
// lanes have distinct residues.
#ifndef MHDPIC_RESIDUES
#define MHDPIC_RESIDUES 16
#endif
constexpr int kResidues = MHDPIC_RESIDUES;

// Code of the move from the item's tile (tx,ty,tz) to the tile holding cell i
// (Codes::STAY and an error bit if that tile is farther than one tile away),
// and in `residue` the bank residue of cell i in the LDS geometry of the
// destination tile (strides T.x + 4, T.y + 4, ghost width 2; the item's own
// tile after an error).
template <int NDIM>
__device__ __forceinline__ int move_code(const BoxDev& bx, int3 T, int tx, int ty, int tz,
                                         const int i[3], uint32_t& errbits, int& residue) {
    int ux = tile_index(bx, 0, i[0], T.x), uy = tile_index(bx, 1, i[1], T.y);
    int uz = NDIM == 3 ? tile_index(bx, 2, i[2], T.z) : 0;
    const int cx = dir_code(tx, ux, bx.nt[0]);
    const int cy = dir_code(ty, uy, bx.nt[1]);
    const int cz = NDIM == 3 ? dir_code(tz, uz, bx.nt[2]) : 0;
    int k = NDIM == 3 ? (cz * 3 + cy) * 3 + cx : cy * 3 + cx;
    if (cx < 0 || cy < 0 || cz < 0) {
        errbits |= ERRBIT_STATE;
        k = Codes<NDIM>::STAY;
        ux = tx;
        uy = ty;
        uz = tz;
    }
    const int lx = i[0] - tile_origin(bx, 0, ux, T.x) + 2;
    const int ly = i[1] - tile_origin(bx, 1, uy, T.y) + 2;
    int idx = ly * (T.x + 4) + lx;
    if (NDIM == 3) idx += (i[2] - tile_origin(bx, 2, uz, T.z) + 2) * (T.x + 4) * (T.y + 4);
    residue = idx & (kResidues - 1);
    return k;
}

// Code word of a particle for the binning: direction code k (bits 0-4), bank
// residue of its next half-step cell (bits 5-8) and the class of its
// predicted next predictor shift (bits 9-13).
__device__ __forceinline__ uint16_t pack_code(int k, int residue, int cls) {
    return (uint16_t)(k | (residue << 5) | (cls << 9));
}
__device__ __forceinline__ int code_dir(uint32_t c) { return (int)(c & 31u); }
__device__ __forceinline__ int code_residue(uint32_t c) { return (int)((c >> 5) & 15u); }
__device__ __forceinline__ int code_class(uint32_t c) { return (int)(c >> 9); }

// Class (0 .. 3^NDIM - 1) of the cell shifts s in {-1, 0, 1} per dimension.
template <int NDIM>
__device__ __forceinline__ int shift_class(int s0, int s1, int s2) {
    return NDIM == 3 ? ((s2 + 1) * 3 + (s1 + 1)) * 3 + (s0 + 1) : (s1 + 1) * 3 + (s0 + 1);
}

__device__ __forceinline__ bool item_of_block(const uint32_t* n_items, uint32_t& item) {
    const uint32_t nitems = *n_items;
    const uint32_t per_xcd = (nitems + 7u) / 8u;
    const uint32_t bid = blockIdx.x;
    const uint32_t slot = bid >> 3;
    if (slot >= per_xcd) return false;
    item = (bid & 7u) * per_xcd + slot;
    return item < nitems;
}

// ---------------------------------------------------------------------------
// cell-centred fields: E0 = -v_g x B and the CR-Hall correction (Sec. 2.1)
// ---------------------------------------------------------------------------

// Writes EB[cell] = (Ex, Ey, Ez, Bx, By, Bz) interleaved for the gather, and
// clears the cell's n_CR, J_CR in nJ_next, which the push then fills.
template <typename TF>
__global__ void k_fieldprep(TF* __restrict__ EB, const double* __restrict__ B,
                            const double* __restrict__ vg, const double* __restrict__ rho,
                            const int64_t* __restrict__ nJ, int64_t* __restrict__ nJ_next,
                            const BoxDev* __restrict__ boxes,
                            const int64_t* __restrict__ cell_off, int nb, int64_t NC) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    const BoxDev& bx = boxes[find_box(cell_off, nb, c)];
    double b0 = B[c], b1 = B[NC + c], b2 = B[2 * NC + c];
    double g0 = vg[c], g1 = vg[NC + c], g2 = vg[2 * NC + c];
    double e0[3];
    e0[0] = -(g1 * b2 - g2 * b1);
    e0[1] = -(g2 * b0 - g0 * b2);
    e0[2] = -(g0 * b1 - g1 * b0);
    double e[3] = {e0[0], e0[1], e0[2]};
    if (bx.hall) {
        double n = ((double)nJ[c] * bx.iS) / bx.dV;
        double J0 = ((double)nJ[NC + c] * bx.iS) / bx.dV;
        double J1 = ((double)nJ[2 * NC + c] * bx.iS) / bx.dV;
        double J2 = ((double)nJ[3 * NC + c] * bx.iS) / bx.dV;
        double ng = bx.qg * rho[c];
        double R = n / (ng + n);
        double jxb[3];
        jxb[0] = J1 * b2 - J2 * b1;
        jxb[1] = J2 * b0 - J0 * b2;
        jxb[2] = J0 * b1 - J1 * b0;
        for (int d = 0; d < 3; ++d) {
            double F = (1.0 - R) * (n * e0[d] + jxb[d]);
            e[d] = e0[d] - F / ng;
        }
    }
    TF* o = EB + 6 * c;
    o[0] = (TF)e[0];
    o[1] = (TF)e[1];
    o[2] = (TF)e[2];
    o[3] = (TF)b0;
    o[4] = (TF)b1;
    o[5] = (TF)b2;
#pragma unroll
    for (int q = 0; q < 4; ++q) nJ_next[q * NC + c] = 0;
}

// Cell-centred feedback of the predictor step (App. A.3), in code units
// (c = 1, no 4 pi), from n_CR, J_CR at the particles' current positions:
//   out[0..2] -F_CR = -(1-R)(n_CR E0 + J_CR x B)      (eq. lorentz2, gasmotion)
//   out[3]    -(1-R) J_CR . E0                         (eq. engeq)
//   out[4..6] (E - E0) x B                             (eq. engeq, energy flux)
//   out[7..9] R (u_CR - v_g) / v_A, v_A = |B|/sqrt(rho), 0 where n_CR = 0 or
//             B = 0                                    (eq. lambda)
// Without the Hall term R is 0 in out[0..6]; Lambda keeps n_CR/(n_g + n_CR).
// The operations are those of the field preparation, in the same order.
__global__ void k_feedback(double* __restrict__ out, const double* __restrict__ B,
                           const double* __restrict__ vg, const double* __restrict__ rho,
                           const int64_t* __restrict__ nJ, const BoxDev* __restrict__ boxes,
                           const int64_t* __restrict__ cell_off, int nb, int64_t NC) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= NC) return;
    const BoxDev& bx = boxes[find_box(cell_off, nb, c)];
    const double b0 = B[c], b1 = B[NC + c], b2 = B[2 * NC + c];
    const double g0 = vg[c], g1 = vg[NC + c], g2 = vg[2 * NC + c];
    double e0[3];
    e0[0] = -(g1 * b2 - g2 * b1);
    e0[1] = -(g2 * b0 - g0 * b2);
    e0[2] = -(g0 * b1 - g1 * b0);
    const double n = ((double)nJ[c] * bx.iS) / bx.dV;
    double J[3];
    J[0] = ((double)nJ[NC + c] * bx.iS) / bx.dV;
    J[1] = ((double)nJ[2 * NC + c] * bx.iS) / bx.dV;
    J[2] = ((double)nJ[3 * NC + c] * bx.iS) / bx.dV;
    const double r = rho[c];
    const double ng = bx.qg * r;
    const double RL = n / (ng + n);
    const double R = bx.hall ? RL : 0.0;
    double jxb[3];
    jxb[0] = J[1] * b2 - J[2] * b1;
    jxb[1] = J[2] * b0 - J[0] * b2;
    jxb[2] = J[0] * b1 - J[1] * b0;
    double de[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double F = (1.0 - R) * (n * e0[d] + jxb[d]);
        out[d * NC + c] = -F;
        const double e = bx.hall ? e0[d] - F / ng : e0[d];
        de[d] = e - e0[d];
    }
    const double je0 = (J[0] * e0[0] + J[1] * e0[1]) + J[2] * e0[2];
    out[3 * NC + c] = -((1.0 - R) * je0);
    out[4 * NC + c] = de[1] * b2 - de[2] * b1;
    out[5 * NC + c] = de[2] * b0 - de[0] * b2;
    out[6 * NC + c] = de[0] * b1 - de[1] * b0;
    const double bb = (b0 * b0 + b1 * b1) + b2 * b2;
    double lam[3] = {0.0, 0.0, 0.0};
    if (n != 0.0 && bb > 0.0) {
        const double vA = sqrt(bb / r);
        lam[0] = (RL * (J[0] / n - g0)) / vA;
        lam[1] = (RL * (J[1] / n - g1)) / vA;
        lam[2] = (RL * (J[2] / n - g2)) / vA;
    }
    out[7 * NC + c] = lam[0];
    out[8 * NC + c] = lam[1];
    out[9 * NC + c] = lam[2];
}

// ---------------------------------------------------------------------------
// read-out in the original particle order
// ---------------------------------------------------------------------------

template <int NDIM, typename PS>
__global__ void k_read_particles(PS P, double* __restrict__ x, double* __restrict__ v,
                                 const BoxDev* __restrict__ boxes,
                                 const int64_t* __restrict__ part_off, int nb, int64_t N) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const BoxDev& bx = boxes[find_box(part_off, nb, j)];
    int64_t p = P.pid[j];
    int i[3];
    unpack_cell<NDIM>(P.cell[j], i[0], i[1], i[2]);
    for (int d = 0; d < 3; ++d) {
        double xd = 0.0;
        if (d < NDIM) xd = bx.x0[d] + bx.dx[d] * (((double)i[d] + 0.5) + (double)P.d[d][j]);
        x[d * N + p] = xd;
        v[d * N + p] = (double)P.v[d][j];
    }
}

// ---------------------------------------------------------------------------
// arithmetic self-test
// ---------------------------------------------------------------------------

__global__ void k_selftest(const double* a, const double* b, const double* c, double* out,
                           int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = __builtin_sqrt(a[i]);
    out[n + i] = a[i] / b[i];
    out[2 * n + i] = __builtin_fma(a[i], b[i], c[i]);
    out[3 * n + i] = (double)(long long)__double_as_longlong(c[i]);
}

}  // namespace mhdpic
