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

// Largest offset below 1/2 (a particle mirrored onto the upper face).
__device__ __forceinline__ double below_half(double) { return 0x1.fffffffffffffp-2; }
__device__ __forceinline__ float below_half(float) { return 0x1.fffffep-2f; }

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

// Tables derived from the box records: first particle and first cell of each
// box (with the totals at index nb), and the box of every tile.
__global__ void k_box_tables(const BoxDev* __restrict__ boxes, int nb, int64_t* __restrict__ part_off,
                             int64_t* __restrict__ cell_off, int32_t* __restrict__ tile_box, int NT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        part_off[i] = boxes[i].part_off;
        cell_off[i] = boxes[i].cell_off;
    } else if (i == nb) {
        const BoxDev& l = boxes[nb - 1];
        part_off[nb] = l.part_off + l.part_n;
        cell_off[nb] = l.cell_off + (int64_t)l.n[0] * l.n[1] * l.n[2];
    }
    if (i < NT) {
        int lo = 0, hi = nb - 1;  // last box whose first tile is <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boxes[mid].tile_off <= i) lo = mid; else hi = mid - 1;
        }
        tile_box[i] = lo;
    }
}

// Converts new particles j = 0 .. N-1 (global positions x, four-velocities
// v, [3][N]; m, qm, optional tags, [N]) of the boxes new_off[] describes
// into slots slot0 + j of P, with ids pid0 + j.  Without tags a particle's
// tag is +infinity (no removal by tag ever takes it).
template <int NDIM, typename PS, typename T>
__global__ void k_init_convert(PS P, const double* __restrict__ x, const double* __restrict__ v,
                               const double* __restrict__ m, const double* __restrict__ qm,
                               const double* __restrict__ tag, const BoxDev* __restrict__ boxes,
                               const int64_t* __restrict__ new_off, int nb, int64_t N,
                               int64_t slot0, int32_t pid0, uint32_t* err) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    int b = find_box(new_off, nb, j);
    const BoxDev& bx = boxes[b];
    const int64_t sl = slot0 + j;
    int ic[3] = {0, 0, 0};
    bool bad = false, far = false;
    for (int d = 0; d < NDIM; ++d) {
        double s = (x[d * N + j] - bx.x0[d]) / bx.dx[d];
        double fl = floor(s);
        if (!isfinite(s)) bad = true;
        // the cell count from x0 must fit a 32-bit int; on a non-periodic
        // axis the position must lie inside the box
        else if (!(fl >= -2147483648.0 && fl < 2147483648.0)) far = true;
        else if (bx.face[d][0] != FACE_PERIODIC && !(fl >= 0.0 && fl < (double)bx.n[d])) far = true;
        double off = (s - fl) - 0.5;
        ic[d] = (bad || far) ? 0 : pmod((int)(long long)fl, bx.n[d]);
        T o = (T)off;
        if (o >= (T)0.5) {  // binary32 rounding can reach the upper edge
            if (bx.face[d][0] != FACE_PERIODIC && ic[d] == bx.n[d] - 1) {
                o = below_half(T(0));
            } else {
                o = o - (T)1;
                ic[d] = wrap_shift(ic[d], 1, bx.n[d]);
            }
        }
        P.d[d][sl] = o;
    }
    for (int d = 0; d < 3; ++d) {
        double vd = v[d * N + j];
        if (!isfinite(vd)) bad = true;
        P.v[d][sl] = (T)vd;
    }
    if (!isfinite(m[j]) || !isfinite(qm[j])) bad = true;
    if (bad) latch(err, ERRBIT_NONFINITE);
    if (far) latch(err, ERRBIT_RANGE);
    P.cell[sl] = pack_cell<NDIM>(ic[0], ic[1], ic[2]);
    P.m[sl] = m[j];
    P.qm[sl] = qm[j];
    P.pid[sl] = pid0 + (int32_t)j;
    if (P.tag) P.tag[sl] = tag ? tag[j] : (double)INFINITY;
}

// ---------------------------------------------------------------------------
// binning by tile of the half-step cell x^(n+1/2)
// ---------------------------------------------------------------------------

// Cell index along axis d of a coordinate that may lie beyond the box (by at
// most two cells past a non-periodic face): wrapped on a periodic axis,
// mirrored at a non-periodic face (cell -1-k is cell k, cell n+k is n-1-k).
__device__ __forceinline__ int map_index(const BoxDev& bx, int d, int i) {
    const int n = bx.n[d];
    if (bx.face[d][0] == FACE_PERIODIC) return pmod(i, n);
    return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

// Global index of cell (x, y, z) of a box; coordinates may lie outside
// [0, n) and are wrapped or mirrored (map_index).
template <int NDIM>
__device__ __forceinline__ int64_t global_cell(const BoxDev& bx, int x, int y, int z) {
    x = map_index(bx, 0, x);
    y = map_index(bx, 1, y);
    z = NDIM == 3 ? map_index(bx, 2, z) : 0;
    return bx.cell_off + ((int64_t)z * bx.n[1] + y) * bx.n[0] + x;
}

// Shift value of half_drift for a particle that left through an absorbing face.
constexpr int kGone = 8;

// After a half drift has moved the cell index along axis d by one cell at
// most (i is then -1 .. n): wraps it on a periodic axis; at a reflecting face
// mirrors the position back (offset, the axis's four-velocity v and
// three-velocity u negated); at an absorbing face returns true (the particle
// leaves the box).  From cell 0 the offset in cell -1 is above -1/2, so its
// negation stays below 1/2; at the upper face it can be exactly -1/2.
template <typename R>
__device__ __forceinline__ bool cross_face(const BoxDev& bx, int d, int& i, R& dl, R& v, R& u) {
    const int n = bx.n[d];
    if (i >= 0 && i < n) return false;
    if (bx.face[d][0] == FACE_PERIODIC) {
        i = i < 0 ? i + n : i - n;
        return false;
    }
    const int side = i < 0 ? 0 : 1;
    if (bx.face[d][side] == FACE_ABSORB) return true;
    dl = -dl;
    v = -v;
    u = -u;
    if (side == 0) {
        i = 0;
    } else {
        i = n - 1;
        if (dl >= R(0.5)) dl = below_half(R(0));
    }
    return false;
}

// One half drift along axis d (App. A.2: x += u dt/2) of a particle in cell i
// at offset dl, then the face it may have crossed.  Returns the cell shift as
// the tile's LDS boxes see it (-1, 0, +1; a mirrored particle is back in its
// own cell, a wrapped one moved by one cell across the periodic seam), or
// kGone if the particle left through an absorbing face.
template <class Pol, typename R>
__device__ __forceinline__ int half_drift(const BoxDev& bx, int d, int& i, R& dl, R& v, R& u, R h) {
    const int s = Pol::drift(dl, u, h);
    if (s == 0) return 0;
    i += s;
    if (i >= 0 && i < bx.n[d]) return s;
    const bool periodic = bx.face[d][0] == FACE_PERIODIC;
    if (cross_face(bx, d, i, dl, v, u)) return kGone;
    return periodic ? s : 0;
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

// Key of a particle that a sort drops (it has left its box).
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// Box of slot j of a sort's source: slots are filled box by box, off[b] being
// box b's first (off has nb + 1 entries).
struct SlotBoxes {
    const int64_t* off;
    int nb;
    __device__ __forceinline__ int box(int64_t j) const { return find_box(off, nb, j); }
};

// Exclusive scan of tile counts and the work list: each tile's particles are
// split into items of at most P particles; items name slots from base on.
// One block of 1024 threads.
__global__ void __launch_bounds__(1024)
k_scan(const uint32_t* __restrict__ count, uint32_t* __restrict__ start,
       uint32_t* __restrict__ cursor, const int32_t* __restrict__ tile_box,
       WorkItem* __restrict__ items, uint32_t* __restrict__ item_first,
       uint32_t* __restrict__ n_items, int NT, int P, uint32_t base) {
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
            w.begin = (int32_t)(base + off + k);
            w.end = (int32_t)(base + off + min(k + (uint32_t)P, c));
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

// Copies particle j of A to slot s of Bo (every array).
template <int NDIM, typename PS>
__device__ __forceinline__ void copy_particle(const PS& A, const PS& Bo, int64_t j, int64_t s) {
    Bo.cell[s] = A.cell[j];
    for (int d = 0; d < NDIM; ++d) Bo.d[d][s] = A.d[d][j];
    for (int d = 0; d < 3; ++d) Bo.v[d][s] = A.v[d][j];
    Bo.m[s] = A.m[j];
    Bo.qm[s] = A.qm[j];
    Bo.pid[s] = A.pid[j];
    if (A.tag) Bo.tag[s] = A.tag[j];
}

// Work list of the current buffer after a sorted tail of new particles was
// appended: tile t's items are its old items followed by its tail items.
// The first item of each tile is the sum of the two lists' prefix sums.
__global__ void k_merge_items(const WorkItem* __restrict__ a, const uint32_t* __restrict__ a_first,
                              const uint32_t* __restrict__ a_n, const WorkItem* __restrict__ b,
                              const uint32_t* __restrict__ b_first, const uint32_t* __restrict__ b_n,
                              WorkItem* __restrict__ out, uint32_t* __restrict__ out_first,
                              uint32_t* __restrict__ out_n, int NT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > NT) return;
    uint32_t o = a_first[t] + b_first[t];
    out_first[t] = o;
    if (t == NT) {
        *out_n = *a_n + *b_n;
        return;
    }
    for (uint32_t k = a_first[t]; k < a_first[t + 1]; ++k) out[o++] = a[k];
    for (uint32_t k = b_first[t]; k < b_first[t + 1]; ++k) out[o++] = b[k];
}

// Moves every particle to its slot in the tile-sorted order (dropping those
// keyed kNoTile).
template <int NDIM, typename PS>
__global__ void k_scatter(PS A, PS Bo, const uint32_t* __restrict__ key,
                          uint32_t* __restrict__ cursor, int64_t N) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t k = j < N ? key[j] : kNoTile;
    bool act = k != kNoTile;
    uint32_t s = wave_claim(cursor, act ? k : 0u, act);
    if (!act) return;
    copy_particle<NDIM>(A, Bo, j, s);
}

// ---------------------------------------------------------------------------
// direction codes of tile-to-tile moves
// ---------------------------------------------------------------------------

template <int NDIM>
struct Codes {
    static constexpr int K = NDIM == 3 ? 27 : 9;
    static constexpr int STAY = NDIM == 3 ? 13 : 4;
    static constexpr int GONE = 31;  // leaves the box: dropped by the binning
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
    int idx = ly * bx.lds_sx + lx;
    if (NDIM == 3) idx += (i[2] - tile_origin(bx, 2, uz, T.z) + 2) * bx.lds_sp;
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

// Code word of a particle at cell i, offset dl, with four-velocity v and
// three-velocity u, for the next binning: the operations of the next step's
// first half drift (faces included) give its half-step cell, whose tile
// (relative to the item's tile tx, ty, tz) and bank residue go into the code,
// with the class of the predicted second-drift shift.  A particle that has
// left (gone) or that this drift takes through an absorbing face gets the
// gone code.  Returns the direction code.
template <class Pol, int NDIM, typename R>
__device__ __forceinline__ int next_code(const BoxDev& bx, int3 T, int tx, int ty, int tz,
                                         const int i[3], const R dl[3], const R v[3], const R u[3],
                                         R hx, R hy, R hz, bool gone, uint32_t& errbits,
                                         uint16_t& code) {
    int ni[3] = {i[0], i[1], i[2]};
    R e[3] = {dl[0], dl[1], dl[2]}, w[3] = {v[0], v[1], v[2]}, q[3] = {u[0], u[1], u[2]};
    if (!gone) gone = half_drift<Pol>(bx, 0, ni[0], e[0], w[0], q[0], hx) == kGone;
    if (!gone) gone = half_drift<Pol>(bx, 1, ni[1], e[1], w[1], q[1], hy) == kGone;
    if (NDIM == 3 && !gone) gone = half_drift<Pol>(bx, 2, ni[2], e[2], w[2], q[2], hz) == kGone;
    if (gone) {
        code = pack_code(Codes<NDIM>::GONE, 0, 0);
        return Codes<NDIM>::GONE;
    }
    int res;
    const int k = move_code<NDIM>(bx, T, tx, ty, tz, ni, errbits, res);
    // predicted shift of the predictor deposit after that drift (velocity as now)
    const int p0 = Pol::drift(e[0], q[0], hx), p1 = Pol::drift(e[1], q[1], hy);
    const int p2 = NDIM == 3 ? Pol::drift(e[2], q[2], hz) : 0;
    code = pack_code(k, res, shift_class<NDIM>(p0, p1, p2));
    return k;
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

// Global position of slot j: x0 + dx((i + 1/2) + d) per axis (z = 0 in 2D).
template <int NDIM, typename PS>
__device__ __forceinline__ void slot_position(const PS& P, const BoxDev& bx, int64_t j, double x[3]) {
    int i[3];
    unpack_cell<NDIM>(P.cell[j], i[0], i[1], i[2]);
    for (int d = 0; d < 3; ++d)
        x[d] = d < NDIM ? bx.x0[d] + bx.dx[d] * (((double)i[d] + 0.5) + (double)P.d[d][j]) : 0.0;
}

// Particles in the order of their ids: slot j goes to column pid of the
// [3][N] outputs (N: the ids given at initialisation).  One block per work
// item; a particle that has left its box is skipped (its columns keep what
// the caller filled them with).
template <int NDIM, typename PS>
__global__ void k_read_particles(PS P, double* __restrict__ x, double* __restrict__ v,
                                 const BoxDev* __restrict__ boxes, const WorkItem* __restrict__ items,
                                 const uint32_t* __restrict__ n_items, int64_t N) {
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    const BoxDev& bx = boxes[w.box];
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += blockDim.x) {
        if (P.cell[j] == kDeadCell) continue;
        const int64_t p = P.pid[j];
        double xx[3];
        slot_position<NDIM>(P, bx, j, xx);
        for (int d = 0; d < 3; ++d) {
            x[d * N + p] = xx[d];
            v[d * N + p] = (double)P.v[d][j];
        }
    }
}

// The particles in the boxes, compacted: each live slot takes the next
// output column from *n_out (one atomic per wave); [3][n_max] outputs,
// columns beyond n_max are not written (*n_out still counts them).
template <int NDIM, typename PS>
__global__ void k_read_ids(PS P, double* __restrict__ x, double* __restrict__ v,
                           int32_t* __restrict__ ids, double* __restrict__ tags,
                           const BoxDev* __restrict__ boxes, const WorkItem* __restrict__ items,
                           const uint32_t* __restrict__ n_items, uint32_t* __restrict__ n_out,
                           int64_t n_max) {
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    const BoxDev& bx = boxes[w.box];
    const int lane = lane_id();
    // the same trip count in every lane of a wave (ballot below)
    for (int j0 = w.begin; j0 < w.end; j0 += blockDim.x) {
        const int j = j0 + (int)threadIdx.x;
        const bool live = j < w.end && P.cell[j] != kDeadCell;
        const uint64_t mask = __ballot(live);
        uint32_t base = 0;
        const int leader = mask ? __ffsll((unsigned long long)mask) - 1 : 0;
        if (mask && lane == leader) base = atomicAdd(n_out, (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (!live) continue;
        const int64_t o = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (o >= n_max) continue;
        double xx[3];
        slot_position<NDIM>(P, bx, j, xx);
        for (int d = 0; d < 3; ++d) {
            x[d * n_max + o] = xx[d];
            v[d * n_max + o] = (double)P.v[d][j];
        }
        ids[o] = P.pid[j];
        if (tags) tags[o] = P.tag ? P.tag[j] : (double)INFINITY;
    }
}

// Live particles per box (counts[b], zeroed by the caller).
template <typename PS>
__global__ void k_box_counts(PS P, const WorkItem* __restrict__ items,
                             const uint32_t* __restrict__ n_items,
                             unsigned long long* __restrict__ counts) {
    __shared__ uint32_t s_n;
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint32_t n = 0;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += blockDim.x) n += P.cell[j] != kDeadCell;
    atomicAdd(&s_n, n);
    __syncthreads();
    if (threadIdx.x == 0 && s_n) atomicAdd(&counts[w.box], (unsigned long long)s_n);
}

__global__ void k_fill_f64(double* p, int64_t n, double val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = val;
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
