// Binning of particles by the tile of their half-step cell, without global
// atomics on shared counters.
//
// Between steps a particle moves at most one tile in each dimension (tiles
// are at least two cells wide and a step moves at most two cells), so each
// particle's next tile is given by a direction code relative to the tile of
// the work item that processed it: code = (cz*3 + cy)*3 + cx with c = 0, 1, 2
// for -1, 0, +1 tiles (2D: cy*3 + cx).  A work item counts its particles per
// code in LDS and stores the counts; one scan block turns all counts into the
// destination offset of every (item, code) group and into the next work list;
// the scatter then moves each particle to its group's offset plus a rank taken
// from an LDS counter.  No counter is shared between blocks.
#pragma once
#include "kernels.h"
#include "push.h"

namespace mhdpic {

// Code words for this call's dt (the push computes them for the later steps
// of the call): next_code of each particle's stored state, with the
// operations of the step's first half drift.
template <class Pol, int NDIM>
__global__ void __launch_bounds__(256)
k_rekey_items(typename Pol::Part P, uint16_t* __restrict__ code, uint32_t* __restrict__ cnt,
              const WorkItem* __restrict__ items, const uint32_t* __restrict__ n_items,
              const BoxDev* __restrict__ boxes, uint32_t* err) {
    using R = typename Pol::R;
    constexpr int K = Codes<NDIM>::K;
    __shared__ uint32_t s_cnt[K];
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    const BoxDev bx = boxes[w.box];
    const int3 T = make_int3(bx.T[0], bx.T[1], bx.T[2]);
    int tx, ty, tz;
    tile_coords<NDIM>(bx, w.tile, tx, ty, tz);
    for (int c = threadIdx.x; c < K; c += blockDim.x) s_cnt[c] = 0;
    __syncthreads();
    const R hx = Pol::hdx(bx.hdx[0]), hy = Pol::hdx(bx.hdx[1]), hz = Pol::hdx(bx.hdx[2]);
    uint32_t errbits = 0;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += blockDim.x) {
        const uint32_t cell = P.cell[j];
        int i[3];
        unpack_cell<NDIM>(cell, i[0], i[1], i[2]);
        R dl[3] = {P.d[0][j], P.d[1][j], NDIM == 3 ? P.d[2][j] : R(0)};
        R v[3] = {P.v[0][j], P.v[1][j], P.v[2][j]};
        typename Pol::K kn = Pol::kin(v, bx.C, bx.C2, bx.iC);
        const int k = next_code<Pol, NDIM>(bx, T, tx, ty, tz, i, dl, v, kn.u, hx, hy, hz,
                                           cell == kDeadCell, errbits, code[j]);
        if (k != Codes<NDIM>::GONE) atomicAdd(&s_cnt[k], 1u);
    }
    if (errbits) latch(err, errbits);
    __syncthreads();
    for (int c = threadIdx.x; c < K; c += blockDim.x) cnt[(size_t)item * K + c] = s_cnt[c];
}

// Codes of a binning in which no particle moves: STAY, or GONE for an empty
// slot (a particle taken out), with each item's counts.
template <typename PS, int NDIM>
__global__ void __launch_bounds__(256)
k_stay_items(PS P, uint16_t* __restrict__ code, uint32_t* __restrict__ cnt,
             const WorkItem* __restrict__ items, const uint32_t* __restrict__ n_items) {
    constexpr int K = Codes<NDIM>::K;
    __shared__ uint32_t s_stay;
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    if (threadIdx.x == 0) s_stay = 0;
    __syncthreads();
    uint32_t n = 0;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += blockDim.x) {
        const bool live = P.cell[j] != kDeadCell;
        code[j] = (uint16_t)(live ? Codes<NDIM>::STAY : Codes<NDIM>::GONE);
        n += live;
    }
    atomicAdd(&s_stay, n);
    __syncthreads();
    for (int c = threadIdx.x; c < K; c += blockDim.x)
        cnt[(size_t)item * K + c] = c == Codes<NDIM>::STAY ? s_stay : 0u;
}

// Source tile of destination tile d for code k.
template <int NDIM>
__device__ __forceinline__ int source_tile(const BoxDev& bx, int d, int k) {
    int tx, ty, tz;
    tile_coords<NDIM>(bx, d, tx, ty, tz);
    int cx = k % 3, cy = (k / 3) % 3, cz = NDIM == 3 ? k / 9 : 1;
    int sx = pmod(tx - (cx - 1), bx.nt[0]);
    int sy = pmod(ty - (cy - 1), bx.nt[1]);
    int sz = NDIM == 3 ? pmod(tz - (cz - 1), bx.nt[2]) : 0;
    return bx.tile_off + (sz * bx.nt[1] + sy) * bx.nt[0] + sx;
}

// The groups arriving at destination tile d, in order (code by code, and
// within a code the source tile's items in order), spread over the lanes of
// one wave: lane k < K holds code k's first source item and its number of
// items, and group g of the list is code k_of(g), item i_of(g).
template <int NDIM>
struct TileGroups {
    static constexpr int K = Codes<NDIM>::K;
    uint32_t i0, pre, total;  // lane k: first item of code k, groups before code k
    __device__ __forceinline__ void load(const BoxDev& bx, int d, const uint32_t* item_first,
                                         int lane) {
        uint32_t n = 0;
        i0 = 0;
        if (lane < K) {
            const int s = source_tile<NDIM>(bx, d, lane);
            i0 = item_first[s];
            n = item_first[s + 1] - i0;
        }
        uint32_t x = n;  // inclusive scan over the lanes
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        pre = x - n;
        total = __shfl(x, 63);
    }
    // code and item of group g (g < total); every lane of the wave calls it
    __device__ __forceinline__ void group(uint32_t g, int& k, uint32_t& item) const {
        k = 0;
        for (int q = 1; q < K; ++q)
            if ((uint32_t)__shfl(pre, q) <= g) k = q;
        item = (uint32_t)__shfl(i0, k) + (g - (uint32_t)__shfl(pre, k));
    }
};

// Per destination tile: particles arriving from the (item, code) groups of
// the current work list, and the number of next-step work items.  One wave
// per tile.
template <int NDIM>
__global__ void __launch_bounds__(256)
k_bin_count(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ item_first,
            const int32_t* __restrict__ tile_box, const BoxDev* __restrict__ boxes,
            uint32_t* __restrict__ tile_count, uint32_t* __restrict__ tile_items, int NT, int P) {
    constexpr int K = Codes<NDIM>::K;
    const int lane = threadIdx.x & 63;
    const int d = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (d >= NT) return;  // whole wave
    TileGroups<NDIM> tg;
    tg.load(boxes[tile_box[d]], d, item_first, lane);
    uint32_t tot = 0;
    for (uint32_t g0 = 0; g0 < tg.total; g0 += 64) {  // the same trip count in every lane
        int k;
        uint32_t i;
        tg.group(g0 + lane, k, i);
        if (g0 + lane < tg.total) tot += cnt[(size_t)i * K + k];
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if (lane == 0) {
        tile_count[d] = tot;
        tile_items[d] = (tot + (uint32_t)P - 1) / (uint32_t)P;
    }
}

// One block: exclusive scans of tile_count (-> start) and tile_items
// (-> item_first_next, with the total in n_items_next).
__global__ void __launch_bounds__(1024)
k_scan2(const uint32_t* __restrict__ tile_count, const uint32_t* __restrict__ tile_items,
        uint32_t* __restrict__ start, uint32_t* __restrict__ item_first_next,
        uint32_t* __restrict__ n_items_next, int NT) {
    __shared__ uint32_t s_a[1024], s_b[1024];
    const int t = threadIdx.x;
    const int per = (NT + 1023) / 1024;
    const int t0 = min(t * per, NT), t1 = min(t0 + per, NT);
    uint32_t sa = 0, sb = 0;
    for (int i = t0; i < t1; ++i) {
        sa += tile_count[i];
        sb += tile_items[i];
    }
    s_a[t] = sa;
    s_b[t] = sb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint32_t a = t >= o ? s_a[t - o] : 0u;
        uint32_t b = t >= o ? s_b[t - o] : 0u;
        __syncthreads();
        s_a[t] += a;
        s_b[t] += b;
        __syncthreads();
    }
    uint32_t ra = s_a[t] - sa, rb = s_b[t] - sb;
    for (int i = t0; i < t1; ++i) {
        start[i] = ra;
        item_first_next[i] = rb;
        ra += tile_count[i];
        rb += tile_items[i];
    }
    if (t == 1023) {
        start[NT] = s_a[1023];
        item_first_next[NT] = s_b[1023];
        *n_items_next = s_b[1023];
    }
}

// Per destination tile: the offset of every arriving (item, code) group, in
// the order of TileGroups, and the tile's next-step work items.  One wave per
// tile; group counts are scanned across the wave.
template <int NDIM>
__global__ void __launch_bounds__(256)
k_bin_offsets(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ item_first,
              uint32_t* __restrict__ off, const int32_t* __restrict__ tile_box,
              const BoxDev* __restrict__ boxes, const uint32_t* __restrict__ start,
              const uint32_t* __restrict__ item_first_next,
              WorkItem* __restrict__ items_next, int NT, int P) {
    constexpr int K = Codes<NDIM>::K;
    const int lane = threadIdx.x & 63;
    const int d = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (d >= NT) return;  // whole wave
    TileGroups<NDIM> tg;
    tg.load(boxes[tile_box[d]], d, item_first, lane);
    const uint32_t s0 = start[d];
    uint32_t run = s0;
    for (uint32_t g0 = 0; g0 < tg.total; g0 += 64) {  // the same trip count in every lane
        int k;
        uint32_t i;
        tg.group(g0 + lane, k, i);
        const bool in = g0 + lane < tg.total;
        const uint32_t c = in ? cnt[(size_t)i * K + k] : 0u;
        uint32_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (in) off[(size_t)i * K + k] = run + x - c;
        run += __shfl(x, 63);
    }
    const uint32_t c = run - s0;
    const uint32_t io = item_first_next[d];
    for (uint32_t q = (uint32_t)lane; q * (uint32_t)P < c; q += 64) {
        WorkItem w;
        w.tile = d;
        w.begin = (int32_t)(s0 + q * (uint32_t)P);
        w.end = (int32_t)(s0 + min((q + 1) * (uint32_t)P, c));
        w.box = tile_box[d];
        items_next[io + q] = w;
    }
}

// Moving the arrays of one item through LDS: each array is loaded in source
// order (coalesced) into registers, written to an LDS staging buffer, and
// stored in destination order (coalesced).  The next array's loads are issued
// while the current one is being stored.
struct MoveMap {
    const uint16_t* from;  // local slot -> source index in the item
    const uint8_t* grp;    // local slot -> group
    const uint32_t* goff;  // group -> destination of local slot 0
    int begin, n;          // first source slot, source particles
    int nd;                // destination slots (the particles that stay in a box)
};

template <int BLOCK, typename T>
struct ItemRegs {  // this thread's elements threadIdx.x + u*BLOCK of one array
    static constexpr int U = kItemParticles / BLOCK;
    T v[U];
    __device__ __forceinline__ void load(const T* __restrict__ src, const MoveMap& mm) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = threadIdx.x + u * BLOCK;
            if (i < mm.n) v[u] = src[mm.begin + i];
        }
    }
    __device__ __forceinline__ void stage(T* st, const MoveMap& mm) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = threadIdx.x + u * BLOCK;
            if (i < mm.n) st[i] = v[u];
        }
    }
};

// Stages `cur`, then stores it in destination order while `nxt` (if given)
// is loaded.  Every thread of the block calls it.
template <int BLOCK, typename TC, typename TN>
__device__ __forceinline__ void move_step(const ItemRegs<BLOCK, TC>& cur, TC* __restrict__ dst,
                                          void* stage, ItemRegs<BLOCK, TN>& nxt,
                                          const TN* __restrict__ nsrc, const MoveMap& mm) {
    TC* st = reinterpret_cast<TC*>(stage);
    cur.stage(st, mm);
    __syncthreads();
    if (nsrc) nxt.load(nsrc, mm);
    // a fixed trip count, so the LDS reads of all the thread's slots overlap
    constexpr int U = kItemParticles / BLOCK;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int L = threadIdx.x + u * BLOCK;
        if (L < mm.nd) dst[mm.goff[mm.grp[L]] + (uint32_t)L] = st[mm.from[L]];
    }
    __syncthreads();
}

// Source slots per chunk of the level order of a 2D binning whose push reads
// the particles through the map (a power of two dividing kItemParticles).
#ifndef MHDPIC_MAP_CHUNK_2D
#define MHDPIC_MAP_CHUNK_2D 256
#endif
constexpr int kMapChunk2D = MHDPIC_MAP_CHUNK_2D;

// Moves the particles of each current work item to their groups' offsets.
//
// Order within a group (the particles of one item with one direction code):
// the particles that stay in the tile are grouped by the class of their
// predicted predictor shift, and each class, like each moving group, is laid
// out level by level: level r holds the r-th particle of every bank residue
// present, in residue order.  Sixteen consecutive particles of a level have
// distinct residues at their next half-step cell and, sharing one shift, at
// their predictor cell too, so the lanes of the next push fall on distinct
// LDS bank pairs in both deposits.
//
// Pass 1 ranks every particle within its (group, residue) by an LDS counter;
// pass 2 turns the ranks into an LDS map from destination to source, and the
// particles are moved one array at a time through LDS (MoveMap, move_step).
// TAGGED: the context carries particle tags (binary64), moved last; the
// staging buffer is then 8 bytes per particle in both precisions.
// MAP: only the ids (and tags) are moved; the kernel writes, for every
// destination slot, the slot its particle has in A, and the next push reads
// the particle there and stores it, updated, at the destination (the push
// reads and writes every particle anyway, so the other arrays need no move
// of their own).  The push's reads are then gathers, and a level order over
// a whole group of isotropic particles, whose residues change at random from
// step to step, draws the 64 particles of a wave from some 26 lines of
// 16 slots (a random walk of the residue counts); in 2D the levels therefore
// run over chunks of kMapChunk2D source slots, without the stay classes,
// which brings it to about 10 lines for a few more same-residue lanes.  The
// particles of the 3D boxes (drifting beams) keep their order from step to
// step well enough, and there the stay classes pay for themselves.
template <int NDIM, typename PS, int BLOCK, bool TAGGED, bool MAP>
__global__ void __launch_bounds__(BLOCK)
k_bin_scatter_class(PS A, PS Bo, const uint16_t* __restrict__ code, const uint32_t* __restrict__ off,
                    const WorkItem* __restrict__ items, const uint32_t* __restrict__ n_items,
                    uint32_t* __restrict__ map) {
    constexpr int K = Codes<NDIM>::K;
    constexpr int STAY = Codes<NDIM>::STAY;
    constexpr int NCL = K;        // shift classes (3^NDIM)
    constexpr int NG = NCL + K;   // groups: stay classes, then moving codes
    constexpr int RS = kResidues;
    // levels run over a whole group, or over each chunk of CH source slots
    // of it (then without stay classes) when a 2D push reads through the map
    constexpr int CH = (MAP && NDIM == 2) ? kMapChunk2D : kItemParticles;
    constexpr int NCH = kItemParticles / CH;
    constexpr bool CLASSES = NCH == 1;
    __shared__ uint32_t s_n[NCH * NG * RS];
    __shared__ uint32_t s_cb[NCH * NG];  // slots of the group's earlier chunks
    __shared__ uint32_t s_off[NG], s_lbase[NG], s_nd;
    __shared__ uint16_t s_src[kItemParticles];
    __shared__ uint8_t s_grp[kItemParticles];
    using SR = typename std::conditional<
        TAGGED, double, typename std::conditional<MAP, uint32_t, typename PS::R>::type>::type;
    __shared__ SR s_stage[kItemParticles];
    uint32_t* s_key = reinterpret_cast<uint32_t*>(s_stage);  // ranks, until the moves
    uint32_t item;
    if (!item_of_block(n_items, item)) return;
    const WorkItem w = items[item];
    if (w.end - w.begin > kItemParticles) return;  // never built larger
    using R = typename PS::R;
    constexpr int NR = NDIM + 5;  // offsets, four-velocity, m, q/m
    constexpr int U = kItemParticles / BLOCK;
    MoveMap mm{s_src, s_grp, s_off, w.begin, w.end - w.begin, 0};
    const R* rsrc[NR];
    R* rdst[NR];
#pragma unroll
    for (int q = 0; q < NDIM; ++q) {
        rsrc[q] = A.d[q];
        rdst[q] = Bo.d[q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        rsrc[NDIM + q] = A.v[q];
        rdst[NDIM + q] = Bo.v[q];
    }
    rsrc[NDIM + 3] = A.m;
    rdst[NDIM + 3] = Bo.m;
    rsrc[NDIM + 4] = A.qm;
    rdst[NDIM + 4] = Bo.qm;
    // the codes, the cells and the first array are loaded before the ranking
    // so that their latency overlaps it
    uint32_t cr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int L = threadIdx.x + u * BLOCK;
        cr[u] = L < mm.n ? code[w.begin + L] : 0u;
    }
    ItemRegs<BLOCK, uint32_t> rcell;
    ItemRegs<BLOCK, int32_t> rpid;
    ItemRegs<BLOCK, R> rbuf[2];
    if (MAP) {
        rpid.load(A.pid, mm);
    } else {
        rcell.load(A.cell, mm);
        rbuf[0].load(rsrc[0], mm);
    }
    for (int c = threadIdx.x; c < NCH * NG * RS; c += BLOCK) s_n[c] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int L = threadIdx.x + u * BLOCK;
        if (L < mm.n) {
            const int k = code_dir(cr[u]), b = code_residue(cr[u]);
            if (k == Codes<NDIM>::GONE) {  // left the box: no destination slot
                s_key[L] = 0xFFFFFFFFu;
                continue;
            }
            const int c = NCH > 1 ? L / CH : 0;
            const int g = k == STAY ? (CLASSES ? code_class(cr[u]) : 0) : NCL + k;
            const uint32_t r = atomicAdd(&s_n[(c * NG + g) * RS + b], 1u);
            s_key[L] = r | ((uint32_t)b << 12) | ((uint32_t)g << 16) | ((uint32_t)c << 22);
        }
    }
    __syncthreads();
    if (NCH > 1) {  // particles of each (chunk, group)
        for (int t = threadIdx.x; t < NCH * NG; t += BLOCK) {
            uint32_t n = 0;
#pragma unroll
            for (int b = 0; b < RS; ++b) n += s_n[t * RS + b];
            s_cb[t] = n;
        }
        __syncthreads();
    }
    // group bases: the stay classes in class order from the stay group's
    // offset, the moving groups at their own offsets; lane g of the first
    // wave scans the group sizes (and turns its chunk counts into bases)
    static_assert(NG <= 64, "one lane per group");
    static_assert(NCH <= 64 && CH <= 4096, "chunk and rank fields of the key");
    if (threadIdx.x < 64) {
        const int g = threadIdx.x;
        uint32_t t = 0;
        if (g < NG) {
            if (NCH > 1) {
                for (int c = 0; c < NCH; ++c) {
                    const uint32_t n = s_cb[c * NG + g];
                    s_cb[c * NG + g] = t;
                    t += n;
                }
            } else {
#pragma unroll
                for (int b = 0; b < RS; ++b) t += s_n[g * RS + b];
            }
        }
        uint32_t x = t;  // inclusive scan over the lanes
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (g >= o) x += y;
        }
        const uint32_t lb = x - t;  // slots of the groups before g
        if (g == 63) s_nd = x;      // all groups: the particles that stay
        if (g < NG) {
            const uint32_t base = g < NCL ? off[(size_t)item * K + STAY] + lb
                                          : off[(size_t)item * K + (g - NCL)];
            s_off[g] = base - lb;  // destination of local slot L of group g: s_off[g] + L
            s_lbase[g] = lb;
        }
    }
    __syncthreads();
    mm.nd = (int)s_nd;
    for (int j = w.begin + (int)threadIdx.x; j < w.end; j += BLOCK) {
        const uint32_t key = s_key[j - w.begin];
        if (key == 0xFFFFFFFFu) continue;
        const uint32_t r = key & 4095u;
        const int b = (int)((key >> 12) & 15u), g = (int)((key >> 16) & 63u), c = (int)(key >> 22);
        const uint32_t* nk = s_n + (c * NG + g) * RS;
        uint32_t pos = NCH > 1 ? s_cb[c * NG + g] : 0u;
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const uint32_t nq = nk[q];
            pos += min(nq, r) + ((q < b && nq > r) ? 1u : 0u);
        }
        s_src[s_lbase[g] + pos] = (uint16_t)(j - w.begin);
        s_grp[s_lbase[g] + pos] = (uint8_t)g;
    }
    __syncthreads();
    if (MAP) {
        constexpr int UD = kItemParticles / BLOCK;
#pragma unroll
        for (int u = 0; u < UD; ++u) {
            const int L = threadIdx.x + u * BLOCK;
            if (L < mm.nd) map[mm.goff[mm.grp[L]] + (uint32_t)L] = (uint32_t)mm.begin + mm.from[L];
        }
        if (TAGGED) {
            ItemRegs<BLOCK, double> rtag;
            move_step<BLOCK>(rpid, Bo.pid, s_stage, rtag, (const double*)A.tag, mm);
            move_step<BLOCK>(rtag, Bo.tag, s_stage, rcell, (const uint32_t*)nullptr, mm);
        } else {
            move_step<BLOCK>(rpid, Bo.pid, s_stage, rcell, (const uint32_t*)nullptr, mm);
        }
        return;
    }
    // the arrays one after another, through LDS, in destination order, with
    // two arrays in flight: array q+2 is loaded while array q is stored
    move_step<BLOCK>(rcell, Bo.cell, s_stage, rbuf[1], rsrc[1], mm);
#pragma unroll
    for (int q = 0; q + 2 < NR; ++q)
        move_step<BLOCK>(rbuf[q & 1], rdst[q], s_stage, rbuf[q & 1], rsrc[q + 2], mm);
    move_step<BLOCK>(rbuf[(NR - 2) & 1], rdst[NR - 2], s_stage, rpid, A.pid, mm);
    move_step<BLOCK>(rbuf[(NR - 1) & 1], rdst[NR - 1], s_stage, rcell, (const uint32_t*)nullptr, mm);
    if (TAGGED) {
        ItemRegs<BLOCK, double> rtag;
        move_step<BLOCK>(rpid, Bo.pid, s_stage, rtag, (const double*)A.tag, mm);
        move_step<BLOCK>(rtag, Bo.tag, s_stage, rcell, (const uint32_t*)nullptr, mm);
    } else {
        move_step<BLOCK>(rpid, Bo.pid, s_stage, rcell, (const uint32_t*)nullptr, mm);
    }
}

// Sort key of slot j: the tile of the particle's current cell (any tile of
// its box), or kNoTile for a particle that has left its box.
template <int NDIM, typename PS>
__device__ __forceinline__ uint32_t sort_key(const PS& P, int64_t j, const SlotBoxes& sb,
                                             const BoxDev* boxes) {
    const uint32_t c = P.cell[j];
    if (c == kDeadCell) return kNoTile;
    const BoxDev& bx = boxes[sb.box(j)];
    int i[3];
    unpack_cell<NDIM>(c, i[0], i[1], i[2]);
    return tile_of<NDIM>(bx, make_int3(bx.T[0], bx.T[1], bx.T[2]), i[0], i[1], i[2]);
}

// Sort by tile (first sort of a context, and re-sorts after particles are
// added or removed), with global counters.
template <int NDIM, typename PS>
__global__ void k_key_cell(PS P, uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                           const BoxDev* __restrict__ boxes, SlotBoxes sb, int64_t N) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t k = kNoTile;
    if (j < N) {
        k = sort_key<NDIM>(P, j, sb, boxes);
        key[j] = k;
    }
    const bool act = k != kNoTile;
    wave_claim(count, act ? k : 0u, act);
}

// The same sort with per-block tile histograms in LDS, for a tile count that
// fits (NT <= kSortLdsTiles): each block takes kSortChunk consecutive
// particles, counts their tiles in LDS and adds each non-zero count to the
// global counter once, so a counter sees one atomic per block however the
// particles are ordered.
constexpr int kSortChunk = 4096;
constexpr int kSortLdsTiles = 32768;  // 128 KB of LDS histogram at most

template <int NDIM, typename PS>
__global__ void __launch_bounds__(256)
k_key_count_lds(PS P, uint32_t* __restrict__ key, uint32_t* __restrict__ count,
                const BoxDev* __restrict__ boxes, SlotBoxes sb, int64_t N, int NT) {
    extern __shared__ uint32_t s_h[];
    constexpr int U = kSortChunk / 256;
    for (int t = threadIdx.x; t < NT; t += 256) s_h[t] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * kSortChunk;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + threadIdx.x + u * 256;
        if (j < N) {
            const uint32_t k = sort_key<NDIM>(P, j, sb, boxes);
            key[j] = k;
            if (k != kNoTile) atomicAdd(&s_h[k], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NT; t += 256)
        if (s_h[t]) atomicAdd(&count[t], s_h[t]);
}

// Moves every particle to its slot in the tile-sorted order: the same chunks
// and LDS histograms as k_key_count_lds; each block claims one range per
// tile from the global cursor and hands out its slots in LDS.  Particles
// keyed kNoTile are dropped.
template <int NDIM, typename PS>
__global__ void __launch_bounds__(256)
k_scatter_lds(PS A, PS Bo, const uint32_t* __restrict__ key, uint32_t* __restrict__ cursor,
              int64_t N, int NT) {
    extern __shared__ uint32_t s_h[];
    constexpr int U = kSortChunk / 256;
    for (int t = threadIdx.x; t < NT; t += 256) s_h[t] = 0;
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * kSortChunk;
    uint32_t k[U], r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + threadIdx.x + u * 256;
        k[u] = j < N ? key[j] : kNoTile;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = k[u] != kNoTile ? atomicAdd(&s_h[k[u]], 1u) : 0u;
    __syncthreads();
    for (int t = threadIdx.x; t < NT; t += 256) {
        const uint32_t c = s_h[t];
        if (c) s_h[t] = atomicAdd(&cursor[t], c);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + threadIdx.x + u * 256;
        if (k[u] != kNoTile) copy_particle<NDIM>(A, Bo, j, s_h[k[u]] + r[u]);
    }
}

}  // namespace mhdpic
