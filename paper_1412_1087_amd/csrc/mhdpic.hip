// Host runtime and C ABI of the MHD-PIC cosmic-ray particle library.
//
// Per mhdpic_step call (fields fixed, dt per box):
//   rekey -> scan -> scatter          bin particles by the tile of x^(n+1/2)
//   per step:
//     fieldprep                       cell-centred E (Sec. 2.1)
//     push                            gather + Boris + deposits (App. A.2, A.3);
//                                     also counts particles per next tile
//     scan -> scatter (not after the last step)
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/mhdpic.h"
#include "common.h"
#include "kernels.h"
#include "push.h"
#include "binning.h"

using namespace mhdpic;

namespace {

// Message of the last failure on this thread.  A fixed buffer: reporting an
// error allocates nothing.
thread_local char g_last_error[512] = "";

int fail(int code, const char* msg) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
    return code;
}

int fail_hip(const char* what, hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return MHDPIC_EDEVICE;
}

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return fail_hip(#expr, e_); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int32_t kMaxSubsteps = 1024;  // particle sub-steps per step, at most

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Tile shapes with compiled push kernels.
struct TileShape {
    int x, y, z;
};

constexpr size_t kLdsPerCU = 160 * 1024;

// LDS bytes of the push kernel for a tile shape (the kernel's Geo layout).
size_t push_lds_bytes(int ndim, int prec, const TileShape& t) {
    const LdsStrides st = lds_strides(t.x, t.y, t.z, ndim);
    size_t NP = ndim == 3 ? (size_t)st.sp * (t.z + 4) : (size_t)st.sx * (t.y + 4);
    size_t FOFF = ndim == 3 ? st.sp : st.sx;
    size_t NFF = NP - 2 * FOFF;
    // fields: binary64 6 words per cell, binary32 8 (two 16-byte planes)
    size_t fbytes = prec == MHDPIC_FP64 ? 6 * 8 : 8 * 4;
    return NFF * 4 * 8 + NP * 4 * 8 + NFF * fbytes + NP * 4;
}

bool tile_compiled(int ndim, const TileShape& t) {
    if (ndim == 2) {
        return (t.x == 16 && t.y == 16) || (t.x == 32 && t.y == 16) || (t.x == 8 && t.y == 8) ||
               (t.x == 32 && t.y == 32) || (t.x == 64 && t.y == 16);
    }
    return (t.x == 8 && t.y == 4 && t.z == 4) || (t.x == 8 && t.y == 8 && t.z == 4) ||
           (t.x == 4 && t.y == 4 && t.z == 4) || (t.x == 8 && t.y == 8 && t.z == 8) ||
           (t.x == 16 && t.y == 4 && t.z == 4);
}

bool tile_supported(int ndim, int prec, const TileShape& t) {
    return tile_compiled(ndim, t) && push_lds_bytes(ndim, prec, t) <= kLdsPerCU;
}

// Events that only time launches between kernels: without the system-scope
// fence, recording one does not write back and invalidate the caches between
// the kernels it separates (with it, each pair cost about 6 us of idle GPU
// around every timed launch).
constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;

// The library's tile for a box of `cells` cells and np particles: in 3D the
// shape that holds about 2048 particles (measured on the beam boxes: 8x4x4
// at 16 per cell, 4x4x4 at 32, in both precisions).
TileShape default_tile(int ndim, int64_t cells, int64_t np) {
    if (ndim == 2) return {32, 16, 1};
    if (cells > 0 && np >= 24 * cells) return {4, 4, 4};
    return {8, 4, 4};
}

struct Layout {
    // sizes: N particle slots (the capacity), N0 particles at initialisation
    int64_t N = 0, N0 = 0, NC = 0;
    int32_t NT = 0, NW = 0;
    bool tagged = false;  // particles carry tags (the context has a capacity for additions)
    // offsets into the workspace
    size_t partA = 0, partB = 0, part_bytes = 0;
    size_t key = 0, code = 0, EB = 0, Dcorr = 0, nJ0 = 0, nJ1 = 0;
    size_t count = 0, start = 0, cursor = 0, tile_box = 0, err = 0;
    size_t items[2] = {0, 0}, n_items[2] = {0, 0}, item_first[2] = {0, 0};
    size_t cnt = 0, off = 0;
    int K = 27;
    size_t boxes = 0, part_off = 0, cell_off = 0, box_count = 0, n_out = 0;
    // a sorted tail of added particles: its tile starts and work list
    size_t tail_start = 0, tail_items = 0, tail_first = 0, tail_n = 0;
    size_t total = 0;
};

// What a captured graph depends on: its arguments and the buffer state it was
// captured in (which particle, work-list and n, J buffers are current).
struct GraphKey {
    const double* B = nullptr;
    const double* vg = nullptr;
    const double* rho = nullptr;
    int32_t n_steps = 0, n_sub = 1;
    std::vector<double> dt;
    int cur = 0, it = 0, nj = 0;
    int32_t moves = 0;
    bool operator==(const GraphKey& o) const {
        return B == o.B && vg == o.vg && rho == o.rho && n_steps == o.n_steps && n_sub == o.n_sub &&
               dt == o.dt && cur == o.cur && it == o.it && nj == o.nj && moves == o.moves;
    }
};

}  // namespace

struct mhdpic_ctx {
    int ndim = 0, precision = 0, nb = 0;
    // launch groups: the boxes of one tile shape (and, while the autotuner
    // times them, one size class) go through one push launch
    std::vector<TileShape> grp_shape;
    std::vector<int32_t> box_grp;
    std::vector<TileShape> box_tile;
    // optional push time per launch group (the autotuner)
    bool grp_timing = false;
    struct GrpMark {
        int grp;
        hipEvent_t a, b;
    };
    std::vector<GrpMark> grp_marks;
    std::vector<mhdpic_box> boxes;
    std::vector<BoxDev> bdev;
    Layout L;
    unsigned char* ws = nullptr;
    int cur = 0;   // which particle buffer (0 = A, 1 = B) holds the state
    // events a timed push launch records (PhaseTimer)
    hipEvent_t push_ev[2] = {nullptr, nullptr};
    // a binning has left the map from the other buffer's slots to the
    // current one's, and the push that reads it has not run yet
    bool map_pending = false;
    // where the particles of a step move to their new slots
    // (mhdpic_set_particle_moves); automatic: in the push
    int32_t moves = MHDPIC_MOVES_AUTO;
    bool moves_in_push() const {
        return moves != MHDPIC_MOVES_IN_BINNING;
    }
    int it = 0;    // which work list describes that buffer
    int nj = 0;    // which nJ buffer is current
    hipStream_t last_stream = nullptr;
    uint32_t* err_host = nullptr;  // pinned copy of the error word
    hipEvent_t err_event = nullptr;
    bool err_pending = false;
    // optional per-phase timing: bit k set times phase k
    uint32_t timing = 0;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    bool dt_uploaded = false;
    int64_t n_init = 0;   // particles given at initialisation (ids 0 .. n_init-1)
    int64_t tail = 0;     // added particles after the slots the last sort or binning filled
    // the code words of the current buffer are those the last push wrote for
    // this dt and n_sub (so the next call's first binning needs no rekey)
    bool codes_fresh = false;
    std::vector<double> codes_dt;
    int32_t codes_nsub = 0;
    int32_t next_id = 0;  // id of the next added particle
    // cached graph of mhdpic_step_graph
    hipGraphExec_t graph_exec = nullptr;
    GraphKey graph_key;
};

namespace {

int validate_boxes(const mhdpic_box* boxes, int32_t nb, const int64_t* np, int32_t precision,
                   int& ndim, std::vector<TileShape>& tiles) {
    if (!boxes || nb < 1 || !np) return fail(MHDPIC_EINVAL, "boxes, n_boxes or n_particles invalid");
    if (precision != MHDPIC_FP64 && precision != MHDPIC_FP32_MIXED)
        return fail(MHDPIC_EINVAL, "precision must be MHDPIC_FP64 or MHDPIC_FP32_MIXED");
    ndim = boxes[0].ndim;
    if (ndim != 2 && ndim != 3) return fail(MHDPIC_EINVAL, "ndim must be 2 or 3");
    tiles.assign(nb, TileShape{});
    int64_t N = 0, NC = 0;
    for (int b = 0; b < nb; ++b) {
        const mhdpic_box& B = boxes[b];
        if (B.ndim != ndim) return fail(MHDPIC_EINVAL, "all boxes must have the same ndim");
        TileShape t{B.tile[0], B.tile[1], ndim == 3 ? B.tile[2] : 1};
        if (t.x == 0 && t.y == 0) {
            int64_t cells = 1;
            for (int d = 0; d < ndim; ++d) cells *= std::max<int64_t>(B.n[d], 0);
            t = default_tile(ndim, cells, np[b]);
        }
        if (!tile_supported(ndim, precision, t))
            return fail(MHDPIC_ENOTSUP, "tile shape has no compiled kernel or exceeds the LDS");
        tiles[b] = t;
        for (int d = 0; d < ndim; ++d) {
            if (B.n[d] < 1) return fail(MHDPIC_EINVAL, "cell counts must be >= 1");
            if (!(B.dx[d] > 0.0) || !std::isfinite(B.dx[d])) return fail(MHDPIC_EINVAL, "dx must be > 0");
            if (!std::isfinite(B.x0[d])) return fail(MHDPIC_EINVAL, "x0 must be finite");
        }
        if (ndim == 2 && B.n[2] != 1) return fail(MHDPIC_EINVAL, "n[2] must be 1 in 2D");
        if (ndim == 2 && (B.n[0] > 65536 || B.n[1] > 65536)) return fail(MHDPIC_ERANGE, "2D box too large");
        if (ndim == 3 && (B.n[0] > 2048 || B.n[1] > 2048 || B.n[2] > 1024))
            return fail(MHDPIC_ERANGE, "3D box too large");
        if (!(B.C > 0.0) || !std::isfinite(B.C)) return fail(MHDPIC_EINVAL, "C must be > 0");
        if (B.frac_bits < 0 || B.frac_bits > 60) return fail(MHDPIC_EINVAL, "frac_bits must be in 0..60");
        if (B.max_move_cells < 1 || B.max_move_cells > 2) return fail(MHDPIC_EINVAL, "max_move_cells must be 1 or 2");
        if (B.hall && !(B.qomc_gas != 0.0 && std::isfinite(B.qomc_gas)))
            return fail(MHDPIC_EINVAL, "qomc_gas must be finite and nonzero with hall = 1");
        if (np[b] < 0) return fail(MHDPIC_EINVAL, "negative particle count");
        if (B.capacity < 0) return fail(MHDPIC_EINVAL, "negative capacity");
        for (int d = 0; d < 3; ++d) {
            const int32_t lo = B.boundary[d][0], hi = B.boundary[d][1];
            if (lo < MHDPIC_PERIODIC || lo > MHDPIC_ABSORB || hi < MHDPIC_PERIODIC || hi > MHDPIC_ABSORB)
                return fail(MHDPIC_EINVAL, "boundary must be MHDPIC_PERIODIC, MHDPIC_REFLECT or MHDPIC_ABSORB");
            if ((lo == MHDPIC_PERIODIC) != (hi == MHDPIC_PERIODIC))
                return fail(MHDPIC_EINVAL, "an axis is periodic on both faces or on neither");
            if (lo != MHDPIC_PERIODIC && (d >= ndim || B.n[d] < 2))
                return fail(MHDPIC_EINVAL, "a non-periodic axis needs at least 2 cells (and z only in 3D)");
        }
        N += std::max<int64_t>(np[b], B.capacity);
        NC += (int64_t)B.n[0] * B.n[1] * (ndim == 3 ? B.n[2] : 1);
    }
    if (N >= (int64_t)1 << 31) return fail(MHDPIC_ERANGE, "at most 2^31-1 particle slots");
    if (NC >= (int64_t)1 << 31) return fail(MHDPIC_ERANGE, "at most 2^31-1 cells");
    return MHDPIC_OK;
}

Layout make_layout(const mhdpic_box* boxes, int32_t nb, const int64_t* np, int32_t precision,
                   int ndim, const std::vector<TileShape>& tiles) {
    Layout L;
    for (int b = 0; b < nb; ++b) {
        const mhdpic_box& B = boxes[b];
        L.N += std::max<int64_t>(np[b], B.capacity);
        L.N0 += np[b];
        L.tagged = L.tagged || B.capacity > 0;
        L.NC += (int64_t)B.n[0] * B.n[1] * (ndim == 3 ? B.n[2] : 1);
        const TileShape& tile = tiles[b];
        int ntx = (B.n[0] + tile.x - 1) / tile.x, nty = (B.n[1] + tile.y - 1) / tile.y;
        int ntz = ndim == 3 ? (B.n[2] + tile.z - 1) / tile.z : 1;
        L.NT += ntx * nty * ntz;
    }
    // work items: one per tile and one per 4096 slots, and as many again for a
    // tail of added particles in contexts with a capacity
    L.NW = L.NT + (int32_t)(L.N / kItemParticles) + 1;
    if (L.tagged) L.NW = 2 * L.NW;
    const size_t N = (size_t)L.N, NC = (size_t)L.NC;
    const size_t fsz = precision == MHDPIC_FP64 ? 8 : 4;
    // cell, d[ndim], v[3], m, qm (fsz each), pid, tags (binary64, if any)
    L.part_bytes = align_up(N * 4) + (size_t)ndim * align_up(N * fsz) + 3 * align_up(N * fsz) +
                   2 * align_up(N * fsz) + align_up(N * 4) + (L.tagged ? align_up(N * 8) : 0);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align_up(bytes);
        return r;
    };
    L.partA = take(L.part_bytes);
    L.partB = take(L.part_bytes);
    L.K = ndim == 3 ? 27 : 9;
    L.key = take(N * 4);
    L.code = take(N * 2);
    L.EB = take(NC * 6 * fsz);
    L.Dcorr = take(NC * 4 * 8);
    L.nJ0 = take(NC * 4 * 8);
    L.nJ1 = take(NC * 4 * 8);
    L.count = take((size_t)L.NT * 4);
    L.start = take((size_t)(L.NT + 1) * 4);
    L.cursor = take((size_t)L.NT * 4);
    L.tile_box = take((size_t)L.NT * 4);
    for (int q = 0; q < 2; ++q) {
        L.items[q] = take((size_t)L.NW * sizeof(WorkItem));
        L.n_items[q] = take(4);
        L.item_first[q] = take((size_t)(L.NT + 1) * 4);
    }
    L.cnt = take((size_t)L.NW * L.K * 4);
    L.off = take((size_t)L.NW * L.K * 4);
    L.err = take(4);
    L.boxes = take((size_t)nb * sizeof(BoxDev));
    L.part_off = take((size_t)(nb + 1) * 8);
    L.cell_off = take((size_t)(nb + 1) * 8);
    L.box_count = take((size_t)nb * 8);
    L.n_out = take(4);
    L.tail_start = take((size_t)(L.NT + 1) * 4);
    L.tail_items = take((size_t)L.NW * sizeof(WorkItem));
    L.tail_first = take((size_t)(L.NT + 1) * 4);
    L.tail_n = take(4);
    L.total = o;
    return L;
}

template <typename PS, typename T>
PS carve_particles(unsigned char* base, size_t N, int ndim, bool tagged) {
    PS P{};
    size_t o = 0;
    P.cell = reinterpret_cast<uint32_t*>(base + o);
    o += align_up(N * 4);
    for (int d = 0; d < 3; ++d) {
        if (d < ndim) {
            P.d[d] = reinterpret_cast<T*>(base + o);
            o += align_up(N * sizeof(T));
        } else {
            P.d[d] = nullptr;
        }
    }
    for (int d = 0; d < 3; ++d) {
        P.v[d] = reinterpret_cast<T*>(base + o);
        o += align_up(N * sizeof(T));
    }
    P.m = reinterpret_cast<T*>(base + o);
    o += align_up(N * sizeof(T));
    P.qm = reinterpret_cast<T*>(base + o);
    o += align_up(N * sizeof(T));
    P.pid = reinterpret_cast<int32_t*>(base + o);
    o += align_up(N * 4);
    P.tag = tagged ? reinterpret_cast<double*>(base + o) : nullptr;
    return P;
}

template <typename PS, typename T>
PS part(mhdpic_ctx* c, int which) {
    size_t off = which == 0 ? c->L.partA : c->L.partB;
    return carve_particles<PS, T>(c->ws + off, (size_t)c->L.N, c->ndim, c->L.tagged);
}

template <typename T>
T* at(mhdpic_ctx* c, size_t off) {
    return reinterpret_cast<T*>(c->ws + off);
}

unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>(grid_for(n, 256), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, n, val);
}

void fill_i64(int64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>(grid_for(n, 256), 8192);
    hipLaunchKernelGGL(k_fill_i64, dim3(g), dim3(256), 0, s, p, n);
}

// Latched device error -> code.
int code_of(uint32_t bits) {
    if (bits & ERRBIT_NONFINITE) return MHDPIC_ENONFINITE;
    if (bits & ERRBIT_RANGE) return MHDPIC_ERANGE;
    if (bits & ERRBIT_STATE) return MHDPIC_ESTATE;
    return MHDPIC_OK;
}

const char* msg_of(uint32_t bits) {
    if (bits & ERRBIT_NONFINITE) return "device: a position or velocity is not finite";
    if (bits & ERRBIT_RANGE)
        return "device: a deposit amount reached 2^51 quanta, or a position lies 2^31 or more "
               "cells from its box origin";
    if (bits & ERRBIT_STATE) return "device: a particle was outside its tile";
    return "";
}

// ---------------------------------------------------------------------------
// launch helpers, dispatched on (ndim, precision, tile)
// ---------------------------------------------------------------------------

unsigned item_grid(const Layout& L) { return (unsigned)((L.NW + 7) / 8 * 8); }

// Where a binning takes the particles' direction codes from.
enum BinKeys {
    kKeysPushed = 0,  // the push has just written them
    kKeysRekey = 1,   // recomputed for this call's dt
    kKeysStay = 2,    // none moves: a compaction that drops empty slots
};

// Re-bins the particles of the current buffer into the other one.
template <int NDIM, typename PS, typename T>
int launch_bin(mhdpic_ctx* c, hipStream_t s, int keys) {
    const Layout& L = c->L;
    PS A = part<PS, T>(c, c->cur);
    PS Bo = part<PS, T>(c, 1 - c->cur);
    const BoxDev* bd = at<BoxDev>(c, L.boxes);
    const int it = c->it;
    using Pol = typename std::conditional<std::is_same<PS, PartF64>::value, F64Pol, F32Pol>::type;
    if (keys == kKeysRekey)
        hipLaunchKernelGGL((k_rekey_items<Pol, NDIM>), dim3(item_grid(L)), dim3(256), 0, s, A,
                           at<uint16_t>(c, L.code), at<uint32_t>(c, L.cnt), at<WorkItem>(c, L.items[it]),
                           at<uint32_t>(c, L.n_items[it]), bd, at<uint32_t>(c, L.err));
    else if (keys == kKeysStay)
        hipLaunchKernelGGL((k_stay_items<PS, NDIM>), dim3(item_grid(L)), dim3(256), 0, s, A,
                           at<uint16_t>(c, L.code), at<uint32_t>(c, L.cnt), at<WorkItem>(c, L.items[it]),
                           at<uint32_t>(c, L.n_items[it]));
    const unsigned gT = grid_for(L.NT, 4);  // one wave per tile, 4 waves per block
    hipLaunchKernelGGL(k_bin_count<NDIM>, dim3(gT), dim3(256), 0, s, at<uint32_t>(c, L.cnt),
                       at<uint32_t>(c, L.item_first[it]), at<int32_t>(c, L.tile_box), bd,
                       at<uint32_t>(c, L.count), at<uint32_t>(c, L.cursor), L.NT, kItemParticles);
    hipLaunchKernelGGL(k_scan2, dim3(1), dim3(1024), 0, s, at<uint32_t>(c, L.count),
                       at<uint32_t>(c, L.cursor), at<uint32_t>(c, L.start),
                       at<uint32_t>(c, L.item_first[1 - it]), at<uint32_t>(c, L.n_items[1 - it]), L.NT);
    hipLaunchKernelGGL(k_bin_offsets<NDIM>, dim3(gT), dim3(256), 0, s, at<uint32_t>(c, L.cnt),
                       at<uint32_t>(c, L.item_first[it]), at<uint32_t>(c, L.off),
                       at<int32_t>(c, L.tile_box), bd, at<uint32_t>(c, L.start),
                       at<uint32_t>(c, L.item_first[1 - it]), at<WorkItem>(c, L.items[1 - it]),
                       L.NT, kItemParticles);
    // where the particles move (mhdpic_set_particle_moves): in the push, the
    // binning moves only the ids (and tags) and leaves the map from new slots
    // to old ones, through which the push reads the particles and writes them,
    // updated, to the other buffer; a compaction always moves them itself
    const bool map = keys != kKeysStay && c->moves_in_push();
    // (moving only ids, a block needs few registers: twice the threads per item
    // hide more of the ranking's latency)
    constexpr int BM = 512;
    auto kern = L.tagged ? (map ? k_bin_scatter_class<NDIM, PS, BM, true, true>
                                : k_bin_scatter_class<NDIM, PS, 256, true, false>)
                         : (map ? k_bin_scatter_class<NDIM, PS, BM, false, true>
                                : k_bin_scatter_class<NDIM, PS, 256, false, false>);
    hipLaunchKernelGGL(kern, dim3(item_grid(L)), dim3(map ? BM : 256), 0, s, A, Bo, at<uint16_t>(c, L.code),
                       at<uint32_t>(c, L.off), at<WorkItem>(c, L.items[it]),
                       at<uint32_t>(c, L.n_items[it]), at<uint32_t>(c, L.key));
    if (map)
        c->map_pending = true;
    else
        c->cur = 1 - c->cur;
    c->it = 1 - it;
    c->tail = 0;
    if (keys == kKeysStay) c->codes_fresh = false;  // stay codes carry no next tile
    return MHDPIC_OK;
}

// Particle arrays of P from slot off on.
template <typename PS>
PS shifted(PS P, int64_t off) {
    P.cell += off;
    for (int d = 0; d < 3; ++d) {
        if (P.d[d]) P.d[d] += off;
        P.v[d] += off;
    }
    P.m += off;
    P.qm += off;
    P.pid += off;
    if (P.tag) P.tag += off;
    return P;
}

// Sorts n particles by the tile of their cell (the boxes the part_off table
// lists, box by box), dropping those that have left their box.
//   first sort of a context: buffer cur slots [0, n) -> the other buffer,
//     which becomes current, with the work list rebuilt in list 0;
//   tail (added particles): the other buffer's slots [slot0, slot0 + n) ->
//     the current buffer's same slots, with the tail's work list in the
//     tail arrays (items name slots from slot0 on).
template <int NDIM, typename PS, typename T>
int launch_sort(mhdpic_ctx* c, hipStream_t s, int64_t n, int64_t slot0, bool tail) {
    const Layout& L = c->L;
    const int src = tail ? 1 - c->cur : c->cur, dst = tail ? c->cur : 1 - c->cur;
    PS A = shifted(part<PS, T>(c, src), slot0);
    PS Bo = shifted(part<PS, T>(c, dst), slot0);
    const SlotBoxes sb{at<int64_t>(c, L.part_off), c->nb};
    fill_u32(at<uint32_t>(c, L.count), L.NT, 0u, s);
    // per-block LDS histograms when the tiles fit (up to 128 KB of LDS), else
    // one atomic per distinct tile in each wave
    const bool lds = L.NT <= kSortLdsTiles;
    const unsigned gC = (unsigned)((n + kSortChunk - 1) / kSortChunk);
    const size_t hbytes = (size_t)L.NT * sizeof(uint32_t);
    if (lds && hbytes > 65536) {
        HIP_TRY(hipFuncSetAttribute((const void*)k_key_count_lds<NDIM, PS>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)hbytes));
        HIP_TRY(hipFuncSetAttribute((const void*)k_scatter_lds<NDIM, PS>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)hbytes));
    }
    if (n > 0 && lds)
        hipLaunchKernelGGL((k_key_count_lds<NDIM, PS>), dim3(gC), dim3(256), hbytes, s, A,
                           at<uint32_t>(c, L.key), at<uint32_t>(c, L.count), at<BoxDev>(c, L.boxes),
                           sb, n, L.NT);
    else if (n > 0)
        hipLaunchKernelGGL((k_key_cell<NDIM, PS>), dim3(grid_for(n, 256)), dim3(256), 0, s, A,
                           at<uint32_t>(c, L.key), at<uint32_t>(c, L.count), at<BoxDev>(c, L.boxes),
                           sb, n);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, at<uint32_t>(c, L.count),
                       at<uint32_t>(c, tail ? L.tail_start : L.start), at<uint32_t>(c, L.cursor),
                       at<int32_t>(c, L.tile_box), at<WorkItem>(c, tail ? L.tail_items : L.items[0]),
                       at<uint32_t>(c, tail ? L.tail_first : L.item_first[0]),
                       at<uint32_t>(c, tail ? L.tail_n : L.n_items[0]), L.NT, kItemParticles,
                       (uint32_t)slot0);
    if (n > 0 && lds)
        hipLaunchKernelGGL((k_scatter_lds<NDIM, PS>), dim3(gC), dim3(256), hbytes, s, A, Bo,
                           at<uint32_t>(c, L.key), at<uint32_t>(c, L.cursor), n, L.NT);
    else if (n > 0)
        hipLaunchKernelGGL((k_scatter<NDIM, PS>), dim3(grid_for(n, 256)), dim3(256), 0, s, A, Bo,
                           at<uint32_t>(c, L.key), at<uint32_t>(c, L.cursor), n);
    if (!tail) {
        c->cur = 1 - c->cur;
        c->it = 0;
        c->tail = 0;
    }
    return MHDPIC_OK;
}

int launch_sort_any(mhdpic_ctx* c, hipStream_t s, int64_t n, int64_t slot0, bool tail) {
    if (c->precision == MHDPIC_FP64) {
        if (c->ndim == 2) return launch_sort<2, PartF64, double>(c, s, n, slot0, tail);
        return launch_sort<3, PartF64, double>(c, s, n, slot0, tail);
    }
    if (c->ndim == 2) return launch_sort<2, PartF32, float>(c, s, n, slot0, tail);
    return launch_sort<3, PartF32, float>(c, s, n, slot0, tail);
}

template <class Pol, int NDIM, int TX, int TY, int TZ>
int launch_push_pol(mhdpic_ctx* c, hipStream_t s, bool do_pred, int grp) {
    // four waves per SIMD: two blocks of eight waves per CU, or one of
    // sixteen when the LDS boxes of the tile take more than half the CU's LDS
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    constexpr int BLOCK = G::lds_bytes() > kLdsPerCU / 2 ? 2 * PushShape<Pol, NDIM>::BLOCK
                                                         : PushShape<Pol, NDIM>::BLOCK;
    using R = typename Pol::R;
    const Layout& L = c->L;
    PushArgsT<Pol> a;
    const int dst = c->map_pending ? 1 - c->cur : c->cur;
    a.P = part<typename Pol::Part, R>(c, dst);
    a.src_delta = (int64_t)(c->cur == 0 ? L.partA : L.partB) - (int64_t)(dst == 0 ? L.partA : L.partB);
    a.map = c->map_pending ? at<uint32_t>(c, L.key) : nullptr;
    a.code = at<uint16_t>(c, L.code);
    a.cnt = at<uint32_t>(c, L.cnt);
    a.EB = at<R>(c, L.EB);
    a.Dcorr = at<int64_t>(c, L.Dcorr);
    a.nJ = at<int64_t>(c, c->nj == 0 ? L.nJ1 : L.nJ0);  // next buffer
    a.boxes = at<BoxDev>(c, L.boxes);
    a.items = at<WorkItem>(c, L.items[c->it]);
    a.n_items = at<uint32_t>(c, L.n_items[c->it]);
    a.err = at<uint32_t>(c, L.err);
    a.NC = L.NC;
    a.do_pred = do_pred ? 1 : 0;
    a.grp = c->grp_shape.size() > 1 ? grp : -1;
    size_t lds = G::lds_bytes();
    auto kern = k_push<Pol, NDIM, TX, TY, TZ, BLOCK>;
    if (lds > 65536) HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->grp_timing) {
        HIP_TRY(hipEventCreateWithFlags(&e0, kTimingEventFlags));
        HIP_TRY(hipEventCreateWithFlags(&e1, kTimingEventFlags));
        HIP_TRY(hipEventRecord(e0, s));
    }
    // a timed push carries its phase's events in the launch (start on the
    // first launch group, end on the last)
    const int last = (int)c->grp_shape.size() - 1;
    hipEvent_t ev0 = grp == 0 ? c->push_ev[0] : nullptr, ev1 = grp == last ? c->push_ev[1] : nullptr;
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, dim3(item_grid(L)), dim3(BLOCK), (uint32_t)lds, s, ev0, ev1, 0, a);
    else
        hipLaunchKernelGGL(kern, dim3(item_grid(L)), dim3(BLOCK), lds, s, a);
    if (c->grp_timing) {
        HIP_TRY(hipEventRecord(e1, s));
        c->grp_marks.push_back({grp, e0, e1});
    }
    return MHDPIC_OK;
}

template <int NDIM, int TX, int TY, int TZ>
int launch_push_t(mhdpic_ctx* c, hipStream_t s, bool p, int grp) {
    if (c->precision == MHDPIC_FP64) return launch_push_pol<F64Pol, NDIM, TX, TY, TZ>(c, s, p, grp);
    return launch_push_pol<F32Pol, NDIM, TX, TY, TZ>(c, s, p, grp);
}

// What a tiled n_CR, J_CR deposit covers: a work list and, for a removal by
// tag, the rule's two times.
struct DepositJob {
    const WorkItem* items;
    const uint32_t* n_items;
    bool remove;
    double t_cut, t_now;
};

template <class Pol, int NDIM, int TX, int TY, int TZ>
int launch_deposit_pol(mhdpic_ctx* c, hipStream_t s, const DepositJob& job, int grp) {
    constexpr int BLOCK = 256;
    using G = Geo<Pol, NDIM, TX, TY, TZ>;
    using R = typename Pol::R;
    const Layout& L = c->L;
    const size_t lds = (size_t)G::NP * 4 * 8 + (size_t)G::NP * 4;
    auto kern = job.remove ? k_deposit_nJ_tiled<Pol, NDIM, TX, TY, TZ, BLOCK, true>
                           : k_deposit_nJ_tiled<Pol, NDIM, TX, TY, TZ, BLOCK, false>;
    if (lds > 65536) HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(item_grid(L)), dim3(BLOCK), lds, s,
                       part<typename Pol::Part, R>(c, c->cur),
                       at<int64_t>(c, c->nj == 0 ? L.nJ0 : L.nJ1), L.NC, at<BoxDev>(c, L.boxes),
                       job.items, job.n_items, at<uint32_t>(c, L.err), job.t_cut, job.t_now,
                       c->grp_shape.size() > 1 ? grp : -1);
    return MHDPIC_OK;
}

template <int NDIM, int TX, int TY, int TZ>
int launch_deposit_t(mhdpic_ctx* c, hipStream_t s, const DepositJob& job, int grp) {
    if (c->precision == MHDPIC_FP64) return launch_deposit_pol<F64Pol, NDIM, TX, TY, TZ>(c, s, job, grp);
    return launch_deposit_pol<F32Pol, NDIM, TX, TY, TZ>(c, s, job, grp);
}

// Calls F<NDIM, TX, TY, TZ>(c, s, flag, g) for each launch group g of the
// context, with the group's (compiled) tile shape.
#define MHDPIC_TILE_DISPATCH(F, c, s, flag)                                                  \
    do {                                                                                     \
        for (int g_ = 0; g_ < (int)(c)->grp_shape.size(); ++g_) {                            \
            const TileShape& t_ = (c)->grp_shape[g_];                                        \
            int rc_ = 1; /* no compiled kernel */                                            \
            if ((c)->ndim == 2) {                                                            \
                if (t_.x == 16 && t_.y == 16) rc_ = F<2, 16, 16, 1>(c, s, flag, g_);        \
                else if (t_.x == 32 && t_.y == 16) rc_ = F<2, 32, 16, 1>(c, s, flag, g_);   \
                else if (t_.x == 8 && t_.y == 8) rc_ = F<2, 8, 8, 1>(c, s, flag, g_);       \
                else if (t_.x == 32 && t_.y == 32) rc_ = F<2, 32, 32, 1>(c, s, flag, g_);   \
                else if (t_.x == 64 && t_.y == 16) rc_ = F<2, 64, 16, 1>(c, s, flag, g_);   \
            } else {                                                                         \
                if (t_.x == 8 && t_.y == 4 && t_.z == 4) rc_ = F<3, 8, 4, 4>(c, s, flag, g_);        \
                else if (t_.x == 8 && t_.y == 8 && t_.z == 4) rc_ = F<3, 8, 8, 4>(c, s, flag, g_);   \
                else if (t_.x == 4 && t_.y == 4 && t_.z == 4) rc_ = F<3, 4, 4, 4>(c, s, flag, g_);   \
                else if (t_.x == 8 && t_.y == 8 && t_.z == 8) rc_ = F<3, 8, 8, 8>(c, s, flag, g_);   \
                else if (t_.x == 16 && t_.y == 4 && t_.z == 4) rc_ = F<3, 16, 4, 4>(c, s, flag, g_); \
            }                                                                                \
            if (rc_ == 1) return fail(MHDPIC_ENOTSUP, "tile shape has no compiled kernel");  \
            if (rc_) return rc_;                                                             \
        }                                                                                    \
        return MHDPIC_OK;                                                                    \
    } while (0)

// Adds n_CR, J_CR of the particles of a work list (the current one unless
// given), or takes back those of the particles a removal by tag picks.
int launch_deposit(mhdpic_ctx* c, hipStream_t s, const DepositJob& job) {
    MHDPIC_TILE_DISPATCH(launch_deposit_t, c, s, job);
}

int launch_init_deposit(mhdpic_ctx* c, hipStream_t s) {
    const DepositJob job{at<WorkItem>(c, c->L.items[c->it]), at<uint32_t>(c, c->L.n_items[c->it]),
                         false, 0.0, 0.0};
    return launch_deposit(c, s, job);
}

int launch_push_groups(mhdpic_ctx* c, hipStream_t s, bool p) {
    MHDPIC_TILE_DISPATCH(launch_push_t, c, s, p);
}

// The push of every launch group; after a binning that left a map it moves
// the particles into the other buffer.
int launch_push(mhdpic_ctx* c, hipStream_t s, bool p) {
    const int rc = launch_push_groups(c, s, p);
    if (rc) return rc;
    if (c->map_pending) {
        c->map_pending = false;
        c->cur = 1 - c->cur;
    }
    return MHDPIC_OK;
}

int launch_bin_any(mhdpic_ctx* c, hipStream_t s, int keys) {
    if (c->precision == MHDPIC_FP64) {
        if (c->ndim == 2) return launch_bin<2, PartF64, double>(c, s, keys);
        return launch_bin<3, PartF64, double>(c, s, keys);
    }
    if (c->ndim == 2) return launch_bin<2, PartF32, float>(c, s, keys);
    return launch_bin<3, PartF32, float>(c, s, keys);
}

int launch_fieldprep(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                     hipStream_t s) {
    const Layout& L = c->L;
    const int64_t* nJcur = at<int64_t>(c, c->nj == 0 ? L.nJ0 : L.nJ1);
    int64_t* nJnext = at<int64_t>(c, c->nj == 0 ? L.nJ1 : L.nJ0);
    if (c->precision == MHDPIC_FP64)
        hipLaunchKernelGGL(k_fieldprep<double>, dim3(grid_for(L.NC, 256)), dim3(256), 0, s,
                           at<double>(c, L.EB), B, vg, rho, nJcur, nJnext, at<BoxDev>(c, L.boxes),
                           at<int64_t>(c, L.cell_off), c->nb, L.NC);
    else
        hipLaunchKernelGGL(k_fieldprep<float>, dim3(grid_for(L.NC, 256)), dim3(256), 0, s,
                           at<float>(c, L.EB), B, vg, rho, nJcur, nJnext, at<BoxDev>(c, L.boxes),
                           at<int64_t>(c, L.cell_off), c->nb, L.NC);
    return MHDPIC_OK;
}

// Event pair around a phase when timing is on.
struct PhaseTimer {
    mhdpic_ctx* c;
    hipStream_t s;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    hipEvent_t take() {
        if (!c->pool.empty()) {
            hipEvent_t e = c->pool.back();
            c->pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, kTimingEventFlags) != hipSuccess) return nullptr;
        return e;
    }
    // in_launch: the phase's kernels take the events themselves (the first
    // launch its start, the last its end: mhdpic_ctx::push_ev), so no event
    // is recorded between kernels
    bool in_launch = false;
    PhaseTimer(mhdpic_ctx* c_, hipStream_t s_, int phase_, bool in_launch_ = false)
        : c(c_), s(s_), phase(phase_), in_launch(in_launch_) {
        if (!((c->timing >> phase) & 1u)) return;
        a = take();
        b = take();
        if (!a || !b) return;
        if (in_launch) {
            c->push_ev[0] = a;
            c->push_ev[1] = b;
        } else {
            (void)hipEventRecord(a, s);
        }
    }
    ~PhaseTimer() {
        if (!((c->timing >> phase) & 1u) || !a || !b) return;
        if (in_launch) {
            c->push_ev[0] = c->push_ev[1] = nullptr;
        } else {
            (void)hipEventRecord(b, s);
        }
        c->marks.push_back({phase, a, b});
    }
};

// Pick up a device error latched by earlier work, without waiting for it.
int poll_error(mhdpic_ctx* c) {
    if (!c->err_pending) return MHDPIC_OK;
    hipError_t q = hipEventQuery(c->err_event);
    if (q == hipErrorNotReady) return MHDPIC_OK;
    c->err_pending = false;
    if (q != hipSuccess) return fail(MHDPIC_EDEVICE, hipGetErrorString(q));
    uint32_t bits = *c->err_host;
    if (bits) return fail(code_of(bits), msg_of(bits));
    return MHDPIC_OK;
}

int post_error_copy(mhdpic_ctx* c, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(c->err_host, at<uint32_t>(c, c->L.err), 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(c->err_event, s));
    c->err_pending = true;
    return MHDPIC_OK;
}

// Checks the arguments of a step call against the boxes (move limit per box).
int check_step_boxes(const mhdpic_box* boxes, int32_t nb, int ndim, int64_t NC, const double* B,
                     const double* vg, const double* rho, const double* dt, int32_t n_steps,
                     int32_t n_sub) {
    if (!dt || n_steps < 0) return fail(MHDPIC_EINVAL, "dt is NULL or n_steps < 0");
    if (n_sub < 1 || n_sub > kMaxSubsteps) return fail(MHDPIC_EINVAL, "n_sub out of range");
    if (NC > 0 && (!B || !vg)) return fail(MHDPIC_EINVAL, "B or vg is NULL");
    bool any_hall = false;
    for (int b = 0; b < nb; ++b) any_hall |= boxes[b].hall != 0;
    if (any_hall && !rho) return fail(MHDPIC_EINVAL, "rho is NULL with hall = 1");
    for (int b = 0; b < nb; ++b) {
        const mhdpic_box& bx = boxes[b];
        if (!std::isfinite(dt[b])) return fail(MHDPIC_EINVAL, "dt must be finite");
        for (int d = 0; d < ndim; ++d) {
            double cells = bx.C * std::fabs(dt[b] / (double)n_sub) / bx.dx[d];
            if (!(cells <= bx.max_move_cells * (1.0 - 1e-12)))
                return fail(MHDPIC_ERANGE, "C*|dt|/dx exceeds max_move_cells");
        }
    }
    return MHDPIC_OK;
}

int check_step_args(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                    const double* dt, int32_t n_steps, int32_t n_sub) {
    if (!c) return fail(MHDPIC_EINVAL, "ctx is NULL");
    return check_step_boxes(c->boxes.data(), c->nb, c->ndim, c->L.NC, B, vg, rho, dt, n_steps, n_sub);
}

// The per-call step constants of one box: the particle step dt/n_sub, its
// half, and the half step in cells per unit velocity along each axis.
void set_step(BoxDev& d, const mhdpic_box& B, int ndim, double dt, int32_t n_sub) {
    const double dts = dt / (double)n_sub;
    d.dt = dts;
    d.hdt = 0.5 * dts;
    for (int k = 0; k < 3; ++k) d.hdx[k] = k < ndim ? d.hdt / B.dx[k] : 0.0;
}

// Refreshes the per-call step constants on the device when dt changed.  A
// stream being captured cannot take the upload (it would be replayed from
// host memory): dt must then already be current.
int set_dt(mhdpic_ctx* c, const double* dt, int32_t n_sub, hipStream_t s, bool capturing) {
    bool changed = !c->dt_uploaded;
    for (int b = 0; b < c->nb && !changed; ++b) changed = c->bdev[b].dt != dt[b] / (double)n_sub;
    if (!changed) return MHDPIC_OK;
    if (capturing)
        return fail(MHDPIC_EINVAL, "dt differs from the last call: step once before capturing");
    for (int b = 0; b < c->nb; ++b) set_step(c->bdev[b], c->boxes[b], c->ndim, dt[b], n_sub);
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.boxes, c->bdev.data(), sizeof(BoxDev) * c->nb,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host copy may change after return
    c->dt_uploaded = true;
    return MHDPIC_OK;
}

// The kernels of n_steps steps of n_sub particle sub-steps each: re-binning
// for this call's dt, then per step field preparation and per sub-step the
// push (n_CR, J_CR at the last sub-step only) and, except after the call's
// last push, re-binning.
int enqueue_steps(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                  int32_t n_steps, int32_t n_sub, hipStream_t s, bool allow_timing,
                  bool codes_valid = false) {
    if (!rho) rho = B;  // never read without the Hall term
    const uint32_t saved = c->timing;
    if (!allow_timing) c->timing = 0;
    int rc;
    {
        PhaseTimer t(c, s, 0);
        rc = launch_bin_any(c, s, codes_valid ? kKeysPushed : kKeysRekey);
    }
    for (int st = 0; st < n_steps && !rc; ++st) {
        {
            PhaseTimer t(c, s, 1);  // also clears the next n_CR, J_CR buffer
            rc = launch_fieldprep(c, B, vg, rho, s);
        }
        if (rc) break;
        for (int sub = 0; sub < n_sub && !rc; ++sub) {
            const bool last_sub = sub + 1 == n_sub;
            {
                PhaseTimer t(c, s, 2, true);
                rc = launch_push(c, s, last_sub);
            }
            if (rc) break;
            if (st + 1 < n_steps || !last_sub) {
                PhaseTimer t(c, s, 0);
                rc = launch_bin_any(c, s, kKeysPushed);
            }
        }
        if (rc) break;
        c->nj = 1 - c->nj;
    }
    c->timing = saved;
    if (rc && c->map_pending) {  // the particles never left the current buffer
        c->it = 1 - c->it;
        c->map_pending = false;
    }
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return MHDPIC_OK;
}

}  // namespace

namespace {

std::vector<TileShape> tile_candidates(int ndim, int prec) {
    std::vector<TileShape> all = ndim == 2
        ? std::vector<TileShape>{{16, 16, 1}, {32, 16, 1}, {8, 8, 1}, {32, 32, 1}, {64, 16, 1}}
        : std::vector<TileShape>{{8, 4, 4}, {8, 8, 4}, {4, 4, 4}, {8, 8, 8}, {16, 4, 4}};
    std::vector<TileShape> ok;
    for (const TileShape& t : all)
        if (tile_supported(ndim, prec, t)) ok.push_back(t);
    return ok;
}

std::vector<mhdpic_box> with_tile(const mhdpic_box* boxes, int32_t nb, const TileShape& t) {
    std::vector<mhdpic_box> v(boxes, boxes + nb);
    for (auto& b : v) {
        b.tile[0] = t.x;
        b.tile[1] = t.y;
        b.tile[2] = b.ndim == 3 ? t.z : 1;
    }
    return v;
}

}  // namespace

namespace {

// The device record of box B.  cell_off, part_off and tile_off are the cells,
// particles and tiles of the boxes before it; the step constants stay zero
// until a step sets them.
BoxDev make_boxdev(const mhdpic_box& B, int ndim, const TileShape& tile, int32_t grp,
                   int64_t cell_off, int64_t part_off, int64_t np, int32_t tile_off) {
    BoxDev d{};
    for (int k = 0; k < 3; ++k) {
        d.n[k] = (k < ndim) ? B.n[k] : 1;
        d.dx[k] = (k < ndim) ? B.dx[k] : 1.0;
        d.x0[k] = (k < ndim) ? B.x0[k] : 0.0;
    }
    const int T[3] = {tile.x, tile.y, ndim == 3 ? tile.z : 1};
    for (int k = 0; k < 3; ++k) {
        d.nt[k] = (d.n[k] + T[k] - 1) / T[k];
        d.small_last[k] = (d.nt[k] >= 2 && d.n[k] % T[k] == 1) ? 1 : 0;
    }
    d.tile_off = tile_off;
    const LdsStrides st = lds_strides(tile.x, tile.y, ndim == 3 ? tile.z : 1, ndim);
    d.lds_sx = st.sx;
    d.lds_sp = st.sp;
    for (int k = 0; k < 3; ++k) d.T[k] = T[k];
    d.grp = grp;
    for (int k = 0; k < 3; ++k) {
        d.face[k][0] = B.boundary[k][0];
        d.face[k][1] = B.boundary[k][1];
    }
    d.hall = B.hall;
    d.cell_off = cell_off;
    d.part_off = part_off;
    d.part_n = np;
    d.C = B.C;
    d.C2 = B.C * B.C;
    d.iC = 1.0 / B.C;
    d.qg = B.qomc_gas;
    d.S = std::ldexp(1.0, B.frac_bits);
    d.iS = std::ldexp(1.0, -B.frac_bits);
    d.dV = B.dx[0] * B.dx[1];
    if (ndim == 3) d.dV = d.dV * B.dx[2];
    return d;
}

// Host fields of a context over the caller's workspace; nothing is enqueued.
// Boxes of one tile shape form one launch group; with size_class (the
// autotuner), boxes of one shape and one class do.
int open_context(mhdpic_ctx* c, const mhdpic_box* boxes, int32_t n_boxes, const int64_t* np,
                 int32_t precision, void* workspace, size_t ws_bytes, const double* x,
                 const double* v, const double* m, const double* qm,
                 const int32_t* size_class = nullptr) {
    int ndim;
    std::vector<TileShape> tiles;
    int rc = validate_boxes(boxes, n_boxes, np, precision, ndim, tiles);
    if (rc) return rc;
    Layout L = make_layout(boxes, n_boxes, np, precision, ndim, tiles);
    if (!workspace) return fail(MHDPIC_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace) % kAlign) return fail(MHDPIC_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(MHDPIC_ENOMEM, "workspace too small");
    if (L.N0 > 0 && (!x || !v || !m || !qm)) return fail(MHDPIC_EINVAL, "particle arrays are NULL");
    c->ndim = ndim;
    c->precision = precision;
    c->nb = n_boxes;
    c->box_tile = tiles;
    c->box_grp.assign(n_boxes, 0);
    c->grp_shape.clear();
    std::vector<int32_t> grp_class;
    for (int b = 0; b < n_boxes; ++b) {
        const int32_t cls = size_class ? size_class[b] : 0;
        int g = 0;
        while (g < (int)c->grp_shape.size() &&
               !(c->grp_shape[g].x == tiles[b].x && c->grp_shape[g].y == tiles[b].y &&
                 c->grp_shape[g].z == tiles[b].z && grp_class[g] == cls))
            ++g;
        if (g == (int)c->grp_shape.size()) {
            c->grp_shape.push_back(tiles[b]);
            grp_class.push_back(cls);
        }
        c->box_grp[b] = g;
    }
    c->L = L;
    c->ws = static_cast<unsigned char*>(workspace);
    return MHDPIC_OK;
}

// Waits for the stream and returns the latched device error (then clears it).
// The word is read into host memory of the caller's stack.
int read_error_now(mhdpic_ctx* c, hipStream_t s) {
    uint32_t bits = 0;
    HIP_TRY(hipMemcpyAsync(&bits, c->ws + c->L.err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bits) {
        fill_u32(at<uint32_t>(c, c->L.err), 1, 0u, s);
        HIP_TRY(hipStreamSynchronize(s));
        return fail(code_of(bits), msg_of(bits));
    }
    return MHDPIC_OK;
}

// Converts n new particles (global positions, [3][n] arrays) of the boxes the
// part_off table describes into slots slot0.. of the current buffer, with ids
// pid0 + j.
void launch_convert(mhdpic_ctx* c, hipStream_t s, const double* x, const double* v,
                    const double* m, const double* qm, const double* tag, int64_t n, int64_t slot0,
                    int32_t pid0, int buf) {
    if (n <= 0) return;
    const Layout& L = c->L;
    const BoxDev* bd = at<BoxDev>(c, L.boxes);
    const int64_t* po = at<int64_t>(c, L.part_off);
    uint32_t* err = at<uint32_t>(c, L.err);
    const unsigned g = grid_for(n, 256);
    if (c->precision == MHDPIC_FP64) {
        PartF64 P = part<PartF64, double>(c, buf);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_init_convert<2, PartF64, double>), dim3(g), dim3(256), 0, s, P, x, v, m,
                               qm, tag, bd, po, c->nb, n, slot0, pid0, err);
        else
            hipLaunchKernelGGL((k_init_convert<3, PartF64, double>), dim3(g), dim3(256), 0, s, P, x, v, m,
                               qm, tag, bd, po, c->nb, n, slot0, pid0, err);
    } else {
        PartF32 P = part<PartF32, float>(c, buf);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_init_convert<2, PartF32, float>), dim3(g), dim3(256), 0, s, P, x, v, m,
                               qm, tag, bd, po, c->nb, n, slot0, pid0, err);
        else
            hipLaunchKernelGGL((k_init_convert<3, PartF32, float>), dim3(g), dim3(256), 0, s, P, x, v, m,
                               qm, tag, bd, po, c->nb, n, slot0, pid0, err);
    }
}

// Enqueues the set-up of a context opened by open_context and waits for it:
// box records (with the step constants of dt/n_sub when dt is given), the
// per-box and per-tile tables, conversion of the global positions to (cell,
// offset) form, the first sort and the n_CR, J_CR deposit at the initial
// positions (App. A.3 predictor).  The box records pass through a small host
// buffer in chunks; keep, if given, receives all of them.  Returns the error
// latched by the kernels.
int init_device(mhdpic_ctx* c, const mhdpic_box* boxes, const int64_t* np, const double* dt,
                int32_t n_sub, const double* x, const double* v, const double* m,
                const double* qm, const double* tag, hipStream_t s, BoxDev* keep) {
    const Layout& L = c->L;
    const int nb = c->nb;
    constexpr int kChunk = 16;
    BoxDev chunk[kChunk];
    int64_t cell_off = 0, part_off = 0;
    int32_t tile_off = 0;
    for (int b0 = 0; b0 < nb; b0 += kChunk) {
        const int nc = std::min(kChunk, nb - b0);
        for (int k = 0; k < nc; ++k) {
            const mhdpic_box& B = boxes[b0 + k];
            BoxDev d = make_boxdev(B, c->ndim, c->box_tile[b0 + k], c->box_grp[b0 + k], cell_off,
                                   part_off, np[b0 + k], tile_off);
            if (dt) set_step(d, B, c->ndim, dt[b0 + k], n_sub);
            cell_off += (int64_t)d.n[0] * d.n[1] * d.n[2];
            part_off += np[b0 + k];
            tile_off += d.nt[0] * d.nt[1] * d.nt[2];
            chunk[k] = d;
            if (keep) keep[b0 + k] = d;
        }
        HIP_TRY(hipMemcpyAsync(c->ws + L.boxes + sizeof(BoxDev) * b0, chunk, sizeof(BoxDev) * nc,
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the chunk buffer is reused
    }
    c->dt_uploaded = dt != nullptr;
    const BoxDev* bd = at<BoxDev>(c, L.boxes);
    const int64_t nt = std::max<int64_t>(L.NT, nb + 1);
    hipLaunchKernelGGL(k_box_tables, dim3(grid_for(nt, 256)), dim3(256), 0, s, bd, nb,
                       at<int64_t>(c, L.part_off), at<int64_t>(c, L.cell_off),
                       at<int32_t>(c, L.tile_box), L.NT);
    fill_u32(at<uint32_t>(c, L.err), 1, 0u, s);
    fill_i64(at<int64_t>(c, L.Dcorr), 4 * L.NC, s);
    fill_i64(at<int64_t>(c, L.nJ0), 4 * L.NC, s);
    c->cur = 0;
    c->nj = 0;
    launch_convert(c, s, x, v, m, qm, tag, L.N0, 0, 0, c->cur);
    c->n_init = L.N0;
    c->next_id = (int32_t)L.N0;
    int rc = launch_sort_any(c, s, L.N0, 0, false);
    if (rc) return rc;
    if (L.N0 > 0) {
        rc = launch_init_deposit(c, s);
        if (rc) return rc;
    }
    HIP_TRY(hipGetLastError());
    return read_error_now(c, s);
}

// Particles in the order of their initial ids into [3][N0] arrays; columns
// of particles that have left their box read NaN.  Not defined once particles
// were added (their ids lie beyond N0).
int read_particles(mhdpic_ctx* c, double* x, double* v, hipStream_t s) {
    const Layout& L = c->L;
    if (c->next_id != c->n_init)
        return fail(MHDPIC_ESTATE, "particles were added: read them with mhdpic_particles_read_ids");
    if (c->n_init == 0) return MHDPIC_OK;
    const BoxDev* bd = at<BoxDev>(c, L.boxes);
    const WorkItem* items = at<WorkItem>(c, L.items[c->it]);
    const uint32_t* ni = at<uint32_t>(c, L.n_items[c->it]);
    const unsigned g = item_grid(L);
    const double nan = std::nan("");
    const unsigned gf = (unsigned)std::min<int64_t>(grid_for(3 * c->n_init, 256), 8192);
    hipLaunchKernelGGL(k_fill_f64, dim3(gf), dim3(256), 0, s, x, 3 * c->n_init, nan);
    hipLaunchKernelGGL(k_fill_f64, dim3(gf), dim3(256), 0, s, v, 3 * c->n_init, nan);
    const int64_t N = c->n_init;
    if (c->precision == MHDPIC_FP64) {
        PartF64 P = part<PartF64, double>(c, c->cur);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_read_particles<2, PartF64>), dim3(g), dim3(256), 0, s, P, x, v, bd, items, ni, N);
        else
            hipLaunchKernelGGL((k_read_particles<3, PartF64>), dim3(g), dim3(256), 0, s, P, x, v, bd, items, ni, N);
    } else {
        PartF32 P = part<PartF32, float>(c, c->cur);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_read_particles<2, PartF32>), dim3(g), dim3(256), 0, s, P, x, v, bd, items, ni, N);
        else
            hipLaunchKernelGGL((k_read_particles<3, PartF32>), dim3(g), dim3(256), 0, s, P, x, v, bd, items, ni, N);
    }
    HIP_TRY(hipGetLastError());
    return MHDPIC_OK;
}

int read_deposits(mhdpic_ctx* c, int64_t* out, hipStream_t s) {
    const int64_t NC = c->L.NC;
    if (NC == 0) return MHDPIC_OK;
    const int64_t* nJ = at<int64_t>(c, c->nj == 0 ? c->L.nJ0 : c->L.nJ1);
    HIP_TRY(hipMemcpyAsync(out, nJ, 4 * NC * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(out + 4 * NC, at<int64_t>(c, c->L.Dcorr), 4 * NC * 8,
                           hipMemcpyDeviceToDevice, s));
    return MHDPIC_OK;
}

// One call from global particles to stepped particles and deposits, through
// a context that lives on this function's stack and in `ws` (nothing of it is
// kept): open, set up with the step constants, n_steps steps, read back.
// Waits for the stream.  Host memory: the context's fixed fields and a
// 16-record staging buffer, both on the stack.
int advance_impl(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* np, int32_t precision,
                 const double* x, const double* v, const double* m, const double* qm,
                 const double* B, const double* vg, const double* rho, const double* dt,
                 int32_t n_steps, int32_t n_sub, double* x_out, double* v_out, int64_t* dep_out,
                 void* ws, size_t ws_bytes, hipStream_t s) {
    mhdpic_ctx c;
    int rc = open_context(&c, boxes, n_boxes, np, precision, ws, ws_bytes, x, v, m, qm);
    if (rc) return rc;
    rc = check_step_boxes(boxes, n_boxes, c.ndim, c.L.NC, B, vg, rho, dt, n_steps, n_sub);
    if (rc) return rc;
    if ((c.L.N0 > 0 && (!x_out || !v_out)) || (c.L.NC > 0 && !dep_out))
        return fail(MHDPIC_EINVAL, "x_out, v_out or deposits_out is NULL");
    c.last_stream = s;
    rc = init_device(&c, boxes, np, dt, n_sub, x, v, m, qm, nullptr, s, nullptr);
    if (rc) return rc;
    if (n_steps > 0) rc = enqueue_steps(&c, B, vg, rho, n_steps, n_sub, s, false);
    if (!rc) rc = read_particles(&c, x_out, v_out, s);
    if (!rc) rc = read_deposits(&c, dep_out, s);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return read_error_now(&c, s);
}

}  // namespace

// Device scratch of mhdpic_advance_noalloc: the whole workspace of one call
// (particles, fields, deposits, work lists), so that the call allocates
// nothing.  Each GPU the library runs on holds its own copy until the process
// ends.  Host code never uses this name as an address: it looks up each
// device's copy once with hipGetSymbolAddress and passes that pointer.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch, looked up on the first call on
// that device, with it current, and kept.
int scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MHDPIC_ENOTSUP, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MHDPIC_EDEVICE, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MHDPIC_OK;
}

}  // namespace

namespace {

// n_CR, J_CR of the current particles at their positions, from scratch (after
// particles were added or removed: the same integers as adding or taking
// back each particle's own).

}  // namespace

namespace {
int init_ctx(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
             int32_t precision, const double* x, const double* v, const double* m,
             const double* qm, void* workspace, size_t ws_bytes, void* hip_stream,
             mhdpic_ctx** out, const int32_t* size_class);
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* mhdpic_last_error(void) { return g_last_error; }

int mhdpic_workspace_size(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                          int32_t precision, size_t* bytes) {
    if (!bytes) return fail(MHDPIC_EINVAL, "bytes is NULL");
    int ndim;
    std::vector<TileShape> tiles;
    int rc = validate_boxes(boxes, n_boxes, n_particles, precision, ndim, tiles);
    if (rc) return rc;
    *bytes = make_layout(boxes, n_boxes, n_particles, precision, ndim, tiles).total;
    return MHDPIC_OK;
}

int mhdpic_init(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                int32_t precision, const double* x, const double* v, const double* m,
                const double* qm, void* workspace, size_t ws_bytes, void* hip_stream,
                mhdpic_ctx** out) {
    return init_ctx(boxes, n_boxes, n_particles, precision, x, v, m, qm, workspace, ws_bytes,
                    hip_stream, out, nullptr);
}

}  // extern "C"

namespace {

int init_ctx(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
             int32_t precision, const double* x, const double* v, const double* m,
             const double* qm, void* workspace, size_t ws_bytes, void* hip_stream,
             mhdpic_ctx** out, const int32_t* size_class) {
    if (!out) return fail(MHDPIC_EINVAL, "out is NULL");
    *out = nullptr;
    mhdpic_ctx* c = new mhdpic_ctx();
    int rc = open_context(c, boxes, n_boxes, n_particles, precision, workspace, ws_bytes, x, v, m, qm,
                          size_class);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    if (!rc && hipHostMalloc((void**)&c->err_host, 4, hipHostMallocDefault) != hipSuccess)
        rc = fail(MHDPIC_EDEVICE, "hipHostMalloc failed");
    if (!rc) {
        *c->err_host = 0;
        if (hipEventCreateWithFlags(&c->err_event, hipEventDisableTiming) != hipSuccess)
            rc = fail(MHDPIC_EDEVICE, "hipEventCreate failed");
    }
    if (!rc) {
        c->boxes.assign(boxes, boxes + n_boxes);
        c->bdev.resize(n_boxes);
        rc = init_device(c, boxes, n_particles, nullptr, 1, x, v, m, qm, nullptr, s, c->bdev.data());
    }
    if (rc) {
        if (c->err_host) (void)hipHostFree(c->err_host);
        if (c->err_event) (void)hipEventDestroy(c->err_event);
        delete c;
        return rc;
    }
    *out = c;
    return MHDPIC_OK;
}

}  // namespace

extern "C" {

int mhdpic_advance_noalloc(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                           int32_t precision, const double* x, const double* v, const double* m,
                           const double* qm, const double* B, const double* vg, const double* rho,
                           const double* dt, int32_t n_steps, int32_t n_sub, double* x_out,
                           double* v_out, int64_t* deposits_out, void* hip_stream) {
    int ndim;
    std::vector<TileShape> tiles;
    int rc = validate_boxes(boxes, n_boxes, n_particles, precision, ndim, tiles);
    if (rc) return rc;
    const size_t need = make_layout(boxes, n_boxes, n_particles, precision, ndim, tiles).total;
    if (need > kScratchBytes) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "mhdpic_advance_noalloc: these boxes and particles need %zu bytes of scratch; "
                      "the static scratch holds %zu (use mhdpic_advance with a workspace)",
                      need, kScratchBytes);
        return MHDPIC_ENOMEM;
    }
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return advance_impl(boxes, n_boxes, n_particles, precision, x, v, m, qm, B, vg, rho, dt,
                        n_steps, n_sub, x_out, v_out, deposits_out, ws, kScratchBytes,
                        static_cast<hipStream_t>(hip_stream));
}

int mhdpic_advance(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                   int32_t precision, const double* x, const double* v, const double* m,
                   const double* qm, const double* B, const double* vg, const double* rho,
                   const double* dt, int32_t n_steps, int32_t n_sub, double* x_out, double* v_out,
                   int64_t* deposits_out, void* workspace, size_t ws_bytes, void* hip_stream) {
    return advance_impl(boxes, n_boxes, n_particles, precision, x, v, m, qm, B, vg, rho, dt,
                        n_steps, n_sub, x_out, v_out, deposits_out, workspace, ws_bytes,
                        static_cast<hipStream_t>(hip_stream));
}

int mhdpic_step(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                const double* dt, int32_t n_steps, void* hip_stream) {
    return mhdpic_step_sub(c, B, vg, rho, dt, n_steps, 1, hip_stream);
}

int mhdpic_step_sub(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                    const double* dt, int32_t n_steps, int32_t n_sub, void* hip_stream) {
    int rc = check_step_args(c, B, vg, rho, dt, n_steps, n_sub);
    if (rc) return rc;
    rc = poll_error(c);
    if (rc) return rc;
    if (n_steps == 0) return MHDPIC_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    // a captured call is replayed without this host code: it must leave the
    // particle, work-list and n, J buffers as it found them
    if (capturing && n_steps % 2)
        return fail(MHDPIC_EINVAL, "a captured call needs an even n_steps");
    c->last_stream = s;
    rc = set_dt(c, dt, n_sub, s, capturing);
    if (rc) return rc;
    // an eager call after a push with the same dt and n_sub bins with the
    // codes that push wrote; a captured call is replayed in states this
    // host code does not see, so it always recomputes them
    const bool codes_valid = !capturing && c->codes_fresh && c->codes_nsub == n_sub &&
                             std::equal(c->codes_dt.begin(), c->codes_dt.end(), dt) &&
                             (int)c->codes_dt.size() == c->nb;
    rc = enqueue_steps(c, B, vg, rho, n_steps, n_sub, s, !capturing, codes_valid);
    c->codes_fresh = false;
    if (rc) return rc;
    if (capturing) return MHDPIC_OK;
    c->codes_fresh = true;
    c->codes_dt.assign(dt, dt + c->nb);
    c->codes_nsub = n_sub;
    return post_error_copy(c, s);
}

int mhdpic_step_graph(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                      const double* dt, int32_t n_steps, void* hip_stream) {
    return mhdpic_step_graph_sub(c, B, vg, rho, dt, n_steps, 1, hip_stream);
}

int mhdpic_step_graph_sub(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                          const double* dt, int32_t n_steps, int32_t n_sub, void* hip_stream) {
    int rc = check_step_args(c, B, vg, rho, dt, n_steps, n_sub);
    if (rc) return rc;
    if (n_steps <= 0 || n_steps % 2) return fail(MHDPIC_EINVAL, "n_steps must be even and > 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (!s) return fail(MHDPIC_EINVAL, "graph capture needs a non-default stream");
    rc = poll_error(c);
    if (rc) return rc;
    c->last_stream = s;
    // the step constants live in device memory that the graph reads: bring
    // them to this dt first (a no-op when they are current)
    rc = set_dt(c, dt, n_sub, s, false);
    if (rc) return rc;
    GraphKey key{B, vg, rho, n_steps, n_sub, std::vector<double>(dt, dt + c->nb), c->cur, c->it, c->nj,
                 c->moves};
    if (!c->graph_exec || !(c->graph_key == key)) {
        if (c->graph_exec) {
            HIP_TRY(hipGraphExecDestroy(c->graph_exec));
            c->graph_exec = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = enqueue_steps(c, B, vg, rho, n_steps, n_sub, s, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail_hip("hipStreamEndCapture", e);
        e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph_exec = nullptr;
            return fail_hip("hipGraphInstantiate", e);
        }
        c->graph_key = key;  // n_steps is even: the buffers end as they began
    }
    HIP_TRY(hipGraphLaunch(c->graph_exec, s));
    c->tail = 0;  // its binnings took in any added particles
    c->codes_fresh = true;
    c->codes_dt.assign(dt, dt + c->nb);
    c->codes_nsub = n_sub;
    return post_error_copy(c, s);
}


int mhdpic_autotune_workspace_size(const mhdpic_box* boxes, int32_t n_boxes,
                                   const int64_t* n_particles, int32_t precision, size_t* bytes) {
    if (!bytes || !boxes || n_boxes < 1) return fail(MHDPIC_EINVAL, "NULL argument");
    size_t best = 0;
    for (const TileShape& t : tile_candidates(boxes[0].ndim, precision)) {
        std::vector<mhdpic_box> b = with_tile(boxes, n_boxes, t);
        size_t sz = 0;
        int rc = mhdpic_workspace_size(b.data(), n_boxes, n_particles, precision, &sz);
        if (rc) return rc;
        best = std::max(best, sz);
    }
    *bytes = best;
    return MHDPIC_OK;
}

int mhdpic_autotune(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                    int32_t precision, const double* x, const double* v, const double* m,
                    const double* qm, const double* B, const double* vg, const double* rho,
                    const double* dt, int32_t n_steps, void* workspace, size_t ws_bytes,
                    void* hip_stream, int32_t* tile_out, double* ms_per_step) {
    if (!boxes || n_boxes < 1 || !tile_out || n_steps < 1)
        return fail(MHDPIC_EINVAL, "NULL argument or n_steps < 1");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.0f;
    TileShape best{0, 0, 0};
    int rc = MHDPIC_OK;
    for (const TileShape& t : tile_candidates(boxes[0].ndim, precision)) {
        std::vector<mhdpic_box> b = with_tile(boxes, n_boxes, t);
        mhdpic_ctx* c = nullptr;
        rc = mhdpic_init(b.data(), n_boxes, n_particles, precision, x, v, m, qm, workspace, ws_bytes,
                         hip_stream, &c);
        if (rc) break;
        rc = mhdpic_step(c, B, vg, rho, dt, 2, hip_stream);  // warm-up, uploads dt
        if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventRecord");
        if (!rc) rc = mhdpic_step(c, B, vg, rho, dt, n_steps, hip_stream);
        if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventRecord");
        float ms = 0.0f;
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventSynchronize");
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventElapsedTime");
        if (!rc) rc = mhdpic_check(c, hip_stream);
        mhdpic_destroy(c);
        if (rc) break;
        if (best.x == 0 || ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    tile_out[0] = best.x;
    tile_out[1] = best.y;
    tile_out[2] = best.z;
    if (ms_per_step) *ms_per_step = best_ms / n_steps;
    return MHDPIC_OK;
}

int mhdpic_autotune_classes_workspace_size(const mhdpic_box* boxes, int32_t n_boxes,
                                           const int64_t* n_particles, int32_t precision,
                                           size_t* bytes) {
    if (!bytes || !boxes || n_boxes < 1) return fail(MHDPIC_EINVAL, "NULL argument");
    size_t best = 0;
    int rc = mhdpic_autotune_workspace_size(boxes, n_boxes, n_particles, precision, &best);
    if (rc) return rc;
    // the mix with the most tiles: each box with its candidate of most tiles
    const int ndim = boxes[0].ndim;
    std::vector<mhdpic_box> b(boxes, boxes + n_boxes);
    for (mhdpic_box& B : b) {
        int most = -1;
        for (const TileShape& t : tile_candidates(ndim, precision)) {
            const int nt = ((B.n[0] + t.x - 1) / t.x) * ((B.n[1] + t.y - 1) / t.y) *
                           (ndim == 3 ? (B.n[2] + t.z - 1) / t.z : 1);
            if (nt > most) {
                most = nt;
                B.tile[0] = t.x;
                B.tile[1] = t.y;
                B.tile[2] = ndim == 3 ? t.z : 1;
            }
        }
    }
    size_t sz = 0;
    rc = mhdpic_workspace_size(b.data(), n_boxes, n_particles, precision, &sz);
    if (rc) return rc;
    *bytes = std::max(best, sz);
    return MHDPIC_OK;
}

}  // extern "C"

namespace {

// Size class of a box for the autotuner: cells in [4^k, 4^(k+1)).
int32_t size_class_of(const mhdpic_box& B) {
    int64_t cells = (int64_t)B.n[0] * B.n[1] * (B.ndim == 3 ? B.n[2] : 1);
    int32_t k = 0;
    while (cells >= 4) {
        cells /= 4;
        ++k;
    }
    return k;
}

// Times n_steps steps of a context built from boxes b (events on stream s);
// with size classes, also the push time of each launch group (ms, summed).
int time_steps(const std::vector<mhdpic_box>& b, const int64_t* np, int32_t precision,
               const double* x, const double* v, const double* m, const double* qm,
               const double* B, const double* vg, const double* rho, const double* dt,
               int32_t n_steps, void* ws, size_t ws_bytes, void* stream, const int32_t* cls,
               float* ms_out, std::vector<float>* grp_ms, std::vector<TileShape>* grp_shape,
               std::vector<int32_t>* box_grp) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    mhdpic_ctx* c = nullptr;
    int rc = init_ctx(b.data(), (int32_t)b.size(), np, precision, x, v, m, qm, ws, ws_bytes, stream,
                      &c, cls);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = mhdpic_step(c, B, vg, rho, dt, 2, stream);  // warm-up, uploads dt
    if (!rc && hipEventCreate(&e0) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventCreate");
    if (!rc && hipEventCreate(&e1) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventCreate");
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipStreamSynchronize");
    c->grp_timing = grp_ms != nullptr;
    if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventRecord");
    if (!rc) rc = mhdpic_step(c, B, vg, rho, dt, n_steps, stream);
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventRecord");
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventSynchronize");
    if (!rc && hipEventElapsedTime(ms_out, e0, e1) != hipSuccess) rc = fail(MHDPIC_EDEVICE, "hipEventElapsedTime");
    if (!rc && grp_ms) {
        grp_ms->assign(c->grp_shape.size(), 0.0f);
        for (auto& mk : c->grp_marks) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, mk.a, mk.b) == hipSuccess) (*grp_ms)[mk.grp] += t;
        }
        if (grp_shape) *grp_shape = c->grp_shape;
        if (box_grp) *box_grp = c->box_grp;
    }
    if (!rc) rc = mhdpic_check(c, stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    mhdpic_destroy(c);
    return rc;
}

}  // namespace

extern "C" {

int mhdpic_autotune_classes(const mhdpic_box* boxes, int32_t n_boxes, const int64_t* n_particles,
                            int32_t precision, const double* x, const double* v, const double* m,
                            const double* qm, const double* B, const double* vg, const double* rho,
                            const double* dt, int32_t n_steps, void* workspace, size_t ws_bytes,
                            void* hip_stream, int32_t* tiles_out, double* ms_per_step) {
    if (!boxes || n_boxes < 1 || !tiles_out || n_steps < 1)
        return fail(MHDPIC_EINVAL, "NULL argument or n_steps < 1");
    const int ndim = boxes[0].ndim;
    std::vector<int32_t> cls(n_boxes);
    int32_t ncls = 0;
    for (int b = 0; b < n_boxes; ++b) {
        cls[b] = size_class_of(boxes[b]);
        ncls = std::max(ncls, cls[b] + 1);
    }
    // push time of each size class under each candidate shape, and the whole
    // step with one shape for all boxes
    std::vector<float> best_cls_ms(ncls, 0.0f);
    std::vector<TileShape> best_cls(ncls, TileShape{0, 0, 0});
    float best_all_ms = 0.0f;
    TileShape best_all{0, 0, 0};
    for (const TileShape& t : tile_candidates(ndim, precision)) {
        std::vector<mhdpic_box> b = with_tile(boxes, n_boxes, t);
        float ms = 0.0f;
        std::vector<float> gms;
        std::vector<TileShape> gshape;
        std::vector<int32_t> bgrp;
        int rc = time_steps(b, n_particles, precision, x, v, m, qm, B, vg, rho, dt, n_steps, workspace,
                            ws_bytes, hip_stream, cls.data(), &ms, &gms, &gshape, &bgrp);
        if (rc) return rc;
        if (best_all.x == 0 || ms < best_all_ms) {
            best_all_ms = ms;
            best_all = t;
        }
        std::vector<float> per_cls(ncls, 0.0f);
        std::vector<bool> seen(ncls, false);
        for (int bx = 0; bx < n_boxes; ++bx) {
            if (seen[cls[bx]]) continue;
            seen[cls[bx]] = true;
            per_cls[cls[bx]] = gms[bgrp[bx]];
        }
        for (int k = 0; k < ncls; ++k)
            if (seen[k] && (best_cls[k].x == 0 || per_cls[k] < best_cls_ms[k])) {
                best_cls_ms[k] = per_cls[k];
                best_cls[k] = t;
            }
    }
    // the per-class choice, kept only if its whole step beats the best single shape
    std::vector<mhdpic_box> mix(boxes, boxes + n_boxes);
    for (int b = 0; b < n_boxes; ++b) {
        const TileShape& t = best_cls[cls[b]];
        mix[b].tile[0] = t.x;
        mix[b].tile[1] = t.y;
        mix[b].tile[2] = ndim == 3 ? t.z : 1;
    }
    float mix_ms = 0.0f;
    int rc = time_steps(mix, n_particles, precision, x, v, m, qm, B, vg, rho, dt, n_steps, workspace,
                        ws_bytes, hip_stream, nullptr, &mix_ms, nullptr, nullptr, nullptr);
    if (rc) return rc;
    const bool use_mix = mix_ms < best_all_ms;
    for (int b = 0; b < n_boxes; ++b) {
        const TileShape& t = use_mix ? best_cls[cls[b]] : best_all;
        tiles_out[3 * b + 0] = t.x;
        tiles_out[3 * b + 1] = t.y;
        tiles_out[3 * b + 2] = ndim == 3 ? t.z : 1;
    }
    if (ms_per_step) *ms_per_step = (use_mix ? mix_ms : best_all_ms) / n_steps;
    return MHDPIC_OK;
}

int mhdpic_deposit_read(mhdpic_ctx* c, int64_t* out, int32_t reset_accumulated, void* hip_stream) {
    if (!c || !out) return fail(MHDPIC_EINVAL, "ctx or out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    int rc = read_deposits(c, out, s);
    if (rc) return rc;
    if (reset_accumulated) fill_i64(at<int64_t>(c, c->L.Dcorr), 4 * c->L.NC, s);
    HIP_TRY(hipGetLastError());
    return MHDPIC_OK;
}

int mhdpic_feedback(mhdpic_ctx* c, const double* B, const double* vg, const double* rho,
                    double* out, void* hip_stream) {
    if (!c || !out) return fail(MHDPIC_EINVAL, "ctx or out is NULL");
    const Layout& L = c->L;
    if (L.NC > 0 && (!B || !vg || !rho)) return fail(MHDPIC_EINVAL, "B, vg or rho is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    if (L.NC == 0) return MHDPIC_OK;
    const int64_t* nJcur = at<int64_t>(c, c->nj == 0 ? L.nJ0 : L.nJ1);
    hipLaunchKernelGGL(k_feedback, dim3(grid_for(L.NC, 256)), dim3(256), 0, s, out, B, vg, rho,
                       nJcur, at<BoxDev>(c, L.boxes), at<int64_t>(c, L.cell_off), c->nb, L.NC);
    HIP_TRY(hipGetLastError());
    return MHDPIC_OK;
}

int mhdpic_particles_read(mhdpic_ctx* c, double* x, double* v, void* hip_stream) {
    if (!c || !x || !v) return fail(MHDPIC_EINVAL, "ctx, x or v is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    return read_particles(c, x, v, s);
}

int mhdpic_counts(mhdpic_ctx* c, int64_t* counts, void* hip_stream) {
    if (!c || !counts) return fail(MHDPIC_EINVAL, "ctx or counts is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    const Layout& L = c->L;
    unsigned long long* dc = at<unsigned long long>(c, L.box_count);
    fill_i64(reinterpret_cast<int64_t*>(dc), c->nb, s);
    const WorkItem* items = at<WorkItem>(c, L.items[c->it]);
    const uint32_t* ni = at<uint32_t>(c, L.n_items[c->it]);
    if (c->precision == MHDPIC_FP64)
        hipLaunchKernelGGL(k_box_counts<PartF64>, dim3(item_grid(L)), dim3(256), 0, s,
                           part<PartF64, double>(c, c->cur), items, ni, dc);
    else
        hipLaunchKernelGGL(k_box_counts<PartF32>, dim3(item_grid(L)), dim3(256), 0, s,
                           part<PartF32, float>(c, c->cur), items, ni, dc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(counts, dc, 8 * c->nb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MHDPIC_OK;
}

int mhdpic_particles_read_ids(mhdpic_ctx* c, double* x, double* v, int32_t* ids, double* tags,
                              int64_t n_max, int64_t* n_out, void* hip_stream) {
    if (!c || !n_out || n_max < 0 || (n_max > 0 && (!x || !v || !ids)))
        return fail(MHDPIC_EINVAL, "ctx, outputs or n_max invalid");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    c->last_stream = s;
    const Layout& L = c->L;
    uint32_t* dn = at<uint32_t>(c, L.n_out);
    fill_u32(dn, 1, 0u, s);
    const BoxDev* bd = at<BoxDev>(c, L.boxes);
    const WorkItem* items = at<WorkItem>(c, L.items[c->it]);
    const uint32_t* ni = at<uint32_t>(c, L.n_items[c->it]);
    const unsigned g = item_grid(L);
    if (c->precision == MHDPIC_FP64) {
        PartF64 P = part<PartF64, double>(c, c->cur);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_read_ids<2, PartF64>), dim3(g), dim3(256), 0, s, P, x, v, ids, tags, bd, items, ni, dn, n_max);
        else
            hipLaunchKernelGGL((k_read_ids<3, PartF64>), dim3(g), dim3(256), 0, s, P, x, v, ids, tags, bd, items, ni, dn, n_max);
    } else {
        PartF32 P = part<PartF32, float>(c, c->cur);
        if (c->ndim == 2)
            hipLaunchKernelGGL((k_read_ids<2, PartF32>), dim3(g), dim3(256), 0, s, P, x, v, ids, tags, bd, items, ni, dn, n_max);
        else
            hipLaunchKernelGGL((k_read_ids<3, PartF32>), dim3(g), dim3(256), 0, s, P, x, v, ids, tags, bd, items, ni, dn, n_max);
    }
    HIP_TRY(hipGetLastError());
    uint32_t n = 0;
    HIP_TRY(hipMemcpyAsync(&n, dn, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_out = n;
    if ((int64_t)n > n_max) return fail(MHDPIC_ENOMEM, "more particles than n_max; *n_out holds their number");
    return MHDPIC_OK;
}

int mhdpic_inject(mhdpic_ctx* c, const int64_t* n_new, const double* x, const double* v,
                  const double* m, const double* qm, const double* tag, void* hip_stream) {
    if (!c || !n_new) return fail(MHDPIC_EINVAL, "ctx or n_new is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int rc = poll_error(c);
    if (rc) return rc;
    c->last_stream = s;
    const Layout& L = c->L;
    // offsets of the new particles per box, through a small host buffer
    constexpr int kChunk = 64;
    int64_t off[kChunk];
    int64_t total = 0;
    for (int b0 = 0; b0 <= c->nb; b0 += kChunk) {
        const int nc = std::min(kChunk, c->nb + 1 - b0);
        for (int k = 0; k < nc; ++k) {
            const int b = b0 + k;
            off[k] = total;
            if (b < c->nb) {
                if (n_new[b] < 0) return fail(MHDPIC_EINVAL, "negative particle count");
                total += n_new[b];
            }
        }
        HIP_TRY(hipMemcpyAsync(c->ws + L.part_off + 8 * b0, off, 8 * nc, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (total == 0) return MHDPIC_OK;
    if (!x || !v || !m || !qm) return fail(MHDPIC_EINVAL, "particle arrays are NULL");
    if ((int64_t)c->next_id + total >= ((int64_t)1 << 31)) return fail(MHDPIC_ERANGE, "particle ids exhausted");
    // room for the tail: slots after the last sorted one, and work items; a
    // compaction (a binning in which no particle moves) frees the slots of
    // removed particles and merges earlier tails
    uint32_t used[2];
    for (int pass = 0;; ++pass) {
        HIP_TRY(hipMemcpyAsync(&used[0], c->ws + L.start + 4 * (size_t)L.NT, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&used[1], c->ws + L.n_items[c->it], 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int64_t s0 = (int64_t)used[0] + c->tail;
        const int64_t items_max = (int64_t)used[1] + std::min<int64_t>(L.NT, total) + total / kItemParticles + 1;
        if (s0 + total <= L.N && items_max <= L.NW) break;
        if (pass == 1)
            return fail(MHDPIC_ENOMEM, "the context's particle slots (the boxes' capacity) are full");
        rc = launch_bin_any(c, s, kKeysStay);
        if (rc) return rc;
    }
    const int64_t s0 = (int64_t)used[0] + c->tail;
    launch_convert(c, s, x, v, m, qm, tag, total, s0, c->next_id, 1 - c->cur);
    c->next_id += (int32_t)total;
    rc = launch_sort_any(c, s, total, s0, true);
    if (rc) return rc;
    const int it = c->it;
    hipLaunchKernelGGL(k_merge_items, dim3(grid_for(L.NT + 1, 256)), dim3(256), 0, s,
                       at<WorkItem>(c, L.items[it]), at<uint32_t>(c, L.item_first[it]),
                       at<uint32_t>(c, L.n_items[it]), at<WorkItem>(c, L.tail_items),
                       at<uint32_t>(c, L.tail_first), at<uint32_t>(c, L.tail_n),
                       at<WorkItem>(c, L.items[1 - it]), at<uint32_t>(c, L.item_first[1 - it]),
                       at<uint32_t>(c, L.n_items[1 - it]), L.NT);
    c->it = 1 - it;
    c->tail += total;
    c->codes_fresh = false;  // the added particles have no code words yet
    // the new particles' n_CR, J_CR join the deposits of the state
    const DepositJob job{at<WorkItem>(c, L.tail_items), at<uint32_t>(c, L.tail_n), false, 0.0, 0.0};
    rc = launch_deposit(c, s, job);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return read_error_now(c, s);
}

int mhdpic_remove_tagged(mhdpic_ctx* c, double t_cut, double t_now, void* hip_stream) {
    if (!c) return fail(MHDPIC_EINVAL, "ctx is NULL");
    if (!c->L.tagged) return fail(MHDPIC_EINVAL, "the context has no particle tags (no capacity was given)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int rc = poll_error(c);
    if (rc) return rc;
    c->last_stream = s;
    const Layout& L = c->L;
    // the picked particles' n_CR, J_CR are taken back from the deposits of the
    // state and their slots marked empty; the next binning drops them (with
    // codes recomputed: an empty slot takes the gone code)
    c->codes_fresh = false;
    const DepositJob job{at<WorkItem>(c, L.items[c->it]), at<uint32_t>(c, L.n_items[c->it]), true,
                         t_cut, t_now};
    rc = launch_deposit(c, s, job);
    if (rc) return rc;
    HIP_TRY(hipGetLastError());
    return read_error_now(c, s);
}

int mhdpic_check(mhdpic_ctx* c, void* hip_stream) {
    if (!c) return fail(MHDPIC_EINVAL, "ctx is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(c->err_host, at<uint32_t>(c, c->L.err), 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    c->err_pending = false;
    uint32_t bits = *c->err_host;
    fill_u32(at<uint32_t>(c, c->L.err), 1, 0u, s);
    HIP_TRY(hipStreamSynchronize(s));
    if (bits) return fail(code_of(bits), msg_of(bits));
    return MHDPIC_OK;
}

int mhdpic_set_particle_moves(mhdpic_ctx* c, int32_t where) {
    if (!c) return fail(MHDPIC_EINVAL, "ctx is NULL");
    if (where != MHDPIC_MOVES_AUTO && where != MHDPIC_MOVES_IN_BINNING && where != MHDPIC_MOVES_IN_PUSH)
        return fail(MHDPIC_EINVAL, "unknown particle move setting");
    c->moves = where;
    return MHDPIC_OK;
}

int mhdpic_timing_enable(mhdpic_ctx* c, int32_t phases) {
    if (!c) return fail(MHDPIC_EINVAL, "ctx is NULL");
    if (phases < 0 || phases > MHDPIC_TIMING_ALL) return fail(MHDPIC_EINVAL, "phases must be a mask of bits 0..3");
    c->timing = (uint32_t)phases;
    return MHDPIC_OK;
}

int mhdpic_timing_read(mhdpic_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(MHDPIC_EINVAL, "NULL argument");
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& mk : c->marks) {
        HIP_TRY(hipEventSynchronize(mk.b));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, mk.a, mk.b));
        ms[mk.phase] += t;
        launches[mk.phase] += 1;
        c->pool.push_back(mk.a);
        c->pool.push_back(mk.b);
    }
    c->marks.clear();
    return MHDPIC_OK;
}

int mhdpic_destroy(mhdpic_ctx* c) {
    if (!c) return MHDPIC_OK;
    if (c->graph_exec) {
        if (c->last_stream) (void)hipStreamSynchronize(c->last_stream);
        (void)hipGraphExecDestroy(c->graph_exec);
    }
    for (auto& mk : c->marks) {
        (void)hipEventSynchronize(mk.b);
        c->pool.push_back(mk.a);
        c->pool.push_back(mk.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    for (auto& mk : c->grp_marks) {
        (void)hipEventSynchronize(mk.b);
        (void)hipEventDestroy(mk.a);
        (void)hipEventDestroy(mk.b);
    }
    if (c->err_event) {
        (void)hipEventSynchronize(c->err_event);
        (void)hipEventDestroy(c->err_event);
    }
    if (c->err_host) (void)hipHostFree(c->err_host);
    delete c;
    return MHDPIC_OK;
}

int mhdpic_selftest_arith(const double* a, const double* b, const double* cc, double* out,
                          int64_t n, void* hip_stream) {
    if (n <= 0) return MHDPIC_OK;
    if (!a || !b || !cc || !out) return fail(MHDPIC_EINVAL, "NULL pointer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(k_selftest, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, cc, out, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return MHDPIC_OK;
}

}  // extern "C"
