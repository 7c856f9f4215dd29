// Device-side data structures shared by the kernels and the host runtime of
// the MHD-PIC cosmic-ray particle library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mhdpic {

// Particle boundary of a face.
enum : int32_t { FACE_PERIODIC = 0, FACE_REFLECT = 1, FACE_ABSORB = 2 };

// Packed cell of a particle that has left its box through an absorbing face;
// it stays in its slot until the next binning drops it.
constexpr uint32_t kDeadCell = 0xFFFFFFFFu;

// Error bits latched by kernels in the device error word.
enum : uint32_t {
    ERRBIT_NONFINITE = 1u,  // a velocity or position became non-finite
    ERRBIT_RANGE = 2u,      // a deposit amount |V| >= 2^51 quanta, or a position
                            // more than 2^31 cells from the box origin
    ERRBIT_STATE = 4u,      // a particle was not inside the tile it was binned to
};

// 1.5 * 2^52: adding a double of magnitude < 2^51 to it rounds that double to
// an integer (round-half-even) held exactly in the low mantissa bits.  The
// low 32 bits of its bit pattern are zero.
constexpr double kMagic = 6755399441055744.0;
constexpr uint32_t kMagicHi = 0x43380000u;
constexpr double kMaxAmount = 2251799813685248.0;  // 2^51
constexpr int kItemParticles = 4096;  // particles per work item (at most)

// Box descriptor as the kernels see it.  Per-call fields (dt, hdt, hdx) are
// refreshed by mhdpic_step before its kernels are enqueued.
// Row and plane strides of a tile's LDS boxes (tile + 2 ghost cells per
// side).  The push's LDS accesses are served 16 lanes at a time over 16 bank
// groups, and the bank group of a cell is its box index modulo 16; the binning
// orders each group of particles (those arriving from one direction, or
// staying) over those residues.  Particles arriving through a face of the
// tile fill one layer of cells, so the strides are padded (at most 3 cells
// per row, 15 per plane) for the layers normal to each axis, and the whole
// tile, to spread over the 16 residues as evenly as their cell counts allow
// (the smallest boxes among the best).
struct LdsStrides {
    int sx, sp;
};
// Largest count of one residue, minus the even share, over the cells
// s0*i + s1*j + s2*k (0 <= i < n0, 0 <= j < n1, 0 <= k < n2).
__host__ __device__ constexpr int residue_excess(int n0, int n1, int n2, int s0, int s1, int s2) {
    int cnt[16] = {};
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) cnt[(s0 * i + s1 * j + s2 * k) % 16]++;
    int mx = 0;
    for (int r = 0; r < 16; ++r) mx = cnt[r] > mx ? cnt[r] : mx;
    return mx - (n0 * n1 * n2 + 15) / 16;
}
__host__ __device__ constexpr LdsStrides lds_strides(int tx, int ty, int tz, int ndim) {
    const int rx = tx + 4, ry = ty + 4;
    LdsStrides best{rx, rx * ry};
    int best_score = 1 << 30, best_cells = 1 << 30;
    for (int px = 0; px < 4; ++px) {
        for (int pz = 0; pz < (ndim == 3 ? 16 : 1); ++pz) {
            const int sx = rx + px, sp = sx * ry + pz;
            int score = 0;
            if (ndim == 2)
                score = residue_excess(ty, 1, 1, sx, 0, 0) + residue_excess(tx, 1, 1, 1, 0, 0) +
                        residue_excess(tx, ty, 1, 1, sx, 0);
            else
                score = residue_excess(ty, tz, 1, sx, sp, 0) + residue_excess(tx, tz, 1, 1, sp, 0) +
                        residue_excess(tx, ty, 1, 1, sx, 0) + residue_excess(tx, ty, tz, 1, sx, sp);
            const int cells = ndim == 3 ? sp * (tz + 4) : sx * ry;
            if (score < best_score || (score == best_score && cells < best_cells)) {
                best_score = score;
                best_cells = cells;
                best = LdsStrides{sx, sp};
            }
        }
    }
    return best;
}

struct BoxDev {
    int32_t n[3];      // cells per dimension (n[2] = 1 in 2D)
    int32_t nt[3];     // tiles per dimension
    int32_t tile_off;  // global index of this box's first tile
    int32_t hall;
    int32_t small_last[3];  // 1: the last tile starts at n-2 (no 1-cell tiles)
    int32_t face[3][2];     // per axis, low/high: FACE_PERIODIC, FACE_REFLECT, FACE_ABSORB
    int32_t lds_sx, lds_sp; // row and plane strides (cells) of the tile's LDS boxes
    int32_t T[3];           // tile shape (T[2] = 1 in 2D)
    int32_t grp;            // launch group: the boxes one push launch takes
    int32_t pad0;
    int64_t cell_off;  // global index of this box's first cell
    int64_t part_off;  // first particle slot of this box
    int64_t part_n;    // particles in this box
    double dx[3];
    double x0[3];
    double C, C2, iC;  // C, C*C, 1/C
    double qg;         // (q/mc) of the gas ions
    double S, iS;      // 2^frac_bits, 2^-frac_bits
    double dV;         // cell volume
    double dt, hdt;    // step and half step of the current call
    double hdx[3];     // hdt / dx[d]
};

// Particle store, structure of arrays.  cell holds the packed cell indices
// (2D: ix | iy<<16; 3D: ix | iy<<11 | iz<<22); d holds the offsets from the
// cell centre in cell units; v the spatial four-velocity gamma*u.
// pid is the particle's id (its index in the initial arrays, then numbered
// on from there for added particles); tag, present only in contexts with a
// particle capacity for additions, is the caller's tag of each particle (the
// injection time of Sec. 5), moved with the particle and never read by the
// step.
struct PartF64 {
    using R = double;
    uint32_t* cell;
    double* d[3];
    double* v[3];
    double* m;
    double* qm;
    int32_t* pid;
    double* tag;
};

// Precision form: every per-particle value in single precision (the tag
// stays binary64).
struct PartF32 {
    using R = float;
    uint32_t* cell;
    float* d[3];
    float* v[3];
    float* m;
    float* qm;
    int32_t* pid;
    double* tag;
};

struct WorkItem {
    int32_t tile;   // global tile index
    int32_t begin;  // first particle slot
    int32_t end;    // one past the last slot
    int32_t box;
};

template <int NDIM>
__host__ __device__ inline uint32_t pack_cell(int ix, int iy, int iz) {
    if (NDIM == 2) return (uint32_t)ix | ((uint32_t)iy << 16);
    return (uint32_t)ix | ((uint32_t)iy << 11) | ((uint32_t)iz << 22);
}

template <int NDIM>
__host__ __device__ inline void unpack_cell(uint32_t c, int& ix, int& iy, int& iz) {
    if (NDIM == 2) {
        ix = (int)(c & 0xFFFFu);
        iy = (int)(c >> 16);
        iz = 0;
    } else {
        ix = (int)(c & 0x7FFu);
        iy = (int)((c >> 11) & 0x7FFu);
        iz = (int)(c >> 22);
    }
}

}  // namespace mhdpic
