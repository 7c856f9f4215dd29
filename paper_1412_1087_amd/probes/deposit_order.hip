// Measurement program (not part of the library): the LDS deposit step of the
// 2D push, 3 x 3 TSC cells x 4 channels of int64 amounts per particle
// (App. A.1 weights, amounts rounded to the nearest integer through
// fma(W, V, 1.5*2^52)), in three orders of particles over the lanes:
//  mode 0: the binning's order: 16 consecutive lanes on cells distinct
//          modulo 16, one LDS atomic per lane and amount;
//  mode 1: cell order in a dense band (every lane of a wave in one cell),
//          one LDS atomic per lane and amount (all on one address);
//  mode 2: cell order with the wave's 64 amounts summed across lanes first
//          (DPP row shifts and broadcasts, 64-bit), one lane's atomics.
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang
// -packed-fp32-ops -o deposit_order deposit_order.hip; each kernel's time
// comes from rocprofv3 --kernel-trace --stats.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>

constexpr int SX = 37, NB = 37 * 20;  // 32x16 tile + ghosts, padded row
constexpr int ROUNDS = 64;
constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ uint32_t hsh(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

template <int CTRL, int RMASK, int BMASK>
__device__ __forceinline__ uint64_t dpp_step(uint64_t x) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    const uint32_t l2 = __builtin_amdgcn_update_dpp(0u, lo, CTRL, RMASK, BMASK, false);
    const uint32_t h2 = __builtin_amdgcn_update_dpp(0u, hi, CTRL, RMASK, BMASK, false);
    return x + (((uint64_t)h2 << 32) | l2);
}
__device__ __forceinline__ uint64_t dpp_sum_to_last(uint64_t v) {
    // inclusive scan steps to lane 63: row_shr 1,2,4,8 (rows of 16), row_bcast15, row_bcast31
    v = dpp_step<0x111, 0xf, 0xf>(v);
    v = dpp_step<0x112, 0xf, 0xf>(v);
    v = dpp_step<0x114, 0xf, 0xe>(v);
    v = dpp_step<0x118, 0xf, 0xc>(v);
    v = dpp_step<0x142, 0xa, 0xf>(v);
    v = dpp_step<0x143, 0xc, 0xf>(v);
    return v;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_dep(const double* dd, unsigned long long* out) {
    __shared__ unsigned long long box[4 * NB];
    for (int i = threadIdx.x; i < 4 * NB; i += blockDim.x) box[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t h = hsh((blockIdx.x * 4 + wave) * 1315423911u + r * 2654435761u);
        int cell;
        if (MODE == 0) {
            // 16 lanes over 16 distinct residues; rows of 37 cells, lx 2..33, ly 2..17
            const int res = ((lane & 15) * 7 + (h & 15)) & 15;
            const int ly = 2 + ((h >> 4) + (lane >> 4) * 5) % 16;
            int lx = 2 + ((res - (ly * SX + 2)) % 16 + 16) % 16;  // lx with (ly*SX+lx) % 16 == res
            lx += 16 * ((h >> 8) & 1);
            cell = ly * SX + lx;
        } else {
            cell = (2 + (h % 16)) * SX + 2 + ((h >> 5) % 32);  // one cell for the whole wave
        }
        const double dx = dd[(lane + r * 64) & 4095], dy = dd[(lane * 7 + r * 64 + 1) & 4095];
        const double wx[3] = {0.5 * (0.5 - dx) * (0.5 - dx), 0.75 - dx * dx, 0.5 * (0.5 + dx) * (0.5 + dx)};
        const double wy[3] = {0.5 * (0.5 - dy) * (0.5 - dy), 0.75 - dy * dy, 0.5 * (0.5 + dy) * (0.5 + dy)};
        const double V[4] = {1e9 * (1.0 + dx), 1e9 * dy, 2e9 * dx * dy, 3e8};
        unsigned long long* p0 = box + cell - SX - 1;
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const double W = wx[ox] * wy[oy];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint64_t q = (uint64_t)__double_as_longlong(__builtin_fma(W, V[c], kMagic));
                    unsigned long long* p = p0 + oy * SX + ox + c * NB;
                    if (MODE == 2) {
                        q = dpp_sum_to_last(q);
                        if (lane == 63) atomicAdd(p, (unsigned long long)q);
                    } else {
                        atomicAdd(p, (unsigned long long)q);
                    }
                }
            }
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = box[SX * 5 + 7];
}

int main() {
    double* dd;
    unsigned long long* o;
    if (hipMalloc(&dd, 4096 * 8) != hipSuccess || hipMalloc(&o, 8192 * 8) != hipSuccess) return 1;
    double h[4096];
    for (int i = 0; i < 4096; ++i) h[i] = ((i * 2654435761u) % 1000) / 1000.0 - 0.5;
    if (hipMemcpy(dd, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return 1;
    for (int rep = 0; rep < 3; ++rep)
        for (int mode = 0; mode < 3; ++mode) {
            printf("probe3 mode %d rep %d\n", mode, rep);
            fflush(stdout);
            if (mode == 0) hipLaunchKernelGGL(k_dep<0>, dim3(8192), dim3(256), 0, 0, dd, o);
            if (mode == 1) hipLaunchKernelGGL(k_dep<1>, dim3(8192), dim3(256), 0, 0, dd, o);
            if (mode == 2) hipLaunchKernelGGL(k_dep<2>, dim3(8192), dim3(256), 0, 0, dd, o);
            if (hipDeviceSynchronize() != hipSuccess) return 1;
        }
    printf("done\n");
    return 0;
}
