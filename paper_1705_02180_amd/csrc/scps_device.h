// Device helpers shared by the stepping kernels (scps_kernels.hip) and the
// reference-map / SCPS matrix-core kernels (scps_maps.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace scps {

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Squared distance of a pair, and the vector d = x_i - x_j.
__device__ __forceinline__ float pair_r2(const float4 &pi, const float4 &pj, float &dx, float &dy, float &dz) {
    dx = pi.x - pj.x;
    dy = pi.y - pj.y;
    dz = pi.z - pj.z;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Sum over the 64 lanes of a wavefront, returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Tile pair (I, J), I <= J, of linear index t in row-major order over the
// upper triangle of an nb x nb block grid.
__device__ __forceinline__ void tile_decode(int t, int nb, int &I, int &J) {
    int row = 0;
    while (t >= nb - row) {
        t -= nb - row;
        ++row;
    }
    I = row;
    J = row + t;
}

}  // namespace scps
