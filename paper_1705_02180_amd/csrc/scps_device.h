// Device helpers shared by the stepping kernels (scps_kernels.hip) and the
// reference-map / SCPS matrix-core kernels (scps_maps.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace scps {

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Lane l receives what lane (l + 1) mod 64 holds (DPP wave_rol:1).  Every
// lane has a valid source, so the "old" operand is never used; passing the
// value itself lets the move happen in place.
__device__ __forceinline__ float rot1(float v) {
    const int u = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(u, u, 0x134, 0xF, 0xF, false));
}

// Squared distance of a pair, and the vector d = x_i - x_j.
__device__ __forceinline__ float pair_r2(const float4 &pi, const float4 &pj, float &dx, float &dy, float &dz) {
    dx = pi.x - pj.x;
    dy = pi.y - pj.y;
    dz = pi.z - pj.z;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds, Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t a = c[0], b = c[2];
        const uint32_t hi0 = __umulhi(0xD2511F53u, a), lo0 = 0xD2511F53u * a;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, b), lo1 = 0xCD9E8D57u * b;
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ float unit_open_f(uint32_t w) {
    return (float)(2u * (w >> 9) + 1u) * 0x1p-24f;
}

// Sum over the 64 lanes of a wavefront, returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Tube variables of one replica from its squared distances to the K <= 128
// frames of a stack, one wavefront (lane holds frames lane and lane + 64):
// d_k = max(Q - 2 X_k + R2_k, 0) / Z0, a = max_k (-lambda d_k),
// e_k = exp(-lambda d_k - a), s0 = sum_k e_k, s1 = sum_k k e_k; then
// s = 1 - (s1 / s0) / (K - 1) and w = -(a + log s0) / lambda, the discrete
// forms of eqs (asXa), (awXa) with a log-sum-exp shift.
struct TubeSums {
    double e[2];
    double a, s0, s1;
};
__device__ __forceinline__ TubeSums tube_sums(int lane, int K, double q, const double *xr, const double *R2,
                                              double Z0, double lam) {
    TubeSums t;
    double dk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        dk[h] = k < K ? fmax(q - 2.0 * xr[k] + R2[k], 0.0) / Z0 : 0.0;
    }
    double a = -INFINITY;
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (lane + 64 * h < K) a = fmax(a, -lam * dk[h]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, 64));
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        t.e[h] = 0.0;
        if (k < K) {
            t.e[h] = exp(-lam * dk[h] - a);
            s0 += t.e[h];
            s1 += (double)k * t.e[h];
        }
    }
    t.a = a;
    t.s0 = wave_sum(s0);
    t.s1 = wave_sum(s1);
    return t;
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
