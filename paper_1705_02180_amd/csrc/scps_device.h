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
        // one 32 x 32 -> 64-bit product per word gives both halves (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // three-input XORs, one v_bitop3_b32 each (truth table 0x96)
        c[0] = __builtin_amdgcn_bitop3_b32(hi1, c[1], k0, 0x96);
        c[1] = lo1;
        c[2] = __builtin_amdgcn_bitop3_b32(hi0, c[3], k1, 0x96);
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// w = -wscale (a + log s0) rounded as written: the ratchet's w - w_m must be
// exactly 0 when w_m was just set to w, so the product may not be fused into
// that difference (an FMA would leave its rounding error behind).
__device__ __forceinline__ double tube_w(double a, double s0, double wscale) {
#pragma clang fp contract(off)
    const double t = a + log(s0);
    return -t * wscale;
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
// frames of a stack, one wavefront (lane holds frames lane and lane + 64).
// The distances are expanded around a reference frame j of the stack: with
// u_p = C_p - R_jp,
//   d_k Z0 = sum_p (C_p - R_kp)^2 = sum_p u_p^2 + 2 (Y_j - Y_k) + G_jk,
//   Y_k = sum_p u_p R_kp,  G_jk = sum_p (R_jp - R_kp)^2,
// so d_j carries no cancellation at all and the rounding of the Y sums
// scales with the distance to frame j (q = sum u^2, yr = Y, Gj = row j of G).
// Then a = max_k (-lambda d_k), e_k = exp(-lambda d_k - a), s0 = sum_k e_k,
// s1 = sum_k k e_k: s = 1 - (s1 / s0) / (K - 1) and w = -wscale (a + log s0),
// the discrete forms of eqs (asXa), (awXa) with a log-sum-exp shift.  kmax is
// the frame of largest weight (the lowest such k), the reference frame to
// use next.
struct TubeSums {
    double e[2];
    double a, s0, s1;
    int kmax;
};
__device__ __forceinline__ TubeSums tube_sums(int lane, int K, double q, const double *yr, int j, const double *Gj,
                                              double Z0, double lam) {
    TubeSums t;
    double dk[2];
    const double yj = yr[j];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        dk[h] = k < K ? fmax(q + 2.0 * (yj - yr[k]) + Gj[k], 0.0) / Z0 : 0.0;
    }
    double a = -INFINITY;
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (lane + 64 * h < K) a = fmax(a, -lam * dk[h]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, 64));
    double s0 = 0.0, s1 = 0.0;
    int best = K;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        t.e[h] = 0.0;
        if (k < K) {
            const double x = -lam * dk[h] - a;
            if (x == 0.0 && k < best) best = k;
            t.e[h] = exp(x);
            s0 += t.e[h];
            s1 += (double)k * t.e[h];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    t.a = a;
    t.s0 = wave_sum(s0);
    t.s1 = wave_sum(s1);
    t.kmax = best < K ? best : 0;
    return t;
}

// Reference frame of a replica for the distance expansion: the one kept from
// its previous evaluation when it lies in the stack, else frame 0.  The
// distance pass and the tube-variable kernels must take the same one.
__device__ __forceinline__ int ref_frame(const int *jref, int r, int K) {
    const int j = jref ? jref[r] : 0;
    return (j >= 0 && j < K) ? j : 0;
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
