// HIP kernels for gfx950: batched rMD / SCPS Langevin stepping.
//
// Pair work is organised in 64x64 tile pairs (I <= J) of a chain's internal
// particle order.  In a tile pass lane l of a wavefront owns particle
// i = 64 I + l and, at sub-step k, meets particle j = 64 J + ((l + k) mod 64),
// read from LDS (persistent kernel) or L1/L2 (per-step kernels).  Every
// unordered pair is met once: k = 0..63 in an off-diagonal tile, and
// k = 1..32 in a diagonal tile with only lanes 0..31 active at k = 32.
// Newton's third law is applied without atomics inside the loop: the j-side
// partial sums live in registers and move one lane down after every
// sub-step (DPP wavefront rotate), so that lane l always holds the partial
// of the particle it meets next.  Pair arithmetic is float32; every tile's
// partial sums (at most 64 terms) are added into float64 accumulators.
//
// Contact function, eq (Cij) of Orioli, a Beccara, Faccioli (arXiv:1705.02180),
// with q = (r/r0)^2:
//   C(q)  = (1 + q + q^2) / (1 + q + q^2 + q^3 + q^4)
//   C'(q) = -q^2 (3 + 6q + 4q^2 + 2q^3) / (1 + q + q^2 + q^3 + q^4)^2
// (the numerator of the quotient rule expanded, so no cancellation at small q).
// z = sum over contact pairs of (C - R)^2, eq (zrMD); dz/dx_i = sum_j
// (4/r0^2) (C - R) C'(q) (x_i - x_j).
#include <math.h>

#include "scps_internal.h"

#ifndef SCPS_PAIR_GROUP
#define SCPS_PAIR_GROUP 4
#endif
#ifndef SCPS_PAIR_GROUP2
#define SCPS_PAIR_GROUP2 2
#endif

namespace scps {

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
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

// Reference maps live in global memory; telling the compiler so lets it use
// global loads with a scalar base instead of flat loads.
typedef const float __attribute__((address_space(1))) gfloat;
__device__ __forceinline__ float ldg(const float *p, int64_t i) {
    return ((gfloat *)p)[i];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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

// Three standard normals for (particle, replica, step).  The uniforms are odd
// multiples of 2^-24, exact in float32; Box-Muller runs in float32 (logf,
// sqrtf, sincospif: within a few ulp of the float64 transform).
__device__ __forceinline__ void normals3(const KParams &P, uint32_t atom, uint32_t rep, uint64_t step,
                                         double &g0, double &g1, double &g2) {
    uint32_t c[4] = {atom, rep, (uint32_t)step, (uint32_t)(step >> 32)};
    philox4x32_10(c, P.seed_lo, P.seed_hi);
    const float r01 = sqrtf(-2.f * logf(unit_open_f(c[0])));
    const float r23 = sqrtf(-2.f * logf(unit_open_f(c[2])));
    float sn, cs;
    sincospif(2.f * unit_open_f(c[1]), &sn, &cs);
    g0 = (double)(r01 * cs);
    g1 = (double)(r01 * sn);
    sincospif(2.f * unit_open_f(c[3]), &sn, &cs);
    g2 = (double)(r23 * cs);
}

// ---------------------------------------------------------------------------
// the pair tile pass
// ---------------------------------------------------------------------------
// PM_SCPS: the SCPS bias (contact gradient against each replica's effective
// reference E) plus the nonbonded forces.
enum { PM_RMD = 0, PM_Z = 1, PM_ZG = 2, PM_SCPS = 3 };

template <int MODE> struct ModeTraits {
    static constexpr bool nb = (MODE == PM_RMD || MODE == PM_SCPS);
    static constexpr bool grad = (MODE == PM_RMD || MODE == PM_ZG || MODE == PM_SCPS);
    static constexpr bool z = (MODE == PM_RMD || MODE == PM_Z || MODE == PM_ZG);
};

// Lane-side state of a tile pass.
struct LaneI {
    float4 p;     // x, y, z, charge of particle i
    float qp;     // k_e/eps_r * charge of i
    int o;        // chain index of i
    bool valid;   // i < n
    bool contact; // i in the contact set
};

// Squared distance of a pair, and the vector d = x_i - x_j.
__device__ __forceinline__ float pair_r2(const float4 &pi, const float4 &pj, float &dx, float &dy, float &dz) {
    dx = pi.x - pj.x;
    dy = pi.y - pj.y;
    dz = pi.z - pj.z;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Nonbonded scalar f with F_i += f (x_i - x_j):
// f = [24 eps (2 s^12 - s^6) + k_e/eps_r q_i q_j e^{-kappa r} (kappa + 1/r)] / r^2, s = sigma / r,
// the Lennard-Jones part evaluated as r^-6 (A r^-6 - B), A = 48 eps sigma^12, B = 24 eps sigma^6.
// qp_i = k_e/eps_r * q_i.  NBK bit 0: Lennard-Jones, bit 1: Debye-Hueckel.
template <int NBK>
__device__ __forceinline__ float nb_scalar(const KParams &P, const float r2, const float qp_i, const float q_j) {
    if constexpr (NBK == 1) {
        const float inv_r2 = frcp(r2);
        const float inv_r6 = inv_r2 * inv_r2 * inv_r2;
        return fmaf(inv_r6, P.lj_A, -P.lj_B) * inv_r6 * inv_r2;
    } else if constexpr (NBK == 0) {
        return 0.f;
    } else {
        const float inv_r = frsq(r2);
        const float inv_r2 = inv_r * inv_r;
        const float r = r2 * inv_r;
        const float e = fexp2(P.dh_kl2 * r) * (qp_i * q_j);
        float S = e * (P.dh_kappa + inv_r);
        if constexpr (NBK == 3) {
            const float inv_r6 = inv_r2 * inv_r2 * inv_r2;
            S = fmaf(fmaf(inv_r6, P.lj_A, -P.lj_B), inv_r6, S);
        }
        return S * inv_r2;
    }
}

// One sub-step k of a tile pass: lane l meets particle j = 64 J + ((l + k) mod 64).
// posj2 points at block J stored twice in a row, so posj2[l + k] needs no wrap.
// Padding particles sit far away with zero charge, so their nonbonded and
// contact terms vanish without a mask.  MASK tiles (host-computed flag) hold
// a pair excluded from the nonbonded sum (chain neighbours) or need the
// contact predicate (a block that straddles the end of the contact set, a
// sequence separation, a cutoff); every other tile runs predicate-free.
// act0 is false only for lanes 32..63 at k = 32 of a diagonal tile, where the
// pair was already met at the mirrored sub-step.  rv[u] is the lane's
// reference value at sub-step k0 + u (the native map, or in PM_SCPS the
// replica's effective reference E = sum_k c_k R_k, against which the
// difference is csum C - E).
template <int MODE, bool DIAG, bool CONTACT, bool MASK, int NBK, int U>
__device__ __forceinline__ void pair_group(const KParams &P, const int lane, const int k0, const bool low,
                                           const LaneI &A, const float4 *__restrict__ posj2,
                                           const int *__restrict__ orgj, const int ncj, const float *rv,
                                           const float csum, float fi[6], float fj[6], float &zt) {
    // Sub-steps k0 .. k0+U-1, computed phase by phase so that the U pair
    // evaluations are independent instruction streams; only the
    // accumulation (and the rotation of the j-side partials) is sequential.
    using T = ModeTraits<MODE>;
    float dx[U], dy[U], dz[U], r2[U], f[U], g[U];
    bool nbon[U], con[U], inside[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + u;
        const float4 pj = posj2[lane + k];
        r2[u] = pair_r2(A.p, pj, dx[u], dy[u], dz[u]);
        const bool act0 = DIAG ? (low | (k != 32)) : true;
        nbon[u] = act0;
        con[u] = act0;
        inside[u] = true;
        if constexpr (MASK) {
            const int jl = (lane + k) & 63;
            const int sep = abs(A.o - orgj[jl]);
            nbon[u] = act0 & (sep > P.nb_excl);
            con[u] = act0 & A.contact & (jl < ncj) & (sep > P.min_sep);
            inside[u] = !P.has_cut | (r2[u] <= P.r_cut2);   // beyond a cutoff C_ij = 0 (R_ij still counts)
        }
        f[u] = 0.f;
        if constexpr (T::nb && NBK != 0) {
            const float fs = nb_scalar<NBK>(P, r2[u], A.qp, pj.w);
            f[u] = nbon[u] ? fs : 0.f;
        }
    }
    if constexpr (CONTACT) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float q = r2[u] * P.inv_r0sq;
            const float q2 = q * q;
            const float num = 1.f + q + q2;
            const float den = fmaf(q2, q + q2, num);
            const float inv_den = inside[u] ? frcp(den) : 0.f;
            const float C = num * inv_den;
            g[u] = 0.f;
            float diff;
            if constexpr (MODE == PM_SCPS)
                diff = fmaf(csum, C, -rv[u]);
            else
                diff = C - rv[u];
            diff = con[u] ? diff : 0.f;
            if constexpr (T::z) zt = fmaf(diff, diff, zt);
            if constexpr (T::grad) {
                // C'(q) = -q^2 (3 + 6q + 4q^2 + 2q^3) / den^2, evaluated as
                // (q^2/den) (poly/den) so nothing overflows at large q;
                // g = (4/r0^2) (C - R) C'(q), the factor -4/r0^2 folded into poly
                const float poly = fmaf(q, fmaf(q, fmaf(q, P.cp[0], P.cp[1]), P.cp[2]), P.cp[3]);
                g[u] = (diff * (q2 * inv_den)) * (poly * inv_den);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if constexpr (T::nb && NBK != 0) {
            fi[0] = fmaf(f[u], dx[u], fi[0]);
            fi[1] = fmaf(f[u], dy[u], fi[1]);
            fi[2] = fmaf(f[u], dz[u], fi[2]);
            fj[0] = rot1(fmaf(-f[u], dx[u], fj[0]));
            fj[1] = rot1(fmaf(-f[u], dy[u], fj[1]));
            fj[2] = rot1(fmaf(-f[u], dz[u], fj[2]));
        }
        if constexpr (T::grad && CONTACT) {
            fi[3] = fmaf(g[u], dx[u], fi[3]);
            fi[4] = fmaf(g[u], dy[u], fi[4]);
            fi[5] = fmaf(g[u], dz[u], fi[5]);
            fj[3] = rot1(fmaf(-g[u], dx[u], fj[3]));
            fj[4] = rot1(fmaf(-g[u], dy[u], fj[4]));
            fj[5] = rot1(fmaf(-g[u], dz[u], fj[5]));
        }
    }
}

// Two off-diagonal tiles (I1, J) and (I2, J) in one pass: lane l holds
// particle l of blocks I1 (A) and I2 (B); at sub-step k both meet the same j,
// so their j-side terms share one register and one rotation, and the j
// position is read once.  Sub-steps k0 .. k0+U-1.
template <int MODE, bool CONTACT, bool MASK, int NBK, int U>
__device__ __forceinline__ void pair_group2(const KParams &P, const int lane, const int k0, const LaneI &A,
                                            const LaneI &B, const float4 *__restrict__ posj2,
                                            const int *__restrict__ orgj, const int ncj,
                                            const float *__restrict__ rtA, const float *__restrict__ rtB,
                                            float fa[6], float fb[6], float fj[6], float &zt) {
    using T = ModeTraits<MODE>;
    static_assert(MODE != PM_SCPS, "double tiles are for the rMD and z modes");
    float dxa[U], dya[U], dza[U], fA[U], gA[U];
    float dxb[U], dyb[U], dzb[U], fB[U], gB[U];
    float r2a[U], r2b[U];
    bool nba[U], nbb[U], ca[U], cb[U], ina[U], inb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = k0 + u;
        const float4 pj = posj2[lane + k];
        r2a[u] = pair_r2(A.p, pj, dxa[u], dya[u], dza[u]);
        r2b[u] = pair_r2(B.p, pj, dxb[u], dyb[u], dzb[u]);
        nba[u] = nbb[u] = ca[u] = cb[u] = ina[u] = inb[u] = true;
        if constexpr (MASK) {
            const int jl = (lane + k) & 63;
            const int oj = orgj[jl];
            const int sa = abs(A.o - oj), sb = abs(B.o - oj);
            nba[u] = sa > P.nb_excl;
            nbb[u] = sb > P.nb_excl;
            ca[u] = A.contact & (jl < ncj) & (sa > P.min_sep);
            cb[u] = B.contact & (jl < ncj) & (sb > P.min_sep);
            ina[u] = !P.has_cut | (r2a[u] <= P.r_cut2);
            inb[u] = !P.has_cut | (r2b[u] <= P.r_cut2);
        }
        fA[u] = fB[u] = 0.f;
        if constexpr (T::nb && NBK != 0) {
            const float xa = nb_scalar<NBK>(P, r2a[u], A.qp, pj.w);
            const float xb = nb_scalar<NBK>(P, r2b[u], B.qp, pj.w);
            fA[u] = nba[u] ? xa : 0.f;
            fB[u] = nbb[u] ? xb : 0.f;
        }
    }
    if constexpr (CONTACT) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float r2 = h ? r2b[u] : r2a[u];
                const float q = r2 * P.inv_r0sq;
                const float q2 = q * q;
                const float num = 1.f + q + q2;
                const float den = fmaf(q2, q + q2, num);
                const float inv_den = (h ? inb[u] : ina[u]) ? frcp(den) : 0.f;
                float diff = num * inv_den - ldg(h ? rtB : rtA, k * 64 + lane);
                diff = (h ? cb[u] : ca[u]) ? diff : 0.f;
                if constexpr (T::z) zt = fmaf(diff, diff, zt);
                if constexpr (T::grad) {
                    const float poly = fmaf(q, fmaf(q, fmaf(q, P.cp[0], P.cp[1]), P.cp[2]), P.cp[3]);
                    const float g = (diff * (q2 * inv_den)) * (poly * inv_den);
                    if (h) gB[u] = g; else gA[u] = g;
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if constexpr (T::nb && NBK != 0) {
            fa[0] = fmaf(fA[u], dxa[u], fa[0]);
            fa[1] = fmaf(fA[u], dya[u], fa[1]);
            fa[2] = fmaf(fA[u], dza[u], fa[2]);
            fb[0] = fmaf(fB[u], dxb[u], fb[0]);
            fb[1] = fmaf(fB[u], dyb[u], fb[1]);
            fb[2] = fmaf(fB[u], dzb[u], fb[2]);
            fj[0] = rot1(fmaf(-fB[u], dxb[u], fmaf(-fA[u], dxa[u], fj[0])));
            fj[1] = rot1(fmaf(-fB[u], dyb[u], fmaf(-fA[u], dya[u], fj[1])));
            fj[2] = rot1(fmaf(-fB[u], dzb[u], fmaf(-fA[u], dza[u], fj[2])));
        }
        if constexpr (T::grad && CONTACT) {
            fa[3] = fmaf(gA[u], dxa[u], fa[3]);
            fa[4] = fmaf(gA[u], dya[u], fa[4]);
            fa[5] = fmaf(gA[u], dza[u], fa[5]);
            fb[3] = fmaf(gB[u], dxb[u], fb[3]);
            fb[4] = fmaf(gB[u], dyb[u], fb[4]);
            fb[5] = fmaf(gB[u], dzb[u], fb[5]);
            fj[3] = rot1(fmaf(-gB[u], dxb[u], fmaf(-gA[u], dxa[u], fj[3])));
            fj[4] = rot1(fmaf(-gB[u], dyb[u], fmaf(-gA[u], dya[u], fj[4])));
            fj[5] = rot1(fmaf(-gB[u], dzb[u], fmaf(-gA[u], dza[u], fj[5])));
        }
    }
}

// MASK tiles evaluate the per-pair predicates only on the sub-step groups
// whose bits are set in mk (bit k: some pair met at sub-step k needs one).
template <int MODE, bool CONTACT, bool MASK, int NBK>
__device__ __forceinline__ void tile_pass2(const KParams &P, const int lane, const int kb, const int ke,
                                           const uint64_t mk, const LaneI &A, const LaneI &B,
                                           const float4 *__restrict__ posj2, const int *__restrict__ orgj,
                                           const int ncj, const float *__restrict__ rtA,
                                           const float *__restrict__ rtB, float fa[6], float fb[6], float fj[6],
                                           float &zt) {
    constexpr int U = SCPS_PAIR_GROUP2;
    constexpr uint64_t GB = (1ull << U) - 1;
#pragma unroll 1
    for (int k0 = kb; k0 < ke; k0 += U) {
        if (MASK && ((mk >> k0) & GB))
            pair_group2<MODE, CONTACT, true, NBK, U>(P, lane, k0, A, B, posj2, orgj, ncj, rtA, rtB, fa, fb, fj, zt);
        else
            pair_group2<MODE, CONTACT, false, NBK, U>(P, lane, k0, A, B, posj2, orgj, ncj, rtA, rtB, fa, fb, fj, zt);
    }
}

template <int MODE, int NBK>
__device__ __forceinline__ void tile_dispatch2(const int flags, const int kb, const int ke, const uint64_t mk,
                                               const KParams &P, const int lane, const LaneI &A, const LaneI &B,
                                               const float4 *__restrict__ posj2, const int *__restrict__ orgj,
                                               const int ncj, const float *__restrict__ rtA,
                                               const float *__restrict__ rtB, float fa[6], float fb[6], float fj[6],
                                               float &zt) {
#define SCPS_TILE2(C, M)                                                                                     \
    tile_pass2<MODE, C, M, NBK>(P, lane, kb, ke, mk, A, B, posj2, orgj, ncj, rtA, rtB, fa, fb, fj, zt)
    const bool con = flags & TILE_CONTACT, mask = flags & TILE_MASK;
    if (con) { if (mask) SCPS_TILE2(true, true); else SCPS_TILE2(true, false); }
    else     { if (mask) SCPS_TILE2(false, true); else SCPS_TILE2(false, false); }
#undef SCPS_TILE2
}

// A whole tile pair, or a segment of one: sub-steps kb .. ke-1, a multiple of
// D (every caller uses 32 or 64), evaluated SCPS_PAIR_GROUP at a time; a
// MASK tile evaluates the per-pair predicates only on the groups whose
// sub-step bits are set in mk.  The
// lane's reference values are loaded D sub-steps ahead of their use into a
// ring of registers: D = 4 groups in the per-step kernels, whose maps stream
// from HBM, one group where the map is cache-resident (persistent kernel).
// Outputs: fi[0..2] nonbonded, fi[3..5] contact gradient (i side); fj
// likewise for the j particle lane l holds at the end (see jflush_at); zt:
// this lane's z partial.
template <int MODE, bool DIAG, bool CONTACT, bool MASK, int NBK, int D>
__device__ __forceinline__ void tile_pass(const KParams &P, const int lane, const int kb, const int ke,
                                          const uint64_t mk, const LaneI &A, const float4 *__restrict__ posj2,
                                          const int *__restrict__ orgj, const int ncj, const float *__restrict__ rt,
                                          const float csum, float fi[6], float fj[6], float &zt) {
    constexpr int U = SCPS_PAIR_GROUP;
    static_assert(D % U == 0, "prefetch depth is whole groups");
    const bool low = lane < 32;
    float ring[D];
    if constexpr (CONTACT) {
#pragma unroll
        for (int d = 0; d < D; ++d) ring[d] = ldg(rt, (kb + d) * 64 + lane);
    }
#pragma unroll 1
    for (int k0 = kb; k0 < ke; k0 += D) {
#pragma unroll
        for (int g = 0; g < D / U; ++g) {
            float rv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) rv[u] = CONTACT ? ring[g * U + u] : 0.f;
            if constexpr (CONTACT) {
                const int kn = k0 + D + g * U;
                if (kn < ke) {
#pragma unroll
                    for (int u = 0; u < U; ++u) ring[g * U + u] = ldg(rt, (kn + u) * 64 + lane);
                }
            }
            if (MASK && ((mk >> (k0 + g * U)) & ((1ull << U) - 1)))
                pair_group<MODE, DIAG, CONTACT, true, NBK, U>(P, lane, k0 + g * U, low, A, posj2, orgj, ncj, rv,
                                                              csum, fi, fj, zt);
            else
                pair_group<MODE, DIAG, CONTACT, false, NBK, U>(P, lane, k0 + g * U, low, A, posj2, orgj, ncj, rv,
                                                               csum, fi, fj, zt);
        }
    }
}

// Sub-step range of a whole tile: 1..32 on a diagonal tile (lanes 0..31 only
// at k = 32), 0..63 otherwise.
__device__ __forceinline__ int tile_kbeg(bool diag) { return diag ? 1 : 0; }
__device__ __forceinline__ int tile_kend(bool diag) { return diag ? 33 : 64; }

// After sub-steps kb .. ke-1 the j-side partials have rotated ke - kb times:
// lane l holds particle (l + ke) mod 64 of block J.
__device__ __forceinline__ int jflush_at(int lane, int ke) { return (lane + ke) & 63; }

// Dispatch on the tile's flags (uniform across the wavefront).
enum { TF_DIAG = TILE_DIAG, TF_CONTACT = TILE_CONTACT, TF_MASK = TILE_MASK };

template <int MODE, int NBK, int D>
__device__ __forceinline__ void tile_dispatch(const int flags, const int kb, const int ke, const uint64_t mk,
                                              const KParams &P,
                                              const int lane, const LaneI &A,
                                              const float4 *__restrict__ posj2, const int *__restrict__ orgj,
                                              const int ncj, const float *__restrict__ rt, const float csum,
                                              float fi[6], float fj[6], float &zt) {
#define SCPS_TILE(DG, C, M)                                                                                 \
    tile_pass<MODE, DG, C, M, NBK, D>(P, lane, kb, ke, mk, A, posj2, orgj, ncj, rt, csum, fi, fj, zt)
    const bool diag = flags & TF_DIAG, con = flags & TF_CONTACT, mask = flags & TF_MASK;
    if (ModeTraits<MODE>::nb) {
        if (diag) {
            if (con) { if (mask) SCPS_TILE(true, true, true); else SCPS_TILE(true, true, false); }
            else     { if (mask) SCPS_TILE(true, false, true); else SCPS_TILE(true, false, false); }
        } else {
            if (con) { if (mask) SCPS_TILE(false, true, true); else SCPS_TILE(false, true, false); }
            else     { if (mask) SCPS_TILE(false, false, true); else SCPS_TILE(false, false, false); }
        }
    } else if (con) {
        if (diag) { if (mask) SCPS_TILE(true, true, true); else SCPS_TILE(true, true, false); }
        else      { if (mask) SCPS_TILE(false, true, true); else SCPS_TILE(false, true, false); }
    }
#undef SCPS_TILE
}


// Padding particle a: uncharged, 1e6 A away from the chain and 1e3 A from
// every other pad, so its Lennard-Jones, Debye-Hueckel and contact terms are
// zero in float32 (the contact denominator overflows to inf, C = C' = 0).
__device__ __forceinline__ float4 pad_position(int a) {
    return make_float4(1.0e6f + 1.0e3f * (float)(a & 7), 1.0e3f * (float)((a >> 3) & 7), 1.0e3f * (float)(a >> 6),
                       0.f);
}

// Index of internal particle a in a position array that stores every block of
// 64 twice in a row (block b occupies [128 b, 128 b + 128)).
__device__ __forceinline__ int dup_index(int a) { return ((a >> 6) << 7) + (a & 63); }

// Harmonic bond between internal particle a and its chain successor b, float64.
__device__ __forceinline__ void bond_force(const KParams &P, float4 pa, float4 pb, double f[3]) {
    const double dx = (double)pa.x - (double)pb.x;
    const double dy = (double)pa.y - (double)pb.y;
    const double dz = (double)pa.z - (double)pb.z;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double s = -P.k_bond * (r - P.r_bond) / r;
    f[0] = s * dx;
    f[1] = s * dy;
    f[2] = s * dz;
}

// ---------------------------------------------------------------------------
// persistent rMD kernel: one workgroup runs one replica for all n_steps
// ---------------------------------------------------------------------------
// LDS per padded particle: positions twice (2 x float4), chain index (int),
// six float64 accumulators, velocity (3 x float).
// Plus a reduction slot per wavefront.
constexpr size_t PERSIST_BYTES_PER_PARTICLE = 32 + 4 + 48 + 12;

static size_t persistent_fixed_bytes(int wg) {
    return (size_t)(wg / 64) * 8 + 64;
}

size_t persistent_lds_bytes(int n_pad, int wg) {
    return (size_t)n_pad * PERSIST_BYTES_PER_PARTICLE + persistent_fixed_bytes(wg);
}

int persistent_max_npad(int wg) {
    const size_t lds = 160 * 1024;
    int n = (int)((lds - persistent_fixed_bytes(wg)) / PERSIST_BYTES_PER_PARTICLE);
    return (n / 64) * 64;
}

__device__ __forceinline__ void tile_decode(int t, int nb, int &I, int &J) {
    int row = 0;
    while (t >= nb - row) {
        t -= nb - row;
        ++row;
    }
    I = row;
    J = row + t;
}

// One workgroup per replica is resident per CU in the benchmark shapes, so
// the register budget is WG/64/4 waves per SIMD: let the scheduler use it for
// latency hiding instead of aiming for a higher occupancy it cannot reach.
template <int WG, int NBK>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WG / 256 > 0 ? WG / 256 : 1, WG / 256 > 0 ? WG / 256 : 1))) void k_rmd_persistent(
    const KParams P, const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
    const int *__restrict__ order, float *__restrict__ x, float *__restrict__ v,
    double *__restrict__ cv, const int64_t n_steps, const uint64_t step0, const int record_every,
    float *__restrict__ frames, const int64_t frame_stride, int *__restrict__ flags) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NW = WG / 64;
    const int r = order[blockIdx.x];
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    const int n = S.n, n_pad = S.n_pad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    float4 *pos = reinterpret_cast<float4 *>(smem);                   // [2 n_pad], blocks twice
    double *acc = reinterpret_cast<double *>(pos + 2 * n_pad);        // [6][n_pad]
    float *vel = reinterpret_cast<float *>(acc + 6 * (size_t)n_pad);  // [3][n_pad]
    int *org = reinterpret_cast<int *>(vel + 3 * (size_t)n_pad);      // [n_pad]
    double *red = reinterpret_cast<double *>(org + n_pad);            // [NW]
    __shared__ double sh_scale;
    __shared__ int sh_next;   // dynamic tile queue

    float *xr = x + 3 * rd.off;
    float *vr = v ? v + 3 * rd.off : nullptr;
    for (int a = tid; a < n_pad; a += WG) {
        const int o = S.perm[a];
        float4 p;
        if (a < n) {
            p = make_float4(xr[o], xr[n + o], xr[2 * n + o], S.charge[a]);
            vel[a] = vr ? vr[o] : 0.f;
            vel[n_pad + a] = vr ? vr[n + o] : 0.f;
            vel[2 * n_pad + a] = vr ? vr[2 * n + o] : 0.f;
        } else {
            p = pad_position(a);
            vel[a] = vel[n_pad + a] = vel[2 * n_pad + a] = 0.f;
        }
        pos[dup_index(a)] = p;
        pos[dup_index(a) + 64] = p;
        org[a] = o;
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c * n_pad + a] = 0.0;
    }
    if (tid == 0) sh_next = NW;
    double zm = cv[(int64_t)r * CV_STRIDE + CV_ZM];
    double z_last = cv[(int64_t)r * CV_STRIDE + CV_Z];
    double eb_last = cv[(int64_t)r * CV_STRIDE + CV_EB];
    double tsum = 0.0;   // this thread's share of sum over steps, particles of |F_bias|^2 / m
    bool bad = false;
    __syncthreads();

    const int ntile = S.ntile;
    const double c1 = P.c1;
    for (int64_t m = 0;; ++m) {
        if (record_every > 0 && frames && (m % record_every) == 0) {
            float *fr = frames + (m / record_every) * frame_stride + 3 * rd.off;
            for (int a = tid; a < n; a += WG) {
                const int o = org[a];
                const float4 p = pos[dup_index(a)];
                fr[o] = p.x;
                fr[n + o] = p.y;
                fr[2 * n + o] = p.z;
            }
        }
        if (m == n_steps) break;

        // ---- pair phase: nonbonded + contact z and grad z, bonds ----------
        double zacc = 0.0;
        // tiles are sorted costliest first; wavefront w starts with tile w and
        // then takes the next unclaimed one
        for (int t = wave; t < ntile;) {
            const int2 td = S.tiles[t];
            const int I = td.x >> 16, J = td.x & 0xFFFF, tf = td.y & 0xFF, I2 = ((td.y >> 8) & 0xFF) - 1;
            const int kb = (td.y >> 16) & 0x7F, ke = (td.y >> 23) & 0x7F;
            const uint64_t mk = S.tmask[t];
            if (I2 >= 0) {
                // two off-diagonal tiles (I, J) and (I2, J) of the same class
                LaneI A, B;
                A.p = pos[I * 128 + lane];
                B.p = pos[I2 * 128 + lane];
                A.qp = P.dh_pref * A.p.w;
                B.qp = P.dh_pref * B.p.w;
                A.o = org[I * 64 + lane];
                B.o = org[I2 * 64 + lane];
                A.valid = I * 64 + lane < n;
                B.valid = I2 * 64 + lane < n;
                A.contact = I * 64 + lane < S.nc;
                B.contact = I2 * 64 + lane < S.nc;
                float fa[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float fb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float fj[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float zt = 0.f;
                const bool con = tf & TF_CONTACT;
                const float *rtA = con ? S.ref + (int64_t)tile_index(I, J, S.ncb) * 4096 : nullptr;
                const float *rtB = con ? S.ref + (int64_t)tile_index(I2, J, S.ncb) * 4096 : nullptr;
                int nxt = 0;
                if (lane == 0) nxt = atomicAdd(&sh_next, 1);
                tile_dispatch2<PM_RMD, NBK>(tf, kb, ke, mk, P, lane, A, B, pos + J * 128, org + J * 64, S.nc - J * 64,
                                            rtA, rtB, fa, fb, fj, zt);
                zacc += (double)zt;
                const int ncomp = con ? 6 : 3;
                const int jo = J * 64 + jflush_at(lane, ke);
                for (int c = 0; c < ncomp; ++c) {
                    unsafeAtomicAdd(&acc[c * n_pad + I * 64 + lane], (double)fa[c]);
                    unsafeAtomicAdd(&acc[c * n_pad + I2 * 64 + lane], (double)fb[c]);
                    unsafeAtomicAdd(&acc[c * n_pad + jo], (double)fj[c]);
                }
                t = __builtin_amdgcn_readfirstlane(nxt);
                continue;
            }
            LaneI A;
            const int i = I * 64 + lane;
            A.p = pos[I * 128 + lane];
            A.qp = P.dh_pref * A.p.w;
            A.o = org[i];
            A.valid = i < n;
            A.contact = i < S.nc;
            float fi[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float fj[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float zt = 0.f;
            const float *rt = (tf & TF_CONTACT) ? S.ref + (int64_t)tile_index(I, J, S.ncb) * 4096 : nullptr;
            int nxt = 0;
            if (lane == 0) nxt = atomicAdd(&sh_next, 1);
            tile_dispatch<PM_RMD, NBK, SCPS_PAIR_GROUP>(tf, kb, ke, mk, P, lane, A, pos + J * 128, org + J * 64,
                                                        S.nc - J * 64, rt, 0.f, fi, fj, zt);
            zacc += (double)zt;
            const int jo = J * 64 + jflush_at(lane, ke);
            const int ncomp = (tf & TF_CONTACT) ? 6 : 3;
            for (int c = 0; c < ncomp; ++c) {
                unsafeAtomicAdd(&acc[c * n_pad + i], (double)fi[c]);
                unsafeAtomicAdd(&acc[c * n_pad + jo], (double)fj[c]);
            }
            t = __builtin_amdgcn_readfirstlane(nxt);
        }
        for (int a = tid; a < n && P.has_bond; a += WG) {
            const int b = S.bond_next[a];
            if (b >= 0) {
                double f[3];
                bond_force(P, pos[dup_index(a)], pos[dup_index(b)], f);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unsafeAtomicAdd(&acc[c * n_pad + a], f[c]);
                    unsafeAtomicAdd(&acc[c * n_pad + b], -f[c]);
                }
            }
        }
        zacc = wave_sum(zacc);
        if (lane == 0) red[wave] = zacc;
        __syncthreads();

        // ---- ratchet, eq (FrMD): z_m updated before the force is used -----
        if (tid == 0) {
            sh_next = NW;
            double z = 0.0;
            for (int w = 0; w < NW; ++w) z += red[w];
            zm = fmin(zm, z);
            const double dzr = z - zm;
            sh_scale = -P.k_R * dzr;
            z_last = z;
            eb_last = 0.5 * P.k_R * dzr * dzr;
        }
        __syncthreads();
        const double scale = sh_scale;

        // ---- Langevin update, float64 per particle -------------------------
        const uint64_t step = step0 + (uint64_t)m;
        for (int a = tid; a < n; a += WG) {
            const double inv_m = 1.0 / (double)S.mass[a];
            double F[3], fb2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double fb = scale * acc[(c + 3) * n_pad + a];
                F[c] = acc[c * n_pad + a] + fb;
                fb2 = fma(fb, fb, fb2);
                acc[c * n_pad + a] = 0.0;
                acc[(c + 3) * n_pad + a] = 0.0;
            }
            tsum = fma(fb2, inv_m, tsum);
            double g[3];
            normals3(P, (uint32_t)org[a], P.rep_base + (uint32_t)r, step, g[0], g[1], g[2]);
            const int da = dup_index(a);
            const float4 p = pos[da];
            double X[3] = {(double)p.x, (double)p.y, (double)p.z};
            if (P.integrator == 0) {
                const double mob = P.dt * inv_m / P.gamma;
                const double amp = sqrt(2.0 * P.kT * mob);
#pragma unroll
                for (int c = 0; c < 3; ++c) X[c] += mob * F[c] + amp * g[c];
            } else {
                const double amp = sqrt((1.0 - c1 * c1) * P.kT * inv_m);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double u = (double)vel[c * n_pad + a] + P.dt * F[c] * inv_m;
                    X[c] += 0.5 * P.dt * u;
                    u = c1 * u + amp * g[c];
                    X[c] += 0.5 * P.dt * u;
                    vel[c * n_pad + a] = (float)u;
                }
            }
            const float4 np = make_float4((float)X[0], (float)X[1], (float)X[2], p.w);
            bad |= !(isfinite(np.x) && isfinite(np.y) && isfinite(np.z));
            pos[da] = np;
            pos[da + 64] = np;
        }
        __syncthreads();
    }

    for (int a = tid; a < n; a += WG) {
        const int o = org[a];
        const float4 p = pos[dup_index(a)];
        xr[o] = p.x;
        xr[n + o] = p.y;
        xr[2 * n + o] = p.z;
        if (vr) {
            vr[o] = vel[a];
            vr[n + o] = vel[n_pad + a];
            vr[2 * n + o] = vel[2 * n_pad + a];
        }
    }
    if (bad) flags[r] = 1;
    // bias functional: T += dt sum_steps sum_i |F_bias,i|^2 / (m_i gamma)
    tsum = wave_sum(tsum);
    if (lane == 0) red[wave] = tsum;
    __syncthreads();
    if (tid == 0 && n_steps > 0) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += red[w];
        cv[(int64_t)r * CV_STRIDE + CV_Z] = z_last;
        cv[(int64_t)r * CV_STRIDE + CV_ZM] = zm;
        cv[(int64_t)r * CV_STRIDE + CV_EB] = eb_last;
        cv[(int64_t)r * CV_STRIDE + CV_T] += P.dt / P.gamma * t;
    }
}

template <int WG>
static void launch_persistent_wg(int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps,
                                 const int *order, int R, size_t lds, float *x, float *v, double *cv,
                                 int64_t n_steps, uint64_t step0, int record_every, float *frames,
                                 int64_t frame_stride, int *flags, hipStream_t st) {
#define SCPS_LAUNCH(K)                                                                                      \
    hipLaunchKernelGGL((k_rmd_persistent<WG, K>), dim3(R), dim3(WG), lds, st, P, sysd, reps, order, x, v, cv, \
                       n_steps, step0, record_every, frames, frame_stride, flags)
    switch (nbk) {
    case 0: SCPS_LAUNCH(0); break;
    case 1: SCPS_LAUNCH(1); break;
    case 2: SCPS_LAUNCH(2); break;
    default: SCPS_LAUNCH(3); break;
    }
#undef SCPS_LAUNCH
}

hipError_t launch_persistent_rmd(int wg, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps,
                                 const int *order, int R, int n_pad_max, float *x, float *v,
                                 double *cv, int64_t n_steps, uint64_t step0, int record_every,
                                 float *frames, int64_t frame_stride, int *flags, hipStream_t st) {
    const size_t lds = persistent_lds_bytes(n_pad_max, wg);
    switch (wg) {
    case 256:
        launch_persistent_wg<256>(nbk, P, sysd, reps, order, R, lds, x, v, cv, n_steps, step0, record_every,
                                  frames, frame_stride, flags, st);
        break;
    case 512:
        launch_persistent_wg<512>(nbk, P, sysd, reps, order, R, lds, x, v, cv, n_steps, step0, record_every,
                                  frames, frame_stride, flags, st);
        break;
    case 1024:
        launch_persistent_wg<1024>(nbk, P, sysd, reps, order, R, lds, x, v, cv, n_steps, step0, record_every,
                                   frames, frame_stride, flags, st);
        break;
    default:
        launch_persistent_wg<64>(nbk, P, sysd, reps, order, R, lds, x, v, cv, n_steps, step0, record_every,
                                 frames, frame_stride, flags, st);
        break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-step path: gather / pairs / finalize / integrate / scatter
// Positions live in xs as float4 (x, y, z, charge), internal order, every
// block of 64 stored twice (replica r at 2 poff_r); velocities in vs
// (float4, single copy, at poff_r).
// ---------------------------------------------------------------------------
__global__ void k_gather(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                         const float *__restrict__ x, const float *__restrict__ v, float4 *__restrict__ xs,
                         float4 *__restrict__ vs) {
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n_pad) return;
    const int n = S.n;
    const float *xr = x + 3 * rd.off;
    float4 p, q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a < n) {
        const int o = S.perm[a];
        p = make_float4(xr[o], xr[n + o], xr[2 * n + o], S.charge[a]);
        if (v) {
            const float *vr = v + 3 * rd.off;
            q = make_float4(vr[o], vr[n + o], vr[2 * n + o], 0.f);
        }
    } else {
        p = pad_position(a);
    }
    float4 *xr2 = xs + 2 * rd.poff;
    xr2[dup_index(a)] = p;
    xr2[dup_index(a) + 64] = p;
    if (vs) vs[rd.poff + a] = q;
}

hipError_t launch_gather(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, const float *x,
                         const float *v, float4 *xs, float4 *vs, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3((n_pad_max + 255) / 256, R), dim3(256), 0, st, sysd, reps, x, v, xs, vs);
    return hipGetLastError();
}

__global__ void k_scatter(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                          const float4 *__restrict__ xs, const float4 *__restrict__ vs, float *__restrict__ x,
                          float *__restrict__ v, float *__restrict__ frames_slot) {
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n) return;
    const int n = S.n;
    const int o = S.perm[a];
    const float4 p = xs[2 * rd.poff + dup_index(a)];
    if (x) {
        float *xr = x + 3 * rd.off;
        xr[o] = p.x;
        xr[n + o] = p.y;
        xr[2 * n + o] = p.z;
    }
    if (frames_slot) {
        float *fr = frames_slot + 3 * rd.off;
        fr[o] = p.x;
        fr[n + o] = p.y;
        fr[2 * n + o] = p.z;
    }
    if (v && vs) {
        const float4 q = vs[rd.poff + a];
        float *vr = v + 3 * rd.off;
        vr[o] = q.x;
        vr[n + o] = q.y;
        vr[2 * n + o] = q.z;
    }
}

hipError_t launch_scatter(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, const float4 *xs,
                          const float4 *vs, float *x, float *v, float *frames_slot, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3((n_pad_max + 255) / 256, R), dim3(256), 0, st, sysd, reps, xs, vs, x, v,
                       frames_slot);
    return hipGetLastError();
}

// One wavefront per tile item; four per workgroup.  Force partial sums go to
// the float64 accumulators in global memory with hardware float64 atomics;
// the item's z partial to zpart[item] (summed per replica in a fixed order by
// k_finalize_rmd / k_reduce_z, so no two tiles meet on one address).  In
// PM_SCPS the contact reference of replica r is its effective reference
// E + eoff_r (written by k_scps_eff) and csum[r] = sum_k c_k.
template <int MODE, int NBK>
__global__ __launch_bounds__(256) void k_pairs(const KParams P, const SysDesc *__restrict__ sysd,
                                               const RepDesc *__restrict__ reps,
                                               const TileItem *__restrict__ items, const int n_items,
                                               const float4 *__restrict__ xs, double *__restrict__ acc,
                                               double *__restrict__ zpart, const float *__restrict__ eff,
                                               const double *__restrict__ csum) {
    using T = ModeTraits<MODE>;
    __shared__ float4 shpos[4][128];   // block J of each wavefront's item, stored twice
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = blockIdx.x * 4 + wave;
    const bool live = item < n_items;
    const TileItem it = items[live ? item : 0];
    const RepDesc rd = reps[it.rep];
    const SysDesc S = sysd[rd.sys];
    const int I = it.I, J = it.J, tf = it.flags;
    const int n = S.n, n_pad = S.n_pad;
    const float4 *xr2 = xs + 2 * rd.poff;
    {
        const float4 pj = xr2[J * 128 + lane];
        shpos[wave][lane] = pj;
        shpos[wave][64 + lane] = pj;
    }
    __syncthreads();
    if (!live) return;
    LaneI A;
    const int i = I * 64 + lane;
    A.p = xr2[I * 128 + lane];
    A.qp = P.dh_pref * A.p.w;
    A.o = S.perm[i];
    A.valid = i < n;
    A.contact = i < S.nc;
    float fi[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float fj[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float zt = 0.f;
    const bool contact_tile = tf & TF_CONTACT;
    const int64_t toff = contact_tile ? (int64_t)tile_index(I, J, S.ncb) * 4096 : 0;
    const float *rt;
    float cs = 0.f;
    if constexpr (MODE == PM_SCPS) {
        rt = eff + rd.eoff + toff;
        cs = (float)csum[it.rep];
    } else {
        rt = S.ref + toff;
    }
    if constexpr (!T::nb) {
        if (!contact_tile) return;
    }
    const bool diag = tf & TF_DIAG;
    const int kb = tile_kbeg(diag), ke = tile_kend(diag);
    tile_dispatch<MODE, NBK, 4 * SCPS_PAIR_GROUP>(tf, kb, ke, it.mask, P, lane, A, shpos[wave], S.perm + J * 64,
                                                  S.nc - J * 64, rt, cs, fi, fj, zt);
    const int jo = J * 64 + jflush_at(lane, ke);
    double *ar = acc + 6 * rd.poff;
    if constexpr (T::nb) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            unsafeAtomicAdd(&ar[c * n_pad + i], (double)fi[c]);
            unsafeAtomicAdd(&ar[c * n_pad + jo], (double)fj[c]);
        }
        // bonds of the particles of block I, once per block (diagonal tile)
        if ((tf & TF_DIAG) && A.valid && P.has_bond) {
            const int b = S.bond_next[i];
            if (b >= 0) {
                double f[3];
                bond_force(P, A.p, xr2[dup_index(b)], f);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unsafeAtomicAdd(&ar[c * n_pad + i], f[c]);
                    unsafeAtomicAdd(&ar[c * n_pad + b], -f[c]);
                }
            }
        }
    }
    if constexpr (T::grad) {
        if (contact_tile) {
#pragma unroll
            for (int c = 3; c < 6; ++c) {
                unsafeAtomicAdd(&ar[c * n_pad + i], (double)fi[c]);
                unsafeAtomicAdd(&ar[c * n_pad + jo], (double)fj[c]);
            }
        }
    }
    if constexpr (T::z) {
        const double zw = wave_sum((double)zt);
        if (lane == 0) zpart[item] = contact_tile ? zw : 0.0;
    }
}

template <int MODE>
static void launch_pairs_mode(int nbk, dim3 grid, dim3 block, hipStream_t st, const KParams &P,
                              const SysDesc *sysd, const RepDesc *reps, const TileItem *items, int n_items,
                              const float4 *xs, double *acc, double *zpart, const float *eff, const double *csum) {
#define SCPS_LAUNCH(K)                                                                                   \
    hipLaunchKernelGGL((k_pairs<MODE, K>), grid, block, 0, st, P, sysd, reps, items, n_items, xs, acc, zpart, \
                       eff, csum)
    if constexpr (!ModeTraits<MODE>::nb) {
        SCPS_LAUNCH(0);
    } else {
        switch (nbk) {
        case 0: SCPS_LAUNCH(0); break;
        case 1: SCPS_LAUNCH(1); break;
        case 2: SCPS_LAUNCH(2); break;
        default: SCPS_LAUNCH(3); break;
        }
    }
#undef SCPS_LAUNCH
}

hipError_t launch_pairs(int mode, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps,
                        const TileItem *items, int n_items, const float4 *xs, double *acc, double *zpart,
                        const float *eff, const double *csum, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    const dim3 grid((n_items + 3) / 4), block(256);
    switch (mode) {
    case PM_RMD:
        launch_pairs_mode<PM_RMD>(nbk, grid, block, st, P, sysd, reps, items, n_items, xs, acc, zpart, eff, csum);
        break;
    case PM_Z:
        launch_pairs_mode<PM_Z>(nbk, grid, block, st, P, sysd, reps, items, n_items, xs, acc, zpart, eff, csum);
        break;
    case PM_ZG:
        launch_pairs_mode<PM_ZG>(nbk, grid, block, st, P, sysd, reps, items, n_items, xs, acc, zpart, eff, csum);
        break;
    default:
        launch_pairs_mode<PM_SCPS>(nbk, grid, block, st, P, sysd, reps, items, n_items, xs, acc, zpart, eff, csum);
        break;
    }
    return hipGetLastError();
}

// z of replica r: the sum of its items' partials zpart[first[r] .. first[r+1])
// (items are stored replica by replica), one wavefront per replica, in a
// fixed order.
__device__ __forceinline__ double replica_z(const int *__restrict__ first, const double *__restrict__ zpart, int r,
                                           int lane) {
    double z = 0.0;
    for (int t = first[r] + lane; t < first[r + 1]; t += 64) z += zpart[t];
    return wave_sum(z);
}

// rMD ratchet per replica, eq (FrMD), from the replica's z.
__global__ void k_finalize_rmd(const KParams P, const int *__restrict__ first, const double *__restrict__ zpart,
                               double *__restrict__ cv, double *__restrict__ scale) {
    const int r = blockIdx.x;
    const double z = replica_z(first, zpart, r, threadIdx.x);
    if (threadIdx.x != 0) return;
    double *c = cv + (int64_t)r * CV_STRIDE;
    const double zm = fmin(c[CV_ZM], z);
    const double dz = z - zm;
    c[CV_Z] = z;
    c[CV_ZM] = zm;
    c[CV_EB] = 0.5 * P.k_R * dz * dz;
    scale[r] = -P.k_R * dz;
}

hipError_t launch_finalize_rmd(const KParams &P, int R, const int *first, const double *zpart, double *cv,
                               double *scale, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_rmd, dim3(R), dim3(64), 0, st, P, first, zpart, cv, scale);
    return hipGetLastError();
}

__global__ void k_reduce_z(const int *__restrict__ first, const double *__restrict__ zpart, double *__restrict__ z) {
    const int r = blockIdx.x;
    const double v = replica_z(first, zpart, r, threadIdx.x);
    if (threadIdx.x == 0) z[r] = v;
}


// SCPS tube variables per replica (one wavefront each), from the squared
// distances d_k Z0 = sum_p (C_p - R_kp)^2 to every frame k = 0..M of the
// stack, assembled in float64 as Q - 2 X_k + R2_k (Q = sum C^2 and
// X_k = sum C R_k from k_scps_dist, R2_k = sum R_k^2 of the stack):
//   s = 1 - (1/M) sum_k k p_k,  w = -(1/lambda) log sum_k exp(-lambda d_k),
//   p_k = softmax(-lambda d_k); ratchets on s and w, eqs (Fw),(Fs).
// The bias force is -sum_k c_k grad d_k with
//   c_k = p_k [k_s (s - s_m)(lambda/M)(k - kbar) + k_w (w - w_m)];
// coef receives c_k / Z0 and csum sum_k c_k / Z0 for the gradient pass.
// X and Q are consumed and cleared.
__global__ void k_finalize_scps(const KParams P, const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                                const int kmax, double *__restrict__ X, double *__restrict__ Q,
                                double *__restrict__ cv, float *__restrict__ coef, double *__restrict__ csum) {
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const SysDesc S = sysd[reps[r].sys];
    const int K = S.K, M = K - 1;
    double *xr = X + (int64_t)r * kmax;
    const double q = Q[r];
    const double lam = P.lambda;
    // d_k for the (at most two) frames this lane holds
    double dk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        dk[h] = k < K ? fmax(q - 2.0 * xr[k] + S.R2[k], 0.0) / S.Z0 : 0.0;
    }
    double a = -INFINITY;
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (lane + 64 * h < K) a = fmax(a, -lam * dk[h]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o, 64));
    double s0 = 0.0, s1 = 0.0, e[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        if (k < K) {
            e[h] = exp(-lam * dk[h] - a);
            s0 += e[h];
            s1 += (double)k * e[h];
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const double kbar = s1 / s0;
    const double sv = 1.0 - kbar / (double)M;
    const double wv = -(a + log(s0)) / lam;
    double *c = cv + (int64_t)r * CV_STRIDE;
    const double sm = fmin(c[CV_SM], sv);
    const double wm = fmin(c[CV_WM], wv);
    const double ds = sv - sm, dw = wv - wm;
    double tot = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = lane + 64 * h;
        if (k < K) {
            const double pk = e[h] / s0;
            const double ckv = pk * (P.k_s * ds * (lam / (double)M) * ((double)k - kbar) + P.k_w * dw);
            coef[(int64_t)r * kmax + k] = (float)(ckv / S.Z0);
            tot += ckv;
            xr[k] = 0.0;
        }
    }
    tot = wave_sum(tot);
    if (lane == 0) {
        Q[r] = 0.0;
        csum[r] = tot / S.Z0;
        c[CV_S] = sv;
        c[CV_W] = wv;
        c[CV_SM] = sm;
        c[CV_WM] = wm;
        c[CV_EB] = 0.5 * P.k_s * ds * ds + 0.5 * P.k_w * dw * dw;
    }
}

hipError_t launch_finalize_scps(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R, int kmax,
                                double *X, double *Q, double *cv, float *coef, double *csum, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_scps, dim3(R), dim3(64), 0, st, P, sysd, reps, kmax, X, Q, cv, coef, csum);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// SCPS on matrix cores.  The squared distance of replica r to frame k,
// d_k Z0 = sum_p (C_rp - R_kp)^2, splits into sum_p C_rp^2 - 2 X_rk +
// sum_p R_kp^2 with X_rk = sum_p C_rp R_kp: for a group of up to 32 replicas
// of one system that is a dense contraction over the contact pairs p, done
// here with float32 MFMA whose sums are moved into float64 every 64 pairs
// (the three terms are then accurate to float64 rounding of float32-exact
// partial sums, which keeps the cancellation in Q - 2X + R2 harmless).  The
// bias pass needs each replica's effective reference E_rp = sum_k c_rk R_kp, a
// contraction over the frames, also float32 MFMA (the same rounding as a
// float32 dot product).  Both read every stack tile once per group instead of
// once per replica.
// ---------------------------------------------------------------------------
typedef float fvec16 __attribute__((ext_vector_type(16)));

// Unordered contact pair (64 I + l, 64 J + ((l + s) mod 64)) of a tile in the
// diagonal-major layout: in a diagonal tile every pair appears twice; the
// copy at sub-steps 1..31, or at 32 for l < 32, is the one that counts.
__device__ __forceinline__ bool tile_pair_counts(bool diag, int s, int l) {
    return !diag || (s >= 1 && (s < 32 || (s == 32 && l < 32)));
}

// Pair-major copy of a frame stack: stack_pm[tile][p][k] = stack[tile][k][p]
// for k < K (zero for K <= k < K4), and R2[k] += sum over the counted pairs of
// R_kp^2 (float64; pairs within min_seq_sep, outside the contact set or
// repeated in a diagonal tile are not counted).  One workgroup per (tile,
// sub-step s): the 64 pairs of that sub-step.  R2 must be zero on entry.
__global__ __launch_bounds__(256) void k_stack_pairmajor(int nc, int ncb, int ntile, int K, int min_sep,
                                                         const int *__restrict__ perm,
                                                         const float *__restrict__ stack,
                                                         float *__restrict__ stack_pm, double *__restrict__ R2) {
    __shared__ float buf[64][KMAX + 1];
    __shared__ double r2s[KMAX];
    const int tile = blockIdx.x, s = blockIdx.y;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int tid = threadIdx.x;
    if (tid < KMAX) r2s[tid] = 0.0;
    __syncthreads();
    for (int e = tid; e < 64 * K; e += 256) {
        const int k = e >> 6, l = e & 63;
        const float v = stack[((int64_t)tile * K + k) * 4096 + s * 64 + l];
        buf[l][k] = v;
        const int a = I * 64 + l, b = J * 64 + ((l + s) & 63);
        const bool counts = a < nc && b < nc && tile_pair_counts(I == J, s, l) && abs(perm[a] - perm[b]) > min_sep;
        if (counts) atomicAdd(&r2s[k], (double)v * (double)v);
    }
    __syncthreads();
    const int K4 = stack_pm_width(K);
    float *out = stack_pm + ((int64_t)tile * 4096 + s * 64) * K4;
    for (int e = tid; e < 64 * K4; e += 256) {
        const int l = e / K4, k = e - l * K4;
        out[e] = k < K ? buf[l][k] : 0.f;
    }
    if (tid < K) unsafeAtomicAdd(&R2[tid], r2s[tid]);
}

hipError_t launch_stack_pairmajor(int nc, int ncb, int K, int min_sep, const int *perm, const float *stack,
                                  float *stack_pm, double *R2, hipStream_t st) {
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0 || K == 0) return hipSuccess;
    if (K > KMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stack_pairmajor, dim3(nt, 64), dim3(256), 0, st, nc, ncb, nt, K, min_sep, perm, stack,
                       stack_pm, R2);
    return hipGetLastError();
}

// Contact value of one replica-pair for the MFMA operand (0 when the pair
// does not count).
__device__ __forceinline__ float contact_operand(const KParams &P, const float4 &pi, const float4 &pj, bool ok) {
    float dx, dy, dz;
    const float r2 = pair_r2(pi, pj, dx, dy, dz);
    const float q = r2 * P.inv_r0sq;
    const float q2 = q * q;
    const float num = 1.f + q + q2;
    const float den = fmaf(q2, q + q2, num);
    const bool inside = !P.has_cut | (r2 <= P.r_cut2);
    return (ok & inside) ? num * frcp(den) : 0.f;
}

#ifndef SCPS_DIST_AHEAD
#define SCPS_DIST_AHEAD 8
#endif
// Pass 1: X[r][k] += sum_p C_rp R_kp and Q[r] += sum_p C_rp^2 over the contact
// pairs of each work item (group of replicas, tile); workgroups stride over
// the items and flush their sums when the group changes and at the end.
// The pairs of a tile are taken row by row: wavefront w takes rows
// i = w, w+4, ... of block I and, per row, 32 MFMA steps of 2 pairs
// (i, 2m + (l >> 5)); lane l evaluates that pair for replica l & 31 (A operand
// of 32x32x2 float32 MFMAs) with particle i's position held in a register and
// particle j's read from the block-J positions in LDS, and loads frames
// 2 (l & 31) and 2 (l & 31) + 1 of the pair with one 8-byte load,
// SCPS_DIST_AHEAD steps ahead of their use; frame block h holds frames 2j + h,
// so component h of that load is the lane's B operand of block h.  A diagonal
// tile counts the pairs j > i.  The float32 accumulators hold one row (64
// pairs per element) and are added after every row into the workgroup's
// float64 sums xl[slot][frame] in LDS.  Element v of lane l in block h is
// replica slot 8 (v >> 2) + 4 (l >> 5) + (v & 3), frame 2 (l & 31) + h.
template <bool MASK>
__device__ __forceinline__ void scps_dist_tile(const KParams &P, const SysDesc &S, const int nrep,
                                               const ScpsItem &it, const float4 (*posj)[32], const int *orgj,
                                               const float4 *__restrict__ xs, const RepDesc *__restrict__ reps,
                                               const int myrep, const int lane, const int wave, double *xl,
                                               double &q) {
    const int I = it.IJ >> 16, J = it.IJ & 0xFFFF;
    const bool diag = I == J;
    const int K4 = stack_pm_width(S.K);
    const int rs = lane & 31, pq = lane >> 5;
    const bool rep = rs < nrep;
    const bool bload = 2 * rs < K4;
    const float *Rt = S.stack_pm + (int64_t)it.tile * 4096 * K4 + 2 * rs;
    const float4 *xr = xs + 2 * reps[myrep].poff + I * 128;
    constexpr int D = SCPS_DIST_AHEAD;
    const float2 zero2 = make_float2(0.f, 0.f);
    // pair (i, j) sits at s * 64 + i in the tile, s = (j - i) mod 64
    auto bop = [&](int i_, int m_) {
        const int s_ = (2 * m_ + pq - i_) & 63;
        return (bload && i_ < 64) ? *reinterpret_cast<const float2 *>(Rt + (int64_t)(s_ * 64 + i_) * K4) : zero2;
    };
    float2 ring[D];
#pragma unroll
    for (int u = 0; u < D; ++u) ring[u] = bop(wave, u);
#pragma unroll 1
    for (int i = wave; i < 64; i += 4) {
        const float4 pi = rep ? xr[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const int oi = MASK ? S.perm[I * 64 + i] : 0;
        const bool icon = I * 64 + i < S.nc;
        fvec16 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[h][v] = 0.f;
#pragma unroll 1
        for (int mg = 0; mg < 32 / D; ++mg) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int m = D * mg + u;
                const float2 b = ring[u];
                const int nm = m + D < 32 ? m + D : m + D - 32, ni = m + D < 32 ? i : i + 4;
                ring[u] = bop(ni, nm);
                const int jl = 2 * m + pq;
                bool ok = !diag | (jl > i);
                if constexpr (MASK) {
                    ok = ok & icon & (J * 64 + jl < S.nc) & (abs(oi - orgj[jl]) > P.min_sep);
                }
                const float c = contact_operand(P, pi, posj[jl][rs], ok & rep);
                q = fma((double)c, (double)c, q);
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(c, b.x, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(c, b.y, acc[1], 0, 0, 0);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                atomicAdd(&xl[(8 * (v >> 2) + 4 * pq + (v & 3)) * 64 + 2 * rs + h], (double)acc[h][v]);
    }
}

#ifndef SCPS_DIST_WPE
#define SCPS_DIST_WPE 3
#endif
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SCPS_DIST_WPE, SCPS_DIST_WPE))) void k_scps_dist(const KParams P, const SysDesc *__restrict__ sysd,
                                                   const RepDesc *__restrict__ reps,
                                                   const ScpsGroup *__restrict__ groups,
                                                   const ScpsItem *__restrict__ items, const int n_items,
                                                   const float4 *__restrict__ xs, double *__restrict__ X,
                                                   double *__restrict__ Q, const int kmax) {
    __shared__ __align__(16) float4 posj[64][32];   // block J of every replica slot
    __shared__ double xl[32 * 64];                   // float64 sums X[slot][frame] of the current group
    __shared__ double ql[4][64];
    __shared__ int orgj[64];
    __shared__ int sh_rep[32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < 32 * 64; e += 256) xl[e] = 0.0;
    double q = 0.0;
    int cur = -1, nrep = 0;
    SysDesc S;
    for (int t = blockIdx.x;; t += gridDim.x) {
        const bool more = t < n_items;
        const ScpsItem it = more ? items[t] : ScpsItem{-1, 0, 0, 0};
        if (cur >= 0 && it.group != cur) {
            // flush the group's sums to the replicas' float64 totals
            ql[wave][lane] = q;
            __syncthreads();
            for (int e = tid; e < 32 * 64; e += 256) {
                const int slot = e >> 6, k = e & 63;
                if (slot < nrep && k < S.K) unsafeAtomicAdd(&X[(int64_t)sh_rep[slot] * kmax + k], xl[e]);
                xl[e] = 0.0;
            }
            if (tid < 32) {
                double sum = 0.0;
                for (int w = 0; w < 4; ++w) sum += ql[w][tid] + ql[w][32 + tid];
                if (tid < nrep) unsafeAtomicAdd(&Q[sh_rep[tid]], sum);
            }
            q = 0.0;
        }
        if (!more) break;
        __syncthreads();
        if (it.group != cur) {
            cur = it.group;
            const ScpsGroup *gp = groups + cur;
            nrep = gp->nrep;
            S = sysd[gp->sys];
            if (tid < 32) sh_rep[tid] = tid < nrep ? gp->rep[tid] : 0;
            __syncthreads();
        }
        // stage block J of every replica of the group
        const int J = it.IJ & 0xFFFF;
        for (int e = tid; e < 64 * 32; e += 256) {
            const int pl = e >> 5, slot = e & 31;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (slot < nrep) p = xs[2 * reps[sh_rep[slot]].poff + J * 128 + pl];
            posj[pl][slot] = p;
        }
        if (tid < 64) orgj[tid] = S.perm[J * 64 + tid];
        __syncthreads();
        const int myrep = sh_rep[lane & 31];
        if (it.flags & TILE_MASK)
            scps_dist_tile<true>(P, S, nrep, it, posj, orgj, xs, reps, myrep, lane, wave, xl, q);
        else
            scps_dist_tile<false>(P, S, nrep, it, posj, orgj, xs, reps, myrep, lane, wave, xl, q);
    }
}

// Pass 2 operand: E[eoff_r + tile * 4096 + p] = sum_k c_rk R_kp for every
// pair p of each work item's tile and replica r of its group (coef holds
// c_rk).  Wavefront w takes chunks of 32 EFF_NB pairs w, w+4, ...; a chunk is
// EFF_NB 32-pair MFMA blocks interleaved so that block b holds pairs
// EFF_NB j + b: lane l reads pairs EFF_NB (l & 31) .. +EFF_NB-1 of frame
// 2 kk + (l >> 5) with one load (component b is its B operand of block b)
// and supplies c of replica l & 31 for that frame (A operand, 32x32x2
// float32 MFMA).  Result element v of lane l in block b is replica
// 8 (v >> 2) + 4 (l >> 5) + (v & 3), pair EFF_NB (l & 31) + b: the blocks give
// one EFF_NB-wide store per replica.
#ifndef SCPS_EFF_BLOCKS
#define SCPS_EFF_BLOCKS 4
#endif
#ifndef SCPS_EFF_WPE
#define SCPS_EFF_WPE (SCPS_EFF_BLOCKS == 4 ? 2 : 3)
#endif
constexpr int EFF_NB = SCPS_EFF_BLOCKS;
static_assert(EFF_NB == 2 || EFF_NB == 4, "chunks of 2 or 4 MFMA blocks");
typedef float effvec __attribute__((ext_vector_type(EFF_NB)));

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SCPS_EFF_WPE, SCPS_EFF_WPE))) void k_scps_eff(
    const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps, const ScpsGroup *__restrict__ groups,
    const ScpsItem *__restrict__ items, const int n_items, const float *__restrict__ coef, const int kmax,
    float *__restrict__ E) {
    __shared__ int64_t sh_eoff[SCPS_GROUP];   // -1 for an empty slot
    constexpr int CH = 32 * EFF_NB;            // pairs per chunk
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = lane & 31, half = lane >> 5;
    int cur = -1;
    SysDesc S;
    float creg[KMAX / 2];
    for (int t = blockIdx.x; t < n_items; t += gridDim.x) {
        const ScpsItem it = items[t];
        if (it.group != cur) {
            cur = it.group;
            const ScpsGroup *gp = groups + cur;
            const int nrep = gp->nrep;
            S = sysd[gp->sys];
            const int myrep = slot < nrep ? gp->rep[slot] : 0;
#pragma unroll
            for (int kk = 0; kk < KMAX / 2; ++kk) {
                const int k = 2 * kk + half;
                creg[kk] = (slot < nrep && k < S.K) ? coef[(int64_t)myrep * kmax + k] : 0.f;
            }
            __syncthreads();
            if (tid < SCPS_GROUP) sh_eoff[tid] = tid < nrep ? reps[gp->rep[tid]].eoff : -1;
            __syncthreads();
        }
        const int K = S.K;
        const float *Rt = S.stack + (int64_t)it.tile * K * 4096;
#pragma unroll 1
        for (int ch = wave; ch < 4096 / CH; ch += 4) {
            const int p = ch * CH + EFF_NB * slot;
            fvec16 acc[EFF_NB];
#pragma unroll
            for (int bl = 0; bl < EFF_NB; ++bl)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[bl][v] = 0.f;
#pragma unroll
            for (int kk = 0; kk < KMAX / 2; ++kk) {
                if (2 * kk < K) {
                    const int k = 2 * kk + half;
                    effvec b;
                    if (k < K)
                        b = *reinterpret_cast<const effvec *>(Rt + k * 4096 + p);
                    else
#pragma unroll
                        for (int bl = 0; bl < EFF_NB; ++bl) b[bl] = 0.f;
#pragma unroll
                    for (int bl = 0; bl < EFF_NB; ++bl)
                        acc[bl] = __builtin_amdgcn_mfma_f32_32x32x2f32(creg[kk], b[bl], acc[bl], 0, 0, 0);
                }
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t eo = sh_eoff[8 * (v >> 2) + 4 * half + (v & 3)];
                if (eo >= 0) {
                    effvec o;
#pragma unroll
                    for (int bl = 0; bl < EFF_NB; ++bl) o[bl] = acc[bl][v];
                    *reinterpret_cast<effvec *>(E + eo + (int64_t)it.tile * 4096 + p) = o;
                }
            }
        }
    }
}

hipError_t launch_scps_dist(const KParams &P, const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups,
                            const ScpsItem *items, int n_items, const float4 *xs, double *X, double *Q, int kmax,
                            hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    const int cap = 256 * SCPS_DIST_WPE;   // resident workgroups: WPE per SIMD, four waves each
    const int grid = n_items < cap ? n_items : cap;
    hipLaunchKernelGGL(k_scps_dist, dim3(grid), dim3(256), 0, st, P, sysd, reps, groups, items, n_items, xs, X, Q,
                       kmax);
    return hipGetLastError();
}

hipError_t launch_scps_eff(const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups, const ScpsItem *items,
                           int n_items, const float *coef, int kmax, float *E, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    const int grid = n_items < 1024 ? n_items : 1024;
    hipLaunchKernelGGL(k_scps_eff, dim3(grid), dim3(256), 0, st, sysd, reps, groups, items, n_items, coef, kmax,
                       E);
    return hipGetLastError();
}

// Langevin update of every particle; consumes and clears the accumulators.
// The force is acc[0..2] + scale[r] * acc[3..5], the second term being the
// bias; each workgroup adds its particles' dt |F_bias|^2 / (m gamma) to the
// replica's bias functional cv[r][CV_T].
__global__ __launch_bounds__(256) void k_integrate(const KParams P, const SysDesc *__restrict__ sysd,
                                                   const RepDesc *__restrict__ reps, float4 *__restrict__ xs,
                                                   float4 *__restrict__ vs, double *__restrict__ acc,
                                                   const double *__restrict__ scale, double *__restrict__ cv,
                                                   const uint64_t step, int *__restrict__ flags) {
    __shared__ double tred[4];
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double tb = 0.0;
    if (a < S.n) {
        const int n_pad = S.n_pad;
        double *ar = acc + 6 * rd.poff;
        const double sc = scale[r];
        const double inv_m = 1.0 / (double)S.mass[a];
        double F[3], fb2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double fb = sc * ar[(c + 3) * n_pad + a];
            F[c] = ar[c * n_pad + a] + fb;
            fb2 = fma(fb, fb, fb2);
            ar[c * n_pad + a] = 0.0;
            ar[(c + 3) * n_pad + a] = 0.0;
        }
        tb = fb2 * inv_m;
        double g[3];
        normals3(P, (uint32_t)S.perm[a], P.rep_base + (uint32_t)r, step, g[0], g[1], g[2]);
        float4 *xr2 = xs + 2 * rd.poff;
        const int da = dup_index(a);
        const float4 p = xr2[da];
        double X[3] = {(double)p.x, (double)p.y, (double)p.z};
        if (P.integrator == 0) {
            const double mob = P.dt * inv_m / P.gamma;
            const double amp = sqrt(2.0 * P.kT * mob);
#pragma unroll
            for (int c = 0; c < 3; ++c) X[c] += mob * F[c] + amp * g[c];
        } else {
            const float4 q = vs[rd.poff + a];
            double V[3] = {(double)q.x, (double)q.y, (double)q.z};
            const double amp = sqrt((1.0 - P.c1 * P.c1) * P.kT * inv_m);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                V[c] += P.dt * F[c] * inv_m;
                X[c] += 0.5 * P.dt * V[c];
                V[c] = P.c1 * V[c] + amp * g[c];
                X[c] += 0.5 * P.dt * V[c];
            }
            vs[rd.poff + a] = make_float4((float)V[0], (float)V[1], (float)V[2], 0.f);
        }
        const float4 np = make_float4((float)X[0], (float)X[1], (float)X[2], p.w);
        if (!(isfinite(np.x) && isfinite(np.y) && isfinite(np.z))) flags[r] = 1;
        xr2[da] = np;
        xr2[da + 64] = np;
    }
    tb = wave_sum(tb);
    if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = tb;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = tred[0] + tred[1] + tred[2] + tred[3];
        if (t != 0.0) unsafeAtomicAdd(&cv[(int64_t)r * CV_STRIDE + CV_T], P.dt / P.gamma * t);
    }
}

hipError_t launch_integrate(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max,
                            float4 *xs, float4 *vs, double *acc, const double *scale, double *cv, uint64_t step,
                            int *flags, hipStream_t st) {
    hipLaunchKernelGGL(k_integrate, dim3((n_pad_max + 255) / 256, R), dim3(256), 0, st, P, sysd, reps, xs, vs, acc,
                       scale, cv, step, flags);
    return hipGetLastError();
}

// z and coef * grad z out of the accumulators (eval_z_and_grad); clears them.
__global__ void k_eval_out(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                           double *__restrict__ acc, float *__restrict__ grad, const double *__restrict__ grad_coef) {
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= S.n) return;
    const int n = S.n, n_pad = S.n_pad;
    double *ar = acc + 6 * rd.poff;
    const double cf = grad_coef ? grad_coef[r] : 1.0;
    const int o = S.perm[a];
    float *gr = grad + 3 * rd.off;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        gr[c * n + o] = (float)(cf * ar[(c + 3) * n_pad + a]);
        ar[(c + 3) * n_pad + a] = 0.0;
    }
}

hipError_t launch_eval_out(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, double *acc,
                           const int *first, const double *zpart, double *z_out, float *grad, const double *grad_coef,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_z, dim3(R), dim3(64), 0, st, first, zpart, z_out);
    if (grad)
        hipLaunchKernelGGL(k_eval_out, dim3((n_pad_max + 255) / 256, R), dim3(256), 0, st, sysd, reps, acc, grad,
                           grad_coef);
    return hipGetLastError();
}

__global__ void k_ratchet_energy(int R, double k_R, const double *__restrict__ z, const double *__restrict__ zm,
                                 double *__restrict__ Eb, const double *__restrict__ gz,
                                 const double *__restrict__ gE, double *__restrict__ coef) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double d = z[r] - zm[r];
    const double th = d >= 0.0 ? 1.0 : 0.0;  // theta(0) = 1
    if (Eb) Eb[r] = 0.5 * k_R * d * d * th;
    if (coef) coef[r] = (gz ? gz[r] : 0.0) + (gE ? gE[r] : 0.0) * k_R * d * th;
}

hipError_t launch_ratchet_energy(int R, double k_R, const double *z, const double *zm, double *Eb,
                                 const double *gz, const double *gE, double *coef, hipStream_t st) {
    hipLaunchKernelGGL(k_ratchet_energy, dim3((R + 255) / 256), dim3(256), 0, st, R, k_R, z, zm, Eb, gz, gE, coef);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reference maps
// ---------------------------------------------------------------------------
__device__ __forceinline__ double contact_f64(double r2, double r0, double r_cut) {
    if (r_cut > 0.0 && r2 > r_cut * r_cut) return 0.0;
    const double q = r2 / (r0 * r0);
    const double q2 = q * q;
    const double num = 1.0 + q + q2;
    return num / (num + q2 * (q + q2));
}

__device__ __forceinline__ int64_t packed_index(int nc, int a, int b) {
    return (int64_t)a * nc - (int64_t)a * (a + 1) / 2 + (b - a - 1);
}

// One workgroup of 256 threads per contact tile pair; thread (w, l) fills
// rows k = w, w+4, ... of the diagonal-major layout element [k][l] =
// R(64I + l, 64J + ((l + k) mod 64)).  Internal contact positions equal the
// positions in contact_idx, so tiles and packed maps share indices.
__global__ void k_native_map(int n, int nc, int ncb, const int *__restrict__ perm, const double *__restrict__ xyz,
                             double r0, double r_cut, float *__restrict__ tiles, double *__restrict__ packed) {
    int I, J;
    tile_decode(blockIdx.x, ncb, I, J);
    const int l = threadIdx.x & 63;
    const int a = I * 64 + l;
    float *t = tiles + (int64_t)blockIdx.x * 4096;
    for (int k = threadIdx.x >> 6; k < 64; k += 4) {
        const int b = J * 64 + ((l + k) & 63);
        double C = 0.0;
        if (a < nc && b < nc && a != b) {
            const int oa = perm[a], ob = perm[b];
            const double dx = xyz[oa] - xyz[ob];
            const double dy = xyz[n + oa] - xyz[n + ob];
            const double dz = xyz[2 * n + oa] - xyz[2 * n + ob];
            C = contact_f64(dx * dx + dy * dy + dz * dz, r0, r_cut);
            if (packed && a < b) packed[packed_index(nc, a, b)] = C;
        }
        t[k * 64 + l] = (float)C;
    }
}

hipError_t launch_native_map(int n, int n_pad, int nc, int ncb, const int *perm_dev, const double *xyz_dev,
                             double r0, double r_cut, float *tiles, double *packed, hipStream_t st) {
    (void)n_pad;
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_native_map, dim3(nt), dim3(256), 0, st, n, nc, ncb, perm_dev, xyz_dev, r0, r_cut, tiles,
                       packed);
    return hipGetLastError();
}

__global__ void k_pack_to_tiles(int nc, int ncb, int ntile, const double *__restrict__ packed,
                                float *__restrict__ tiles) {
    const int tile = blockIdx.x;
    const int map = blockIdx.y;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int64_t P = (int64_t)nc * (nc - 1) / 2;
    const double *pm = packed + (int64_t)map * P;
    float *t = tiles + ((int64_t)tile * gridDim.y + map) * 4096;   // [tile][map][4096]
    const int l = threadIdx.x & 63;
    const int a = I * 64 + l;
    for (int k = threadIdx.x >> 6; k < 64; k += 4) {
        const int b = J * 64 + ((l + k) & 63);
        float v = 0.f;
        if (a < nc && b < nc && a != b) v = (float)pm[a < b ? packed_index(nc, a, b) : packed_index(nc, b, a)];
        t[k * 64 + l] = v;
    }
}

hipError_t launch_pack_to_tiles(int n_maps, int nc, int ncb, const double *packed, float *tiles, hipStream_t st) {
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0 || n_maps == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_to_tiles, dim3(nt, n_maps), dim3(256), 0, st, nc, ncb, nt, packed, tiles);
    return hipGetLastError();
}

// sum_i v_i^2 in two fixed-order phases: SUMSQ_BLOCKS workgroups each reduce
// a contiguous chunk into part[], then one workgroup adds the partials.
constexpr int SUMSQ_BLOCKS = 256;
__global__ void k_sum_squares(int64_t m, const double *__restrict__ v, double *__restrict__ part,
                              double *__restrict__ out) {
    __shared__ double red[4];
    const int64_t chunk = (m + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < m ? lo + chunk : m;
    double s = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) s += v[e] * v[e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_parts(int n, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += blockDim.x) s += part[e];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

int sum_squares_scratch() { return SUMSQ_BLOCKS; }

hipError_t launch_sum_squares(int64_t m, const double *v, double *part, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_squares, dim3(SUMSQ_BLOCKS), dim3(256), 0, st, m, v, part, out);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, SUMSQ_BLOCKS, part, out);
    return hipGetLastError();
}

// eq (avCij): mean over successful paths of C(X_p(t_k)), float64 sums.
// Grid (contact tile pair, frame); thread (w, l) owns 16 rows k of the
// diagonal-major tile and loops over the successful paths.
__global__ __launch_bounds__(256) void k_update_reference(int n, int nc, int ncb, int ntile,
                                                          const int *__restrict__ perm,
                                                          const float *__restrict__ frames, int n_paths,
                                                          const int *__restrict__ succ, int n_succ, double r0,
                                                          double r_cut, float *__restrict__ tiles,
                                                          double *__restrict__ packed) {
    __shared__ float4 blk[2][64];
    const int tile = blockIdx.x, f = blockIdx.y;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int a = I * 64 + l;
    double sum[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) sum[k] = 0.0;
    for (int s = 0; s < n_succ; ++s) {
        const float *X = frames + ((int64_t)f * n_paths + succ[s]) * 3 * (int64_t)n;
        __syncthreads();
        if (threadIdx.x < 128) {
            const int which = threadIdx.x >> 6;
            const int c = (which ? J : I) * 64 + l;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < nc) {
                const int o = perm[c];
                p = make_float4(X[o], X[n + o], X[2 * n + o], 0.f);
            }
            blk[which][l] = p;
        }
        __syncthreads();
        const float4 pa = blk[0][l];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int k = w * 16 + kk;
            const float4 pb = blk[1][(l + k) & 63];
            const double dx = (double)pa.x - (double)pb.x;
            const double dy = (double)pa.y - (double)pb.y;
            const double dz = (double)pa.z - (double)pb.z;
            sum[kk] += contact_f64(dx * dx + dy * dy + dz * dz, r0, r_cut);
        }
    }
    float *t = tiles + ((int64_t)tile * gridDim.y + f) * 4096;     // [tile][frame][4096]
    const int64_t P = (int64_t)nc * (nc - 1) / 2;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
        const int k = w * 16 + kk;
        const int b = J * 64 + ((l + k) & 63);
        double mean = 0.0;
        if (a < nc && b < nc && a != b) {
            mean = sum[kk] / (double)n_succ;
            if (packed && a < b) packed[(int64_t)f * P + packed_index(nc, a, b)] = mean;
        }
        t[k * 64 + l] = (float)mean;
    }
}

hipError_t launch_update_reference(int n, int n_pad, int nc, int ncb, const int *perm_dev, const float *frames,
                                   int n_paths, int n_frames, const int *succ_idx, int n_succ, double r0,
                                   double r_cut, float *tiles, double *packed, hipStream_t st) {
    (void)n_pad;
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_reference, dim3(nt, n_frames), dim3(256), 0, st, n, nc, ncb, nt, perm_dev, frames,
                       n_paths, succ_idx, n_succ, r0, r_cut, tiles, packed);
    return hipGetLastError();
}

}  // namespace scps
