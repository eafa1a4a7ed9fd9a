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
#include <limits.h>
#include <math.h>

#include "scps_device.h"
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


// Reference maps live in global memory; telling the compiler so lets it use
// global loads with a scalar base instead of flat loads.
typedef const float __attribute__((address_space(1))) gfloat;
__device__ __forceinline__ float ldg(const float *p, int64_t i) {
    return ((gfloat *)p)[i];
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
enum { PM_RMD = 0, PM_Z = 1, PM_ZG = 2, PM_SCPS = 3, PM_NB = 4 };

template <int MODE> struct ModeTraits {
    static constexpr bool nb = (MODE == PM_RMD || MODE == PM_SCPS || MODE == PM_NB);
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
            nbon[u] = act0 & (sep > P.nb_excl) & (!P.has_cut_nb | (r2[u] <= P.r_cut_nb2));
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
            const float t = q + q2;             // num = 1 + t, den = num + q^2 t
            const float num = 1.f + t;
            const float den = fmaf(q2, t, num);
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
            nba[u] = (sa > P.nb_excl) & (!P.has_cut_nb | (r2a[u] <= P.r_cut_nb2));
            nbb[u] = (sb > P.nb_excl) & (!P.has_cut_nb | (r2b[u] <= P.r_cut_nb2));
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
                const float t = q + q2;
                const float num = 1.f + t;
                const float den = fmaf(q2, t, num);
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
    // -k (r - r0) / r as k (r0 / r - 1): one float64 reciprocal square root, no division
    const double s = P.k_bond * (P.r_bond * rsqrt(dx * dx + dy * dy + dz * dz) - 1.0);
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
// packed persistent rMD kernel: several short chains per wavefront
// ---------------------------------------------------------------------------
// A chain of at most W <= 64 particles runs in a segment of W lanes: a
// wavefront holds P = 64 / W replicas (segment s: lanes s W .. s W + W - 1,
// lane s W + a owns internal particle a), a workgroup blockDim.x / 64
// wavefronts, and the kernel runs all n_steps of every replica it holds.
// Each wavefront works alone on its own part of LDS (no workgroup barrier):
// the lanes publish their positions each step and read their partners'.
// Every pair is evaluated once: lane a meets b = (a + k) mod n at step
// k = 1 .. n/2 (even n: lanes a < n/2 only at the last step), adds its own
// side and keeps b's side in j-side partials that move one lane back within
// the segment after each step and reach their owner lane at the end.
// Float32 pair math over at most 32 steps per lane, then float64 per particle,
// as in the tile kernels; bonds, the ratchet and the Langevin update in
// float64.  Segment sums (z each step, T at the end) run as a fixed binary
// tree over the segment's lanes (ds_bpermute) whose total the first lane
// hands to the others, so every lane of a replica holds the same z.
constexpr int PACK_WMAX = 64;

// Lanes of one wavefront exchanging values through LDS: what the lanes stored
// before this point is visible to every lane's loads after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// a double from the lane whose byte address (4 x lane) is given
__device__ __forceinline__ double bpermute_f64(int from, double v) {
    const int lo = __builtin_amdgcn_ds_bpermute(from, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(from, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// LDS of one wavefront: positions (x, y, z, charge), chain indices, the
// chain predecessors and the lane's native-map value at every partner step
// (rows 1 .. W/2; row 0 unused).
__host__ __device__ inline size_t packed_wave_lds_bytes(int W) {
    return 64 * (sizeof(float4) + sizeof(int) + sizeof(int)) + (size_t)(W / 2 + 1) * 64 * sizeof(float);
}

template <int NBK>
__global__ __launch_bounds__(512) void k_rmd_packed(const KParams P, const SysDesc *__restrict__ sysd,
                                                    const RepDesc *__restrict__ reps, const int R, const int W,
                                                    float *__restrict__ x, float *__restrict__ v,
                                                    double *__restrict__ cv, const int64_t n_steps,
                                                    const uint64_t step0, const int record_every,
                                                    float *__restrict__ frames, const int64_t frame_stride,
                                                    int *__restrict__ flags) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned char *wl = smem + (size_t)wave * packed_wave_lds_bytes(W);
    float4 *posl = reinterpret_cast<float4 *>(wl);                 // [64]
    int *orgl = reinterpret_cast<int *>(posl + 64);                 // [64]
    int *prevl = orgl + 64;                                          // [64]
    float *refl = reinterpret_cast<float *>(prevl + 64);           // [W/2 + 1][64]: R(a, partner at step k)

    const int PR = 64 / W;                           // replicas per wavefront
    const int seg = lane / W, a = lane - seg * W, sbase = seg * W;
    const int slot = ((int)blockIdx.x * (int)(blockDim.x >> 6) + wave) * PR + seg;
    const int r = (seg < PR && slot < R) ? slot : -1;
    RepDesc rd{};
    SysDesc S{};
    int n = 0;
    if (r >= 0) {
        rd = reps[r];
        S = sysd[rd.sys];
        n = S.n;
    }
    const bool act = a < n;                          // a particle of a replica
    float *xr = r >= 0 ? x + 3 * rd.off : nullptr;
    float *vr = (r >= 0 && v) ? v + 3 * rd.off : nullptr;
    int o = lane, nxt = -1;
    float4 p = pad_position(lane);
    float vel[3] = {0.f, 0.f, 0.f};
    double inv_m = 1.0;
    if (act) {
        o = S.perm[a];
        p = make_float4(xr[o], xr[n + o], xr[2 * n + o], S.charge[a]);
        if (vr) {
            vel[0] = vr[o];
            vel[1] = vr[n + o];
            vel[2] = vr[2 * n + o];
        }
        inv_m = 1.0 / (double)S.mass[a];
        nxt = S.bond_next[a];
    }
    const bool icon = act && a < S.nc;
    const float qp = P.dh_pref * p.w;
    orgl[lane] = o;
    prevl[lane] = -1;
    wave_lds_sync();
    if (act && nxt >= 0) prevl[sbase + nxt] = a;
    // native-map value of the pair met at partner step k (0 outside the contact set)
    for (int k = 1; k <= (W >> 1); ++k) {
        float rv = 0.f;
        if (icon && k < n) {
            const int b = a + k < n ? a + k : a + k - n;
            if (b < S.nc) rv = S.ref[((b - a) & 63) * 64 + a];
        }
        refl[k * 64 + lane] = rv;
    }
    wave_lds_sync();
    const int prv = act ? prevl[lane] : -1;

    double zm = 0.0, z_last = 0.0, eb_last = 0.0;
    if (r >= 0) {
        zm = cv[(int64_t)r * CV_STRIDE + CV_ZM];
        z_last = cv[(int64_t)r * CV_STRIDE + CV_Z];
        eb_last = cv[(int64_t)r * CV_STRIDE + CV_EB];
    }
    double tsum = 0.0;
    bool bad = false;
    // the step loop's partner schedule, fixed for the call: bit k - 1 of
    // nbmask / cmask is set when the pair (a, (a + k) mod n) is met at partner
    // step k (this segment's steps 1 .. n/2; for even n, at k = n/2 only by the
    // lanes a < n/2) and counts in the nonbonded sum (beyond nb_excl in
    // sequence) / in the contact set (both particles in it, beyond min_sep)
    const int kend = n >> 1, kend_max = W >> 1;
    uint32_t nbmask = 0u, cmask = 0u;
    for (int k = 1; k <= kend_max; ++k) {
        if (act && k <= kend && (2 * k < n || a < kend)) {
            const int b = a + k < n ? a + k : a + k - n;
            const int sep = abs(o - orgl[sbase + b]);
            if (sep > P.nb_excl) nbmask |= 1u << (k - 1);
            if (icon && b < S.nc && sep > P.min_sep) cmask |= 1u << (k - 1);
        }
    }
    // the partner's lane at step 1 and its wrap, the lane each step's j
    // partials come from ((a + 1) mod n: every lane rotates at every step of
    // the widest segment) and the lane holding this particle's partials at the
    // end ((a - kend_max - 1) mod n); lanes without a particle stay on themselves
    const int bl1 = act ? sbase + (a + 1 < n ? a + 1 : 0) : lane;
    const int bl_inc = act ? 1 : 0, bl_wrap = act ? sbase + n : -1;
    const int rot_from = bl1 << 2;
    int home = act ? (a - kend_max - 1) % n : 0;
    home = home < 0 ? home + n : home;
    const int home_from = (act ? sbase + home : lane) << 2;
    const double c1 = P.c1;
    // the particle's update constants (overdamped: mobility dt / (m gamma) and
    // noise amplitude sqrt(2 kT mob); BAOAB: sqrt((1 - c1^2) kT / m))
    const double mob = P.dt * inv_m / P.gamma;
    const double amp = P.integrator == 0 ? sqrt(2.0 * P.kT * mob) : sqrt((1.0 - c1 * c1) * P.kT * inv_m);
    // the sum over the lanes of this lane's segment: a binary tree in a fixed
    // order (lane a takes a + s for s = 1, 2, 4, ... while a is a multiple of
    // 2s), then the segment's first lane's total to every lane, so that all
    // lanes of a replica hold the same value.  Each level's take flag (bit l
    // of seg_take) and partner address are fixed for the call.
    constexpr int SEG_LEVELS = 6;   // W <= 64
    uint32_t seg_take = 0u;
    int seg_from[SEG_LEVELS];
#pragma unroll
    for (int l = 0; l < SEG_LEVELS; ++l) {
        const int s = 1 << l;
        const bool take = s < W && ((a & (2 * s - 1)) == 0) && a + s < n;
        seg_take |= take ? 1u << l : 0u;
        seg_from[l] = (take ? lane + s : lane) << 2;
    }
    auto seg_sum = [&](double val) {
        // an opaque copy: tests of a loop-invariant value would be hoisted out
        // of the step loop as lane masks held in (spilled) scalar registers
        uint32_t tk = seg_take;
        asm volatile("" : "+v"(tk));
#pragma unroll
        for (int l = 0; l < SEG_LEVELS; ++l) {
            if ((1 << l) < W) {   // uniform
                const double o = bpermute_f64(seg_from[l], val);
                val = ((tk >> l) & 1u) ? val + o : val;
            }
        }
        return bpermute_f64(sbase << 2, val);
    };
    for (int64_t m = 0;; ++m) {
        if (record_every > 0 && frames && (m % record_every) == 0 && act) {
            float *fr = frames + (m / record_every) * frame_stride + 3 * rd.off;
            fr[o] = p.x;
            fr[n + o] = p.y;
            fr[2 * n + o] = p.z;
        }
        if (m == n_steps) break;
        posl[lane] = p;
        wave_lds_sync();
        // ---- pair phase: every pair once.  Lane a meets b = (a + k) mod n at
        // step k = 1 .. n/2 (for even n only lanes a < n/2 at k = n/2); its
        // j-side partials belong to particle (a + k) mod n and move one lane
        // back within the segment after each step (ds_bpermute: segments are
        // not DPP rows), and go to their owner lane at the end.
        float fn[3] = {0.f, 0.f, 0.f}, fg[3] = {0.f, 0.f, 0.f}, jn[3] = {0.f, 0.f, 0.f},
              jg[3] = {0.f, 0.f, 0.f}, zt = 0.f;
        int bl = bl1;
        for (int k = 1; k <= kend_max; ++k) {
            const uint32_t bit = 1u << (k - 1);
            const float4 pj = posl[bl];
            float dx, dy, dz;
            const float r2 = pair_r2(p, pj, dx, dy, dz);
            bl += bl_inc;
            bl = bl == bl_wrap ? sbase : bl;
            if constexpr (NBK != 0) {
                const bool nbon = ((nbmask & bit) != 0u) & (!P.has_cut_nb | (r2 <= P.r_cut_nb2));
                const float fs = nb_scalar<NBK>(P, r2, qp, pj.w);
                const float f = nbon ? fs : 0.f;
                fn[0] = fmaf(f, dx, fn[0]);
                fn[1] = fmaf(f, dy, fn[1]);
                fn[2] = fmaf(f, dz, fn[2]);
                jn[0] = fmaf(-f, dx, jn[0]);
                jn[1] = fmaf(-f, dy, jn[1]);
                jn[2] = fmaf(-f, dz, jn[2]);
            }
            const bool con = (cmask & bit) != 0u;
            const bool inside = !P.has_cut | (r2 <= P.r_cut2);   // beyond a cutoff C = 0 (R still counts)
            const float q = r2 * P.inv_r0sq;
            const float q2 = q * q;
            const float t = q + q2;
            const float num = 1.f + t;
            const float den = fmaf(q2, t, num);
            const float inv_den = inside ? frcp(den) : 0.f;
            float diff = num * inv_den - refl[k * 64 + lane];
            diff = con ? diff : 0.f;
            zt = fmaf(diff, diff, zt);
            const float poly = fmaf(q, fmaf(q, fmaf(q, P.cp[0], P.cp[1]), P.cp[2]), P.cp[3]);
            const float g = (diff * (q2 * inv_den)) * (poly * inv_den);
            fg[0] = fmaf(g, dx, fg[0]);
            fg[1] = fmaf(g, dy, fg[1]);
            fg[2] = fmaf(g, dz, fg[2]);
            jg[0] = fmaf(-g, dx, jg[0]);
            jg[1] = fmaf(-g, dy, jg[1]);
            jg[2] = fmaf(-g, dz, jg[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (NBK != 0)
                    jn[c] = __int_as_float(__builtin_amdgcn_ds_bpermute(rot_from, __float_as_int(jn[c])));
                jg[c] = __int_as_float(__builtin_amdgcn_ds_bpermute(rot_from, __float_as_int(jg[c])));
            }
        }
        // lane a now holds the j-side partials of particle (a + kend_max + 1) mod n
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (NBK != 0) fn[c] += __int_as_float(__builtin_amdgcn_ds_bpermute(home_from, __float_as_int(jn[c])));
            fg[c] += __int_as_float(__builtin_amdgcn_ds_bpermute(home_from, __float_as_int(jg[c])));
        }
        double F[3] = {(double)fn[0], (double)fn[1], (double)fn[2]};
        if (P.has_bond) {
            // each bond once, by the lane of its first particle; the second
            // particle's lane takes the opposite force from it
            double f[3] = {0.0, 0.0, 0.0};
            if (nxt >= 0) bond_force(P, p, posl[sbase + nxt], f);
            const int from = (prv >= 0 ? sbase + prv : lane) << 2;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double g = bpermute_f64(from, f[c]);
                F[c] += prv >= 0 ? f[c] - g : f[c];
            }
        }
        // ---- ratchet, eq (FrMD): z_m updated before the force is used ----
        const double z = seg_sum((double)zt);
        zm = fmin(zm, z);
        const double dzr = z - zm;
        const double scale = -P.k_R * dzr;
        z_last = z;
        eb_last = 0.5 * P.k_R * dzr * dzr;
        // ---- Langevin update, float64 per particle ----------------------
        if (act) {
            double fb2 = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double fb = scale * (double)fg[c];
                F[c] += fb;
                fb2 = fma(fb, fb, fb2);
            }
            tsum = fma(fb2, inv_m, tsum);
            double gn[3];
            normals3(P, (uint32_t)o, P.rep_base + (uint32_t)r, step0 + (uint64_t)m, gn[0], gn[1], gn[2]);
            double X[3] = {(double)p.x, (double)p.y, (double)p.z};
            if (P.integrator == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) X[c] += mob * F[c] + amp * gn[c];
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double u = (double)vel[c] + P.dt * F[c] * inv_m;
                    X[c] += 0.5 * P.dt * u;
                    u = c1 * u + amp * gn[c];
                    X[c] += 0.5 * P.dt * u;
                    vel[c] = (float)u;
                }
            }
            p = make_float4((float)X[0], (float)X[1], (float)X[2], p.w);
            bad |= !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z));
        }
        wave_lds_sync();
    }
    if (act) {
        xr[o] = p.x;
        xr[n + o] = p.y;
        xr[2 * n + o] = p.z;
        if (vr) {
            vr[o] = vel[0];
            vr[n + o] = vel[1];
            vr[2 * n + o] = vel[2];
        }
        if (bad) flags[r] = 1;
    }
    // bias functional: T += dt sum_steps sum_i |F_bias,i|^2 / (m_i gamma)
    const double tt = seg_sum(tsum);
    if (r >= 0 && a == 0 && n_steps > 0) {
        cv[(int64_t)r * CV_STRIDE + CV_Z] = z_last;
        cv[(int64_t)r * CV_STRIDE + CV_ZM] = zm;
        cv[(int64_t)r * CV_STRIDE + CV_EB] = eb_last;
        cv[(int64_t)r * CV_STRIDE + CV_T] += P.dt / P.gamma * tt;
    }
}

int packed_width_ok(int n_max) { return n_max >= 2 && n_max <= PACK_WMAX; }
// Without tuning: chains of up to 48 particles (one replica per wavefront at
// most 3/4 full still beats a 64-lane persistent tile, which pads to 64), and
// up to 64 once the batch gives every SIMD (256 CUs x 4) two wavefronts.
int packed_default(int n_max, int n_replicas) {
    return packed_width_ok(n_max) && (4 * n_max <= 3 * PACK_WMAX || n_replicas >= 2048);
}

hipError_t launch_packed_rmd(int waves, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                             int n_max, float *x, float *v, double *cv, int64_t n_steps, uint64_t step0,
                             int record_every, float *frames, int64_t frame_stride, int *flags, hipStream_t st) {
    if (!packed_width_ok(n_max) || waves < 1 || waves > 8) return hipErrorInvalidValue;
    const int W = n_max, per_wg = waves * (64 / W);
    const int grid = (R + per_wg - 1) / per_wg;
    const size_t lds = (size_t)waves * packed_wave_lds_bytes(W);
#define SCPS_LAUNCH(K)                                                                                          \
    hipLaunchKernelGGL((k_rmd_packed<K>), dim3(grid), dim3(64 * waves), lds, st, P, sysd, reps, R, W, x, v, cv, \
                       n_steps, step0, record_every, frames, frame_stride, flags)
    switch (nbk) {
    case 0: SCPS_LAUNCH(0); break;
    case 1: SCPS_LAUNCH(1); break;
    case 2: SCPS_LAUNCH(2); break;
    default: SCPS_LAUNCH(3); break;
    }
#undef SCPS_LAUNCH
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
// k_integrate / k_eval_out, so no two tiles meet on one address).  In
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
    __shared__ int shorg[4][64];       // and its chain indices (read by the per-pair predicates)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = blockIdx.x * 4 + wave;
    const bool live = item < n_items;
    const TileItem it = items[live ? item : 0];
    const RepDesc rd = reps[it.rep];
    const SysDesc S = sysd[rd.sys];
    // PM_NB: nonbonded forces and bonds only (the contact terms come from another pass)
    const int I = it.I, J = it.J, tf = MODE == PM_NB ? (it.flags & ~TF_CONTACT) : it.flags;
    const int n = S.n, n_pad = S.n_pad;
    const float4 *xr2 = xs + 2 * rd.poff;
    {
        const float4 pj = xr2[J * 128 + lane];
        shpos[wave][lane] = pj;
        shpos[wave][64 + lane] = pj;
        shorg[wave][lane] = S.perm[J * 64 + lane];
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
    tile_dispatch<MODE, NBK, 4 * SCPS_PAIR_GROUP>(tf, kb, ke, it.mask, P, lane, A, shpos[wave], shorg[wave],
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
                              const float4 *xs, double *acc, double *zpart, const float *eff,
                              const double *csum) {
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
#define SCPS_MODE(M)                                                                                       \
    launch_pairs_mode<M>(nbk, grid, block, st, P, sysd, reps, items, n_items, xs, acc, zpart, eff, csum)
    switch (mode) {
    case PM_RMD: SCPS_MODE(PM_RMD); break;
    case PM_Z: SCPS_MODE(PM_Z); break;
    case PM_ZG: SCPS_MODE(PM_ZG); break;
    case PM_NB: SCPS_MODE(PM_NB); break;
    default: SCPS_MODE(PM_SCPS); break;
    }
#undef SCPS_MODE
    return hipGetLastError();
}

// z of replica r: the sum of its items' partials zpart[first[r] .. first[r+1])
// (items are stored replica by replica), one wavefront per replica, in a
// fixed order.  Eight partial sums per lane keep eight loads in flight (one
// sum waited on every load: ~10 us for the ~1100 items of a 3000-particle
// chain).
__device__ __forceinline__ double replica_z(const int *__restrict__ first, const double *__restrict__ zpart, int r,
                                           int lane) {
    constexpr int U = 8;
    double z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = 0.0;
    const int end = first[r + 1];
    int t = first[r] + lane;
    for (; t + 64 * (U - 1) < end; t += 64 * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) z[u] += zpart[t + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < U - 1; ++u)   // the rest: at most U - 1 more, one per sum
        if (t + 64 * u < end) z[u] += zpart[t + 64 * u];
    double zl = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) zl += z[u];
    return wave_sum(zl);
}


// ---------------------------------------------------------------------------
// cutoff variant: neighbour lists (per-step rMD path)
// ---------------------------------------------------------------------------
// With both cutoffs set, every particle keeps a full list of the particles
// within r_list = (larger cutoff) + NL_SKIN of it, rebuilt for a replica when
// one of its particles has moved more than NL_SKIN / 2 since the last build
// (whatever moved it: steps, or the caller between calls), so no pair within
// the cutoffs is ever missing.  The host forces a rebuild of every replica
// when the lists are new or the reference map they carry has changed.  The build tests only the tile pairs whose blocks' bounding
// spheres come within r_list.  Entry: x = j | contact << 30 | nonbonded << 29
// (j internal, predicates of the pair), y = the bits of R_ij (float32).
// Skipped contact pairs have C = 0, so
//   z = sum over all counted pairs of R^2 + sum over listed pairs of C (C - 2R)
// and each unordered pair is listed twice (once per side).

// Per block b of replica r (one wavefront): its bounding sphere (centroid of
// its real particles and the largest distance from it) into bounds, and the
// largest squared displacement of its particles since the last build into
// bmax[first[r] + b].
__global__ __launch_bounds__(64) void k_nl_blocks(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                                                  int nb_max, const int *__restrict__ first,
                                                  const float4 *__restrict__ xs, const float4 *__restrict__ xref,
                                                  float4 *__restrict__ bounds, float *__restrict__ bmax) {
    const int b = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
    const RepDesc rd = reps[r];
    const int n = sysd[rd.sys].n, nb = sysd[rd.sys].nb;
    if (b >= nb) return;
    const int i = b * 64 + lane;
    const bool valid = i < n;
    const float4 p = xs[2 * rd.poff + b * 128 + lane];
    float m2 = 0.f;
    if (valid) {
        const float4 q = xref[rd.poff + i];
        const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
        m2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (!(m2 <= 3.0e38f)) m2 = 3.0e38f;           // a non-finite position forces a rebuild
    }
    const double cnt = wave_sum(valid ? 1.0 : 0.0);
    const double cx = wave_sum(valid ? (double)p.x : 0.0) / cnt;
    const double cy = wave_sum(valid ? (double)p.y : 0.0) / cnt;
    const double cz = wave_sum(valid ? (double)p.z : 0.0) / cnt;
    const double dx = (double)p.x - cx, dy = (double)p.y - cy, dz = (double)p.z - cz;
    double d2 = valid ? dx * dx + dy * dy + dz * dz : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d2 = fmax(d2, __shfl_xor(d2, o, 64));
        m2 = fmaxf(m2, __shfl_xor(m2, o, 64));
    }
    if (lane == 0) {
        bounds[(int64_t)r * nb_max + b] = make_float4((float)cx, (float)cy, (float)cz, (float)sqrt(d2));
        bmax[first[r] + b] = m2;
    }
}

// Decide per replica whether to rebuild (force, or a displacement beyond
// NL_SKIN / 2 in any of its blocks); for a rebuild, clear the block's counts
// and record the reference positions.
__global__ __launch_bounds__(64) void k_nl_reset(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                                                 const int *__restrict__ first, const float4 *__restrict__ xs,
                                                 float4 *__restrict__ xref, const float *__restrict__ bmax, int force,
                                                 int *__restrict__ rebuild, int *__restrict__ cnt) {
    const int b = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
    const RepDesc rd = reps[r];
    const int nb = sysd[rd.sys].nb;
    if (b >= nb) return;
    float d2 = 0.f;
    for (int q = lane; q < nb; q += 64) d2 = fmaxf(d2, bmax[first[r] + q]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, o, 64));
    const float half = 0.5f * NL_SKIN;
    const bool rb = force || d2 > half * half;
    if (b == 0 && lane == 0) rebuild[r] = rb;
    if (!rb) return;
    const int i = b * 64 + lane;
    xref[rd.poff + i] = xs[2 * rd.poff + b * 128 + lane];
    cnt[rd.poff + i] = 0;
}

// List build on a fixed grid of NL_BUILD_WG workgroups: wavefront w takes
// the work items g = w (mod all wavefronts) of every rebuilding replica (the
// flags are read 64 replicas at a time), so one replica's rebuild is spread
// over the whole grid and a step without rebuilds costs a few loads.  A
// tile pair whose blocks come
// within r_list is walked twice in the sub-step order of the force kernels
// (lane l meets j = (l + k) mod 64 of block J, read from LDS): the first walk
// counts each lane's i-side entries and, in a counter that rotates with the
// j partner (DPP, as the j-side force partials do), the j-side ones; one
// atomic per particle and tile reserves the slots; the second walk writes
// the entries.  A list that would pass NL_CAP entries marks the replica
// (flags[r] = 2) and keeps its first NL_CAP entries.
constexpr int NL_BUILD_WG = 2048;

__device__ __forceinline__ int rot1i(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x134, 0xF, 0xF, false); }

__global__ __launch_bounds__(256) void k_nl_build(const KParams P, const SysDesc *__restrict__ sysd,
                                                  const RepDesc *__restrict__ reps, int R,
                                                  const TileItem *__restrict__ items,
                                                  const int *__restrict__ first_all, const float4 *__restrict__ xs,
                                                  const float4 *__restrict__ bounds, int nb_max, float r_list,
                                                  const int *__restrict__ rebuild, int *__restrict__ cnt,
                                                  int2 *__restrict__ nl, int *__restrict__ flags) {
    __shared__ float4 shpos[4][128];
    // block J's chain indices and list indices, stored twice like its positions:
    // .x = chain index, .y = j (-1 past the end of the system) with bit 30 set
    // inside the contact set
    __shared__ int2 shorg[4][128];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int W = gridDim.x * 4, w = blockIdx.x * 4 + wave;
    const float rl2 = r_list * r_list;
    for (int r0 = 0; r0 < R; r0 += 64) {
        uint64_t todo = __ballot(r0 + lane < R && rebuild[min(r0 + lane, R - 1)]);
        while (todo) {
            const int r = r0 + __builtin_ctzll(todo);
            todo &= todo - 1;
            const RepDesc rd = reps[r];
            const SysDesc S = sysd[rd.sys];
            const float4 *xr2 = xs + 2 * rd.poff;
            int *ci = cnt + rd.poff;
            int2 *li = nl + rd.poff * (int64_t)NL_CAP;
            const int t0 = first_all[r], t_end = first_all[r + 1];
            for (int t = t0 + ((w - t0) % W + W) % W; t < t_end; t += W) {
                const TileItem it = items[t];
                const int I = it.I, J = it.J;
                if (I != J) {
                    const float4 a = bounds[(int64_t)r * nb_max + I], b = bounds[(int64_t)r * nb_max + J];
                    const double dx = (double)a.x - b.x, dy = (double)a.y - b.y, dz = (double)a.z - b.z;
                    if (sqrt(dx * dx + dy * dy + dz * dz) - (double)a.w - (double)b.w > (double)r_list + 0.01)
                        continue;
                }
                // block J of this wavefront's tile (stored twice: j = lane + k needs no wrap)
                const float4 pjl = xr2[J * 128 + lane];
                shpos[wave][lane] = pjl;
                shpos[wave][64 + lane] = pjl;
                const int jw = J * 64 + lane;
                const int2 orgj = make_int2(S.perm[jw], jw < S.n ? (jw | (jw < S.nc ? 1 << 30 : 0)) : -1);
                shorg[wave][lane] = orgj;
                shorg[wave][64 + lane] = orgj;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int i = I * 64 + lane;
                const float4 pi = xr2[I * 128 + lane];
                const int oi = S.perm[i];
                const bool diag = I == J, ival = i < S.n, icon = i < S.nc;
                // the tag bits of the pair met at sub-step k (0: no entry), without
                // branches; every tile runs all 64 sub-steps, a diagonal tile counting
                // only k = 1..32 (lanes 0..31 at k = 32), so each unordered pair is met
                // once.  Everything that depends on the partner comes from LDS, so
                // nothing per sub-step is loop-invariant (hoisted values of all 64
                // sub-steps would hold 64 registers).
                auto tag_at = [&](int k) -> int {
                    float dx, dy, dz;
                    const float r2 = pair_r2(pi, shpos[wave][lane + k], dx, dy, dz);
                    const int2 oj = shorg[wave][lane + k];
                    const int sep = abs(oi - oj.x);
                    const bool in_tile = !diag | ((k >= 1) & ((k < 32) | ((k == 32) & (lane < 32))));
                    const bool act = ival & (oj.y >= 0) & in_tile & (r2 <= rl2);
                    const int con = (icon & ((oj.y >> 30) & 1) & (sep > P.min_sep)) ? 1 << 30 : 0;
                    const int nbp = (sep > P.nb_excl) ? 1 << 29 : 0;
                    return act ? (con | nbp) : 0;
                };
                // the lane's reference values of this tile stream through a ring of
                // 32 registers: sub-steps 0..31 load before the first walk, so that
                // their latency hides behind it, and the first half of the second
                // walk reloads each slot it has used with the value 32 sub-steps
                // ahead.  HR (a tile inside the contact set, which has a reference
                // tile) is uniform, so the loads are unconditional within a form.
                const float *rt =
                    (I < S.ncb && J < S.ncb) ? S.ref + (int64_t)tile_index(I, J, S.ncb) * 4096 : nullptr;
                auto walks = [&](auto hr) {
                    constexpr bool HR = decltype(hr)::value;
                    float ring[32];
#pragma unroll
                    for (int k = 0; k < 32; ++k) ring[k] = HR ? ldg(rt, k * 64 + lane) : 0.f;
                    // first walk: count the entries, and keep each sub-step's two tag
                    // bits (nonbonded, contact) in tb for the second walk
                    // (16 sub-steps per word; after the four blocks tb[3 - q] holds
                    // block q, the words having moved down one place per block)
                    uint32_t tb[4] = {0u, 0u, 0u, 0u};
                    int n_i = 0, n_j = 0;
#pragma unroll 1
                    for (int q = 0; q < 4; ++q) {
                        uint32_t cur = 0u;
#pragma unroll
                        for (int kk = 0; kk < 16; ++kk) {
                            const uint32_t b = (uint32_t)tag_at(16 * q + kk) >> 29;
                            cur |= b << (2 * kk);
                            const int hit = b != 0u;
                            n_i += hit;
                            n_j = rot1i(n_j + hit);
                            if ((kk & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                        }
                        tb[3] = tb[2];
                        tb[2] = tb[1];
                        tb[1] = tb[0];
                        tb[0] = cur;
                    }
                    // after 64 rotations lane l holds the j-side count of particle l of block J
                    const int base_i = n_i ? atomicAdd(&ci[i], n_i) : 0;
                    const int base_j = n_j ? atomicAdd(&ci[J * 64 + lane], n_j) : 0;
                    if (base_i + n_i > NL_CAP || base_j + n_j > NL_CAP) flags[r] = 2;
                    // second walk, over the kept tags: the j-side write offset travels
                    // with its particle
                    int o_i = base_i, o_j = base_j;
                    auto put = [&](const int k, const float Rk) {
                        const uint32_t b = (tb[3 - (k >> 4)] >> (2 * (k & 15))) & 3u;
                        if (b) {
                            const int j = shorg[wave][lane + k].y & 0x1FFFFFFF, tag = (int)(b << 29);
                            const float Rv = (b & 2u) ? Rk : 0.f;
                            if (o_i < NL_CAP) li[(int64_t)i * NL_CAP + o_i] = make_int2(j | tag, __float_as_int(Rv));
                            if (o_j < NL_CAP) li[(int64_t)j * NL_CAP + o_j] = make_int2(i | tag, __float_as_int(Rv));
                            ++o_i;
                            ++o_j;
                        }
                        o_j = rot1i(o_j);
                    };
#pragma unroll
                    for (int k = 0; k < 32; ++k) {
                        const float Rk = ring[k];
                        if constexpr (HR) ring[k] = ldg(rt, (32 + k) * 64 + lane);
                        put(k, Rk);
                        // issue the reloads as the slots free up, not all at once
                        if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                    }
#pragma unroll
                    for (int k = 32; k < 64; ++k) put(k, ring[k - 32]);
                };
                if (rt)
                    walks(std::true_type{});
                else
                    walks(std::false_type{});
                __builtin_amdgcn_wave_barrier();   // shpos / shorg are rewritten for the next tile
            }
        }
    }
}

// Forces and z over the lists.  NL_LANES lanes share a particle and take its
// entries e = t, t + NL_LANES, ... (consecutive entries, so a wavefront's
// loads are coalesced per particle); a workgroup of 256 threads covers
// 256 / NL_LANES particles.  Only i's side of each listed pair is added (the
// pair is listed for j as well).  zpart[first[r] + chunk] = the chunk's sum
// of C (C - 2R) / 2.
constexpr int NL_LANES = 4;
constexpr int NL_CHUNK = 256 / NL_LANES;
constexpr int NL_BATCH = 8;
template <int NBK>
__global__ __launch_bounds__(256) void k_nl_force(const KParams P, const SysDesc *__restrict__ sysd,
                                                  const RepDesc *__restrict__ reps, const int *__restrict__ first,
                                                  const float4 *__restrict__ xs, const int *__restrict__ cnt,
                                                  const int2 *__restrict__ nl, double *__restrict__ acc,
                                                  double *__restrict__ zpart) {
    __shared__ double zw[4];
    const int chunk = blockIdx.x, r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    if (chunk * NL_CHUNK >= S.n_pad) return;
    const int tid = threadIdx.x, t = tid % NL_LANES;
    const int i = chunk * NL_CHUNK + tid / NL_LANES;
    const float4 *xr2 = xs + 2 * rd.poff;
    const float4 pi = xr2[dup_index(i)];
    const float qp = P.dh_pref * pi.w;
    const int m = i < S.n ? min(cnt[rd.poff + i], NL_CAP) : 0;
    const int2 *li = nl + (rd.poff + i) * (int64_t)NL_CAP;
    float f[3] = {0.f, 0.f, 0.f}, g[3] = {0.f, 0.f, 0.f};
    float zt = 0.f;
    // NL_BATCH entries per lane at a time: their list loads, then their
    // position gathers, are all issued before the first pair is computed, so
    // each wave keeps NL_BATCH dependent load pairs in flight instead of one.
    // Slots past the end read as (particle 0, no tag) and add nothing.
    for (int e0 = t; e0 < m; e0 += NL_BATCH * NL_LANES) {
        int2 en[NL_BATCH];
        float4 pj[NL_BATCH];
#pragma unroll
        for (int u = 0; u < NL_BATCH; ++u) {
            const int e = e0 + u * NL_LANES;
            en[u] = e < m ? li[e] : make_int2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < NL_BATCH; ++u) pj[u] = xr2[dup_index(en[u].x & 0x1FFFFFFF)];
#pragma unroll
        for (int u = 0; u < NL_BATCH; ++u) {
            float dx, dy, dz;
            const float r2 = pair_r2(pi, pj[u], dx, dy, dz);
            if (NBK != 0 && (en[u].x & (1 << 29)) && (!P.has_cut_nb || r2 <= P.r_cut_nb2)) {
                const float s = nb_scalar<NBK>(P, r2, qp, pj[u].w);
                f[0] = fmaf(s, dx, f[0]);
                f[1] = fmaf(s, dy, f[1]);
                f[2] = fmaf(s, dz, f[2]);
            }
            if (en[u].x & (1 << 30)) {
                const float R = __int_as_float(en[u].y);
                const float q = r2 * P.inv_r0sq;
                const float q2 = q * q;
                const float t = q + q2;             // num = 1 + t, den = num + q^2 t
                const float num = 1.f + t;
                const float den = fmaf(q2, t, num);
                const float inv_den = (!P.has_cut || r2 <= P.r_cut2) ? frcp(den) : 0.f;
                const float C = num * inv_den;
                zt = fmaf(C, C - 2.f * R, zt);
                const float poly = fmaf(q, fmaf(q, fmaf(q, P.cp[0], P.cp[1]), P.cp[2]), P.cp[3]);
                const float gg = ((C - R) * (q2 * inv_den)) * (poly * inv_den);
                g[0] = fmaf(gg, dx, g[0]);
                g[1] = fmaf(gg, dy, g[1]);
                g[2] = fmaf(gg, dz, g[2]);
            }
        }
    }
#pragma unroll
    for (int o = 1; o < NL_LANES; o <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f[c] += __shfl_xor(f[c], o, 64);
            g[c] += __shfl_xor(g[c], o, 64);
        }
    }
    double *ar = acc + 6 * rd.poff;
    if (t == 0 && i < S.n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            unsafeAtomicAdd(&ar[c * S.n_pad + i], (double)f[c]);
            unsafeAtomicAdd(&ar[(3 + c) * S.n_pad + i], (double)g[c]);
        }
        if (P.has_bond) {
            const int bn = S.bond_next[i];
            if (bn >= 0) {
                double fb[3];
                bond_force(P, pi, xr2[dup_index(bn)], fb);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unsafeAtomicAdd(&ar[c * S.n_pad + i], fb[c]);
                    unsafeAtomicAdd(&ar[c * S.n_pad + bn], -fb[c]);
                }
            }
        }
    }
    const double w = wave_sum(0.5 * (double)zt);
    if ((tid & 63) == 0) zw[tid >> 6] = w;
    __syncthreads();
    if (tid == 0) zpart[first[r] + chunk] = (zw[0] + zw[1]) + (zw[2] + zw[3]);
}

hipError_t launch_nl_update(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R, int nb_max,
                            const int *first_blk, const float4 *xs, float4 *bounds, float4 *xref, float *bmax,
                            int *rebuild, int force, const TileItem *items_all, const int *first_all, float r_list,
                            int *cnt, int2 *nl, int *flags, hipStream_t st) {
    const dim3 blocks(nb_max, R);
    hipLaunchKernelGGL(k_nl_blocks, blocks, dim3(64), 0, st, sysd, reps, nb_max, first_blk, xs, xref, bounds, bmax);
    hipLaunchKernelGGL(k_nl_reset, blocks, dim3(64), 0, st, sysd, reps, first_blk, xs, xref, bmax, force, rebuild,
                       cnt);
    hipLaunchKernelGGL(k_nl_build, dim3(NL_BUILD_WG), dim3(256), 0, st, P, sysd, reps, R, items_all, first_all, xs,
                       bounds, nb_max, r_list, rebuild, cnt, nl, flags);
    return hipGetLastError();
}

int nl_chunks(int n_pad) { return (n_pad + NL_CHUNK - 1) / NL_CHUNK; }

hipError_t launch_nl_force(int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                           int n_pad_max, const int *first_chunk, const float4 *xs, const int *cnt, const int2 *nl,
                           double *acc, double *zpart, hipStream_t st) {
    const dim3 blocks(nl_chunks(n_pad_max), R);
#define SCPS_NL(K)                                                                                      \
    hipLaunchKernelGGL(k_nl_force<K>, blocks, dim3(256), 0, st, P, sysd, reps, first_chunk, xs, cnt, nl, acc, \
                       zpart)
    switch (nbk) {
    case 0: SCPS_NL(0); break;
    case 1: SCPS_NL(1); break;
    case 2: SCPS_NL(2); break;
    default: SCPS_NL(3); break;
    }
#undef SCPS_NL
    return hipGetLastError();
}


// SCPS tube variables per replica (one wavefront each), from the squared
// distances d_k Z0 = sum_p (C_p - R_kp)^2 to every frame k = 0..M of the
// stack, assembled in float64 around the replica's reference frame j as
// Q + 2 (X_j - X_k) + G_jk (Q = sum (C - R_j)^2 and X_k = sum (C - R_j) R_k
// from k_scps_dist, G_jk = sum (R_j - R_k)^2 of the stack; see tube_sums):
//   s = 1 - (1/M) sum_k k p_k,  w = -wscale log sum_k exp(-lambda d_k),
//   p_k = softmax(-lambda d_k), wscale = 1/lambda (eq (wX)) or 1 (eq (awXa));
//   ratchets on s and w, eqs (Fw),(Fs).
// The bias force is -sum_k c_k grad d_k with
//   c_k = p_k [k_s (s - s_m)(lambda/M)(k - kbar) + k_w (w - w_m) lambda wscale];
// coef receives c_k / Z0 and csum sum_k c_k / Z0 for the gradient pass, and
// jref[r] the frame of largest weight, the reference of the next step's
// distance pass.  X and Q are consumed and cleared.
__global__ void k_finalize_scps(const KParams P, const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                                const int kmax, int *__restrict__ jref, double *__restrict__ X,
                                double *__restrict__ Q, double *__restrict__ cv, float *__restrict__ coef,
                                double *__restrict__ csum) {
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const SysDesc S = sysd[reps[r].sys];
    const int K = S.K, M = K - 1;
    double *xr = X + (int64_t)r * kmax;
    const double lam = P.lambda;
    const int j = ref_frame(jref, r, K);
    const TubeSums ts = tube_sums(lane, K, Q[r], xr, j, S.G + (int64_t)j * K, S.Z0, lam);
    const double *e = ts.e;
    const double a = ts.a, s0 = ts.s0, s1 = ts.s1;
    const double kbar = s1 / s0;
    const double sv = 1.0 - kbar / (double)M;
    const double wv = tube_w(a, s0, P.wscale);
    const double lw = lam * P.wscale;   // dw/dd_k = lw p_k
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
            const double ckv = pk * (P.k_s * ds * (lam / (double)M) * ((double)k - kbar) + P.k_w * dw * lw);
            coef[(int64_t)r * kmax + k] = (float)(ckv / S.Z0);
            tot += ckv;
            xr[k] = 0.0;
        }
    }
    tot = wave_sum(tot);
    if (lane == 0) {
        Q[r] = 0.0;
        csum[r] = tot / S.Z0;
        if (jref) jref[r] = ts.kmax;
        c[CV_S] = sv;
        c[CV_W] = wv;
        c[CV_SM] = sm;
        c[CV_WM] = wm;
        c[CV_EB] = 0.5 * P.k_s * ds * ds + 0.5 * P.k_w * dw * dw;
    }
}

hipError_t launch_finalize_scps(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R, int kmax,
                                int *jref, double *X, double *Q, double *cv, float *coef, double *csum,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_finalize_scps, dim3(R), dim3(64), 0, st, P, sysd, reps, kmax, jref, X, Q, cv, coef, csum);
    return hipGetLastError();
}

// Langevin update of every particle; consumes and clears the accumulators.
// The force is acc[0..2] + scale[r] * acc[3..5], the second term being the
// bias; each workgroup adds its particles' dt |F_bias|^2 / (m gamma) to the
// replica's bias functional cv[r][CV_T].  The noise is drawn for step
// step_off + *step_base (step_base: nullable device word, so that a captured
// sequence of steps can be replayed from any step).
__global__ __launch_bounds__(256) void k_integrate(const KParams P, const SysDesc *__restrict__ sysd,
                                                   const RepDesc *__restrict__ reps, float4 *__restrict__ xs,
                                                   float4 *__restrict__ vs, double *__restrict__ acc,
                                                   const double *__restrict__ scale, double *__restrict__ cv,
                                                   const uint64_t step_off, const uint64_t *__restrict__ step_base,
                                                   int *__restrict__ flags, const int *__restrict__ zfirst,
                                                   const double *__restrict__ zpart, const double *__restrict__ zbase) {
    __shared__ double tred[4];
    __shared__ double sh_scale;
    const uint64_t step = step_off + (step_base ? *step_base : 0u);
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const SysDesc S = sysd[rd.sys];
    if ((int)(blockIdx.x * blockDim.x) >= S.n) return;   // past a shorter chain's particles (uniform)
    if (zpart) {
        // the rMD ratchet, eq (FrMD), in every workgroup of the replica: z from
        // its partials (the same fixed-order sum in each), z_m updated before
        // the force is used; column 0 writes cvstate (a workgroup that reads
        // the z_m column 0 has already written computes the same min again)
        if (threadIdx.x < 64) {
            const double z = (zbase ? zbase[r] : 0.0) + replica_z(zfirst, zpart, r, threadIdx.x);
            if (threadIdx.x == 0) {
                double *c = cv + (int64_t)r * CV_STRIDE;
                // z_m is read here while column 0 may be writing it: both as
                // relaxed atomics, so either value is read whole
                const double zm =
                    fmin(__hip_atomic_load(&c[CV_ZM], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), z);
                const double dz = z - zm;
                if (blockIdx.x == 0) {
                    c[CV_Z] = z;
                    __hip_atomic_store(&c[CV_ZM], zm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    c[CV_EB] = 0.5 * P.k_R * dz * dz;
                }
                sh_scale = -P.k_R * dz;
            }
        }
        __syncthreads();
    }
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double tb = 0.0;
    if (a < S.n) {
        const int n_pad = S.n_pad;
        double *ar = acc + 6 * rd.poff;
        const double sc = zpart ? sh_scale : scale[r];
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
                            const uint64_t *step_base, int *flags, hipStream_t st, const int *zfirst,
                            const double *zpart, const double *zbase) {
    hipLaunchKernelGGL(k_integrate, dim3((n_pad_max + 255) / 256, R), dim3(256), 0, st, P, sysd, reps, xs, vs, acc,
                       scale, cv, step, step_base, flags, zfirst, zpart, zbase);
    return hipGetLastError();
}

__global__ void k_set_step(uint64_t *__restrict__ d, const uint64_t v) { *d = v; }

hipError_t launch_set_step(uint64_t *d, uint64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, st, d, v);
    return hipGetLastError();
}

// Output of the z pass (eval_z_and_grad, eval_zbias), one launch: the first
// wavefront of column 0 sums replica r's z partials into z[r] and, when zm is
// given, writes the ratchet energy Eb[r] = 1/2 k_R (z - z_m)^2 theta(z - z_m)
// (eq (FrMD)); when grad is given, every column writes coef * grad z out of the
// accumulators and clears them.  The grid has one column without grad.
__global__ void k_eval_out(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                           const int *__restrict__ first, const double *__restrict__ zpart, double *__restrict__ z_out,
                           const double k_R, const double *__restrict__ zm, double *__restrict__ Eb,
                           double *__restrict__ acc, float *__restrict__ grad, const double *__restrict__ grad_coef) {
    const int r = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        const double z = replica_z(first, zpart, r, threadIdx.x);
        if (threadIdx.x == 0) {
            z_out[r] = z;
            if (zm) {
                const double d = z - zm[r];
                const double th = d >= 0.0 ? 1.0 : 0.0;  // theta(0) = 1
                Eb[r] = 0.5 * k_R * d * d * th;
            }
        }
    }
    if (!grad) return;
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
                           const int *first, const double *zpart, double *z_out, double k_R, const double *zm,
                           double *Eb, float *grad, const double *grad_coef, hipStream_t st) {
    const int cols = grad ? (n_pad_max + 255) / 256 : 1;
    hipLaunchKernelGGL(k_eval_out, dim3(cols, R), dim3(256), 0, st, sysd, reps, first, zpart, z_out, k_R, zm, Eb, acc,
                       grad, grad_coef);
    return hipGetLastError();
}

// grad_x = grad_z * (g_z + g_E k_R (z - z_m) theta(z - z_m)) over replica r's
// coordinates (x layout), for every replica: the backward of z and E_b from
// a kept dz/dx in one launch.  g_z and g_E are read with element strides
// (0: one value for all replicas) and may be NULL (taken as 0).
__global__ void k_zbias_backward(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps, const double k_R,
                                 const double *__restrict__ z, const double *__restrict__ zm,
                                 const double *__restrict__ gz, const int64_t sz, const double *__restrict__ gE,
                                 const int64_t sE, const float *__restrict__ in, float *__restrict__ out) {
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const int n3 = 3 * sysd[rd.sys].n;
    const double d = z[r] - zm[r];
    const double th = d >= 0.0 ? 1.0 : 0.0;  // theta(0) = 1
    const double c = (gz ? gz[r * sz] : 0.0) + (gE ? gE[r * sE] : 0.0) * k_R * d * th;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += gridDim.x * blockDim.x)
        out[3 * rd.off + e] = (float)(c * (double)in[3 * rd.off + e]);
}

hipError_t launch_zbias_backward(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, double k_R,
                                 const double *z, const double *zm, const double *gz, int64_t sz, const double *gE,
                                 int64_t sE, const float *in, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_zbias_backward, dim3((3 * n_pad_max + 255) / 256, R), dim3(256), 0, st, sysd, reps, k_R, z,
                       zm, gz, sz, gE, sE, in, out);
    return hipGetLastError();
}

// out = coef[r] * in over replica r's coordinates (x layout), for every
// replica: the backward of the z wrapper from a kept dz/dx.
__global__ void k_scale_by_replica(const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
                                   const float *__restrict__ in, const double *__restrict__ coef,
                                   float *__restrict__ out) {
    const int r = blockIdx.y;
    const RepDesc rd = reps[r];
    const int n3 = 3 * sysd[rd.sys].n;
    const double c = coef[r];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n3; e += gridDim.x * blockDim.x)
        out[3 * rd.off + e] = (float)(c * (double)in[3 * rd.off + e]);
}

hipError_t launch_scale_by_replica(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, const float *in,
                                   const double *coef, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_by_replica, dim3((3 * n_pad_max + 255) / 256, R), dim3(256), 0, st, sysd, reps, in,
                       coef, out);
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

// Least-biased path: the replica with the smallest bias functional T[X]
// (cvstate slot CV_T) among the listed ones, ties to the lowest replica id.
// One workgroup; out_i = {index, number of listed replicas with a non-finite T},
// out_t = that replica's T.
__global__ __launch_bounds__(256) void k_least_biased(const double *__restrict__ cv, const int *__restrict__ list,
                                                      int n, int *__restrict__ out_i, double *__restrict__ out_t) {
    __shared__ double st[256];
    __shared__ int si[256], sbad[256];
    const int tid = threadIdx.x;
    double best = INFINITY;
    int bi = INT_MAX, bad = 0;
    for (int s = tid; s < n; s += 256) {
        const int r = list[s];
        const double t = cv[(int64_t)r * CV_STRIDE + CV_T];
        if (!isfinite(t)) {
            ++bad;
        } else if (t < best || (t == best && r < bi)) {
            best = t;
            bi = r;
        }
    }
    st[tid] = best;
    si[tid] = bi;
    sbad[tid] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            const double t = st[tid + h];
            const int r = si[tid + h];
            if (t < st[tid] || (t == st[tid] && r < si[tid])) {
                st[tid] = t;
                si[tid] = r;
            }
            sbad[tid] += sbad[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out_i[0] = si[0];
        out_i[1] = sbad[0];
        out_t[0] = st[0];
    }
}

hipError_t launch_least_biased(const double *cv, const int *list, int n, int *out_i, double *out_t, hipStream_t st) {
    hipLaunchKernelGGL(k_least_biased, dim3(1), dim3(256), 0, st, cv, list, n, out_i, out_t);
    return hipGetLastError();
}

}  // namespace scps
