// HIP kernels for gfx950: reference contact maps and the SCPS tube-variable
// passes on matrix cores.
//
// Contact maps are stored per system as float32 tiles of 64 x 64 contact
// pairs in the diagonal-major layout of the stepping kernels: element [s][l]
// of tile (I, J) is the pair (64 I + l, 64 J + ((l + s) mod 64)) of the
// contact set's internal order.  A stack of K frame maps is tile-major,
// [tile][K][4096]; the SCPS passes read a pair-major copy [tile][4096][K4]
// (K4 = K rounded up to a multiple of 4, zero-padded).
//
// Reference maps, eq (avCij) of Orioli, a Beccara, Faccioli
// (arXiv:1705.02180): R_k(i, j) is the mean over the successful paths of the
// contact function C at frame k, with C(q) = (1 + q + q^2) / (1 + q + q^2 +
// q^3 + q^4), q = (r/r0)^2.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "scps_device.h"
#include "scps_internal.h"

namespace scps {

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

// The sum over the packed contact pairs a < b with |perm[a] - perm[b]| >
// min_sep of v^2: one workgroup per row a into part[a], then the rows in
// order.  perm[a] is the chain index of contact position a.
__global__ void k_sum_squares_sep(int nc, int min_sep, const int *__restrict__ perm, const double *__restrict__ v,
                                  double *__restrict__ part) {
    __shared__ double red[4];
    const int a = blockIdx.x;
    const int oa = perm[a];
    const double *row = v + (packed_index(nc, a, a + 1) - (a + 1));   // row[b] = v(a, b) for b > a
    double s = 0.0;
    for (int b = a + 1 + threadIdx.x; b < nc; b += blockDim.x)
        if (abs(oa - perm[b]) > min_sep) s += row[b] * row[b];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[a] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sum_squares_sep(int nc, int min_sep, const int *perm, const double *v, double *part, double *out,
                                  hipStream_t st) {
    if (nc < 2) {
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, 0, part, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_sum_squares_sep, dim3(nc), dim3(256), 0, st, nc, min_sep, perm, v, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, nc, part, out);
    return hipGetLastError();
}

// Contact function in float64 with the quotient from the hardware reciprocal
// estimate: two Newton steps r <- r (2 - den r), then one residual correction
// of num * r.  den >= 1 here, so no scaling or special cases are needed; the
// result is within an ulp or two of the correctly rounded quotient.
__device__ __forceinline__ double contact_f64_fast(double r2, double inv_r0sq) {
    const double q = r2 * inv_r0sq;
    const double q2 = q * q;
    const double t = q + q2;
    const double num = t + 1.0;
    const double den = fma(q2, t, num);
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double c = num * r;
    return fma(fma(-den, c, num), r, c);
}

#ifndef UPDREF_PATHS
#define UPDREF_PATHS 8
#endif
// eq (avCij): mean over successful paths of C(X_p(t_k)), float64 sums.
// Grid (contact tile pair, frame); thread (w, l) owns rows k = 16 w .. 16 w + 15
// of the diagonal-major tile.  The positions of blocks I and J of
// UPDREF_PATHS paths at a time are staged in LDS as float64 components (the
// differences of float32 coordinates are then exact); every thread adds its
// 16 contact values per path in path order, so the sums do not depend on the
// launch shape.
template <bool CUT>
__global__ __launch_bounds__(256) void k_update_reference(int n, int nc, int ncb, const int *__restrict__ perm,
                                                          const float *__restrict__ frames, int n_paths,
                                                          const int *__restrict__ succ, int n_succ,
                                                          double inv_r0sq, double r_cut2, float *__restrict__ tiles,
                                                          double *__restrict__ packed) {
    constexpr int PB = UPDREF_PATHS;
    __shared__ double pos[2][3][PB][64];   // [block I/J][component][path][particle]
    const int tile = blockIdx.x, f = blockIdx.y;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int a = I * 64 + l;
    double sum[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) sum[k] = 0.0;
    for (int s0 = 0; s0 < n_succ; s0 += PB) {
        const int np = min(PB, n_succ - s0);
        __syncthreads();
        for (int e = tid; e < 2 * PB * 64; e += 256) {
            const int which = e / (PB * 64), pp = (e >> 6) % PB, c = (which ? J : I) * 64 + (e & 63);
            double x = 0.0, y = 0.0, z = 0.0;
            if (pp < np && c < nc) {
                const float *X = frames + ((int64_t)f * n_paths + succ[s0 + pp]) * 3 * (int64_t)n;
                const int o = perm[c];
                x = X[o];
                y = X[n + o];
                z = X[2 * n + o];
            }
            pos[which][0][pp][e & 63] = x;
            pos[which][1][pp][e & 63] = y;
            pos[which][2][pp][e & 63] = z;
        }
        __syncthreads();
        for (int pp = 0; pp < np; ++pp) {
            const double ax = pos[0][0][pp][l], ay = pos[0][1][pp][l], az = pos[0][2][pp][l];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int j = (l + w * 16 + kk) & 63;
                const double dx = ax - pos[1][0][pp][j];
                const double dy = ay - pos[1][1][pp][j];
                const double dz = az - pos[1][2][pp][j];
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const double c = contact_f64_fast(r2, inv_r0sq);
                sum[kk] += (CUT && r2 > r_cut2) ? 0.0 : c;
            }
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
    const double inv_r0sq = 1.0 / (r0 * r0);
    if (r_cut > 0.0)
        hipLaunchKernelGGL(k_update_reference<true>, dim3(nt, n_frames), dim3(256), 0, st, n, nc, ncb, perm_dev,
                           frames, n_paths, succ_idx, n_succ, inv_r0sq, r_cut * r_cut, tiles, packed);
    else
        hipLaunchKernelGGL(k_update_reference<false>, dim3(nt, n_frames), dim3(256), 0, st, n, nc, ncb, perm_dev,
                           frames, n_paths, succ_idx, n_succ, inv_r0sq, 0.0, tiles, packed);
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

// Per contact tile of a map [tile][4096]: the float64 sum of the squared
// entries over the tile's counted pairs (both in the contact set, beyond
// min_seq_sep, each unordered pair once).  One workgroup per tile; thread
// (w, l) takes sub-steps s = w, w + 4, ... of column l.
__global__ __launch_bounds__(256) void k_tile_sumsq(int nc, int ncb, int min_sep, const int *__restrict__ perm,
                                                    const float *__restrict__ tiles, double *__restrict__ out) {
    __shared__ double ws[4];
    const int tile = blockIdx.x;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int a = I * 64 + l;
    const float *t = tiles + (int64_t)tile * 4096;
    double sum = 0.0;
    for (int s = w; s < 64; s += 4) {
        const int b = J * 64 + ((l + s) & 63);
        if (a < nc && b < nc && tile_pair_counts(I == J, s, l) && abs(perm[a] - perm[b]) > min_sep) {
            const double v = t[s * 64 + l];
            sum = fma(v, v, sum);
        }
    }
    sum = wave_sum(sum);
    if (l == 0) ws[w] = sum;
    __syncthreads();
    if (tid == 0) out[tile] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

hipError_t launch_tile_sumsq(int nc, int ncb, int min_sep, const int *perm, const float *tiles, double *out,
                             hipStream_t st) {
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_sumsq, dim3(nt), dim3(256), 0, st, nc, ncb, min_sep, perm, tiles, out);
    return hipGetLastError();
}

// Pair-major copy of a frame stack: stack_pm[tile][p][k] = stack[tile][k][p]
// for k < K (zero for K <= k < K4).  Grid (tile, STACKPM_SPLIT): each
// workgroup transposes 64 / STACKPM_SPLIT sub-steps of one tile, 64 pairs at
// a time through LDS; thread (w, l) reads rows k = w, w + 4, ...
#ifndef STACKPM_SPLIT
#define STACKPM_SPLIT 1
#endif
__global__ __launch_bounds__(256) void k_stack_pairmajor(int K, const float *__restrict__ stack,
                                                         float *__restrict__ stack_pm) {
    __shared__ float buf[64][KMAX + 1];
    const int tile = blockIdx.x;
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int K4 = stack_pm_width(K);
    const int per = 64 / STACKPM_SPLIT, s_beg = blockIdx.y * per;
    const float *src = stack + (int64_t)tile * K * 4096 + l;
    for (int s = s_beg; s < s_beg + per; ++s) {
        __syncthreads();
        for (int k = w; k < K; k += 4) buf[l][k] = src[(int64_t)k * 4096 + s * 64];
        __syncthreads();
        float *out = stack_pm + ((int64_t)tile * 4096 + s * 64) * K4;
        for (int e = tid; e < 64 * K4; e += 256) {
            const int pl = e / K4, k = e - pl * K4;
            out[e] = k < K ? buf[pl][k] : 0.f;
        }
    }
}

hipError_t launch_stack_pairmajor(int nc, int ncb, int K, const float *stack, float *stack_pm, hipStream_t st) {
    (void)nc;
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0 || K == 0) return hipSuccess;
    if (K > KMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stack_pairmajor, dim3(nt, STACKPM_SPLIT), dim3(256), 0, st, K, stack, stack_pm);
    return hipGetLastError();
}

// The stack's frame distances G[j][k] = sum over the counted contact pairs
// (both in the contact set, beyond min_seq_sep, each unordered pair once) of
// (R_jp - R_kp)^2, in float64 from the float32 frames (differences of float32
// values are exact in float64), for j != k; the diagonal stays 0.  Grid
// (tile, chunk): the workgroup stages the K frames of 64 pairs at a time in
// LDS and each thread adds GRAM_EPT frame pairs j < k, numbered row by row,
// over them; one float64 atomic per frame pair and workgroup at the end
// (both G[j][k] and G[k][j]).  G must be zero on entry.
constexpr int GRAM_EPT = 8;
__global__ __launch_bounds__(256) void k_stack_gram(int nc, int ncb, int K, int min_sep,
                                                    const int *__restrict__ perm, const float *__restrict__ stack,
                                                    double *__restrict__ G) {
    __shared__ float buf[64][KMAX + 1];
    __shared__ int cnt[64];
    __shared__ int orig[2][64];
    const int tile = blockIdx.x;
    int I, J;
    tile_decode(tile, ncb, I, J);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid < 128) {
        const int c = ((tid >> 6) ? J : I) * 64 + l;
        orig[tid >> 6][l] = c < nc ? perm[c] : 0;
    }
    const int E = K * (K - 1) / 2;
    int fj[GRAM_EPT], fk[GRAM_EPT];
    double acc[GRAM_EPT];
#pragma unroll
    for (int m = 0; m < GRAM_EPT; ++m) {
        int e = (blockIdx.y * GRAM_EPT + m) * 256 + tid;
        int j = 0, k = 0;   // an entry past the end reads frame 0 twice and adds 0
        if (e < E) {
            while (e >= K - 1 - j) {
                e -= K - 1 - j;
                ++j;
            }
            k = j + 1 + e;
        }
        fj[m] = j;
        fk[m] = k;
        acc[m] = 0.0;
    }
    const float *src = stack + (int64_t)tile * K * 4096 + l;
    for (int s = 0; s < 64; ++s) {
        __syncthreads();
        for (int k = w; k < K; k += 4) buf[l][k] = src[(int64_t)k * 4096 + s * 64];
        if (w == 0) {
            const int a = I * 64 + l, jl = (l + s) & 63, b = J * 64 + jl;
            cnt[l] = a < nc && b < nc && tile_pair_counts(I == J, s, l) && abs(orig[0][l] - orig[1][jl]) > min_sep;
        }
        __syncthreads();
        for (int p = 0; p < 64; ++p) {
            if (!cnt[p]) continue;   // uniform across the workgroup
#pragma unroll
            for (int m = 0; m < GRAM_EPT; ++m) {
                const double d = (double)buf[p][fj[m]] - (double)buf[p][fk[m]];
                acc[m] = fma(d, d, acc[m]);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < GRAM_EPT; ++m)
        if (fj[m] != fk[m]) {
            unsafeAtomicAdd(&G[fj[m] * K + fk[m]], acc[m]);
            unsafeAtomicAdd(&G[fk[m] * K + fj[m]], acc[m]);
        }
}

hipError_t launch_stack_gram(int nc, int ncb, int K, int min_sep, const int *perm, const float *stack, double *G,
                             hipStream_t st) {
    const int nt = ncb * (ncb + 1) / 2;
    if (nt == 0 || K < 2) return hipSuccess;
    if (K > KMAX) return hipErrorInvalidValue;
    const int E = K * (K - 1) / 2, chunks = (E + GRAM_EPT * 256 - 1) / (GRAM_EPT * 256);
    hipLaunchKernelGGL(k_stack_gram, dim3(nt, chunks), dim3(256), 0, st, nc, ncb, K, min_sep, perm, stack, G);
    return hipGetLastError();
}

// Contact value of one replica-pair for the MFMA operand (0 when the pair
// does not count).  CUT: test the contact cutoff (a cutoff marks every
// contact tile MASK, so the other tiles need no test).
template <bool CUT>
__device__ __forceinline__ float contact_operand(const KParams &P, const float4 &pi, const float4 &pj, bool ok) {
    float dx, dy, dz;
    const float r2 = pair_r2(pi, pj, dx, dy, dz);
    const float q = r2 * P.inv_r0sq;
    const float q2 = q * q;
    const float t = q + q2;   // num = 1 + t, den = num + q^2 t
    const float num = 1.f + t;
    const float den = fmaf(q2, t, num);
    const bool inside = CUT ? (!P.has_cut | (r2 <= P.r_cut2)) : true;
    return (ok & inside) ? num * frcp(den) : 0.f;
}

#ifndef SCPS_DIST_AHEAD
#define SCPS_DIST_AHEAD 8
#endif
#ifndef SCPS_DIST_REF_AHEAD
#define SCPS_DIST_REF_AHEAD 4   // the reference values ride a shorter ring (registers)
#endif
#ifndef SCPS_DIST_REF_GLOBAL
#define SCPS_DIST_REF_GLOBAL 0  // 1: R_j from its own load also for stacks of at most 64 frames
#endif
// Pass 1, around each replica's reference frame j_r (see tube_sums): with
// u_rp = C_rp - R_{j_r}p, X[r][k] += sum_p u_rp R_kp and Q[r] += sum_p u_rp^2
// over the contact pairs of each work item (group of replicas, tile);
// workgroups stride over the items and flush their sums when the group
// changes and at the end.
// The pairs of a tile are taken row by row: wavefront w takes rows
// i = w, w+4, ... of block I and, per row, 32 MFMA steps of 2 pairs
// (i, 2m + (l >> 5)); lane l evaluates u of that pair for replica l & 31 (A
// operand of 32x32x2 float32 MFMAs) with particle i's position held in a
// register, particle j's read from the block-J positions in LDS and R_j of
// the pair, and loads frames 2 (l & 31) and 2 (l & 31) + 1 of the pair with
// one 8-byte load SCPS_DIST_AHEAD steps ahead of their use.  R_j is one of
// those loaded values (lane (j >> 1) + 32 (l >> 5), component j & 1), fetched
// across lanes with ds_bpermute; a stack of more than 64 frames (REFLOAD)
// loads it from the pair's frames instead, SCPS_DIST_REF_AHEAD steps ahead,
// since frame j need not lie in the current frame block.  Frame block h holds frames 2j + h,
// so component h of that load is the lane's B operand of block h.  A diagonal
// tile counts the pairs j > i.  The float32 accumulators hold one row (64
// pairs per element) and are added after every row into the workgroup's
// float64 sums xl[slot][frame] in LDS; u^2 goes to float64 term by term (a
// Q that carries float32 partial sums moves w by more than the ratchets
// near the appendix limit allow).  Element v of lane l in block h is
// replica slot 8 (v >> 2) + 4 (l >> 5) + (v & 3), frame 64 fb + 2 (l & 31) + h:
// a stack of more than 64 frames is taken in frame blocks fb of 64, each a
// pass of its own over the tile (the contact values are recomputed; Q is
// summed in block 0 only).
// Addressing: pair (i, j) sits at s * 64 + i in the tile, s = (j - i) mod 64.
// At step m of row i the uniform row b = (2m - i) mod 64 gives s = b + (l >> 5)
// except for b = 63 and l >> 5 = 1 (s = 0), so every load is a uniform base
// (scalar registers) plus one of two per-lane offsets fixed for the tile.
// Lanes of slots without a replica (l & 31 >= nrep) compute finite values
// from zero positions that reach only their own output rows and Q partials,
// which the flush drops; MASK and DIAG tiles zero u of pairs that do not count.
template <bool MASK, bool REFLOAD, bool DIAG, int NW>
__device__ __forceinline__ void scps_dist_tile(const KParams &P, const SysDesc &S, const int nrep,
                                               const ScpsItem &it, const int fb_in, const float4 (*posj)[32],
                                               const int *orgj, const float4 *__restrict__ xs,
                                               const RepDesc *__restrict__ reps, const int myrep, const int jr,
                                               const int lane, const int wave, const int r0, const int r1, double *xl,
                                               double &q) {
    const int I = it.IJ >> 16, J = it.IJ & 0xFFFF;
    const int K4 = stack_pm_width(S.K);
    const int rs = lane & 31, pq = lane >> 5;
    const bool rep = rs < nrep;
    // a stack of at most 64 frames has the one frame block 0: known at compile
    // time, so the step loop below has no branch
    const int fb = REFLOAD ? fb_in : 0;
    const bool bload = 64 * fb + 2 * rs < K4;
    const bool sum_q = fb == 0;
    constexpr bool REF_LD = REFLOAD || SCPS_DIST_REF_GLOBAL;
    // global (not flat) loads from a uniform base with 32-bit lane offsets:
    // flat loads would also count against the LDS wait counter and drain the ring
    typedef float v2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) char *gbytes;
    const gbytes tile_base = (gbytes)(S.stack_pm + (int64_t)it.tile * 4096 * K4);
    const uint32_t row_bytes = 4u * (uint32_t)K4;   // one pair of the tile, all frames
    // byte offsets in a row pair: B operands (frames 2 rs, 2 rs + 1 of frame block fb;
    // lanes past the stack width re-read the pair's first frames, whose columns
    // the flush drops) and R_j
    const uint32_t fo = bload ? 8u * (uint32_t)(32 * fb + rs) : 0u, ro = 4u * (uint32_t)jr;
    const uint32_t up = (uint32_t)pq * 64u * row_bytes;              // s = b + 1 for the upper half
    const uint32_t wrap = (uint32_t)(1 - pq) * 63u * 64u * row_bytes; // b = 63: lower half s = 63, upper s = 0
    const float4 *xr = xs + 2 * reps[myrep].poff + I * 128;
    constexpr int D = SCPS_DIST_AHEAD, DR = SCPS_DIST_REF_AHEAD;
    static_assert(D % DR == 0 && 32 % D == 0, "the rings advance together");
    // the base of step m_ of row i_ (a row past the last, i_ = 64, is never consumed:
    // clamped to 63) and the lane offset
    auto at = [&](int i_, int m_, uint32_t lane_bytes) {
        const int ic = i_ < 64 ? i_ : 63;
        const int b = (2 * m_ - ic) & 63;
        const bool w = b == 63;
        const gbytes base = tile_base + (uint32_t)((w ? 0 : b) * 64 + ic) * row_bytes;
        return base + ((w ? wrap : up) + lane_bytes);
    };
    auto bop = [&](int i_, int m_) {
        typedef const __attribute__((address_space(1))) v2 *gv2;
        return *(gv2)at(i_, m_, fo);
    };
    auto rop = [&](int i_, int m_) {   // R_j of the same pair, the reference of slot rs
        typedef const __attribute__((address_space(1))) float *gf;
        return *(gf)at(i_, m_, ro);
    };
    v2 ring[D];
    float rring[REF_LD ? DR : 1];
#pragma unroll
    for (int u = 0; u < D; ++u) ring[u] = bop(r0 + wave, u);
    if constexpr (REF_LD) {
#pragma unroll
        for (int u = 0; u < DR; ++u) rring[u] = rop(r0 + wave, u);
    }
    const int ref_lane = ((jr >> 1) + 32 * pq) << 2;   // ds_bpermute byte address of the lane holding R_j
    // R_j of a step from the B operands of that step (one step ahead of its use,
    // so the cross-lane move is off the contact value -> MFMA chain)
    auto ref_of = [&](const v2 &bb) {
        const float rx = __int_as_float(__builtin_amdgcn_ds_bpermute(ref_lane, __float_as_int(bb.x)));
        const float ry = __int_as_float(__builtin_amdgcn_ds_bpermute(ref_lane, __float_as_int(bb.y)));
        return (jr & 1) ? ry : rx;
    };
    float rj_next = 0.f;
    if constexpr (!REF_LD) rj_next = ref_of(ring[0]);
#pragma unroll 1
    for (int i = r0 + wave; i < r1; i += NW) {
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
                const v2 b = ring[u];
                float rj;
                if constexpr (REF_LD) {
                    rj = rring[u % DR];
                    const int rm = m + DR < 32 ? m + DR : m + DR - 32, ri = m + DR < 32 ? i : i + NW;
                    rring[u % DR] = rop(ri, rm);
                } else {
                    rj = rj_next;
                    rj_next = ref_of(ring[(u + 1) % D]);   // holds the next step's B operands
                }
                const int nm = m + D < 32 ? m + D : m + D - 32, ni = m + D < 32 ? i : i + NW;
                ring[u] = bop(ni, nm);
                const int jl = 2 * m + pq;
                float c;
                if constexpr (MASK || DIAG) {
                    bool ok = rep;
                    if constexpr (DIAG) ok = ok & (jl > i);
                    if constexpr (MASK) ok = ok & icon & (J * 64 + jl < S.nc) & (abs(oi - orgj[jl]) > P.min_sep);
                    const float cv = contact_operand<MASK>(P, pi, posj[jl][rs], ok);
                    c = ok ? cv - rj : 0.f;   // u = C - R_j of a counted pair
                } else {
                    c = contact_operand<false>(P, pi, posj[jl][rs], true) - rj;
                }
                if (sum_q) q = fma((double)c, (double)c, q);
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
#ifndef SCPS_DIST_NW
#define SCPS_DIST_NW 8      // wavefronts per workgroup for stacks of at most 64 frames
#endif
#ifndef SCPS_DIST_NW_WPE
#define SCPS_DIST_NW_WPE 4  // waves per SIMD with that workgroup (two workgroups per CU)
#endif
// Launch shape of k_scps_dist: stacks of at most 64 frames take SCPS_DIST_NW
// wavefronts per workgroup sharing one staging of block J and one set of
// float64 sums (more wavefronts per CU in the LDS of fewer workgroups); the
// larger stacks (more registers per lane) take four.
template <bool BIGK>
struct DistShape {
    static constexpr int NW = BIGK ? 4 : SCPS_DIST_NW;
    static constexpr int WPE = BIGK ? SCPS_DIST_WPE : SCPS_DIST_NW_WPE;
    static constexpr int WG = 64 * NW;
    static constexpr int RESIDENT = 4 * WPE / NW;   // workgroups per CU
};
// Work unit t covers item t mod n_items in frame block t / n_items (nfb
// blocks of 64 frames); the sums are flushed when (group, frame block) changes.
// BIGK: stacks of more than 64 frames (a kernel of its own).
template <bool BIGK>
__global__ __launch_bounds__(DistShape<BIGK>::WG)
__attribute__((amdgpu_waves_per_eu(DistShape<BIGK>::WPE, DistShape<BIGK>::WPE))) void k_scps_dist(
    const KParams P, const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
    const ScpsGroup *__restrict__ groups, const ScpsItem *__restrict__ items, const int n_items, const int nfb,
    const int nsplit, const int *__restrict__ jref, const float4 *__restrict__ xs, double *__restrict__ X,
    double *__restrict__ Q, const int kmax, const int stack_sys) {
    __shared__ __align__(16) float4 posj[64][32];   // block J of every replica slot
    __shared__ double xl[32 * 64];                   // float64 sums X[slot][frame] of the current group
    constexpr int NW = DistShape<BIGK>::NW, WG = DistShape<BIGK>::WG;
    __shared__ double ql[NW][64];
    __shared__ int orgj[64];
    __shared__ int sh_rep[32];
    __shared__ int sh_jref[32];                      // reference frame of every replica slot
    // the wavefront index is uniform: in a scalar register, the row and step
    // arithmetic of the tile loop (and its load bases) stay scalar
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int e = tid; e < 32 * 64; e += WG) xl[e] = 0.0;
    double q = 0.0;
    int cur = -1, cur_fb = 0, nrep = 0;
    SysDesc S;
    // work unit t: rows [r0, r0 + 64 / nsplit) of item u mod n_items in frame
    // block u / n_items, u = t / nsplit (nsplit > 1 when there are too few
    // items to fill the chip)
    const int n_units = n_items * nfb * nsplit, rows = 64 / nsplit;
    for (int t = blockIdx.x;; t += gridDim.x) {
        const bool more = t < n_units;
        const int u = t / nsplit, r0 = (t - u * nsplit) * rows;
        const int fb = (BIGK && more) ? u / n_items : 0;
        const ScpsItem it = more ? items[u - fb * n_items] : ScpsItem{-1, 0, 0, 0};
        const bool change = it.group != cur || fb != cur_fb;
        if (cur >= 0 && change) {
            // flush the sums of (group, frame block) to the replicas' float64 totals
            ql[wave][lane] = q;
            __syncthreads();
            for (int e = tid; e < 32 * 64; e += WG) {
                const int slot = e >> 6, k = 64 * cur_fb + (e & 63);
                if (slot < nrep && k < S.K) unsafeAtomicAdd(&X[(int64_t)sh_rep[slot] * kmax + k], xl[e]);
                xl[e] = 0.0;
            }
            if (tid < 32 && cur_fb == 0) {
                double sum = 0.0;
                for (int w = 0; w < NW; ++w) sum += ql[w][tid] + ql[w][32 + tid];
                if (tid < nrep) unsafeAtomicAdd(&Q[sh_rep[tid]], sum);
            }
            q = 0.0;
        }
        if (!more) break;
        __syncthreads();
        if (change) {
            cur = it.group;
            cur_fb = fb;
            const ScpsGroup *gp = groups + cur;
            nrep = gp->nrep;
            S = sysd[gp->sys];
            if (stack_sys >= 0) {   // another system's stack (same chain and contact set)
                S.stack_pm = sysd[stack_sys].stack_pm;
                S.K = sysd[stack_sys].K;
            }
            if (tid < 32) {
                sh_rep[tid] = tid < nrep ? gp->rep[tid] : 0;
                sh_jref[tid] = tid < nrep ? ref_frame(jref, gp->rep[tid], S.K) : 0;
            }
            __syncthreads();
        }
        if (64 * fb >= S.K) continue;   // the group's stack has no frame in this block (uniform per workgroup)
        // stage block J of every replica of the group
        const int J = it.IJ & 0xFFFF;
        for (int e = tid; e < 64 * 32; e += WG) {
            const int pl = e >> 5, slot = e & 31;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (slot < nrep) p = xs[2 * reps[sh_rep[slot]].poff + J * 128 + pl];
            posj[pl][slot] = p;
        }
        if (tid < 64) orgj[tid] = S.perm[J * 64 + tid];
        __syncthreads();
        const int myrep = sh_rep[lane & 31], myj = sh_jref[lane & 31];
        const bool diag = (it.IJ >> 16) == J;
        if (it.flags & TILE_MASK) {
            if (diag)
                scps_dist_tile<true, BIGK, true, NW>(P, S, nrep, it, fb, posj, orgj, xs, reps, myrep, myj, lane, wave,
                                                 r0, r0 + rows, xl, q);
            else
                scps_dist_tile<true, BIGK, false, NW>(P, S, nrep, it, fb, posj, orgj, xs, reps, myrep, myj, lane, wave,
                                                  r0, r0 + rows, xl, q);
        } else if (diag) {
            scps_dist_tile<false, BIGK, true, NW>(P, S, nrep, it, fb, posj, orgj, xs, reps, myrep, myj, lane, wave, r0,
                                              r0 + rows, xl, q);
        } else {
            scps_dist_tile<false, BIGK, false, NW>(P, S, nrep, it, fb, posj, orgj, xs, reps, myrep, myj, lane, wave, r0,
                                               r0 + rows, xl, q);
        }
    }
}

// Pass 2 operand of the two-pass form (exec mode 2; the default forms it inside
// k_scps_bias): E[eoff_r + tile * 4096 + p] = sum_k c_rk R_kp for every
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
#ifndef SCPS_EFF_NT
#define SCPS_EFF_NT 3   // bit 0: non-temporal stores of E, bit 1: non-temporal loads of the stack
#endif                  // (each is used once per step; measured 1.7 % faster per SCPS step with both)
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
                    if (k < K) {
#if SCPS_EFF_NT & 2
                        b = __builtin_nontemporal_load(reinterpret_cast<const effvec *>(Rt + k * 4096 + p));
#else
                        b = *reinterpret_cast<const effvec *>(Rt + k * 4096 + p);
#endif
                    } else
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
#if SCPS_EFF_NT & 1
                    __builtin_nontemporal_store(o, reinterpret_cast<effvec *>(E + eo + (int64_t)it.tile * 4096 + p));
#else
                    *reinterpret_cast<effvec *>(E + eo + (int64_t)it.tile * 4096 + p) = o;
#endif
                }
            }
        }
    }
}

// Pass 2 fused with the bias forces: the effective references never leave
// the chip.  A workgroup takes one work item (group of replicas, contact tile
// pair I, J) at a time, with blocks I and J of every replica slot in LDS, and
// walks the tile's sub-steps (lane i of block I meets particle (i + k) mod 64
// of block J) in chunks of BIAS_CH.  Its wavefronts split into a producer
// and a consumer half that work on neighbouring chunks at the same time
// (double-buffered E in LDS, one barrier per chunk):
//  - matrix wavefront w forms E[slot][i] = sum_f c_f,slot R_f,(i, k) of
//    sub-step k = chunk + w with 32x32x2 float32 MFMAs (rows: the pairs
//    i = 2 row + b of block b, read with one 8-byte load per lane from frames
//    2 kk + (l >> 5); columns: the slots, B operand c of slot l & 31 as in
//    k_scps_eff), stores it, and issues the stack loads of its next sub-step;
//  - pair wavefront p takes slots p, p + BIAS_NPW, ... with lane = i, as the
//    tile kernels do: the contact gradient term (csum C - E) C' of the bias
//    goes to the lane's i-side partials and to j-side partials that rotate
//    with the j partner (DPP), over every sub-step of the tile.
// The partials of each slot go to the replica's float64 bias accumulators
// (components 3..5) once per item, 64 consecutive particles per atomic
// instruction.  A diagonal tile takes sub-steps 1..32 (lanes i < 32 at
// k = 32), so each pair is met once; MASK tiles evaluate the contact
// predicate and the cutoff per pair.  Nonbonded forces and bonds are not
// computed here.
constexpr int BIAS_WG = 768;
constexpr int BIAS_NMW = 4;                      // matrix wavefronts = sub-steps per chunk
constexpr int BIAS_NPW = BIAS_WG / 64 - BIAS_NMW;  // pair wavefronts
constexpr int BIAS_CH = BIAS_NMW;
constexpr int BIAS_SPW = SCPS_GROUP / BIAS_NPW;  // replica slots per pair wavefront

struct BiasLds {
    float4 pos[2][SCPS_GROUP][64];        // blocks I, J: [slot][particle]
    float E[2][BIAS_CH][SCPS_GROUP][65];  // two chunks: [sub-step][slot][i], padded for the matrix stores
    float c[KMAX / 2][64];                // B operand: c of slot l & 31, frame 2 kk + (l >> 5)
    float cs[SCPS_GROUP];
    int org[2][64];
    int rep[SCPS_GROUP];                  // -1: empty slot
    int64_t poff[SCPS_GROUP];
};
static_assert(BIAS_WG % 64 == 0 && BIAS_NPW > 0 && SCPS_GROUP % BIAS_NPW == 0,
              "every pair wavefront takes the same number of replica slots");
static_assert(sizeof(BiasLds) <= 160 * 1024, "the fused bias pass keeps one workgroup's state in LDS");

typedef float bias_f2 __attribute__((ext_vector_type(2)));

// Frames 2 (f0 + kk) + half of pairs 2 slot, 2 slot + 1 of sub-step k: a
// uniform tile base and a 32-bit lane offset per load.
template <int KKN>
__device__ __forceinline__ void bias_loads(const float *tile_base, const int k, const int f0, const int K,
                                           const int slot, const int half, bias_f2 r[KKN]) {
    typedef const __attribute__((address_space(1))) bias_f2 *gptr;
    const gptr gb = (gptr)tile_base;
    const int o = (half * 4096 + k * 64 + 2 * slot) >> 1;   // in float pairs
#pragma unroll
    for (int kk = 0; kk < KKN; ++kk) {
        r[kk] = bias_f2{0.f, 0.f};
        if (2 * (f0 + kk) + half < K) r[kk] = __builtin_nontemporal_load(gb + (o + (f0 + kk) * 4096));
    }
}

// KKN frame pairs per MFMA chain, NH chains per sub-step (2 KKN NH >= K;
// frames beyond K have zero coefficients and are not loaded), fixed at
// compile time so that a chain has no branches and its loads are issued
// together.  With NH = 2 (stacks of more than 64 frames) the loads of the
// next half are issued after the MFMAs of the current one.
template <bool MASK, int KKN, int NH>
__device__ __forceinline__ void scps_bias_tile(const KParams &P, const SysDesc &S, const ScpsItem &it,
                                               const int lane, const int wave, const int kb, const int ke, BiasLds &L,
                                               float fi[][3], float fj[][3]) {
    const int I = it.IJ >> 16, J = it.IJ & 0xFFFF;
    const bool diag = it.flags & TILE_DIAG;
    const int nch = (ke - kb + BIAS_CH - 1) / BIAS_CH;
    if (wave < BIAS_NMW) {
        // ---- producer: E of sub-step kb + BIAS_CH st + wave, chunk st -> buffer st & 1
        const int K = S.K;
        const int slot = lane & 31, half = lane >> 5;
        const float *Rt = S.stack + (int64_t)it.tile * K * 4096;   // uniform
        bias_f2 r[KKN];
        if (kb + wave < ke) bias_loads<KKN>(Rt, kb + wave, 0, K, slot, half, r);
#pragma unroll 1
        for (int st = 0; st <= nch; ++st) {
            const int k = kb + BIAS_CH * st + wave;
            if (st < nch && k < ke) {
                fvec16 acc[2];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
                // one chain per KKN frame pairs; a second chain's loads go out after
                // the first chain's MFMAs, into the same registers
#pragma unroll
                for (int h = 0; h < NH; ++h) {
#pragma unroll
                    for (int kk = 0; kk < KKN; ++kk) {
                        const float c = L.c[KKN * h + kk][lane];
                        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(r[kk].x, c, acc[0], 0, 0, 0);
                        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(r[kk].y, c, acc[1], 0, 0, 0);
                    }
                    if (h + 1 < NH) bias_loads<KKN>(Rt, k, KKN * (h + 1), K, slot, half, r);
                }
                float(*E)[65] = L.E[st & 1][wave];
#pragma unroll
                for (int v = 0; v < 16; ++v)
#pragma unroll
                    for (int b = 0; b < 2; ++b) E[slot][16 * (v >> 2) + 8 * half + 2 * (v & 3) + b] = acc[b][v];
                if (k + BIAS_CH < ke) bias_loads<KKN>(Rt, k + BIAS_CH, 0, K, slot, half, r);
            }
            __syncthreads();
        }
        return;
    }
    // ---- consumer: chunk st - 1 from buffer (st - 1) & 1
    const int pw = wave - BIAS_NMW;
    const int nc = S.nc, min_sep = P.min_sep;
    const bool has_cut = P.has_cut;
    const float inv_r0sq = P.inv_r0sq, r_cut2 = P.r_cut2;
    const float cp0 = P.cp[0], cp1 = P.cp[1], cp2 = P.cp[2], cp3 = P.cp[3];
    const bool icon = I * 64 + lane < nc;
    const int oi = L.org[0][lane];
    float px[BIAS_SPW], py[BIAS_SPW], pz[BIAS_SPW], csm[BIAS_SPW];
#pragma unroll
    for (int m = 0; m < BIAS_SPW; ++m) {
        const float4 p = L.pos[0][pw + BIAS_NPW * m][lane];
        px[m] = p.x;
        py[m] = p.y;
        pz[m] = p.z;
        csm[m] = L.cs[pw + BIAS_NPW * m];
    }
#pragma unroll 1
    for (int st = 0; st <= nch; ++st) {
        if (st > 0) {
            const int c0 = kb + BIAS_CH * (st - 1), nk = min(BIAS_CH, ke - c0);
            float(*E)[SCPS_GROUP][65] = L.E[(st - 1) & 1];
            // sub-steps in order (the j-side partials rotate once per sub-step);
            // the slots of one sub-step are independent, so they run interleaved
#pragma unroll
            for (int u = 0; u < BIAS_CH; ++u) {
                if (u < nk) {
                    const int k = c0 + u, jl = (lane + k) & 63;
                    const bool con0 = !diag | (k != 32) | (lane < 32);
                    bool conm = true;
                    if constexpr (MASK) conm = icon & (J * 64 + jl < nc) & (abs(oi - L.org[1][jl]) > min_sep);
#pragma unroll
                    for (int m = 0; m < BIAS_SPW; ++m) {
                        const int sl = pw + BIAS_NPW * m;
                        const float4 pj = L.pos[1][sl][jl];
                        const float dx = px[m] - pj.x, dy = py[m] - pj.y, dz = pz[m] - pj.z;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        bool inside = true;
                        if constexpr (MASK) inside = !has_cut | (r2 <= r_cut2);
                        const float q = r2 * inv_r0sq;
                        const float q2 = q * q;
                        const float t = q + q2;
                        const float num = 1.f + t;
                        const float den = fmaf(q2, t, num);
                        const float inv_den = inside ? frcp(den) : 0.f;
                        float diff = fmaf(csm[m], num * inv_den, -E[u][sl][lane]);
                        diff = (con0 & conm) ? diff : 0.f;
                        const float poly = fmaf(q, fmaf(q, fmaf(q, cp0, cp1), cp2), cp3);
                        const float g = (diff * (q2 * inv_den)) * (poly * inv_den);
                        fi[m][0] = fmaf(g, dx, fi[m][0]);
                        fi[m][1] = fmaf(g, dy, fi[m][1]);
                        fi[m][2] = fmaf(g, dz, fi[m][2]);
                        fj[m][0] = rot1(fmaf(-g, dx, fj[m][0]));
                        fj[m][1] = rot1(fmaf(-g, dy, fj[m][1]));
                        fj[m][2] = rot1(fmaf(-g, dz, fj[m][2]));
                    }
                }
            }
        }
        __syncthreads();
    }
}

// BIG: stacks of 65 .. KMAX frames, in a kernel of its own so that the
// common sizes keep their register allocation.
template <bool MASK, bool BIG>
__device__ __forceinline__ void scps_bias_dispatch(const KParams &P, const SysDesc &S, const ScpsItem &it,
                                                   const int lane, const int wave, const int kb, const int ke,
                                                   BiasLds &L, float fi[][3], float fj[][3]) {
    if constexpr (BIG)
        scps_bias_tile<MASK, 32, 2>(P, S, it, lane, wave, kb, ke, L, fi, fj);
    else if (S.K <= 16)
        scps_bias_tile<MASK, 8, 1>(P, S, it, lane, wave, kb, ke, L, fi, fj);
    else if (S.K <= 32)
        scps_bias_tile<MASK, 16, 1>(P, S, it, lane, wave, kb, ke, L, fi, fj);
    else if (S.K <= 52)
        scps_bias_tile<MASK, 26, 1>(P, S, it, lane, wave, kb, ke, L, fi, fj);
    else
        scps_bias_tile<MASK, 32, 1>(P, S, it, lane, wave, kb, ke, L, fi, fj);
}

template <bool BIG>
__global__ __launch_bounds__(BIAS_WG) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_scps_bias(
    const KParams P, const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps,
    const ScpsGroup *__restrict__ groups, const ScpsItem *__restrict__ items, const int n_items,
    const float4 *__restrict__ xs, const float *__restrict__ coef, const double *__restrict__ csum, const int kmax,
    const int ksplit, double *__restrict__ acc) {
    __shared__ BiasLds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int cur = -1;
    SysDesc S;
    // work unit t: a range of the sub-steps of item t / ksplit (ksplit > 1
    // when there are too few items to fill the chip), in whole chunks
    for (int t = blockIdx.x; t < n_items * ksplit; t += gridDim.x) {
        const ScpsItem it = items[t / ksplit];
        const bool tdiag = it.flags & TILE_DIAG;
        const int kb0 = tdiag ? 1 : 0, ke0 = tdiag ? 33 : 64;   // a diagonal tile meets each pair by sub-step 32
        const int per = ((ke0 - kb0 + ksplit - 1) / ksplit + BIAS_CH - 1) / BIAS_CH * BIAS_CH;
        const int kb = min(ke0, kb0 + (t % ksplit) * per), ke = min(ke0, kb + per);
        __syncthreads();   // the previous item's positions are no longer read
        if (it.group != cur) {
            cur = it.group;
            const ScpsGroup *gp = groups + cur;
            const int nrep = gp->nrep;
            S = sysd[gp->sys];
            for (int e = tid; e < KMAX / 2 * 64; e += BIAS_WG) {
                const int kk = e >> 6, l = e & 63, sl = l & 31, k = 2 * kk + (l >> 5);
                L.c[kk][l] = (sl < nrep && k < S.K) ? coef[(int64_t)gp->rep[sl] * kmax + k] : 0.f;
            }
            if (tid < SCPS_GROUP) {
                const bool live = tid < nrep;
                L.rep[tid] = live ? gp->rep[tid] : -1;
                L.poff[tid] = live ? reps[gp->rep[tid]].poff : 0;
                L.cs[tid] = live ? (float)csum[gp->rep[tid]] : 0.f;
            }
            __syncthreads();
        }
        const int I = it.IJ >> 16, J = it.IJ & 0xFFFF;
        for (int e = tid; e < 2 * SCPS_GROUP * 64; e += BIAS_WG) {
            const int pl = e & 63, sl = (e >> 6) & 31, side = e >> 11;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            if (L.rep[sl] >= 0) p = xs[2 * L.poff[sl] + (side ? J : I) * 128 + pl];
            L.pos[side][sl][pl] = p;
        }
        if (tid < 128) L.org[tid >> 6][tid & 63] = S.perm[((tid >> 6) ? J : I) * 64 + (tid & 63)];
        __syncthreads();
        float fi[BIAS_SPW][3], fj[BIAS_SPW][3];
#pragma unroll
        for (int m = 0; m < BIAS_SPW; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) fi[m][c] = fj[m][c] = 0.f;
        if (it.flags & TILE_MASK)
            scps_bias_dispatch<true, BIG>(P, S, it, lane, wave, kb, ke, L, fi, fj);
        else
            scps_bias_dispatch<false, BIG>(P, S, it, lane, wave, kb, ke, L, fi, fj);
        if (wave < BIAS_NMW || kb == ke) continue;
        // after sub-steps kb .. ke-1 lane l holds the j-side partials of particle (l + ke) mod 64
        const int jo = J * 64 + ((lane + ke) & 63);
        const int n_pad = S.n_pad;
#pragma unroll
        for (int m = 0; m < BIAS_SPW; ++m) {
            const int sl = (wave - BIAS_NMW) + BIAS_NPW * m;
            if (L.rep[sl] >= 0) {
                double *ar = acc + 6 * L.poff[sl];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    unsafeAtomicAdd(&ar[(3 + c) * n_pad + I * 64 + lane], (double)fi[m][c]);
                    unsafeAtomicAdd(&ar[(3 + c) * n_pad + jo], (double)fj[m][c]);
                }
            }
        }
    }
}

hipError_t launch_scps_dist(const KParams &P, const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups,
                            const ScpsItem *items, int n_items, int max_frames, const int *jref, const float4 *xs,
                            double *X, double *Q, int kmax, int stack_sys, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (max_frames < 1 || max_frames > KMAX || max_frames > kmax) return hipErrorInvalidValue;
    const int nfb = (max_frames + 63) / 64;
    // a grid of the resident workgroups (256 CUs) striding over the work
    // units; too few items for that (small systems) split each tile's rows
    // over up to 16 workgroups (4 rows each, half the wavefronts without a
    // row: still faster than 8 at 32 x 560, while 16 sub-step ranges of the
    // bias pass were slower than 8)
    auto split = [&](int resident) {
        int ns = 1;
        while (ns < 16 && n_items * nfb * ns * 2 <= resident) ns *= 2;
        return ns;
    };
    if (nfb > 1) {
        typedef DistShape<true> DS;
        const int ns = split(256 * DS::RESIDENT);
        const int grid = std::min(n_items * nfb * ns, 256 * DS::RESIDENT);
        hipLaunchKernelGGL(k_scps_dist<true>, dim3(grid), dim3(DS::WG), 0, st, P, sysd, reps, groups, items, n_items,
                           nfb, ns, jref, xs, X, Q, kmax, stack_sys);
    } else {
        typedef DistShape<false> DS;
        const int ns = split(256 * DS::RESIDENT);
        const int grid = std::min(n_items * ns, 256 * DS::RESIDENT);
        hipLaunchKernelGGL(k_scps_dist<false>, dim3(grid), dim3(DS::WG), 0, st, P, sysd, reps, groups, items,
                           n_items, nfb, ns, jref, xs, X, Q, kmax, stack_sys);
    }
    return hipGetLastError();
}

// Tube variables of every replica against the frame stack of system
// stack_sys (-1: its own system's), from the sums k_scps_dist left in X and
// Q around the reference frames jref_in, which are cleared for the next
// pass.  s, w: nullable [R]; sigma: nullable [R], set to weight (1 - s) when
// first, else incremented by it (the mean of 1 - s over several stacks is
// the progress coordinate sigma); jref_out: nullable [R], each replica's
// frame of largest weight.
__global__ void k_tube_eval(double lam, double wscale, const int *__restrict__ jref_in, int *__restrict__ jref_out,
                            const SysDesc *__restrict__ sysd, const RepDesc *__restrict__ reps, int kmax,
                            int stack_sys, double *__restrict__ X, double *__restrict__ Q, double *__restrict__ s,
                            double *__restrict__ w, double *__restrict__ sigma, double weight, int first) {
    const int r = blockIdx.x, lane = threadIdx.x;
    const SysDesc S = sysd[stack_sys >= 0 ? stack_sys : reps[r].sys];
    const int K = S.K;
    double *xr = X + (int64_t)r * kmax;
    const int j = ref_frame(jref_in, r, K);
    const TubeSums ts = tube_sums(lane, K, Q[r], xr, j, S.G + (int64_t)j * K, S.Z0, lam);
    const double sv = 1.0 - (ts.s1 / ts.s0) / (double)(K - 1);
    const double wv = tube_w(ts.a, ts.s0, wscale);
#pragma unroll
    for (int h = 0; h < 2; ++h)
        if (lane + 64 * h < K) xr[lane + 64 * h] = 0.0;
    if (lane == 0) {
        Q[r] = 0.0;
        if (s) s[r] = sv;
        if (w) w[r] = wv;
        if (sigma) sigma[r] = (first ? 0.0 : sigma[r]) + weight * (1.0 - sv);
        if (jref_out) jref_out[r] = ts.kmax;
    }
}

hipError_t launch_tube_eval(double lam, double wscale, const int *jref_in, int *jref_out, const SysDesc *sysd,
                            const RepDesc *reps, int R, int kmax, int stack_sys, double *X, double *Q, double *s,
                            double *w, double *sigma, double weight, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_tube_eval, dim3(R), dim3(64), 0, st, lam, wscale, jref_in, jref_out, sysd, reps, kmax,
                       stack_sys, X, Q, s, w, sigma, weight, first);
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

hipError_t launch_scps_bias(const KParams &P, const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups,
                            const ScpsItem *items, int n_items, int max_frames, const float4 *xs, const float *coef,
                            const double *csum, int kmax, double *acc, hipStream_t st) {
    if (n_items == 0) return hipSuccess;
    if (max_frames < 1 || max_frames > KMAX || max_frames > kmax) return hipErrorInvalidValue;
    // one workgroup per compute unit (LDS); too few items for 256 (small
    // systems) split each tile's sub-steps over up to 8 workgroups
    int ks = 1;
    while (ks < 8 && n_items * ks * 2 <= 256) ks *= 2;
    const int grid = std::min(n_items * ks, 256);
    if (max_frames > 64)
        hipLaunchKernelGGL(k_scps_bias<true>, dim3(grid), dim3(BIAS_WG), 0, st, P, sysd, reps, groups, items, n_items,
                           xs, coef, csum, kmax, ks, acc);
    else
        hipLaunchKernelGGL(k_scps_bias<false>, dim3(grid), dim3(BIAS_WG), 0, st, P, sysd, reps, groups, items,
                           n_items, xs, coef, csum, kmax, ks, acc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// convergence measure between iterations
// ---------------------------------------------------------------------------
// Occupancy of an nx x ny grid of square cells (side cell, lower corner
// (x0, y0), half-open) by 2-D points xy [n][2]: occ[cy * nx + cx] = 1 for
// every cell holding a point; points outside the grid are ignored.  Cell
// indices are taken in float64.  occ must be zero on entry.
__global__ void k_occupancy(const float *__restrict__ xy, int64_t n, double x0, double y0, double cell, int nx, int ny,
                            int *__restrict__ occ) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double u = floor(((double)xy[2 * e] - x0) / cell), v = floor(((double)xy[2 * e + 1] - y0) / cell);
        if (u >= 0.0 && u < (double)nx && v >= 0.0 && v < (double)ny) occ[(int)v * nx + (int)u] = 1;
    }
}

// Counts of occupied cells in a, in b, and in both (one workgroup).
__global__ __launch_bounds__(256) void k_occupancy_overlap(const int *__restrict__ a, const int *__restrict__ b,
                                                           int m, long long *__restrict__ out) {
    __shared__ long long sh[3][256];
    long long na = 0, nb = 0, nab = 0;
    for (int e = threadIdx.x; e < m; e += 256) {
        na += a[e];
        nb += b[e];
        nab += a[e] & b[e];
    }
    sh[0][threadIdx.x] = na;
    sh[1][threadIdx.x] = nb;
    sh[2][threadIdx.x] = nab;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_fill_int(int *__restrict__ v, int m) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x) v[e] = 0;
}

// Scratch of the convergence measure for callers that cannot allocate: the
// four counts (long long) first, then the two occupancy grids, in a file-scope
// device array each GPU holds until the process ends.  Host code must not
// pass `scratch` itself to a kernel (in host code the name is a stand-in, not
// a device address): path_scratch() returns this GPU's address of it.
static __device__ __align__(256) int scratch[8 + 2 * PATH_NOALLOC_MAX_CELLS];

hipError_t path_scratch(int **occ, long long **counts) {
    static std::mutex lock;
    static void *addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // with this device current: its own copy
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *counts = reinterpret_cast<long long *>(addr[dev]);
    *occ = reinterpret_cast<int *>(addr[dev]) + 8;
    return hipSuccess;
}

hipError_t launch_path_occupancy(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                                 double y0, double cell, int nx, int ny, int *occ, long long *counts,
                                 hipStream_t st) {
    const int m = nx * ny;
    hipLaunchKernelGGL(k_fill_int, dim3((2 * m + 255) / 256), dim3(256), 0, st, occ, 2 * m);
    if (n_a > 0)
        hipLaunchKernelGGL(k_occupancy, dim3((unsigned)std::min<int64_t>((n_a + 255) / 256, 4096)), dim3(256), 0, st,
                           xy_a, n_a, x0, y0, cell, nx, ny, occ);
    if (n_b > 0)
        hipLaunchKernelGGL(k_occupancy, dim3((unsigned)std::min<int64_t>((n_b + 255) / 256, 4096)), dim3(256), 0, st,
                           xy_b, n_b, x0, y0, cell, nx, ny, occ + m);
    hipLaunchKernelGGL(k_occupancy_overlap, dim3(1), dim3(256), 0, st, occ, occ + m, m, counts);
    return hipGetLastError();
}

}  // namespace scps
