// Internal declarations shared by the kernels and the host side of libscps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scps {

constexpr int TILE = 64;          // tile edge = wavefront width
constexpr int KMAX = 128;         // largest SCPS frame stack (the distance pass takes it in blocks of 64)
constexpr int CV_STRIDE = 8;
enum { CV_Z = 0, CV_ZM = 1, CV_EB = 2, CV_S = 3, CV_W = 4, CV_SM = 5, CV_WM = 6, CV_T = 7 };

// Scalars every kernel needs, passed by value.
struct KParams {
    float inv_r0sq;      // 1/r0^2
    float g_scale;       // 4/r0^2: dz/dx_i = sum_j g_scale (C - R) C'(q) (x_i - x_j)
    float cp[4];         // -g_scale * {2, 4, 6, 3}: coefficients of -g_scale (3 + 6q + 4q^2 + 2q^3)
    float r_cut2;        // contact cutoff squared (used when has_cut)
    float r_cut_nb2;     // nonbonded cutoff squared (used when has_cut_nb)
    float lj_A;          // 48 epsilon sigma^12
    float lj_B;          // 24 epsilon sigma^6
    float dh_pref;       // k_e/eps_r
    float dh_kappa;
    float dh_kl2;        // -kappa * log2(e)
    int nb_excl, min_sep;
    int has_lj, has_dh, has_cut, has_cut_nb, has_bond;
    int integrator;
    double dt, kT, gamma, c1;
    double k_bond, r_bond;
    double k_R;
    double lambda, k_s, k_w;
    double wscale;       // w = -wscale log sum_k exp(-lambda d_k): 1/lambda, or 1 without the 1/lambda
    uint32_t seed_lo, seed_hi;
    uint32_t rep_base;
};

// One chain, in the library's internal particle order: contact-set particles
// first (ascending), then the rest (ascending), padded to a multiple of 64.
struct SysDesc {
    int n, n_pad, nb;        // particles, padded count, blocks of 64
    int nc, ncb, ntile_c;    // contact-set size, its blocks, contact tile pairs
    int K;                   // SCPS frames in the stack
    int pad0;
    const int *perm;         // [n_pad] internal -> chain index (pads: n + k)
    const int *bond_next;    // [n_pad] internal index of chain neighbour i+1, -1 if none
    const float *mass;       // [n_pad] internal order (pads: 1)
    const float *charge;     // [n_pad] internal order (pads: 0)
    const float *ref;        // native map tiles [ntile_c][64*64]
    const float *stack;      // SCPS frames [ntile_c][K][64*64]
    const float *stack_pm;   // the same frames pair-major: [ntile_c][64*64][stack_pm_width(K)]
    const double *G;         // [K][K] sum over the counted contact pairs of (R_j - R_k)^2
    const double *R2tile;    // [ntile_c] per native-map tile: sum over its counted contact pairs of R^2
    const int2 *tiles;       // persistent work list, costliest first (see build_schedule)
    const uint64_t *tmask;   // per work-list item: sub-steps that need the per-pair predicates
    int ntile;
    int pad1;
    double Z0;
};

struct RepDesc {
    int sys;
    int pad0;
    int64_t off;             // particle offset of the replica in the flat x layout
    int64_t poff;            // particle offset in the padded internal-order buffers
    int64_t eoff;            // SCPS: offset of its effective reference [ntile_c][64*64]
};

// SCPS: up to 32 replicas of one system share every read of the frame stack.
constexpr int SCPS_GROUP = 32;
struct ScpsGroup {
    int sys, nrep;
    int rep[SCPS_GROUP];
};
// A unit of SCPS stack work: one contact tile pair (I, J) = (IJ >> 16, IJ &
// 0xFFFF), numbered tile, for every replica of a group.
struct ScpsItem {
    int group, tile, IJ, flags;
};

// A unit of pair work for the per-step kernels: one tile pair of one replica.
// mask: bit k set when some pair the tile meets at sub-step k needs a per-pair
// predicate (only MASK tiles evaluate them, and only on those sub-steps).
struct TileItem {
    int rep, I, J, flags;
    uint64_t mask;
};

// Tile flags, computed on the host.  CONTACT: both blocks hold contact-set
// particles.  MASK: a per-pair predicate is needed, because the tile holds a
// pair excluded from the nonbonded sum (|i-j| <= nb_excl) or its contact sum
// does (a block that straddles the end of the contact set, a pair within
// min_seq_sep, or a contact cutoff).  With it goes a 64-bit mask of the
// sub-steps k at which such a pair is met: lane l of block I meets particle
// (l + k) mod 64 of block J (a diagonal tile meets each pair at the smaller
// of its two separations); a straddling block or a cutoff sets every bit.
enum { TILE_DIAG = 1, TILE_CONTACT = 2, TILE_MASK = 4 };

// The persistent kernel's work items are segments of sub-steps k_begin ..
// k_end-1 of a tile (or of two tiles that share the J block): {I1 << 16 | J,
// flags | (I2 + 1) << 8 | k_begin << 16 | k_end << 23}, I2 = -1 for a single
// tile (so I2 < 255: the persistent kernel's chains have far fewer blocks).
// Segments are SEG_STEPS long; the TAIL_ITEMS cheapest items of the
// cost-sorted list are cut further into TAIL_STEPS-long pieces, so that the
// wavefronts of a workgroup run out of work at nearly the same time.
#ifndef SCPS_SEG_STEPS
#define SCPS_SEG_STEPS 32
#endif
#ifndef SCPS_TAIL_ITEMS
#define SCPS_TAIL_ITEMS 32
#endif
#ifndef SCPS_TAIL_STEPS
#define SCPS_TAIL_STEPS 16
#endif
constexpr int SEG_STEPS = SCPS_SEG_STEPS;
constexpr int TAIL_ITEMS = SCPS_TAIL_ITEMS;
constexpr int TAIL_STEPS = SCPS_TAIL_STEPS;

// Frames per pair in the pair-major stack: K rounded up to a multiple of 4
// (zero-filled), so a lane reads four frames of a pair with one 16-byte load.
__host__ __device__ inline int stack_pm_width(int K) { return (K + 3) & ~3; }

// Contact tile pairs (I <= J < ncb) are numbered row by row.
__host__ __device__ inline int tile_index(int I, int J, int ncb) {
    return I * ncb - (I * (I - 1)) / 2 + (J - I);
}

// ---- launch wrappers (defined in scps_kernels.hip) -------------------------
size_t persistent_lds_bytes(int n_pad, int wg);
int persistent_max_npad(int wg);

hipError_t launch_persistent_rmd(int wg, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps,
                                 const int *order, int R, int n_pad_max, float *x, float *v,
                                 double *cv, int64_t n_steps, uint64_t step0, int record_every,
                                 float *frames, int64_t frame_stride, int *flags, hipStream_t st);
// Chains of at most 64 particles, 64 / n_max per wavefront, `waves` wavefronts
// per workgroup, all n_steps in one launch; the untuned default for chains that
// pack at least two to a wavefront.
int packed_width_ok(int n_max);
int packed_default(int n_max, int n_replicas);
hipError_t launch_packed_rmd(int waves, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                             int n_max, float *x, float *v, double *cv, int64_t n_steps, uint64_t step0,
                             int record_every, float *frames, int64_t frame_stride, int *flags, hipStream_t st);

hipError_t launch_gather(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max,
                         const float *x, const float *v, float4 *xs, float4 *vs, hipStream_t st);
hipError_t launch_scatter(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max,
                          const float4 *xs, const float4 *vs, float *x, float *v, float *frames_slot,
                          hipStream_t st);

// mode: 0 rMD forces (contact z + grad, nonbonded, bonds); 1 z only; 2 z and grad;
//       3 SCPS bias against the effective references eff (+ nonbonded + bonds)
// nbk: nonbonded terms, bit 0 Lennard-Jones, bit 1 Debye-Hueckel
hipError_t launch_pairs(int mode, int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps,
                        const TileItem *items, int n_items, const float4 *xs, double *acc, double *zpart,
                        const float *eff, const double *csum, hipStream_t st);
// stack_sys: -1 for each group's own system's stack, else that system's
// (same chain and contact set as every group's).  max_frames: the largest K
// of the stacks read (1 .. KMAX), which sets the number of 64-frame blocks.
// jref [R]: each replica's reference frame j of the distance expansion (NULL:
// frame 0); X receives Y_k = sum_p (C_p - R_jp) R_kp and Q sum_p (C_p - R_jp)^2.
hipError_t launch_scps_dist(const KParams &P, const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups,
                            const ScpsItem *items, int n_items, int max_frames, const int *jref, const float4 *xs,
                            double *X, double *Q, int kmax, int stack_sys, hipStream_t st);
// s, w, sigma of every replica from the distances in X, Q (which it clears);
// jref_in: the reference frames the distance pass used (NULL: frame 0);
// jref_out (nullable): each replica's frame of largest weight.
hipError_t launch_tube_eval(double lam, double wscale, const int *jref_in, int *jref_out, const SysDesc *sysd,
                            const RepDesc *reps, int R, int kmax, int stack_sys, double *X, double *Q, double *s,
                            double *w, double *sigma, double weight, int first, hipStream_t st);
hipError_t launch_scps_eff(const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups, const ScpsItem *items,
                           int n_items, const float *coef, int kmax, float *E, hipStream_t st);
// Effective references and the contact bias forces in one pass (no E in
// device memory): adds the bias gradient terms to acc components 3..5.
hipError_t launch_scps_bias(const KParams &P, const SysDesc *sysd, const RepDesc *reps, const ScpsGroup *groups,
                            const ScpsItem *items, int n_items, int max_frames, const float4 *xs, const float *coef,
                            const double *csum, int kmax, double *acc, hipStream_t st);
hipError_t launch_stack_pairmajor(int nc, int ncb, int K, const float *stack, float *stack_pm, hipStream_t st);
// G[j][k] = sum over the counted contact pairs of (R_j - R_k)^2 in float64 from
// a tile-major stack; G must be zero on entry.
hipError_t launch_stack_gram(int nc, int ncb, int K, int min_sep, const int *perm, const float *stack, double *G,
                             hipStream_t st);

// Neighbour lists of the cutoff variant (rMD with both cutoffs): NL_CAP
// entries per particle, radius (larger cutoff) + NL_SKIN.
constexpr int NL_CAP = 512;
constexpr float NL_SKIN = 2.0f;
// Rebuild the lists of the replicas that need it (force: all of them).
// first_blk [R+1]: blocks of 64 before each replica; bounds [R][nb_max],
// xref [sum n_pad], bmax [sum nb], rebuild [R], cnt [sum n_pad],
// nl [sum n_pad][NL_CAP]; flags[r] = 2 when a list of replica r overflowed.
hipError_t launch_nl_update(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R, int nb_max,
                            const int *first_blk, const float4 *xs, float4 *bounds, float4 *xref, float *bmax,
                            int *rebuild, int force, const TileItem *items_all, const int *first_all, float r_list,
                            int *cnt, int2 *nl, int *flags, hipStream_t st);
// Particle chunks of the list force kernel for a system of n_pad particles.
int nl_chunks(int n_pad);
// Forces (added to acc) and z partials zpart[first_chunk[r] + chunk] over the lists.
hipError_t launch_nl_force(int nbk, const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                           int n_pad_max, const int *first_chunk, const float4 *xs, const int *cnt, const int2 *nl,
                           double *acc, double *zpart, hipStream_t st);
// Per contact tile of a map: sum over its counted pairs of the squared
// (float32) entries, in float64.
hipError_t launch_tile_sumsq(int nc, int ncb, int min_sep, const int *perm, const float *tiles, double *out,
                             hipStream_t st);
// jref [R]: read as the distance pass's reference frames, then set to each
// replica's frame of largest weight for the next step.
hipError_t launch_finalize_scps(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                                int kmax, int *jref, double *X, double *Q, double *cv, float *coef, double *csum,
                                hipStream_t st);
// The update of one step.  The contact-gradient accumulators are scaled by
// scale[r], or, when zpart is not NULL, by the rMD ratchet of eq (FrMD)
// computed in the same launch (cvstate's z, z_m and E_b written): z of
// replica r = zbase[r] (when not NULL) + the sum of zpart[zfirst[r] ..
// zfirst[r+1]).
hipError_t launch_integrate(const KParams &P, const SysDesc *sysd, const RepDesc *reps, int R,
                            int n_pad_max, float4 *xs, float4 *vs, double *acc,
                            const double *scale, double *cv, uint64_t step, const uint64_t *step_base,
                            int *flags, hipStream_t st, const int *zfirst = nullptr,
                            const double *zpart = nullptr, const double *zbase = nullptr);
// *d = v (one thread), in stream order
hipError_t launch_set_step(uint64_t *d, uint64_t v, hipStream_t st);

// z[r] from the pass's partials, E_b[r] when zm is not NULL, and (grad not
// NULL) grad_coef * grad z out of the accumulators, clearing them
hipError_t launch_eval_out(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, double *acc,
                           const int *first, const double *zpart, double *z_out, double k_R, const double *zm,
                           double *Eb, float *grad, const double *grad_coef, hipStream_t st);
// out = in * (gz[r sz] + gE[r sE] k_R (z - zm) theta) per replica
hipError_t launch_zbias_backward(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, double k_R,
                                 const double *z, const double *zm, const double *gz, int64_t sz, const double *gE,
                                 int64_t sE, const float *in, float *out, hipStream_t st);
hipError_t launch_ratchet_energy(int R, double k_R, const double *z, const double *zm, double *Eb,
                                 const double *gz, const double *gE, double *coef, hipStream_t st);

hipError_t launch_native_map(int n, int n_pad, int nc, int ncb, const int *perm_dev,
                             const double *xyz_dev, double r0, double r_cut, float *tiles,
                             double *packed, hipStream_t st);
hipError_t launch_pack_to_tiles(int n_maps, int nc, int ncb, const double *packed, float *tiles,
                                hipStream_t st);
int sum_squares_scratch();   // doubles of scratch launch_sum_squares needs
hipError_t launch_sum_squares(int64_t m, const double *v, double *part, double *out, hipStream_t st);
// The sum over the packed contact pairs a < b with |perm[a] - perm[b]| >
// min_sep of v^2 (part: scratch of nc doubles).
hipError_t launch_sum_squares_sep(int nc, int min_sep, const int *perm, const double *v, double *part, double *out,
                                  hipStream_t st);
// Binary occupancy of an nx x ny grid by the points of a and of b (occ:
// scratch int [2 nx ny]) and counts[3] = {cells of a, cells of b, cells of both}.
hipError_t launch_path_occupancy(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                                 double y0, double cell, int nx, int ny, int *occ, long long *counts,
                                 hipStream_t st);
// The convergence measure without allocation: grids of at most
// PATH_NOALLOC_MAX_CELLS cells in a file-scope device array (8 MiB per GPU);
// path_scratch gives the current GPU's address of its grids and counts.
constexpr int PATH_NOALLOC_MAX_CELLS = 1 << 20;
hipError_t path_scratch(int **occ, long long **counts);
hipError_t launch_scale_by_replica(const SysDesc *sysd, const RepDesc *reps, int R, int n_pad_max, const float *in,
                                   const double *coef, float *out, hipStream_t st);
hipError_t launch_least_biased(const double *cv, const int *list, int n, int *out_i, double *out_t, hipStream_t st);
hipError_t launch_update_reference(int n, int n_pad, int nc, int ncb, const int *perm_dev,
                                   const float *frames, int n_paths, int n_frames,
                                   const int *succ_idx, int n_succ, double r0, double r_cut,
                                   float *tiles, double *packed, hipStream_t st);

}  // namespace scps
