// Host side of libscps: validation, ownership, work lists and launches.
// Every entry point of include/scps.h is defined here.
#include <math.h>
#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <exception>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/scps.h"
#include "scps_internal.h"
#include "scps_funnel.h"

using namespace scps;

static_assert(KMAX == SCPS_MAX_FRAMES, "the header states the frame-stack limit the kernels are built for");
static_assert(FUNNEL_KMAX == SCPS_MAX_FRAMES, "mean paths of the toy model take as many frames as stacks");

namespace {

thread_local std::string g_err;

scps_status fail(scps_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

struct SysHost {
    int n = 0, n_pad = 0, nb = 0, nc = 0, ncb = 0, ntile_c = 0;
    std::vector<int> perm, bond_next;
    std::vector<int> tile_flags;        // [nb * nb], entry I * nb + J for I <= J
    std::vector<uint64_t> tile_mask;    // [nb * nb]: sub-steps that need the per-pair predicates
    std::vector<int2> sched;            // persistent-kernel tile list, costliest first
    std::vector<uint64_t> sched_mask;   // its sub-step masks
    int2 *d_sched = nullptr;
    uint64_t *d_sched_mask = nullptr;
    std::vector<float> mass, charge;
    int *d_perm = nullptr, *d_bond_next = nullptr;
    float *d_mass = nullptr, *d_charge = nullptr;
    float *d_ref = nullptr;
    bool has_native = false;
    double Z0 = 0.0;
    float *d_stack = nullptr;      // [ntile_c][K][4096]
    float *d_stack_pm = nullptr;   // [ntile_c][4096][stack_pm_width(K)]
    double *d_G = nullptr;         // [K][K] frame distances sum_p (R_j - R_k)^2
    int K = 0;
    int K_pm = 0;                  // K the pair-major copy and G are allocated for
    double *d_R2tile = nullptr;    // [ntile_c] native map: sum of R^2 over each tile's counted pairs
    double R2total = 0.0;          // their sum (added to z for the tiles the culled path skips)
};

}  // namespace

struct scps_ctx {
    scps_params prm{};
    KParams kp{};
    hipStream_t stream = nullptr;
    // SCPS, fused form: the nonbonded pass runs on a second stream beside the
    // distance pass (fork and join through events on the caller's stream)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool overlap_nb = false;          // SCPS: nonbonded pass beside the distance pass (scps_autotune may turn it on)
    hipEvent_t ev_switch = nullptr;   // orders a new stream after the old one (scps_set_stream)
    // per-step path: whole blocks of graph_steps steps replay one captured
    // HIP graph (scps_set_graph_steps; 0, the default: every kernel launched
    // on its own)
    int graph_steps = 0;
    hipStream_t cap = nullptr;        // private stream the graph is captured on
    hipGraphExec_t gexec = nullptr;
    const double *g_cv = nullptr;     // what the graph was captured for
    int g_frames = 0, g_steps = 0;
    bool g_overlap = false;
    uint64_t *d_step = nullptr;       // the replayed block's first step
    // scps_time_passes: HIP events around the SCPS step's two stack passes, in a ring
    // of PASS_RING slots (4 events each) whose oldest slot is read back before reuse
    static constexpr int PASS_RING = 256;
    bool timing = false;
    int timing_period = 1;           // time every timing_period-th SCPS step
    int64_t timing_tick = 0;
    std::vector<hipEvent_t> pass_ev;  // [PASS_RING][4]: distance start, end, bias start, end
    int64_t pass_recorded = 0, pass_read = 0;
    double pass_ms[2] = {0.0, 0.0};
    int R = 0;
    std::vector<SysHost> sys;
    std::vector<int> rep_sys;
    std::vector<int64_t> rep_off, rep_poff;
    int64_t sumN = 0, sumNpad = 0;
    int n_pad_max = 0;
    bool poisoned = false;
    // device
    SysDesc *d_sysd = nullptr;
    RepDesc *d_reps = nullptr;
    int *d_order = nullptr;
    int *d_flags = nullptr;
    TileItem *d_items_all = nullptr;
    int n_items_all = 0;
    TileItem *d_items_contact = nullptr;
    int n_items_contact = 0;
    float4 *d_xs = nullptr, *d_vs = nullptr;
    double *d_acc = nullptr, *d_negone = nullptr;
    double *d_zpart = nullptr;                       // z partial of every tile item
    int *d_first_all = nullptr, *d_first_con = nullptr;   // [R+1] item ranges per replica
    double *d_X = nullptr, *d_Q = nullptr, *d_csum = nullptr;   // SCPS: sum u R_k, sum u^2, sum c_k (u = C - R_j)
    int *d_succ = nullptr;        // update_reference_from_paths: the successful paths' indices
    int succ_cap = 0;
    int *d_jref = nullptr;        // SCPS: reference frame j of each replica's distance expansion
    int *d_jref_eval = nullptr;   // the same for the tube evaluation calls
    bool jref_init = true;        // a stack changed: pick every replica's reference frame before stepping
    float *d_coef = nullptr;      // SCPS: c_k / Z0 per replica
    float *d_E = nullptr;         // SCPS, two-pass form: effective references, replica r at RepDesc::eoff
    ScpsGroup *d_groups = nullptr;
    ScpsItem *d_sitems = nullptr;
    int n_sitems = 0;
    int kmax = KMAX;
    int wg = 64;     // persistent workgroup size
    int tuned = -1;  // -1 untuned; else 0 persistent (with wg), 1 per-step, 2 packed (with pk_waves),
                     // from scps_autotune or scps_set_launch
    int pk_waves = 4;  // packed kernel: wavefronts per workgroup
    int n_max = 0;     // longest chain among the replicas' systems
    int nbk = 0;     // nonbonded terms: bit 0 LJ, bit 1 Debye-Hueckel
    // cutoff variant: neighbour lists on the per-step path (rMD with both cutoffs set)
    bool nl = false;
    bool nl_stale = true;            // lists unbuilt, or built on a reference map since replaced
    float r_list = 0.f;
    int nb_max = 0;
    float4 *d_bounds = nullptr;      // [R][nb_max] block bounding spheres
    float4 *d_xref = nullptr;        // [sumNpad] positions at the last build
    float *d_bmax = nullptr;         // [sum nb] largest squared displacement per block since then
    int *d_rebuild = nullptr;        // [R]
    int *d_nl_cnt = nullptr;         // [sumNpad]
    int2 *d_nl = nullptr;            // [sumNpad][NL_CAP]
    int *d_first_blk = nullptr;      // [R + 1] blocks of 64 particles before each replica
    int *d_first_chunk = nullptr;    // [R + 1] chunks of the list force kernel before each replica
    double *d_zpart_nl = nullptr;    // [chunks] z partials of the list force kernel
    double *d_zbase = nullptr;       // [R] R2total of each replica's system
    std::vector<void *> owned;
};

namespace {

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            if (ctx) (ctx)->poisoned = true;                                                \
            return fail(SCPS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));  \
        }                                                                                   \
    } while (0)

template <typename T>
hipError_t dalloc(scps_ctx *c, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) c->owned.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return e;
}

void dfree(scps_ctx *c, void *p) {
    if (!p) return;
    auto it = std::find(c->owned.begin(), c->owned.end(), p);
    if (it != c->owned.end()) c->owned.erase(it);
    (void)hipFree(p);
}

KParams make_kparams(const scps_params &p) {
    KParams k{};
    k.inv_r0sq = (float)(1.0 / (p.r0_contact * p.r0_contact));
    k.g_scale = (float)(4.0 / (p.r0_contact * p.r0_contact));
    k.cp[0] = (float)(-2.0 * 4.0 / (p.r0_contact * p.r0_contact));
    k.cp[1] = (float)(-4.0 * 4.0 / (p.r0_contact * p.r0_contact));
    k.cp[2] = (float)(-6.0 * 4.0 / (p.r0_contact * p.r0_contact));
    k.cp[3] = (float)(-3.0 * 4.0 / (p.r0_contact * p.r0_contact));
    k.has_cut = p.r_cut_contact > 0.0;
    k.r_cut2 = (float)(p.r_cut_contact * p.r_cut_contact);
    k.has_cut_nb = p.r_cut_nb > 0.0;
    k.r_cut_nb2 = (float)(p.r_cut_nb * p.r_cut_nb);
    k.lj_A = (float)(48.0 * p.lj_eps * pow(p.lj_sigma, 12));
    k.lj_B = (float)(24.0 * p.lj_eps * pow(p.lj_sigma, 6));
    k.has_lj = p.lj_eps != 0.0;
    k.dh_pref = (float)p.dh_prefactor;
    k.dh_kappa = (float)p.dh_kappa;
    k.dh_kl2 = (float)(-p.dh_kappa * 1.4426950408889634);
    k.has_dh = p.dh_prefactor != 0.0;
    k.nb_excl = p.nb_excl;
    k.min_sep = p.min_seq_sep;
    k.integrator = p.integrator;
    k.dt = p.dt;
    k.kT = p.kT;
    k.gamma = p.gamma;
    k.c1 = exp(-p.gamma * p.dt);
    k.k_bond = p.k_bond;
    k.has_bond = p.k_bond != 0.0;
    k.r_bond = p.r_bond;
    k.k_R = p.k_R;
    k.lambda = p.lambda;
    k.k_s = p.k_s;
    k.k_w = p.k_w;
    k.wscale = p.w_form == SCPS_W_NO_INV_LAMBDA ? 1.0 : (p.lambda > 0 ? 1.0 / p.lambda : 0.0);
    k.seed_lo = (uint32_t)p.seed;
    k.seed_hi = (uint32_t)(p.seed >> 32);
    k.rep_base = (uint32_t)p.replica_base;
    return k;
}

scps_status upload_sysdesc(scps_ctx *c) {
    std::vector<SysDesc> d(c->sys.size());
    for (size_t s = 0; s < c->sys.size(); ++s) {
        const SysHost &h = c->sys[s];
        SysDesc &o = d[s];
        o.n = h.n;
        o.n_pad = h.n_pad;
        o.nb = h.nb;
        o.nc = h.nc;
        o.ncb = h.ncb;
        o.ntile_c = h.ntile_c;
        o.K = h.K;
        o.perm = h.d_perm;
        o.bond_next = h.d_bond_next;
        o.mass = h.d_mass;
        o.charge = h.d_charge;
        o.ref = h.d_ref;
        o.stack = h.d_stack;
        o.stack_pm = h.d_stack_pm;
        o.G = h.d_G;
        o.R2tile = h.d_R2tile;
        o.tiles = h.d_sched;
        o.tmask = h.d_sched_mask;
        o.ntile = (int)h.sched.size();
        o.Z0 = h.Z0;
    }
    HIP_TRY(c, hipMemcpy(c->d_sysd, d.data(), d.size() * sizeof(SysDesc), hipMemcpyHostToDevice));
    return SCPS_OK;
}

bool usable(scps_ctx *c, scps_status *st) {
    if (!c) {
        *st = fail(SCPS_ERR_INVALID_ARG, "context is NULL");
        return false;
    }
    if (c->poisoned) {
        *st = fail(SCPS_ERR_STATE, "context is poisoned by an earlier HIP or non-finite error");
        return false;
    }
    return true;
}

int pick_wg(int nb, int n_replicas) {
    const int ntile = nb * (nb + 1) / 2;
    if (ntile >= 16) return 1024;
    if (ntile >= 8) return 512;
    if (ntile >= 4) return 256;
    // a batch too small to give half the SIMDs (256 CUs x 4) a wavefront:
    // four wavefronts per replica share its tiles
    return n_replicas < 512 ? 256 : 64;
}

// Per-tile flags and sub-step masks of a system (see TILE_* in scps_internal.h).
void compute_tile_flags(SysHost &h, const scps_params &p) {
    const int nb = h.nb;
    h.tile_flags.assign((size_t)nb * nb, 0);
    h.tile_mask.assign((size_t)nb * nb, 0);
    std::vector<int> inv(h.n);
    for (int a = 0; a < h.n; ++a) inv[h.perm[a]] = a;
    // pairs that need a predicate: chain neighbours excluded from the
    // nonbonded sum, contact pairs within min_seq_sep
    for (int a = 0; a < h.n; ++a) {
        const int o = h.perm[a];
        for (int d = 1; d <= std::max(p.nb_excl, p.min_seq_sep) && o + d < h.n; ++d) {
            const int b = inv[o + d];
            const bool contact_close = d <= p.min_seq_sep && a < h.nc && b < h.nc;
            if (!(d <= p.nb_excl || contact_close)) continue;
            const int lo = std::min(a, b), hi = std::max(a, b);
            const int I = lo / TILE, J = hi / TILE;
            int k = ((hi % TILE) - (lo % TILE) + TILE) % TILE;
            if (I == J) k = std::min(k, TILE - k);   // a diagonal tile meets the pair at separations 1..32
            h.tile_mask[(size_t)I * nb + J] |= 1ull << k;
        }
    }
    for (int I = 0; I < nb; ++I)
        for (int J = I; J < nb; ++J) {
            int f = 0;
            uint64_t &m = h.tile_mask[(size_t)I * nb + J];
            if (I == J) f |= TILE_DIAG;
            if (I < h.ncb && J < h.ncb) {
                f |= TILE_CONTACT;
                if ((J + 1) * TILE > h.nc || p.r_cut_contact > 0.0) m = ~0ull;
            }
            if (p.r_cut_nb > 0.0) m = ~0ull;   // every pair tests the nonbonded cutoff
            if (m) f |= TILE_MASK;
            h.tile_flags[(size_t)I * nb + J] = f;
        }
}

// Relative cost of a tile pair, for load balancing: a contact tile costs
// about 1.85 nonbonded-only tiles; the predicated sub-steps about 25 % more.
double tile_cost(int f, uint64_t mask) {
    double c = (f & TILE_CONTACT) ? 1.85 : 1.0;
    const double steps = (f & TILE_DIAG) ? 32.0 : 64.0;
    c *= 1.0 + 0.25 * std::min(1.0, __builtin_popcountll(mask) / steps);
    if (f & TILE_DIAG) c *= 0.5;
    return c;
}

// The persistent kernel's work list, costliest first; its wavefronts claim
// entries dynamically in this order.  Off-diagonal tiles (I1, J), (I2, J) of
// the same class (contact, mask) are paired; every tile or pair is cut into
// segments of SEG_STEPS sub-steps (see SEG_STEPS for the encoding).
void build_schedule(SysHost &h) {
    struct Item {
        double cost;
        int2 code;
        uint64_t mask;
    };
    std::vector<Item> all;
    auto code = [](int I1, int I2, int J, int f, int kb, int ke) {
        return make_int2((I1 << 16) | J, f | ((I2 + 1) << 8) | (kb << 16) | (ke << 23));
    };
    auto push = [&](int I1, int I2, int J, int f, double cost) {
        const int kb = (f & TILE_DIAG) ? 1 : 0, ke = (f & TILE_DIAG) ? 33 : 64;
        uint64_t m = h.tile_mask[(size_t)I1 * h.nb + J];
        if (I2 >= 0) m |= h.tile_mask[(size_t)I2 * h.nb + J];
        if (m) f |= TILE_MASK;
        for (int k = kb; k < ke; k += SEG_STEPS) {
            const int k2 = std::min(k + SEG_STEPS, ke);
            all.push_back({cost * (k2 - k) / 64.0, code(I1, I2, J, f, k, k2), m});
        }
    };
    for (int J = 0; J < h.nb; ++J) {
        std::vector<int> waiting(8, -1);   // per class, an unpaired row I
        for (int I = 0; I <= J; ++I) {
            const int f = h.tile_flags[(size_t)I * h.nb + J];
            if (I == J) {
                push(I, -1, J, f, 2.0 * tile_cost(f, h.tile_mask[(size_t)I * h.nb + J]));   // half the sub-steps, same cost per sub-step
                continue;
            }
            const int cls = f & (TILE_CONTACT | TILE_MASK);
            if (waiting[cls] < 0) {
                waiting[cls] = I;
            } else {
                push(waiting[cls], I, J, f,
                     2.0 * tile_cost(f, h.tile_mask[(size_t)I * h.nb + J] |
                                            h.tile_mask[(size_t)waiting[cls] * h.nb + J]));
                waiting[cls] = -1;
            }
        }
        for (int cls = 0; cls < 8; ++cls)
            if (waiting[cls] >= 0) {
                const int f = h.tile_flags[(size_t)waiting[cls] * h.nb + J];
                push(waiting[cls], -1, J, f, tile_cost(f, h.tile_mask[(size_t)waiting[cls] * h.nb + J]));
            }
    }
    auto by_cost = [](const Item &a, const Item &b) { return a.cost > b.cost; };
    std::stable_sort(all.begin(), all.end(), by_cost);
    // cut the cheapest items into TAIL_STEPS-long pieces
    const size_t first_tail = all.size() > (size_t)TAIL_ITEMS ? all.size() - TAIL_ITEMS : 0;
    std::vector<Item> tail;
    for (size_t t = first_tail; t < all.size(); ++t) {
        const Item &it = all[t];
        const int f = it.code.y & 0xFF, I2 = ((it.code.y >> 8) & 0xFF) - 1;
        const int kb = (it.code.y >> 16) & 0x7F, ke = (it.code.y >> 23) & 0x7F;
        for (int k = kb; k < ke; k += TAIL_STEPS) {
            const int k2 = std::min(k + TAIL_STEPS, ke);
            tail.push_back({it.cost * (k2 - k) / (ke - kb), code(it.code.x >> 16, I2, it.code.x & 0xFFFF, f, k, k2),
                            it.mask});
        }
    }
    all.resize(first_tail);
    std::stable_sort(tail.begin(), tail.end(), by_cost);
    all.insert(all.end(), tail.begin(), tail.end());
    h.sched.clear();
    h.sched_mask.clear();
    for (const auto &t : all) {
        h.sched.push_back(t.code);
        h.sched_mask.push_back(t.mask);
    }
}

// Replicas of each system in groups of up to SCPS_GROUP, one item per
// (group, contact tile pair), and the distance accumulators X, Q: what the
// matrix-core tube-variable passes need.  Built at init for SCPS contexts and
// on first use by the evaluation calls otherwise.
scps_status ensure_scps_groups(scps_ctx *c) {
    if (c->d_groups) return SCPS_OK;
    const int R = c->R;
    HIP_TRY(c, dalloc(c, &c->d_X, (size_t)R * c->kmax));
    HIP_TRY(c, hipMemset(c->d_X, 0, (size_t)R * c->kmax * sizeof(double)));
    HIP_TRY(c, dalloc(c, &c->d_Q, R));
    HIP_TRY(c, hipMemset(c->d_Q, 0, R * sizeof(double)));
    HIP_TRY(c, dalloc(c, &c->d_jref, R));
    HIP_TRY(c, hipMemset(c->d_jref, 0, R * sizeof(int)));
    HIP_TRY(c, dalloc(c, &c->d_jref_eval, R));
    c->jref_init = true;
    std::vector<ScpsGroup> groups;
    std::vector<ScpsItem> items;
    for (int s = 0; s < (int)c->sys.size(); ++s) {
        std::vector<int> mine;
        for (int r = 0; r < R; ++r)
            if (c->rep_sys[r] == s) mine.push_back(r);
        const SysHost &h = c->sys[s];
        for (size_t b = 0; b < mine.size(); b += SCPS_GROUP) {
            ScpsGroup g{};
            g.sys = s;
            g.nrep = (int)std::min<size_t>(SCPS_GROUP, mine.size() - b);
            for (int k = 0; k < g.nrep; ++k) g.rep[k] = mine[b + k];
            const int gi = (int)groups.size();
            groups.push_back(g);
            // diagonal by diagonal (J - I = d), so that the items that run at the
            // same time add their forces to different blocks
            for (int d = 0; d < h.ncb; ++d)
                for (int I = 0; I + d < h.ncb; ++I) {
                    const int J = I + d;
                    items.push_back(ScpsItem{gi, tile_index(I, J, h.ncb), (I << 16) | J,
                                             h.tile_flags[(size_t)I * h.nb + J]});
                }
        }
    }
    c->n_sitems = (int)items.size();
    HIP_TRY(c, dalloc(c, &c->d_groups, groups.size()));
    HIP_TRY(c, hipMemcpy(c->d_groups, groups.data(), groups.size() * sizeof(ScpsGroup), hipMemcpyHostToDevice));
    HIP_TRY(c, dalloc(c, &c->d_sitems, items.size()));
    if (!items.empty())
        HIP_TRY(c, hipMemcpy(c->d_sitems, items.data(), items.size() * sizeof(ScpsItem), hipMemcpyHostToDevice));
    return SCPS_OK;
}

scps_status init_impl(const scps_params *params, const scps_topology *topo, int32_t R, const int32_t *rsys,
                      void *stream, scps_ctx **out) {
    if (!params || !topo || !rsys || !out) return fail(SCPS_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const scps_params &p = *params;
    if (p.integrator != SCPS_INTEGRATOR_OVERDAMPED && p.integrator != SCPS_INTEGRATOR_BAOAB)
        return fail(SCPS_ERR_INVALID_ARG, "integrator must be 0 (overdamped) or 1 (BAOAB)");
    if (p.bias_mode != SCPS_BIAS_RMD && p.bias_mode != SCPS_BIAS_SCPS)
        return fail(SCPS_ERR_INVALID_ARG, "bias_mode must be 0 (rMD) or 1 (SCPS)");
    if (p.exec_mode != SCPS_EXEC_AUTO && p.exec_mode != SCPS_EXEC_PER_STEP &&
        p.exec_mode != SCPS_EXEC_PER_STEP_ALL_TILES && p.exec_mode != SCPS_EXEC_PER_STEP_OVERLAP)
        return fail(SCPS_ERR_INVALID_ARG, "exec_mode must be 0, 1, 2 or 3");
    if (p.exec_mode == SCPS_EXEC_PER_STEP_OVERLAP && p.bias_mode != SCPS_BIAS_SCPS)
        return fail(SCPS_ERR_INVALID_ARG, "exec_mode 3 (nonbonded pass beside the distance pass) needs SCPS bias");
    if (!(p.dt > 0) || !(p.gamma > 0) || !(p.kT >= 0) || !(p.r0_contact > 0))
        return fail(SCPS_ERR_INVALID_ARG, "dt, gamma, r0_contact must be > 0 and kT >= 0");
    if (p.w_form != SCPS_W_INV_LAMBDA && p.w_form != SCPS_W_NO_INV_LAMBDA)
        return fail(SCPS_ERR_INVALID_ARG, "w_form must be 0 (w with 1/lambda) or 1 (without)");
    if (p.nb_excl < 1 || p.min_seq_sep < 0 || p.replica_base < 0)
        return fail(SCPS_ERR_INVALID_ARG, "nb_excl must be >= 1, min_seq_sep and replica_base >= 0");
    if (p.bias_mode == SCPS_BIAS_SCPS && !(p.lambda > 0))
        return fail(SCPS_ERR_INVALID_ARG, "lambda must be > 0 in SCPS mode");
    if (p.lj_eps != 0.0 && !(p.lj_sigma > 0)) return fail(SCPS_ERR_INVALID_ARG, "lj_sigma must be > 0");
    if (topo->n_systems < 1 || !topo->n_particles || !topo->n_contact || !topo->mass || !topo->charge)
        return fail(SCPS_ERR_INVALID_ARG, "topology needs n_systems >= 1 and non-NULL arrays");
    if (R < 1) return fail(SCPS_ERR_INVALID_ARG, "n_replicas must be >= 1");
    if (R > 65535) return fail(SCPS_ERR_SHAPE, "n_replicas must be <= 65535 (one grid row per replica)");

    scps_ctx *c = new (std::nothrow) scps_ctx();
    if (!c) return fail(SCPS_ERR_OOM, "host allocation failed");
    std::unique_ptr<scps_ctx, void (*)(scps_ctx *)> guard(c, scps_destroy);
    c->prm = p;
    c->kp = make_kparams(p);
    c->stream = (hipStream_t)stream;
    c->R = R;

    int64_t poff_part = 0, poff_cidx = 0;
    c->sys.resize(topo->n_systems);
    for (int s = 0; s < topo->n_systems; ++s) {
        SysHost &h = c->sys[s];
        h.n = topo->n_particles[s];
        h.nc = topo->n_contact[s];
        if (h.n < 2 || h.n > (1 << 20)) return fail(SCPS_ERR_SHAPE, "n_particles must be in [2, 2^20]");
        if (h.nc < 0 || h.nc > h.n) return fail(SCPS_ERR_SHAPE, "n_contact must be in [0, n_particles]");
        if (h.nc > 0 && !topo->contact_idx) return fail(SCPS_ERR_INVALID_ARG, "contact_idx is NULL");
        h.n_pad = (h.n + TILE - 1) / TILE * TILE;
        h.nb = h.n_pad / TILE;
        h.ncb = (h.nc + TILE - 1) / TILE;
        h.ntile_c = h.ncb * (h.ncb + 1) / 2;
        const int32_t *ci = topo->contact_idx + poff_cidx;
        std::vector<char> in_c(h.n, 0);
        for (int a = 0; a < h.nc; ++a) {
            if (ci[a] < 0 || ci[a] >= h.n || (a > 0 && ci[a] <= ci[a - 1]))
                return fail(SCPS_ERR_INVALID_ARG, "contact_idx must be strictly ascending within [0, N)");
            in_c[ci[a]] = 1;
        }
        h.perm.resize(h.n_pad);
        std::vector<int> inv(h.n);
        int k = 0;
        for (int a = 0; a < h.nc; ++a) h.perm[k++] = ci[a];
        for (int i = 0; i < h.n; ++i)
            if (!in_c[i]) h.perm[k++] = i;
        for (int a = h.n; a < h.n_pad; ++a) h.perm[a] = a;  // pads: indices >= n
        for (int a = 0; a < h.n; ++a) inv[h.perm[a]] = a;
        h.bond_next.assign(h.n_pad, -1);
        h.mass.assign(h.n_pad, 1.f);
        h.charge.assign(h.n_pad, 0.f);
        for (int a = 0; a < h.n; ++a) {
            const int o = h.perm[a];
            if (o + 1 < h.n) h.bond_next[a] = inv[o + 1];
            const float m = topo->mass[poff_part + o];
            if (!(m > 0.f)) return fail(SCPS_ERR_INVALID_ARG, "masses must be > 0");
            h.mass[a] = m;
            h.charge[a] = topo->charge[poff_part + o];
        }
        poff_part += h.n;
        poff_cidx += h.nc;
        c->n_pad_max = std::max(c->n_pad_max, h.n_pad);
    }
    c->rep_sys.assign(rsys, rsys + R);
    c->rep_off.resize(R + 1);
    c->rep_poff.resize(R + 1);
    c->rep_off[0] = c->rep_poff[0] = 0;
    for (int r = 0; r < R; ++r) {
        if (rsys[r] < 0 || rsys[r] >= topo->n_systems)
            return fail(SCPS_ERR_INVALID_ARG, "replica_system entry out of range");
        c->rep_off[r + 1] = c->rep_off[r] + c->sys[rsys[r]].n;
        c->n_max = std::max(c->n_max, c->sys[rsys[r]].n);
        c->rep_poff[r + 1] = c->rep_poff[r] + c->sys[rsys[r]].n_pad;
    }
    c->sumN = c->rep_off[R];
    c->sumNpad = c->rep_poff[R];
    c->wg = pick_wg(c->n_pad_max / TILE, c->R);
    c->nbk = (p.lj_eps != 0.0 ? 1 : 0) | (p.dh_prefactor != 0.0 ? 2 : 0);
    for (auto &h : c->sys) {
        compute_tile_flags(h, p);
        build_schedule(h);
    }

    // device buffers
    for (auto &h : c->sys) {
        HIP_TRY(c, dalloc(c, &h.d_perm, h.n_pad));
        HIP_TRY(c, dalloc(c, &h.d_bond_next, h.n_pad));
        HIP_TRY(c, dalloc(c, &h.d_mass, h.n_pad));
        HIP_TRY(c, dalloc(c, &h.d_charge, h.n_pad));
        HIP_TRY(c, hipMemcpy(h.d_perm, h.perm.data(), h.n_pad * sizeof(int), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(h.d_bond_next, h.bond_next.data(), h.n_pad * sizeof(int), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(h.d_mass, h.mass.data(), h.n_pad * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(h.d_charge, h.charge.data(), h.n_pad * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(c, dalloc(c, &h.d_sched, h.sched.size()));
        HIP_TRY(c, hipMemcpy(h.d_sched, h.sched.data(), h.sched.size() * sizeof(int2), hipMemcpyHostToDevice));
        HIP_TRY(c, dalloc(c, &h.d_sched_mask, h.sched_mask.size()));
        HIP_TRY(c, hipMemcpy(h.d_sched_mask, h.sched_mask.data(), h.sched_mask.size() * sizeof(uint64_t),
                             hipMemcpyHostToDevice));
    }
    HIP_TRY(c, dalloc(c, &c->d_sysd, c->sys.size()));
    scps_status st = upload_sysdesc(c);
    if (st != SCPS_OK) return st;

    std::vector<RepDesc> reps(R);
    int64_t eoff = 0;
    for (int r = 0; r < R; ++r) {
        reps[r].sys = rsys[r];
        reps[r].off = c->rep_off[r];
        reps[r].poff = c->rep_poff[r];
        reps[r].eoff = eoff;
        eoff += (int64_t)c->sys[rsys[r]].ntile_c * 4096;
    }
    HIP_TRY(c, dalloc(c, &c->d_reps, R));
    HIP_TRY(c, hipMemcpy(c->d_reps, reps.data(), R * sizeof(RepDesc), hipMemcpyHostToDevice));

    // persistent launch order: longest replicas first
    std::vector<int> order(R);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return c->sys[rsys[a]].n > c->sys[rsys[b]].n; });
    HIP_TRY(c, dalloc(c, &c->d_order, R));
    HIP_TRY(c, hipMemcpy(c->d_order, order.data(), R * sizeof(int), hipMemcpyHostToDevice));

    // per-step work lists: every tile pair, and the contact tile pairs,
    // replica by replica
    std::vector<TileItem> all, con;
    std::vector<int> first_all(R + 1), first_con(R + 1);
    for (int r = 0; r < R; ++r) {
        first_all[r] = (int)all.size();
        first_con[r] = (int)con.size();
        const SysHost &h = c->sys[rsys[r]];
        for (int I = 0; I < h.nb; ++I)
            for (int J = I; J < h.nb; ++J) {
                TileItem t{r, I, J, h.tile_flags[(size_t)I * h.nb + J], h.tile_mask[(size_t)I * h.nb + J]};
                all.push_back(t);
                if (I < h.ncb && J < h.ncb) con.push_back(t);
            }
    }
    first_all[R] = (int)all.size();
    first_con[R] = (int)con.size();
    c->n_items_all = (int)all.size();
    c->n_items_contact = (int)con.size();
    HIP_TRY(c, dalloc(c, &c->d_zpart, all.size()));
    HIP_TRY(c, dalloc(c, &c->d_first_all, R + 1));
    HIP_TRY(c, dalloc(c, &c->d_first_con, R + 1));
    HIP_TRY(c, hipMemcpy(c->d_first_all, first_all.data(), (R + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_first_con, first_con.data(), (R + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(c, dalloc(c, &c->d_items_all, all.size()));
    HIP_TRY(c, dalloc(c, &c->d_items_contact, con.size()));
    if (!all.empty())
        HIP_TRY(c, hipMemcpy(c->d_items_all, all.data(), all.size() * sizeof(TileItem), hipMemcpyHostToDevice));
    if (!con.empty())
        HIP_TRY(c, hipMemcpy(c->d_items_contact, con.data(), con.size() * sizeof(TileItem),
                             hipMemcpyHostToDevice));

    c->nl = p.bias_mode == SCPS_BIAS_RMD && p.r_cut_contact > 0.0 && p.r_cut_nb > 0.0 &&
            p.exec_mode != SCPS_EXEC_PER_STEP_ALL_TILES && !all.empty();
    if (c->nl) {
        c->r_list = (float)std::max(p.r_cut_contact, p.r_cut_nb) + NL_SKIN;
        std::vector<int> fb(R + 1, 0), fc(R + 1, 0);
        for (int r = 0; r < R; ++r) {
            const SysHost &h = c->sys[rsys[r]];
            c->nb_max = std::max(c->nb_max, h.nb);
            fb[r + 1] = fb[r] + h.nb;
            fc[r + 1] = fc[r] + nl_chunks(h.n_pad);
        }
        HIP_TRY(c, dalloc(c, &c->d_bounds, (size_t)R * c->nb_max));
        HIP_TRY(c, dalloc(c, &c->d_xref, c->sumNpad));
        HIP_TRY(c, dalloc(c, &c->d_bmax, fb[R]));
        HIP_TRY(c, dalloc(c, &c->d_rebuild, R));
        HIP_TRY(c, dalloc(c, &c->d_nl_cnt, c->sumNpad));
        HIP_TRY(c, dalloc(c, &c->d_nl, (size_t)c->sumNpad * NL_CAP));
        HIP_TRY(c, dalloc(c, &c->d_first_blk, R + 1));
        HIP_TRY(c, hipMemcpy(c->d_first_blk, fb.data(), (R + 1) * sizeof(int), hipMemcpyHostToDevice));
        HIP_TRY(c, dalloc(c, &c->d_first_chunk, R + 1));
        HIP_TRY(c, hipMemcpy(c->d_first_chunk, fc.data(), (R + 1) * sizeof(int), hipMemcpyHostToDevice));
        HIP_TRY(c, dalloc(c, &c->d_zpart_nl, fc[R]));
        HIP_TRY(c, dalloc(c, &c->d_zbase, R));
        HIP_TRY(c, hipMemset(c->d_zbase, 0, R * sizeof(double)));
    }
    HIP_TRY(c, dalloc(c, &c->d_flags, R));
    HIP_TRY(c, hipMemset(c->d_flags, 0, R * sizeof(int)));
    HIP_TRY(c, dalloc(c, &c->d_xs, 2 * c->sumNpad));
    HIP_TRY(c, dalloc(c, &c->d_vs, c->sumNpad));
    HIP_TRY(c, dalloc(c, &c->d_acc, 6 * c->sumNpad));
    HIP_TRY(c, hipMemset(c->d_acc, 0, 6 * c->sumNpad * sizeof(double)));
    HIP_TRY(c, dalloc(c, &c->d_negone, R));
    std::vector<double> neg(R, -1.0);
    HIP_TRY(c, hipMemcpy(c->d_negone, neg.data(), R * sizeof(double), hipMemcpyHostToDevice));
    if (p.bias_mode == SCPS_BIAS_SCPS) {
        HIP_TRY(c, dalloc(c, &c->d_coef, (size_t)R * c->kmax));
        HIP_TRY(c, dalloc(c, &c->d_csum, R));
        if (p.exec_mode == SCPS_EXEC_PER_STEP_ALL_TILES) {   // the two-pass form keeps E in device memory
            HIP_TRY(c, dalloc(c, &c->d_E, (size_t)eoff));
        } else {
            HIP_TRY(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
            HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
            HIP_TRY(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
            c->overlap_nb = p.exec_mode == SCPS_EXEC_PER_STEP_OVERLAP;
        }
        scps_status st2 = ensure_scps_groups(c);
        if (st2 != SCPS_OK) return st2;
    }
    *out = guard.release();
    return SCPS_OK;
}

// The pair-major copy of a system's frame stack and its frame distances G,
// rebuilt whenever the stack changes; every replica's reference frame is
// picked again before the next SCPS step.
scps_status make_pairmajor(scps_ctx *c, SysHost &h) {
    if (h.K_pm != h.K) {   // multi-GB buffers: allocated again only when the frame count changes
        dfree(c, h.d_stack_pm);
        dfree(c, h.d_G);
        h.d_stack_pm = nullptr;
        h.d_G = nullptr;
        h.K_pm = 0;
        HIP_TRY(c, dalloc(c, &h.d_stack_pm, (size_t)stack_pm_width(h.K) * h.ntile_c * 4096));
        HIP_TRY(c, dalloc(c, &h.d_G, (size_t)h.K * h.K));
        h.K_pm = h.K;
    }
    HIP_TRY(c, hipMemsetAsync(h.d_G, 0, (size_t)h.K * h.K * sizeof(double), c->stream));
    HIP_TRY(c, launch_stack_pairmajor(h.nc, h.ncb, h.K, h.d_stack, h.d_stack_pm, c->stream));
    HIP_TRY(c, launch_stack_gram(h.nc, h.ncb, h.K, c->prm.min_seq_sep, h.d_perm, h.d_stack, h.d_G, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->jref_init = true;
    return SCPS_OK;
}

scps_status set_ref_impl(scps_ctx *c, int32_t s, int32_t n_maps, const double *maps, const double *xyz,
                         double z0) {
    if (s < 0 || s >= (int)c->sys.size()) return fail(SCPS_ERR_INVALID_ARG, "system index out of range");
    SysHost &h = c->sys[s];
    const int64_t P = (int64_t)h.nc * (h.nc - 1) / 2;
    if (n_maps < 1) return fail(SCPS_ERR_INVALID_ARG, "n_maps must be >= 1");
    if (n_maps == 1) {
        if (!maps && !xyz) return fail(SCPS_ERR_INVALID_ARG, "need maps or native_xyz");
        if (!h.d_ref) HIP_TRY(c, dalloc(c, &h.d_ref, (size_t)h.ntile_c * 4096));
        double *d_packed = nullptr, *d_sum = nullptr;
        HIP_TRY(c, dalloc(c, &d_packed, (size_t)std::max<int64_t>(P, 1)));
        HIP_TRY(c, dalloc(c, &d_sum, 1 + std::max(sum_squares_scratch(), h.nc)));
        if (maps) {
            HIP_TRY(c, hipMemcpy(d_packed, maps, P * sizeof(double), hipMemcpyHostToDevice));
            HIP_TRY(c, launch_pack_to_tiles(1, h.nc, h.ncb, d_packed, h.d_ref, c->stream));
        } else {
            double *d_xyz = nullptr;
            HIP_TRY(c, dalloc(c, &d_xyz, 3 * (size_t)h.n));
            HIP_TRY(c, hipMemcpy(d_xyz, xyz, 3 * h.n * sizeof(double), hipMemcpyHostToDevice));
            HIP_TRY(c, launch_native_map(h.n, h.n_pad, h.nc, h.ncb, h.d_perm, d_xyz, c->prm.r0_contact,
                                         c->prm.r_cut_contact, h.d_ref, d_packed, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            dfree(c, d_xyz);
        }
        double zz = z0;
        if (!(z0 > 0.0)) {
            // the denominator of the normalised distance sums over the pairs its
            // numerator does: |i-j| > min_seq_sep
            if (c->prm.min_seq_sep > 0)
                HIP_TRY(c, launch_sum_squares_sep(h.nc, c->prm.min_seq_sep, h.d_perm, d_packed, d_sum + 1, d_sum,
                                                  c->stream));
            else
                HIP_TRY(c, launch_sum_squares(P, d_packed, d_sum + 1, d_sum, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipMemcpy(&zz, d_sum, sizeof(double), hipMemcpyDeviceToHost));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c, d_packed);
        dfree(c, d_sum);
        h.Z0 = zz;
        h.has_native = true;
        // per-tile sums of R^2 (the culled path's z offset)
        if (h.ntile_c > 0) {
            if (!h.d_R2tile) HIP_TRY(c, dalloc(c, &h.d_R2tile, h.ntile_c));
            HIP_TRY(c, launch_tile_sumsq(h.nc, h.ncb, c->prm.min_seq_sep, h.d_perm, h.d_ref, h.d_R2tile, c->stream));
            std::vector<double> r2(h.ntile_c);
            HIP_TRY(c, hipMemcpyAsync(r2.data(), h.d_R2tile, h.ntile_c * sizeof(double), hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            h.R2total = 0.0;
            for (double v : r2) h.R2total += v;
        }
        c->nl_stale = true;
        if (c->nl) {
            std::vector<double> zb(c->R);
            for (int r = 0; r < c->R; ++r) zb[r] = c->sys[c->rep_sys[r]].R2total;
            HIP_TRY(c, hipMemcpyAsync(c->d_zbase, zb.data(), c->R * sizeof(double), hipMemcpyHostToDevice,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
        }
    } else {
        if (!maps || xyz) return fail(SCPS_ERR_INVALID_ARG, "a frame stack needs maps and no native_xyz");
        if (n_maps > KMAX) return fail(SCPS_ERR_SHAPE, "at most " + std::to_string(KMAX) + " frames in an SCPS stack");
        if (h.K != n_maps) {
            dfree(c, h.d_stack);
            h.d_stack = nullptr;
            h.K = 0;
            HIP_TRY(c, dalloc(c, &h.d_stack, (size_t)n_maps * h.ntile_c * 4096));
        }
        double *d_packed = nullptr;
        HIP_TRY(c, dalloc(c, &d_packed, (size_t)std::max<int64_t>(P * n_maps, 1)));
        HIP_TRY(c, hipMemcpy(d_packed, maps, (size_t)P * n_maps * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(c, launch_pack_to_tiles(n_maps, h.nc, h.ncb, d_packed, h.d_stack, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c, d_packed);
        h.K = n_maps;
        scps_status st = make_pairmajor(c, h);
        if (st != SCPS_OK) return st;
    }
    return upload_sysdesc(c);
}

// Read back the oldest recorded slot of the pass-timing ring (waits for it).
scps_status read_pass_slot(scps_ctx *c) {
    const int slot = (int)(c->pass_read % scps_ctx::PASS_RING);
    hipEvent_t *e = &c->pass_ev[4 * slot];
    HIP_TRY(c, hipEventSynchronize(e[3]));
    float a = 0.f, b = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&a, e[0], e[1]));
    HIP_TRY(c, hipEventElapsedTime(&b, e[2], e[3]));
    c->pass_ms[0] += a;
    c->pass_ms[1] += b;
    ++c->pass_read;
    return SCPS_OK;
}

// The events of the current step's slot (recycling the oldest one when the
// ring is full), or nullptr when pass timing is off.
hipEvent_t *pass_slot(scps_ctx *c, scps_status *st) {
    *st = SCPS_OK;
    if (!c->timing) return nullptr;
    if (c->timing_tick++ % c->timing_period != 0) return nullptr;
    if (c->pass_recorded - c->pass_read == scps_ctx::PASS_RING) {
        *st = read_pass_slot(c);
        if (*st != SCPS_OK) return nullptr;
    }
    return &c->pass_ev[4 * (int)(c->pass_recorded % scps_ctx::PASS_RING)];
}

// The largest frame stack among the systems the replicas run (SCPS passes).
int max_stack_frames(const scps_ctx *c) {
    int k = 1;
    for (int r = 0; r < c->R; ++r) k = std::max(k, c->sys[c->rep_sys[r]].K);
    return k;
}

// The launch scps_step_replicas takes: 0 the persistent kernel (c->wg
// threads per replica), 1 the per-step path, 2 the packed kernel (c->pk_waves
// wavefronts per workgroup).
int launch_path(const scps_ctx *c) {
    if (c->prm.bias_mode == SCPS_BIAS_SCPS || c->prm.exec_mode != SCPS_EXEC_AUTO) return 1;
    // untuned, short chains run packed (several, or one, per wavefront)
    if (c->tuned == 2 || (c->tuned == -1 && packed_default(c->n_max, c->R))) return 2;
    if (c->tuned == 1 || c->n_pad_max > persistent_max_npad(c->wg)) return 1;
    return 0;
}

// {path, parameter} as scps_autotune and scps_get_launch report them.
void launch_report(const scps_ctx *c, int path, int32_t *out) {
    out[0] = path;
    out[1] = path == 0   ? c->wg
             : path == 2 ? c->pk_waves * (64 / c->n_max)
                         : (c->prm.bias_mode == SCPS_BIAS_SCPS && c->overlap_nb ? 1 : 0);
}

// The kernel launches of one step of the per-step path (all tile pairs for
// rMD; the SCPS passes), on stream st, the update drawing its noise for step
// step (+ *step_base when given).  eager: the overlapped SCPS schedule and
// pass timing may be used (never while a graph is being captured).
scps_status step_launches(scps_ctx *c, double *cv, uint64_t step, const uint64_t *step_base, bool eager,
                          hipStream_t st) {
    if (c->prm.bias_mode != SCPS_BIAS_SCPS) {
        HIP_TRY(c, launch_pairs(0, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_items_all, c->n_items_all, c->d_xs,
                                c->d_acc, c->d_zpart, nullptr, nullptr, st));
        HIP_TRY(c, launch_integrate(c->kp, c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_xs, c->d_vs, c->d_acc,
                                    nullptr, cv, step, step_base, c->d_flags, st, c->d_first_all, c->d_zpart,
                                    nullptr));
        return SCPS_OK;
    }
    // distances to every frame (matrix cores), tube variables and ratchets,
    // effective references (matrix cores), bias + physics
    // (also while the step is captured into a graph: the fork and join become
    // the graph's branch and merge, with no per-step event cost at replay)
    const bool overlap = (eager || st == c->cap) && c->side && c->overlap_nb;
    if (overlap) {
        // nonbonded forces (acc components 0..2) need only the positions:
        // they overlap the bandwidth-bound distance pass
        HIP_TRY(c, hipEventRecord(c->ev_fork, st));
        HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
        HIP_TRY(c, launch_pairs(4, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_items_all, c->n_items_all, c->d_xs,
                                c->d_acc, c->d_zpart, nullptr, nullptr, c->side));
        HIP_TRY(c, hipEventRecord(c->ev_join, c->side));
    }
    hipEvent_t *tev = nullptr;
    if (eager) {
        scps_status tst;
        tev = pass_slot(c, &tst);
        if (tst != SCPS_OK) return tst;
    }
    if (tev) HIP_TRY(c, hipEventRecord(tev[0], st));
    HIP_TRY(c, launch_scps_dist(c->kp, c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems,
                                max_stack_frames(c), c->d_jref, c->d_xs, c->d_X, c->d_Q, c->kmax, -1, st));
    if (tev) HIP_TRY(c, hipEventRecord(tev[1], st));
    HIP_TRY(c, launch_finalize_scps(c->kp, c->d_sysd, c->d_reps, c->R, c->kmax, c->d_jref, c->d_X, c->d_Q, cv,
                                    c->d_coef, c->d_csum, st));
    if (tev) HIP_TRY(c, hipEventRecord(tev[2], st));
    if (c->prm.exec_mode == SCPS_EXEC_PER_STEP_ALL_TILES) {
        // two passes: effective references to device memory, then every tile pair
        HIP_TRY(c, launch_scps_eff(c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems, c->d_coef, c->kmax,
                                   c->d_E, st));
        HIP_TRY(c, launch_pairs(3, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_items_all, c->n_items_all, c->d_xs,
                                c->d_acc, c->d_zpart, c->d_E, c->d_csum, st));
        if (tev) HIP_TRY(c, hipEventRecord(tev[3], st));
    } else {
        // the effective references and the bias in one pass over the contact tiles;
        // the nonbonded forces and bonds (mode 4, every tile pair) after it, or
        // joined from the side stream
        HIP_TRY(c, launch_scps_bias(c->kp, c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems,
                                    max_stack_frames(c), c->d_xs, c->d_coef, c->d_csum, c->kmax, c->d_acc, st));
        if (tev) HIP_TRY(c, hipEventRecord(tev[3], st));
        if (overlap)
            HIP_TRY(c, hipStreamWaitEvent(st, c->ev_join, 0));
        else
            HIP_TRY(c, launch_pairs(4, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_items_all, c->n_items_all,
                                    c->d_xs, c->d_acc, c->d_zpart, nullptr, nullptr, st));
    }
    if (tev) ++c->pass_recorded;
    HIP_TRY(c, launch_integrate(c->kp, c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_xs, c->d_vs, c->d_acc,
                                c->d_negone, cv, step, step_base, c->d_flags, st));
    return SCPS_OK;
}

void drop_step_graph(scps_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_cv = nullptr;
}

// The executable graph of graph_steps consecutive steps (captured on the
// context's private capture stream; replayed on its stream).  Its kernels
// read the state from the context's buffers, the replicas' cvstate from cv
// and the step from d_step, so a new capture is needed only when cv, the
// largest stack or the block length changes.
scps_status ensure_step_graph(scps_ctx *c, double *cv) {
    const int kf = max_stack_frames(c);
    if (c->gexec && c->g_cv == cv && c->g_frames == kf && c->g_steps == c->graph_steps &&
        c->g_overlap == c->overlap_nb)
        return SCPS_OK;
    drop_step_graph(c);
    if (!c->cap) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    if (!c->d_step) HIP_TRY(c, dalloc(c, &c->d_step, 1));
    HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    scps_status st = SCPS_OK;
    for (int u = 0; u < c->graph_steps && st == SCPS_OK; ++u)
        st = step_launches(c, cv, (uint64_t)u, c->d_step, false, c->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (st != SCPS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIP_TRY(c, e);
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(c, ei);
    c->g_cv = cv;
    c->g_frames = kf;
    c->g_steps = c->graph_steps;
    c->g_overlap = c->overlap_nb;
    return SCPS_OK;
}

scps_status step_impl(scps_ctx *c, float *x, float *v, double *cv, int64_t n_steps, uint64_t step0,
                      int32_t record_every, float *frames) {
    if (!x || !cv) return fail(SCPS_ERR_INVALID_ARG, "x and cvstate must not be NULL");
    if (n_steps < 0 || record_every < 0) return fail(SCPS_ERR_INVALID_ARG, "n_steps and record_every must be >= 0");
    if (record_every > 0 && !frames) return fail(SCPS_ERR_INVALID_ARG, "frames is NULL but record_every > 0");
    if (c->prm.integrator == SCPS_INTEGRATOR_BAOAB && !v)
        return fail(SCPS_ERR_INVALID_ARG, "BAOAB needs velocities");
    const bool scps = c->prm.bias_mode == SCPS_BIAS_SCPS;
    for (int r = 0; r < c->R; ++r) {
        const SysHost &h = c->sys[c->rep_sys[r]];
        if (!h.has_native) return fail(SCPS_ERR_STATE, "a system has no native map (scps_set_reference_map)");
        if (scps && h.K < 2) return fail(SCPS_ERR_STATE, "SCPS mode needs a frame stack of >= 2 maps");
    }
    const int64_t frame_stride = 3 * c->sumN;
    const int path = launch_path(c);
    if (path == 2) {
        HIP_TRY(c, launch_packed_rmd(c->pk_waves, c->nbk, c->kp, c->d_sysd, c->d_reps, c->R, c->n_max, x, v, cv,
                                     n_steps, step0, record_every, frames, frame_stride, c->d_flags, c->stream));
        return SCPS_OK;
    }
    if (path == 0) {
        HIP_TRY(c, launch_persistent_rmd(c->wg, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_order, c->R, c->n_pad_max, x, v, cv,
                                         n_steps, step0, record_every, frames, frame_stride, c->d_flags,
                                         c->stream));
        return SCPS_OK;
    }
    HIP_TRY(c, launch_gather(c->d_sysd, c->d_reps, c->R, c->n_pad_max, x, v, c->d_xs, v ? c->d_vs : nullptr,
                             c->stream));
    // whole blocks of graph_steps steps replay one captured graph (not with
    // neighbour lists or pass timing; the overlapped SCPS schedule is captured
    // as two branches); a block never crosses a recorded frame or the end of
    // the call
    const int B = c->graph_steps;
    const bool graphs = B > 0 && !(!scps && c->nl) && !c->timing;
    for (int64_t m = 0;;) {
        if (record_every > 0 && m % record_every == 0)
            HIP_TRY(c, launch_scatter(c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_xs, nullptr, nullptr, nullptr,
                                      frames + (m / record_every) * frame_stride, c->stream));
        if (m == n_steps) break;
        if (scps && c->jref_init) {
            // a new stack: every replica's reference frame is its nearest frame,
            // from one distance pass around frame 0
            HIP_TRY(c, launch_scps_dist(c->kp, c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems,
                                        max_stack_frames(c), nullptr, c->d_xs, c->d_X, c->d_Q, c->kmax, -1,
                                        c->stream));
            HIP_TRY(c, launch_tube_eval(c->prm.lambda, c->kp.wscale, nullptr, c->d_jref, c->d_sysd, c->d_reps,
                                        c->R, c->kmax, -1, c->d_X, c->d_Q, nullptr, nullptr, nullptr, 0.0, 1,
                                        c->stream));
            c->jref_init = false;
        }
        const int64_t until = record_every > 0 ? std::min(n_steps, (m / record_every + 1) * record_every) : n_steps;
        if (graphs && until - m >= B) {
            scps_status gs = ensure_step_graph(c, cv);
            if (gs != SCPS_OK) return gs;
            HIP_TRY(c, launch_set_step(c->d_step, step0 + (uint64_t)m, c->stream));
            HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
            m += B;
            continue;
        }
        if (!scps && c->nl) {
            // cutoff variant: neighbour lists, rebuilt where a particle moved more than half the skin
            HIP_TRY(c, launch_nl_update(c->kp, c->d_sysd, c->d_reps, c->R, c->nb_max, c->d_first_blk, c->d_xs,
                                        c->d_bounds, c->d_xref, c->d_bmax, c->d_rebuild, c->nl_stale, c->d_items_all,
                                        c->d_first_all, c->r_list, c->d_nl_cnt, c->d_nl, c->d_flags, c->stream));
            c->nl_stale = false;
            HIP_TRY(c, launch_nl_force(c->nbk, c->kp, c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_first_chunk,
                                       c->d_xs, c->d_nl_cnt, c->d_nl, c->d_acc, c->d_zpart_nl, c->stream));
            HIP_TRY(c, launch_integrate(c->kp, c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_xs, c->d_vs, c->d_acc,
                                        nullptr, cv, step0 + (uint64_t)m, nullptr, c->d_flags, c->stream,
                                        c->d_first_chunk, c->d_zpart_nl, c->d_zbase));
        } else {
            scps_status ss = step_launches(c, cv, step0 + (uint64_t)m, nullptr, true, c->stream);
            if (ss != SCPS_OK) return ss;
        }
        ++m;
    }
    HIP_TRY(c, launch_scatter(c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_xs, v ? c->d_vs : nullptr, x, v,
                              nullptr, c->stream));
    return SCPS_OK;
}

scps_status eval_impl(scps_ctx *c, const float *x, double *z, float *grad, const double *coef,
                      const double *z_m = nullptr, double *E_b = nullptr) {
    if (!x || !z) return fail(SCPS_ERR_INVALID_ARG, "x and z must not be NULL");
    for (int r = 0; r < c->R; ++r)
        if (!c->sys[c->rep_sys[r]].has_native)
            return fail(SCPS_ERR_STATE, "a system has no native map (scps_set_reference_map)");
    HIP_TRY(c, launch_gather(c->d_sysd, c->d_reps, c->R, c->n_pad_max, x, nullptr, c->d_xs, nullptr, c->stream));
    HIP_TRY(c, launch_pairs(grad ? 2 : 1, c->nbk, c->kp, c->d_sysd, c->d_reps, c->d_items_contact, c->n_items_contact,
                            c->d_xs, c->d_acc, c->d_zpart, nullptr, nullptr, c->stream));
    HIP_TRY(c, launch_eval_out(c->d_sysd, c->d_reps, c->R, c->n_pad_max, c->d_acc, c->d_first_con, c->d_zpart, z,
                               c->prm.k_R, z_m, E_b, grad, coef, c->stream));
    return SCPS_OK;
}

scps_status update_ref_impl(scps_ctx *c, int32_t s, const float *frames, int32_t n_paths, int32_t n_frames,
                            const uint8_t *success, double *maps_out) {
    if (s < 0 || s >= (int)c->sys.size()) return fail(SCPS_ERR_INVALID_ARG, "system index out of range");
    if (!frames || !success) return fail(SCPS_ERR_INVALID_ARG, "frames and success must not be NULL");
    if (n_paths < 1 || n_frames < 1) return fail(SCPS_ERR_INVALID_ARG, "n_paths and n_frames must be >= 1");
    if (n_frames > KMAX) return fail(SCPS_ERR_SHAPE, "at most " + std::to_string(KMAX) + " frames in an SCPS stack");
    SysHost &h = c->sys[s];
    std::vector<int> succ;
    for (int q = 0; q < n_paths; ++q)
        if (success[q]) succ.push_back(q);
    if (succ.empty()) return fail(SCPS_ERR_NO_SUCCESS, "no successful path; the frame stack is unchanged");
    const int64_t P = (int64_t)h.nc * (h.nc - 1) / 2;
    if (c->succ_cap < (int)succ.size()) {
        dfree(c, c->d_succ);
        c->d_succ = nullptr;
        c->succ_cap = 0;
        HIP_TRY(c, dalloc(c, &c->d_succ, succ.size()));
        c->succ_cap = (int)succ.size();
    }
    int *d_succ = c->d_succ;
    HIP_TRY(c, hipMemcpyAsync(d_succ, succ.data(), succ.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    // the new stack replaces the old one in place when it has as many frames
    // (no kernel reads the old stack while eq (avCij) runs)
    float *d_new = (h.d_stack && h.K == n_frames) ? h.d_stack : nullptr;
    if (!d_new) HIP_TRY(c, dalloc(c, &d_new, (size_t)n_frames * h.ntile_c * 4096));
    double *d_packed = nullptr;
    if (maps_out) HIP_TRY(c, dalloc(c, &d_packed, (size_t)std::max<int64_t>(P * n_frames, 1)));
    HIP_TRY(c, launch_update_reference(h.n, h.n_pad, h.nc, h.ncb, h.d_perm, frames, n_paths, n_frames, d_succ,
                                       (int)succ.size(), c->prm.r0_contact, c->prm.r_cut_contact, d_new, d_packed,
                                       c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (maps_out)
        HIP_TRY(c, hipMemcpy(maps_out, d_packed, (size_t)P * n_frames * sizeof(double), hipMemcpyDeviceToHost));
    dfree(c, d_packed);
    if (d_new != h.d_stack) dfree(c, h.d_stack);
    h.d_stack = d_new;
    h.K = n_frames;
    scps_status st = make_pairmajor(c, h);
    if (st != SCPS_OK) return st;
    return upload_sysdesc(c);
}

scps_status least_biased_impl(scps_ctx *c, const double *cv, const uint8_t *success, int32_t *index,
                              double *t_min) {
    if (!cv || !index) return fail(SCPS_ERR_INVALID_ARG, "cvstate and index must not be NULL");
    std::vector<int> list;
    for (int r = 0; r < c->R; ++r)
        if (!success || success[r]) list.push_back(r);
    if (list.empty()) return fail(SCPS_ERR_NO_SUCCESS, "no successful path to select from");
    const int n = (int)list.size();
    int *d_list = nullptr;             // n replica ids, then {index, non-finite count}
    double *d_t = nullptr;
    HIP_TRY(c, dalloc(c, &d_list, (size_t)n + 2));
    HIP_TRY(c, dalloc(c, &d_t, 1));
    HIP_TRY(c, hipMemcpyAsync(d_list, list.data(), n * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_least_biased(cv, d_list, n, d_list + n, d_t, c->stream));
    int out[2];
    double t = 0.0;
    HIP_TRY(c, hipMemcpyAsync(out, d_list + n, sizeof(out), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&t, d_t, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c, d_list);
    dfree(c, d_t);
    if (out[1] > 0)
        return fail(SCPS_ERR_INVALID_ARG, std::to_string(out[1]) + " listed replica(s) have a non-finite T");
    *index = out[0];
    if (t_min) *t_min = t;
    return SCPS_OK;
}

// s, w (nullable) against one stack, or sigma (nullable) as the mean of
// 1 - s over several stacks; every replica's system must be the same chain
// and contact set as each stack's system.
scps_status eval_tube_impl(scps_ctx *c, int32_t n_stacks, const int32_t *stacks, const float *x, double *s,
                           double *w, double *sigma) {
    if (!x || !stacks || n_stacks < 1) return fail(SCPS_ERR_INVALID_ARG, "x and at least one stack system are needed");
    if (c->prm.bias_mode != SCPS_BIAS_SCPS && !(c->prm.lambda > 0))
        return fail(SCPS_ERR_INVALID_ARG, "lambda must be > 0 to evaluate tube variables");
    for (int k = 0; k < n_stacks; ++k) {
        const int b = stacks[k];
        if (b < 0 || b >= (int)c->sys.size()) return fail(SCPS_ERR_INVALID_ARG, "stack system index out of range");
        const SysHost &hb = c->sys[b];
        if (!hb.has_native || hb.K < 2)
            return fail(SCPS_ERR_STATE, "a stack system has no native map or no frame stack of >= 2 maps");
        for (int r = 0; r < c->R; ++r) {
            const SysHost &ha = c->sys[c->rep_sys[r]];
            if (ha.n != hb.n || ha.nc != hb.nc || ha.perm != hb.perm)
                return fail(SCPS_ERR_SHAPE, "every replica's chain and contact set must match the stack system's");
        }
    }
    scps_status st = ensure_scps_groups(c);
    if (st != SCPS_OK) return st;
    HIP_TRY(c, launch_gather(c->d_sysd, c->d_reps, c->R, c->n_pad_max, x, nullptr, c->d_xs, nullptr, c->stream));
    for (int k = 0; k < n_stacks; ++k) {
        // two passes: around frame 0, to find each replica's nearest frame, then around that frame
        const int K = c->sys[stacks[k]].K;
        HIP_TRY(c, launch_scps_dist(c->kp, c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems, K, nullptr,
                                    c->d_xs, c->d_X, c->d_Q, c->kmax, stacks[k], c->stream));
        HIP_TRY(c, launch_tube_eval(c->prm.lambda, c->kp.wscale, nullptr, c->d_jref_eval, c->d_sysd, c->d_reps, c->R,
                                    c->kmax, stacks[k], c->d_X, c->d_Q, nullptr, nullptr, nullptr, 0.0, 1,
                                    c->stream));
        HIP_TRY(c, launch_scps_dist(c->kp, c->d_sysd, c->d_reps, c->d_groups, c->d_sitems, c->n_sitems, K,
                                    c->d_jref_eval, c->d_xs, c->d_X, c->d_Q, c->kmax, stacks[k], c->stream));
        HIP_TRY(c, launch_tube_eval(c->prm.lambda, c->kp.wscale, c->d_jref_eval, nullptr, c->d_sysd, c->d_reps, c->R,
                                    c->kmax, stacks[k], c->d_X, c->d_Q, s, w, sigma, 1.0 / n_stacks, k == 0,
                                    c->stream));
    }
    return SCPS_OK;
}

scps_status autotune_impl(scps_ctx *c, const float *x, const float *v, const double *cv, int64_t n_steps,
                          int32_t *chosen) {
    if (!x || !cv) return fail(SCPS_ERR_INVALID_ARG, "x and cvstate must not be NULL");
    if (n_steps < 1) return fail(SCPS_ERR_INVALID_ARG, "n_steps must be >= 1");
    if (c->prm.integrator == SCPS_INTEGRATOR_BAOAB && !v) return fail(SCPS_ERR_INVALID_ARG, "BAOAB needs velocities");
    for (int r = 0; r < c->R; ++r)
        if (!c->sys[c->rep_sys[r]].has_native)
            return fail(SCPS_ERR_STATE, "a system has no native map (scps_set_reference_map)");
    // candidates: {path, workgroup of the persistent kernel, nonbonded pass beside the distance pass (SCPS)}
    struct Cand {
        int path, wg;
        bool overlap;
    };
    std::vector<Cand> cand;
    const bool scps = c->prm.bias_mode == SCPS_BIAS_SCPS;
    if (!scps && c->prm.exec_mode == SCPS_EXEC_AUTO) {
        // chains of at most 64 particles: 64 / n replicas per wavefront, 1 .. 8 wavefronts per workgroup
        if (packed_width_ok(c->n_max))
            for (int w : {1, 2, 4, 8}) cand.push_back({2, w, false});
        // one wavefront per replica can win for chains of a few blocks (several replicas then share a CU)
        if (c->n_pad_max <= 4 * TILE) cand.push_back({0, 64, false});
        for (int wg : {256, 512, 1024})
            if (c->n_pad_max <= persistent_max_npad(wg)) cand.push_back({0, wg, false});
    }
    if (scps && c->prm.exec_mode != SCPS_EXEC_AUTO) {
        cand.push_back({1, 0, c->overlap_nb});     // a fixed schedule: timed, kept
    } else {
        cand.push_back({1, 0, false});
        if (scps && c->side) cand.push_back({1, 0, true});
    }
    const size_t nx = 3 * (size_t)c->sumN;
    float *tx = nullptr, *tv = nullptr;
    double *tcv = nullptr;
    int *tflags = nullptr;   // the caller's non-finite flags, kept across the trial runs
    HIP_TRY(c, dalloc(c, &tflags, c->R));
    HIP_TRY(c, hipMemcpyAsync(tflags, c->d_flags, c->R * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    int *tjref = nullptr;    // SCPS: the reference frames, also kept across the trial runs
    const bool saved_jref_init = c->jref_init;
    if (c->d_jref) {
        HIP_TRY(c, dalloc(c, &tjref, c->R));
        HIP_TRY(c, hipMemcpyAsync(tjref, c->d_jref, c->R * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_TRY(c, dalloc(c, &tx, nx));
    if (v) HIP_TRY(c, dalloc(c, &tv, nx));
    HIP_TRY(c, dalloc(c, &tcv, (size_t)c->R * CV_STRIDE));
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    const int saved_tuned = c->tuned, saved_wg = c->wg, saved_pk = c->pk_waves;
    const bool saved_overlap = c->overlap_nb;
    // every candidate once untimed (first-launch costs), then TUNE_ROUNDS timed
    // runs taken in turns, each from the caller's state; a candidate's time is
    // its fastest run (configurations a few per cent apart stay apart)
    constexpr int TUNE_ROUNDS = 3;
    std::vector<float> fastest(cand.size(), 0.f);
    scps_status st = SCPS_OK;
    for (int round = 0; round <= TUNE_ROUNDS && st == SCPS_OK; ++round)
        for (size_t i = 0; i < cand.size() && st == SCPS_OK; ++i) {
            c->tuned = cand[i].path;
            if (cand[i].path == 0) c->wg = cand[i].wg;
            if (cand[i].path == 2) c->pk_waves = cand[i].wg;
            if (scps) c->overlap_nb = cand[i].overlap;
            float ms = 0.f;
            HIP_TRY(c, hipMemcpyAsync(tx, x, nx * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
            if (v) HIP_TRY(c, hipMemcpyAsync(tv, v, nx * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(tcv, cv, (size_t)c->R * CV_STRIDE * sizeof(double), hipMemcpyDeviceToDevice,
                                      c->stream));
            HIP_TRY(c, hipEventRecord(e0, c->stream));
            st = step_impl(c, tx, tv, tcv, round ? n_steps : 1, 0, 0, nullptr);
            HIP_TRY(c, hipEventRecord(e1, c->stream));
            HIP_TRY(c, hipEventSynchronize(e1));
            HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
            if (round > 0 && (round == 1 || ms < fastest[i])) fastest[i] = ms;
        }
    // the overlapped SCPS schedule has to win clearly: in sustained runs the two
    // passes sharing the CUs slow the distance pass by more than the nonbonded
    // pass costs alone, which runs of a few steps do not show
    constexpr float OVERLAP_MARGIN = 0.97f;
    int best_i = 0;
    for (size_t i = 1; i < cand.size(); ++i) {
        const float bar = cand[i].overlap ? OVERLAP_MARGIN * fastest[best_i] : fastest[best_i];
        if (fastest[i] < bar) best_i = (int)i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // flags raised by the trial runs on the copies do not count
    HIP_TRY(c, hipMemcpyAsync(c->d_flags, tflags, c->R * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    if (tjref) HIP_TRY(c, hipMemcpyAsync(c->d_jref, tjref, c->R * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    c->jref_init = saved_jref_init;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c, tflags);
    dfree(c, tjref);
    dfree(c, tx);
    dfree(c, tv);
    dfree(c, tcv);
    if (st != SCPS_OK) {
        c->tuned = saved_tuned;
        c->wg = saved_wg;
        c->pk_waves = saved_pk;
        c->overlap_nb = saved_overlap;
        return st;
    }
    c->tuned = cand[best_i].path;
    c->wg = c->tuned == 0 ? cand[best_i].wg : saved_wg;
    c->pk_waves = c->tuned == 2 ? cand[best_i].wg : saved_pk;
    c->overlap_nb = scps ? cand[best_i].overlap : saved_overlap;
    if (chosen) launch_report(c, c->tuned, chosen);
    return SCPS_OK;
}

scps_status set_launch_impl(scps_ctx *c, int32_t path, int32_t param) {
    if (c->prm.exec_mode != SCPS_EXEC_AUTO)
        return fail(SCPS_ERR_STATE, "a launch configuration can be set with exec_mode AUTO only");
    const bool scps = c->prm.bias_mode == SCPS_BIAS_SCPS;
    if (path == 1) {
        c->tuned = 1;
        return SCPS_OK;
    }
    if (scps) return fail(SCPS_ERR_INVALID_ARG, "an SCPS context steps on the per-step path (path 1) only");
    if (path == 0) {
        if (param != 64 && param != 256 && param != 512 && param != 1024)
            return fail(SCPS_ERR_INVALID_ARG, "the persistent kernel takes 64, 256, 512 or 1024 threads");
        if (c->n_pad_max > persistent_max_npad(param))
            return fail(SCPS_ERR_SHAPE, "a replica's state does not fit one workgroup's LDS");
        c->tuned = 0;
        c->wg = param;
        return SCPS_OK;
    }
    if (path == 2) {
        if (param < 1 || param > 8) return fail(SCPS_ERR_INVALID_ARG, "the packed kernel takes 1 .. 8 wavefronts");
        if (!packed_width_ok(c->n_max)) return fail(SCPS_ERR_SHAPE, "the packed kernel needs chains of <= 64 particles");
        c->tuned = 2;
        c->pk_waves = param;
        return SCPS_OK;
    }
    return fail(SCPS_ERR_INVALID_ARG, "path must be 0 (persistent), 1 (per-step) or 2 (packed)");
}

}  // namespace

extern "C" {

scps_status scps_init_system(const scps_params *params, const scps_topology *topology, int32_t n_replicas,
                             const int32_t *replica_system, void *hip_stream, scps_ctx **out) {
    try {
        return init_impl(params, topology, n_replicas, replica_system, hip_stream, out);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SCPS_ERR_INVALID_ARG, e.what());
    }
}

scps_status scps_set_reference_map(scps_ctx *ctx, int32_t system, int32_t n_maps, const double *maps,
                                   const double *native_xyz, double z0_norm) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    try {
        return set_ref_impl(ctx, system, n_maps, maps, native_xyz, z0_norm);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_step_replicas(scps_ctx *ctx, float *x, float *v, double *cvstate, int64_t n_steps, uint64_t step0,
                               int32_t record_every, float *frames) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    return step_impl(ctx, x, v, cvstate, n_steps, step0, record_every, frames);
}

scps_status scps_eval_z_and_grad(scps_ctx *ctx, const float *x, double *z, float *grad, const double *grad_coef) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    return eval_impl(ctx, x, z, grad, grad_coef);
}

scps_status scps_eval_zbias(scps_ctx *ctx, const float *x, const double *z_m, double *z, double *E_b, float *grad_z) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!z_m || !E_b) return fail(SCPS_ERR_INVALID_ARG, "z_m and E_b must not be NULL");
    return eval_impl(ctx, x, z, grad_z, nullptr, z_m, E_b);
}

scps_status scps_zbias_backward(scps_ctx *ctx, const double *z, const double *z_m, const double *g_z,
                                int64_t g_z_stride, const double *g_E, int64_t g_E_stride, const float *grad_z,
                                float *grad_x) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!z || !z_m || !grad_z || !grad_x) return fail(SCPS_ERR_INVALID_ARG, "z, z_m, grad_z and grad_x must not be NULL");
    if (g_z_stride < 0 || g_E_stride < 0) return fail(SCPS_ERR_INVALID_ARG, "gradient strides must be >= 0");
    HIP_TRY(ctx, launch_zbias_backward(ctx->d_sysd, ctx->d_reps, ctx->R, ctx->n_pad_max, ctx->prm.k_R, z, z_m, g_z,
                                       g_z_stride, g_E, g_E_stride, grad_z, grad_x, ctx->stream));
    return SCPS_OK;
}

scps_status scps_ratchet_energy(scps_ctx *ctx, const double *z, const double *z_m, double *E_b, const double *gz,
                                const double *gE, double *coef) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!z || !z_m) return fail(SCPS_ERR_INVALID_ARG, "z and z_m must not be NULL");
    HIP_TRY(ctx, launch_ratchet_energy(ctx->R, ctx->prm.k_R, z, z_m, E_b, gz, gE, coef, ctx->stream));
    return SCPS_OK;
}

scps_status scps_update_reference_from_paths(scps_ctx *ctx, int32_t system, const float *frames, int32_t n_paths,
                                             int32_t n_frames, const uint8_t *success, double *maps_out) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    try {
        return update_ref_impl(ctx, system, frames, n_paths, n_frames, success, maps_out);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_autotune(scps_ctx *ctx, const float *x, const float *v, const double *cvstate, int64_t n_steps,
                          int32_t *chosen) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    try {
        return autotune_impl(ctx, x, v, cvstate, n_steps, chosen);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_set_launch(scps_ctx *ctx, int32_t path, int32_t param) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    return set_launch_impl(ctx, path, param);
}

scps_status scps_set_graph_steps(scps_ctx *ctx, int32_t steps) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (steps < 0 || steps > SCPS_MAX_GRAPH_STEPS)
        return fail(SCPS_ERR_INVALID_ARG, "graph steps must be 0 .. " + std::to_string(SCPS_MAX_GRAPH_STEPS));
    if (steps != ctx->graph_steps) {
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));   // the old graph may still be running
        drop_step_graph(ctx);
        ctx->graph_steps = steps;
    }
    return SCPS_OK;
}

scps_status scps_get_launch(scps_ctx *ctx, int32_t *launch) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!launch) return fail(SCPS_ERR_INVALID_ARG, "launch must not be NULL");
    launch_report(ctx, launch_path(ctx), launch);
    return SCPS_OK;
}

scps_status scps_least_biased_path(scps_ctx *ctx, const double *cvstate, const uint8_t *success, int32_t *index,
                                  double *t_min) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    try {
        return least_biased_impl(ctx, cvstate, success, index, t_min);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_scale_by_replica(scps_ctx *ctx, const float *in, const double *coef, float *out) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!in || !coef || !out) return fail(SCPS_ERR_INVALID_ARG, "in, coef and out must not be NULL");
    HIP_TRY(ctx, launch_scale_by_replica(ctx->d_sysd, ctx->d_reps, ctx->R, ctx->n_pad_max, in, coef, out,
                                         ctx->stream));
    return SCPS_OK;
}

scps_status scps_eval_tube(scps_ctx *ctx, int32_t stack_system, const float *x, double *s, double *w) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!s && !w) return fail(SCPS_ERR_INVALID_ARG, "s and w are both NULL");
    try {
        return eval_tube_impl(ctx, 1, &stack_system, x, s, w, nullptr);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_eval_sigma(scps_ctx *ctx, int32_t n_stacks, const int32_t *stack_systems, const float *x,
                            double *sigma) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!sigma) return fail(SCPS_ERR_INVALID_ARG, "sigma is NULL");
    try {
        return eval_tube_impl(ctx, n_stacks, stack_systems, x, nullptr, nullptr, sigma);
    } catch (const std::bad_alloc &) {
        return fail(SCPS_ERR_OOM, "host allocation failed");
    }
}

scps_status scps_set_stream(scps_ctx *ctx, void *hip_stream) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    hipStream_t next = (hipStream_t)hip_stream;
    if (next == ctx->stream) return SCPS_OK;
    // every call shares the context's scratch buffers: work queued from now on
    // waits for what is still queued on the old stream
    if (!ctx->ev_switch) HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ev_switch, hipEventDisableTiming));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_switch, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(next, ctx->ev_switch, 0));
    ctx->stream = next;
    return SCPS_OK;
}

scps_status scps_time_passes(scps_ctx *ctx, int32_t enable) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (ctx->prm.bias_mode != SCPS_BIAS_SCPS) return fail(SCPS_ERR_STATE, "pass timing needs an SCPS context");
    if (enable < 0) return fail(SCPS_ERR_INVALID_ARG, "the timing period must be >= 0");
    if (ctx->pass_ev.empty()) {
        ctx->pass_ev.assign(4 * scps_ctx::PASS_RING, nullptr);
        for (auto &e : ctx->pass_ev) HIP_TRY(ctx, hipEventCreate(&e));
    }
    while (ctx->pass_read < ctx->pass_recorded) {   // what an earlier period recorded
        st = read_pass_slot(ctx);
        if (st != SCPS_OK) return st;
    }
    ctx->timing = enable != 0;
    ctx->timing_period = enable > 0 ? enable : 1;
    ctx->timing_tick = 0;
    ctx->pass_ms[0] = ctx->pass_ms[1] = 0.0;
    ctx->pass_recorded = ctx->pass_read = 0;
    return SCPS_OK;
}

scps_status scps_pass_times(scps_ctx *ctx, double *ms, int64_t *launches) {
    scps_status st;
    if (!usable(ctx, &st)) return st;
    if (!ms || !launches) return fail(SCPS_ERR_INVALID_ARG, "ms and launches must not be NULL");
    while (ctx->pass_read < ctx->pass_recorded) {
        st = read_pass_slot(ctx);
        if (st != SCPS_OK) return st;
    }
    ms[0] = ctx->pass_ms[0];
    ms[1] = ctx->pass_ms[1];
    launches[0] = launches[1] = ctx->pass_read;
    return SCPS_OK;
}

scps_status scps_sync(scps_ctx *ctx, int32_t *bad_replicas, int32_t *n_bad) {
    if (!ctx) return fail(SCPS_ERR_INVALID_ARG, "context is NULL");
    if (n_bad) *n_bad = 0;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(SCPS_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    std::vector<int> flags(ctx->R);
    e = hipMemcpy(flags.data(), ctx->d_flags, ctx->R * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(SCPS_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    int nb = 0, full = 0;
    for (int r = 0; r < ctx->R; ++r)
        if (flags[r]) {
            if (bad_replicas) bad_replicas[nb] = r;
            ++nb;
            full += flags[r] == 2;
        }
    if (n_bad) *n_bad = nb;
    if (nb) {
        ctx->poisoned = true;
        if (full)
            return fail(SCPS_ERR_NONFINITE, std::to_string(full) + " replica(s) had a particle with more than " +
                                                std::to_string(NL_CAP) + " neighbours within the list radius");
        return fail(SCPS_ERR_NONFINITE, std::to_string(nb) + " replica(s) produced non-finite coordinates");
    }
    return SCPS_OK;
}

scps_status scps_path_distance(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                               double y0, double cell, int32_t nx, int32_t ny, void *hip_stream, double *D) {
    if ((!xy_a && n_a > 0) || (!xy_b && n_b > 0) || !D || n_a < 0 || n_b < 0)
        return fail(SCPS_ERR_INVALID_ARG, "NULL point array or output, or a negative count");
    if (!(cell > 0) || nx < 1 || ny < 1 || (int64_t)nx * ny > (1 << 24))
        return fail(SCPS_ERR_INVALID_ARG, "cell must be > 0 and the grid 1 .. 2^24 cells");
    hipStream_t st = (hipStream_t)hip_stream;
    const int m = nx * ny;
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, 2 * (size_t)m * sizeof(int) + 4 * sizeof(long long));
    if (e != hipSuccess) return fail(SCPS_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    long long *d_counts = reinterpret_cast<long long *>(buf);
    int *d_occ = reinterpret_cast<int *>(d_counts + 4);
    long long counts[3] = {0, 0, 0};
    e = launch_path_occupancy(xy_a, n_a, xy_b, n_b, x0, y0, cell, nx, ny, d_occ, d_counts, st);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, d_counts, sizeof(counts), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(SCPS_ERR_HIP, std::string("path distance: ") + hipGetErrorString(e));
    if (counts[0] == 0 || counts[1] == 0)
        return fail(SCPS_ERR_INVALID_ARG, "a point set occupies no cell of the grid");
    // unit-norm binary matrices: |A/|A| - B/|B||^2 = 2 - 2 n_ab / sqrt(n_a n_b)
    const double c = (double)counts[2] / std::sqrt((double)counts[0] * (double)counts[1]);
    *D = std::sqrt(std::max(0.0, 2.0 - 2.0 * c));
    return SCPS_OK;
}

scps_status scps_path_distance_noalloc(const float *xy_a, int64_t n_a, const float *xy_b, int64_t n_b, double x0,
                                       double y0, double cell, int32_t nx, int32_t ny, void *hip_stream,
                                       double *D) {
    if ((!xy_a && n_a > 0) || (!xy_b && n_b > 0) || !D || n_a < 0 || n_b < 0)
        return fail(SCPS_ERR_INVALID_ARG, "NULL point array or output, or a negative count");
    if (!(cell > 0) || nx < 1 || ny < 1)
        return fail(SCPS_ERR_INVALID_ARG, "cell must be > 0 and the grid at least 1 x 1");
    if ((int64_t)nx * ny > PATH_NOALLOC_MAX_CELLS)
        return fail(SCPS_ERR_SHAPE, "a grid of more than " + std::to_string(PATH_NOALLOC_MAX_CELLS) +
                                        " cells needs scps_path_distance (this call allocates nothing)");
    hipStream_t st = (hipStream_t)hip_stream;
    int *d_occ = nullptr;
    long long *d_counts = nullptr;
    hipError_t e = path_scratch(&d_occ, &d_counts);
    long long counts[3] = {0, 0, 0};
    if (e == hipSuccess)
        e = launch_path_occupancy(xy_a, n_a, xy_b, n_b, x0, y0, cell, nx, ny, d_occ, d_counts, st);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, d_counts, sizeof(counts), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(SCPS_ERR_HIP, std::string("path distance: ") + hipGetErrorString(e));
    if (counts[0] == 0 || counts[1] == 0)
        return fail(SCPS_ERR_INVALID_ARG, "a point set occupies no cell of the grid");
    const double c = (double)counts[2] / std::sqrt((double)counts[0] * (double)counts[1]);
    *D = std::sqrt(std::max(0.0, 2.0 - 2.0 * c));
    return SCPS_OK;
}

scps_status scps_funnel_steps(const scps_funnel_params *p, int32_t n_traj, int32_t first_id, double *xy,
                              double *cvstate, int64_t n_steps, uint64_t step0, int32_t record_every, double *frames,
                              int32_t n_path_frames, const double *mean_path, void *hip_stream) {
    if (!p || !xy || !cvstate) return fail(SCPS_ERR_INVALID_ARG, "params, xy and cvstate must not be NULL");
    if (n_traj < 1 || first_id < 0 || n_steps < 0 || record_every < 0)
        return fail(SCPS_ERR_INVALID_ARG, "n_traj >= 1, first_id, n_steps and record_every >= 0 are required");
    if (record_every > 0 && !frames) return fail(SCPS_ERR_INVALID_ARG, "frames is NULL but record_every > 0");
    if (!(p->mobility_dt > 0) || !(p->kT >= 0)) return fail(SCPS_ERR_INVALID_ARG, "mobility_dt > 0, kT >= 0");
    if (p->bias_mode != SCPS_BIAS_RMD && p->bias_mode != SCPS_BIAS_SCPS)
        return fail(SCPS_ERR_INVALID_ARG, "bias_mode must be 0 (rMD) or 1 (tube ratchets)");
    if (p->w_form != SCPS_W_INV_LAMBDA && p->w_form != SCPS_W_NO_INV_LAMBDA)
        return fail(SCPS_ERR_INVALID_ARG, "w_form must be 0 (w with 1/lambda) or 1 (without)");
    if (p->bias_mode == SCPS_BIAS_SCPS) {
        if (!mean_path) return fail(SCPS_ERR_INVALID_ARG, "the tube ratchets need a mean path");
        if (n_path_frames < 2 || n_path_frames > FUNNEL_KMAX)
            return fail(SCPS_ERR_SHAPE, "a mean path has 2 .. " + std::to_string(FUNNEL_KMAX) + " frames");
        if (!(p->lambda > 0)) return fail(SCPS_ERR_INVALID_ARG, "lambda must be > 0");
    }
    FunnelK k{};
    k.A1 = p->A1; k.A2 = p->A2; k.A3 = p->A3;
    k.s1 = p->s1; k.s2 = p->s2; k.s3 = p->s3;
    k.w = p->w; k.xm = p->xm; k.ym = p->ym;
    k.kT = p->kT; k.mob_dt = p->mobility_dt;
    k.k_R = p->k_R; k.lambda = p->lambda; k.k_s = p->k_s; k.k_w = p->k_w;
    k.wscale = p->w_form == SCPS_W_NO_INV_LAMBDA ? 1.0 : (p->lambda > 0 ? 1.0 / p->lambda : 0.0);
    k.seed_lo = (uint32_t)p->seed; k.seed_hi = (uint32_t)(p->seed >> 32);
    k.bias_mode = p->bias_mode;
    hipError_t e = launch_funnel_steps(k, n_traj, first_id, reinterpret_cast<double2 *>(xy), cvstate, n_steps, step0,
                                       record_every, reinterpret_cast<double2 *>(frames),
                                       p->bias_mode == SCPS_BIAS_SCPS ? n_path_frames : 0,
                                       reinterpret_cast<const double2 *>(mean_path), (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(SCPS_ERR_HIP, std::string("funnel steps: ") + hipGetErrorString(e));
    return SCPS_OK;
}

scps_status scps_funnel_mean_path(int32_t n_traj, int32_t n_frames, const double *frames, const uint8_t *success,
                                  double *mean_path, void *hip_stream) {
    if (!frames || !success || !mean_path) return fail(SCPS_ERR_INVALID_ARG, "NULL argument");
    if (n_traj < 1 || n_frames < 1) return fail(SCPS_ERR_INVALID_ARG, "n_traj and n_frames must be >= 1");
    std::vector<int> list;
    for (int t = 0; t < n_traj; ++t)
        if (success[t]) list.push_back(t);
    if (list.empty()) return fail(SCPS_ERR_NO_SUCCESS, "no successful trajectory");
    hipStream_t st = (hipStream_t)hip_stream;
    void *d_list = nullptr;
    hipError_t e = hipMalloc(&d_list, list.size() * sizeof(int));
    if (e != hipSuccess) return fail(SCPS_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = hipMemcpyAsync(d_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_funnel_mean(n_traj, n_frames, reinterpret_cast<const double2 *>(frames), (const int *)d_list,
                               (int)list.size(), reinterpret_cast<double2 *>(mean_path), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_list);
    if (e != hipSuccess) return fail(SCPS_ERR_HIP, std::string("funnel mean path: ") + hipGetErrorString(e));
    return SCPS_OK;
}

void scps_destroy(scps_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_switch) (void)hipEventDestroy(ctx->ev_switch);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (hipEvent_t e : ctx->pass_ev)
        if (e) (void)hipEventDestroy(e);
    for (void *p : ctx->owned) (void)hipFree(p);
    delete ctx;
}

const char *scps_last_error(void) { return g_err.c_str(); }

}  // extern "C"
