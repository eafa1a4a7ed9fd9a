/*
 * Plain FP64 CPU oracle of the batched rMD / SCPS hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the HIP library and must never sit on the product path.
 *
 * Everything is double precision, straightforward loops over unordered
 * pairs i<j, no blocking, no fusion, no fast-math.  OpenMP is used only to
 * run independent replicas side by side.
 *
 * What is computed (Orioli, a Beccara, Faccioli, "Self Consistent Path
 * Sampling", arXiv:1705.02180):
 *   - contact map entries, eq (Cij), and the collective coordinate z,
 *     eq (zrMD), with its analytic gradient;
 *   - the ratchet-and-pawl force, eq (FrMD), with the running minimum z_m
 *     of the section on rMD (z_m(0) = z(X(0)), theta(0) = 1);
 *   - a synthetic chain force field standing in for the all-atom one:
 *     harmonic bonds, Lennard-Jones 12-6 and Debye-Hueckel pair terms;
 *   - Langevin dynamics, eq (Lang): overdamped Euler-Maruyama or BAOAB,
 *     driven by Philox4x32-10 noise (Salmon, Moraes, Dror, Shaw, SC'11);
 *   - the path-ensemble mean contact map, eq (avCij);
 *   - the mean-field tube variables s_lambda, w_lambda, eqs (asXa),(awXa)
 *     discretised as in the appendix, and their ratchet forces (Fw),(Fs);
 *   - the bias functional T[X] of the bias-functional variational principle
 *     (rMD section, eq (T) and the protocol's variational correction),
 *     accumulated over the path as T += dt sum_i |F_bias,i|^2 / (m_i gamma).
 *
 * Readings where the paper is silent (all documented in the design notes):
 *   - the sum in eq (zrMD) runs over unordered pairs i<j of the contact
 *     set with |i-j| > min_seq_sep (the paper's all-atom value is 35);
 *   - eq (Cij) is evaluated in the algebraically identical form
 *     (1+q+q^2)/(1+q+q^2+q^3+q^4), q = (r/r0)^2, which has no 0/0 at r0;
 *   - w_lambda keeps the 1/lambda of eq (wX) by default; w_form = 1 drops
 *     it, as eq (awXa), the protocol and the toy-model formulas print w
 *     (then w and its gradient are lambda times larger).  The constant w0
 *     is dropped because only differences w - w_m and gradients enter the
 *     forces;
 *   - the norm of the tube distance divides by Z0 = the sum of (C0_ij)^2 over
 *     the same pairs as its numerator (|i-j| > min_seq_sep), as the
 *     normalised Frobenius-type distance of the SCPS section is defined;
 *   - the SCPS ratchets use (s - s_m) and (w - w_m) as in eqs (Fw),(Fs);
 *   - BAOAB is used for the underdamped equation and its state velocity
 *     is the one right after the friction/noise substep;
 *   - the cutoff the paper introduces for linear scaling (C = 0 beyond r_c,
 *     remark after eq (Cij)) is offered for the synthetic nonbonded terms as
 *     well: with r_cut_nb > 0 a Lennard-Jones / Debye-Hueckel pair farther
 *     apart than r_cut_nb contributes no force and no energy (plain
 *     truncation, like the contact cutoff);
 *   - T[X] takes the prefactor 1/(m_i gamma_i) of the rMD section and of the
 *     protocol (eq (T) writes Gamma_i = 1/(4 gamma_i m_i k_B T), which only
 *     rescales every path's T by the same constant), and the time integral
 *     as a left Riemann sum over the force evaluations of the steps taken.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CV_STRIDE 8
enum { CV_Z = 0, CV_ZM = 1, CV_EB = 2, CV_S = 3, CV_W = 4, CV_SM = 5, CV_WM = 6, CV_T = 7 };

typedef struct {
    int32_t integrator;      /* 0 overdamped Euler-Maruyama, 1 BAOAB */
    int32_t bias_mode;       /* 0 rMD on z, 1 SCPS tube variables */
    double dt, gamma, kT;
    double k_bond, r_bond;
    double lj_eps, lj_sigma;
    double dh_prefactor, dh_kappa;
    int32_t nb_excl;         /* nonbonded pairs need |i-j| > nb_excl */
    int32_t min_seq_sep;     /* contact pairs need |i-j| > min_seq_sep */
    int32_t w_form;          /* 0: w = -(1/lambda) log sum_k e^{-lambda d_k}; 1: without the 1/lambda */
    int32_t pad_w;
    double r0;               /* contact reference distance */
    double r_cut;            /* <= 0: no cutoff */
    double r_cut_nb;         /* <= 0: no cutoff; else nonbonded pairs with r > r_cut_nb contribute nothing */
    double k_R;
    double lambda, k_s, k_w;
    uint64_t seed;
} orc_params;

/* ------------------------------------------------------------------------
 * Contact function, eq (Cij):  C = (1 - (r/r0)^6) / (1 - (r/r0)^10).
 * With q = (r/r0)^2 numerator and denominator share the factor (1-q).
 * ---------------------------------------------------------------------- */
double orc_contact(double r2, double r0, double r_cut, double *dC_dr2)
{
    if (r_cut > 0.0 && r2 > r_cut * r_cut) {
        if (dC_dr2) *dC_dr2 = 0.0;
        return 0.0;
    }
    double q = r2 / (r0 * r0);
    double num = 1.0 + q + q * q;
    double den = 1.0 + q + q * q + q * q * q + q * q * q * q;
    double C = num / den;
    if (dC_dr2) {
        double dnum = 1.0 + 2.0 * q;
        double dden = 1.0 + 2.0 * q + 3.0 * q * q + 4.0 * q * q * q;
        double dC_dq = (dnum * den - num * dden) / (den * den);
        *dC_dr2 = dC_dq / (r0 * r0);
    }
    return C;
}

static double dist2(const double *x, int n, int i, int j, double d[3])
{
    d[0] = x[i] - x[j];
    d[1] = x[n + i] - x[n + j];
    d[2] = x[2 * n + i] - x[2 * n + j];
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

static int64_t npairs(int nc) { return (int64_t)nc * (nc - 1) / 2; }

/* packed index of the unordered contact-set pair a<b */
static int64_t pidx(int nc, int a, int b)
{
    return (int64_t)a * nc - (int64_t)a * (a + 1) / 2 + (b - a - 1);
}

/* Contact map of a configuration over the contact set, packed a<b. */
void orc_contact_map(int n, const double *x, int nc, const int32_t *cidx,
                     double r0, double r_cut, double *out)
{
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            double d[3];
            double r2 = dist2(x, n, cidx[a], cidx[b], d);
            out[pidx(nc, a, b)] = orc_contact(r2, r0, r_cut, NULL);
        }
}

/* z = sum over contact pairs of (C_ij(X) - R_ij)^2, eq (zrMD), and its
 * gradient dz/dx_i = sum_j 2 (C_ij - R_ij) dC_ij/dx_i (grad may be NULL). */
double orc_z_grad(int n, const double *x, int nc, const int32_t *cidx,
                  const double *ref, double r0, double r_cut, int min_sep,
                  double *grad)
{
    double z = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * 3 * n);
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            int i = cidx[a], j = cidx[b];
            if (abs(i - j) <= min_sep) continue;
            double d[3], dC;
            double r2 = dist2(x, n, i, j, d);
            double C = orc_contact(r2, r0, r_cut, &dC);
            double diff = C - ref[pidx(nc, a, b)];
            z += diff * diff;
            if (grad) {
                /* dC/dx_i = dC/dr2 * 2 (x_i - x_j) */
                double g = 2.0 * diff * dC * 2.0;
                for (int c = 0; c < 3; ++c) {
                    grad[c * n + i] += g * d[c];
                    grad[c * n + j] -= g * d[c];
                }
            }
        }
    return z;
}

/* Denominator of the normalised distance between contact maps (SCPS
 * section): the sum of (C0_ij)^2 over the contact pairs with |i-j| >
 * min_sep, the same pairs its numerator and z sum over. */
double orc_norm_z0(int nc, const int32_t *cidx, const double *native, int min_sep)
{
    double z0 = 0.0;
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            if (abs(cidx[a] - cidx[b]) <= min_sep) continue;
            double c0 = native[pidx(nc, a, b)];
            z0 += c0 * c0;
        }
    return z0;
}

/* ------------------------------------------------------------------------
 * Synthetic chain force field (stand-in for the all-atom force field):
 * harmonic bonds i,i+1; Lennard-Jones 12-6 and Debye-Hueckel over pairs
 * with |i-j| > nb_excl.  F = -grad U.  Returns U.
 * ---------------------------------------------------------------------- */
double orc_phys_forces(int n, const double *x, const float *charge,
                       const orc_params *p, double *F)
{
    double U = 0.0;
    memset(F, 0, sizeof(double) * 3 * n);
    for (int i = 0; i + 1 < n; ++i) {
        double d[3];
        double r = sqrt(dist2(x, n, i, i + 1, d));
        double dr = r - p->r_bond;
        U += 0.5 * p->k_bond * dr * dr;
        /* dU/dx_i = k (r - r_b) (x_i - x_{i+1}) / r */
        double f = -p->k_bond * dr / r;
        for (int c = 0; c < 3; ++c) {
            F[c * n + i] += f * d[c];
            F[c * n + i + 1] -= f * d[c];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (j - i <= p->nb_excl) continue;
            double d[3];
            double r2 = dist2(x, n, i, j, d);
            if (p->r_cut_nb > 0.0 && r2 > p->r_cut_nb * p->r_cut_nb) continue;   /* truncated, as the contact cutoff */
            double r = sqrt(r2);
            double f_over_r = 0.0;          /* -dU/dr / r */
            if (p->lj_eps != 0.0) {
                double sr6 = pow(p->lj_sigma / r, 6.0);
                U += 4.0 * p->lj_eps * (sr6 * sr6 - sr6);
                f_over_r += 24.0 * p->lj_eps * (2.0 * sr6 * sr6 - sr6) / r2;
            }
            if (p->dh_prefactor != 0.0) {
                double qq = (double)charge[i] * (double)charge[j];
                double u = p->dh_prefactor * qq * exp(-p->dh_kappa * r) / r;
                U += u;
                /* dU/dr = -u (kappa + 1/r) */
                f_over_r += u * (p->dh_kappa + 1.0 / r) / r;
            }
            for (int c = 0; c < 3; ++c) {
                F[c * n + i] += f_over_r * d[c];
                F[c * n + j] -= f_over_r * d[c];
            }
        }
    return U;
}

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
 * multiplications with the Weyl-sequence key schedule.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k[0] += W0; k[1] += W1;
    }
    memcpy(out, c, sizeof(c));
}

/* 32-bit word -> odd multiple of 2^-24 in (0,1); exact in float and double */
double orc_uniform(uint32_t w)
{
    return (2.0 * (double)(w >> 9) + 1.0) * (1.0 / 16777216.0);
}

/* Three standard normals for (atom, replica, step): counter = (atom,
 * replica, step_lo, step_hi), key = seed.  Box-Muller on (u0,u1) gives the
 * first two, on (u2,u3) the third; the fourth is not used. */
void orc_normals(uint64_t seed, uint32_t atom, uint32_t replica, uint64_t step, double out[3])
{
    uint32_t ctr[4] = {atom, replica, (uint32_t)step, (uint32_t)(step >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = orc_uniform(w[0]), u1 = orc_uniform(w[1]);
    double u2 = orc_uniform(w[2]), u3 = orc_uniform(w[3]);
    double r01 = sqrt(-2.0 * log(u0));
    double r23 = sqrt(-2.0 * log(u2));
    out[0] = r01 * cos(two_pi * u1);
    out[1] = r01 * sin(two_pi * u1);
    out[2] = r23 * cos(two_pi * u3);
}

/* ------------------------------------------------------------------------
 * Mean-field tube variables (eqs (asXa),(awXa), discretised over reference
 * frames k = 0..M as in the appendix) and their gradients.
 *   d_k = ||C(X) - R_k||^2 = sum_p (C_p - R_{k,p})^2 / Z0
 *   s   = 1 - (1/M) sum_k k e^{-lambda d_k} / sum_k e^{-lambda d_k}
 *   w   = -(1/lambda) log sum_k e^{-lambda d_k}      (w_form 0, eqs (wX), (wXapp))
 *   w   = -log sum_k e^{-lambda d_k}                (w_form 1, eq (awXa))
 * grad_s / grad_w may be NULL; dk (length K) may be NULL.
 * ---------------------------------------------------------------------- */
void orc_tube(int n, const double *x, int nc, const int32_t *cidx, int K,
              const double *stack, double Z0, double lambda, double r0,
              double r_cut, int min_sep, int w_form, double *s_out, double *w_out,
              double *grad_s, double *grad_w, double *dk)
{
    int64_t P = npairs(nc);
    double *d = (double *)calloc((size_t)K, sizeof(double));
    double *C = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    double *dCdr2 = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            double dd[3];
            double r2 = dist2(x, n, cidx[a], cidx[b], dd);
            int64_t p = pidx(nc, a, b);
            C[p] = orc_contact(r2, r0, r_cut, &dCdr2[p]);
        }
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int a = 0; a < nc; ++a)
            for (int b = a + 1; b < nc; ++b) {
                if (abs(cidx[a] - cidx[b]) <= min_sep) continue;
                int64_t p = pidx(nc, a, b);
                double diff = C[p] - stack[(int64_t)k * P + p];
                acc += diff * diff;
            }
        d[k] = acc / Z0;
    }
    /* log-sum-exp with the largest exponent factored out */
    double amax = -INFINITY;
    for (int k = 0; k < K; ++k) amax = fmax(amax, -lambda * d[k]);
    double S = 0.0, Sk = 0.0;
    for (int k = 0; k < K; ++k) {
        double e = exp(-lambda * d[k] - amax);
        S += e;
        Sk += (double)k * e;
    }
    int M = K - 1;
    double kbar = Sk / S;
    *s_out = 1.0 - kbar / (double)M;
    /* w_form 0: w = -(1/lambda) log sum; w_form 1: w = -log sum */
    double wscale = w_form ? 1.0 : 1.0 / lambda;
    *w_out = -(amax + log(S)) * wscale;
    if (dk) memcpy(dk, d, sizeof(double) * K);

    if (grad_s || grad_w) {
        /* ds/dd_k = (lambda/M) p_k (k - kbar);  dw/dd_k = lambda wscale p_k;
         * dd_k/dx = (2/Z0) sum_p (C_p - R_{k,p}) dC_p/dx                     */
        if (grad_s) memset(grad_s, 0, sizeof(double) * 3 * n);
        if (grad_w) memset(grad_w, 0, sizeof(double) * 3 * n);
        for (int k = 0; k < K; ++k) {
            double pk = exp(-lambda * d[k] - amax) / S;
            double cs = (lambda / (double)M) * pk * ((double)k - kbar);
            double cw = lambda * wscale * pk;
            for (int a = 0; a < nc; ++a)
                for (int b = a + 1; b < nc; ++b) {
                    int i = cidx[a], j = cidx[b];
                    if (abs(i - j) <= min_sep) continue;
                    int64_t p = pidx(nc, a, b);
                    double dd[3];
                    dist2(x, n, i, j, dd);
                    double g = (2.0 / Z0) * (C[p] - stack[(int64_t)k * P + p]) * dCdr2[p] * 2.0;
                    for (int c = 0; c < 3; ++c) {
                        if (grad_s) {
                            grad_s[c * n + i] += cs * g * dd[c];
                            grad_s[c * n + j] -= cs * g * dd[c];
                        }
                        if (grad_w) {
                            grad_w[c * n + i] += cw * g * dd[c];
                            grad_w[c * n + j] -= cw * g * dd[c];
                        }
                    }
                }
        }
    }
    free(d);
    free(C);
    free(dCdr2);
}

/* ------------------------------------------------------------------------
 * Total force at X with the history-dependent bias.  Updates the running
 * minima in cv (z_m, or s_m and w_m) before using them, and stores the
 * collective variables and the bias energy.
 *   rMD  (eq (FrMD)):  F_bias = -k_R (z - z_m) theta(z - z_m) grad z
 *   SCPS (eqs (Fw),(Fs)): F_bias = -k_s (s - s_m) grad s - k_w (w - w_m) grad w
 * Optionally returns the bias part alone in Fbias (may be NULL).
 * ---------------------------------------------------------------------- */
typedef struct {
    int n, nc;
    const int32_t *cidx;
    const float *mass, *charge;
    const double *native;        /* packed native map [P] */
    int K;                       /* SCPS reference frames */
    const double *stack;         /* [K][P] */
    double Z0;
} orc_system;

void orc_total_force(const orc_params *p, const orc_system *s, const double *x,
                     double *cv, double *F, double *Fbias)
{
    int n = s->n;
    double *Fb = (double *)calloc((size_t)3 * n, sizeof(double));
    orc_phys_forces(n, x, s->charge, p, F);
    if (p->bias_mode == 0) {
        double *gz = (double *)malloc(sizeof(double) * 3 * n);
        double z = orc_z_grad(n, x, s->nc, s->cidx, s->native, p->r0, p->r_cut,
                              p->min_seq_sep, gz);
        double zm = fmin(cv[CV_ZM], z);       /* z_m(0) = z(X(0)) when cv starts at +inf */
        double dz = z - zm;
        double theta = (dz >= 0.0) ? 1.0 : 0.0;
        for (int i = 0; i < 3 * n; ++i) Fb[i] = -p->k_R * gz[i] * dz * theta;
        cv[CV_Z] = z;
        cv[CV_ZM] = zm;
        cv[CV_EB] = 0.5 * p->k_R * dz * dz * theta;
        free(gz);
    } else {
        double *gs = (double *)malloc(sizeof(double) * 3 * n);
        double *gw = (double *)malloc(sizeof(double) * 3 * n);
        double sv, wv;
        orc_tube(n, x, s->nc, s->cidx, s->K, s->stack, s->Z0, p->lambda, p->r0,
                 p->r_cut, p->min_seq_sep, p->w_form, &sv, &wv, gs, gw, NULL);
        double sm = fmin(cv[CV_SM], sv);
        double wm = fmin(cv[CV_WM], wv);
        double ds = sv - sm, dw = wv - wm;
        double ts = (ds >= 0.0) ? 1.0 : 0.0, tw = (dw >= 0.0) ? 1.0 : 0.0;
        for (int i = 0; i < 3 * n; ++i)
            Fb[i] = -p->k_s * gs[i] * ds * ts - p->k_w * gw[i] * dw * tw;
        cv[CV_S] = sv;
        cv[CV_W] = wv;
        cv[CV_SM] = sm;
        cv[CV_WM] = wm;
        cv[CV_EB] = 0.5 * p->k_s * ds * ds * ts + 0.5 * p->k_w * dw * dw * tw;
        free(gs);
        free(gw);
    }
    for (int i = 0; i < 3 * n; ++i) F[i] += Fb[i];
    if (Fbias) memcpy(Fbias, Fb, sizeof(double) * 3 * n);
    free(Fb);
}

/* ------------------------------------------------------------------------
 * Langevin steps for one replica, eq (Lang), with global step counter
 * step0 + m.  Each step starts with a force evaluation at the current X.
 *   overdamped:  x += dt F/(m gamma) + sqrt(2 kT dt/(m gamma)) xi
 *   BAOAB (v = velocity after the friction/noise substep):
 *     v += dt F/m   (the closing half kick of the previous step and the
 *                    opening half kick of this one)
 *     x += dt/2 v;  v = c1 v + sqrt((1-c1^2) kT/m) xi, c1 = exp(-gamma dt);
 *     x += dt/2 v
 * Every force evaluation also adds dt sum_i |F_bias,i|^2 / (m_i gamma) to
 * the bias functional cv[CV_T].
 * Frames (may be NULL) receive X at local step indices 0, E, 2E, ... <=
 * n_steps, each as [3][n], stride frame_stride doubles.
 * ---------------------------------------------------------------------- */
void orc_steps(const orc_params *p, const orc_system *s, uint32_t replica_id,
               double *x, double *v, double *cv, int64_t n_steps, uint64_t step0,
               int record_every, double *frames, int64_t frame_stride)
{
    int n = s->n;
    double *F = (double *)malloc(sizeof(double) * 3 * n);
    double *Fb = (double *)malloc(sizeof(double) * 3 * n);
    double c1 = exp(-p->gamma * p->dt);
    for (int64_t m = 0; m <= n_steps; ++m) {
        if (frames && record_every > 0 && m % record_every == 0)
            memcpy(frames + (m / record_every) * frame_stride, x, sizeof(double) * 3 * n);
        if (m == n_steps) break;
        uint64_t step = step0 + (uint64_t)m;
        orc_total_force(p, s, x, cv, F, Fb);
        /* bias functional: T += dt sum_i |F_bias,i|^2 / (m_i gamma) */
        double t = 0.0;
        for (int i = 0; i < n; ++i) {
            double f2 = 0.0;
            for (int c = 0; c < 3; ++c) f2 += Fb[c * n + i] * Fb[c * n + i];
            t += f2 / ((double)s->mass[i] * p->gamma);
        }
        cv[CV_T] += p->dt * t;
        for (int i = 0; i < n; ++i) {
            double xi[3];
            orc_normals(p->seed, (uint32_t)i, replica_id, step, xi);
            double mi = (double)s->mass[i];
            for (int c = 0; c < 3; ++c) {
                int k = c * n + i;
                if (p->integrator == 0) {
                    double mob = p->dt / (mi * p->gamma);
                    x[k] += mob * F[k] + sqrt(2.0 * p->kT * mob) * xi[c];
                } else {
                    v[k] += p->dt * F[k] / mi;
                    x[k] += 0.5 * p->dt * v[k];
                    v[k] = c1 * v[k] + sqrt((1.0 - c1 * c1) * p->kT / mi) * xi[c];
                    x[k] += 0.5 * p->dt * v[k];
                }
            }
        }
    }
    free(F);
    free(Fb);
}

/* Batched driver: replicas r = 0..R-1 of systems replica_system[r], state
 * in flat buffers, replica r at particle offset off[r] as [3][N_r].
 * Replicas run in parallel with OpenMP; returns the thread count used. */
int orc_run_batch(const orc_params *p, const orc_system *systems, int R,
                  const int32_t *replica_system, const int64_t *off, double *x,
                  double *v, double *cv, int64_t n_steps, uint64_t step0, int n_threads)
{
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int r = 0; r < R; ++r) {
        const orc_system *s = &systems[replica_system[r]];
        orc_steps(p, s, (uint32_t)r, x + 3 * off[r], v ? v + 3 * off[r] : NULL,
                  cv + (int64_t)r * ORC_CV_STRIDE, n_steps, step0, 0, NULL, 0);
    }
    return used;
}

/* Path-ensemble mean contact map, eq (avCij), over paths with success[p]
 * != 0.  frames: [n_frames][n_paths][3][n].  out: [n_frames][P].  Returns
 * the number of successful paths (out untouched when zero). */
int orc_update_reference(int n, int nc, const int32_t *cidx, double r0, double r_cut,
                         int n_frames, int n_paths, const double *frames,
                         const uint8_t *success, double *out)
{
    int64_t P = npairs(nc);
    int nsucc = 0;
    for (int q = 0; q < n_paths; ++q) nsucc += success[q] ? 1 : 0;
    if (nsucc == 0) return 0;
    double *map = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
    for (int k = 0; k < n_frames; ++k) {
        double *o = out + (int64_t)k * P;
        for (int64_t e = 0; e < P; ++e) o[e] = 0.0;
        for (int q = 0; q < n_paths; ++q) {
            if (!success[q]) continue;
            const double *X = frames + ((int64_t)k * n_paths + q) * 3 * n;
            orc_contact_map(n, X, nc, cidx, r0, r_cut, map);
            for (int64_t e = 0; e < P; ++e) o[e] += map[e];
        }
        for (int64_t e = 0; e < P; ++e) o[e] /= (double)nsucc;
    }
    free(map);
    return nsucc;
}

/* Least-biased path (the protocol's final selection): the path with the
 * smallest bias functional T[X], eq (T), among those with success[r] != 0
 * (success NULL = all).  T of path r is cv[r * ORC_CV_STRIDE + CV_T].  Equal
 * values go to the lowest r.  Returns r, -1 when there is no candidate, -2
 * when a candidate's T is not finite. */
int orc_least_biased(int R, const double *cv, const uint8_t *success)
{
    int best = -1;
    for (int r = 0; r < R; ++r) {
        if (success && !success[r]) continue;
        double t = cv[(int64_t)r * ORC_CV_STRIDE + CV_T];
        if (!isfinite(t)) return -2;
        if (best < 0 || t < cv[(int64_t)best * ORC_CV_STRIDE + CV_T]) best = r;
    }
    return best;
}

/* ------------------------------------------------------------------------
 * Toy model: diffusion of one particle on the two-dimensional asymmetric
 * funnel of eq (U) with the parameters of Table 1 (section "Diffusion in a
 * 2-dimensional asymmetric funnel").  Overdamped Langevin steps
 *   X += D F + sqrt(2 kT D) xi,   D = dt / (m gamma)  (the paper's gamma dt),
 * with the noise of orc_normals (atom 0, replica = trajectory id; the first
 * two normals drive x and y).  Bias: rMD on z = |X| (eq (FrMD) with the
 * running minimum), or the ratchets on the tube variables of eqs (Fw),(Fs)
 * with the Euclidean distance to the frames of the mean path,
 *   d_k = |X - <X(t_k)>|^2,  s = 1 - (1/M) sum_k k p_k,  w = -(1/lambda) log sum_k e^{-lambda d_k}.
 * T accumulates D |F_bias|^2 per step (the 1/(m gamma) weight of T[X]).
 * ---------------------------------------------------------------------- */
typedef struct {
    double A1, A2, A3, s1, s2, s3, w, xm, ym;
    double kT, mob_dt;
    int32_t bias_mode, w_form;   /* w_form as for the chains */
    double k_R, lambda, k_s, k_w;
    uint64_t seed;
} orc_funnel_params;

/* U(x, y) of eq (U); F = -grad U. */
double orc_funnel_force(const orc_funnel_params *p, double x, double y, double F[2])
{
    double r2 = x * x + y * y;
    double a1 = r2 + p->s1 * p->s1, a2 = r2 + p->s2 * p->s2;
    double dx = x - p->xm, dy = y - p->ym;
    double a3 = dx * dx + dy * dy + p->s3 * p->s3;
    double U = p->w * p->w * r2 * r2
             - p->A1 * p->s1 * p->s1 / (a1 * a1)
             + p->A2 * p->s2 * p->s2 / (a2 * a2)
             - p->A3 * p->s3 * p->s3 / (a3 * a3);
    /* dU/dx for each term: 4 w^2 r^2 x, +4 A1 s1^2 x / a1^3, -4 A2 s2^2 x / a2^3, +4 A3 s3^2 (x - xm) / a3^3 */
    double g_r = 4.0 * p->w * p->w * r2
               + 4.0 * p->A1 * p->s1 * p->s1 / (a1 * a1 * a1)
               - 4.0 * p->A2 * p->s2 * p->s2 / (a2 * a2 * a2);
    double g_3 = 4.0 * p->A3 * p->s3 * p->s3 / (a3 * a3 * a3);
    F[0] = -(g_r * x + g_3 * dx);
    F[1] = -(g_r * y + g_3 * dy);
    return U;
}

/* Euclidean tube variables of (x, y) on the mean path mp [K][2]; gradients
 * optional.  w_form 0 keeps the 1/lambda of eq (wX) in w; w_form 1 drops it,
 * as the toy-model section prints w. */
void orc_funnel_tube(double x, double y, int K, const double *mp, double lambda, int w_form,
                     double *s, double *w, double gs[2], double gw[2])
{
    int M = K - 1;
    double *d = (double *)malloc(sizeof(double) * (size_t)K);
    double amax = -INFINITY;
    for (int k = 0; k < K; ++k) {
        double ex = x - mp[2 * k], ey = y - mp[2 * k + 1];
        d[k] = ex * ex + ey * ey;
        if (-lambda * d[k] > amax) amax = -lambda * d[k];
    }
    double z = 0.0, kz = 0.0;
    for (int k = 0; k < K; ++k) {
        double e = exp(-lambda * d[k] - amax);
        z += e;
        kz += k * e;
    }
    double kbar = kz / z;
    double wscale = w_form ? 1.0 : 1.0 / lambda;
    *s = 1.0 - kbar / M;
    *w = -(amax + log(z)) * wscale;
    if (gs || gw) {
        double as[2] = {0.0, 0.0}, aw[2] = {0.0, 0.0};
        for (int k = 0; k < K; ++k) {
            double pk = exp(-lambda * d[k] - amax) / z;
            double gd[2] = {2.0 * (x - mp[2 * k]), 2.0 * (y - mp[2 * k + 1])};
            for (int c = 0; c < 2; ++c) {
                as[c] += pk * (k - kbar) * gd[c];
                aw[c] += pk * gd[c];
            }
        }
        for (int c = 0; c < 2; ++c) {
            if (gs) gs[c] = (lambda / M) * as[c];
            if (gw) gw[c] = lambda * wscale * aw[c];
        }
    }
    free(d);
}

/* One trajectory, n_steps steps from global step step0.  xy[2], cv[8] in/out
 * (z, z_m, E_b, s, w, s_m, w_m, T as in the chain model).  frames: NULL or
 * [n_steps / record_every + 1][2] (frame 0 = the start). */
void orc_funnel_steps(const orc_funnel_params *p, uint32_t traj, double *xy, double *cv, int64_t n_steps,
                      uint64_t step0, int record_every, double *frames, int K, const double *mp)
{
    double x = xy[0], y = xy[1];
    double D = p->mob_dt, amp = sqrt(2.0 * p->kT * p->mob_dt);
    for (int64_t n = 0;; ++n) {
        if (frames && record_every > 0 && n % record_every == 0) {
            frames[2 * (n / record_every)] = x;
            frames[2 * (n / record_every) + 1] = y;
        }
        if (n == n_steps) break;
        double F[2], Fb[2] = {0.0, 0.0};
        orc_funnel_force(p, x, y, F);
        if (p->bias_mode == 0) {
            double z = sqrt(x * x + y * y);
            double zm = fmin(cv[CV_ZM], z);
            double dz = z - zm;
            if (z > 0.0) {
                Fb[0] = -p->k_R * dz * x / z;
                Fb[1] = -p->k_R * dz * y / z;
            }
            cv[CV_Z] = z;
            cv[CV_ZM] = zm;
            cv[CV_EB] = 0.5 * p->k_R * dz * dz;
        } else {
            double sv, wv, gs[2], gw[2];
            orc_funnel_tube(x, y, K, mp, p->lambda, p->w_form, &sv, &wv, gs, gw);
            double sm = fmin(cv[CV_SM], sv), wm = fmin(cv[CV_WM], wv);
            for (int c = 0; c < 2; ++c) Fb[c] = -p->k_s * (sv - sm) * gs[c] - p->k_w * (wv - wm) * gw[c];
            cv[CV_S] = sv;
            cv[CV_W] = wv;
            cv[CV_SM] = sm;
            cv[CV_WM] = wm;
            cv[CV_EB] = 0.5 * p->k_s * (sv - sm) * (sv - sm) + 0.5 * p->k_w * (wv - wm) * (wv - wm);
        }
        cv[CV_T] += D * (Fb[0] * Fb[0] + Fb[1] * Fb[1]);
        double g[3];
        orc_normals(p->seed, 0u, traj, step0 + (uint64_t)n, g);
        x += D * (F[0] + Fb[0]) + amp * g[0];
        y += D * (F[1] + Fb[1]) + amp * g[1];
    }
    xy[0] = x;
    xy[1] = y;
}

/* n_traj trajectories side by side (OpenMP); trajectory t uses id t0 + t.
 * xy [n_traj][2], cv [n_traj][8], frames NULL or [n_rec][n_traj][2]. */
int orc_funnel_batch(const orc_funnel_params *p, int n_traj, uint32_t t0, double *xy, double *cv, int64_t n_steps,
                     uint64_t step0, int record_every, double *frames, int K, const double *mp, int threads)
{
    int n_rec = (frames && record_every > 0) ? (int)(n_steps / record_every) + 1 : 0;
    int used = 1;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
#pragma omp single
        used = omp_get_num_threads();
        double *fr = n_rec ? (double *)malloc(sizeof(double) * 2 * (size_t)n_rec) : NULL;
#pragma omp for schedule(dynamic, 4)
        for (int t = 0; t < n_traj; ++t) {
            orc_funnel_steps(p, t0 + (uint32_t)t, xy + 2 * t, cv + (int64_t)ORC_CV_STRIDE * t, n_steps, step0,
                             record_every, fr, K, mp);
            for (int f = 0; f < n_rec; ++f) {
                frames[((int64_t)f * n_traj + t) * 2] = fr[2 * f];
                frames[((int64_t)f * n_traj + t) * 2 + 1] = fr[2 * f + 1];
            }
        }
        free(fr);
    }
    return used;
}

/* ---- array helpers for the test suite -------------------------------- */
void orc_contact_array(int64_t m, const double *r2, double r0, double r_cut,
                       double *C, double *dC_dr2)
{
    for (int64_t e = 0; e < m; ++e) C[e] = orc_contact(r2[e], r0, r_cut, dC_dr2 ? &dC_dr2[e] : NULL);
}

void orc_philox_array(int64_t m, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t e = 0; e < m; ++e) orc_philox4x32_10(ctr + 4 * e, key + 2 * e, out + 4 * e);
}

void orc_normals_array(int64_t m, uint64_t seed, const uint32_t *atom, const uint32_t *replica,
                       const uint64_t *step, double *out)
{
    for (int64_t e = 0; e < m; ++e) orc_normals(seed, atom[e], replica[e], step[e], out + 3 * e);
}
