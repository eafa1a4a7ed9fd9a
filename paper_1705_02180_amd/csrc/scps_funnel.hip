// HIP kernels for gfx950: the toy model of the paper's illustration, one
// particle diffusing on the two-dimensional asymmetric funnel of eq (U)
// (parameters of Table 1), many trajectories at once.
//
// One thread per trajectory, float64 throughout (a few hundred flops per step,
// so the trajectories are cheap and exact arithmetic costs nothing that
// matters).  Overdamped Langevin steps X += D F + sqrt(2 kT D) xi with
// D = dt / (m gamma); noise from Philox4x32-10 with counter (0, trajectory,
// step_lo, step_hi) and the Box-Muller transform of its first two words.
// Bias: the rMD ratchet on z = |X| (eq (FrMD)), or the ratchets on the tube
// variables of eqs (Fw),(Fs) with the Euclidean distance to the frames of
// the mean path (d_k = |X - <X(t_k)>|^2), the toy model's stand-in for the
// contact map, one exponential per frame and step.  T accumulates
// D |F_bias|^2 per step.
#include <math.h>

#include "scps_device.h"
#include "scps_funnel.h"
#include "scps_internal.h"

namespace scps {

__device__ __forceinline__ double unit_open_d(uint32_t w) { return (double)(2u * (w >> 9) + 1u) * 0x1p-24; }

// U of eq (U) is not needed on the step; F = -grad U.
__device__ __forceinline__ void funnel_force(const FunnelK &P, double x, double y, double &fx, double &fy) {
    const double r2 = x * x + y * y;
    const double a1 = r2 + P.s1 * P.s1, a2 = r2 + P.s2 * P.s2;
    const double dx = x - P.xm, dy = y - P.ym;
    const double a3 = dx * dx + dy * dy + P.s3 * P.s3;
    // radial part: d/dr^2 of w^2 r^4 - A1 s1^2 / a1^2 + A2 s2^2 / a2^2, times 2
    const double g_r = 4.0 * P.w * P.w * r2 + 4.0 * P.A1 * P.s1 * P.s1 / (a1 * a1 * a1) -
                       4.0 * P.A2 * P.s2 * P.s2 / (a2 * a2 * a2);
    const double g_3 = 4.0 * P.A3 * P.s3 * P.s3 / (a3 * a3 * a3);
    fx = -(g_r * x + g_3 * dx);
    fy = -(g_r * y + g_3 * dy);
}

template <int BIAS>
__global__ __launch_bounds__(256) void k_funnel_steps(const FunnelK P, int n_traj, int first_id,
                                                      double2 *__restrict__ xy, double *__restrict__ cv,
                                                      int64_t n_steps, uint64_t step0, int record_every,
                                                      double2 *__restrict__ frames, int K,
                                                      const double2 *__restrict__ mp) {
    __shared__ double2 path[FUNNEL_KMAX];
    if (BIAS == 1) {
        for (int k = threadIdx.x; k < K; k += blockDim.x) path[k] = mp[k];
        __syncthreads();
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_traj) return;
    double x = xy[t].x, y = xy[t].y;
    double *c = cv + (int64_t)t * CV_STRIDE;
    double zm = c[CV_ZM], sm = c[CV_SM], wm = c[CV_WM], T = c[CV_T];
    double z = c[CV_Z], eb = c[CV_EB], sv = c[CV_S], wv = c[CV_W];
    const double D = P.mob_dt, amp = sqrt(2.0 * P.kT * P.mob_dt);
    const int M = K - 1;
    for (int64_t n = 0;; ++n) {
        if (frames && record_every > 0 && n % record_every == 0)
            frames[(n / record_every) * n_traj + t] = make_double2(x, y);
        if (n == n_steps) break;
        double fx, fy, bx = 0.0, by = 0.0;
        funnel_force(P, x, y, fx, fy);
        if (BIAS == 0) {
            z = sqrt(x * x + y * y);
            zm = fmin(zm, z);
            const double dz = z - zm;
            if (z > 0.0) {
                bx = -P.k_R * dz * x / z;
                by = -P.k_R * dz * y / z;
            }
            eb = 0.5 * P.k_R * dz * dz;
        } else {
            // tube variables: the largest exponent, then the weights with the sums
            // sum_k e_k grad d_k and sum_k k e_k grad d_k, from which
            // grad s = (lambda / M) sum_k p_k (k - kbar) grad d_k and grad w = lambda wscale sum_k p_k grad d_k
            double a = -INFINITY;
            for (int k = 0; k < K; ++k) {
                const double ex = x - path[k].x, ey = y - path[k].y;
                a = fmax(a, -P.lambda * (ex * ex + ey * ey));
            }
            double s0 = 0.0, s1 = 0.0, ax = 0.0, ay = 0.0, bx_ = 0.0, by_ = 0.0;
            for (int k = 0; k < K; ++k) {
                const double ex = x - path[k].x, ey = y - path[k].y;
                const double e = exp(-P.lambda * (ex * ex + ey * ey) - a);
                s0 += e;
                s1 += k * e;
                ax += e * 2.0 * ex;
                ay += e * 2.0 * ey;
                bx_ += k * e * 2.0 * ex;
                by_ += k * e * 2.0 * ey;
            }
            const double kbar = s1 / s0;
            sv = 1.0 - kbar / M;
            wv = tube_w(a, s0, P.wscale);
            const double gsx = (P.lambda / M) * (bx_ - kbar * ax) / s0, gsy = (P.lambda / M) * (by_ - kbar * ay) / s0;
            const double lw = P.lambda * P.wscale;
            const double gwx = lw * ax / s0, gwy = lw * ay / s0;
            sm = fmin(sm, sv);
            wm = fmin(wm, wv);
            const double ds = sv - sm, dw = wv - wm;
            bx = -P.k_s * ds * gsx - P.k_w * dw * gwx;
            by = -P.k_s * ds * gsy - P.k_w * dw * gwy;
            eb = 0.5 * P.k_s * ds * ds + 0.5 * P.k_w * dw * dw;
        }
        T += D * (bx * bx + by * by);
        uint32_t ctr[4] = {0u, (uint32_t)(first_id + t), (uint32_t)(step0 + n), (uint32_t)((step0 + n) >> 32)};
        philox4x32_10(ctr, P.seed_lo, P.seed_hi);
        const double rad = sqrt(-2.0 * log(unit_open_d(ctr[0])));
        const double ang = 6.283185307179586476925286766559 * unit_open_d(ctr[1]);
        x += D * (fx + bx) + amp * rad * cos(ang);
        y += D * (fy + by) + amp * rad * sin(ang);
    }
    xy[t] = make_double2(x, y);
    c[CV_Z] = z;
    c[CV_ZM] = zm;
    c[CV_EB] = eb;
    c[CV_S] = sv;
    c[CV_W] = wv;
    c[CV_SM] = sm;
    c[CV_WM] = wm;
    c[CV_T] = T;
}

hipError_t launch_funnel_steps(const FunnelK &P, int n_traj, int first_id, double2 *xy, double *cv, int64_t n_steps,
                               uint64_t step0, int record_every, double2 *frames, int K, const double2 *mp,
                               hipStream_t st) {
    const dim3 grid((n_traj + 255) / 256), block(256);
    if (P.bias_mode == 1)
        hipLaunchKernelGGL(k_funnel_steps<1>, grid, block, 0, st, P, n_traj, first_id, xy, cv, n_steps, step0,
                           record_every, frames, K, mp);
    else
        hipLaunchKernelGGL(k_funnel_steps<0>, grid, block, 0, st, P, n_traj, first_id, xy, cv, n_steps, step0,
                           record_every, frames, K, mp);
    return hipGetLastError();
}

// The mean path: frame f averaged over the listed trajectories, one
// workgroup per frame, a fixed-order float64 sum.
__global__ __launch_bounds__(256) void k_funnel_mean(int n_traj, const double2 *__restrict__ frames,
                                                     const int *__restrict__ list, int n_list,
                                                     double2 *__restrict__ out) {
    __shared__ double sx[256], sy[256];
    const int f = blockIdx.x, tid = threadIdx.x;
    double ax = 0.0, ay = 0.0;
    for (int q = tid; q < n_list; q += 256) {
        const double2 p = frames[(int64_t)f * n_traj + list[q]];
        ax += p.x;
        ay += p.y;
    }
    sx[tid] = ax;
    sy[tid] = ay;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            sx[tid] += sx[tid + h];
            sy[tid] += sy[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) out[f] = make_double2(sx[0] / n_list, sy[0] / n_list);
}

hipError_t launch_funnel_mean(int n_traj, int n_frames, const double2 *frames, const int *list, int n_list,
                              double2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_funnel_mean, dim3(n_frames), dim3(256), 0, st, n_traj, frames, list, n_list, out);
    return hipGetLastError();
}

}  // namespace scps
