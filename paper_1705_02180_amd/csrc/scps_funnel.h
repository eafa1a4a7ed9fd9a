// Toy model of the paper's illustration (one particle on the two-dimensional
// asymmetric funnel of eq (U)): device parameters and launches.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scps {

constexpr int FUNNEL_KMAX = 128;  // frames of a mean path

struct FunnelK {
    double A1, A2, A3, s1, s2, s3, w, xm, ym;
    double kT, mob_dt;            // overdamped step: X += mob_dt F + sqrt(2 kT mob_dt) xi
    double k_R, lambda, k_s, k_w;
    double wscale;                // w = -wscale log sum_k exp(-lambda d_k): 1/lambda, or 1 without the 1/lambda
    uint32_t seed_lo, seed_hi;
    int bias_mode;                // 0: rMD on z = |X|; 1: tube ratchets on the mean path
};

// n_traj trajectories (noise ids first_id + t) by n_steps steps from global
// step step0.  xy [n_traj] (x, y), cv [n_traj][8]; frames nullable
// [n_steps / record_every + 1][n_traj]; mean path mp [K] (bias_mode 1).
hipError_t launch_funnel_steps(const FunnelK &P, int n_traj, int first_id, double2 *xy, double *cv, int64_t n_steps,
                               uint64_t step0, int record_every, double2 *frames, int K, const double2 *mp,
                               hipStream_t st);
// Mean over the listed trajectories of every recorded frame: out [n_frames].
hipError_t launch_funnel_mean(int n_traj, int n_frames, const double2 *frames, const int *list, int n_list,
                              double2 *out, hipStream_t st);

}  // namespace scps
