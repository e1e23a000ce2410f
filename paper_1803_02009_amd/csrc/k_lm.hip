// Adaptive Levenberg-Marquardt damping (Sec. II-F): the paper names the
// method only; the schedule is the classical one.  A step dx solved with
// damping lambda is evaluated at x + dx; it is taken when the weighted Eq.(3)
// objective there is lower than at x, and lambda then shrinks by `down`
// (not below lambda_min); otherwise x stays and lambda grows by `up` (not
// above lambda_max).  lambda lives in one device float that the assembly and
// the solve of the next step read, so the whole schedule runs without a host
// round trip.
#include "frame.h"

namespace msl {

__global__ void lm_init_kernel(float *lambda_slot, float lambda0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *lambda_slot = lambda0;
}

__global__ void __launch_bounds__(256) lm_trial_kernel(const float *__restrict__ x, const float *__restrict__ dx,
                                                       float *__restrict__ xt, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) xt[i] = x[i] + dx[i];
}

__device__ __forceinline__ double lm_objective(const misslam_report &r, float w_data, float w_rot, float w_reg,
                                               float w_corr) {
    return (((double)w_data * r.e_data + (double)w_rot * r.e_rot) + (double)w_reg * r.e_reg) +
           (double)w_corr * r.e_corr;
}

// Every block takes the same decision from the same two reports; each copies its slice of x_trial when
// the step is taken, and block 0 alone updates lambda and the report (no block reads lambda).
__global__ void __launch_bounds__(256) lm_decide_kernel(misslam_report *rep_x, const misslam_report *rep_t,
                                                        misslam_lm_params lm, float w_data, float w_rot, float w_reg,
                                                        float w_corr, float *__restrict__ x,
                                                        const float *__restrict__ xt, int n, float *lambda_slot) {
    const double E = lm_objective(*rep_x, w_data, w_rot, w_reg, w_corr);
    const double Et = lm_objective(*rep_t, w_data, w_rot, w_reg, w_corr);
    // never a step whose solve timed out or met a non-finite value; false too for a non-finite objective
    const bool take = Et < E && !(rep_x->flags & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT));
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (take && i < n) x[i] = xt[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const float lam = *lambda_slot;
        rep_x->lm_e = E;
        rep_x->lm_e_trial = Et;
        rep_x->lm_lambda = lam;
        rep_x->lm_accepted = take ? 1 : 0;
        *lambda_slot = take ? fmaxf(lam * lm.down, lm.lambda_min) : fminf(lam * lm.up, lm.lambda_max);
    }
}

hipError_t launch_lm_init(float *lambda_slot, float lambda0, hipStream_t st) {
    hipLaunchKernelGGL(lm_init_kernel, dim3(1), dim3(64), 0, st, lambda_slot, lambda0);
    return hipGetLastError();
}

hipError_t launch_lm_trial(const float *x, const float *dx, float *x_trial, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lm_trial_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, dx, x_trial, n);
    return hipGetLastError();
}

hipError_t launch_lm_decide(misslam_report *rep_x, const misslam_report *rep_t, const misslam_lm_params &lm,
                            float w_data, float w_rot, float w_reg, float w_corr, float *x, const float *x_trial,
                            int n, float *lambda_slot, hipStream_t st) {
    const unsigned blocks = (unsigned)((n > 0 ? n : 1) + 255) / 256;
    hipLaunchKernelGGL(lm_decide_kernel, dim3(blocks), dim3(256), 0, st, rep_x, rep_t, lm, w_data, w_rot, w_reg,
                       w_corr, x, x_trial, n, lambda_slot);
    return hipGetLastError();
}

}  // namespace msl
