// Key-point correspondence term, Eq.(9): E_corr = sum_s |V~_s - V_s|^2 over
// matched key points, V~_s the Eq.(1) warp (pose included) of the key point's
// carrying model point p_s and V_s its matched position (both in the
// frame's camera coordinates).
//
// Each key point contributes three rows with unit-axis normals, so for nodes
// j, l of p_s (weights w_j, w_l, d_j = (v - g_j, 1)):
//   H_jl += w_corr w_j w_l (d_j d_l^T) (x) I3      (R orthonormal)
//   g_j  += w_corr w_j d_j (x) R^T r_s
// Per Gauss-Newton step, one thread per key point evaluates the warp and the
// residual once; then one workgroup per node row adds the contributions of
// the key points whose k nodes include the row's node, in key-point order (no
// atomics: bitwise reproducible), and re-inverts the row's damped diagonal
// block for the block-Jacobi preconditioner, since the term changes it.
#include "frame.h"

namespace msl {

constexpr int kCorrThreads = 64;

template <int K>
constexpr int kp_stride() { return 3 + 4 * K; }   // R^T r, then per node q: w_q, d_q (3)

// Once per registration: the k nodes of each key point's carrying point (-1 for an index outside [0, n)),
// so that the rows scan one compact array instead of gathering from the kNN table.
template <int K>
__global__ void __launch_bounds__(256) kp_nodes_kernel(StepArgs a, KeyArgs kp, int32_t *kp_nodes) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= kp.count) return;
    const int64_t n = a.pts.n;
    const int p = kp.point[s];
    const bool ok = p >= 0 && p < n;
#pragma unroll
    for (int q = 0; q < K; ++q) kp_nodes[(size_t)s * K + q] = ok ? a.g.knn_idx[(int64_t)q * n + p] : -1;
}

// Per step, one thread per key point: residual r = V~ - V (float32), R^T r, the k weights and
// d_q = v - g_q, and the key point's energy |r|^2 (float64; 0 for a skipped key point).
template <int K>
__global__ void __launch_bounds__(256) kp_eval_kernel(StepArgs a, KeyArgs kp, const int32_t *__restrict__ kp_nodes,
                                                      float *kp_data, double *kp_energy) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= kp.count) return;
    float *o = kp_data + (size_t)s * kp_stride<K>();
    if (kp_nodes[(size_t)s * K] < 0) {
        for (int t = 0; t < kp_stride<K>(); ++t) o[t] = 0.f;
        kp_energy[s] = 0.0;
        return;
    }
    const int64_t n = a.pts.n;
    const int p = kp.point[s];
    const float vx = a.pts.px[p], vy = a.pts.py[p], vz = a.pts.pz[p];
    float ox, oy, oz;
    ed_blend<K>(vx, vy, vz, a.g.knn_idx, a.g.knn_w, n, p, a.nd, ox, oy, oz);
    apply_pose(a.pose, ox, oy, oz);
    const float rx = ox - kp.target[3 * (size_t)s], ry = oy - kp.target[3 * (size_t)s + 1],
                rz = oz - kp.target[3 * (size_t)s + 2];
    const float *R = a.pose.R;
    o[0] = fmaf(R[6], rz, fmaf(R[3], ry, R[0] * rx));
    o[1] = fmaf(R[7], rz, fmaf(R[4], ry, R[1] * rx));
    o[2] = fmaf(R[8], rz, fmaf(R[5], ry, R[2] * rx));
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int l = kp_nodes[(size_t)s * K + q];
        o[3 + 4 * q] = a.g.knn_w[(int64_t)q * n + p];
        o[4 + 4 * q] = vx - a.nd.gx[l];
        o[5 + 4 * q] = vy - a.nd.gy[l];
        o[6 + 4 * q] = vz - a.nd.gz[l];
    }
    kp_energy[s] = ((double)rx * rx + (double)ry * ry) + (double)rz * rz;
}

template <int K>
__global__ void __launch_bounds__(kCorrThreads) corr_rows_kernel(StepArgs a, KeyArgs kp,
                                                                 const int32_t *__restrict__ kp_nodes,
                                                                 const float *__restrict__ kp_data) {
    __shared__ int cols[MISSLAM_MAX_ROW];
    __shared__ float cacc[MISSLAM_MAX_ROW * 144];   // this term's part of the row's blocks
    __shared__ double Hd[12][12];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap);
    const int re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    const int nslots = min(re - rb, MISSLAM_MAX_ROW);
    for (int t = tid; t < nslots; t += kCorrThreads) cols[t] = a.g.col_idx[rb + t];
    for (int t = tid; t < nslots * 144; t += kCorrThreads) cacc[t] = 0.f;
    __syncthreads();
    double gacc = 0.0;     // gradient entry tid (< 12) of row j
    bool any = false;      // workgroup-uniform
    for (int s0 = 0; s0 < kp.count; s0 += kCorrThreads) {
        // the key points of this chunk whose carrying point has node j among its k nodes
        const int s = s0 + tid;
        bool mine = false;
        if (s < kp.count)
#pragma unroll
            for (int q = 0; q < K; ++q) mine = mine || kp_nodes[(size_t)s * K + q] == j;
        for (uint64_t todo = __ballot(mine); todo; todo &= todo - 1) {
            any = true;
            const int sk = s0 + __builtin_ctzll(todo);
            const float *d = kp_data + (size_t)sk * kp_stride<K>();
            int qj = 0;   // position of node j in the key point's set
#pragma unroll
            for (int q = 0; q < K; ++q)
                if (kp_nodes[(size_t)sk * K + q] == j) qj = q;
            const float wj = d[3 + 4 * qj];
            const float dj[4] = {d[4 + 4 * qj], d[5 + 4 * qj], d[6 + 4 * qj], 1.f};
            if (tid < 12) gacc = fma((double)(kp.w_corr * wj * dj[tid / 3]), (double)d[tid % 3], gacc);
            // entries (R, C) = (3c + a, 3c' + a') of the k blocks: only a = a' is non-zero
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int l = kp_nodes[(size_t)sk * K + q];
                int lo = 0, hi = nslots;   // slot of node l in the ascending row
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (cols[mid] < l)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo >= nslots || cols[lo] != l) continue;
                const float f = kp.w_corr * wj * d[3 + 4 * q];
                const float dl[4] = {d[4 + 4 * q], d[5 + 4 * q], d[6 + 4 * q], 1.f};
                for (int t = tid; t < 144; t += kCorrThreads) {
                    const int R = t / 12, C = t % 12;
                    if (R % 3 == C % 3) cacc[lo * 144 + t] = fmaf(f * dj[R / 3], dl[C / 3], cacc[lo * 144 + t]);
                }
            }
        }
    }
    if (!any) return;   // workgroup-uniform
    __syncthreads();
    // add this term to the row's blocks and gradient
    float *outb = a.blocks + (size_t)rb * 144;
    for (int t = tid; t < nslots * 144; t += kCorrThreads) {
        const float h = outb[t] + cacc[t];
        outb[t] = h;
        const int sl = t / 144, en = t % 144;
        if (cols[sl] == j) Hd[en / 12][en % 12] = (double)h + (en / 12 == en % 12 ? (double)a.lambda : 0.0);
    }
    if (tid < 12) a.gvec[(size_t)j * 12 + tid] = (float)((double)a.gvec[(size_t)j * 12 + tid] + gacc);
    if (a.minv) {
        __syncthreads();
        const bool ok = gj_inverse_block<kCorrThreads>(Hd, a.minv + (size_t)j * 144);
        if (!ok && tid == 0) atomicOr(a.flags, MISSLAM_FLAG_NONSPD_BLOCK);
    }
}

// rep->e_corr = sum of the key points' energies, in a fixed order (strided, wave butterflies, waves in order).
__global__ void __launch_bounds__(256) corr_report_kernel(const double *__restrict__ kp_energy, int count,
                                                          misslam_report *rep) {
    __shared__ double red[256 / kWave];
    double v = 0.0;
    for (int t = threadIdx.x; t < count; t += 256) v += kp_energy[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double e = ((red[0] + red[1]) + red[2]) + red[3];
        rep->e_corr = e;
        if (!isfinite(e)) rep->flags |= MISSLAM_FLAG_NONFINITE;
    }
}

hipError_t launch_kp_nodes(const StepArgs &a, const KeyArgs &kp, int32_t *kp_nodes, hipStream_t st) {
    if (kp.count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((kp.count + 255) / 256);
    switch (a.g.k) {
#define MSL_KN_CASE(KK) \
    case KK: hipLaunchKernelGGL((kp_nodes_kernel<KK>), dim3(blocks), dim3(256), 0, st, a, kp, kp_nodes); break;
        MSL_KN_CASE(1) MSL_KN_CASE(2) MSL_KN_CASE(3) MSL_KN_CASE(4)
        MSL_KN_CASE(5) MSL_KN_CASE(6) MSL_KN_CASE(7) MSL_KN_CASE(8)
#undef MSL_KN_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_corr_rows(const StepArgs &a, const KeyArgs &kp, const CorrScratch &c, bool assemble,
                            misslam_report *rep, hipStream_t st) {
    const int m = a.nd.m;
    if (kp.count <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((kp.count + 255) / 256);
    switch (a.g.k) {
#define MSL_KP_CASE(KK)                                                                                         \
    case KK:                                                                                                    \
        hipLaunchKernelGGL((kp_eval_kernel<KK>), dim3(blocks), dim3(256), 0, st, a, kp, c.kp_nodes, c.kp_data, \
                           c.kp_energy);                                                                        \
        if (assemble && m > 0)                                                                                  \
            hipLaunchKernelGGL((corr_rows_kernel<KK>), dim3(m), dim3(kCorrThreads), 0, st, a, kp, c.kp_nodes,  \
                               c.kp_data);                                                                      \
        break;
        MSL_KP_CASE(1) MSL_KP_CASE(2) MSL_KP_CASE(3) MSL_KP_CASE(4)
        MSL_KP_CASE(5) MSL_KP_CASE(6) MSL_KP_CASE(7) MSL_KP_CASE(8)
#undef MSL_KP_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(corr_report_kernel, dim3(1), dim3(256), 0, st, c.kp_energy, kp.count, rep);
    return hipGetLastError();
}

}  // namespace msl
