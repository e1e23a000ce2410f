// Key-point correspondence term, Eq.(9): E_corr = sum_s |V~_s - V_s|^2 over
// matched key points, V~_s the Eq.(1) warp (pose included) of the key point's
// carrying model point p_s and V_s its matched position (both in the
// frame's camera coordinates).
//
// Each key point contributes three rows with unit-axis normals, so for nodes
// j, l of p_s (weights w_j, w_l, d_j = (v - g_j, 1)):
//   H_jl += w_corr w_j w_l (d_j d_l^T) (x) I3      (R orthonormal)
//   g_j  += w_corr w_j d_j (x) R^T r_s
// Per Gauss-Newton step, the point pass evaluates each key point's warp and
// residual once (kp_eval_body); then one workgroup per node row adds the contributions of
// the key points whose k nodes include the row's node, in key-point order (no
// atomics: bitwise reproducible), and re-inverts the row's damped diagonal
// block for the block-Jacobi preconditioner, since the term changes it.  The
// energy is summed by the step's energy report.
#include "frame.h"

namespace msl {

constexpr int kCorrThreads = 64;

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

// One single-wave workgroup per node row j.  A scan of kp_nodes (kScanChunks x 64 key points per pass,
// all loads issued together) lists, in key-point order, the key points whose k nodes include j; the
// listed ones then load their data (written by the point pass) and find their nodes' slots in this row,
// 64 at a time in parallel, and are accumulated in list order.  Since the term's block (j, l) is
// M_jl (x) I3 with the 4x4 M_jl = sum w_corr w_j w_l d_j d_l^T, only M is accumulated; the write-back
// touches the 48 entries of each touched block that the pattern makes non-zero (all loads issued before
// the stores) and reads the rest of the diagonal block for the re-inversion.
constexpr int kScanChunks = 8;
constexpr int kWbPerThread = 8;

template <int K>
__global__ void __launch_bounds__(kCorrThreads) corr_rows_kernel(StepArgs a, KeyArgs kp,
                                                                 const int32_t *__restrict__ kp_nodes,
                                                                 const float *__restrict__ kp_data, float *Bout) {
    constexpr int S = kp_stride<K>();
    constexpr int kPass = kScanChunks * kCorrThreads;   // key points scanned per pass
    static_assert(MISSLAM_MAX_ROW <= kCorrThreads, "one thread per slot");
    __shared__ int cols[MISSLAM_MAX_ROW];
    __shared__ int tslot[MISSLAM_MAX_ROW];              // touched slots, ascending
    __shared__ int touched[MISSLAM_MAX_ROW];
    __shared__ float macc[MISSLAM_MAX_ROW * 16];        // this term's M per slot
    __shared__ int hits[kPass];                         // the pass's listed key points: s K + (position of j)
    __shared__ float kd[kCorrThreads][S];               // listed key points' R^T r, w_q, d_q (64 at a time)
    __shared__ int kslot[kCorrThreads][K];              // slot of each of their nodes in this row (-1: none)
    __shared__ int kqj[kCorrThreads];
    __shared__ double Hd[12][12];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap);
    const int re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    const int nslots = min(re - rb, MISSLAM_MAX_ROW);
    if (tid < MISSLAM_MAX_ROW) {
        cols[tid] = tid < nslots ? a.g.col_idx[rb + tid] : -1;
        touched[tid] = 0;
    }
    for (int t = tid; t < MISSLAM_MAX_ROW * 16; t += kCorrThreads) macc[t] = 0.f;
    double gacc = 0.0;     // gradient entry tid (< 12) of row j
    bool any = false;      // workgroup-uniform
    // joint pose form: entries tid and tid + 64 (< 72) of this row's border B_j, (3c + a) * 6 + k:
    //   w_corr w_j d_c R[:, a]^T [-[v~]x, I][:, k] = w_corr w_j d_c ((v~ x R[:, a])_k, or R[k - 3][a])
    float bacc0 = 0.f, bacc1 = 0.f;
    const Pose P = step_pose(a);
    const uint64_t below = (1ull << tid) - 1ull;
    for (int s0 = 0; s0 < kp.count; s0 += kPass) {
        int nd[kScanChunks][K];
#pragma unroll
        for (int u = 0; u < kScanChunks; ++u) {
            const int s = s0 + u * kCorrThreads + tid;
#pragma unroll
            for (int q = 0; q < K; ++q) nd[u][q] = s < kp.count ? kp_nodes[(size_t)s * K + q] : -1;
        }
        int nh = 0;   // wave-uniform
#pragma unroll
        for (int u = 0; u < kScanChunks; ++u) {
            int qj = -1;
#pragma unroll
            for (int q = 0; q < K; ++q)
                if (nd[u][q] == j) qj = q;
            const uint64_t hm = __ballot(qj >= 0);
            if (qj >= 0) hits[nh + __popcll(hm & below)] = (s0 + u * kCorrThreads + tid) * K + qj;
            nh += __popcll(hm);
        }
        if (nh == 0) continue;
        any = true;
        __syncthreads();
        for (int h0 = 0; h0 < nh; h0 += kCorrThreads) {
            const int cnt = min(nh - h0, kCorrThreads);
            if (tid < cnt) {
                const int e = hits[h0 + tid], s = e / K;
                const float *d = kp_data + (size_t)s * S;
                float v[S];
                int l[K];
#pragma unroll
                for (int t = 0; t < S; ++t) v[t] = d[t];
#pragma unroll
                for (int q = 0; q < K; ++q) l[q] = kp_nodes[(size_t)s * K + q];
#pragma unroll
                for (int t = 0; t < S; ++t) kd[tid][t] = v[t];
                kqj[tid] = e % K;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    int lo = 0, hi = nslots;   // slot of node l[q] in the ascending row
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (cols[mid] < l[q])
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    const bool in = lo < nslots && cols[lo] == l[q];
                    kslot[tid][q] = in ? lo : -1;
                    if (in) touched[lo] = 1;
                }
            }
            __syncthreads();
            if (tid < 16) {
                const int c = tid / 4, c2 = tid % 4;
                for (int L = 0; L < cnt; ++L) {
                    const int qjL = kqj[L];
                    const float wj = kd[L][3 + 4 * qjL];
                    const float djc = c < 3 ? kd[L][4 + 4 * qjL + c] : 1.f;
                    if (tid < 12) {
                        const float djg = tid / 3 < 3 ? kd[L][4 + 4 * qjL + tid / 3] : 1.f;
                        gacc = fma((double)(kp.w_corr * wj * djg), (double)kd[L][tid % 3], gacc);
                    }
                    // node by node, so that a repeated node would add twice, in order
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        const int sl = kslot[L][q];
                        if (sl >= 0) {
                            const float f = kp.w_corr * wj * kd[L][3 + 4 * q];
                            const float dlc = c2 < 3 ? kd[L][4 + 4 * q + c2] : 1.f;
                            macc[sl * 16 + tid] = fmaf(f * djc, dlc, macc[sl * 16 + tid]);
                        }
                    }
                }
            }
            if (Bout) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = tid + 64 * h;
                    if (e >= 72) continue;
                    const int c = (e / 6) / 3, ax = (e / 6) % 3, k = e % 6;
                    const float ux = P.R[ax], uy = P.R[3 + ax], uz = P.R[6 + ax];   // R[:, a]
                    float acc = h ? bacc1 : bacc0;
                    for (int L = 0; L < cnt; ++L) {
                        const int qjL = kqj[L];
                        const float wj = kd[L][3 + 4 * qjL];
                        const float dc = c < 3 ? kd[L][4 + 4 * qjL + c] : 1.f;
                        const float vx = kd[L][3 + 4 * K], vy = kd[L][4 + 4 * K], vz = kd[L][5 + 4 * K];
                        float col;
                        if (k == 0) col = fmaf(vy, uz, -vz * uy);
                        else if (k == 1) col = fmaf(vz, ux, -vx * uz);
                        else if (k == 2) col = fmaf(vx, uy, -vy * ux);
                        else col = k == 3 ? ux : (k == 4 ? uy : uz);
                        acc = fmaf(kp.w_corr * wj * dc, col, acc);
                    }
                    if (h) bacc1 = acc;
                    else bacc0 = acc;
                }
            }
            __syncthreads();   // hits, kd, kslot and kqj are refilled next
        }
    }
    if (!any) return;   // workgroup-uniform
    const uint64_t tm = __ballot(tid < nslots && touched[tid] != 0);
    const uint64_t dm = __ballot(tid < nslots && cols[tid] == j);
    const int nts = __popcll(tm);
    const int dslot = dm ? __builtin_ctzll(dm) : -1;
    if (tid < nslots && touched[tid]) tslot[__popcll(tm & below)] = tid;
    __syncthreads();
    const bool inv = a.minv && dslot >= 0;
    const int npat = nts * 48;                 // pattern entries of the touched blocks
    const int items = npat + (inv ? 96 : 0);   // + the diagonal block's other entries
    float *outb = a.blocks + (size_t)rb * 144;
    for (int base = 0; base < items; base += kWbPerThread * kCorrThreads) {
        float h[kWbPerThread];
        int off[kWbPerThread], mi[kWbPerThread];
#pragma unroll
        for (int e = 0; e < kWbPerThread; ++e) {
            const int it = base + e * kCorrThreads + tid;
            off[e] = -1;
            mi[e] = -1;
            h[e] = 0.f;
            if (it < npat) {
                // entry (3c + x, 3c' + x) of touched block it / 48, with cc = 4c + c'
                const int sl = tslot[it / 48], w = it % 48, x = w % 3, cc = w / 3;
                off[e] = sl * 144 + (3 * (cc / 4) + x) * 12 + 3 * (cc % 4) + x;
                mi[e] = sl * 16 + cc;
            } else if (it < items) {
                // entry (R, C) of the diagonal block with R % 3 != C % 3 (8 per row R)
                const int w = it - npat, R = w / 8, k = w % 8;
                off[e] = dslot * 144 + R * 12 + 3 * (k / 2) + (R % 3 + 1 + k % 2) % 3;
            }
            if (off[e] >= 0) h[e] = outb[off[e]];
        }
#pragma unroll
        for (int e = 0; e < kWbPerThread; ++e) {
            if (off[e] < 0) continue;
            if (mi[e] >= 0) {
                h[e] = h[e] + macc[mi[e]];
                outb[off[e]] = h[e];
            }
            if (inv && off[e] / 144 == dslot) {
                const int en = off[e] % 144;
                Hd[en / 12][en % 12] = (double)h[e] + (en / 12 == en % 12 ? (double)step_lambda(a) : 0.0);
            }
        }
    }
    if (tid < 12) a.gvec[(size_t)j * 12 + tid] = (float)((double)a.gvec[(size_t)j * 12 + tid] + gacc);
    if (Bout) {
        Bout[(size_t)j * 72 + tid] += bacc0;
        if (tid + 64 < 72) Bout[(size_t)j * 72 + tid + 64] += bacc1;
    }
    if (inv) {
        __syncthreads();
        const bool ok = gj_inverse_block<kCorrThreads>(Hd, a.minv + (size_t)j * 144);
        if (!ok && tid == 0) atomicOr(a.flags, MISSLAM_FLAG_NONSPD_BLOCK);
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

hipError_t launch_corr_rows(const StepArgs &a, const KeyArgs &kp, const CorrScratch &c, hipStream_t st, float *B) {
    const int m = a.nd.m;
    if (kp.count <= 0 || m <= 0) return hipSuccess;
    switch (a.g.k) {
#define MSL_KP_CASE(KK)                                                                                      \
    case KK:                                                                                                 \
        hipLaunchKernelGGL((corr_rows_kernel<KK>), dim3(m), dim3(kCorrThreads), 0, st, a, kp, c.kp_nodes,   \
                           c.kp_data, B);                                                                       \
        break;
        MSL_KP_CASE(1) MSL_KP_CASE(2) MSL_KP_CASE(3) MSL_KP_CASE(4)
        MSL_KP_CASE(5) MSL_KP_CASE(6) MSL_KP_CASE(7) MSL_KP_CASE(8)
#undef MSL_KP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace msl
