// Joint rigid pose + ED registration (Eq.(3) with the Eq.(10) pose terms;
// Sec. II-F: six more unknowns).  The pose perturbation xi = (dw, dt) acts as
// R <- exp([dw]x) R, T <- exp([dw]x) T + dt, so a data row gains the pose
// columns Jp = (v~ x N, N).  Per Gauss-Newton step:
//   - the joint point pass writes Jp per point and per-block partials of
//     sum Jp Jp^T and sum Jp r;
//   - border_rows_kernel forms B_j = w_data sum_i w_ij kron(d_ij, n'_i) Jp_i^T
//     (12 x 6 per node) from the node's list, one workgroup per node;
//   - pose_setup_kernel reduces the partials, adds the priors w_r |log(R R0^T)|^2
//     and w_p |C - C0|^2 (C = -R^T T; Jacobians I and -R^T, the first exact for
//     the gradient) and factors the damped 6x6 block;
//   - the joint PCG runs the textbook recurrence of the ED solve over the joint
//     vector (the pose part in float64, computed redundantly by every block from
//     the same partials, so every block holds the same values), then applies
//     x += dx and the pose step.
#include "frame.h"

namespace msl {

constexpr int kJThreads = 256;
constexpr int kJRows = 21;          // node rows per block, 12 threads per row
constexpr int kJKinds = 10;         // partial kinds per iteration: r.z, r.r, p.q, #non-finite, B^T z (6)
constexpr int kPst = 32;            // pose state per iteration: r, z, p, q, x (6 each)

__global__ void pose_init_kernel(Pose P, float *pose_dev) {
    const int t = threadIdx.x;
    if (t < 9) pose_dev[t] = P.R[t];
    else if (t < 12) pose_dev[t] = P.T[t - 9];
}

// ---------------------------------------------------------------- border B_j

constexpr int kBorderWaves = 4;
constexpr int kBorderSlices = 5;   // entry slices per wave: lane = 12 * slice + (3c + a); lanes 60-63 only load

// One workgroup per node row.  Each wave stages 64 of the row's list entries at a time (w d, n', Jp, all
// float4-aligned) and only reads its own: lane (slice, 3c + a) adds, over the staged entries t = slice,
// slice + 5, ..., (w d_c n'_a) Jp_k into its six columns k.  The partial sums are added slice by slice and wave
// by wave in a fixed order.
__global__ void __launch_bounds__(kBorderWaves * 64) border_rows_kernel(StepArgs a, StepScratch s, float *B) {
    __shared__ float4 ent[kBorderWaves][64][4];   // per wave: (w d, w), (n', 0), Jp 0-3, (Jp 4-5, 0, 0)
    __shared__ float part[kBorderWaves][kBorderSlices][72];
    const int j = blockIdx.x;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int l0 = a.g.list_ptr[j], l1 = a.g.list_ptr[j + 1];
    const int slice = lane / 12, ca = lane % 12, c = ca / 3, aa = ca % 3;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float4 (*E)[4] = ent[wave];
    for (int base0 = l0; base0 < l1; base0 += 64 * kBorderWaves) {
        const int base = base0 + 64 * wave;
        const int le = base + lane;
        if (le < l1) {
            const int p = a.g.list_pts[le];
            const float4 dw = s.lpa[le];
            const float4 nr = s.nr[p];
            const float4 j0 = s.jp[2 * (size_t)p], j1 = s.jp[2 * (size_t)p + 1];
            E[lane][0] = make_float4(dw.w * dw.x, dw.w * dw.y, dw.w * dw.z, dw.w);
            E[lane][1] = make_float4(nr.x, nr.y, nr.z, 0.f);
            E[lane][2] = j0;
            E[lane][3] = j1;
        }
        wave_sync();
        const int cnt = max(0, min(64, l1 - base));
        if (slice < kBorderSlices)
            for (int t = slice; t < cnt; t += kBorderSlices) {
                const float *wd = reinterpret_cast<const float *>(&E[t][0]);
                const float *nn = reinterpret_cast<const float *>(&E[t][1]);
                const float f = wd[c] * nn[aa];
                const float4 ja = E[t][2], jb = E[t][3];
                acc[0] = fmaf(f, ja.x, acc[0]);
                acc[1] = fmaf(f, ja.y, acc[1]);
                acc[2] = fmaf(f, ja.z, acc[2]);
                acc[3] = fmaf(f, ja.w, acc[3]);
                acc[4] = fmaf(f, jb.x, acc[4]);
                acc[5] = fmaf(f, jb.y, acc[5]);
            }
        wave_sync();   // the wave's reads of this pass before its next writes
    }
    if (slice < kBorderSlices)
#pragma unroll
        for (int k = 0; k < 6; ++k) part[wave][slice][ca * 6 + k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 72) {
        const int e = threadIdx.x;
        float t = part[0][0][e];
        for (int sl = 1; sl < kBorderSlices; ++sl) t += part[0][sl][e];
#pragma unroll
        for (int w = 1; w < kBorderWaves; ++w)
            for (int sl = 0; sl < kBorderSlices; ++sl) t += part[w][sl][e];
        B[(size_t)j * 72 + e] = a.w_data * t;
    }
}

hipError_t launch_border_rows(const StepArgs &a, const StepScratch &s, float *B, hipStream_t st) {
    if (a.nd.m <= 0) return hipSuccess;
    hipLaunchKernelGGL(border_rows_kernel, dim3(a.nd.m), dim3(kBorderWaves * 64), 0, st, a, s, B);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pose block

__device__ inline void so3_log_d(const double R[9], double w[3]) {
    const double c = fmin(1.0, fmax(-1.0, (R[0] + R[4] + R[8] - 1.0) * 0.5));
    const double th = acos(c);
    const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    const double f = th < 1e-8 ? 0.5 : th / (2.0 * sin(th));
#pragma unroll
    for (int t = 0; t < 3; ++t) w[t] = f * v[t];
}

__device__ inline void so3_exp_d(const double w[3], double E[9]) {
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    double KK[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) KK[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    const double f1 = th < 1e-12 ? 1.0 : sin(th) / th;
    const double f2 = th < 1e-12 ? 0.5 : (1.0 - cos(th)) / (th * th);
#pragma unroll
    for (int t = 0; t < 9; ++t) E[t] = (t % 4 == 0 ? 1.0 : 0.0) + f1 * K[t] + f2 * KK[t];
}

// Gauss-Jordan on the diagonal pivots of a 6x6 SPD float64 matrix (one thread,
// fully unrolled so that the matrix stays in registers).  A non-positive pivot
// (not SPD) returns false.
__device__ inline bool inverse6(const double A_in[36], double out[36]) {
    double A[6][12];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 12; ++c) A[r][c] = c < 6 ? A_in[6 * r + c] : (c - 6 == r ? 1.0 : 0.0);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        ok = ok && A[k][k] > 0.0;
        const double ip = A[k][k] > 0.0 ? 1.0 / A[k][k] : 1.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) A[k][c] *= ip;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (r == k) continue;
            const double f = A[r][k];
#pragma unroll
            for (int c = 0; c < 12; ++c) A[r][c] -= f * A[k][c];
        }
    }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) out[6 * r + c] = A[r][6 + c];
    return ok;
}

struct PoseKeys {
    int count;
    float w_corr;
    const int32_t *point;
    const float *data;     // kp_data
    int stride;            // 9 + 4k
    int off_v;             // offset of v~ (then r) in a record: 3 + 4k
    int64_t n;
};

__global__ void __launch_bounds__(256) pose_setup_kernel(const float *pose_dev, PosePrior pr,
                                                         const double *__restrict__ part, int nblk_pts, float lambda,
                                                         double *sys, misslam_report *rep,
                                                         unsigned long long *jbar, int jbar_words, PoseKeys pk) {
    __shared__ double wred[2][256 / kWave][kPosePart];
    for (int t = threadIdx.x; t < jbar_words; t += 256) jbar[t] = 0ull;   // the next joint solve's sync area
    double v[kPosePart], vk[kPosePart];
#pragma unroll
    for (int q = 0; q < kPosePart; ++q) {
        v[q] = 0.0;
        vk[q] = 0.0;
    }
    for (int b = threadIdx.x; b < nblk_pts; b += 256)
#pragma unroll
        for (int q = 0; q < kPosePart; ++q) v[q] += part[(size_t)kPosePart * b + q];
    // key points: rows [-[v~]x, I] with residual r, weight w_corr
    for (int s = threadIdx.x; s < pk.count; s += 256) {
        const int p = pk.point[s];
        if (p < 0 || p >= pk.n) continue;
        const float *o = pk.data + (size_t)s * pk.stride + pk.off_v;
        const double vx = o[0], vy = o[1], vz = o[2], r3[3] = {o[3], o[4], o[5]};
        const double J[3][6] = {{0.0, vz, -vy, 1.0, 0.0, 0.0}, {-vz, 0.0, vx, 0.0, 1.0, 0.0},
                                {vy, -vx, 0.0, 0.0, 0.0, 1.0}};
        const double wc = (double)pk.w_corr;
        int e = 0;
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int w = u; w < 6; ++w) vk[e++] += wc * ((J[0][u] * J[0][w] + J[1][u] * J[1][w]) + J[2][u] * J[2][w]);
#pragma unroll
        for (int u = 0; u < 6; ++u) vk[21 + u] += wc * ((J[0][u] * r3[0] + J[1][u] * r3[1]) + J[2][u] * r3[2]);
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    wave_sums(v);
    if (pk.count > 0) wave_sums(vk);   // else every vk is +0.0, and so is its sum
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < kPosePart; ++q) {
            wred[0][wave][q] = v[q];
            wred[1][wave][q] = vk[q];
        }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double S[kPosePart], SK[kPosePart];
#pragma unroll
    for (int q = 0; q < kPosePart; ++q) {
        S[q] = ((wred[0][0][q] + wred[0][1][q]) + wred[0][2][q]) + wred[0][3][q];
        SK[q] = ((wred[1][0][q] + wred[1][1][q]) + wred[1][2][q]) + wred[1][3][q];
    }
    double H[36], g[6];
    int e = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
        for (int w = u; w < 6; ++w) {
            H[6 * u + w] = (double)pr.w_data * S[e] + SK[e];
            H[6 * w + u] = (double)pr.w_data * S[e] + SK[e];
            ++e;
        }
#pragma unroll
    for (int u = 0; u < 6; ++u) g[u] = (double)pr.w_data * S[21 + u] + SK[21 + u];
    // priors: rho_r = log(R R0^T), rho_p = C - C0
    double R[9], T[3], R0[9], T0[3], M[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        R[t] = pose_dev[t];
        R0[t] = pr.R0[t];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        T[t] = pose_dev[9 + t];
        T0[t] = pr.T0[t];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            M[3 * r + c] = (R[3 * r] * R0[3 * c] + R[3 * r + 1] * R0[3 * c + 1]) + R[3 * r + 2] * R0[3 * c + 2];
    double rr[3], rp[3];
    so3_log_d(M, rr);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double C = -((R[a] * T[0] + R[3 + a] * T[1]) + R[6 + a] * T[2]);
        const double C0 = -((R0[a] * T0[0] + R0[3 + a] * T0[1]) + R0[6 + a] * T0[2]);
        rp[a] = C - C0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        H[6 * a + a] += (double)pr.w_r;
        g[a] += (double)pr.w_r * rr[a];
        g[3 + a] -= (double)pr.w_p * ((R[3 * a] * rp[0] + R[3 * a + 1] * rp[1]) + R[3 * a + 2] * rp[2]);
#pragma unroll
        for (int b = 0; b < 3; ++b)
            H[6 * (3 + a) + 3 + b] +=
                (double)pr.w_p * ((R[3 * a] * R[3 * b] + R[3 * a + 1] * R[3 * b + 1]) + R[3 * a + 2] * R[3 * b + 2]);
    }
    if (rep) {
        rep->e_pose_r = (rr[0] * rr[0] + rr[1] * rr[1]) + rr[2] * rr[2];
        rep->e_pose_p = (rp[0] * rp[0] + rp[1] * rp[1]) + rp[2] * rp[2];
    }
    if (!sys) return;
    double Hd[36], Mi[36];
#pragma unroll
    for (int t = 0; t < 36; ++t) Hd[t] = H[t] + (t % 7 == 0 ? (double)lambda : 0.0);
    const bool ok = inverse6(Hd, Mi);
#pragma unroll
    for (int t = 0; t < 36; ++t) {
        sys[t] = H[t];
        sys[42 + t] = ok ? Mi[t] : (t % 7 == 0 ? 1.0 : 0.0);
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) sys[36 + t] = g[t];
    if (!ok && rep) rep->flags |= MISSLAM_FLAG_NONSPD_BLOCK;
}

hipError_t launch_pose_init(const Pose &pose, float *pose_dev, hipStream_t st) {
    hipLaunchKernelGGL(pose_init_kernel, dim3(1), dim3(64), 0, st, pose, pose_dev);
    return hipGetLastError();
}

hipError_t launch_pose_setup(const float *pose_dev, const PosePrior &pr, const double *pose_part, int nblk_pts,
                             float lambda, double *sys, misslam_report *rep, hipStream_t st,
                             unsigned long long *jbar, int m, const KeyArgs *kp, const CorrScratch *c, int64_t n,
                             int k) {
    const int words = jbar ? joint_sync_words(m) : 0;
    PoseKeys pk{};
    if (kp && c && kp->count > 0) {
        pk.count = kp->count;
        pk.w_corr = kp->w_corr;
        pk.point = kp->point;
        pk.data = c->kp_data;
        pk.stride = 9 + 4 * k;
        pk.off_v = 3 + 4 * k;
        pk.n = n;
    }
    hipLaunchKernelGGL(pose_setup_kernel, dim3(1), dim3(256), 0, st, pose_dev, pr, pose_part, nblk_pts, lambda, sys,
                       rep, jbar, words, pk);
    return hipGetLastError();
}

// ---------------------------------------------------------------- joint PCG

struct JArgs {
    PcgArgs A;
    const float *B;
    const double *sys;    // H_pp (36), g_p (6), (H_pp + lambda I)^-1 (36)
    double *jpart;
    double *pst;
};

// Sums N values over the block (wave butterflies, then the waves in order); every thread gets the totals.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double (*lds)[kJThreads / kWave]) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    wave_sums(v);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) lds[q][wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = ((lds[q][0] + lds[q][1]) + lds[q][2]) + lds[q][3];
    __syncthreads();
}

// The block totals of N partial kinds: (iteration, kind) pairs its[q], kinds[q].
template <int N>
__device__ __forceinline__ void jgather(const JArgs &J, const int (&its)[N], const int (&kinds)[N], double (&out)[N],
                                        double (*lds)[kJThreads / kWave]) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
        out[q] = 0.0;
        const double *p = J.jpart + (size_t)(its[q] * kJKinds + kinds[q]) * J.A.nblk;
        for (int t = threadIdx.x; t < J.A.nblk; t += kJThreads) out[q] += p[t];
    }
    block_sums<N>(out, lds);
}

__device__ __forceinline__ float jprecond(const float *minv, int j, int a, const float *rl) {
    const float *M = minv + (size_t)j * 144 + a * 12;
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < 12; ++b) s = fmaf(M[b], rl[b], s);
    return s;
}

__global__ void __launch_bounds__(kJThreads) jpcg_init_kernel(JArgs J) {
    const PcgArgs &A = J.A;
    __shared__ double red[16][kJThreads / kWave];
    __shared__ float rl[kJRows][12];
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kJRows + row;
    const bool act = row < kJRows && j < A.m;
    float r = 0.f, z = 0.f;
    if (act) {
        r = -A.g[(size_t)j * 12 + a];
        rl[row][a] = r;
    }
    __syncthreads();
    if (act) {
        z = jprecond(A.minv, j, a, rl[row]);
        A.r[(size_t)j * 12 + a] = r;
        A.z[(size_t)j * 12 + a] = z;
        A.x[(size_t)j * 12 + a] = 0.f;
    }
    double sums[2] = {(double)r * (double)z, (double)r * (double)r};
    block_sums<2>(sums, red);
    double rz = sums[0], rr = sums[1];
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) {   // the pose part: r_p = -g_p, z_p = M_p r_p
            double rp[6], zp[6];
            for (int u = 0; u < 6; ++u) rp[u] = -J.sys[36 + u];
            for (int u = 0; u < 6; ++u) {
                double t = 0.0;
                for (int w = 0; w < 6; ++w) t += J.sys[42 + 6 * u + w] * rp[w];
                zp[u] = t;
            }
            double rz_p = 0.0, rr_p = 0.0;   // summed apart, then added: the one-launch solve's order
            for (int u = 0; u < 6; ++u) {
                rz_p += rp[u] * zp[u];
                rr_p += rp[u] * rp[u];
                J.pst[u] = rp[u];
                J.pst[6 + u] = zp[u];
                J.pst[12 + u] = 0.0;
                J.pst[18 + u] = 0.0;
                J.pst[24 + u] = 0.0;
            }
            rz += rz_p;
            rr += rr_p;
        }
        J.jpart[(size_t)0 * A.nblk + blockIdx.x] = rz;
        J.jpart[(size_t)1 * A.nblk + blockIdx.x] = rr;
        J.jpart[(size_t)3 * A.nblk + blockIdx.x] = 0.0;
    }
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t <= A.iters; t += kJThreads) {
            A.status[t] = 0;
            A.done[t] = 0;
        }
}

// q_e = H z_e + lambda z_e + B z_p + beta q_e, p_e = z_e + beta p_e; partials p_e.q_e and B^T z_e.
__global__ void __launch_bounds__(kJThreads) jpcg_dir_kernel(JArgs J, int it) {
    const PcgArgs &A = J.A;
    __shared__ double red[16][kJThreads / kWave];
    __shared__ double zp[6];
    double gz[2];
    jgather<2>(J, {it, it > 0 ? it - 1 : 0}, {0, 0}, gz, red);
    const double rz = gz[0];
    const double rz_prev = it > 0 ? gz[1] : 1.0;
    if (threadIdx.x < 6) zp[threadIdx.x] = J.pst[(size_t)it * kPst + 6 + threadIdx.x];
    __syncthreads();
    const bool skip = A.status[it] != 0 || rz == 0.0;
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kJRows + row;
    const bool act = row < kJRows && j < A.m && !skip;
    double pq = 0.0, btz[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (act) {
        const float beta = it > 0 ? (float)(rz / rz_prev) : 0.f;
        double az = 0.0;
        const int p0 = A.row_ptr[j], p1 = min(A.row_ptr[j + 1], A.cap);
        for (int pb = p0; pb < p1; ++pb) {
            const int l = A.col_idx[pb];
            const float *Bk = A.blocks + (size_t)pb * 144 + a * 12;
            const float *zl = A.z + (size_t)l * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) az = fma((double)Bk[b], (double)zl[b], az);
        }
        const size_t o = (size_t)j * 12 + a;
        const float zj = A.z[o];
        az = fma((double)A.lambda, (double)zj, az);
        const float *Bj = J.B + (size_t)j * 72 + a * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            az = fma((double)Bj[k], zp[k], az);
            btz[k] = (double)Bj[k] * (double)zj;
        }
        float p, q;
        if (it > 0) {
            p = fmaf(beta, A.p[o], zj);
            q = (float)fma((double)beta, (double)A.q[o], az);
        } else {
            p = zj;
            q = (float)az;
        }
        A.p[o] = p;
        A.q[o] = q;
        pq = (double)p * (double)q;
    }
    double sums[7] = {pq, btz[0], btz[1], btz[2], btz[3], btz[4], btz[5]};
    block_sums<7>(sums, red);
    if (threadIdx.x == 0) {
        J.jpart[(size_t)(it * kJKinds + 2) * A.nblk + blockIdx.x] = sums[0];
        for (int k = 0; k < 6; ++k) J.jpart[(size_t)(it * kJKinds + 4 + k) * A.nblk + blockIdx.x] = sums[1 + k];
    }
}

// The pose part of the product and the step, then the ED step: alpha = r.z / p.q over the joint vector.
__global__ void __launch_bounds__(kJThreads) jpcg_step_kernel(JArgs J, int it) {
    const PcgArgs &A = J.A;
    __shared__ double red[16][kJThreads / kWave];
    __shared__ float rl[kJRows][12];
    __shared__ double ps[kPst];   // this iteration's pose r, z, p, q, x after the step
    __shared__ double pq_pose;
    const int ip = it > 0 ? it - 1 : 0;
    double gs[9];
    jgather<9>(J, {it, ip, it, it, it, it, it, it, it}, {0, 0, 2, 4, 5, 6, 7, 8, 9}, gs, red);
    const double rz = gs[0];
    const double rz_prev = it > 0 ? gs[1] : 1.0;
    const double pq_e = gs[2];
    const double btz[6] = {gs[3], gs[4], gs[5], gs[6], gs[7], gs[8]};
    const int st = A.status[it];
    const bool skip = st != 0 || rz == 0.0;
    const float beta = it > 0 ? (float)(rz / rz_prev) : 0.f;
    if (threadIdx.x == 0) {
        const double *cur = J.pst + (size_t)it * kPst;
        double zp[6], pp[6], qp[6];
        for (int u = 0; u < 6; ++u) {
            double az = btz[u];
            for (int w = 0; w < 6; ++w) az += J.sys[6 * u + w] * cur[6 + w];
            az += (double)A.lambda * cur[6 + u];
            zp[u] = cur[6 + u];
            qp[u] = it > 0 ? (double)beta * cur[18 + u] + az : az;
            pp[u] = it > 0 ? (double)beta * cur[12 + u] + zp[u] : zp[u];
        }
        double t = 0.0;
        for (int u = 0; u < 6; ++u) t += pp[u] * qp[u];
        pq_pose = t;
        for (int u = 0; u < 6; ++u) {
            ps[u] = cur[u];
            ps[6 + u] = cur[6 + u];
            ps[12 + u] = skip ? cur[12 + u] : pp[u];
            ps[18 + u] = skip ? cur[18 + u] : qp[u];
            ps[24 + u] = cur[24 + u];
        }
    }
    __syncthreads();
    const double pq = pq_e + pq_pose;
    const bool brk = !skip && !(pq > 0.0);
    const bool upd = !skip && !brk;
    const float alpha = upd ? (float)(rz / pq) : 0.f;
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kJRows + row;
    const bool in = row < kJRows && j < A.m;
    const size_t o = (size_t)j * 12 + a;
    float r = 0.f;
    double bad = 0.0;
    if (in) {
        r = A.r[o];
        float xv = A.x[o];
        if (upd) {
            xv = fmaf(alpha, A.p[o], xv);
            A.x[o] = xv;
            r = fmaf(-alpha, A.q[o], r);
            A.r[o] = r;
        }
        bad = isfinite(xv) ? 0.0 : 1.0;
        rl[row][a] = r;
    }
    __syncthreads();
    float z = 0.f;
    if (in) {
        if (upd) {
            z = jprecond(A.minv, j, a, rl[row]);
            A.z[o] = z;
        } else {
            z = A.z[o];
        }
    }
    double sums[3] = {(double)r * (double)z, (double)r * (double)r, bad};
    block_sums<3>(sums, red);
    double rzn = sums[0], rrn = sums[1], nb = sums[2];
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) {   // the pose step, stored for the next iteration
            double *nxt = J.pst + (size_t)(it + 1) * kPst;
            double rp[6], zp[6], rz_p = 0.0, rr_p = 0.0, nb_p = 0.0;
            for (int u = 0; u < 6; ++u) {
                rp[u] = upd ? ps[u] - (double)alpha * ps[18 + u] : ps[u];
                nxt[24 + u] = upd ? ps[24 + u] + (double)alpha * ps[12 + u] : ps[24 + u];
                if (!isfinite(nxt[24 + u])) nb_p += 1.0;
            }
            for (int u = 0; u < 6; ++u) {
                double t = 0.0;
                for (int w = 0; w < 6; ++w) t += J.sys[42 + 6 * u + w] * rp[w];
                zp[u] = upd ? t : ps[6 + u];
            }
            for (int u = 0; u < 6; ++u) {   // summed apart, then added: the one-launch solve's order
                rz_p += rp[u] * zp[u];
                rr_p += rp[u] * rp[u];
                nxt[u] = rp[u];
                nxt[6 + u] = zp[u];
                nxt[12 + u] = ps[12 + u];
                nxt[18 + u] = ps[18 + u];
            }
            rzn += rz_p;
            rrn += rr_p;
            nb += nb_p;
            A.status[it + 1] = st != 0 ? st : (brk ? 2 : 0);
            A.done[it] = upd ? 1 : 0;
        }
        J.jpart[(size_t)((it + 1) * kJKinds + 0) * A.nblk + blockIdx.x] = rzn;
        J.jpart[(size_t)((it + 1) * kJKinds + 1) * A.nblk + blockIdx.x] = rrn;
        J.jpart[(size_t)((it + 1) * kJKinds + 3) * A.nblk + blockIdx.x] = nb;
    }
}

// Report (block 0), params += x_e and the pose step unless anything is non-finite.
__global__ void __launch_bounds__(kJThreads) jpcg_finish_kernel(JArgs J, misslam_report *rep,
                                                                float *__restrict__ params, float *pose_dev) {
    const PcgArgs &A = J.A;
    __shared__ double red[16][kJThreads / kWave];
    double nb1[1];
    jgather<1>(J, {A.iters}, {3}, nb1, red);
    const double nbad = nb1[0];
    const int total = A.m * 12;
    const int t = blockIdx.x * kJThreads + threadIdx.x;
    if (params && nbad == 0.0 && t < total) params[t] += A.x[t];
    if (blockIdx.x != 0) return;
    int done = 0;
    for (int q = 0; q < A.iters; ++q) done += A.done[q];
    for (int q = 0; q <= done; ++q) {
        double rr[1];
        jgather<1>(J, {q}, {1}, rr, red);
        if (threadIdx.x == 0 && q <= MISSLAM_MAX_PCG) rep->pcg_resid[q] = sqrt(rr[0]);
    }
    if (threadIdx.x == 0) {
        rep->pcg_iters_done = done;
        int f = rep->flags;
        if (A.status[A.iters] & 2) f |= MISSLAM_FLAG_PCG_BREAKDOWN;
        if (nbad != 0.0) f |= MISSLAM_FLAG_NONFINITE;
        rep->flags = f;
        if (nbad == 0.0) {
            const double *xp = J.pst + (size_t)A.iters * kPst + 24;
            double E[9], R[9], T[3];
            so3_exp_d(xp, E);
            for (int u = 0; u < 9; ++u) R[u] = pose_dev[u];
            for (int u = 0; u < 3; ++u) T[u] = pose_dev[9 + u];
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c)
                    pose_dev[3 * r + c] =
                        (float)((E[3 * r] * R[c] + E[3 * r + 1] * R[3 + c]) + E[3 * r + 2] * R[6 + c]);
                pose_dev[9 + r] = (float)(((E[3 * r] * T[0] + E[3 * r + 1] * T[1]) + E[3 * r + 2] * T[2]) + xp[3 + r]);
            }
        }
    }
}

// After the one-launch joint solve: params += delta and the pose step (stored by its first workgroup at
// pst), unless the step's report carries a non-finite value or a timeout of any workgroup.
__global__ void __launch_bounds__(256) joint_commit_kernel(float *__restrict__ params, const float *__restrict__ dx,
                                                           int n, const misslam_report *rep, float *pose_dev,
                                                           const double *xp) {
    if (rep->flags & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (params && i < n) params[i] += dx[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double E[9], R[9], T[3];
        so3_exp_d(xp, E);
        for (int u = 0; u < 9; ++u) R[u] = pose_dev[u];
        for (int u = 0; u < 3; ++u) T[u] = pose_dev[9 + u];
        for (int rr = 0; rr < 3; ++rr) {
            for (int c = 0; c < 3; ++c)
                pose_dev[3 * rr + c] = (float)((E[3 * rr] * R[c] + E[3 * rr + 1] * R[3 + c]) + E[3 * rr + 2] * R[6 + c]);
            pose_dev[9 + rr] = (float)(((E[3 * rr] * T[0] + E[3 * rr + 1] * T[1]) + E[3 * rr + 2] * T[2]) + xp[3 + rr]);
        }
    }
}

hipError_t launch_joint_pcg(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                            float lambda, int iters, float *delta, const PcgScratch &s, const JointScratch &js,
                            misslam_report *rep, float *params, float *pose_dev, hipStream_t st, bool kernels,
                            unsigned spin) {
    JArgs J;
    PcgArgs &A = J.A;
    A.row_ptr = g.row_ptr;
    A.col_idx = g.col_idx;
    A.blocks = blocks;
    A.minv = minv;
    A.g = gvec;
    A.lambda = lambda;
    A.m = m;
    A.nblk = (m + kJRows - 1) / kJRows;
    A.iters = iters;
    A.cap = g.bsr_cap;
    A.x = delta;
    A.r = s.r;
    A.z = s.z;
    A.p = s.p;
    A.q = s.q;
    A.part = nullptr;
    A.status = s.status;
    A.done = s.status + (iters + 2);
    J.B = js.B;
    J.sys = js.sys;
    J.jpart = js.jpart;
    J.pst = js.pst;
    if (!kernels && js.jbar) {   // one launch when every workgroup fits on the device at once
        PcgArgs P = A;
        P.part = s.part;
        if (spin > 0) P.spin = spin;
        JointExtra jx;
        jx.B = js.B;
        jx.sys = js.sys;
        jx.xp_out = J.pst + (size_t)iters * kPst + 24;
        bool used = false;
        hipError_t e = launch_joint_pcg_persistent(P, jx, js.jbar, joint_sync_words(m), rep, st, &used);
        if (e != hipSuccess) return e;
        if (used) {
            hipLaunchKernelGGL(joint_commit_kernel, dim3((12 * m + 255) / 256), dim3(256), 0, st, params, delta,
                               12 * m, rep, pose_dev, jx.xp_out);
            return hipGetLastError();
        }
    }
    const dim3 grid(A.nblk), blk(kJThreads);
    hipLaunchKernelGGL(jpcg_init_kernel, grid, blk, 0, st, J);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(jpcg_dir_kernel, grid, blk, 0, st, J, it);
        hipLaunchKernelGGL(jpcg_step_kernel, grid, blk, 0, st, J, it);
    }
    hipLaunchKernelGGL(jpcg_finish_kernel, dim3((12 * m + kJThreads - 1) / kJThreads), blk, 0, st, J, rep, params,
                       pose_dev);
    return hipGetLastError();
}

}  // namespace msl
