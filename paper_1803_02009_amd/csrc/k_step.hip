// Per-iteration kernels of the Gauss-Newton registration (Sec. II-E, II-F):
// the ED warp (Eq.(1)), projective association with the Eq.(7) gates and the
// point-to-plane residual (Eq.(8)), and the row-wise assembly of the normal
// equations with the rotation (Eq.(5)) and regularisation (Eq.(6)) terms.
#include "frame.h"

namespace msl {

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- standalone warp

template <int K>
__global__ void __launch_bounds__(256) warp_kernel(PointsView pts, NodesView nd, const int32_t *__restrict__ idx,
                                                   const float *__restrict__ w, Pose pose, int has_pose,
                                                   float *__restrict__ out_pos, float *__restrict__ out_nrm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pts.n) return;
    float x, y, z;
    ed_blend<K>(pts.px[i], pts.py[i], pts.pz[i], idx, w, pts.n, i, nd, x, y, z);
    if (has_pose) apply_pose(pose, x, y, z);
    out_pos[i] = x;
    out_pos[pts.n + i] = y;
    out_pos[2 * pts.n + i] = z;
    if (out_nrm) {
        float a, b, c;
        ed_blend_normal<K>(pts.nx[i], pts.ny[i], pts.nz[i], idx, w, pts.n, i, nd, a, b, c);
        if (has_pose) rotate(pose, a, b, c);
        normalize3(a, b, c);
        out_nrm[i] = a;
        out_nrm[pts.n + i] = b;
        out_nrm[2 * pts.n + i] = c;
    }
}

hipError_t launch_warp(const PointsView &pts, const NodesView &nd, const GraphView &g, const Pose *pose,
                       float *out_pos, float *out_nrm, hipStream_t st) {
    if (pts.n == 0) return hipSuccess;
    Pose P{};
    const int hp = pose != nullptr;
    if (hp) P = *pose;
    const dim3 grid(nblk(pts.n, 256)), blk(256);
    switch (g.k) {
#define MSL_WARP_CASE(KK)                                                                                   \
    case KK:                                                                                                \
        hipLaunchKernelGGL((warp_kernel<KK>), grid, blk, 0, st, pts, nd, g.knn_idx, g.knn_w, P, hp, out_pos, \
                           out_nrm);                                                                        \
        break;
        MSL_WARP_CASE(1) MSL_WARP_CASE(2) MSL_WARP_CASE(3) MSL_WARP_CASE(4)
        MSL_WARP_CASE(5) MSL_WARP_CASE(6) MSL_WARP_CASE(7) MSL_WARP_CASE(8)
#undef MSL_WARP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- point pass: warp + association

constexpr int kPtBlock = 256;

// One thread per model point: warps point and normal into the camera, finds
// the matched pixel, stores (n', r) with n' = R^T N for the assembly, and leaves
// per-block float64 sums (r^2, count, |r|) for the energy report.
template <int K>
__global__ void __launch_bounds__(kPtBlock) point_pass_kernel(StepArgs a, StepScratch s) {
    __shared__ double red[kPtBlock];
    const int64_t n = a.pts.n;
    const int64_t i = (int64_t)blockIdx.x * kPtBlock + threadIdx.x;
    double r2 = 0.0, cnt = 0.0, ra = 0.0;
    if (i < n) {
        float x, y, z, nx, ny, nz;
        ed_blend<K>(a.pts.px[i], a.pts.py[i], a.pts.pz[i], a.g.knn_idx, a.g.knn_w, n, i, a.nd, x, y, z);
        apply_pose(a.pose, x, y, z);
        ed_blend_normal<K>(a.pts.nx[i], a.pts.ny[i], a.pts.nz[i], a.g.knn_idx, a.g.knn_w, n, i, a.nd, nx, ny, nz);
        rotate(a.pose, nx, ny, nz);
        normalize3(nx, ny, nz);
        const Match mt = associate(x, y, z, nx, ny, nz, a.nmap, a.cam, a.eps_d, a.cos_eps_n);
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, rr = 0.f;
        if (mt.pix >= 0) {
            const float *R = a.pose.R;
            // n' = R^T N
            p0 = fmaf(R[6], mt.Nz, fmaf(R[3], mt.Ny, R[0] * mt.Nx));
            p1 = fmaf(R[7], mt.Nz, fmaf(R[4], mt.Ny, R[1] * mt.Nx));
            p2 = fmaf(R[8], mt.Nz, fmaf(R[5], mt.Ny, R[2] * mt.Nx));
            rr = mt.r;
            r2 = (double)rr * (double)rr;
            cnt = 1.0;
            ra = fabs((double)rr);
        }
        s.nr[i] = make_float4(p0, p1, p2, rr);
        s.corr[i] = mt.pix;
        if (a.corr_out) a.corr_out[i] = mt.pix;
    }
    const double t0 = block_sum<kPtBlock>(r2, red);
    const double t1 = block_sum<kPtBlock>(cnt, red);
    const double t2 = block_sum<kPtBlock>(ra, red);
    if (threadIdx.x == 0) {
        s.pt_part[3 * blockIdx.x + 0] = t0;
        s.pt_part[3 * blockIdx.x + 1] = t1;
        s.pt_part[3 * blockIdx.x + 2] = t2;
    }
}

// ---------------------------------------------------------------- row assembly

// Unique entries of the data-term statistic of one node pair (j, l):
//   S[c, c', a, a'] = sum_p w_pj w_pl u_c u_c' n'_a n'_a',  u = (v_p - g_j, 1), n' = R^T N_p
// symmetric in (c, c') and in (a, a'): 10 x 6 = 60 values.  The 12x12 block is
//   H_jl[(c,a),(c',a')] = S[c,c',a,a'] + delta_c' S[c,3,a,a'],  delta = (g_j - g_l, 0)
// because the second factor of the data Jacobian is (v_p - g_l, 1) = u + delta.
__constant__ int kPairC0[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__constant__ int kPairC1[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
__constant__ int kPairA0[6] = {0, 0, 0, 1, 1, 2};
__constant__ int kPairA1[6] = {0, 1, 2, 1, 2, 2};

__device__ __forceinline__ int pc_index(int c, int d) {  // c, d in 0..3
    const int lo = c < d ? c : d, hi = c < d ? d : c;
    // rows of the upper triangle: lo=0 -> 0..3, lo=1 -> 4..6, lo=2 -> 7..8, lo=3 -> 9
    const int start[4] = {0, 4, 7, 9};
    return start[lo] + (hi - lo);
}
__device__ __forceinline__ int na_index(int a, int b) {  // a, b in 0..2
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int start[3] = {0, 3, 5};
    return start[lo] + (hi - lo);
}

constexpr int kAsmThreads = 256;
constexpr int kAsmWaves = kAsmThreads / kWave;
constexpr int kBatch = 64;

template <int K>
struct AsmShared {
    float accS[kAsmWaves][MISSLAM_MAX_ROW][64];
    float Pc[kAsmWaves][kBatch][10];
    float Na[kAsmWaves][kBatch][6];
    float4 W[kAsmWaves][kBatch][(K + 3) / 4];
    uint32_t key[kAsmWaves][kBatch][2];
    float gw[kAsmWaves][12];
    int cols[MISSLAM_MAX_ROW];
    float rg[MISSLAM_MAX_ROW][9];    // per neighbour slot: e = g_l - g_j, r_jl, r_lj
    float EE[10];                    // sum over neighbours of e^_c e^_c', e^ = (e, 1)
    float Jr[6][9];                  // rotation-term Jacobian of node j
    float rr[6];
    float xj[12];
    double Hd[12][12];               // damped diagonal block for the preconditioner
    double Li[12][12];
    double red[kAsmThreads];
};

// Registers of one list entry between its global loads and its LDS staging.
template <int K>
struct EntryRegs {
    int q[K];
    float wq[K];
    float4 nr;
    float vx, vy, vz;
    uint32_t k0, k1;
};

template <int K>
__device__ __forceinline__ void entry_load(const StepArgs &a, const StepScratch &s, int64_t n, int le,
                                           EntryRegs<K> &r) {
    const int p = a.g.list_pts[le];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        r.q[t] = a.g.knn_idx[(int64_t)t * n + p];
        r.wq[t] = a.g.knn_w[(int64_t)t * n + p];
    }
    r.nr = s.nr[p];
    r.vx = a.pts.px[p];
    r.vy = a.pts.py[p];
    r.vz = a.pts.pz[p];
    r.k0 = a.g.list_key[2 * (size_t)le];
    r.k1 = a.g.list_key[2 * (size_t)le + 1];
}

// One workgroup per node row j (rows spread so each XCD owns a contiguous band).
// Four waves split the row's point list and run independently: each stages 64
// list entries at a time (lane = entry) while the next 64 are already being
// fetched, then accumulates the 60 statistic entries (lane = entry of the
// statistic) for the k node pairs of each run of equal kNN sets.  Then the
// node terms (Eqs.(5)-(6)) are added, the row's blocks and gradient are
// written, and the damped diagonal block is inverted for the block-Jacobi
// preconditioner.  Fixed summation order throughout: bitwise reproducible.
template <int K>
__global__ void __launch_bounds__(kAsmThreads) assemble_rows_kernel(StepArgs a, StepScratch s) {
    __shared__ AsmShared<K> sh;
    const int m = a.nd.m;
    const int per = (int)((m + 7) / 8);
    const int j = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (j >= m) return;
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    const int64_t n = a.pts.n;

    // an overflowed pattern (flagged by the graph build) is clamped to the capacity
    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap);
    const int re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    const int nslots = min(re - rb, MISSLAM_MAX_ROW);
    for (int t = tid; t < (re - rb - nslots) * 144; t += kAsmThreads)
        a.blocks[(size_t)(rb + nslots) * 144 + t] = 0.f;   // blocks of a row longer than MISSLAM_MAX_ROW
    for (int t = tid; t < nslots; t += kAsmThreads) sh.cols[t] = a.g.col_idx[rb + t];
    for (int t = lane; t < MISSLAM_MAX_ROW * 64; t += kWave) (&sh.accS[wave][0][0])[t] = 0.f;

    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    const int lb = a.g.list_ptr[j];
    const int cnt = min(a.g.list_ptr[j + 1] - lb, MISSLAM_MAX_LIST);
    const int quota = (cnt + kAsmWaves - 1) / kAsmWaves;
    const int my0 = min(cnt, wave * quota), my1 = min(cnt, my0 + quota);
    const int nbatch = (my1 - my0 + kBatch - 1) / kBatch;

    const int e = lane;                      // statistic entry owned in phase 2 (e < 60)
    const int pci = e < 60 ? e / 6 : 0, nai = e < 60 ? e % 6 : 0;
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.f;
    uint32_t cur0 = 0xFFFFFFFFu, cur1 = 0xFFFFFFFFu;
    float gacc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) gacc[q] = 0.f;

    EntryRegs<K> nxt;
    if (nbatch > 0 && lane < min(kBatch, my1 - my0)) entry_load<K>(a, s, n, lb + my0 + lane, nxt);
    for (int bt = 0; bt < nbatch; ++bt) {
        const int e0 = my0 + bt * kBatch;
        const int nb = min(kBatch, my1 - e0);
        EntryRegs<K> cu = nxt;
        // prefetch the next batch while this one is staged and accumulated
        if (bt + 1 < nbatch && lane < min(kBatch, my1 - e0 - kBatch))
            entry_load<K>(a, s, n, lb + e0 + kBatch + lane, nxt);
        // ---- phase 1: lane = list entry
        bool start = false;
        if (lane < nb) {
            float wj = 0.f;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (cu.q[t] == j) wj = cu.wq[t];
            // weights in node-index order, matching the entry's row positions
#pragma unroll
            for (int u = 1; u < K; ++u)
#pragma unroll
                for (int v = u; v > 0; --v)
                    if (cu.q[v] < cu.q[v - 1]) {
                        const int ti = cu.q[v];
                        cu.q[v] = cu.q[v - 1];
                        cu.q[v - 1] = ti;
                        const float tw = cu.wq[v];
                        cu.wq[v] = cu.wq[v - 1];
                        cu.wq[v - 1] = tw;
                    }
            const float uu[4] = {cu.vx - gjx, cu.vy - gjy, cu.vz - gjz, 1.f};
            const float nn[3] = {cu.nr.x, cu.nr.y, cu.nr.z};
#pragma unroll
            for (int t = 0; t < 10; ++t) sh.Pc[wave][lane][t] = uu[kPairC0[t]] * uu[kPairC1[t]];
#pragma unroll
            for (int t = 0; t < 6; ++t) sh.Na[wave][lane][t] = nn[kPairA0[t]] * nn[kPairA1[t]];
            float wv[4 * ((K + 3) / 4)];
#pragma unroll
            for (int t = 0; t < 4 * ((K + 3) / 4); ++t) wv[t] = t < K ? wj * cu.wq[t] : 0.f;
#pragma unroll
            for (int t = 0; t < (K + 3) / 4; ++t)
                sh.W[wave][lane][t] = make_float4(wv[4 * t], wv[4 * t + 1], wv[4 * t + 2], wv[4 * t + 3]);
            sh.key[wave][lane][0] = cu.k0;
            sh.key[wave][lane][1] = cu.k1;
            const float wr = wj * cu.nr.w;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float f = wr * uu[c];
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) gacc[3 * c + aa] = fmaf(f, nn[aa], gacc[3 * c + aa]);
            }
        }
        // run starts: an entry whose kNN set differs from the previous entry's
        {
            const uint32_t p0 = __shfl_up(cu.k0, 1, 64), p1 = __shfl_up(cu.k1, 1, 64);
            const uint32_t q0 = lane == 0 ? cur0 : p0, q1 = lane == 0 ? cur1 : p1;
            start = lane < nb && (cu.k0 != q0 || cu.k1 != q1);
        }
        uint64_t starts = __ballot(start);
        wave_sync();
        // ---- phase 2: lane = statistic entry, one run of equal sets at a time
        int t = 0;
        while (t < nb) {
            if (starts & (1ull << t)) {
                if (cur0 != 0xFFFFFFFFu && e < 60) {
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        const uint32_t slot = q < 4 ? (cur0 >> (8 * q)) & 0xFF : (cur1 >> (8 * (q - 4))) & 0xFF;
                        if (slot < (uint32_t)nslots) sh.accS[wave][slot][e] += acc[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < K; ++q) acc[q] = 0.f;
                cur0 = sh.key[wave][t][0];
                cur1 = sh.key[wave][t][1];
            }
            // end of this run: next start after t, or the batch end
            const uint64_t later = t + 1 < 64 ? (starts >> (t + 1)) : 0ull;
            const int t1 = later ? min(nb, t + 1 + __builtin_ctzll(later)) : nb;
            int u = t;
            for (; u + 1 < t1; u += 2) {
                const float m0 = sh.Pc[wave][u][pci] * sh.Na[wave][u][nai];
                const float m1 = sh.Pc[wave][u + 1][pci] * sh.Na[wave][u + 1][nai];
#pragma unroll
                for (int g4 = 0; g4 < (K + 3) / 4; ++g4) {
                    const float4 w0 = sh.W[wave][u][g4], w1 = sh.W[wave][u + 1][g4];
                    const float w0v[4] = {w0.x, w0.y, w0.z, w0.w}, w1v[4] = {w1.x, w1.y, w1.z, w1.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (4 * g4 + q < K) acc[4 * g4 + q] = fmaf(w1v[q], m1, fmaf(w0v[q], m0, acc[4 * g4 + q]));
                }
            }
            if (u < t1) {
                const float m0 = sh.Pc[wave][u][pci] * sh.Na[wave][u][nai];
#pragma unroll
                for (int g4 = 0; g4 < (K + 3) / 4; ++g4) {
                    const float4 w0 = sh.W[wave][u][g4];
                    const float w0v[4] = {w0.x, w0.y, w0.z, w0.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (4 * g4 + q < K) acc[4 * g4 + q] = fmaf(w0v[q], m0, acc[4 * g4 + q]);
                }
            }
            t = t1;
        }
        wave_sync();
    }
    if (cur0 != 0xFFFFFFFFu && e < 60) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const uint32_t slot = q < 4 ? (cur0 >> (8 * q)) & 0xFF : (cur1 >> (8 * (q - 4))) & 0xFF;
            if (slot < (uint32_t)nslots) sh.accS[wave][slot][e] += acc[q];
        }
    }
    // wave reduction of the data gradient (fixed butterfly order)
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        float v = gacc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        gacc[q] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 12; ++q) sh.gw[wave][q] = gacc[q];
    }
    // ---- node-level terms: parameters, regulariser residuals, rotation Jacobian
    if (tid < 12) sh.xj[tid] = a.nd.x[(size_t)j * 12 + tid];
    __syncthreads();
    for (int t = tid; t < nslots * 64; t += kAsmThreads) {
        const int sl = t / 64, en = t % 64;
        if (en < 60) {
            const float v = sh.accS[0][sl][en] + sh.accS[1][sl][en] + sh.accS[2][sl][en] + sh.accS[3][sl][en];
            sh.accS[0][sl][en] = v;
        }
    }
    double e_reg = 0.0;
    if (tid < nslots) {
        const int l = sh.cols[tid];
        float ex = 0.f, ey = 0.f, ez = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f;
        if (l != j) {
            const float glx = a.nd.gx[l], gly = a.nd.gy[l], glz = a.nd.gz[l];
            const float *xl = a.nd.x + (size_t)l * 12;
            const float *xj = sh.xj;
            ex = glx - gjx;
            ey = gly - gjy;
            ez = glz - gjz;
            // r_jl = A_j e + g_j + t_j - g_l - t_l   (edge j -> l)
            r0 = fmaf(xj[6], ez, fmaf(xj[3], ey, xj[0] * ex)) + gjx + xj[9] - glx - xl[9];
            r1 = fmaf(xj[7], ez, fmaf(xj[4], ey, xj[1] * ex)) + gjy + xj[10] - gly - xl[10];
            r2 = fmaf(xj[8], ez, fmaf(xj[5], ey, xj[2] * ex)) + gjz + xj[11] - glz - xl[11];
            // r_lj = A_l (-e) + g_l + t_l - g_j - t_j   (edge l -> j)
            q0 = -fmaf(xl[6], ez, fmaf(xl[3], ey, xl[0] * ex)) + glx + xl[9] - gjx - xj[9];
            q1 = -fmaf(xl[7], ez, fmaf(xl[4], ey, xl[1] * ex)) + gly + xl[10] - gjy - xj[10];
            q2 = -fmaf(xl[8], ez, fmaf(xl[5], ey, xl[2] * ex)) + glz + xl[11] - gjz - xj[11];
            e_reg = ((double)r0 * r0 + (double)r1 * r1) + (double)r2 * r2;
        }
        float *rg = sh.rg[tid];
        rg[0] = ex; rg[1] = ey; rg[2] = ez;
        rg[3] = r0; rg[4] = r1; rg[5] = r2;
        rg[6] = q0; rg[7] = q1; rg[8] = q2;
    }
    if (tid == 0) {
        const float *x = sh.xj;
        const float *c[3] = {x, x + 3, x + 6};
        auto dot = [](const float *u, const float *v) { return fmaf(u[2], v[2], fmaf(u[1], v[1], u[0] * v[0])); };
        sh.rr[0] = dot(c[0], c[1]);
        sh.rr[1] = dot(c[0], c[2]);
        sh.rr[2] = dot(c[1], c[2]);
        sh.rr[3] = dot(c[0], c[0]) - 1.f;
        sh.rr[4] = dot(c[1], c[1]) - 1.f;
        sh.rr[5] = dot(c[2], c[2]) - 1.f;
        for (int q = 0; q < 6; ++q)
            for (int t = 0; t < 9; ++t) sh.Jr[q][t] = 0.f;
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        for (int q = 0; q < 3; ++q) {
            for (int t = 0; t < 3; ++t) {
                sh.Jr[q][3 * pa[q] + t] = c[pb[q]][t];
                sh.Jr[q][3 * pb[q] + t] = c[pa[q]][t];
            }
        }
        for (int q = 0; q < 3; ++q)
            for (int t = 0; t < 3; ++t) sh.Jr[3 + q][3 * q + t] = 2.f * c[q][t];
    }
    const double ereg_tot = block_sum<kAsmThreads>(e_reg, sh.red);   // also a barrier
    if (tid < 10) {
        float sacc = 0.f;
        for (int t = 0; t < nslots; ++t) {
            if (sh.cols[t] == j) continue;
            const float eh[4] = {sh.rg[t][0], sh.rg[t][1], sh.rg[t][2], 1.f};
            sacc = fmaf(eh[kPairC0[tid]], eh[kPairC1[tid]], sacc);
        }
        sh.EE[tid] = sacc;
    }
    __syncthreads();
    if (tid == 0) {
        double erot = 0.0;
        for (int q = 0; q < 6; ++q) erot += (double)sh.rr[q] * sh.rr[q];
        s.node_part[2 * j + 0] = erot;
        s.node_part[2 * j + 1] = ereg_tot;
    }
    int deg = 0;
    for (int q = 0; q < nslots; ++q) deg += sh.cols[q] != j;
    if (tid < 144) sh.Hd[tid / 12][tid % 12] = tid / 12 == tid % 12 ? (double)a.lambda : 0.0;
    __syncthreads();
    const float wd = a.w_data, wreg = a.w_reg, wrot = a.w_rot;
    // ---- expand statistics into 12x12 blocks and add the regularisers
    float *outb = a.blocks + (size_t)rb * 144;
    const int nent = nslots * 144;
    for (int t = tid; t < nent; t += kAsmThreads) {
        const int sl = t / 144, en = t % 144;
        const int R = en / 12, C = en % 12;
        const int c = R / 3, aa = R % 3, c2 = C / 3, a2 = C % 3;
        const int l = sh.cols[sl];
        const float *S = sh.accS[0][sl];
        const int ni = na_index(aa, a2);
        float h = S[pc_index(c, c2) * 6 + ni];
        float reg = 0.f;
        if (l != j) {
            // delta = g_j - g_l = -e
            const float dl = c2 < 3 ? -sh.rg[sl][c2] : 0.f;
            h = fmaf(dl, S[pc_index(c, 3) * 6 + ni], h);
            if (aa == a2) {
                const float eh_c = c < 3 ? sh.rg[sl][c] : 1.f;
                const float fh_c2 = c2 < 3 ? -sh.rg[sl][c2] : 1.f;
                if (c2 == 3) reg -= eh_c;      // edge j -> l
                if (c == 3) reg -= fh_c2;      // edge l -> j
            }
            h = fmaf(wreg, reg, wd * h);
        } else {
            h = wd * h;
            if (aa == a2) {
                reg = sh.EE[pc_index(c, c2)];
                if (c == 3 && c2 == 3) reg += (float)deg;
            }
            float rot = 0.f;
            if (c < 3 && c2 < 3) {
#pragma unroll
                for (int q = 0; q < 6; ++q) rot = fmaf(sh.Jr[q][R], sh.Jr[q][C], rot);
            }
            h = fmaf(wrot, rot, fmaf(wreg, reg, h));
            sh.Hd[R][C] = (double)h + (R == C ? (double)a.lambda : 0.0);
        }
        outb[(size_t)sl * 144 + en] = h;
    }
    if (tid < 12) {
        const int c = tid / 3, aa = tid % 3;
        const float gd = sh.gw[0][tid] + sh.gw[1][tid] + sh.gw[2][tid] + sh.gw[3][tid];
        float reg = 0.f;
        for (int t = 0; t < nslots; ++t) {
            if (sh.cols[t] == j) continue;
            const float eh_c = c < 3 ? sh.rg[t][c] : 1.f;
            reg = fmaf(eh_c, sh.rg[t][3 + aa], reg);
            if (c == 3) reg -= sh.rg[t][6 + aa];
        }
        float rot = 0.f;
        if (c < 3) {
#pragma unroll
            for (int q = 0; q < 6; ++q) rot = fmaf(sh.Jr[q][tid], sh.rr[q], rot);
        }
        a.gvec[(size_t)j * 12 + tid] = fmaf(wrot, rot, fmaf(wreg, reg, wd * gd));
    }
    // ---- block-Jacobi preconditioner of this row: (H_jj + lambda I)^-1 in float64, by wave 0
    if (a.minv) {
        __syncthreads();
        if (wave == 0) {
            const bool ok = chol_inverse_wave(sh.Hd, sh.Li, a.minv + (size_t)j * 144);
            if (!ok && lane == 0) atomicOr(a.flags, MISSLAM_FLAG_NONSPD_BLOCK);
        }
    }
}

// ---------------------------------------------------------------- energy report

__global__ void __launch_bounds__(256) energy_report_kernel(const double *__restrict__ pt_part, int npb,
                                                            const double *__restrict__ node_part, int m,
                                                            misslam_report *rep, float reject_thr) {
    __shared__ double red[256];
    double a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0;
    for (int t = threadIdx.x; t < npb; t += 256) {
        a0 += pt_part[3 * t];
        a1 += pt_part[3 * t + 1];
        a2 += pt_part[3 * t + 2];
    }
    for (int t = threadIdx.x; t < m; t += 256) {
        b0 += node_part[2 * t];
        b1 += node_part[2 * t + 1];
    }
    const double ed = block_sum<256>(a0, red);
    const double nv = block_sum<256>(a1, red);
    const double sa = block_sum<256>(a2, red);
    const double er = block_sum<256>(b0, red);
    const double eg = block_sum<256>(b1, red);
    if (threadIdx.x == 0) {
        rep->e_data = ed;
        rep->e_rot = er;
        rep->e_reg = eg;
        rep->n_valid = (int32_t)nv;
        int flags = 0;
        if (!isfinite(ed) || !isfinite(er) || !isfinite(eg)) flags |= MISSLAM_FLAG_NONFINITE;
        if (reject_thr > 0.f && nv > 0 && sa / nv > (double)reject_thr) flags |= MISSLAM_FLAG_FRAME_REJECT;
        rep->flags |= flags;
    }
}

hipError_t launch_point_pass(const StepArgs &a, const StepScratch &s, hipStream_t st) {
    const int64_t n = a.pts.n;
    const unsigned ptb = nblk(n > 0 ? n : 1, kPtBlock);
    switch (a.g.k) {
#define MSL_PP_CASE(KK)                                                                                     \
    case KK: hipLaunchKernelGGL((point_pass_kernel<KK>), dim3(ptb), dim3(kPtBlock), 0, st, a, s); break;
        MSL_PP_CASE(1) MSL_PP_CASE(2) MSL_PP_CASE(3) MSL_PP_CASE(4)
        MSL_PP_CASE(5) MSL_PP_CASE(6) MSL_PP_CASE(7) MSL_PP_CASE(8)
#undef MSL_PP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const StepArgs &a, const StepScratch &s, hipStream_t st) {
    const int m = a.nd.m;
    const unsigned rows = 8 * (unsigned)((m + 7) / 8);
    switch (a.g.k) {
#define MSL_AS_CASE(KK)                                                                                     \
    case KK: hipLaunchKernelGGL((assemble_rows_kernel<KK>), dim3(rows), dim3(kAsmThreads), 0, st, a, s); break;
        MSL_AS_CASE(1) MSL_AS_CASE(2) MSL_AS_CASE(3) MSL_AS_CASE(4)
        MSL_AS_CASE(5) MSL_AS_CASE(6) MSL_AS_CASE(7) MSL_AS_CASE(8)
#undef MSL_AS_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_energy_report(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                                hipStream_t st) {
    const int npb = (int)nblk(n > 0 ? n : 1, kPtBlock);
    hipLaunchKernelGGL(energy_report_kernel, dim3(1), dim3(256), 0, st, s.pt_part, npb, s.node_part, m, rep,
                       reject_thr);
    return hipGetLastError();
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace msl
