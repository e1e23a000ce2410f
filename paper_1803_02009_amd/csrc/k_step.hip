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
// Joint pose form (JOINT): the pose comes from the device, and each point also
// writes the pose columns Jp = (v~ x N, N) of its data row and adds Jp Jp^T and
// Jp r to per-block float64 partials (27 values, fixed reduction order).
template <int K, bool JOINT = false>
__device__ __forceinline__ void point_pass_body(const StepArgs &a, const StepScratch &s, int64_t blk) {
    __shared__ double red[3 * kPtBlock];
    const int64_t n = a.pts.n;
    const int64_t i = blk * kPtBlock + threadIdx.x;
    const Pose P = JOINT ? step_pose(a) : a.pose;
    double r2 = 0.0, cnt = 0.0, ra = 0.0;
    float jp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, rres = 0.f;
    if (i < n) {
        float x, y, z, nx, ny, nz;
        ed_blend<K>(a.pts.px[i], a.pts.py[i], a.pts.pz[i], a.g.knn_idx, a.g.knn_w, n, i, a.nd, x, y, z);
        apply_pose(P, x, y, z);
        ed_blend_normal<K>(a.pts.nx[i], a.pts.ny[i], a.pts.nz[i], a.g.knn_idx, a.g.knn_w, n, i, a.nd, nx, ny, nz);
        rotate(P, nx, ny, nz);
        normalize3(nx, ny, nz);
        const Match mt = a.corr_in ? match_fixed(x, y, z, a.corr_in[i], a.nmap, a.cam)
                                   : associate(x, y, z, nx, ny, nz, a.nmap, a.cam, a.eps_d, a.cos_eps_n);
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, rr = 0.f;
        if (JOINT && mt.pix >= 0) {
            jp[0] = fmaf(y, mt.Nz, -z * mt.Ny);
            jp[1] = fmaf(z, mt.Nx, -x * mt.Nz);
            jp[2] = fmaf(x, mt.Ny, -y * mt.Nx);
            jp[3] = mt.Nx;
            jp[4] = mt.Ny;
            jp[5] = mt.Nz;
            rres = mt.r;
        }
        if (JOINT) {
            s.jp[2 * i] = make_float4(jp[0], jp[1], jp[2], jp[3]);
            s.jp[2 * i + 1] = make_float4(jp[4], jp[5], 0.f, 0.f);
        }
        if (mt.pix >= 0) {
            const float *R = P.R;
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
    double tv[3] = {r2, cnt, ra};
    block_sums_tree<kPtBlock>(tv, red);
    const double t0 = tv[0], t1 = tv[1], t2 = tv[2];
    if (threadIdx.x == 0) {
        s.pt_part[3 * blk + 0] = t0;
        s.pt_part[3 * blk + 1] = t1;
        s.pt_part[3 * blk + 2] = t2;
    }
    if (JOINT) {
        // 27 sums at once: wave butterflies, then the waves in order
        __shared__ double wred[kPtBlock / kWave][kPosePart];
        double v[kPosePart];
        int e = 0;
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int w = u; w < 6; ++w) v[e++] = (double)jp[u] * (double)jp[w];
#pragma unroll
        for (int u = 0; u < 6; ++u) v[e++] = (double)jp[u] * (double)rres;
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        wave_sums(v);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < kPosePart; ++q) wred[wave][q] = v[q];
        __syncthreads();
        if (threadIdx.x < kPosePart) {
            double t = wred[0][threadIdx.x];
#pragma unroll
            for (int w = 1; w < kPtBlock / kWave; ++w) t += wred[w][threadIdx.x];
            s.pose_part[(size_t)kPosePart * blk + threadIdx.x] = t;
        }
    }
}

template <int K>
__global__ void __launch_bounds__(kPtBlock) point_pass_kernel(StepArgs a, StepScratch s, KeyArgs kp, float *kp_data,
                                                             double *kp_energy, unsigned ptb) {
    if (blockIdx.x < ptb)
        point_pass_body<K>(a, s, blockIdx.x);
    else   // the key points, Eq.(9), one per thread
        kp_eval_body<K>(a, kp, kp_data, kp_energy, (int)(blockIdx.x - ptb) * kPtBlock + (int)threadIdx.x);
}

// ---------------------------------------------------------------- row assembly

// Unique entries of the data-term statistic of one node pair (j, l):
//   S[c, c', a, a'] = sum_p w_pj w_pl u_c u_c' n'_a n'_a',  u = (v_p - g_j, 1), n' = R^T N_p
// symmetric in (c, c') and in (a, a'): 10 x 6 = 60 values.  The 12x12 block is
//   H_jl[(c,a),(c',a')] = S[c,c',a,a'] + delta_c' S[c,3,a,a'],  delta = (g_j - g_l, 0)
// because the second factor of the data Jacobian is (v_p - g_l, 1) = u + delta.
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// pairs c <= c' of 0..3 (t = 0..9) and a <= a' of 0..2 (t = 0..5), as arithmetic so that unrolled
// loops fold them to constants
__device__ __forceinline__ constexpr int pair_c0(int t) { return t < 4 ? 0 : t < 7 ? 1 : t < 9 ? 2 : 3; }
__device__ __forceinline__ constexpr int pair_c1(int t) { return t < 4 ? t : t < 7 ? t - 3 : t < 9 ? t - 5 : 3; }
__device__ __forceinline__ constexpr int pair_a0(int t) { return t < 3 ? 0 : t < 5 ? 1 : 2; }
__device__ __forceinline__ constexpr int pair_a1(int t) { return t < 3 ? t : t < 5 ? t - 2 : 2; }

// (arithmetic, not a table: a table index becomes a memory load)
__device__ __forceinline__ int pc_index(int c, int d) {  // c, d in 0..3
    const int lo = c < d ? c : d, hi = c < d ? d : c;
    // rows of the upper triangle: lo=0 -> 0..3, lo=1 -> 4..6, lo=2 -> 7..8, lo=3 -> 9
    return 4 * lo - (lo * (lo - 1)) / 2 + (hi - lo);
}
__device__ __forceinline__ int na_index(int a, int b) {  // a, b in 0..2
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return 3 * lo - (lo * (lo - 1)) / 2 + (hi - lo);
}

constexpr int kBatch = 64;
// Statistic slots of a row, shared out among its W waves (one or two, the assembly tile): each wave has
// kAsmSlots / W of its own.  A row with more column slots than a wave holds accumulates on its first wave
// alone, over the slots of all waves.
constexpr int kAsmSlots = 36;
static_assert(kAsmSlots >= MISSLAM_MAX_ROW, "a row's slots must fit the statistic area");
// Staged entries per statistic row: the batch plus the four-entry read-ahead; 69 floats keep the rows of the
// staged products (read by lanes with different statistic entries) in distinct banks.
constexpr int kStage = kBatch + 5;

// LDS of the node-level part of a row: columns, regulariser residuals,
// rotation Jacobian and the data gradient.
struct RowNode {
    int cols[MISSLAM_MAX_ROW];
    float rg[MISSLAM_MAX_ROW][9];    // per neighbour slot: e = g_l - g_j, r_jl, r_lj
    float EE[10];                    // sum over neighbours of e^_c e^_c', e^ = (e, 1)
    float Jr[6][9];                  // rotation-term Jacobian of node j
    float rr[6];
    float xj[12];
    double gd[12];                   // data-term gradient of the row (unweighted)
};

// LDS used only once the row's data term is complete (it may share memory with the staging buffers): the
// damped diagonal block, inverted in place for the preconditioner, and a reduction area.
template <int NT>
struct RowFin {
    double Hd[12][12];
    double red[NT];
};

// One wave's staged batch: per entry its products, weights and kNN key.
template <int K>
struct AsmStage {
    float Pc[10][kStage];
    float Na[6][kStage];
    float4 W[kBatch + 4][(K + 3) / 4];
    uint32_t key[kBatch][2];
};

template <int K, int W>
struct AsmShared {
    float accS[kAsmSlots][60];   // statistic per slot; wave w's slots start at w kAsmSlots / W
    union {
        AsmStage<K> st[W];
        // wave w's data gradient (gw[w][0..11]), over its own staging once its batches are done
        double gw[W][sizeof(AsmStage<K>) / sizeof(double)];
        RowFin<kWave * W> fin;
    };
    RowNode rn;
};

// Node-level residuals of row j, computed before the data phase so that their
// loads overlap it: for each neighbour slot (thread tid < nslots) the edge
// vector and both Eq.(6) residuals, and (thread 0) the Eq.(5) residuals and
// Jacobian of node j; threads < 12 stage x_j.  Returns this thread's share of
// E_reg (summed in row_finalize).  The columns must already be in rn.cols.
__device__ __forceinline__ double row_prepare(const StepArgs &a, RowNode &rn, int j, int nslots, float gjx,
                                              float gjy, float gjz) {
    const int tid = threadIdx.x;
    const float *xj = a.nd.x + (size_t)j * 12;
    if (tid < 12) rn.xj[tid] = xj[tid];
    double e_reg = 0.0;
    if (tid < nslots) {
        const int l = a.g.col_idx[min(a.g.row_ptr[j], a.g.bsr_cap) + tid];
        float ex = 0.f, ey = 0.f, ez = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f;
        if (l != j) {
            const float glx = a.nd.gx[l], gly = a.nd.gy[l], glz = a.nd.gz[l];
            const float *xl = a.nd.x + (size_t)l * 12;
            ex = glx - gjx;
            ey = gly - gjy;
            ez = glz - gjz;
            reg_residual(xj, xl, ex, ey, ez, r0, r1, r2);      // edge j -> l
            reg_residual(xl, xj, -ex, -ey, -ez, q0, q1, q2);   // edge l -> j
            e_reg = ((double)r0 * r0 + (double)r1 * r1) + (double)r2 * r2;
        }
        float *rg = rn.rg[tid];
        rg[0] = ex; rg[1] = ey; rg[2] = ez;
        rg[3] = r0; rg[4] = r1; rg[5] = r2;
        rg[6] = q0; rg[7] = q1; rg[8] = q2;
    }
    if (tid == 0) {
        float x[12];
#pragma unroll
        for (int t = 0; t < 12; ++t) x[t] = xj[t];
        const float *c[3] = {x, x + 3, x + 6};
        auto dot = [](const float *u, const float *v) { return fmaf(u[2], v[2], fmaf(u[1], v[1], u[0] * v[0])); };
        rn.rr[0] = dot(c[0], c[1]);
        rn.rr[1] = dot(c[0], c[2]);
        rn.rr[2] = dot(c[1], c[2]);
        rn.rr[3] = unit_residual(c[0], 0);
        rn.rr[4] = unit_residual(c[1], 1);
        rn.rr[5] = unit_residual(c[2], 2);
        for (int q = 0; q < 6; ++q)
            for (int t = 0; t < 9; ++t) rn.Jr[q][t] = 0.f;
        const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
        for (int q = 0; q < 3; ++q) {
            for (int t = 0; t < 3; ++t) {
                rn.Jr[q][3 * pa[q] + t] = c[pb[q]][t];
                rn.Jr[q][3 * pb[q] + t] = c[pa[q]][t];
            }
        }
        for (int q = 0; q < 3; ++q)
            for (int t = 0; t < 3; ++t) rn.Jr[3 + q][3 * q + t] = 2.f * c[q][t];
    }
    return e_reg;
}

// Output of one row, shared by the float32 and the low-precision assembly:
// Eq.(6) regulariser blocks for both edge directions, the Eq.(5) rotation
// block, the gradient, the row's blocks (data term given by data(slot, R, C),
// already weighted by the point weights) and, when requested, the
// block-Jacobi inverse of the damped diagonal block.  rr_out, if set,
// receives the regulariser + rotation part of each block alone.  The
// node-level residuals come from row_prepare (e_reg: this thread's share); lamf is the damping.
template <int NT, class DataFn>
__device__ __forceinline__ void row_finalize(const StepArgs &a, const StepScratch &s, RowNode &rn, RowFin<NT> &fin,
                                             int j, int rb, int nslots, double e_reg, float lamf, DataFn data,
                                             float *rr_out) {
    static_assert(NT % kWave == 0, "whole waves");
    static_assert(MISSLAM_MAX_ROW <= kWave, "one lane per slot");
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    // the diagonal slot and the degree, by a ballot over the slots
    const uint64_t dmask = __ballot(lane < nslots && rn.cols[lane] == j);
    const int dsl = dmask ? (int)__builtin_ctzll(dmask) : -1;
    const int deg = nslots - __popcll(dmask);
    // the row's regulariser energy: its edges' terms added in slot order, as node_energy_kernel adds them, so
    // that the energy of a point in parameter space does not depend on which kernel evaluated it.  Loops over
    // the slots take kChunk slots at a time, their LDS reads issued together, and skip the diagonal slot.
    constexpr int kChunk = 8;
    if (tid < nslots) fin.red[tid] = e_reg;
    const double lam = (double)lamf;
    for (int t = tid; t < 144; t += NT) fin.Hd[t / 12][t % 12] = t / 12 == t % 12 ? lam : 0.0;
    if (tid < 10) {
        const int p0 = pair_c0(tid), p1 = pair_c1(tid);
        float sacc = 0.f;
        for (int t0 = 0; t0 < nslots; t0 += kChunk) {
            float eh0[kChunk], eh1[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int t = min(t0 + u, MISSLAM_MAX_ROW - 1);
                eh0[u] = p0 < 3 ? rn.rg[t][p0 < 3 ? p0 : 0] : 1.f;
                eh1[u] = p1 < 3 ? rn.rg[t][p1 < 3 ? p1 : 0] : 1.f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (t0 + u < nslots && !((dmask >> (t0 + u)) & 1)) sacc = fmaf(eh0[u], eh1[u], sacc);
        }
        rn.EE[tid] = sacc;
    }
    __syncthreads();
    if (tid == 0) {
        double ereg_tot = 0.0;
        for (int t0 = 0; t0 < nslots; t0 += kChunk) {
            double red[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) red[u] = fin.red[min(t0 + u, NT - 1)];
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (t0 + u < nslots && !((dmask >> (t0 + u)) & 1)) ereg_tot += red[u];
        }
        double erot = 0.0;
        for (int q = 0; q < 6; ++q) erot += (double)rn.rr[q] * rn.rr[q];
        s.node_part[2 * j + 0] = erot;
        s.node_part[2 * j + 1] = ereg_tot;
    }
    const float wd = a.w_data, wreg = a.w_reg, wrot = a.w_rot;
    float *outb = a.blocks + (size_t)rb * 144;
    // each thread owns entries en of every block of the row: its index arithmetic is done once, and the slots'
    // loads are independent (straight-line bodies, selects, no branches).  The 144 % NT entries left after the
    // full passes share their slots among NT / (144 % NT) threads each (slots part, part + share, ...), so no
    // wave runs a second pass over every slot alone.
    auto out_entry = [&](int en, int sl0, int sstep) {
        const int R = en / 12, C = en % 12;
        const int c = R / 3, aa = R % 3, c2 = C / 3, a2 = C % 3;
        const int ic = c < 3 ? c : 0, ic2 = c2 < 3 ? c2 : 0;
#pragma unroll 4
        for (int sl = sl0; sl < nslots; sl += sstep) {   // edges j -> l; the diagonal slot is written below
            const float hd = data(sl, R, C, true);
            const float rgc = rn.rg[sl][ic], rgc2 = rn.rg[sl][ic2];
            const float eh_c = c < 3 ? rgc : 1.f;
            const float fh_c2 = c2 < 3 ? -rgc2 : 1.f;
            const float r1 = c2 == 3 ? 0.f - eh_c : 0.f;   // edge j -> l
            const float r2 = c == 3 ? r1 - fh_c2 : r1;     // edge l -> j
            const float reg = aa == a2 ? r2 : 0.f;
            const float rr = fmaf(wrot, 0.f, wreg * reg);
            const float h = fmaf(wreg, reg, wd * hd);
            if (sl != dsl) {
                outb[(size_t)sl * 144 + en] = h;
                if (rr_out) rr_out[(size_t)(rb + sl) * 144 + en] = rr;
            }
        }
        if (dsl >= 0 && dsl % sstep == sl0) {   // the diagonal block: regulariser and rotation terms of node j
            const float hd = data(dsl, R, C, false);
            float reg = 0.f, rot = 0.f;
            if (aa == a2) {
                reg = rn.EE[pc_index(c, c2)];
                if (c == 3 && c2 == 3) reg += (float)deg;
            }
            if (c < 3 && c2 < 3) {
#pragma unroll
                for (int q = 0; q < 6; ++q) rot = fmaf(rn.Jr[q][R], rn.Jr[q][C], rot);
            }
            const float rr = fmaf(wrot, rot, wreg * reg);
            const float h = fmaf(wrot, rot, fmaf(wreg, reg, wd * hd));
            fin.Hd[R][C] = (double)h + (R == C ? lam : 0.0);
            outb[(size_t)dsl * 144 + en] = h;
            if (rr_out) rr_out[(size_t)(rb + dsl) * 144 + en] = rr;
        }
    };
    constexpr int kRem = 144 % NT, kFull = 144 - kRem;
    for (int en = tid; en < kFull; en += NT) out_entry(en, 0, 1);
    if constexpr (kRem > 0) {
        static_assert(NT % kRem == 0, "the remaining entries share whole groups of threads");
        out_entry(kFull + tid % kRem, tid / kRem, NT / kRem);
    }
    __syncthreads();
    // the block-Jacobi preconditioner of this row on wave 0 and the gradient on the last wave (with one wave,
    // one after the other)
    if (wave == 0) {
        // (H_jj + lambda I)^-1 in float64 on lanes 0-11
        if (a.minv) {
            const bool ok = gj_inverse_lanes(fin.Hd, a.minv + (size_t)j * 144);
            if (!ok && lane == 0) atomicOr(a.flags, MISSLAM_FLAG_NONSPD_BLOCK);
        }
    }
    if (wave == NT / kWave - 1 && lane < 12) {
        const int c = lane / 3, aa = lane % 3;
        double reg = 0.0;
        for (int t0 = 0; t0 < nslots; t0 += kChunk) {
            float ehc[kChunk], rja[kChunk], rla[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int t = min(t0 + u, MISSLAM_MAX_ROW - 1);
                ehc[u] = c < 3 ? rn.rg[t][c < 3 ? c : 0] : 1.f;
                rja[u] = rn.rg[t][3 + aa];
                rla[u] = rn.rg[t][6 + aa];
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                if (t0 + u < nslots && !((dmask >> (t0 + u)) & 1)) {
                    reg = fma((double)ehc[u], (double)rja[u], reg);
                    if (c == 3) reg -= rla[u];
                }
            }
        }
        double rot = 0.0;
        if (c < 3) {
#pragma unroll
            for (int q = 0; q < 6; ++q) rot = fma((double)rn.Jr[q][lane], (double)rn.rr[q], rot);
        }
        // the three terms balance near convergence: combined in float64, rounded once
        a.gvec[(size_t)j * 12 + lane] =
            (float)fma((double)wrot, rot, fma((double)wreg, reg, (double)wd * rn.gd[lane]));
    }
}

// Registers of one list entry between its global loads and its LDS staging.
template <int K>
struct EntryRegs {
    int q[K];
    float wq[K];
    float4 nr;
    float vx, vy, vz;
    uint32_t k0, k1;
};

// Registers of one packed list entry: read in list order, except the point's (n', r) (a gather).
template <int K>
struct EntryPack {
    float4 uw;                  // (v_p - g_j, w_pj)
    float4 w[(K + 3) / 4];      // w_pj w_pq, nodes in index order
    float4 nr;
    uint32_t k0, k1;
};

// The data of list entry le whose point p is already known.
template <int K>
__device__ __forceinline__ void entry_pack(const StepArgs &a, const StepScratch &s, int le, int p,
                                           EntryPack<K> &r) {
    constexpr int KW = (K + 3) / 4;
    r.uw = s.lpa[le];
#pragma unroll
    for (int g4 = 0; g4 < KW; ++g4) r.w[g4] = s.lpw[(size_t)le * KW + g4];
    r.nr = s.nr[p];
    r.k0 = a.g.list_key[2 * (size_t)le];
    r.k1 = a.g.list_key[2 * (size_t)le + 1];
}

// Packs the list entries of node j, one per thread: (v_p - g_j, w_pj) and the weight products in the
// order of the entry's row positions (the nodes of its kNN set sorted by index).
template <int K>
__device__ __forceinline__ void list_pack_body(const StepArgs &a, const StepScratch &s, int j) {
    constexpr int KW = (K + 3) / 4;
    if (j >= a.nd.m) return;
    const int64_t n = a.pts.n;
    const int lb = a.g.list_ptr[j];
    const int cnt = a.g.list_ptr[j + 1] - lb;
    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    for (int t = threadIdx.x; t < cnt; t += 256) {
        const int le = lb + t;
        const int p = a.g.list_pts[le];
        int q[K];
        float wq[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            q[u] = a.g.knn_idx[(int64_t)u * n + p];
            wq[u] = a.g.knn_w[(int64_t)u * n + p];
        }
        float wj = 0.f;
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (q[u] == j) wj = wq[u];
#pragma unroll
        for (int u = 1; u < K; ++u)
#pragma unroll
            for (int v = u; v > 0; --v)
                if (q[v] < q[v - 1]) {
                    const int ti = q[v];
                    q[v] = q[v - 1];
                    q[v - 1] = ti;
                    const float tw = wq[v];
                    wq[v] = wq[v - 1];
                    wq[v - 1] = tw;
                }
        s.lpa[le] = make_float4(a.pts.px[p] - gjx, a.pts.py[p] - gjy, a.pts.pz[p] - gjz, wj);
        float wv[4 * KW];
#pragma unroll
        for (int u = 0; u < 4 * KW; ++u) wv[u] = u < K ? wj * wq[u] : 0.f;
#pragma unroll
        for (int g4 = 0; g4 < KW; ++g4)
            s.lpw[(size_t)le * KW + g4] = make_float4(wv[4 * g4], wv[4 * g4 + 1], wv[4 * g4 + 2], wv[4 * g4 + 3]);
    }
}

template <int K>
__global__ void __launch_bounds__(256) list_pack_kernel(StepArgs a, StepScratch s) {
    list_pack_body<K>(a, s, blockIdx.x);
}

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

// One workgroup of W waves (the assembly tile: one or two) per node row j (rows
// spread so each XCD owns a contiguous band).  The waves split the row's point
// list and run independently: each stages 64 list entries at a time (lane =
// entry) while the next 64 are already being fetched, then accumulates the 60
// statistic entries (lane = entry of the statistic) for the k node pairs of
// each run of equal kNN sets, into slots of its own.  With two waves the LDS of
// a row stays under 23 KB, so seven rows fit a CU and a 1600-node graph is
// resident at once.  Then the
// node terms (Eqs.(5)-(6)) are added, the row's blocks and gradient are
// written, and the damped diagonal block is inverted for the block-Jacobi
// preconditioner.  Fixed summation order throughout: bitwise reproducible.
template <int K, int W>
__device__ __forceinline__ void assemble_rows_body(const StepArgs &a, const StepScratch &s, int j) {
    constexpr int kAsmThreads = kWave * W, kAsmWaves = W, kSlotsPerWave = kAsmSlots / W;
    __shared__ AsmShared<K, W> sh;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int64_t n = a.pts.n;

    // an overflowed pattern (flagged by the graph build) is clamped to the capacity
    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap);
    const int re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    const int nslots = min(re - rb, MISSLAM_MAX_ROW);
    for (int t = tid; t < (re - rb - nslots) * 144; t += kAsmThreads)
        a.blocks[(size_t)(rb + nslots) * 144 + t] = 0.f;   // blocks of a row longer than MISSLAM_MAX_ROW
    for (int t = tid; t < nslots; t += kAsmThreads) sh.rn.cols[t] = a.g.col_idx[rb + t];
    // the waves split the point list, each with slots of its own; a row with more slots than a wave holds is
    // accumulated by the first wave alone, over the slots of all waves.  Each wave clears the slots it uses
    // (no other wave touches them until the workgroup barrier after the data phase).
    const bool split = nslots <= kSlotsPerWave;
    const int nw = split ? kAsmWaves : 1;
    float(*accw)[60] = sh.accS + (split ? wave * kSlotsPerWave : 0);
    {
        const int nclr = (wave < nw ? (split ? kSlotsPerWave : kAsmWaves * kSlotsPerWave) : 0) * 60 / 4;
        for (int t = lane; t < nclr; t += kWave)
            reinterpret_cast<float4 *>(&accw[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    const int lb = a.g.list_ptr[j];
    const int cnt = a.g.list_ptr[j + 1] - lb;
    const int quota = (cnt + nw - 1) / nw;
    const int my0 = wave < nw ? min(cnt, wave * quota) : cnt;
    const int my1 = wave < nw ? min(cnt, my0 + quota) : cnt;
    const int nbatch = (my1 - my0 + kBatch - 1) / kBatch;
    AsmStage<K> &st = sh.st[wave];
    // Entries are fetched in two stages: the point index two batches ahead (coalesced), the point's data one
    // batch ahead (gathers whose addresses are known by then), so no wait in the loop is a chain of two
    // dependent loads.  The first batch's entries are fetched before the node-level loads are waited for.
    EntryPack<K> nxt;
    int pnext = 0;   // point of this lane's entry in the next batch
    if (nbatch > 0 && lane < min(kBatch, my1 - my0))
        entry_pack<K>(a, s, lb + my0 + lane, a.g.list_pts[lb + my0 + lane], nxt);
    if (nbatch > 1 && lane < min(kBatch, my1 - my0 - kBatch)) pnext = a.g.list_pts[lb + my0 + kBatch + lane];
    const float lamf = step_lambda(a);
    const double e_reg = row_prepare(a, sh.rn, j, nslots, gjx, gjy, gjz);

    const int e = lane;                      // statistic entry owned in phase 2 (e < 60)
    const int pci = e < 60 ? e / 6 : 0, nai = e < 60 ? e % 6 : 0;
    float acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.f;
    f32x4_t acc4 = {0.f, 0.f, 0.f, 0.f};   // K <= 4: the run's sums on the matrix cores (lane e, register q)
    uint32_t cur0 = 0xFFFFFFFFu, cur1 = 0xFFFFFFFFu;
    // a finished run's sums into the slots of its kNN set's nodes (distinct slots: reads, then writes)
    auto flush = [&](uint32_t k0, uint32_t k1, float(&ac)[K]) {
        if (k0 != 0xFFFFFFFFu && e < 60) {
            uint32_t slot[K];
            float old[K];
#pragma unroll
            for (int q = 0; q < K; ++q) {
                slot[q] = q < 4 ? (k0 >> (8 * q)) & 0xFF : (k1 >> (8 * (q - 4))) & 0xFF;
                old[q] = slot[q] < (uint32_t)nslots ? accw[slot[q]][e] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < K; ++q)
                if (slot[q] < (uint32_t)nslots) accw[slot[q]][e] = old[q] + ac[q];
        }
#pragma unroll
        for (int q = 0; q < K; ++q) ac[q] = 0.f;
    };
    double gacc[12];                 // data gradient: float64, it cancels near convergence
#pragma unroll
    for (int q = 0; q < 12; ++q) gacc[q] = 0.0;

    for (int bt = 0; bt < nbatch; ++bt) {
        const int e0 = my0 + bt * kBatch;
        const int nb = min(kBatch, my1 - e0);
        EntryPack<K> cu = nxt;
        // prefetch: the next batch's data, then the point indices of the batch after next (issued last, so
        // that waiting for this batch's data never waits for them)
        if (bt + 1 < nbatch && lane < min(kBatch, my1 - e0 - kBatch))
            entry_pack<K>(a, s, lb + e0 + kBatch + lane, pnext, nxt);
        if (bt + 2 < nbatch && lane < min(kBatch, my1 - e0 - 2 * kBatch))
            pnext = a.g.list_pts[lb + e0 + 2 * kBatch + lane];
        // ---- phase 1: lane = list entry.  An entry whose point has no correspondence (n' = 0 from the point
        // pass) adds nothing, so the valid entries are packed in order (position pv) for phase 2.
        const bool valid = lane < nb && (cu.nr.x != 0.f || cu.nr.y != 0.f || cu.nr.z != 0.f);
        const uint64_t vmask = __ballot(valid);
        const int pv = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(vmask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)vmask, 0u));
        const int np = __builtin_amdgcn_readfirstlane(__popcll(vmask));
        if (valid) {
            const float wj = cu.uw.w;
            const float uu[4] = {cu.uw.x, cu.uw.y, cu.uw.z, 1.f};
            const float nn[3] = {cu.nr.x, cu.nr.y, cu.nr.z};
#pragma unroll
            for (int t = 0; t < 10; ++t) st.Pc[t][pv] = uu[pair_c0(t)] * uu[pair_c1(t)];
#pragma unroll
            for (int t = 0; t < 6; ++t) st.Na[t][pv] = nn[pair_a0(t)] * nn[pair_a1(t)];
#pragma unroll
            for (int t = 0; t < (K + 3) / 4; ++t) st.W[pv][t] = cu.w[t];
            st.key[pv][0] = cu.k0;
            st.key[pv][1] = cu.k1;
            const float wr = wj * cu.nr.w;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float f = wr * uu[c];
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) gacc[3 * c + aa] = fma((double)f, (double)nn[aa], gacc[3 * c + aa]);
            }
        }
        wave_sync();
        // run starts among the packed entries: an entry whose kNN set differs from the previous one's (the
        // list is ordered by set, so equal sets stay contiguous after packing)
        bool start = false;
        if (lane < np) {
            const uint32_t q0 = lane == 0 ? cur0 : st.key[lane - 1][0];
            const uint32_t q1 = lane == 0 ? cur1 : st.key[lane - 1][1];
            start = st.key[lane][0] != q0 || st.key[lane][1] != q1;
        }
        const uint64_t starts = __ballot(start);
        // ---- phase 2: lane = statistic entry, the entries in order; a run of equal kNN sets ends by adding
        // its sums into the slots of its nodes.  The products of the next four entries are read from LDS
        // while the current four are accumulated.
        if constexpr (K <= 4) {
            // v_mfma_f32_4x4x1 (16 blocks): lane e = 4 b + c gives A = W[u][e % 4] and B = the product of entry u
            // for statistic entry e, so register q of lane e accumulates W[u][q] * product (one fused
            // multiply-add per entry, the same arithmetic as the vector path)
            const float *Wf = reinterpret_cast<const float *>(&st.W[0][0]);
            float cA[4], nA[4], wA[4], cB[4], nB[4], wB[4];
            auto fetch = [&](int u0, float(&cv)[4], float(&nv)[4], float(&wv)[4]) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    cv[h] = st.Pc[pci][u0 + h];
                    nv[h] = st.Na[nai][u0 + h];
                    wv[h] = Wf[(u0 + h) * 4 + (lane & 3)];
                }
            };
            auto consume = [&](int u0, const float(&cv)[4], const float(&nv)[4], const float(&wv)[4]) {
                const uint32_t sbits = (uint32_t)(starts >> u0) & 0xFu;
                if (sbits == 0 && u0 + 4 <= np) {   // inside one run: four products, no checks
#pragma unroll
                    for (int h = 0; h < 4; ++h)
                        acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(wv[h], cv[h] * nv[h], acc4, 0, 0, 0);
                    return;
                }
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int u = u0 + h;
                    if (u >= np) break;
                    if ((sbits >> h) & 1u) {   // a run starts at entry u
#pragma unroll
                        for (int q = 0; q < K; ++q) acc[q] = acc4[q];
                        flush(cur0, cur1, acc);
                        acc4 = f32x4_t{0.f, 0.f, 0.f, 0.f};
                        cur0 = __builtin_amdgcn_readfirstlane(st.key[u][0]);
                        cur1 = __builtin_amdgcn_readfirstlane(st.key[u][1]);
                    }
                    acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(wv[h], cv[h] * nv[h], acc4, 0, 0, 0);
                }
            };
            fetch(0, cA, nA, wA);
            for (int g = 0; g < np; g += 8) {
                fetch(g + 4, cB, nB, wB);
                consume(g, cA, nA, wA);
                fetch(g + 8, cA, nA, wA);
                consume(g + 4, cB, nB, wB);
            }
        } else
        {
            constexpr int KW = (K + 3) / 4;
            float cA[4], nA[4], cB[4], nB[4];
            float4 wA[4][KW], wB[4][KW];
            auto fetch = [&](int u0, float(&cv)[4], float(&nv)[4], float4(&wv)[4][KW]) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    cv[h] = st.Pc[pci][u0 + h];
                    nv[h] = st.Na[nai][u0 + h];
#pragma unroll
                    for (int g4 = 0; g4 < KW; ++g4) wv[h][g4] = st.W[u0 + h][g4];
                }
            };
            auto consume = [&](int u0, const float(&cv)[4], const float(&nv)[4], const float4(&wv)[4][KW]) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int u = u0 + h;
                    if (u >= np) break;
                    if ((starts >> u) & 1ull) {   // a run starts at entry u
                        flush(cur0, cur1, acc);
                        cur0 = __builtin_amdgcn_readfirstlane(st.key[u][0]);
                        cur1 = __builtin_amdgcn_readfirstlane(st.key[u][1]);
                    }
                    const float mv = cv[h] * nv[h];
#pragma unroll
                    for (int g4 = 0; g4 < KW; ++g4) {
                        const float wq4[4] = {wv[h][g4].x, wv[h][g4].y, wv[h][g4].z, wv[h][g4].w};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (4 * g4 + q < K) acc[4 * g4 + q] = fmaf(wq4[q], mv, acc[4 * g4 + q]);
                    }
                }
            };
            // entries beyond np (up to kBatch + 8, inside the arrays) are read and left unused, so that the
            // reads are unconditional and stay in flight across the accumulation
            fetch(0, cA, nA, wA);
            for (int g = 0; g < np; g += 8) {
                fetch(g + 4, cB, nB, wB);
                consume(g, cA, nA, wA);
                fetch(g + 8, cA, nA, wA);
                consume(g + 4, cB, nB, wB);
            }
        }
        wave_sync();
    }
    if constexpr (K <= 4) {
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = acc4[q];
    }
    flush(cur0, cur1, acc);
    // wave reduction of the data gradient (fixed butterfly order)
    wave_sums(gacc);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 12; ++q) sh.gw[wave][q] = gacc[q];
    }
    __syncthreads();
    if (kAsmWaves > 1 && split) {
        for (int t = tid; t < nslots * 60; t += kAsmThreads) {
            const int sl = t / 60, en = t - sl * 60;
            float v = sh.accS[sl][en];
#pragma unroll
            for (int w = 1; w < kAsmWaves; ++w) v += sh.accS[w * kSlotsPerWave + sl][en];   // waves in order
            sh.accS[sl][en] = v;
        }
    }
    if (tid < 12) {
        double v = sh.gw[0][tid];
#pragma unroll
        for (int w = 1; w < kAsmWaves; ++w) v += sh.gw[w][tid];
        sh.rn.gd[tid] = v;
    }
    __syncthreads();
    // data-term block from the statistic: H[(c,a),(c',a')] = S[c,c',a,a'] + delta_c' S[c,3,a,a']
    // off: slot sl is not the diagonal; every operand is read whether used or not (independent loads)
    auto data = [&](int sl, int R, int C, bool off) {
        const int c = R / 3, aa = R % 3, c2 = C / 3, a2 = C % 3;
        const float *S = sh.accS[sl];
        const int ni = na_index(aa, a2);
        const float s1 = S[pc_index(c, c2) * 6 + ni], s3 = S[pc_index(c, 3) * 6 + ni];
        const float e = sh.rn.rg[sl][c2 < 3 ? c2 : 0];
        return off && c2 < 3 ? fmaf(-e, s3, s1) : s1;   // delta = -e
    };
    row_finalize<kAsmThreads>(a, s, sh.rn, sh.fin, j, rb, nslots, e_reg, lamf, data, nullptr);
}

// The first workgroup of a kernel that runs right before a one-launch solve clears the solve's sync area
// (a.zero_words, if set): nothing reads it between that kernel and the solve.
__device__ __forceinline__ void clear_sync_words(const StepArgs &a) {
    if (blockIdx.x == 0 && a.zero_words)
        for (int t = threadIdx.x; t < a.zero_count / 4; t += blockDim.x)
            reinterpret_cast<uint4 *>(a.zero_words)[t] = make_uint4(0u, 0u, 0u, 0u);
}

template <int K, int W>
__global__ void __launch_bounds__(kWave * W) __attribute__((amdgpu_waves_per_eu(4)))
assemble_rows_kernel(StepArgs a, StepScratch s) {
    clear_sync_words(a);
    const int m = a.nd.m;
    const int per = (int)((m + 7) / 8);
    const int j = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (j >= m) return;
    assemble_rows_body<K, W>(a, s, j);
}


// ---------------------------------------------------------------- low-precision assembly on the matrix cores

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<__bf16> {
    typedef bf16x8_t vec;
    static __device__ __forceinline__ f32x4_t run(vec a, vec b, f32x4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaOp<_Float16> {
    typedef f16x8_t vec;
    static __device__ __forceinline__ f32x4_t run(vec a, vec b, f32x4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

constexpr int kLpThreads = 128;
constexpr int kLpWaves = kLpThreads / kWave;

constexpr int kLpSlotsPerWave = kAsmSlots / kLpWaves;

template <int K, typename T>
struct LpShared {
    float acc[kAsmSlots][144];   // blocks per slot; wave w's slots start at w kLpSlotsPerWave
    union {
        // per entry: J of node j (rows 0-11), then of its k set nodes; 16-byte groups of 8 entries
        alignas(16) T Jt[kLpWaves][12 * (K + 1)][kBatch];
        RowFin<kLpThreads> fin;   // once the data term is complete
    };
    uint32_t key[kLpWaves][kBatch][2];
    double gw[kLpWaves][12];
    RowNode rn;
};

// Same rows as assemble_rows_kernel, but the data term is formed from the
// per-point Jacobian rows J_pj = w_pj kron((v_p - g_j, 1), n'_p) rounded to T
// (bfloat16 or float16) and contracted on the matrix cores with float32
// accumulation: for each run of equal kNN sets, chunks of 32 list entries
// give J_j^T J_{set} (16x32 by 32x16 tiles, 12 useful rows).  The
// gradient g and every regulariser block stay float32.  rr_out receives the
// regulariser + rotation blocks alone for the float32 refinement.
template <int K, typename T>
__global__ void __launch_bounds__(kLpThreads) assemble_lp_kernel(StepArgs a, StepScratch s, float *rr_out) {
    __shared__ LpShared<K, T> sh;
    constexpr int NT = (12 * K + 15) / 16;           // column tiles of the set nodes' parameters
    clear_sync_words(a);
    const int m = a.nd.m;
    const int per = (int)((m + 7) / 8);
    const int j = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (j >= m) return;
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave;
    const int64_t n = a.pts.n;

    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap);
    const int re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    const int nslots = min(re - rb, MISSLAM_MAX_ROW);
    for (int t = tid; t < (re - rb - nslots) * 144; t += kLpThreads) a.blocks[(size_t)(rb + nslots) * 144 + t] = 0.f;
    for (int t = tid; t < nslots; t += kLpThreads) sh.rn.cols[t] = a.g.col_idx[rb + t];
    // as in the float32 rows: the waves split the point list, each with slots of its own, unless the row has
    // more slots than a wave holds (then the first wave takes the whole list over every slot); each wave
    // clears the slots it uses
    const bool split = nslots <= kLpSlotsPerWave;
    const int nw = split ? kLpWaves : 1;
    float(*accw)[144] = sh.acc + (split ? wave * kLpSlotsPerWave : 0);
    {
        const int nclr = (wave < nw ? (split ? kLpSlotsPerWave : kLpWaves * kLpSlotsPerWave) : 0) * 144 / 4;
        for (int t = lane; t < nclr; t += kWave)
            reinterpret_cast<float4 *>(&accw[0][0])[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    const float lamf = step_lambda(a);
    const double e_reg = row_prepare(a, sh.rn, j, nslots, gjx, gjy, gjz);
    const int lb = a.g.list_ptr[j];
    const int cnt = a.g.list_ptr[j + 1] - lb;
    const int quota = (cnt + nw - 1) / nw;
    const int my0 = wave < nw ? min(cnt, wave * quota) : cnt;
    const int my1 = wave < nw ? min(cnt, my0 + quota) : cnt;
    const int nbatch = (my1 - my0 + kBatch - 1) / kBatch;
    const int r16 = lane % 16, kb = 8 * (lane / 16);

    f32x4_t D[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) D[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    uint32_t cur0 = 0xFFFFFFFFu, cur1 = 0xFFFFFFFFu;
    double gacc[12];                 // data gradient: float64, it cancels near convergence
#pragma unroll
    for (int q = 0; q < 12; ++q) gacc[q] = 0.0;
    __syncthreads();   // cols visible to every wave

    auto flush = [&]() {
        if (cur0 == 0xFFFFFFFFu) return;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int col = 16 * q + r16;
            const int sidx = col / 12;
            if (sidx < K) {
                const uint32_t slot = sidx < 4 ? (cur0 >> (8 * sidx)) & 0xFF : (cur1 >> (8 * (sidx - 4))) & 0xFF;
                if (slot < (uint32_t)nslots) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = 4 * (lane / 16) + i;
                        if (row < 12) accw[slot][row * 12 + col % 12] += D[q][i];
                    }
                }
            }
            D[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
    };

    EntryRegs<K> nxt;
    if (nbatch > 0 && lane < min(kBatch, my1 - my0)) entry_load<K>(a, s, n, lb + my0 + lane, nxt);
    for (int bt = 0; bt < nbatch; ++bt) {
        const int e0 = my0 + bt * kBatch;
        const int nb = min(kBatch, my1 - e0);
        EntryRegs<K> cu = nxt;
        if (bt + 1 < nbatch && lane < min(kBatch, my1 - e0 - kBatch))
            entry_load<K>(a, s, n, lb + e0 + kBatch + lane, nxt);
        // ---- phase 1: lane = list entry; Jacobian rows in T, gradient in float32
        if (lane < nb) {
            float wj = 0.f;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if (cu.q[t] == j) wj = cu.wq[t];
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
            const float nn[3] = {cu.nr.x, cu.nr.y, cu.nr.z};
            const float uj[4] = {cu.vx - gjx, cu.vy - gjy, cu.vz - gjz, 1.f};
#pragma unroll
            for (int p = 0; p < 12; ++p) sh.Jt[wave][p][lane] = (T)(wj * uj[p / 3] * nn[p % 3]);
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const int l = cu.q[t];
                const float ul[4] = {cu.vx - a.nd.gx[l], cu.vy - a.nd.gy[l], cu.vz - a.nd.gz[l], 1.f};
#pragma unroll
                for (int p = 0; p < 12; ++p) sh.Jt[wave][12 + 12 * t + p][lane] = (T)(cu.wq[t] * ul[p / 3] * nn[p % 3]);
            }
            sh.key[wave][lane][0] = cu.k0;
            sh.key[wave][lane][1] = cu.k1;
            const float wr = wj * cu.nr.w;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float f = wr * uj[c];
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) gacc[3 * c + aa] = fma((double)f, (double)nn[aa], gacc[3 * c + aa]);
            }
        }
        bool start;
        {
            const uint32_t p0 = __shfl_up(cu.k0, 1, 64), p1 = __shfl_up(cu.k1, 1, 64);
            const uint32_t q0 = lane == 0 ? cur0 : p0, q1 = lane == 0 ? cur1 : p1;
            start = lane < nb && (cu.k0 != q0 || cu.k1 != q1);
        }
        const uint64_t starts = __ballot(start);
        wave_sync();
        // ---- phase 2: per run of equal sets, 32-entry chunks on the matrix cores
        int t = 0;
        while (t < nb) {
            if (starts & (1ull << t)) {
                flush();
                cur0 = sh.key[wave][t][0];
                cur1 = sh.key[wave][t][1];
            }
            const uint64_t later = t + 1 < 64 ? (starts >> (t + 1)) : 0ull;
            const int t1 = later ? min(nb, t + 1 + __builtin_ctzll(later)) : nb;
            // 32-entry chunks from the run's first group of 8: each lane reads its 8 entries of a row as one
            // 16-byte group and zeroes those outside [t, t1) with a bit mask (which also keeps out whatever the
            // staging holds there)
            for (int c0 = t & ~7; c0 < t1; c0 += 32) {
                typedef typename MfmaOp<T>::vec vec;
                typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
                const int g = c0 + kb;          // a group that starts before t1 ends inside the 64 entries
                u32x4 mk = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int e = g + 2 * d;
                    mk[d] = (e >= t && e < t1 ? 0x0000FFFFu : 0u) | (e + 1 >= t && e + 1 < t1 ? 0xFFFF0000u : 0u);
                }
                const bool in = g < t1;
                u32x4 ar = {0u, 0u, 0u, 0u};
                if (in && r16 < 12) ar = *reinterpret_cast<const u32x4 *>(&sh.Jt[wave][r16][g]);
                const vec av = __builtin_bit_cast(vec, ar & mk);
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int col = 16 * q + r16;
                    u32x4 br = {0u, 0u, 0u, 0u};
                    if (in && col < 12 * K) br = *reinterpret_cast<const u32x4 *>(&sh.Jt[wave][12 + col][g]);
                    D[q] = MfmaOp<T>::run(av, __builtin_bit_cast(vec, br & mk), D[q]);
                }
            }
            t = t1;
        }
        wave_sync();
    }
    flush();
    wave_sums(gacc);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 12; ++q) sh.gw[wave][q] = gacc[q];
    }
    __syncthreads();
    if (split)
        for (int t = tid; t < nslots * 144; t += kLpThreads) {
            const int sl = t / 144, en = t - sl * 144;
            float v = sh.acc[sl][en];
#pragma unroll
            for (int w = 1; w < kLpWaves; ++w) v += sh.acc[w * kLpSlotsPerWave + sl][en];   // waves in order
            sh.acc[sl][en] = v;
        }
    if (tid < 12) {
        double v = sh.gw[0][tid];
#pragma unroll
        for (int w = 1; w < kLpWaves; ++w) v += sh.gw[w][tid];
        sh.rn.gd[tid] = v;
    }
    __syncthreads();
    auto data = [&](int sl, int R, int C, bool) { return sh.acc[sl][R * 12 + C]; };
    row_finalize<kLpThreads>(a, s, sh.rn, sh.fin, j, rb, nslots, e_reg, lamf, data, rr_out);
}

hipError_t launch_assemble_lp(const StepArgs &a, const StepScratch &s, int precision, float *rr_out,
                              hipStream_t st) {
    if (a.zero_words && (a.zero_count < 0 || a.zero_count > MSL_BAR_WORDS || a.zero_count % 4))
        return hipErrorInvalidValue;
    const unsigned rows = 8 * (unsigned)((a.nd.m + 7) / 8);
    const bool bf = precision == MISSLAM_PREC_BF16;
    switch (a.g.k) {
#define MSL_LP_CASE(KK)                                                                                         \
    case KK:                                                                                                    \
        if (bf)                                                                                                 \
            hipLaunchKernelGGL((assemble_lp_kernel<KK, __bf16>), dim3(rows), dim3(kLpThreads), 0, st, a, s, rr_out); \
        else                                                                                                    \
            hipLaunchKernelGGL((assemble_lp_kernel<KK, _Float16>), dim3(rows), dim3(kLpThreads), 0, st, a, s, rr_out); \
        break;
        MSL_LP_CASE(1) MSL_LP_CASE(2) MSL_LP_CASE(3) MSL_LP_CASE(4)
#undef MSL_LP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- float32 matrix-free data term (refinement)

// (J dx)_p = n'_p . sum_s w_ps (dA_s (v_p - g_s) + dt_s): the linearised data
// residual change of each point for a parameter step dx.
template <int K>
__global__ void __launch_bounds__(256) jv_kernel(StepArgs a, StepScratch s, const float *__restrict__ dx,
                                                 float *__restrict__ out) {
    const int64_t n = a.pts.n;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 nr = s.nr[i];
    const float vx = a.pts.px[i], vy = a.pts.py[i], vz = a.pts.pz[i];
    float ux = 0.f, uy = 0.f, uz = 0.f;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int j = a.g.knn_idx[(int64_t)t * n + i];
        const float w = a.g.knn_w[(int64_t)t * n + i];
        const float *d = dx + (size_t)j * 12;
        const float ex = vx - a.nd.gx[j], ey = vy - a.nd.gy[j], ez = vz - a.nd.gz[j];
        ux = fmaf(w, fmaf(d[6], ez, fmaf(d[3], ey, fmaf(d[0], ex, d[9]))), ux);
        uy = fmaf(w, fmaf(d[7], ez, fmaf(d[4], ey, fmaf(d[1], ex, d[10]))), uy);
        uz = fmaf(w, fmaf(d[8], ez, fmaf(d[5], ey, fmaf(d[2], ex, d[11]))), uz);
    }
    out[i] = fmaf(nr.z, uz, fmaf(nr.y, uy, nr.x * ux));
}

// One wave per row j: y_j = w_data sum_{p in list(j)} w_pj (J dx)_p kron((v_p - g_j, 1), n'_p)
//                            + (H_rr dx)_j + lambda dx_j;  rhs_j = g_j + y_j.
// (The next solve of (H_lo + lambda I) d = -rhs gives d = (H_lo + lambda I)^-1 (-g - y).)
template <int K>
__global__ void __launch_bounds__(64) jtv_row_kernel(StepArgs a, StepScratch s, const float *__restrict__ jv,
                                                     const float *__restrict__ rr, const float *__restrict__ dx,
                                                     const float *__restrict__ g, float *__restrict__ rhs) {
    clear_sync_words(a);
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t n = a.pts.n;
    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    const int lb = a.g.list_ptr[j];
    const int cnt = a.g.list_ptr[j + 1] - lb;
    float acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = 0.f;
    for (int t = lane; t < cnt; t += 64) {
        const int p = a.g.list_pts[lb + t];
        float wj = 0.f;
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (a.g.knn_idx[(int64_t)u * n + p] == j) wj = a.g.knn_w[(int64_t)u * n + p];
        const float4 nr = s.nr[p];
        const float f = wj * jv[p];
        const float uu[4] = {a.pts.px[p] - gjx, a.pts.py[p] - gjy, a.pts.pz[p] - gjz, 1.f};
        const float nn[3] = {nr.x, nr.y, nr.z};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) acc[3 * c + aa] = fmaf(f * uu[c], nn[aa], acc[3 * c + aa]);
    }
    wave_sums(acc);
    if (lane < 12) {
        float y = 0.f;
#pragma unroll
        for (int q = 0; q < 12; ++q) y = q == lane ? acc[q] : y;
        y = a.w_data * y;
        const int rb = min(a.g.row_ptr[j], a.g.bsr_cap), re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
        for (int pb = rb; pb < re; ++pb) {
            const int l = a.g.col_idx[pb];
            const float *B = rr + (size_t)pb * 144 + lane * 12;
            const float *xl = dx + (size_t)l * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) y = fmaf(B[b], xl[b], y);
        }
        y = fmaf(a.lambda, dx[(size_t)j * 12 + lane], y);
        rhs[(size_t)j * 12 + lane] = g[(size_t)j * 12 + lane] + y;
    }
}

__global__ void axpy_kernel(float *__restrict__ y, const float *__restrict__ x, int count) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < count) y[t] += x[t];
}

hipError_t launch_refine_rhs(const StepArgs &a, const StepScratch &s, const float *dx, const float *rr, const float *g,
                             float *jv, float *rhs, hipStream_t st) {
    if (a.zero_words && (a.zero_count < 0 || a.zero_count > MSL_BAR_WORDS || a.zero_count % 4))
        return hipErrorInvalidValue;
    const int64_t n = a.pts.n;
    if (n > 0) {
        switch (a.g.k) {
#define MSL_JV_CASE(KK) \
    case KK: hipLaunchKernelGGL((jv_kernel<KK>), dim3(nblk(n, 256)), dim3(256), 0, st, a, s, dx, jv); break;
            MSL_JV_CASE(1) MSL_JV_CASE(2) MSL_JV_CASE(3) MSL_JV_CASE(4)
            MSL_JV_CASE(5) MSL_JV_CASE(6) MSL_JV_CASE(7) MSL_JV_CASE(8)
#undef MSL_JV_CASE
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.g.k) {
#define MSL_JT_CASE(KK) \
    case KK: hipLaunchKernelGGL((jtv_row_kernel<KK>), dim3(a.nd.m), dim3(64), 0, st, a, s, jv, rr, dx, g, rhs); break;
        MSL_JT_CASE(1) MSL_JT_CASE(2) MSL_JT_CASE(3) MSL_JT_CASE(4)
        MSL_JT_CASE(5) MSL_JT_CASE(6) MSL_JT_CASE(7) MSL_JT_CASE(8)
#undef MSL_JT_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpy(float *y, const float *x, int count, hipStream_t st) {
    hipLaunchKernelGGL(axpy_kernel, dim3(nblk(count, 256)), dim3(256), 0, st, y, x, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- node energies without assembly

// E_rot of node j (Eq.(5)) and E_reg over its outgoing edges (Eq.(6)), float64
// sums of float32 residuals in the assembly's order; one thread per node.
__device__ __forceinline__ void node_energy_body(const StepArgs &a, const StepScratch &s, int blk) {
    const int j = blk * 256 + threadIdx.x;
    if (j >= a.nd.m) return;
    const float *xj = a.nd.x + (size_t)j * 12;
    auto dot = [](const float *u, const float *v) { return fmaf(u[2], v[2], fmaf(u[1], v[1], u[0] * v[0])); };
    const float rr[6] = {dot(xj, xj + 3), dot(xj, xj + 6), dot(xj + 3, xj + 6),
                         unit_residual(xj, 0), unit_residual(xj + 3, 1), unit_residual(xj + 6, 2)};
    double erot = 0.0;
    for (int q = 0; q < 6; ++q) erot += (double)rr[q] * rr[q];
    const float gjx = a.nd.gx[j], gjy = a.nd.gy[j], gjz = a.nd.gz[j];
    const int rb = min(a.g.row_ptr[j], a.g.bsr_cap), re = min(a.g.row_ptr[j + 1], a.g.bsr_cap);
    double ereg = 0.0;
    for (int p = rb; p < re && p - rb < MISSLAM_MAX_ROW; ++p) {
        const int l = a.g.col_idx[p];
        if (l == j) continue;
        const float glx = a.nd.gx[l], gly = a.nd.gy[l], glz = a.nd.gz[l];
        const float *xl = a.nd.x + (size_t)l * 12;
        const float ex = glx - gjx, ey = gly - gjy, ez = glz - gjz;
        float r0, r1, r2;
        reg_residual(xj, xl, ex, ey, ez, r0, r1, r2);
        ereg += ((double)r0 * r0 + (double)r1 * r1) + (double)r2 * r2;
    }
    s.node_part[2 * j + 0] = erot;
    s.node_part[2 * j + 1] = ereg;
}

__global__ void __launch_bounds__(256) node_energy_kernel(StepArgs a, StepScratch s) {
    node_energy_body(a, s, blockIdx.x);
}

hipError_t launch_node_energy(const StepArgs &a, const StepScratch &s, hipStream_t st) {
    hipLaunchKernelGGL(node_energy_kernel, dim3(nblk(a.nd.m, 256)), dim3(256), 0, st, a, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------- adjoint of the energy

// dE/dv_i for frozen correspondences and kNN sets, normalised Gaussian weights:
//   2 w_data r_i n'^T sum_j [w_j A_j + y_j (grad w_j)^T],  y_j = A_j (v - g_j) + g_j + t_j,
//   grad w_j = w_j (-(v - g_j) + sum_l w_l (v - g_l)) / sigma^2
// scaled by the upstream gradient.  One thread per point.
template <int K>
__global__ void __launch_bounds__(256) vjp_points_kernel(StepArgs a, StepScratch s, float sigma,
                                                         const float *__restrict__ grad_e, float *__restrict__ out) {
    const int64_t n = a.pts.n;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 nr = s.nr[i];
    const float ge = grad_e ? grad_e[0] : 1.f;
    const float vx = a.pts.px[i], vy = a.pts.py[i], vz = a.pts.pz[i];
    float d[K][3], wv[K];
    float md[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int j = a.g.knn_idx[(int64_t)t * n + i];
        wv[t] = a.g.knn_w[(int64_t)t * n + i];     // the normalised Gaussian weights of this point
        d[t][0] = vx - a.nd.gx[j];
        d[t][1] = vy - a.nd.gy[j];
        d[t][2] = vz - a.nd.gz[j];
#pragma unroll
        for (int c = 0; c < 3; ++c) md[c] = fmaf(wv[t], d[t][c], md[c]);
    }
    const float is2 = 1.f / (sigma * sigma);
    // row = n'^T M, M = sum_j [w_j A_j + y_j grad_w_j^T]
    float row[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int j = a.g.knn_idx[(int64_t)t * n + i];
        const float *x = a.nd.x + (size_t)j * 12;
        // n'^T A_j: component c = sum_a n'_a A[a][c] = n' . column c
        const float nA[3] = {fmaf(nr.z, x[2], fmaf(nr.y, x[1], nr.x * x[0])),
                             fmaf(nr.z, x[5], fmaf(nr.y, x[4], nr.x * x[3])),
                             fmaf(nr.z, x[8], fmaf(nr.y, x[7], nr.x * x[6]))};
        const float y0 = fmaf(x[6], d[t][2], fmaf(x[3], d[t][1], x[0] * d[t][0])) + a.nd.gx[j] + x[9];
        const float y1 = fmaf(x[7], d[t][2], fmaf(x[4], d[t][1], x[1] * d[t][0])) + a.nd.gy[j] + x[10];
        const float y2 = fmaf(x[8], d[t][2], fmaf(x[5], d[t][1], x[2] * d[t][0])) + a.nd.gz[j] + x[11];
        const float ny = fmaf(nr.z, y2, fmaf(nr.y, y1, nr.x * y0));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float gw = wv[t] * (md[c] - d[t][c]) * is2;
            row[c] = fmaf(wv[t], nA[c], fmaf(ny, gw, row[c]));
        }
    }
    const float sc = 2.f * a.w_data * nr.w * ge;
    out[i] = sc * row[0];
    out[n + i] = sc * row[1];
    out[2 * n + i] = sc * row[2];
}

hipError_t launch_vjp_points(const StepArgs &a, const StepScratch &s, float sigma, const float *grad_e, float *out,
                             hipStream_t st) {
    if (a.pts.n == 0) return hipSuccess;
    const dim3 grid(nblk(a.pts.n, 256)), blk(256);
    switch (a.g.k) {
#define MSL_VJ_CASE(KK) \
    case KK: hipLaunchKernelGGL((vjp_points_kernel<KK>), grid, blk, 0, st, a, s, sigma, grad_e, out); break;
        MSL_VJ_CASE(1) MSL_VJ_CASE(2) MSL_VJ_CASE(3) MSL_VJ_CASE(4)
        MSL_VJ_CASE(5) MSL_VJ_CASE(6) MSL_VJ_CASE(7) MSL_VJ_CASE(8)
#undef MSL_VJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// dE/dx = 2 g (g = sum w J^T r of the normal equations), scaled by the upstream gradient.
__global__ void scale_grad_kernel(const float *__restrict__ g, int count, const float *__restrict__ grad_e,
                                  float *__restrict__ out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < count) out[t] = 2.f * (grad_e ? grad_e[0] : 1.f) * g[t];
}

// E = w_data E_data + w_rot E_rot + w_reg E_reg (Eq.(3) restricted to the hot-path terms).
__global__ void energy_total_kernel(const misslam_report *rep, double w_data, double w_rot, double w_reg,
                                    double *out) {
    if (threadIdx.x == 0) out[0] = (w_data * rep->e_data + w_rot * rep->e_rot) + w_reg * rep->e_reg;
}

hipError_t launch_grad_params(const float *g, int m, const float *grad_e, float *out, hipStream_t st) {
    hipLaunchKernelGGL(scale_grad_kernel, dim3(nblk(12 * (int64_t)m, 256)), dim3(256), 0, st, g, 12 * m, grad_e, out);
    return hipGetLastError();
}

hipError_t launch_energy_total(const misslam_report *rep, float w_data, float w_rot, float w_reg, double *out,
                               hipStream_t st) {
    hipLaunchKernelGGL(energy_total_kernel, dim3(1), dim3(64), 0, st, rep, (double)w_data, (double)w_rot,
                       (double)w_reg, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- energy report

__global__ void __launch_bounds__(256) energy_report_kernel(const double *__restrict__ pt_part, int npb,
                                                            const double *__restrict__ node_part, int m,
                                                            misslam_report *rep, float reject_thr,
                                                            unsigned *__restrict__ zero_words, int zero_count,
                                                            const double *__restrict__ kp_energy, int kp_count) {
    energy_report_body(pt_part, npb, node_part, m, rep, reject_thr, zero_words, zero_count, kp_energy, kp_count);
}

template <int K>
__global__ void __launch_bounds__(kPtBlock) point_pass_joint_kernel(StepArgs a, StepScratch s, KeyArgs kp,
                                                                   float *kp_data, double *kp_energy, unsigned ptb) {
    if (blockIdx.x < ptb)
        point_pass_body<K, true>(a, s, blockIdx.x);
    else   // the key points, Eq.(9), one per thread, at the device pose
        kp_eval_body<K>(a, kp, kp_data, kp_energy, (int)(blockIdx.x - ptb) * kPtBlock + (int)threadIdx.x);
}

int point_blocks(int64_t n) { return (int)nblk(n > 0 ? n : 1, kPtBlock); }

hipError_t launch_point_pass_joint(const StepArgs &a, const StepScratch &s, hipStream_t st, const KeyArgs *kp,
                                  const CorrScratch *c) {
    const unsigned ptb = nblk(a.pts.n > 0 ? a.pts.n : 1, kPtBlock);
    KeyArgs kk{};
    float *kd = nullptr;
    double *ke = nullptr;
    if (kp && c && kp->count > 0) {
        kk = *kp;
        kd = c->kp_data;
        ke = c->kp_energy;
    }
    const unsigned kpb = (unsigned)((kk.count + kPtBlock - 1) / kPtBlock);
    switch (a.g.k) {
#define MSL_PJ_CASE(KK)                                                                                     \
    case KK:                                                                                                \
        hipLaunchKernelGGL((point_pass_joint_kernel<KK>), dim3(ptb + kpb), dim3(kPtBlock), 0, st, a, s, kk, kd, ke, \
                           ptb);                                                                            \
        break;
        MSL_PJ_CASE(1) MSL_PJ_CASE(2) MSL_PJ_CASE(3) MSL_PJ_CASE(4)
        MSL_PJ_CASE(5) MSL_PJ_CASE(6) MSL_PJ_CASE(7) MSL_PJ_CASE(8)
#undef MSL_PJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_point_pass(const StepArgs &a, const StepScratch &s, hipStream_t st, const KeyArgs *kp,
                             const CorrScratch *c) {
    const int64_t n = a.pts.n;
    const unsigned ptb = nblk(n > 0 ? n : 1, kPtBlock);
    KeyArgs kk{};
    float *kd = nullptr;
    double *ke = nullptr;
    if (kp && c && kp->count > 0) {
        kk = *kp;
        kd = c->kp_data;
        ke = c->kp_energy;
    }
    const unsigned kpb = (unsigned)((kk.count + kPtBlock - 1) / kPtBlock);
    switch (a.g.k) {
#define MSL_PP_CASE(KK)                                                                                     \
    case KK:                                                                                                \
        hipLaunchKernelGGL((point_pass_kernel<KK>), dim3(ptb + kpb), dim3(kPtBlock), 0, st, a, s, kk, kd, ke, ptb); \
        break;
        MSL_PP_CASE(1) MSL_PP_CASE(2) MSL_PP_CASE(3) MSL_PP_CASE(4)
        MSL_PP_CASE(5) MSL_PP_CASE(6) MSL_PP_CASE(7) MSL_PP_CASE(8)
#undef MSL_PP_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_list_pack(const StepArgs &a, const StepScratch &s, hipStream_t st) {
    const int m = a.nd.m;
    if (m <= 0) return hipSuccess;
    switch (a.g.k) {
#define MSL_LK_CASE(KK) \
    case KK: hipLaunchKernelGGL((list_pack_kernel<KK>), dim3(m), dim3(256), 0, st, a, s); break;
        MSL_LK_CASE(1) MSL_LK_CASE(2) MSL_LK_CASE(3) MSL_LK_CASE(4)
        MSL_LK_CASE(5) MSL_LK_CASE(6) MSL_LK_CASE(7) MSL_LK_CASE(8)
#undef MSL_LK_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const StepArgs &a, const StepScratch &s, hipStream_t st) {
    if (a.zero_words && (a.zero_count < 0 || a.zero_count > MSL_BAR_WORDS || a.zero_count % 4))
        return hipErrorInvalidValue;
    const int m = a.nd.m;
    const unsigned rows = 8 * (unsigned)((m + 7) / 8);
    const bool one = a.asm_waves == 1;
    switch (a.g.k) {
#define MSL_AS_CASE(KK)                                                                                       \
    case KK:                                                                                                  \
        if (one) hipLaunchKernelGGL((assemble_rows_kernel<KK, 1>), dim3(rows), dim3(kWave), 0, st, a, s);     \
        else hipLaunchKernelGGL((assemble_rows_kernel<KK, 2>), dim3(rows), dim3(2 * kWave), 0, st, a, s);     \
        break;
        MSL_AS_CASE(1) MSL_AS_CASE(2) MSL_AS_CASE(3) MSL_AS_CASE(4)
        MSL_AS_CASE(5) MSL_AS_CASE(6) MSL_AS_CASE(7) MSL_AS_CASE(8)
#undef MSL_AS_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void report_args(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                 const double *kp_energy, int kp_count, ReportArgs &out) {
    out.pt_part = s.pt_part;
    out.npb = (int)nblk(n > 0 ? n : 1, kPtBlock);
    out.node_part = s.node_part;
    out.m = m;
    out.rep = rep;
    out.reject = reject_thr;
    out.kp_energy = kp_energy;
    out.kp_count = kp_energy ? kp_count : 0;
}

hipError_t launch_energy_report(const ReportArgs &ra, hipStream_t st) {
    hipLaunchKernelGGL(energy_report_kernel, dim3(1), dim3(256), 0, st, ra.pt_part, ra.npb, ra.node_part, ra.m,
                       ra.rep, ra.reject, nullptr, 0, ra.kp_energy, ra.kp_count);
    return hipGetLastError();
}

hipError_t launch_energy_report(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                                hipStream_t st, unsigned *zero_words, int zero_count, const double *kp_energy,
                                int kp_count) {
    const int npb = (int)nblk(n > 0 ? n : 1, kPtBlock);
    if (zero_count < 0 || zero_count > MSL_BAR_WORDS || zero_count % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(energy_report_kernel, dim3(1), dim3(256), 0, st, s.pt_part, npb, s.node_part, m, rep,
                       reject_thr, zero_words, zero_count, kp_energy, kp_energy ? kp_count : 0);
    return hipGetLastError();
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ src, int32_t *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------- batched launches

__device__ __forceinline__ int batch_of(const BatchItem *items, int count, int64_t blk, int which) {
    int b = count - 1;
    while (b > 0) {
        const int64_t start = which == 0 ? items[b].pp0 : which == 1 ? items[b].row0 : items[b].ne0;
        if (start <= blk) break;
        --b;
    }
    return b;
}

template <int K>
__global__ void __launch_bounds__(kPtBlock) point_pass_batched_kernel(const BatchItem *__restrict__ items, int count) {
    const BatchItem &it = items[batch_of(items, count, blockIdx.x, 0)];
    point_pass_body<K>(it.a, it.s, (int64_t)blockIdx.x - it.pp0);
}

template <int K>
__global__ void __launch_bounds__(256) list_pack_batched_kernel(const BatchItem *__restrict__ items, int count) {
    const BatchItem &it = items[batch_of(items, count, blockIdx.x, 1)];
    list_pack_body<K>(it.a, it.s, (int)blockIdx.x - it.row0);
}

template <int K, int W>
__global__ void __launch_bounds__(kWave * W) __attribute__((amdgpu_waves_per_eu(4)))
assemble_batched_kernel(const BatchItem *__restrict__ items, int count, int gi) {
    const BatchItem &it = items[batch_of(items, count, blockIdx.x, 1)];
    StepArgs a = it.a;
    a.flags = &it.rep[gi].flags;
    assemble_rows_body<K, W>(a, it.s, (int)blockIdx.x - it.row0);
}

__global__ void __launch_bounds__(256) node_energy_batched_kernel(const BatchItem *__restrict__ items, int count) {
    const BatchItem &it = items[batch_of(items, count, blockIdx.x, 2)];
    node_energy_body(it.a, it.s, (int)blockIdx.x - it.ne0);
}

// One workgroup per problem.
__global__ void __launch_bounds__(256) energy_report_batched_kernel(const BatchItem *__restrict__ items, int gi,
                                                                    unsigned *__restrict__ zero_words,
                                                                    int zero_count) {
    const BatchItem &it = items[blockIdx.x];
    energy_report_body(it.s.pt_part, it.npb, it.s.node_part, it.a.nd.m, it.rep + gi, it.reject,
                       blockIdx.x == 0 ? zero_words : nullptr, zero_count);
}

hipError_t launch_point_pass_batched(const BatchItem *items, int count, int k, int64_t total_blocks, int it,
                                     hipStream_t st) {
    (void)it;
    if (total_blocks <= 0) return hipSuccess;
    switch (k) {
#define MSL_PB_CASE(KK)                                                                                          \
    case KK:                                                                                                     \
        hipLaunchKernelGGL((point_pass_batched_kernel<KK>), dim3((unsigned)total_blocks), dim3(kPtBlock), 0, st, \
                           items, count);                                                                        \
        break;
        MSL_PB_CASE(1) MSL_PB_CASE(2) MSL_PB_CASE(3) MSL_PB_CASE(4)
        MSL_PB_CASE(5) MSL_PB_CASE(6) MSL_PB_CASE(7) MSL_PB_CASE(8)
#undef MSL_PB_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_list_pack_batched(const BatchItem *items, int count, int k, int total_rows, hipStream_t st) {
    if (total_rows <= 0) return hipSuccess;
    switch (k) {
#define MSL_LB_CASE(KK)                                                                                          \
    case KK:                                                                                                     \
        hipLaunchKernelGGL((list_pack_batched_kernel<KK>), dim3(total_rows), dim3(256), 0, st, items, count); \
        break;
        MSL_LB_CASE(1) MSL_LB_CASE(2) MSL_LB_CASE(3) MSL_LB_CASE(4)
        MSL_LB_CASE(5) MSL_LB_CASE(6) MSL_LB_CASE(7) MSL_LB_CASE(8)
#undef MSL_LB_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_assemble_batched(const BatchItem *items, int count, int k, int total_rows, int it, int waves,
                                   hipStream_t st) {
    if (total_rows <= 0) return hipSuccess;
    const bool one = waves == 1;
    switch (k) {
#define MSL_AB_CASE(KK)                                                                                          \
    case KK:                                                                                                     \
        if (one)                                                                                                 \
            hipLaunchKernelGGL((assemble_batched_kernel<KK, 1>), dim3(total_rows), dim3(kWave), 0, st, items,    \
                               count, it);                                                                       \
        else                                                                                                     \
            hipLaunchKernelGGL((assemble_batched_kernel<KK, 2>), dim3(total_rows), dim3(2 * kWave), 0, st, items,\
                               count, it);                                                                       \
        break;
        MSL_AB_CASE(1) MSL_AB_CASE(2) MSL_AB_CASE(3) MSL_AB_CASE(4)
        MSL_AB_CASE(5) MSL_AB_CASE(6) MSL_AB_CASE(7) MSL_AB_CASE(8)
#undef MSL_AB_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_energy_report_batched(const BatchItem *items, int count, int it, unsigned *zero_words,
                                        int zero_count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (zero_count < 0 || zero_count > MSL_BAR_WORDS || zero_count % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(energy_report_batched_kernel, dim3(count), dim3(256), 0, st, items, it, zero_words,
                       zero_count);
    return hipGetLastError();
}

hipError_t launch_node_energy_batched(const BatchItem *items, int count, int total_blocks, hipStream_t st) {
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(node_energy_batched_kernel, dim3(total_blocks), dim3(256), 0, st, items, count);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace msl
