// Linear solve of the Gauss-Newton step (Sec. II-F): block-Jacobi preconditioned
// conjugate gradients on (H + lambda I) dx = -g over the block pattern.
//
// Float32 block products and vector updates, float64 reductions.  Each
// reduction is a two-level fixed-order sum: a block tree per workgroup, then
// every consumer workgroup re-adds the per-workgroup partials in the same
// order, so every workgroup sees the same scalars and the result is bitwise
// reproducible.  The recurrence is the textbook PCG with the direction
// product folded as q = A z + beta q (A p with p = z + beta p, unchanged in
// exact arithmetic), which needs one workgroup-wide sync less per iteration.
#include <hip/hip_cooperative_groups.h>

#include "frame.h"

namespace msl {

constexpr int kRowsPerBlk = 21;          // 12 threads per row
constexpr int kPcgThreads = 256;

// ---------------------------------------------------------------- block-Jacobi preconditioner

// One wave per node: M_j = (H_jj + lambda I)^-1 by a float64 Cholesky in LDS.
// A non-SPD block gets M_j = I and raises MISSLAM_FLAG_NONSPD_BLOCK.
__global__ void __launch_bounds__(64) bjacobi_kernel(const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col_idx,
                                                      const float *__restrict__ blocks, int m, int cap, float lambda,
                                                      float *__restrict__ minv, int32_t *__restrict__ flags) {
    __shared__ double A[12][12];
    __shared__ double Li[12][12];
    const int j = blockIdx.x;
    int pd = -1;
    const int pe = min(row_ptr[j + 1], cap);
    for (int p = row_ptr[j]; p < pe; ++p)
        if (col_idx[p] == j) pd = p;
    for (int t = threadIdx.x; t < 144; t += 64) {
        const int i = t / 12, c = t % 12;
        double v = pd >= 0 ? (double)blocks[(size_t)pd * 144 + t] : 0.0;
        if (i == c) v += (double)lambda;
        A[i][c] = v;
    }
    __syncthreads();
    const bool ok = chol_inverse_wave(A, Li, minv + (size_t)j * 144);
    if (!ok && threadIdx.x == 0) atomicOr(flags, MISSLAM_FLAG_NONSPD_BLOCK);
}

hipError_t launch_bjacobi(const GraphView &g, int m, const float *blocks, float lambda, float *minv, int32_t *flags,
                          hipStream_t st) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(bjacobi_kernel, dim3(m), dim3(64), 0, st, g.row_ptr, g.col_idx, blocks, m, g.bsr_cap,
                       lambda, minv, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------- PCG

__global__ void fill_u32_kernel_pcg(unsigned *p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}


__device__ __forceinline__ double gather_sum(const double *part, int nblk, double *lds) {
    double s = 0.0;
    for (int t = threadIdx.x; t < nblk; t += kPcgThreads) s += part[t];
    return block_sum<kPcgThreads>(s, lds);
}

// z_j = M_j r_j for the rows of this block; rl holds the block's r values.
__device__ __forceinline__ float precond_row(const float *minv, int j, int a, const float *rl) {
    const float *M = minv + (size_t)j * 144 + a * 12;
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < 12; ++b) s = fmaf(M[b], rl[b], s);
    return s;
}

__global__ void __launch_bounds__(kPcgThreads) pcg_init_kernel(PcgArgs A) {
    __shared__ double red[kPcgThreads];
    __shared__ float rl[kRowsPerBlk][12];
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kRowsPerBlk + row;
    const bool act = row < kRowsPerBlk && j < A.m;
    float r = 0.f, z = 0.f;
    if (act) {
        r = -A.g[(size_t)j * 12 + a];
        rl[row][a] = r;
    }
    __syncthreads();
    if (act) {
        z = precond_row(A.minv, j, a, rl[row]);
        A.r[(size_t)j * 12 + a] = r;
        A.z[(size_t)j * 12 + a] = z;
        A.x[(size_t)j * 12 + a] = 0.f;
    }
    const double rz = block_sum<kPcgThreads>((double)r * (double)z, red);
    const double rr = block_sum<kPcgThreads>((double)r * (double)r, red);
    if (threadIdx.x == 0) {
        A.part[(0 * 4 + 0) * A.nblk + blockIdx.x] = rz;
        A.part[(0 * 4 + 1) * A.nblk + blockIdx.x] = rr;
        A.part[(0 * 4 + 3) * A.nblk + blockIdx.x] = 0.0;
    }
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t <= A.iters; t += kPcgThreads) {
            A.status[t] = 0;
            A.done[t] = 0;
        }
}

// Direction update and product: p = z + beta p, q = (H + lambda I) z + beta q, partial p.q.
__global__ void __launch_bounds__(kPcgThreads) pcg_dir_kernel(PcgArgs A, int it) {
    __shared__ double red[kPcgThreads];
    const double rz = gather_sum(A.part + (size_t)(it * 4 + 0) * A.nblk, A.nblk, red);
    const double rz_prev = it > 0 ? gather_sum(A.part + (size_t)((it - 1) * 4 + 0) * A.nblk, A.nblk, red) : 1.0;
    const bool skip = A.status[it] != 0 || rz == 0.0;
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kRowsPerBlk + row;
    const bool act = row < kRowsPerBlk && j < A.m && !skip;
    double pq = 0.0;
    if (act) {
        const float beta = it > 0 ? (float)(rz / rz_prev) : 0.f;
        // float32 products summed exactly in float64: the regulariser blocks
        // cancel each other to a small product, which float32 sums would blur
        double az = 0.0;
        const int p0 = A.row_ptr[j], p1 = min(A.row_ptr[j + 1], A.cap);
        for (int pb = p0; pb < p1; ++pb) {
            const int l = A.col_idx[pb];
            const float *B = A.blocks + (size_t)pb * 144 + a * 12;
            const float *zl = A.z + (size_t)l * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) az = fma((double)B[b], (double)zl[b], az);
        }
        const size_t o = (size_t)j * 12 + a;
        const float zj = A.z[o];
        az = fma((double)(A.lambda_dev ? *A.lambda_dev : A.lambda), (double)zj, az);
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
    const double t = block_sum<kPcgThreads>(pq, red);
    if (threadIdx.x == 0) A.part[(size_t)(it * 4 + 2) * A.nblk + blockIdx.x] = t;
}

// Step: alpha = r.z / p.q, x += alpha p, r -= alpha q, z = M r; partial r.z and r.r of the new residual.
__global__ void __launch_bounds__(kPcgThreads) pcg_step_kernel(PcgArgs A, int it) {
    __shared__ double red[kPcgThreads];
    __shared__ float rl[kRowsPerBlk][12];
    const double rz = gather_sum(A.part + (size_t)(it * 4 + 0) * A.nblk, A.nblk, red);
    const double pq = gather_sum(A.part + (size_t)(it * 4 + 2) * A.nblk, A.nblk, red);
    const int st = A.status[it];
    const bool skip = st != 0 || rz == 0.0;
    const bool brk = !skip && !(pq > 0.0);
    const bool upd = !skip && !brk;
    const int row = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = blockIdx.x * kRowsPerBlk + row;
    const bool in = row < kRowsPerBlk && j < A.m;
    const size_t o = (size_t)j * 12 + a;
    float r = 0.f;
    double bad = 0.0;
    if (in) {
        r = A.r[o];
        float xv = A.x[o];
        if (upd) {
            const float alpha = (float)(rz / pq);
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
            z = precond_row(A.minv, j, a, rl[row]);
            A.z[o] = z;
        } else {
            z = A.z[o];
        }
    }
    const double rzn = block_sum<kPcgThreads>((double)r * (double)z, red);
    const double rrn = block_sum<kPcgThreads>((double)r * (double)r, red);
    const double nb = block_sum<kPcgThreads>(bad, red);
    if (threadIdx.x == 0) {
        A.part[(size_t)((it + 1) * 4 + 0) * A.nblk + blockIdx.x] = rzn;
        A.part[(size_t)((it + 1) * 4 + 1) * A.nblk + blockIdx.x] = rrn;
        A.part[(size_t)((it + 1) * 4 + 3) * A.nblk + blockIdx.x] = nb;
        if (blockIdx.x == 0) {
            A.status[it + 1] = st != 0 ? st : (brk ? 2 : 0);
            A.done[it] = upd ? 1 : 0;
        }
    }
}

// Residual norms, iterations done and flags (block 0); every block applies
// params += x to its slice unless x holds a non-finite value anywhere.
__global__ void __launch_bounds__(kPcgThreads) pcg_finish_kernel(PcgArgs A, misslam_report *rep,
                                                                float *__restrict__ params) {
    __shared__ double red[kPcgThreads];
    const double nbad = gather_sum(A.part + (size_t)(A.iters * 4 + 3) * A.nblk, A.nblk, red);
    const int total = A.m * 12;
    const int t = blockIdx.x * kPcgThreads + threadIdx.x;
    if (params && nbad == 0.0 && t < total) params[t] += A.x[t];
    if (blockIdx.x != 0) return;
    int done = 0;
    for (int q = 0; q < A.iters; ++q) done += A.done[q];
    for (int q = 0; q <= done; ++q) {
        const double rr = gather_sum(A.part + (size_t)(q * 4 + 1) * A.nblk, A.nblk, red);
        if (threadIdx.x == 0 && q <= MISSLAM_MAX_PCG) rep->pcg_resid[q] = sqrt(rr);
    }
    if (threadIdx.x == 0) {
        rep->pcg_iters_done = done;
        int f = rep->flags;
        if (A.status[A.iters] & 2) f |= MISSLAM_FLAG_PCG_BREAKDOWN;
        if (nbad != 0.0) f |= MISSLAM_FLAG_NONFINITE;
        rep->flags = f;
    }
}

hipError_t launch_pcg_update(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                             float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                             float *params, hipStream_t st, const float *lambda_dev) {
    PcgArgs A;
    A.row_ptr = g.row_ptr;
    A.col_idx = g.col_idx;
    A.blocks = blocks;
    A.minv = minv;
    A.g = gvec;
    A.lambda = lambda;
    A.lambda_dev = lambda_dev;
    A.m = m;
    A.nblk = s.nblk;
    A.iters = iters;
    A.cap = g.bsr_cap;
    A.x = delta;
    A.r = s.r;
    A.z = s.z;
    A.p = s.p;
    A.q = s.q;
    A.part = s.part;
    A.status = s.status;
    A.done = s.status + (iters + 2);
    const dim3 grid(s.nblk), blk(kPcgThreads);
    hipLaunchKernelGGL(pcg_init_kernel, grid, blk, 0, st, A);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(pcg_dir_kernel, grid, blk, 0, st, A, it);
        hipLaunchKernelGGL(pcg_step_kernel, grid, blk, 0, st, A, it);
    }
    hipLaunchKernelGGL(pcg_finish_kernel, dim3((12 * m + kPcgThreads - 1) / kPcgThreads), blk, 0, st, A, rep,
                       params);
    return hipGetLastError();
}

__global__ void report_init_batched_kernel(const BatchItem *__restrict__ items, int per_problem) {
    misslam_report *rep = items[blockIdx.x].rep;
    const int32_t *info = items[blockIdx.x].a.g.info;
    const int gf = info[3] != 0 ? MISSLAM_FLAG_GRAPH_OVERFLOW : 0;
    for (int t = threadIdx.x; t < per_problem; t += blockDim.x) {
        rep[t].e_data = 0.0;
        rep[t].e_rot = 0.0;
        rep[t].e_reg = 0.0;
        for (int q = 0; q <= MISSLAM_MAX_PCG; ++q) rep[t].pcg_resid[q] = 0.0;
        rep[t].n_valid = 0;
        rep[t].flags = gf;
        rep[t].pcg_iters_done = 0;
        rep[t].reserved = 0;
        rep[t].e_corr = 0.0;
        rep[t].lm_e = 0.0;
        rep[t].lm_e_trial = 0.0;
        rep[t].lm_lambda = 0.f;
        rep[t].lm_accepted = 0;
        rep[t].e_pose_r = 0.0;
        rep[t].e_pose_p = 0.0;
    }
}

hipError_t launch_report_init_batched(const BatchItem *items, int count, int per_problem, hipStream_t st) {
    if (count <= 0 || per_problem <= 0) return hipSuccess;
    hipLaunchKernelGGL(report_init_batched_kernel, dim3(count), dim3(64), 0, st, items, per_problem);
    return hipGetLastError();
}

__global__ void report_init_kernel(misslam_report *rep, int count, const int32_t *graph_info) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        const int gf = graph_info && graph_info[3] != 0 ? MISSLAM_FLAG_GRAPH_OVERFLOW : 0;
        rep[t].e_data = 0.0;
        rep[t].e_rot = 0.0;
        rep[t].e_reg = 0.0;
        for (int q = 0; q <= MISSLAM_MAX_PCG; ++q) rep[t].pcg_resid[q] = 0.0;
        rep[t].n_valid = 0;
        rep[t].flags = gf;
        rep[t].pcg_iters_done = 0;
        rep[t].reserved = 0;
        rep[t].e_corr = 0.0;
        rep[t].lm_e = 0.0;
        rep[t].lm_e_trial = 0.0;
        rep[t].lm_lambda = 0.f;
        rep[t].lm_accepted = 0;
        rep[t].e_pose_r = 0.0;
        rep[t].e_pose_p = 0.0;
    }
}

hipError_t launch_report_init(misslam_report *rep, int count, hipStream_t st, const int32_t *graph_info) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(report_init_kernel, dim3((count + 63) / 64), dim3(64), 0, st, rep, count, graph_info);
    return hipGetLastError();
}

int pcg_blocks(int m) { return (m + kRowsPerBlk - 1) / kRowsPerBlk; }

// ---------------------------------------------------------------- persistent PCG (one cooperative launch)

// The same recurrence in one launch.  Each workgroup owns a contiguous range
// of up to kRowsPerBlk rows and keeps their H blocks (as many as fit), their
// preconditioner blocks and its slice of x, r, p, q in LDS.  Between
// workgroups only z and the reduction partials travel, through device-scope
// loads and stores (coherent across the XCDs' separate L2 caches without
// cache maintenance).  There is no grid barrier: the two reductions of an
// iteration (p.q, then r.z) are exchanged as tagged words, and a workgroup
// publishes its r.z partial only after its z stores are acknowledged, so the
// wait for the r.z partials is also the wait for the z that the next product
// reads.  Every reduction is re-added by every workgroup in the same order,
// so all take identical decisions.
constexpr int kPersistMaxLds = 160 * 1024;   // LDS of one CU (gfx950)

__device__ __forceinline__ void st_dev(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_dev(const float *p) {
    return __hip_atomic_load(const_cast<float *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The polls of one wait are bounded (PcgArgs::spin).  A workgroup that gives
// up (which a launch whose workgroups are all resident never causes) stops
// waiting from then on and the solve reports it; the step is then discarded
// as a whole by step_commit_kernel, which runs after the solve.

// Sum of up to three doubles over the workgroup: wave butterflies, then the
// waves in order (fixed order: bitwise reproducible).
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double (*lds)[kPcgThreads / kWave]) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double t[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) t[q] = v[q];
    wave_sums(t);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q][wave] = t[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = lds[q][0];
#pragma unroll
        for (int w = 1; w < kPcgThreads / kWave; ++w) t += lds[q][w];
        v[q] = t;
    }
    __syncthreads();
}

// Fixed-order sum of the G partials of one reduction (device-scope loads).
__device__ __forceinline__ double gather_dev(const double *part, int G, double (*lds)[kPcgThreads / kWave]) {
    double v[1] = {0.0};
    for (int t = threadIdx.x; t < G; t += kPcgThreads) v[0] += ld_dev(part + t);
    wg_sum<1>(v, lds);
    return v[0];
}

// Tagged exchange of one double per workgroup, the synchronisation of the
// solve: workgroup g of the launch owns 4 eight-byte words of the sync area,
// (high half | tag, low half | tag) for the direction product and the same for
// r.z.  Each 8-byte word is stored and loaded whole (device scope), so a
// reader that finds the expected tag in both words holds both halves of the
// value published with it.  A slot is rewritten two exchanges later, which no
// workgroup reaches before every workgroup has read it.  The words must be
// zero at launch (tags start at 1).
__device__ __forceinline__ unsigned long long *tag_slots(unsigned *bar) {
    return reinterpret_cast<unsigned long long *>(bar);
}

__device__ __forceinline__ void tag_publish(unsigned *bar, int gid, int which, unsigned tag, double v) {
    unsigned long long *w = tag_slots(bar) + 4 * gid + 2 * which;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    __hip_atomic_store(w, (bits & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (bits << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-order sum of the values that workgroups g0 .. g0+G-1 published with
// `tag`, waiting for each (bounded: a timeout marks the workgroup broken).
__device__ __forceinline__ double tag_sum(unsigned *bar, int g0, int G, int which, unsigned tag, bool &broken,
                                          double (*lds)[kPcgThreads / kWave], unsigned spin_limit) {
    const unsigned long long *base = tag_slots(bar) + 2 * which;
    double v[1] = {0.0};
    bool ok = true;
    for (int t = threadIdx.x; t < G; t += kPcgThreads) {
        unsigned long long *w = const_cast<unsigned long long *>(base) + 4 * (g0 + t);
        unsigned long long hi = 0, lo = 0;
        unsigned spins = 0;
        for (;;) {
            hi = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            lo = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)hi == tag && (unsigned)lo == tag) break;
            if (broken || ++spins > spin_limit) {
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok) v[0] += __longlong_as_double((long long)((hi & 0xFFFFFFFF00000000ull) | (lo >> 32)));
    }
    broken = __syncthreads_or(broken || !ok) != 0;
    wg_sum<1>(v, lds);
    return v[0];
}

constexpr int kMaxBlocksWg = kRowsPerBlk * MISSLAM_MAX_ROW;   // blocks of one workgroup's rows
constexpr int kMaxUnique = 192;                                // distinct columns staged per iteration
constexpr int kZPer = (kMaxUnique * 6 + kPcgThreads - 1) / kPcgThreads;

__device__ __forceinline__ unsigned long long ld_dev64(const float *p) {
    return __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<float *>(p)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// LDS of one workgroup's share of a one-launch solve besides the cached blocks: the columns of its blocks
// reduced to their distinct nodes (each staged once per iteration).
struct TileLds {
    int bmap[kMaxBlocksWg];                 // block -> distinct-column slot (-1: beyond the cap)
    int colL[kMaxBlocksWg];                 // column of each block
    int scan_w[kPcgThreads / kWave];
    int ucol[kMaxUnique];                   // node of each distinct-column slot
    int cnt_u, cmin_s, cmax_s;
    int lslot[kRowsPerBlk];                 // staged slot of each of this workgroup's own columns (-1: none)
};

struct TileRange {
    int r0, r1;      // rows [r0, r1)
    int b0, nb;      // their blocks [b0, b0 + nb) of the system
    int cached;      // blocks held in LDS (the first `cached`)
    int U;           // distinct columns with a slot
};

// n float4 from src (global) straight into LDS at dst, 16 bytes per lane (global_load_lds_dwordx4: lane i of a
// wave fills dst + i, dst the same for the whole wave), every load in flight at once and no registers held.
// The caller waits (vmcnt) and synchronises before reading dst.
__device__ __forceinline__ void lds_copy16(const float4 *src, float4 *dst, int n) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int q0 = wave * kWave; q0 < n; q0 += kPcgThreads)
        if (q0 + lane < n)
            __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + q0 + lane),
                                             (__attribute__((address_space(3))) void *)(dst + q0), 16, 0, 0);
}

// Setup of workgroup wg's share: its rows' blocks (as many as fit) into hc, their preconditioner blocks into
// mc, and the distinct-column map with at most max_unique (<= kMaxUnique) slots.  firstmap: map_ints ints of
// scratch LDS (free again on return).
__device__ __forceinline__ TileRange tile_setup(const PcgArgs &A, int rows_per_wg, int cache_blocks, int wg,
                                                float4 *hc4, float *mc, TileLds &t, int *firstmap, int map_ints,
                                                int max_unique) {
    TileRange R;
    R.r0 = min(A.m, wg * rows_per_wg);
    R.r1 = min(A.m, R.r0 + rows_per_wg);
    R.b0 = min(A.row_ptr[R.r0], A.cap);
    const int b1 = min(A.row_ptr[R.r1], A.cap);
    R.nb = min(b1 - R.b0, kMaxBlocksWg);
    R.cached = min(R.nb, cache_blocks);
    // distinct columns: a block whose column appears at no earlier block of the workgroup gets the next
    // slot (in block order, by a workgroup scan); later blocks of that column share it
    if (threadIdx.x == 0) {
        t.cmin_s = 0x7FFFFFFF;
        t.cmax_s = -1;
    }
    if (threadIdx.x < kRowsPerBlk) t.lslot[threadIdx.x] = -1;
    __syncthreads();
    const int nb = R.nb, b0 = R.b0, r0 = R.r0, r1 = R.r1;
    for (int q = threadIdx.x; q < nb; q += kPcgThreads) {
        const int c = A.col_idx[b0 + q];
        t.colL[q] = c;
        atomicMin(&t.cmin_s, c);
        atomicMax(&t.cmax_s, c);
    }
    // the cached blocks and the rows' preconditioner blocks, straight into LDS: they arrive while the rest of
    // the map is built (LDS work only), and are waited for at its end
    lds_copy16(reinterpret_cast<const float4 *>(A.blocks + (size_t)R.b0 * 144), hc4, R.cached * 36);
    lds_copy16(reinterpret_cast<const float4 *>(A.minv + (size_t)R.r0 * 144), reinterpret_cast<float4 *>(mc),
               (R.r1 - R.r0) * 36);
    __syncthreads();
    const int cmin = t.cmin_s, crange = t.cmax_s - t.cmin_s + 1;
    const bool mapped = nb > 0 && crange <= map_ints;
    if (mapped) {
        for (int q = threadIdx.x; q < crange; q += kPcgThreads) firstmap[q] = 0x7FFFFFFF;
        __syncthreads();
        for (int q = threadIdx.x; q < nb; q += kPcgThreads) atomicMin(&firstmap[t.colL[q] - cmin], q);
        __syncthreads();
    }
    constexpr int kPerT = (kMaxBlocksWg + kPcgThreads - 1) / kPcgThreads;   // entries per thread in the scan
    int firstpos[kPerT];
    int nfirst = 0;
#pragma unroll
    for (int e = 0; e < kPerT; ++e) {
        const int q = threadIdx.x * kPerT + e;
        firstpos[e] = -1;
        if (q < nb) {
            const int c = t.colL[q];
            int f = q;
            if (mapped) {
                f = firstmap[c - cmin];
            } else {
                for (int u = 0; u < q; ++u)
                    if (t.colL[u] == c) {
                        f = u;
                        break;
                    }
            }
            firstpos[e] = f;
            nfirst += f == q;
        }
    }
    __syncthreads();   // the map's space is free again
    // exclusive scan of nfirst over the workgroup: wave scans, then the waves in order
    {
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        int incl = nfirst;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int v = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += v;
        }
        if (lane == kWave - 1) t.scan_w[wave] = incl;
        __syncthreads();
        int base = 0;
        for (int w = 0; w < wave; ++w) base += t.scan_w[w];
        int slot = base + incl - nfirst;
#pragma unroll
        for (int e = 0; e < kPerT; ++e) {
            const int q = threadIdx.x * kPerT + e;
            if (q < nb && firstpos[e] == q) {
                const int sl = slot < max_unique ? slot : -1;
                if (sl >= 0) t.ucol[sl] = t.colL[q];
                if (sl >= 0 && t.colL[q] >= r0 && t.colL[q] < r1) t.lslot[t.colL[q] - r0] = sl;
                t.bmap[q] = sl;
                ++slot;
            }
        }
        if (threadIdx.x == kPcgThreads - 1) {
            int tot = 0;
            for (int w = 0; w < kPcgThreads / kWave; ++w) tot += t.scan_w[w];
            t.cnt_u = tot < max_unique ? tot : max_unique;
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPerT; ++e) {
        const int q = threadIdx.x * kPerT + e;
        if (q < nb && firstpos[e] != q) t.bmap[q] = t.bmap[firstpos[e]];   // a first occurrence: already set
    }
    __builtin_amdgcn_s_waitcnt(0);   // this wave's LDS loads have landed (vmcnt); the barrier covers every wave's
    __syncthreads();
    R.U = t.cnt_u;
    return R;
}

// Joint form (pose + ED unknowns, Eq.(10)): the six pose unknowns border the
// ED system, [[H, B], [B^T, H_pp]].  Their part of every vector (r, z, p, q, x
// of the pose) is recomputed identically by every workgroup from the same
// exchanged sums, so it never travels.  B^T z uses the z of the previous step,
// so its partial sums ride in the r.z exchange (7 values) and the p.q exchange
// stays one value: the same two exchanges per iteration as the ED-only solve.
// Sync area: kJointTagWords 8-byte words per workgroup, the p.q value in words
// 0-1 and the r.z, B^T z values in words 2-15 (high half | tag, low half | tag).
constexpr int kPoseThread = kPcgThreads - 1;   // never holds an ED entry (kRowsPerBlk * 12 < kPcgThreads)

template <int N>
__device__ __forceinline__ void tagn_publish(unsigned *bar, int gid, int word0, unsigned tag, const double (&v)[N]) {
    unsigned long long *w = tag_slots(bar) + (size_t)kJointTagWords * gid + word0;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(v[q]);
        __hip_atomic_store(w + 2 * q, (bits & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 2 * q + 1, (bits << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The workgroup's publication: once every wave's device-scope stores are acknowledged.
template <int N>
__device__ __forceinline__ void tagn_publish_wg(unsigned *bar, int gid, int word0, unsigned tag,
                                                const double (&v)[N]) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) tagn_publish<N>(bar, gid, word0, tag, v);
}

// Fixed-order sums of the N values that workgroups g0 .. g0+G-1 published with `tag` (bounded waits).
template <int N>
__device__ __forceinline__ void tagn_sum(unsigned *bar, int g0, int G, int word0, unsigned tag, bool &broken,
                                         double (*lds)[kPcgThreads / kWave], unsigned spin_limit, double (&out)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = 0.0;
    bool ok = true;
    for (int t = threadIdx.x; t < G; t += kPcgThreads) {
        unsigned long long *w = tag_slots(bar) + (size_t)kJointTagWords * (g0 + t) + word0;
        unsigned long long hv[N], lv[N];
        unsigned spins = 0;
        for (;;) {
            bool all = true;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                hv[q] = __hip_atomic_load(w + 2 * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                lv[q] = __hip_atomic_load(w + 2 * q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                all = all && (unsigned)hv[q] == tag && (unsigned)lv[q] == tag;
            }
            if (all) break;
            if (broken || ++spins > spin_limit) {
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok)
#pragma unroll
            for (int q = 0; q < N; ++q)
                out[q] += __longlong_as_double((long long)((hv[q] & 0xFFFFFFFF00000000ull) | (lv[q] >> 32)));
    }
    broken = __syncthreads_or(broken || !ok) != 0;
    wg_sum<N>(out, lds);
}

// The pose part of one iteration's direction (one thread; ps = pose r, z, p, q, x in LDS, the same in every
// workgroup): q_p = (H_pp + lambda I) z_p + sum_j B_j^T z_j + beta q_p, p_p = z_p + beta p_p; returns p_p.q_p.
__device__ __forceinline__ double pose_direction(double *ps, const double *sysl, const double (&btz)[6], double lam,
                                                 int it, float beta) {
    double z[6], qp[6], pp[6], t = 0.0;
#pragma unroll
    for (int u = 0; u < 6; ++u) z[u] = ps[6 + u];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        double az = btz[u];
#pragma unroll
        for (int w = 0; w < 6; ++w) az += sysl[6 * u + w] * z[w];
        az += lam * z[u];
        qp[u] = it > 0 ? (double)beta * ps[18 + u] + az : az;
        pp[u] = it > 0 ? (double)beta * ps[12 + u] + z[u] : z[u];
        t += pp[u] * qp[u];
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        ps[12 + u] = pp[u];
        ps[18 + u] = qp[u];
    }
    return t;
}

// The pose part of one step: x_p += alpha p_p, r_p -= alpha q_p, z_p = (H_pp + lambda I)^-1 r_p; out = r_p.z_p,
// r_p.r_p and the count of non-finite x_p.
__device__ __forceinline__ void pose_step(double *ps, const double *sysl, float alpha, double (&out)[3]) {
    double r[6], nb = 0.0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        const double x = ps[24 + u] + (double)alpha * ps[12 + u];
        r[u] = ps[u] - (double)alpha * ps[18 + u];
        ps[24 + u] = x;
        ps[u] = r[u];
        if (!isfinite(x)) nb += 1.0;
    }
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 6; ++w) t += sysl[42 + 6 * u + w] * r[w];
        ps[6 + u] = t;
        rz += r[u] * t;
        rr += r[u] * r[u];
    }
    out[0] = rz;
    out[1] = rr;
    out[2] = nb;
}

// One workgroup's share of the solve: workgroup wg of the G that own this
// system's rows, which are workgroups gid0 .. gid0+G-1 of the launch (a batch
// solves several systems side by side, each over its own sync slots).  The
// columns of the workgroup's blocks are reduced to their distinct nodes once;
// each iteration stages z of those nodes in LDS (8-byte device-scope loads,
// all in flight together).  kJoint: the joint form above (one system, first
// workgroup of the launch at gid0 = 0; bar is its own sync area).
template <bool kJoint>
__device__ __forceinline__ void pcg_persistent_body(const PcgArgs &A, int rows_per_wg, int cache_blocks, unsigned *bar,
                                                    int gid0, int wg, int G, misslam_report *rep,
                                                    const JointExtra &jx) {
    extern __shared__ float4 dyn4[];
    __shared__ double red[kJoint ? 9 : 3][kPcgThreads / kWave];
    __shared__ float vx[kRowsPerBlk * 12], vr[kRowsPerBlk * 12], vp[kRowsPerBlk * 12], vq[kRowsPerBlk * 12];
    __shared__ TileLds tl;
    __shared__ float4 zc4[kMaxUnique * 3];             // z of the distinct columns (setup: first-block map)
    // joint form: the pose part (r, z, p, q, x of the pose), H_pp | g_p | (H_pp + lambda I)^-1, this iteration's
    // p_p.q_p, the pose step's r_p.z_p, r_p.r_p, #non-finite x_p, and r_p.r_p after each step (for the report)
    __shared__ double ps[kJoint ? 30 : 1], sysl[kJoint ? 78 : 1], pose_s[kJoint ? 4 : 1];
    __shared__ double rrp[kJoint ? MISSLAM_MAX_PCG + 1 : 1];
    float *zc = reinterpret_cast<float *>(zc4);
    const double lam = (double)(A.lambda_dev ? *A.lambda_dev : A.lambda);
    float *hc = reinterpret_cast<float *>(dyn4);       // cached blocks
    float *mc = hc + (size_t)cache_blocks * 144;       // preconditioner blocks of the rows
    const int lr = threadIdx.x / 12, a = threadIdx.x % 12;
    // what does not depend on the setup is requested before it, so its latency hides behind the block copy:
    // this thread's gradient entry and its row's block range (and, joint form, its row of the border)
    const int r0e = min(A.m, wg * rows_per_wg), r1e = min(A.m, r0e + rows_per_wg);
    const bool act = lr < kRowsPerBlk && r0e + lr < r1e;
    float g_own = 0.f;
    int rp0 = 0, rp1 = 0;
    float brow[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // joint: this entry's row of the border
    if (act) {
        g_own = A.g[(size_t)(r0e + lr) * 12 + a];
        rp0 = A.row_ptr[r0e + lr];
        rp1 = A.row_ptr[r0e + lr + 1];
        if constexpr (kJoint)
#pragma unroll
            for (int k = 0; k < 6; ++k) brow[k] = jx.B[(size_t)(r0e + lr) * 72 + a * 6 + k];
    }
    const TileRange R = tile_setup(A, rows_per_wg, cache_blocks, wg, dyn4, mc, tl, reinterpret_cast<int *>(zc4),
                                   kMaxUnique * 12, kMaxUnique);
    const int r0 = R.r0, r1 = R.r1, b0 = R.b0, nb = R.nb, cached = R.cached, U = R.U;
    const int *bmap = tl.bmap, *colL = tl.colL, *ucol = tl.ucol, *lslot = tl.lslot;
    const int j = r0 + lr;
    const int li = lr * 12 + a;
    bool broken = false;
    // this thread's row: its blocks q in [rq0, rq1) of the workgroup; fast = all cached with a staged column
    const int rq0 = act ? min(rp0, A.cap) - b0 : 0;
    const int rq1 = act ? min(rp1, A.cap) - b0 : 0;
    bool fast = rq1 <= cached;
    for (int q = rq0; q < rq1 && fast; ++q) fast = bmap[q] >= 0;
    // Blocks whose column is one of this workgroup's own rows (bit i: block rq0 + i, fast rows only): their
    // z is produced here and written straight into its staged slot, so their part of the next product is
    // formed while the r.z exchange is in flight; the other blocks wait for the exchange.
    uint32_t lmask = 0, rmask = 0;
    if (act && fast)
        for (int q = rq0; q < rq1; ++q) {
            if (colL[q] >= r0 && colL[q] < r1)
                lmask |= 1u << (q - rq0);
            else
                rmask |= 1u << (q - rq0);
        }
    const int zslot = act ? lslot[lr] : -1;   // staged slot of this row's own column (-1: none)
    // product of one block (workgroup block q, staged column slot sl) and z, into chain t
    auto block_dot = [&](int q, double t) {
        const float4 *Bq = reinterpret_cast<const float4 *>(hc + (size_t)q * 144 + a * 12);
        const float4 *zq = zc4 + bmap[q] * 3;
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            const float4 b4 = Bq[h], z4 = zq[h];
            t = fma((double)b4.x, (double)z4.x, t);
            t = fma((double)b4.y, (double)z4.y, t);
            t = fma((double)b4.z, (double)z4.z, t);
            t = fma((double)b4.w, (double)z4.w, t);
        }
        return t;
    };
    // the local part of the product (own columns, in block order)
    auto local_part = [&]() {
        double t = 0.0;
        for (uint32_t mk = lmask; mk; mk &= mk - 1) t = block_dot(rq0 + __builtin_ctz(mk), t);
        return t;
    };

    // stage z of the distinct columns owned by other workgroups, all loads in flight together (the own
    // columns' slots are written by their rows' threads)
    auto stage = [&]() {
        unsigned long long zv[kZPer];
#pragma unroll
        for (int e = 0; e < kZPer; ++e) {
            const int t = threadIdx.x + e * kPcgThreads;
            if (t < U * 6 && (ucol[t / 6] < r0 || ucol[t / 6] >= r1))
                zv[e] = ld_dev64(A.z + (size_t)ucol[t / 6] * 12 + 2 * (t % 6));
        }
#pragma unroll
        for (int e = 0; e < kZPer; ++e) {
            const int t = threadIdx.x + e * kPcgThreads;
            if (t < U * 6 && (ucol[t / 6] < r0 || ucol[t / 6] >= r1)) {
                zc[(t / 6) * 12 + 2 * (t % 6)] = __uint_as_float((unsigned)(zv[e] & 0xFFFFFFFFull));
                zc[(t / 6) * 12 + 2 * (t % 6) + 1] = __uint_as_float((unsigned)(zv[e] >> 32));
            }
        }
        __syncthreads();
    };
    // publish this workgroup's value once every wave's device-scope stores are acknowledged
    auto publish = [&](int which, unsigned tag, double v) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) tag_publish(bar, gid0 + wg, which, tag, v);
    };

    // init: r = -g, z = M r, x = 0
    float r = 0.f, z = 0.f;
    if (act) {
        r = -g_own;
        vr[li] = r;
        vx[li] = 0.f;
    }
    double btz[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};    // joint: sum_j B_j^T z_j of the current z
    if constexpr (kJoint) {
        if (threadIdx.x < 78) sysl[threadIdx.x] = jx.sys[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == kPoseThread) {   // r_p = -g_p, z_p = M_p r_p, p_p = q_p = x_p = 0
            double rp[6], rz_p = 0.0, rr_p = 0.0;
#pragma unroll
            for (int u = 0; u < 6; ++u) rp[u] = -sysl[36 + u];
#pragma unroll
            for (int u = 0; u < 6; ++u) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < 6; ++w) t += sysl[42 + 6 * u + w] * rp[w];
                ps[u] = rp[u];
                ps[6 + u] = t;
                ps[12 + u] = 0.0;
                ps[18 + u] = 0.0;
                ps[24 + u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < 6; ++u) {
                rz_p += rp[u] * ps[6 + u];
                rr_p += rp[u] * rp[u];
            }
            pose_s[1] = rz_p;
            pose_s[2] = rr_p;
            pose_s[3] = 0.0;
            rrp[0] = rr_p;
        }
    }
    __syncthreads();
    if (act) {
        const float *M = mc + (size_t)lr * 144 + a * 12;
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < 12; ++b) s = fmaf(M[b], vr[lr * 12 + b], s);
        z = s;
        st_dev(A.z + (size_t)j * 12 + a, z);
        if (zslot >= 0) zc[zslot * 12 + a] = z;
    }
    double rz, azl;
    if constexpr (kJoint) {   // r.z and B^T z travel together; the pose's r.z is added by every workgroup
        double v[8] = {(double)r * (double)z, (double)r * (double)r};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[2 + k] = (double)brow[k] * (double)z;
        wg_sum<8>(v, red);
        if (threadIdx.x == 0) st_dev(A.part + (size_t)(0 * 4 + 1) * G + wg, v[1]);
        const double pv7[7] = {v[0], v[2], v[3], v[4], v[5], v[6], v[7]};
        tagn_publish_wg<7>(bar, gid0 + wg, 2, 1u, pv7);
        azl = local_part();
        double t7[7];
        tagn_sum<7>(bar, gid0, G, 2, 1u, broken, red, A.spin, t7);
        rz = t7[0] + pose_s[1];
#pragma unroll
        for (int k = 0; k < 6; ++k) btz[k] = t7[1 + k];
        stage();
    } else {
        double v[2] = {(double)r * (double)z, (double)r * (double)r};
        wg_sum<2>(v, red);
        if (threadIdx.x == 0) st_dev(A.part + (size_t)(0 * 4 + 1) * G + wg, v[1]);
        publish(1, 1u, v[0]);
        azl = local_part();
        rz = tag_sum(bar, gid0, G, 1, 1u, broken, red, A.spin);
        stage();
    }
    bool stopped = false;
    int done = 0;
    double rz_prev = 1.0;
    for (int it = 0; it < A.iters; ++it) {
        const bool skip = stopped || rz == 0.0;
        // ---- direction and product: p = z + beta p, q = (H + lambda I) z + beta q
        double pq = 0.0;
        const float beta = it > 0 ? (float)(rz / rz_prev) : 0.f;
        if constexpr (kJoint)   // the pose part, beside the ED product (the pose thread holds no entry)
            if (threadIdx.x == kPoseThread && !skip) pose_s[0] = pose_direction(ps, sysl, btz, lam, it, beta);
        if (act && !skip) {
            double az = 0.0;                           // exact float64 sums of float32 products
            const int p0 = A.row_ptr[j], p1 = min(A.row_ptr[j + 1], A.cap);
            if (fast) {   // the local part, then the other blocks in two chains (pairs read together)
                double az1 = 0.0;
                az = azl;
                uint32_t mk = rmask;
                while (mk) {
                    const int qa = rq0 + __builtin_ctz(mk);
                    mk &= mk - 1;
                    if (mk) {
                        const int qb = rq0 + __builtin_ctz(mk);
                        mk &= mk - 1;
                        const float4 *Ba = reinterpret_cast<const float4 *>(hc + (size_t)qa * 144 + a * 12);
                        const float4 *Bb = reinterpret_cast<const float4 *>(hc + (size_t)qb * 144 + a * 12);
                        const float4 *za = zc4 + bmap[qa] * 3, *zb = zc4 + bmap[qb] * 3;
                        float4 ba[3], bb[3], zav[3], zbv[3];
#pragma unroll
                        for (int h = 0; h < 3; ++h) {
                            ba[h] = Ba[h];
                            bb[h] = Bb[h];
                            zav[h] = za[h];
                            zbv[h] = zb[h];
                        }
#pragma unroll
                        for (int h = 0; h < 3; ++h) {
                            az = fma((double)ba[h].x, (double)zav[h].x, az);
                            az1 = fma((double)bb[h].x, (double)zbv[h].x, az1);
                            az = fma((double)ba[h].y, (double)zav[h].y, az);
                            az1 = fma((double)bb[h].y, (double)zbv[h].y, az1);
                            az = fma((double)ba[h].z, (double)zav[h].z, az);
                            az1 = fma((double)bb[h].z, (double)zbv[h].z, az1);
                            az = fma((double)ba[h].w, (double)zav[h].w, az);
                            az1 = fma((double)bb[h].w, (double)zbv[h].w, az1);
                        }
                    } else {
                        az = block_dot(qa, az);
                    }
                }
                az += az1;
            } else
            for (int pb = p0; pb < p1; ++pb) {
                const int q = pb - b0;
                const int slot = q < nb ? bmap[q] : -1;
                const float *B = q < cached ? hc + (size_t)q * 144 + a * 12 : A.blocks + (size_t)pb * 144 + a * 12;
                if (slot >= 0 && q < cached) {
                    const float4 *B4 = reinterpret_cast<const float4 *>(B);
                    const float4 *z4 = zc4 + slot * 3;
#pragma unroll
                    for (int h = 0; h < 3; ++h) {
                        const float4 bv = B4[h], zv = z4[h];
                        az = fma((double)bv.x, (double)zv.x, az);
                        az = fma((double)bv.y, (double)zv.y, az);
                        az = fma((double)bv.z, (double)zv.z, az);
                        az = fma((double)bv.w, (double)zv.w, az);
                    }
                } else if (slot >= 0) {
                    const float *zl = zc + slot * 12;
#pragma unroll
                    for (int b = 0; b < 12; ++b) az = fma((double)B[b], (double)zl[b], az);
                } else {
                    const float *zl = A.z + (size_t)A.col_idx[pb] * 12;
#pragma unroll
                    for (int b = 0; b < 12; ++b) az = fma((double)B[b], (double)ld_dev(zl + b), az);
                }
            }
            az = fma(lam, (double)z, az);
            if constexpr (kJoint)   // + B_j z_p
#pragma unroll
                for (int k = 0; k < 6; ++k) az = fma((double)brow[k], ps[6 + k], az);
            const float pv = it > 0 ? fmaf(beta, vp[li], z) : z;
            const float qv = it > 0 ? (float)fma((double)beta, (double)vq[li], az) : (float)az;
            vp[li] = pv;
            vq[li] = qv;
            pq = (double)pv * (double)qv;
        }
        double pqs;
        {
            double v[1] = {pq};
            wg_sum<1>(v, red);
            if constexpr (kJoint) {
                double t1[1];
                const double pv1[1] = {v[0]};
                tagn_publish_wg<1>(bar, gid0 + wg, 0, (unsigned)(it + 1), pv1);
                tagn_sum<1>(bar, gid0, G, 0, (unsigned)(it + 1), broken, red, A.spin, t1);
                pqs = t1[0] + pose_s[0];   // + p_p.q_p, the same in every workgroup
            } else {
                publish(0, (unsigned)(it + 1), v[0]);
                pqs = tag_sum(bar, gid0, G, 0, (unsigned)(it + 1), broken, red, A.spin);
            }
        }
        // ---- step: alpha = r.z / p.q, x += alpha p, r -= alpha q, z = M r
        const bool brk = !skip && !(pqs > 0.0);
        const bool upd = !skip && !brk;
        if (act && upd) {
            const float alpha = (float)(rz / pqs);
            vx[li] = fmaf(alpha, vp[li], vx[li]);
            r = fmaf(-alpha, vq[li], r);
            vr[li] = r;
        }
        const double bad = act ? (isfinite(vx[li]) ? 0.0 : 1.0) : 0.0;
        __syncthreads();
        if (act && upd) {
            const float *M = mc + (size_t)lr * 144 + a * 12;
            float s = 0.f;
#pragma unroll
            for (int b = 0; b < 12; ++b) s = fmaf(M[b], vr[lr * 12 + b], s);
            z = s;
            st_dev(A.z + (size_t)j * 12 + a, z);
            if (zslot >= 0) zc[zslot * 12 + a] = z;
        }
        if (upd) ++done;
        if (brk) stopped = true;
        if (!skip) rz_prev = rz;
        if constexpr (kJoint) {
            double v[9] = {(double)r * (double)z, (double)r * (double)r, bad};
#pragma unroll
            for (int k = 0; k < 6; ++k) v[3 + k] = (double)brow[k] * (double)z;
            wg_sum<9>(v, red);
            if (threadIdx.x == 0) {
                st_dev(A.part + (size_t)((it + 1) * 4 + 1) * G + wg, v[1]);
                st_dev(A.part + (size_t)((it + 1) * 4 + 3) * G + wg, v[2]);
            }
            const double pv7[7] = {v[0], v[3], v[4], v[5], v[6], v[7], v[8]};
            tagn_publish_wg<7>(bar, gid0 + wg, 2, (unsigned)(it + 2), pv7);
            // the pose step, while the exchange is in flight (nothing before this point reads its results)
            if (threadIdx.x == kPoseThread && upd) {
                double o3[3];
                pose_step(ps, sysl, (float)(rz / pqs), o3);
                pose_s[1] = o3[0];
                pose_s[2] = o3[1];
                pose_s[3] = o3[2];
                rrp[min(it + 1, MISSLAM_MAX_PCG)] = o3[1];
            }
            azl = local_part();
            double t7[7];
            tagn_sum<7>(bar, gid0, G, 2, (unsigned)(it + 2), broken, red, A.spin, t7);
            rz = t7[0] + pose_s[1];
#pragma unroll
            for (int k = 0; k < 6; ++k) btz[k] = t7[1 + k];
        } else {
            double v[3] = {(double)r * (double)z, (double)r * (double)r, bad};
            wg_sum<3>(v, red);
            if (threadIdx.x == 0) {
                st_dev(A.part + (size_t)((it + 1) * 4 + 1) * G + wg, v[1]);
                st_dev(A.part + (size_t)((it + 1) * 4 + 3) * G + wg, v[2]);
            }
            publish(1, (unsigned)(it + 2), v[0]);
            azl = local_part();
            rz = tag_sum(bar, gid0, G, 1, (unsigned)(it + 2), broken, red, A.spin);
        }
        stage();
    }
    // ---- finish: report (first workgroup), x out; the update itself is step_commit_kernel's
    double nbad = A.iters > 0 ? gather_dev(A.part + (size_t)(A.iters * 4 + 3) * G, G, red) : 0.0;
    if constexpr (kJoint) nbad += pose_s[3];
    if (act) A.x[(size_t)j * 12 + a] = vx[li];
    if (wg == 0) {
        for (int q = 0; q <= done; ++q) {
            double rr = gather_dev(A.part + (size_t)(q * 4 + 1) * G, G, red);
            if constexpr (kJoint) rr += rrp[min(q, MISSLAM_MAX_PCG)];
            if (threadIdx.x == 0 && q <= MISSLAM_MAX_PCG) rep->pcg_resid[q] = sqrt(rr);
        }
        if constexpr (kJoint)
            if (threadIdx.x == 0)
                for (int u = 0; u < 6; ++u) jx.xp_out[u] = ps[24 + u];
        if (threadIdx.x == 0) {
            rep->pcg_iters_done = done;
            int f = 0;
            if (stopped) f |= MISSLAM_FLAG_PCG_BREAKDOWN;
            if (nbad != 0.0) f |= MISSLAM_FLAG_NONFINITE;
            if (f) atomicOr(&rep->flags, f);   // atomic: other workgroups may be adding the timeout bit
        }
    }
    if (broken && threadIdx.x == 0) atomicOr(&rep->flags, MISSLAM_FLAG_SYNC_TIMEOUT);
}

// The solve's G workgroups, and with ra.rep set one more (the last) that forms the step's energy report and
// exits: it takes no part in the exchanges.
__global__ void __launch_bounds__(kPcgThreads) pcg_persistent_kernel(PcgArgs A, int rows_per_wg, int cache_blocks,
                                                                    unsigned *bar, misslam_report *rep,
                                                                    ReportArgs ra) {
    const int G = (int)gridDim.x - (ra.rep ? 1 : 0);
    if ((int)blockIdx.x == G) {
        energy_report_body(ra.pt_part, ra.npb, ra.node_part, ra.m, ra.rep, ra.reject, nullptr, 0, ra.kp_energy,
                           ra.kp_count);
        return;
    }
    pcg_persistent_body<false>(A, rows_per_wg, cache_blocks, bar, 0, blockIdx.x, G, rep, JointExtra{});
}

__global__ void __launch_bounds__(kPcgThreads) jpcg_tiled_kernel(PcgArgs A, int rows_per_wg, int cache_blocks,
                                                                unsigned *bar, misslam_report *rep, JointExtra jx) {
    pcg_persistent_body<true>(A, rows_per_wg, cache_blocks, bar, 0, blockIdx.x, gridDim.x, rep, jx);
}

// x += dx over n entries as one step, after the solve that produced dx has
// completed: skipped entirely when the step's report carries a non-finite
// value or a solve timeout, so no entry changes unless every workgroup of the
// solve finished.  extra_flags (optional) is ORed into that report first
// (block 0), for steps assembled from several solves.
__global__ void __launch_bounds__(256) step_commit_kernel(float *__restrict__ x, const float *__restrict__ dx,
                                                          int n, misslam_report *rep, const misslam_report *extra) {
    const int xf = extra ? extra->flags : 0;
    const int f = rep->flags | xf;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (!(f & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT)) && i < n) x[i] += dx[i];
    if (extra && blockIdx.x == 0 && threadIdx.x == 0) rep->flags = f;
}

hipError_t launch_step_commit(float *x, const float *dx, int n, misslam_report *rep, hipStream_t st,
                              const misslam_report *extra) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(step_commit_kernel, dim3((n + 255) / 256), dim3(256), 0, st, x, dx, n, rep, extra);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pipelined PCG in one launch

// The default recurrence of the one-launch solve: the preconditioned pipelined
// conjugate gradients of Ghysels and Vanroose (2014), the same iterates as the
// textbook recurrence in exact arithmetic.  Besides x, r and the direction p it
// carries u = M r, w = A u, s = A p, q = M s and z = A q, so that the two inner
// products of an iteration, gamma = r.u and delta = w.u, are formed before the
// iteration's only product n = A m (m = M w) and travel in the same exchange as
// m itself: one exchange per iteration instead of two.  Every vector is kept in
// float64 (in registers: each thread owns one entry of each), which keeps the
// longer recurrence as accurate as the textbook one: the only float32 values
// are the matrix blocks and the preconditioner blocks.  The decisions are the
// textbook ones: gamma = r.z = 0 stops the solve, p.Ap <= 0 (here
// delta - beta gamma / alpha_prev) stops it and flags a breakdown.
//
// Exchange e (tag e = 1 before the first iteration, e = i + 2 in iteration i;
// the sync words are zero at launch) publishes the workgroup's partials of
// gamma and delta as tagged words in the sync slots of parity e & 1 (4
// eight-byte words per workgroup), and the vector it multiplies next (u_0,
// then m_i) through halo buffer e & 1; a workgroup rewrites a buffer or a slot
// only two exchanges later, when every workgroup has read it.
// |r|^2 of every iterate goes to A.part for the report, which ppcg_finish
// completes after the launch (no exchange is spent on it).

__device__ __forceinline__ void tag_publish2(unsigned *bar, int gid, unsigned tag, double v0, double v1) {
    unsigned long long *w = tag_slots(bar) + 8 * gid + 4 * (tag & 1);
    const unsigned long long b0 = (unsigned long long)__double_as_longlong(v0);
    const unsigned long long b1 = (unsigned long long)__double_as_longlong(v1);
    __hip_atomic_store(w, (b0 & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, (b0 << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 2, (b1 & 0xFFFFFFFF00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 3, (b1 << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-order sums of the two values workgroups g0 .. g0+G-1 published with `tag` (bounded waits).
__device__ __forceinline__ void tag_sum2(unsigned *bar, int g0, int G, unsigned tag, bool &broken,
                                         double (*lds)[kPcgThreads / kWave], unsigned spin_limit, double &s0,
                                         double &s1) {
    double v[2] = {0.0, 0.0};
    bool ok = true;
    for (int t = threadIdx.x; t < G; t += kPcgThreads) {
        unsigned long long *w = tag_slots(bar) + 8 * (g0 + t) + 4 * (tag & 1);
        unsigned long long h0 = 0, l0 = 0, h1 = 0, l1 = 0;
        unsigned spins = 0;
        for (;;) {
            h0 = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            l0 = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            h1 = __hip_atomic_load(w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            l1 = __hip_atomic_load(w + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((unsigned)h0 == tag && (unsigned)l0 == tag && (unsigned)h1 == tag && (unsigned)l1 == tag) break;
            if (broken || ++spins > spin_limit) {
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok) {
            v[0] += __longlong_as_double((long long)((h0 & 0xFFFFFFFF00000000ull) | (l0 >> 32)));
            v[1] += __longlong_as_double((long long)((h1 & 0xFFFFFFFF00000000ull) | (l1 >> 32)));
        }
    }
    broken = __syncthreads_or(broken || !ok) != 0;
    wg_sum<2>(v, lds);
    s0 = v[0];
    s1 = v[1];
}

constexpr int kMaxUniqueP = 96;   // distinct columns staged per iteration (float64): 16 rows have about 50
constexpr int kMPer = (kMaxUniqueP * 12 + kPcgThreads - 1) / kPcgThreads;   // staged doubles per thread

__device__ __forceinline__ void ppcg_persistent_body(const PcgArgs &A, int rows_per_wg, int cache_blocks,
                                                     unsigned *bar, int gid0, int wg, int G, misslam_report *rep) {
    extern __shared__ float4 dyn4[];
    __shared__ double red[2][kPcgThreads / kWave];
    __shared__ TileLds tl;
    __shared__ double mz[kMaxUniqueP * 12];           // the multiplied vector at the distinct columns
    __shared__ double vv[kRowsPerBlk * 12];           // the rows' vector going through the preconditioner
    const double lam = (double)(A.lambda_dev ? *A.lambda_dev : A.lambda);
    float *hc = reinterpret_cast<float *>(dyn4);       // cached blocks
    float *mc = hc + (size_t)cache_blocks * 144;       // preconditioner blocks of the rows
    const TileRange R = tile_setup(A, rows_per_wg, cache_blocks, wg, dyn4, mc, tl, reinterpret_cast<int *>(mz),
                                   kMaxUniqueP * 24, kMaxUniqueP);
    const int r0 = R.r0, r1 = R.r1, b0 = R.b0, nb = R.nb, cached = R.cached, U = R.U;
    const int *bmap = tl.bmap, *colL = tl.colL, *ucol = tl.ucol;
    const int lr = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = r0 + lr;
    const bool act = lr < kRowsPerBlk && j < r1;
    const int li = lr * 12 + a;
    const size_t o = (size_t)j * 12 + a;
    bool broken = false;
    // this thread's row: its blocks q in [rq0, rq1) of the workgroup (at most MISSLAM_MAX_ROW), split into the
    // blocks whose column is one of this workgroup's rows (multiplied while the exchange is in flight) and the
    // others.  The summation order is the same whether a block is cached in LDS or read from memory, and
    // whether its column is staged or not: own columns in block order into one chain, then the other blocks
    // alternately into two chains, added at the end.
    const int rq0 = act ? min(A.row_ptr[j], A.cap) - b0 : 0;
    const int rq1 = act ? min(min(A.row_ptr[j + 1], A.cap) - b0, rq0 + MISSLAM_MAX_ROW) : 0;
    uint32_t lmask = 0, rmask = 0;
    for (int q = rq0; q < rq1; ++q) {
        const int c = q < nb ? colL[q] : A.col_idx[b0 + q];
        if (c >= r0 && c < r1)
            lmask |= 1u << (q - rq0);
        else
            rmask |= 1u << (q - rq0);
    }
    const int mslot = act ? tl.lslot[lr] : -1;   // staged slot of this row's own column (-1: none)

    // one block (workgroup block q) times the multiplied vector, float32 entries times float64 values summed
    // in float64 in entry order; the block from LDS when cached, the vector from its staged slot when it has
    // one, else from memory (halo buffer hb)
    auto block_dot = [&](int q, double t, const double *hb) {
        const int slot = q < nb ? bmap[q] : -1;
        if (q < cached && slot >= 0) {
            const float4 *Bq = reinterpret_cast<const float4 *>(hc + (size_t)q * 144 + a * 12);
            const double *mq = mz + slot * 12;
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                const float4 b4 = Bq[h];
                t = fma((double)b4.x, mq[4 * h], t);
                t = fma((double)b4.y, mq[4 * h + 1], t);
                t = fma((double)b4.z, mq[4 * h + 2], t);
                t = fma((double)b4.w, mq[4 * h + 3], t);
            }
            return t;
        }
        const float *B = q < cached ? hc + (size_t)q * 144 + a * 12 : A.blocks + (size_t)(b0 + q) * 144 + a * 12;
        if (slot >= 0) {
            const double *ml = mz + slot * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) t = fma((double)B[b], ml[b], t);
        } else {
            const double *ml = hb + (size_t)A.col_idx[b0 + q] * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) t = fma((double)B[b], ld_dev(ml + b), t);
        }
        return t;
    };
    auto local_part = [&](const double *hb) {
        double t = 0.0;
        for (uint32_t mk = lmask; mk; mk &= mk - 1) t = block_dot(rq0 + __builtin_ctz(mk), t, hb);
        return t;
    };
    // the other blocks of the row's product, the vector staged from halo buffer hb; t holds the local part
    auto remote_part = [&](double t, const double *hb) {
        double t1 = 0.0;
        uint32_t mk = rmask;
        while (mk) {
            const int qa = rq0 + __builtin_ctz(mk);
            mk &= mk - 1;
            if (mk) {
                const int qb = rq0 + __builtin_ctz(mk);
                mk &= mk - 1;
                t = block_dot(qa, t, hb);
                t1 = block_dot(qb, t1, hb);
            } else {
                t = block_dot(qa, t, hb);
            }
        }
        return t + t1;
    };
    // stage the vector at the distinct columns owned by other workgroups (own columns are written by their
    // rows' threads), all loads in flight together
    auto stage = [&](const double *hb) {
        double mv[kMPer];
#pragma unroll
        for (int e = 0; e < kMPer; ++e) {
            const int t = threadIdx.x + e * kPcgThreads;
            if (t < U * 12 && (ucol[t / 12] < r0 || ucol[t / 12] >= r1))
                mv[e] = ld_dev(hb + (size_t)ucol[t / 12] * 12 + t % 12);
        }
#pragma unroll
        for (int e = 0; e < kMPer; ++e) {
            const int t = threadIdx.x + e * kPcgThreads;
            if (t < U * 12 && (ucol[t / 12] < r0 || ucol[t / 12] >= r1)) mz[t] = mv[e];
        }
        __syncthreads();
    };
    // M_j v for this thread's entry, v of the row in vv
    auto precond = [&]() {
        const float *M = mc + (size_t)lr * 144 + a * 12;
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < 12; ++b) t = fma((double)M[b], vv[lr * 12 + b], t);
        return t;
    };
    // this entry of the vector to multiply next: into halo buffer hb and this row's staged slot
    auto put = [&](double *hb, double v) {
        st_dev(hb + o, v);
        if (mslot >= 0) mz[mslot * 12 + a] = v;
    };
    auto publish = [&](unsigned tag, double v0, double v1) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) tag_publish2(bar, gid0 + wg, tag, v0, v1);
    };
    auto rr_out = [&](int it, double rr) {   // |r_it|^2 partial, read by ppcg_finish after the launch
        double v[1] = {rr};
        wg_sum<1>(v, red);
        if (threadIdx.x == 0) A.part[(size_t)it * G + wg] = v[0];
    };

    // init: x = 0, r = -g, u = M r, w = A u (exchange 0 carries u)
    double x = 0.0, r = 0.0, u = 0.0, w = 0.0, p = 0.0, s = 0.0, q = 0.0, z = 0.0;
    if (act) {
        r = -(double)A.g[o];
        vv[li] = r;
    }
    __syncthreads();
    if (act) {
        u = precond();
        put(A.halo[1], u);
    }
    publish(1u, 0.0, 0.0);
    {
        double l = act ? local_part(A.halo[1]) : 0.0;
        double d0, d1;
        tag_sum2(bar, gid0, G, 1u, broken, red, A.spin, d0, d1);
        stage(A.halo[1]);
        if (act) w = fma(lam, u, remote_part(l, A.halo[1]));
    }
    bool stopped = false, brk = false;
    int done = 0;
    double gamma_prev = 1.0, alpha_prev = 1.0;
    for (int it = 0; it < A.iters; ++it) {
        rr_out(it, act ? r * r : 0.0);
        double v[2] = {act ? r * u : 0.0, act ? w * u : 0.0};
        wg_sum<2>(v, red);
        // m = M w: multiplied while gamma and delta are in flight
        double m = 0.0;
        if (act) vv[li] = w;
        __syncthreads();
        double *hb = A.halo[it & 1];
        if (act) {
            m = precond();
            put(hb, m);
        }
        publish((unsigned)(it + 2), v[0], v[1]);
        double n = act ? local_part(hb) : 0.0;
        double gamma, delta;
        tag_sum2(bar, gid0, G, (unsigned)(it + 2), broken, red, A.spin, gamma, delta);
        stage(hb);
        if (act) n = fma(lam, m, remote_part(n, hb));
        // the textbook decisions, from scalars every workgroup holds alike
        if (stopped || gamma == 0.0) {
            stopped = true;
            continue;
        }
        const double beta = it > 0 ? gamma / gamma_prev : 0.0;
        const double pap = it > 0 ? delta - beta * gamma / alpha_prev : delta;   // p.A p
        if (!(pap > 0.0)) {
            stopped = brk = true;
            continue;
        }
        const double alpha = gamma / pap;
        if (act) {
            z = fma(beta, z, n);
            q = fma(beta, q, m);
            s = fma(beta, s, w);
            p = fma(beta, p, u);
            x = fma(alpha, p, x);
            r = fma(-alpha, s, r);
            u = fma(-alpha, q, u);
            w = fma(-alpha, z, w);
        }
        gamma_prev = gamma;
        alpha_prev = alpha;
        ++done;
    }
    rr_out(A.iters, act ? r * r : 0.0);
    // x out (float32), this workgroup's non-finite check, the report's scalars (first workgroup); the
    // residual norms and the update itself are ppcg_finish's
    const float xf = (float)x;
    if (act) A.x[o] = xf;
    const bool bad = __syncthreads_or(act && !isfinite(xf)) != 0;
    if (threadIdx.x == 0) {
        int f = 0;
        if (bad) f |= MISSLAM_FLAG_NONFINITE;
        if (broken) f |= MISSLAM_FLAG_SYNC_TIMEOUT;
        if (wg == 0) {
            rep->pcg_iters_done = done;
            if (brk) f |= MISSLAM_FLAG_PCG_BREAKDOWN;
        }
        if (f) atomicOr(&rep->flags, f);
    }
}

__global__ void __launch_bounds__(kPcgThreads) ppcg_persistent_kernel(PcgArgs A, int rows_per_wg, int cache_blocks,
                                                                     unsigned *bar, misslam_report *rep) {
    ppcg_persistent_body(A, rows_per_wg, cache_blocks, bar, 0, blockIdx.x, gridDim.x, rep);
}

// After a pipelined one-launch solve of G workgroups: the report's residual norms |r_q|, q = 0 .. iterations
// done (the partials every workgroup left, added in workgroup order; first block), and x += dx unless the
// report carries a non-finite value or a timeout (params may be null: the solve alone).
__device__ __forceinline__ void ppcg_finish_body(const double *part, int G, misslam_report *rep, float *params,
                                                 const float *dx, int n, int blk, double *lds) {
    const int f = rep->flags;
    const int i = blk * kPcgThreads + threadIdx.x;
    if (params && !(f & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT)) && i < n) params[i] += dx[i];
    if (blk != 0) return;
    const int done = rep->pcg_iters_done;
    for (int q = 0; q <= done && q <= MISSLAM_MAX_PCG; ++q) {
        double v = 0.0;
        for (int t = threadIdx.x; t < G; t += kPcgThreads) v += part[(size_t)q * G + t];
        v = block_sum<kPcgThreads>(v, lds);
        if (threadIdx.x == 0) rep->pcg_resid[q] = sqrt(v);
    }
}

__global__ void __launch_bounds__(kPcgThreads) ppcg_finish_kernel(const double *part, int G, misslam_report *rep,
                                                                 float *params, const float *dx, int n) {
    __shared__ double lds[kPcgThreads];
    ppcg_finish_body(part, G, rep, params, dx, n, blockIdx.x, lds);
}

// Grid shape of the persistent solve for m rows on this device, or 0 when a
// cooperative launch cannot hold it (the multi-kernel path is used then).
// Rows are packed MISSLAM_SOLVE_ROWS to a workgroup: fewer workgroups make
// the exchanges cheaper, while the blocks of that many rows (about 13 per row
// on a surface graph) still fit the LDS left beside the static arrays.  One
// workgroup per CU must hold them all, so a larger system packs up to
// kRowsPerBlk rows (blocks beyond the LDS cache are read from global memory).

struct PersistentShape {
    int max_blocks = -1, max_lds = 0;
};

// The device limits of one persistent kernel: queried once per process (first device used).
template <typename Kern>
static void persistent_limits(Kern kern, PersistentShape &sh) {
    int dev = 0, cus = 0, coop = 0, shmem = 0;
    hipFuncAttributes fa{};
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&shmem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern)) != hipSuccess || !coop) {
        sh.max_blocks = 0;
        return;
    }
    sh.max_lds = (shmem < kPersistMaxLds ? shmem : kPersistMaxLds) - (int)fa.sharedSizeBytes - 1024;
    int per_cu = 0;
    if (sh.max_lds <= 0 ||
        hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            sh.max_lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPcgThreads, sh.max_lds) != hipSuccess ||
        per_cu < 1)
        sh.max_blocks = 0;
    else
        sh.max_blocks = cus;
}

static int persistent_grid(const PersistentShape &sh, int m, int &rows_per_wg, int &lds_bytes) {
    const int max_blocks = sh.max_blocks, max_lds = sh.max_lds;
    if (max_blocks <= 0 || m <= 0) return 0;
    // more rows per workgroup once one workgroup per CU no longer holds the system
    rows_per_wg = MISSLAM_SOLVE_ROWS;
    if (m > rows_per_wg * max_blocks) rows_per_wg = (m + max_blocks - 1) / max_blocks;
    if (rows_per_wg > kRowsPerBlk) return 0;
    const int G = (m + rows_per_wg - 1) / rows_per_wg;
    if (G > max_blocks || G > MSL_TAG_WGS) return 0;
    lds_bytes = max_lds;
    return G;
}

static int persistent_grid(int m, int &rows_per_wg, int &lds_bytes, bool textbook, int extra_wgs = 0) {
    static PersistentShape tb, pp;
    PersistentShape &sh = textbook ? tb : pp;
    if (sh.max_blocks < 0) {
        if (textbook)
            persistent_limits(pcg_persistent_kernel, sh);
        else
            persistent_limits(ppcg_persistent_kernel, sh);
    }
    const int G = persistent_grid(sh, m, rows_per_wg, lds_bytes);
    return G > 0 && G + extra_wgs <= sh.max_blocks ? G : 0;
}

hipError_t launch_pcg_persistent(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                                 float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                                 float *params, hipStream_t st, bool *used, bool cooperative, int zeroed_words,
                                 const float *lambda_dev, unsigned spin, bool textbook,
                                 const ReportArgs *report) {
    *used = false;
    ReportArgs ra;
    if (report && textbook) ra = *report;   // the report workgroup rides with the textbook solve only
    const int extra = ra.rep ? 1 : 0;
    int rows = 0, lds = 0;
    const int G = persistent_grid(m, rows, lds, textbook, extra);
    if (G <= 0 || G > s.nblk_max) return hipSuccess;
    PcgArgs A;
    A.row_ptr = g.row_ptr;
    A.col_idx = g.col_idx;
    A.blocks = blocks;
    A.minv = minv;
    A.g = gvec;
    A.lambda = lambda;
    A.lambda_dev = lambda_dev;
    A.m = m;
    A.nblk = G;
    A.iters = iters;
    A.cap = g.bsr_cap;
    A.x = delta;
    A.r = s.r;
    A.z = s.z;
    A.p = s.p;
    A.q = s.q;
    A.part = s.part;
    A.status = s.status;
    A.done = s.status + (iters + 2);
    if (spin > 0) A.spin = spin;
    A.halo[0] = s.halo;
    A.halo[1] = s.halo + (size_t)12 * m;
    A.textbook = textbook;
    // dynamic LDS: cached blocks (144 floats each) and the rows' preconditioner
    const int cache_blocks = (lds / 4 - rows * 144) / 144;
    if (cache_blocks < 1) return hipSuccess;
    unsigned *bar = s.bar;
    const int words = MSL_WG_WORDS * G;
    if (zeroed_words < words)
        hipLaunchKernelGGL(fill_u32_kernel_pcg, dim3((words + 255) / 256), dim3(256), 0, st, bar, words);
    hipError_t e = hipSuccess;
    if (report && report->rep && !textbook) e = launch_energy_report(*report, st);   // not formed by the solve
    if (e != hipSuccess) return e;
    if (textbook) {
        if (cooperative) {
            void *args[] = {&A, (void *)&rows, (void *)&cache_blocks, &bar, &rep, &ra};
            e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(pcg_persistent_kernel), dim3(G + extra),
                                           dim3(kPcgThreads), args, (unsigned)lds, st);
        } else {
            hipLaunchKernelGGL(pcg_persistent_kernel, dim3(G + extra), dim3(kPcgThreads), (unsigned)lds, st, A, rows,
                               cache_blocks, bar, rep, ra);
            e = hipGetLastError();
        }
    } else if (cooperative) {
        void *args[] = {&A, (void *)&rows, (void *)&cache_blocks, &bar, &rep};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(ppcg_persistent_kernel), dim3(G),
                                       dim3(kPcgThreads), args, (unsigned)lds, st);
    } else {
        hipLaunchKernelGGL(ppcg_persistent_kernel, dim3(G), dim3(kPcgThreads), (unsigned)lds, st, A, rows,
                           cache_blocks, bar, rep);
        e = hipGetLastError();
    }
    if (e == hipSuccess) *used = true;
    if (e == hipSuccess && textbook && params) e = launch_step_commit(params, delta, 12 * m, rep, st, nullptr);
    if (e == hipSuccess && !textbook) {   // the residual norms, and the step unless it failed
        const int blocks = params ? (12 * m + kPcgThreads - 1) / kPcgThreads : 1;
        hipLaunchKernelGGL(ppcg_finish_kernel, dim3(blocks), dim3(kPcgThreads), 0, st, A.part, G, rep, params,
                           delta, 12 * m);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_joint_pcg_persistent(const PcgArgs &base, const JointExtra &jx, unsigned long long *bar,
                                       int zeroed_words, misslam_report *rep, hipStream_t st, bool *used) {
    *used = false;
    static PersistentShape sh;
    if (sh.max_blocks < 0) persistent_limits(jpcg_tiled_kernel, sh);
    int rows = 0, lds = 0;
    const int G = persistent_grid(sh, base.m, rows, lds);
    if (G <= 0 || G > kJointMaxWgs || !bar || !base.part) return hipSuccess;
    const int cache_blocks = (lds / 4 - rows * 144) / 144;
    if (cache_blocks < 1) return hipSuccess;
    PcgArgs A = base;
    A.nblk = G;
    unsigned *b32 = reinterpret_cast<unsigned *>(bar);
    const int words = kJointTagWords * G;   // 8-byte words
    if (zeroed_words < words)
        hipLaunchKernelGGL(fill_u32_kernel_pcg, dim3((2 * words + 255) / 256), dim3(256), 0, st, b32, 2 * words);
    hipLaunchKernelGGL(jpcg_tiled_kernel, dim3(G), dim3(kPcgThreads), (unsigned)lds, st, A, rows, cache_blocks, b32,
                       rep, jx);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) *used = true;
    return e;
}


}  // namespace msl

namespace msl {

// ---------------------------------------------------------------- side-by-side persistent solves

// Every problem of a batch runs the same recurrence on its own rows: workgroup
// w belongs to the problem whose range holds it, keeps that problem's
// partials, and joins one barrier with every workgroup of the launch.
__global__ void __launch_bounds__(kPcgThreads) pcg_batched_kernel(const BatchItem *__restrict__ items, int count,
                                                                 int rows_per_wg, int cache_blocks, unsigned *bar,
                                                                 int gi) {
    int b = count - 1;
    while (b > 0 && items[b].wg0 > (int)blockIdx.x) --b;
    const BatchItem &it = items[b];
    pcg_persistent_body<false>(it.p, rows_per_wg, cache_blocks, bar, it.wg0, (int)blockIdx.x - it.wg0, it.wgs,
                               it.rep + gi, JointExtra{});
}

// The same with the pipelined recurrence.
__global__ void __launch_bounds__(kPcgThreads) ppcg_batched_kernel(const BatchItem *__restrict__ items, int count,
                                                                  int rows_per_wg, int cache_blocks, unsigned *bar,
                                                                  int gi) {
    int b = count - 1;
    while (b > 0 && items[b].wg0 > (int)blockIdx.x) --b;
    const BatchItem &it = items[b];
    ppcg_persistent_body(it.p, rows_per_wg, cache_blocks, bar, it.wg0, (int)blockIdx.x - it.wg0, it.wgs,
                         it.rep + gi);
}

// ppcg_finish over every problem of a batch: block b < count completes problem b's report; the blocks after
// them apply each problem's step (one thread per parameter entry), unless its report rules it out.
__global__ void __launch_bounds__(kPcgThreads) ppcg_finish_batched_kernel(const BatchItem *__restrict__ items,
                                                                         int count, int total_rows, int gi) {
    __shared__ double lds[kPcgThreads];
    if ((int)blockIdx.x < count) {
        const BatchItem &it = items[blockIdx.x];
        ppcg_finish_body(it.p.part, it.wgs, it.rep + gi, nullptr, nullptr, 0, 0, lds);
        return;
    }
    const int t = ((int)blockIdx.x - count) * kPcgThreads + threadIdx.x;
    if (t >= 12 * total_rows) return;
    const int row = t / 12;
    int b = count - 1;
    while (b > 0 && items[b].row0 > row) --b;
    const BatchItem &it = items[b];
    const int f = it.rep[gi].flags;
    const int o = t - 12 * it.row0;
    if (!(f & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT))) it.params[o] += it.p.x[o];
}

// step_commit_kernel over every problem of a batch: params += dx of problem b unless its step's report
// carries a non-finite value or a solve timeout.  One thread per parameter entry (rows row0 .. of problem b).
__global__ void __launch_bounds__(256) step_commit_batched_kernel(const BatchItem *__restrict__ items, int count,
                                                                  int total_rows, int gi) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= 12 * total_rows) return;
    const int row = t / 12;
    int b = count - 1;
    while (b > 0 && items[b].row0 > row) --b;
    const BatchItem &it = items[b];
    const int f = it.rep[gi].flags;
    const int o = t - 12 * it.row0;
    if (!(f & (MISSLAM_FLAG_NONFINITE | MISSLAM_FLAG_SYNC_TIMEOUT))) it.params[o] += it.p.x[o];
}

using BatchedKernel = void (*)(const BatchItem *, int, int, int, unsigned *, int);

static int batched_static_lds(BatchedKernel kern) {
    hipFuncAttributes fa{};
    return hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern)) == hipSuccess ? (int)fa.sharedSizeBytes
                                                                                         : 1 << 30;
}

// Dynamic LDS per workgroup for total_wgs co-resident workgroups, or 0 if they cannot all be resident.
static int batched_lds(int total_wgs, bool textbook) {
    static int static_lds[2] = {-1, -1};
    const BatchedKernel kern = textbook ? pcg_batched_kernel : ppcg_batched_kernel;
    if (static_lds[textbook] < 0) static_lds[textbook] = batched_static_lds(kern);
    const int sl = static_lds[textbook];
    int dev = 0, cus = 0, shmem = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&shmem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || cus <= 0)
        return 0;
    const int per_cu = (total_wgs + cus - 1) / cus;
    if (per_cu > 4 || total_wgs > MSL_TAG_WGS) return 0;
    const int cu_lds = kPersistMaxLds;
    int lds = cu_lds / per_cu - sl - 1024;
    if (lds > shmem - sl - 1024) lds = shmem - sl - 1024;
    const int min_lds = (kRowsPerBlk * 144 + 144) * 4;   // the rows' preconditioner and one cached block
    if (lds < min_lds) return 0;
    int occ = 0;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kPcgThreads, lds) != hipSuccess ||
        occ * cus < total_wgs)
        return 0;
    return lds;
}

int pcg_batched_fits(int total_wgs, bool textbook) {
    return total_wgs > 0 && batched_lds(total_wgs, textbook) > 0 ? 1 : 0;
}

hipError_t launch_pcg_batched(const BatchItem *items, int count, int rows_per_wg, int total_wgs, int total_rows,
                              int it, unsigned *bar, bool cooperative, hipStream_t st, bool *used, bool textbook) {
    *used = false;
    const int lds = batched_lds(total_wgs, textbook);
    if (lds <= 0 || rows_per_wg < 1 || rows_per_wg > kRowsPerBlk) return hipSuccess;
    const int cache_blocks = (lds / 4 - rows_per_wg * 144) / 144;
    if (cache_blocks < 1) return hipSuccess;
    const BatchedKernel kern = textbook ? pcg_batched_kernel : ppcg_batched_kernel;
    hipError_t e;
    if (cooperative) {
        void *args[] = {(void *)&items, (void *)&count, (void *)&rows_per_wg, (void *)&cache_blocks, (void *)&bar,
                        (void *)&it};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(total_wgs), dim3(kPcgThreads), args,
                                       (unsigned)lds, st);
    } else {
        hipLaunchKernelGGL(kern, dim3(total_wgs), dim3(kPcgThreads), (unsigned)lds, st, items, count, rows_per_wg,
                           cache_blocks, bar, it);
        e = hipGetLastError();
    }
    if (e == hipSuccess) *used = true;
    if (e == hipSuccess && textbook && total_rows > 0) {
        hipLaunchKernelGGL(step_commit_batched_kernel, dim3((12 * total_rows + 255) / 256), dim3(256), 0, st, items,
                           count, total_rows, it);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !textbook) {
        const int blocks = count + (12 * total_rows + kPcgThreads - 1) / kPcgThreads;
        hipLaunchKernelGGL(ppcg_finish_batched_kernel, dim3(blocks), dim3(kPcgThreads), 0, st, items, count,
                           total_rows, it);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace msl
