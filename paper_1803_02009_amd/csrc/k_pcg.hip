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

struct PcgArgs {
    const int32_t *row_ptr, *col_idx;
    const float *blocks, *minv, *g;
    float lambda;
    int m, nblk, iters, cap;
    float *x, *r, *z, *p, *q;
    double *part;     // [(it * 4 + kind) * nblk + block], kind 0 = r.z, 1 = r.r, 2 = p.q, 3 = #non-finite x
    int32_t *status;  // [it]: 0 running, 2 stopped by breakdown (propagates)
    int32_t *done;    // [it]: 1 if iteration it updated x
};

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
        float az = 0.f;
        const int p0 = A.row_ptr[j], p1 = min(A.row_ptr[j + 1], A.cap);
        for (int pb = p0; pb < p1; ++pb) {
            const int l = A.col_idx[pb];
            const float *B = A.blocks + (size_t)pb * 144 + a * 12;
            const float *zl = A.z + (size_t)l * 12;
#pragma unroll
            for (int b = 0; b < 12; ++b) az = fmaf(B[b], zl[b], az);
        }
        const size_t o = (size_t)j * 12 + a;
        const float zj = A.z[o];
        az = fmaf(A.lambda, zj, az);
        float p, q;
        if (it > 0) {
            p = fmaf(beta, A.p[o], zj);
            q = fmaf(beta, A.q[o], az);
        } else {
            p = zj;
            q = az;
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
                             float *params, hipStream_t st) {
    PcgArgs A;
    A.row_ptr = g.row_ptr;
    A.col_idx = g.col_idx;
    A.blocks = blocks;
    A.minv = minv;
    A.g = gvec;
    A.lambda = lambda;
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

__global__ void report_init_kernel(misslam_report *rep, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) {
        rep[t].e_data = 0.0;
        rep[t].e_rot = 0.0;
        rep[t].e_reg = 0.0;
        for (int q = 0; q <= MISSLAM_MAX_PCG; ++q) rep[t].pcg_resid[q] = 0.0;
        rep[t].n_valid = 0;
        rep[t].flags = 0;
        rep[t].pcg_iters_done = 0;
        rep[t].reserved = 0;
    }
}

hipError_t launch_report_init(misslam_report *rep, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(report_init_kernel, dim3((count + 63) / 64), dim3(64), 0, st, rep, count);
    return hipGetLastError();
}

int pcg_blocks(int m) { return (m + kRowsPerBlk - 1) / kRowsPerBlk; }

// ---------------------------------------------------------------- persistent PCG (one cooperative launch)

constexpr int kPersistLdsBytes = 64 * 1024;

// The same recurrence in one launch: each workgroup owns a contiguous range of
// rows, keeps their blocks (as many as fit) and their preconditioner blocks in
// LDS and its slice of x, r, p, q in LDS; only z travels through global memory.
// Two grid-wide barriers per iteration; every reduction is re-added by every
// workgroup in the same order, so all take identical decisions.
__global__ void __launch_bounds__(kPcgThreads) pcg_persistent_kernel(PcgArgs A, int rows_per_wg, int cache_blocks,
                                                                    misslam_report *rep, float *__restrict__ params) {
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    extern __shared__ float dyn[];
    __shared__ double red[kPcgThreads];
    __shared__ float vx[kRowsPerBlk * 12], vr[kRowsPerBlk * 12], vp[kRowsPerBlk * 12], vq[kRowsPerBlk * 12];
    const int G = gridDim.x;
    const int r0 = min(A.m, (int)blockIdx.x * rows_per_wg);
    const int r1 = min(A.m, r0 + rows_per_wg);
    const int b0 = min(A.row_ptr[r0], A.cap), b1 = min(A.row_ptr[r1], A.cap);
    const int cached = min(b1 - b0, cache_blocks);
    float *hc = dyn;                                   // cached blocks
    float *mc = dyn + (size_t)cache_blocks * 144;      // preconditioner blocks of the rows
    for (int t = threadIdx.x; t < cached * 144; t += kPcgThreads) hc[t] = A.blocks[(size_t)b0 * 144 + t];
    for (int t = threadIdx.x; t < (r1 - r0) * 144; t += kPcgThreads) mc[t] = A.minv[(size_t)r0 * 144 + t];
    // thread -> (row, component); rows_per_wg <= kRowsPerBlk
    const int lr = threadIdx.x / 12, a = threadIdx.x % 12;
    const int j = r0 + lr;
    const bool act = lr < kRowsPerBlk && j < r1;
    const int li = lr * 12 + a;
    __syncthreads();

    // init: r = -g, z = M r, x = 0
    float r = 0.f, z = 0.f;
    if (act) {
        r = -A.g[(size_t)j * 12 + a];
        vr[li] = r;
        vx[li] = 0.f;
    }
    __syncthreads();
    if (act) {
        const float *M = mc + (size_t)lr * 144 + a * 12;
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < 12; ++b) s = fmaf(M[b], vr[lr * 12 + b], s);
        z = s;
        A.z[(size_t)j * 12 + a] = z;
    }
    {
        const double rz0 = block_sum<kPcgThreads>((double)r * (double)z, red);
        const double rr0 = block_sum<kPcgThreads>((double)r * (double)r, red);
        if (threadIdx.x == 0) {
            A.part[(size_t)(0 * 4 + 0) * G + blockIdx.x] = rz0;
            A.part[(size_t)(0 * 4 + 1) * G + blockIdx.x] = rr0;
        }
    }
    grid.sync();
    bool stopped = false;
    int done = 0;
    double rz_prev = 1.0;
    for (int it = 0; it < A.iters; ++it) {
        const double rz = gather_sum(A.part + (size_t)(it * 4 + 0) * G, G, red);
        const bool skip = stopped || rz == 0.0;
        // ---- direction and product: p = z + beta p, q = (H + lambda I) z + beta q
        double pq = 0.0;
        if (act && !skip) {
            const float beta = it > 0 ? (float)(rz / rz_prev) : 0.f;
            float az = 0.f;
            const int p0 = A.row_ptr[j], p1 = min(A.row_ptr[j + 1], A.cap);
            for (int pb = p0; pb < p1; ++pb) {
                const int l = A.col_idx[pb];
                const float *B = (pb - b0 < cached) ? hc + (size_t)(pb - b0) * 144 + a * 12
                                                    : A.blocks + (size_t)pb * 144 + a * 12;
                const float *zl = A.z + (size_t)l * 12;
#pragma unroll
                for (int b = 0; b < 12; ++b) az = fmaf(B[b], zl[b], az);
            }
            az = fmaf(A.lambda, z, az);
            const float pv = it > 0 ? fmaf(beta, vp[li], z) : z;
            const float qv = it > 0 ? fmaf(beta, vq[li], az) : az;
            vp[li] = pv;
            vq[li] = qv;
            pq = (double)pv * (double)qv;
        }
        {
            const double t = block_sum<kPcgThreads>(pq, red);
            if (threadIdx.x == 0) A.part[(size_t)(it * 4 + 2) * G + blockIdx.x] = t;
        }
        grid.sync();
        // ---- step: alpha = r.z / p.q, x += alpha p, r -= alpha q, z = M r
        const double pqs = gather_sum(A.part + (size_t)(it * 4 + 2) * G, G, red);
        const bool brk = !skip && !(pqs > 0.0);
        const bool upd = !skip && !brk;
        double bad = 0.0;
        if (act && upd) {
            const float alpha = (float)(rz / pqs);
            vx[li] = fmaf(alpha, vp[li], vx[li]);
            r = fmaf(-alpha, vq[li], r);
            vr[li] = r;
        }
        if (act) bad = isfinite(vx[li]) ? 0.0 : 1.0;
        __syncthreads();
        if (act && upd) {
            const float *M = mc + (size_t)lr * 144 + a * 12;
            float s = 0.f;
#pragma unroll
            for (int b = 0; b < 12; ++b) s = fmaf(M[b], vr[lr * 12 + b], s);
            z = s;
            A.z[(size_t)j * 12 + a] = z;
        }
        {
            const double rzn = block_sum<kPcgThreads>((double)r * (double)z, red);
            const double rrn = block_sum<kPcgThreads>((double)r * (double)r, red);
            const double nb = block_sum<kPcgThreads>(bad, red);
            if (threadIdx.x == 0) {
                A.part[(size_t)((it + 1) * 4 + 0) * G + blockIdx.x] = rzn;
                A.part[(size_t)((it + 1) * 4 + 1) * G + blockIdx.x] = rrn;
                A.part[(size_t)((it + 1) * 4 + 3) * G + blockIdx.x] = nb;
            }
        }
        if (upd) ++done;
        if (brk) stopped = true;
        if (!skip) rz_prev = rz;
        grid.sync();
    }
    // ---- finish: report (block 0), x out, params += x unless non-finite
    const double nbad = A.iters > 0 ? gather_sum(A.part + (size_t)(A.iters * 4 + 3) * G, G, red) : 0.0;
    if (act) {
        A.x[(size_t)j * 12 + a] = vx[li];
        if (params && nbad == 0.0) params[(size_t)j * 12 + a] += vx[li];
    }
    if (blockIdx.x == 0) {
        for (int q = 0; q <= done; ++q) {
            const double rr = gather_sum(A.part + (size_t)(q * 4 + 1) * G, G, red);
            if (threadIdx.x == 0 && q <= MISSLAM_MAX_PCG) rep->pcg_resid[q] = sqrt(rr);
        }
        if (threadIdx.x == 0) {
            rep->pcg_iters_done = done;
            int f = rep->flags;
            if (stopped) f |= MISSLAM_FLAG_PCG_BREAKDOWN;
            if (nbad != 0.0) f |= MISSLAM_FLAG_NONFINITE;
            rep->flags = f;
        }
    }
}

// Grid shape of the persistent solve for m rows on this device, or 0 when a
// cooperative launch cannot hold it (the multi-kernel path is used then).
static int persistent_grid(int m, int &rows_per_wg) {
    static int max_blocks = -1;
    if (max_blocks < 0) {
        int dev = 0, cus = 0, per_cu = 0, coop = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pcg_persistent_kernel, kPcgThreads,
                                                         kPersistLdsBytes) != hipSuccess ||
            !coop)
            max_blocks = 0;
        else
            max_blocks = cus * (per_cu < 1 ? per_cu : 1);   // one workgroup per CU keeps the barriers small
    }
    if (max_blocks <= 0) return 0;
    rows_per_wg = (m + max_blocks - 1) / max_blocks;
    if (rows_per_wg > kRowsPerBlk) return 0;
    return (m + rows_per_wg - 1) / rows_per_wg;
}

hipError_t launch_pcg_persistent(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                                 float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                                 float *params, hipStream_t st, bool *used) {
    *used = false;
    int rows = 0;
    const int G = persistent_grid(m, rows);
    if (G <= 0 || G > s.nblk_max) return hipSuccess;
    PcgArgs A;
    A.row_ptr = g.row_ptr;
    A.col_idx = g.col_idx;
    A.blocks = blocks;
    A.minv = minv;
    A.g = gvec;
    A.lambda = lambda;
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
    const int mc_floats = rows * 144;
    const int cache_blocks = (kPersistLdsBytes / 4 - mc_floats) / 144;
    void *args[] = {&A, (void *)&rows, (void *)&cache_blocks, &rep, &params};
    const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(pcg_persistent_kernel), dim3(G),
                                                    dim3(kPcgThreads), args, kPersistLdsBytes, st);
    if (e == hipSuccess) *used = true;
    return e;
}


}  // namespace msl
