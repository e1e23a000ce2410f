// Model growth and maintenance after fusion (Alg. 2 steps 3-5, Alg. 3):
// removal of old light points, lifting of unregistered pixels (Group 2),
// merging of the points of every touched voxel, node regeneration.
//
// Every order is fixed: the new model is [surviving points in index order,
// lifted pixels in pixel order] with merged voxels kept at their lowest
// index; voxel groups come from a stable LSD radix sort of 63-bit voxel keys
// over the (ascending) point indices, so each group's members are in
// ascending index order and its float64 sums are formed in that order; new
// nodes are appended in ascending voxel-key order.  Compactions rank
// elements with wave ballots and per-block offsets from an exclusive scan.
#include "frame.h"

namespace msl {

constexpr int kGrowBlock = 256;
constexpr int kSortItems = 16;                          // keys per thread in one radix tile
constexpr int kSortTile = kGrowBlock * kSortItems;
constexpr int kKeyBits = 21;                            // per axis; voxel coordinates in [-2^20, 2^20)

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ __forceinline__ unsigned long long voxel_key(float x, float y, float z, double edge) {
    const double q[3] = {floor((double)x / edge), floor((double)y / edge), floor((double)z / edge)};
    unsigned long long k = 0;
#pragma unroll
    for (int a = 2; a >= 0; --a) {
        double v = q[a] + (double)(1 << (kKeyBits - 1));
        v = v < 0.0 ? 0.0 : (v > (double)((1 << kKeyBits) - 1) ? (double)((1 << kKeyBits) - 1) : v);
        if (!(v == v)) v = 0.0;
        k = (k << kKeyBits) | (unsigned long long)v;
    }
    return k;   // (kz, ky, kx) from the most significant bits down
}

// Rank of this thread's flag among the set flags of its block (threads in
// order), and the block's total; every thread of the block must call it.
__device__ __forceinline__ int block_rank(bool flag, int *total, int *lds_w) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const unsigned long long b = __ballot(flag);
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int in_wave = __popcll(b & lt);
    if (lane == 0) lds_w[wave] = __popcll(b);
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < kGrowBlock / kWave; ++w) {
        if (w < wave) base += lds_w[w];
        tot += lds_w[w];
    }
    __syncthreads();
    *total = tot;
    return base + in_wave;
}

// ---------------------------------------------------------------- scans

__global__ void __launch_bounds__(1024) exclusive_scan_kernel(const int32_t *__restrict__ in, int n,
                                                              int32_t *__restrict__ out, int32_t *__restrict__ total) {
    __shared__ int part[1024];
    const int chunk = (n + 1023) / 1024;
    const int c0 = min(n, (int)threadIdx.x * chunk), c1 = min(n, c0 + chunk);
    int s = 0;
    for (int i = c0; i < c1; ++i) s += in[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x == 0 ? 0 : part[threadIdx.x - 1];
    for (int i = c0; i < c1; ++i) {
        const int v = in[i];
        out[i] = run;
        run += v;
    }
    if (threadIdx.x == 1023 && total) *total = part[1023];
}

__global__ void __launch_bounds__(kGrowBlock) count_flags_kernel(const int32_t *__restrict__ flags, int64_t n,
                                                                 int32_t *__restrict__ counts) {
    __shared__ int lds_w[kGrowBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    int tot = 0;
    (void)block_rank(i < n && flags[i] != 0, &tot, lds_w);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// ---------------------------------------------------------------- stable LSD radix sort (keys u64, values u32)

__global__ void __launch_bounds__(kGrowBlock) radix_hist_kernel(const unsigned long long *__restrict__ keys,
                                                                int64_t n, int shift, int nb,
                                                                int32_t *__restrict__ hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    for (int e = 0; e < kSortItems; ++e) {
        const int64_t i = t0 + (int64_t)e * kGrowBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 0xFF)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];   // digit-major
}

// Each chunk of 256 keys (one per thread, tile order) is ranked per digit
// within its wave by 8 ballots, then across the waves and the chunks
// before it: equal digits keep their order.
__global__ void __launch_bounds__(kGrowBlock) radix_scatter_kernel(
    const unsigned long long *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n, int shift, int nb,
    const int32_t *__restrict__ offs, unsigned long long *__restrict__ okeys, uint32_t *__restrict__ ovals) {
    __shared__ int run[256];
    __shared__ int wcnt[kGrowBlock / kWave][256];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int e = 0; e < kSortItems; ++e) {
        for (int w = 0; w < kGrowBlock / kWave; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = t0 + (int64_t)e * kGrowBlock + threadIdx.x;
        const bool live = i < n;
        const unsigned long long k = live ? keys[i] : 0ull;
        const int d = (int)((k >> shift) & 0xFF);
        unsigned long long same = __ballot(live);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bb = __ballot(live && ((d >> bit) & 1));
            same &= ((d >> bit) & 1) ? bb : ~bb;
        }
        const int r_wave = __popcll(same & lt);
        if (live && r_wave == __popcll(same) - 1) wcnt[wave][d] = r_wave + 1;   // the last lane of the digit
        __syncthreads();
        if (live) {
            int base = run[d];
            for (int w = 0; w < wave; ++w) base += wcnt[w][d];
            const int64_t pos = base + r_wave;
            okeys[pos] = k;
            ovals[pos] = vals[i];
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kGrowBlock / kWave; ++w) add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// Sorts n pairs by key (stably) with 8-bit digits over the low `bits` bits;
// the result ends in (k0, v0) (an even pass count) after ping-ponging with (k1, v1).
static hipError_t radix_sort(unsigned long long *k0, uint32_t *v0, unsigned long long *k1, uint32_t *v1, int64_t n,
                             int bits, int32_t *hist, int32_t *offs, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)nblk(n, kSortTile);
    const int passes = ((bits + 7) / 8 + 1) / 2 * 2;
    for (int p = 0; p < passes; ++p) {
        unsigned long long *ki = p % 2 ? k1 : k0, *ko = p % 2 ? k0 : k1;
        uint32_t *vi = p % 2 ? v1 : v0, *vo = p % 2 ? v0 : v1;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kGrowBlock), 0, st, ki, n, 8 * p, nb, hist);
        hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, hist, 256 * nb, offs, nullptr);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kGrowBlock), 0, st, ki, vi, n, 8 * p, nb, offs, ko,
                           vo);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- growth steps

// Stability S_i (Sec. II-G, Alg. 3): stable once the weight (one per registration) has reached tau_weight,
// and from then on; without the flag plane the weight alone decides.
__device__ __forceinline__ bool point_stable(const GrowArgs &g, int64_t e) {
    return g.w[e] >= g.tau_weight || (g.stable && g.stable[e] != 0);
}

// flags over [existing points | pixels]: keep (Alg. 3 removal rule: an unstable point older than tau_time
// goes) and lift (Group 2)
__global__ void __launch_bounds__(kGrowBlock) grow_flags_kernel(GrowArgs g, int32_t *__restrict__ flags) {
    const int64_t e = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    const int64_t n = g.n, npx = (int64_t)g.cam.W * g.cam.H;
    if (e < n) {
        const bool del = (int64_t)g.frame - (int64_t)g.stamp[e] > (int64_t)g.tau_time && !point_stable(g, e);
        flags[e] = del ? 0 : 1;
    } else if (e < n + npx) {
        const int64_t t = e - n;
        const float4 q = g.nmap[t];
        const bool nvalid = !(q.x == 0.f && q.y == 0.f && q.z == 0.f);
        const int win = g.reg_map[t];
        const bool regd = win >= 0 && g.registered[win] != 0;
        flags[e] = (q.w > 0.f && nvalid && !regd) ? 1 : 0;
    }
}

// survivors and lifted pixels into the staging arrays, in order
__global__ void __launch_bounds__(kGrowBlock) grow_scatter_kernel(GrowArgs g, const int32_t *__restrict__ flags,
                                                                  const int32_t *__restrict__ offs) {
    __shared__ int lds_w[kGrowBlock / kWave];
    const int64_t e = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    const int64_t n = g.n, npx = (int64_t)g.cam.W * g.cam.H;
    const bool f = e < n + npx && flags[e] != 0;
    int tot = 0;
    const int r = block_rank(f, &tot, lds_w);
    if (!f) return;
    const int64_t pos = (int64_t)offs[blockIdx.x] + r;
    float *S = g.stage;
    const int64_t C = g.stage_cap;
    if (e < n) {
        S[pos] = g.px[e];
        S[C + pos] = g.py[e];
        S[2 * C + pos] = g.pz[e];
        S[3 * C + pos] = g.nx[e];
        S[4 * C + pos] = g.ny[e];
        S[5 * C + pos] = g.nz[e];
        S[6 * C + pos] = g.w[e];
        g.stage_stamp[pos] = g.stamp[e];
        if (g.stable) g.stage_stable[pos] = point_stable(g, e) ? 1 : 0;
        if (g.color)
#pragma unroll
            for (int c = 0; c < 3; ++c) g.stage_color[c * C + pos] = g.color[c * g.color_stride + e];
    } else {
        const int64_t t = e - n;
        const int u = (int)(t % g.cam.W), v = (int)(t / g.cam.W);
        const float4 q = g.nmap[t];
        const double d = q.w;
        const double V[3] = {d * (((double)u - (double)g.cam.cx) / (double)g.cam.fx),
                             d * (((double)v - (double)g.cam.cy) / (double)g.cam.fy), d};
        const double dv[3] = {V[0] - g.Td[0], V[1] - g.Td[1], V[2] - g.Td[2]};
        const double Nc[3] = {q.x, q.y, q.z};
        const double *R = g.Rd;
#pragma unroll
        for (int a = 0; a < 3; ++a) {   // R^T (V - T), R^T N
            S[a * C + pos] = (float)((R[a] * dv[0] + R[3 + a] * dv[1]) + R[6 + a] * dv[2]);
            S[(3 + a) * C + pos] = (float)((R[a] * Nc[0] + R[3 + a] * Nc[1]) + R[6 + a] * Nc[2]);
        }
        S[6 * C + pos] = 1.f;
        g.stage_stamp[pos] = g.frame;
        if (g.stable) g.stage_stable[pos] = 1.f >= g.tau_weight ? 1 : 0;   // a lifted point has weight 1
        if (g.color)   // a lifted point takes the frame's colour at its pixel
#pragma unroll
            for (int c = 0; c < 3; ++c) g.stage_color[c * C + pos] = g.image[t * 3 + c];
    }
}

// keys of the first min(*count, limit) points; the rest of [0, cap) sort last
__global__ void __launch_bounds__(kGrowBlock) key_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                         const float *__restrict__ z, const int32_t *__restrict__ count,
                                                         int64_t limit, int64_t cap, double edge,
                                                         unsigned long long *__restrict__ keys,
                                                         uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    if (i >= cap) return;
    const int64_t c = min((int64_t)*count, limit);
    keys[i] = i < c ? voxel_key(x[i], y[i], z[i], edge) : ~0ull;
    vals[i] = (uint32_t)i;
}

// One thread per group start in sorted order: merge the members of a touched
// voxel of two or more points into the first (lowest index) member.
__global__ void __launch_bounds__(kGrowBlock) merge_kernel(GrowArgs g, const unsigned long long *__restrict__ keys,
                                                           const uint32_t *__restrict__ idx,
                                                           int32_t *__restrict__ alive) {
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    const int64_t c = g.count[0];
    if (i >= c) return;
    const unsigned long long k = keys[i];
    if (i > 0 && keys[i - 1] == k) return;
    int64_t j1 = i + 1;
    while (j1 < c && keys[j1] == k) ++j1;
    float *S = g.stage;
    const int64_t C = g.stage_cap;
    bool touched = false;
    for (int64_t j = i; j < j1; ++j) touched = touched || g.stage_stamp[idx[j]] == g.frame;
    if (!touched || j1 - i < 2) return;
    double ps[3] = {0.0, 0.0, 0.0}, ns[3] = {0.0, 0.0, 0.0}, cs[3] = {0.0, 0.0, 0.0};
    float wmax = -__builtin_huge_valf();
    int smax = -2147483647 - 1;
    uint8_t sor = 0;
    for (int64_t j = i; j < j1; ++j) {   // ascending index
        const uint32_t q = idx[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ps[a] += (double)S[a * C + q];
            ns[a] += (double)S[(3 + a) * C + q];
            if (g.color) cs[a] += (double)g.stage_color[a * C + q];
        }
        wmax = fmaxf(wmax, S[6 * C + q]);
        smax = max(smax, g.stage_stamp[q]);
        if (g.stable) sor |= g.stage_stable[q];
        if (j > i) alive[q] = 0;
    }
    const double cnt = (double)(j1 - i);
    const uint32_t lead = idx[i];
    double nm[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        S[a * C + lead] = (float)(ps[a] / cnt);
        nm[a] = ns[a] / cnt;
    }
    const double nn = sqrt((nm[0] * nm[0] + nm[1] * nm[1]) + nm[2] * nm[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) S[(3 + a) * C + lead] = (float)(nm[a] / nn);
    S[6 * C + lead] = wmax;
    g.stage_stamp[lead] = smax;
    if (g.stable) g.stage_stable[lead] = sor;   // stable when a member is
    if (g.color)   // mean colour of the voxel
#pragma unroll
        for (int a = 0; a < 3; ++a) g.stage_color[a * C + lead] = (float)(cs[a] / cnt);
}

__global__ void __launch_bounds__(kGrowBlock) alive_init_kernel(int32_t *__restrict__ alive, const int32_t *count,
                                                                int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    if (i < cap) alive[i] = i < *count ? 1 : 0;
}

// surviving staged points back into the caller's arrays (up to its capacity)
__global__ void __launch_bounds__(kGrowBlock) final_scatter_kernel(GrowArgs g, const int32_t *__restrict__ alive,
                                                                   const int32_t *__restrict__ offs) {
    __shared__ int lds_w[kGrowBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    const bool f = i < g.stage_cap && alive[i] != 0;
    int tot = 0;
    const int r = block_rank(f, &tot, lds_w);
    if (!f) return;
    const int64_t pos = (int64_t)offs[blockIdx.x] + r;
    if (pos >= g.capacity) return;
    const float *S = g.stage;
    const int64_t C = g.stage_cap;
    g.px[pos] = S[i];
    g.py[pos] = S[C + i];
    g.pz[pos] = S[2 * C + i];
    g.nx[pos] = S[3 * C + i];
    g.ny[pos] = S[4 * C + i];
    g.nz[pos] = S[5 * C + i];
    g.w[pos] = S[6 * C + i];
    g.stamp[pos] = g.stage_stamp[i];
    if (g.stable) g.stable[pos] = g.stage_stable[i];
    if (g.color)
#pragma unroll
        for (int c = 0; c < 3; ++c) g.color[c * g.color_stride + pos] = g.stage_color[c * C + i];
}

// One thread per node-voxel group start: centroid (float64, ascending index)
// and whether no node of the frame lies within s of it.
__global__ void __launch_bounds__(kGrowBlock) node_candidate_kernel(GrowArgs g,
                                                                    const unsigned long long *__restrict__ keys,
                                                                    const uint32_t *__restrict__ idx,
                                                                    const int32_t *__restrict__ count,
                                                                    int32_t *__restrict__ flag,
                                                                    float *__restrict__ cent) {
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    if (i >= g.stage_cap) return;
    const int64_t c = min((int64_t)*count, g.capacity);
    flag[i] = 0;
    if (i >= c) return;
    const unsigned long long k = keys[i];
    if (i > 0 && keys[i - 1] == k) return;
    int64_t j1 = i + 1;
    while (j1 < c && keys[j1] == k) ++j1;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t j = i; j < j1; ++j) {
        const uint32_t q = idx[j];
        s[0] += (double)g.px[q];
        s[1] += (double)g.py[q];
        s[2] += (double)g.pz[q];
    }
    const double cnt = (double)(j1 - i);
    const double cx = s[0] / cnt, cy = s[1] / cnt, cz = s[2] / cnt;
    const double sp = g.node_spacing, s2 = sp * sp;
    bool near = false;
    for (int j = 0; j < g.m && !near; ++j) {
        const double dx = cx - (double)g.gx[j], dy = cy - (double)g.gy[j], dz = cz - (double)g.gz[j];
        near = ((dx * dx + dy * dy) + dz * dz) < s2;
    }
    if (near) return;
    flag[i] = 1;
    cent[3 * i] = (float)cx;
    cent[3 * i + 1] = (float)cy;
    cent[3 * i + 2] = (float)cz;
}

__global__ void __launch_bounds__(kGrowBlock) node_scatter_kernel(GrowArgs g, const int32_t *__restrict__ flag,
                                                                  const float *__restrict__ cent,
                                                                  const int32_t *__restrict__ offs) {
    __shared__ int lds_w[kGrowBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    const bool f = i < g.stage_cap && flag[i] != 0;
    int tot = 0;
    const int r = block_rank(f, &tot, lds_w);
    if (!f) return;
    const int64_t pos = (int64_t)g.m + offs[blockIdx.x] + r;
    if (pos >= g.node_capacity) return;
    g.gx[pos] = cent[3 * i];
    g.gy[pos] = cent[3 * i + 1];
    g.gz[pos] = cent[3 * i + 2];
    float *x = g.params + pos * 12;
#pragma unroll
    for (int t = 0; t < 12; ++t) x[t] = (t == 0 || t == 4 || t == 8) ? 1.f : 0.f;
}

// counts_out: new n, new m, lifted, removed, merged away, new nodes, overflow (0/1)
__global__ void grow_counts_kernel(GrowArgs g, const int32_t *__restrict__ flags, const int32_t *__restrict__ kept,
                                   const int32_t *__restrict__ alive_total, const int32_t *__restrict__ new_nodes,
                                   int64_t *__restrict__ out) {
    if (threadIdx.x != 0) return;
    (void)flags;
    const int64_t staged = g.count[0];
    const int64_t kept_n = kept[0];
    const int64_t alive = alive_total[0];
    const int64_t nn = new_nodes[0];
    const int64_t n_out = alive < g.capacity ? alive : g.capacity;
    const int64_t m_out = g.m + nn < g.node_capacity ? g.m + nn : g.node_capacity;
    out[0] = n_out;
    out[1] = m_out;
    out[2] = staged - kept_n;
    out[3] = g.n - kept_n;
    out[4] = staged - alive;
    out[5] = m_out - g.m;
    out[6] = (alive > g.capacity || g.m + nn > g.node_capacity) ? 1 : 0;
}

// the kept-point count: the flags of [0, n) summed by a second scan
__global__ void __launch_bounds__(kGrowBlock) kept_count_kernel(const int32_t *__restrict__ flags, int64_t n,
                                                                int32_t *__restrict__ counts) {
    __shared__ int lds_w[kGrowBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kGrowBlock + threadIdx.x;
    int tot = 0;
    (void)block_rank(i < n && flags[i] != 0, &tot, lds_w);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

hipError_t launch_grow(GrowArgs g, const GrowScratch &s, int64_t *counts_out, hipStream_t st) {
    const int64_t npx = (int64_t)g.cam.W * g.cam.H;
    const int64_t E = g.n + npx;                    // [existing | pixels]
    const int64_t C = g.stage_cap;                  // = E
    const unsigned nbE = nblk(E > 0 ? E : 1, kGrowBlock);
    const unsigned nbC = nblk(C > 0 ? C : 1, kGrowBlock);
    // 1. flags, counts, offsets; staged count -> s.count[0]
    hipLaunchKernelGGL(grow_flags_kernel, dim3(nbE), dim3(kGrowBlock), 0, st, g, s.flags);
    hipLaunchKernelGGL(count_flags_kernel, dim3(nbE), dim3(kGrowBlock), 0, st, s.flags, E, s.bcount);
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, s.bcount, (int)nbE, s.boffs, s.count);
    const unsigned nbN = nblk(g.n > 0 ? g.n : 1, kGrowBlock);
    hipLaunchKernelGGL(kept_count_kernel, dim3(nbN), dim3(kGrowBlock), 0, st, s.flags, g.n, s.bcount2);
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, s.bcount2, (int)nbN, s.boffs2, s.count + 1);
    hipLaunchKernelGGL(grow_scatter_kernel, dim3(nbE), dim3(kGrowBlock), 0, st, g, s.flags, s.boffs);
    // 2. voxel groups of the staged model, merge touched voxels
    const float *S = g.stage;
    hipLaunchKernelGGL(key_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, S, S + C, S + 2 * C, s.count, C, C,
                       (double)g.voxel, s.k0, s.v0);
    hipError_t e = radix_sort(s.k0, s.v0, s.k1, s.v1, C, 3 * kKeyBits, s.hist, s.hoffs, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(alive_init_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, s.alive, s.count, C);
    hipLaunchKernelGGL(merge_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, g, s.k0, s.v0, s.alive);
    // 3. compaction into the caller's arrays; final count -> s.count[2]
    hipLaunchKernelGGL(count_flags_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, s.alive, C, s.bcount);
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, s.bcount, (int)nbC, s.boffs, s.count + 2);
    hipLaunchKernelGGL(final_scatter_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, g, s.alive, s.boffs);
    // 4. node regeneration over the final points
    hipLaunchKernelGGL(key_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, g.px, g.py, g.pz, s.count + 2, g.capacity,
                       C, (double)g.node_spacing, s.k0, s.v0);
    e = radix_sort(s.k0, s.v0, s.k1, s.v1, C, 3 * kKeyBits, s.hist, s.hoffs, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(node_candidate_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, g, s.k0, s.v0, s.count + 2,
                       s.alive, s.cent);
    hipLaunchKernelGGL(count_flags_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, s.alive, C, s.bcount);
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, s.bcount, (int)nbC, s.boffs, s.count + 3);
    hipLaunchKernelGGL(node_scatter_kernel, dim3(nbC), dim3(kGrowBlock), 0, st, g, s.alive, s.cent, s.boffs);
    hipLaunchKernelGGL(grow_counts_kernel, dim3(1), dim3(64), 0, st, g, s.flags, s.count + 1, s.count + 2,
                       s.count + 3, counts_out);
    return hipGetLastError();
}

int64_t grow_hist_entries(int64_t cap) { return 256 * (int64_t)nblk(cap > 0 ? cap : 1, kSortTile); }

}  // namespace msl
