// Per-frame setup kernels: depth normal map, k nearest nodes with skinning
// weights (Eq.(2)), node graph N(j) (Eq.(6)) and block pattern, and the
// node -> point lists the assembly walks.  All integer results are
// deterministic: ordering decisions use float64 in a fixed operation order,
// adjacency is an idempotent bitmap, and lists are sorted by a unique key.
// Global atomics are integer only and never decide an order.
#include "frame.h"

namespace msl {

// ---------------------------------------------------------------- depth normal map (Eq.(8) inputs)

// One thread per pixel.  V(u,v) = D ((u-cx)/fx, (v-cy)/fy, 1); N = normalize(b x a)
// with a = V(u+1,v) - V(u-1,v), b = V(u,v+1) - V(u,v-1); float64, rounded at the end.
__global__ void __launch_bounds__(256) normal_map_kernel(const float *__restrict__ depth, Cam cam,
                                                         float4 *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npx = (int64_t)cam.W * cam.H;
    if (t >= npx) return;
    const int u = (int)(t % cam.W), v = (int)(t / cam.W);
    const float d0 = depth[t];
    float4 res = make_float4(0.f, 0.f, 0.f, d0);
    if (u >= 1 && u < cam.W - 1 && v >= 1 && v < cam.H - 1) {
        const float dl = depth[t - 1], dr = depth[t + 1], du = depth[t - cam.W], dd = depth[t + cam.W];
        if (d0 > 0.f && dl > 0.f && dr > 0.f && du > 0.f && dd > 0.f) {
            const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
            const double qxr = ((double)(u + 1) - cx) / fx, qxl = ((double)(u - 1) - cx) / fx;
            const double qxc = ((double)u - cx) / fx;
            const double qyd = ((double)(v + 1) - cy) / fy, qyu = ((double)(v - 1) - cy) / fy;
            const double qyc = ((double)v - cy) / fy;
            // a = V(u+1, v) - V(u-1, v)
            const double ax = (double)dr * qxr - (double)dl * qxl;
            const double ay = (double)dr * qyc - (double)dl * qyc;
            const double az = (double)dr - (double)dl;
            // b = V(u, v+1) - V(u, v-1)
            const double bx = (double)dd * qxc - (double)du * qxc;
            const double by = (double)dd * qyd - (double)du * qyu;
            const double bz = (double)dd - (double)du;
            const double cx_ = by * az - bz * ay;
            const double cy_ = bz * ax - bx * az;
            const double cz_ = bx * ay - by * ax;
            const double nn = sqrt((cx_ * cx_ + cy_ * cy_) + cz_ * cz_);
            if (nn > 0.0) {
                res.x = (float)(cx_ / nn);
                res.y = (float)(cy_ / nn);
                res.z = (float)(cz_ / nn);
            }
        }
    }
    out[t] = res;
}

// ---------------------------------------------------------------- kNN + skinning weights (Eq.(2))

constexpr int kKnnBlock = 256;
constexpr int kNodeTile = 2048;

// One thread per point; node coordinates staged through LDS in tiles.  Keeps
// the k+1 smallest (d^2, index) pairs, d^2 = ((dx dx + dy dy) + dz dz) in float64.
template <int K>
__global__ void __launch_bounds__(kKnnBlock) knn_kernel(PointsView pts, NodesView nd, int wkind, float sigma,
                                                        int32_t *__restrict__ idx_out, float *__restrict__ w_out) {
    __shared__ float sx[kNodeTile], sy[kNodeTile], sz[kNodeTile];
    const int64_t i = (int64_t)blockIdx.x * kKnnBlock + threadIdx.x;
    const bool live = i < pts.n;
    const double px = live ? (double)pts.px[i] : 0.0;
    const double py = live ? (double)pts.py[i] : 0.0;
    const double pz = live ? (double)pts.pz[i] : 0.0;
    constexpr int KK = K + 1;
    double bd[KK];
    int bi[KK];
#pragma unroll
    for (int s = 0; s < KK; ++s) {
        bd[s] = __builtin_huge_val();
        bi[s] = -1;
    }
    for (int base = 0; base < nd.m; base += kNodeTile) {
        const int cnt = min(kNodeTile, nd.m - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kKnnBlock) {
            sx[t] = nd.gx[base + t];
            sy[t] = nd.gy[base + t];
            sz[t] = nd.gz[base + t];
        }
        __syncthreads();
        if (!live) continue;
        for (int t = 0; t < cnt; ++t) {
            const double dx = px - (double)sx[t];
            const double dy = py - (double)sy[t];
            const double dz = pz - (double)sz[t];
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 < bd[KK - 1]) {
                // insert after every entry with distance <= d2 (equal distances keep the lower index first)
                double cd = d2;
                int ci = base + t;
#pragma unroll
                for (int s = 0; s < KK; ++s) {
                    if (cd < bd[s]) {
                        const double td = bd[s];
                        const int ti = bi[s];
                        bd[s] = cd;
                        bi[s] = ci;
                        cd = td;
                        ci = ti;
                    }
                }
            }
        }
    }
    if (!live) return;
    double wv[K];
    double sum = 0.0;
    if (wkind == MISSLAM_WEIGHT_GAUSS) {
        const double s2 = 2.0 * (double)sigma * (double)sigma;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            wv[s] = exp(-bd[s] / s2);
            sum += wv[s];
        }
    } else {
        const double dmax = sqrt(bd[K]);
#pragma unroll
        for (int s = 0; s < K; ++s) {
            double ws = 1.0 - sqrt(bd[s]) / dmax;
            ws = ws > 0.0 ? ws : 0.0;
            if (!(ws == ws) || !isfinite(ws)) ws = 0.0;
            wv[s] = ws;
            sum += wv[s];
        }
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        idx_out[(int64_t)s * pts.n + i] = bi[s];
        w_out[(int64_t)s * pts.n + i] = (float)(sum > 0.0 ? wv[s] / sum : 1.0 / K);
    }
}

// ---------------------------------------------------------------- node -> point lists

__global__ void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// LDS hash of the node ids met by one block of points: open addressing, twice
// as many slots as the block can insert, so probing always ends.
template <int K>
struct NodeHash {
    static constexpr int kSlots = 2 * 256 * K;
    int key[kSlots];
    int cnt[kSlots];
    int base[kSlots];
    int rank[kSlots];
};

template <int K>
__device__ __forceinline__ int hash_insert(NodeHash<K> &h, int j) {
    int s = (int)(((uint32_t)j * 2654435761u) % (uint32_t)NodeHash<K>::kSlots);
    while (true) {
        const int old = atomicCAS(&h.key[s], -1, j);
        if (old == -1 || old == j) return s;
        s = s + 1 == NodeHash<K>::kSlots ? 0 : s + 1;
    }
}

template <int K>
__device__ __forceinline__ int hash_find(const NodeHash<K> &h, int j) {
    int s = (int)(((uint32_t)j * 2654435761u) % (uint32_t)NodeHash<K>::kSlots);
    while (h.key[s] != j) s = s + 1 == NodeHash<K>::kSlots ? 0 : s + 1;
    return s;
}

// Entries per node: counted per block in LDS, one global add per distinct node.
template <int K>
__global__ void __launch_bounds__(256) list_count_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                         int32_t *__restrict__ cnt) {
    __shared__ NodeHash<K> h;
    for (int t = threadIdx.x; t < NodeHash<K>::kSlots; t += 256) {
        h.key[t] = -1;
        h.cnt[t] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
#pragma unroll
        for (int s = 0; s < K; ++s) atomicAdd(&h.cnt[hash_insert<K>(h, idx[(int64_t)s * n + i])], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NodeHash<K>::kSlots; t += 256)
        if (h.key[t] >= 0) atomicAdd(&cnt[h.key[t]], h.cnt[t]);
}

// Unordered placement (list_sort_kernel imposes the order): each block reserves
// one contiguous range per distinct node, then ranks its entries in LDS.
template <int K>
__global__ void __launch_bounds__(256) list_fill_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                        const int32_t *__restrict__ ptr, int32_t *__restrict__ cursor,
                                                        int32_t *__restrict__ list) {
    __shared__ NodeHash<K> h;
    for (int t = threadIdx.x; t < NodeHash<K>::kSlots; t += 256) {
        h.key[t] = -1;
        h.cnt[t] = 0;
        h.rank[t] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int q[K];
    if (i < n) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            q[s] = idx[(int64_t)s * n + i];
            atomicAdd(&h.cnt[hash_insert<K>(h, q[s])], 1);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NodeHash<K>::kSlots; t += 256)
        if (h.key[t] >= 0) h.base[t] = atomicAdd(&cursor[h.key[t]], h.cnt[t]);
    __syncthreads();
    if (i < n) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int sl = hash_find<K>(h, q[s]);
            const int r = atomicAdd(&h.rank[sl], 1);
            list[ptr[q[s]] + h.base[sl] + r] = (int32_t)i;
        }
    }
}

// Sorted k-node set of a point packed 16 bits per node: hi = nodes 0..3, lo = nodes 4..7,
// unused slots 0xFFFF.
template <int K>
__device__ __forceinline__ void sorted_set(const int32_t *__restrict__ idx, int64_t n, int64_t i, int *q) {
#pragma unroll
    for (int s = 0; s < 8; ++s) q[s] = s < K ? idx[(int64_t)s * n + i] : 0xFFFF;
#pragma unroll
    for (int a = 1; a < K; ++a)
#pragma unroll
        for (int b = a; b > 0; --b)
            if (q[b] < q[b - 1]) {
                const int t = q[b];
                q[b] = q[b - 1];
                q[b - 1] = t;
            }
}

template <int K>
__device__ __forceinline__ void set_key(const int32_t *__restrict__ idx, int64_t n, int64_t i, uint64_t &hi,
                                        uint64_t &lo) {
    int q[8];
    sorted_set<K>(idx, n, i, q);
    hi = ((uint64_t)q[0] << 48) | ((uint64_t)q[1] << 32) | ((uint64_t)q[2] << 16) | (uint64_t)q[3];
    lo = ((uint64_t)q[4] << 48) | ((uint64_t)q[5] << 32) | ((uint64_t)q[6] << 16) | (uint64_t)q[7];
}

__device__ __forceinline__ bool key_less(uint64_t ah, uint64_t al, uint32_t ap, uint64_t bh, uint64_t bl,
                                         uint32_t bp) {
    if (ah != bh) return ah < bh;
    if (al != bl) return al < bl;
    return ap < bp;
}

// One block per node: bitonic sort of its list by (sorted node set, point index) in LDS.
template <int K>
__global__ void __launch_bounds__(256) list_sort_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                        const int32_t *__restrict__ ptr,
                                                        int32_t *__restrict__ list) {
    __shared__ uint64_t kh[MISSLAM_MAX_LIST];
    __shared__ uint64_t kl[K > 4 ? MISSLAM_MAX_LIST : 1];
    __shared__ uint32_t kp[MISSLAM_MAX_LIST];
    const int j = blockIdx.x;
    const int b = ptr[j];
    const int c = min(ptr[j + 1] - b, MISSLAM_MAX_LIST);
    int P = 1;
    while (P < c) P <<= 1;
    for (int t = threadIdx.x; t < P; t += 256) {
        uint64_t h = ~0ull, l = ~0ull;
        uint32_t p = 0xFFFFFFFFu;
        if (t < c) {
            p = (uint32_t)list[b + t];
            set_key<K>(idx, n, p, h, l);
        }
        kh[t] = h;
        if (K > 4) kl[t] = l;
        kp[t] = p;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P; t += 256) {
                const int o = t ^ stride;
                if (o > t) {
                    const bool up = (t & size) == 0;
                    const uint64_t th = kh[t], oh = kh[o];
                    const uint32_t tp = kp[t], op = kp[o];
                    const uint64_t tl = K > 4 ? kl[t] : 0, ol = K > 4 ? kl[o] : 0;
                    if (key_less(oh, ol, op, th, tl, tp) == up) {
                        kh[t] = oh;
                        kh[o] = th;
                        kp[t] = op;
                        kp[o] = tp;
                        if (K > 4) {
                            kl[t] = ol;
                            kl[o] = tl;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < c; t += 256) list[b + t] = (int32_t)kp[t];
}

// ---------------------------------------------------------------- node graph and block pattern

// One block per node j: row j = {j} U {nodes sharing a point with j}, read off
// the sorted list (one representative per distinct set) into an LDS bitmap,
// then extracted in ascending order.  Rows longer than MISSLAM_MAX_ROW are cut
// there and flagged.
template <int K>
__global__ void __launch_bounds__(256) row_collect_kernel(const int32_t *__restrict__ idx, int64_t n, int m,
                                                          const int32_t *__restrict__ lptr,
                                                          const int32_t *__restrict__ list, int32_t *__restrict__ tmp,
                                                          int32_t *__restrict__ cnt, int32_t *__restrict__ info) {
    __shared__ uint32_t bm[2048];
    __shared__ int wsum[257];
    const int j = blockIdx.x;
    const int words = (m + 31) / 32;
    for (int t = threadIdx.x; t < words; t += 256) bm[t] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) atomicOr(&bm[j >> 5], 1u << (j & 31));
    const int b = lptr[j];
    const int c = min(lptr[j + 1] - b, MISSLAM_MAX_LIST);
    for (int t = threadIdx.x; t < c; t += 256) {
        const int p = list[b + t];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int q = idx[(int64_t)s * n + p];
            const uint32_t bit = 1u << (q & 31);
            if (!(bm[q >> 5] & bit)) atomicOr(&bm[q >> 5], bit);
        }
    }
    __syncthreads();
    // per-thread contiguous word range, block prefix of bit counts
    const int per = (words + 255) / 256;
    const int w0 = min(words, (int)threadIdx.x * per), w1 = min(words, w0 + per);
    int mine = 0;
    for (int w = w0; w < w1; ++w) mine += __popc(bm[w]);
    wsum[threadIdx.x + 1] = mine;
    if (threadIdx.x == 0) wsum[0] = 0;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int t = 1; t <= 256; ++t) wsum[t] += wsum[t - 1];
    __syncthreads();
    int pos = wsum[threadIdx.x];
    for (int w = w0; w < w1; ++w) {
        uint32_t bb = bm[w];
        while (bb) {
            const int bit = __ffs(bb) - 1;
            bb &= bb - 1;
            if (pos < MISSLAM_MAX_ROW) tmp[(size_t)j * MISSLAM_MAX_ROW + pos] = w * 32 + bit;
            ++pos;
        }
    }
    if (threadIdx.x == 0) {
        const int total = wsum[256];
        cnt[j] = min(total, MISSLAM_MAX_ROW);
        if (total > MISSLAM_MAX_ROW) atomicOr(&info[3], MISSLAM_FLAG_GRAPH_OVERFLOW);
    }
}

// One block per node j: writes row j's columns and, for every entry of list(j),
// the row positions of the entry's k nodes (sorted by node index), 8 bits each
// (0xFF = not in the row), two words per entry.
template <int K>
__global__ void __launch_bounds__(256) row_keys_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                       const int32_t *__restrict__ tmp,
                                                       const int32_t *__restrict__ row_ptr, int cap,
                                                       int32_t *__restrict__ col_idx, const int32_t *__restrict__ lptr,
                                                       const int32_t *__restrict__ list, uint32_t *__restrict__ key) {
    __shared__ int cols[MISSLAM_MAX_ROW];
    const int j = blockIdx.x;
    const int rb = row_ptr[j];
    const int len = row_ptr[j + 1] - rb;
    for (int t = threadIdx.x; t < len; t += 256) {
        const int c = tmp[(size_t)j * MISSLAM_MAX_ROW + t];
        cols[t] = c;
        if (rb + t < cap) col_idx[rb + t] = c;
    }
    __syncthreads();
    const int b = lptr[j];
    const int c = lptr[j + 1] - b;
    for (int t = threadIdx.x; t < c; t += 256) {
        int q[8];
        sorted_set<K>(idx, n, list[b + t], q);
        uint32_t k0 = 0, k1 = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            int lo = 0, hi = len;   // binary search in the ascending row
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cols[mid] < q[s])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            const uint32_t slot = (lo < len && cols[lo] == q[s]) ? (uint32_t)lo : 0xFFu;
            if (s < 4)
                k0 |= slot << (8 * s);
            else
                k1 |= slot << (8 * (s - 4));
        }
        key[2 * (size_t)(b + t)] = k0;
        key[2 * (size_t)(b + t) + 1] = k1;
    }
}

// Exclusive scan of m counts into ptr[0..m] in one block; also records the
// largest count and whether it exceeded cap_each / the total exceeded cap_total.
__global__ void __launch_bounds__(1024) scan_kernel(const int32_t *__restrict__ cnt, int m, int32_t *__restrict__ ptr,
                                                    int32_t *__restrict__ info, int info_total, int info_max,
                                                    int cap_each, int64_t cap_total) {
    __shared__ int64_t part[1024];
    __shared__ int mx[1024];
    const int T = 1024;
    const int per = (m + T - 1) / T;
    const int b0 = threadIdx.x * per;
    const int b1 = min(m, b0 + per);
    int64_t s = 0;
    int lm = 0;
    for (int j = b0; j < b1; ++j) {
        s += cnt[j];
        lm = max(lm, cnt[j]);
    }
    part[threadIdx.x] = s;
    mx[threadIdx.x] = lm;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        int64_t v = ((int)threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
        int w = ((int)threadIdx.x >= off) ? mx[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        mx[threadIdx.x] = max(mx[threadIdx.x], w);
        __syncthreads();
    }
    int64_t run = threadIdx.x == 0 ? 0 : part[threadIdx.x - 1];
    for (int j = b0; j < b1; ++j) {
        ptr[j] = (int32_t)run;
        run += cnt[j];
    }
    if (threadIdx.x == T - 1) {
        const int64_t total = part[T - 1];
        ptr[m] = (int32_t)total;
        if (info_total >= 0) info[info_total] = (int32_t)total;
        if (info_max >= 0) info[info_max] = mx[T - 1];
        if (mx[T - 1] > cap_each || total > cap_total) atomicOr(&info[3], MISSLAM_FLAG_GRAPH_OVERFLOW);
    }
}

// ---------------------------------------------------------------- launch wrappers

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_normal_map(const float *depth, const Cam &cam, float4 *out, hipStream_t st) {
    const int64_t npx = (int64_t)cam.W * cam.H;
    if (npx == 0) return hipSuccess;
    hipLaunchKernelGGL(normal_map_kernel, dim3(nblk(npx, 256)), dim3(256), 0, st, depth, cam, out);
    return hipGetLastError();
}

template <int K>
static hipError_t graph_k(const PointsView &pts, const NodesView &nd, int wkind, float sigma, const GraphView &g,
                          const GraphScratch &s, hipStream_t st) {
    const int64_t n = pts.n;
    const int m = nd.m;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(nblk(2 * (int64_t)m + 8, 256)), dim3(256), 0, st, (uint32_t *)s.cnt,
                       (size_t)(2 * m + 8), 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)g.info, (size_t)8, 0u);
    int32_t *lcnt = s.cnt + m;
    if (n > 0) {
        hipLaunchKernelGGL((knn_kernel<K>), dim3(nblk(n, kKnnBlock)), dim3(kKnnBlock), 0, st, pts, nd, wkind, sigma,
                           g.knn_idx, g.knn_w);
        hipLaunchKernelGGL((list_count_kernel<K>), dim3(nblk(n, 256)), dim3(256), 0, st, g.knn_idx, n, lcnt);
    }
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, lcnt, m, g.list_ptr, g.info, -1, 2,
                       MISSLAM_MAX_LIST, (int64_t)K * n);
    if (n > 0) {
        hipLaunchKernelGGL((list_fill_kernel<K>), dim3(nblk(n, 256)), dim3(256), 0, st, g.knn_idx, n, g.list_ptr,
                           s.cnt, g.list_pts);
        hipLaunchKernelGGL((list_sort_kernel<K>), dim3(m), dim3(256), 0, st, g.knn_idx, n, g.list_ptr, g.list_pts);
    }
    hipLaunchKernelGGL((row_collect_kernel<K>), dim3(m), dim3(256), 0, st, g.knn_idx, n, m, g.list_ptr, g.list_pts,
                       s.tmp, s.cnt, g.info);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, s.cnt, m, g.row_ptr, g.info, 0, 1, MISSLAM_MAX_ROW,
                       (int64_t)g.bsr_cap);
    hipLaunchKernelGGL((row_keys_kernel<K>), dim3(m), dim3(256), 0, st, g.knn_idx, n, s.tmp, g.row_ptr, g.bsr_cap,
                       g.col_idx, g.list_ptr, g.list_pts, g.list_key);
    return hipGetLastError();
}

hipError_t launch_build_graph(const PointsView &pts, const NodesView &nd, int k, int wkind, float sigma,
                              const GraphView &g, const GraphScratch &s, hipStream_t st) {
    switch (k) {
        case 1: return graph_k<1>(pts, nd, wkind, sigma, g, s, st);
        case 2: return graph_k<2>(pts, nd, wkind, sigma, g, s, st);
        case 3: return graph_k<3>(pts, nd, wkind, sigma, g, s, st);
        case 4: return graph_k<4>(pts, nd, wkind, sigma, g, s, st);
        case 5: return graph_k<5>(pts, nd, wkind, sigma, g, s, st);
        case 6: return graph_k<6>(pts, nd, wkind, sigma, g, s, st);
        case 7: return graph_k<7>(pts, nd, wkind, sigma, g, s, st);
        case 8: return graph_k<8>(pts, nd, wkind, sigma, g, s, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace msl
