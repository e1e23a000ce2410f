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
__device__ __forceinline__ void normal_map_body(const float *__restrict__ depth, const Cam &cam,
                                                float4 *__restrict__ out, int64_t blk) {
    const int64_t t = blk * 256 + threadIdx.x;
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

__global__ void __launch_bounds__(256) normal_map_kernel(const float *__restrict__ depth, Cam cam,
                                                         float4 *__restrict__ out) {
    normal_map_body(depth, cam, out, blockIdx.x);
}

// The normal maps of a batch of problems in one grid.
__global__ void __launch_bounds__(256) normal_map_batched_kernel(const BatchItem *__restrict__ items, int count) {
    int b = count - 1;
    while (b > 0 && items[b].nm0 > (int)blockIdx.x) --b;
    const BatchItem &it = items[b];
    normal_map_body(it.depth, it.a.cam, const_cast<float4 *>(it.a.nmap), (int64_t)blockIdx.x - it.nm0);
}

// ---------------------------------------------------------------- kNN + skinning weights (Eq.(2))

constexpr int kKnnBlock = 256;
constexpr int kGridThreads = 1024;

// Uniform grid over the node bounding box: header, cell offsets (counting
// sort) and the nodes in cell order as (x, y, z, index bits).  Cell width
// h = 2 sqrt(A / m), A the product of the two largest box extents (about
// twice the node spacing of a surface-sampled graph), widened until the
// cell count fits MSL_GRID_CELLS.  The width only affects speed: the search
// below is exact for any h.  One workgroup.
constexpr int kGridLdsCells = 4096;   // grids up to this many cells are sorted in LDS

// zero_a / zero_b (na / nb words, may be null): counters the graph build clears before its later kernels.
__global__ void __launch_bounds__(kGridThreads) node_grid_kernel(NodesView nd, GridView gv, uint32_t *zero_a,
                                                                 size_t na, uint32_t *zero_b, size_t nb) {
    __shared__ float red[6][kGridThreads];
    __shared__ int part[kGridThreads];
    __shared__ int cell_s[kGridLdsCells + 1];   // counts, then fill cursors, of a grid that fits
    const int m = nd.m, tid = threadIdx.x;
    for (size_t t = tid; t < na; t += kGridThreads) zero_a[t] = 0u;
    for (size_t t = tid; t < nb; t += kGridThreads) zero_b[t] = 0u;
    float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
    float hi[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
    for (int t = tid; t < m; t += kGridThreads) {
        const float c[3] = {nd.gx[t], nd.gy[t], nd.gz[t]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], c[a]);
            hi[a] = fmaxf(hi[a], c[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        red[a][tid] = lo[a];
        red[3 + a][tid] = hi[a];
    }
    __syncthreads();
    for (int off = kGridThreads / 2; off > 0; off >>= 1) {
        if (tid < off) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                red[a][tid] = fminf(red[a][tid], red[a][tid + off]);
                red[3 + a][tid] = fmaxf(red[3 + a][tid], red[3 + a][tid + off]);
            }
        }
        __syncthreads();
    }
    // header (identical in every thread)
    double org[3], ext[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        org[a] = m > 0 ? (double)red[a][0] : 0.0;
        ext[a] = m > 0 ? (double)red[3 + a][0] - org[a] : 0.0;
        if (!(ext[a] >= 0.0) || !isfinite(ext[a])) ext[a] = 0.0;   // non-finite nodes: one cell on that axis
    }
    double e0 = fmax(ext[0], fmax(ext[1], ext[2]));
    double e2 = fmin(ext[0], fmin(ext[1], ext[2]));
    double e1 = ext[0] + ext[1] + ext[2] - e0 - e2;
    double h = 2.0 * sqrt(fmax(e0 * e1, 1e-12) / (double)(m > 0 ? m : 1));
    if (!(h > 0.0) || !isfinite(h)) h = 1.0;
    int dim[3];
    for (int guard = 0; guard < 200; ++guard) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            const double q = floor(ext[a] / h) + 1.0;
            dim[a] = q < 1e6 ? (int)q : 1000000;
            tot *= dim[a];
        }
        if (tot <= MSL_GRID_CELLS) break;
        h *= 1.25;
    }
    const int ncell = m > 0 ? dim[0] * dim[1] * dim[2] : 0;
    if (tid == 0) {
        gv.hdr[0] = org[0];
        gv.hdr[1] = org[1];
        gv.hdr[2] = org[2];
        gv.hdr[3] = h;
        gv.dims[0] = m > 0 ? dim[0] : 0;
        gv.dims[1] = m > 0 ? dim[1] : 0;
        gv.dims[2] = m > 0 ? dim[2] : 0;
    }
    const double ih = 1.0 / h;
    auto cell_of = [&](int t) {
        const double c[3] = {(double)nd.gx[t], (double)nd.gy[t], (double)nd.gz[t]};
        int q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double f = floor((c[a] - org[a]) * ih);
            q[a] = f >= 0.0 ? (f < (double)(dim[a] - 1) ? (int)f : dim[a] - 1) : 0;   // NaN -> 0
        }
        return (q[2] * dim[1] + q[1]) * dim[0] + q[0];
    };
    if (ncell <= kGridLdsCells) {   // counting sort in LDS: counts, an exclusive scan, cursors
        for (int c = tid; c <= ncell; c += kGridThreads) cell_s[c] = 0;
        __syncthreads();
        for (int t = tid; t < m; t += kGridThreads) atomicAdd(&cell_s[cell_of(t)], 1);
        __syncthreads();
        const int chunk = (ncell + kGridThreads - 1) / kGridThreads;
        const int c0 = min(ncell, tid * chunk), c1 = min(ncell, c0 + chunk);
        int sum = 0;
        for (int c = c0; c < c1; ++c) sum += cell_s[c];
        part[tid] = sum;
        __syncthreads();
        for (int off = 1; off < kGridThreads; off <<= 1) {
            const int v = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        int run = tid == 0 ? 0 : part[tid - 1];
        for (int c = c0; c < c1; ++c) {
            const int v = cell_s[c];
            gv.start[c] = run;
            cell_s[c] = run;
            run += v;
        }
        if (tid == 0) gv.start[ncell] = m;
        __syncthreads();
        for (int t = tid; t < m; t += kGridThreads) {
            const int pos = atomicAdd(&cell_s[cell_of(t)], 1);
            gv.nodes[pos] = make_float4(nd.gx[t], nd.gy[t], nd.gz[t], __int_as_float(t));
        }
        return;
    }
    // a larger grid: the same in global memory
    for (int c = tid; c <= ncell; c += kGridThreads) gv.start[c] = 0;
    __syncthreads();
    for (int t = tid; t < m; t += kGridThreads) atomicAdd(&gv.start[cell_of(t)], 1);
    __syncthreads();
    // exclusive scan of ncell counts: each thread a contiguous chunk
    const int chunk = (ncell + kGridThreads - 1) / kGridThreads;
    const int c0 = min(ncell, tid * chunk), c1 = min(ncell, c0 + chunk);
    int sum = 0;
    // counts were formed by atomics in the L2: read them from there
    for (int c = c0; c < c1; ++c) sum += __hip_atomic_load(&gv.start[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kGridThreads; off <<= 1) {
        const int v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = tid == 0 ? 0 : part[tid - 1];
    for (int c = c0; c < c1; ++c) {
        const int v = __hip_atomic_load(&gv.start[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        gv.start[c] = run;
        gv.cursor[c] = run;
        run += v;
    }
    if (tid == 0) gv.start[ncell] = m;
    __syncthreads();
    for (int t = tid; t < m; t += kGridThreads) {
        const int pos = atomicAdd(&gv.cursor[cell_of(t)], 1);
        gv.nodes[pos] = make_float4(nd.gx[t], nd.gy[t], nd.gz[t], __int_as_float(t));
    }
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

// The node counts alone (the kNN kernel's share of the list lengths).
template <int K>
struct NodeCount {
    static constexpr int kSlots = NodeHash<K>::kSlots;
    int key[kSlots];
    int cnt[kSlots];
};

template <int K, class H>
__device__ __forceinline__ int hash_insert(H &h, int j) {
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
// Keeps the KK smallest (d^2, index) pairs in lexicographic order (equal
// distances: lower index first), so the result does not depend on the order
// in which candidates arrive.
template <int KK>
__device__ __forceinline__ void knn_insert(double (&bd)[KK], int (&bi)[KK], double d2, int idx) {
    if (!(d2 < bd[KK - 1] || (d2 == bd[KK - 1] && (unsigned)idx < (unsigned)bi[KK - 1]))) return;
    double cd = d2;
    int ci = idx;
#pragma unroll
    for (int s = 0; s < KK; ++s) {
        if (cd < bd[s] || (cd == bd[s] && (unsigned)ci < (unsigned)bi[s])) {
            const double td = bd[s];
            const int ti = bi[s];
            bd[s] = cd;
            bi[s] = ci;
            cd = td;
            ci = ti;
        }
    }
}

// One thread per point.  d^2 = ((dx dx + dy dy) + dz dz) in float64 against
// the nodes of the point's grid cell, then of the shells of cells at
// Chebyshev cell distance r = 1, 2, ...  Every node outside the cells seen
// lies farther than r h from the point, so the search stops once the
// (k+1)-th best d^2 is below (r h)^2 (with a margin for the rounding of the
// cell index) or the cube covers the grid: the result equals the exhaustive
// search.  The weights of Eq.(2) follow in float64.
template <int K>
__device__ __forceinline__ void knn_point(PointsView pts, GridView gv, int wkind, float sigma,
                                          int32_t *__restrict__ idx_out, float *__restrict__ w_out, int64_t i,
                                          NodeCount<K> &hc) {
    const double px = (double)pts.px[i], py = (double)pts.py[i], pz = (double)pts.pz[i];
    constexpr int KK = K + 1;
    double bd[KK];
    int bi[KK];
#pragma unroll
    for (int s = 0; s < KK; ++s) {
        bd[s] = __builtin_huge_val();
        bi[s] = -1;
    }
    const int dx = gv.dims[0], dy = gv.dims[1], dz = gv.dims[2];
    if (dx > 0) {
        const double h = gv.hdr[3], ih = 1.0 / h;
        const double p[3] = {px, py, pz};
        const int dim[3] = {dx, dy, dz};
        int q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double f = floor((p[a] - gv.hdr[a]) * ih);
            q[a] = f >= 0.0 ? (f < (double)(dim[a] - 1) ? (int)f : dim[a] - 1) : 0;
        }
        const int rmax = max(max(max(q[0], dx - 1 - q[0]), max(q[1], dy - 1 - q[1])), max(q[2], dz - 1 - q[2]));
        for (int r = 0; r <= rmax; ++r) {
            const int z0 = max(0, q[2] - r), z1 = min(dz - 1, q[2] + r);
            const int y0 = max(0, q[1] - r), y1 = min(dy - 1, q[1] + r);
            const int x0 = max(0, q[0] - r), x1 = min(dx - 1, q[0] + r);
            for (int cz = z0; cz <= z1; ++cz) {
                for (int cy = y0; cy <= y1; ++cy) {
                    const bool face = abs(cz - q[2]) == r || abs(cy - q[1]) == r;
                    // on a face row every x; otherwise only the two x ends of the shell
                    const int step = face ? 1 : 2 * r;
                    for (int cx = face ? x0 : q[0] - r; cx <= (face ? x1 : q[0] + r); cx += step > 0 ? step : 1) {
                        if (cx < 0 || cx >= dx) continue;
                        const int c = (cz * dy + cy) * dx + cx;
                        const int n0 = gv.start[c], n1 = gv.start[c + 1];
                        for (int t = n0; t < n1; ++t) {
                            const float4 g = gv.nodes[t];
                            const double ex = px - (double)g.x;
                            const double ey = py - (double)g.y;
                            const double ez = pz - (double)g.z;
                            knn_insert<KK>(bd, bi, (ex * ex + ey * ey) + ez * ez, __float_as_int(g.w));
                        }
                    }
                }
            }
            const double b = ((double)r - 1e-6) * h;
            if (b > 0.0 && bd[KK - 1] < b * b) break;
        }
    }
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
        atomicAdd(&hc.cnt[hash_insert<K>(hc, bi[s])], 1);
    }
}

template <int K>
__global__ void __launch_bounds__(kKnnBlock) knn_kernel(PointsView pts, GridView gv, int wkind, float sigma,
                                                        int32_t *__restrict__ idx_out, float *__restrict__ w_out,
                                                        int32_t *__restrict__ list_cnt) {
    // the block's kNN sets are also counted per node (an LDS hash, then one device atomic per distinct node):
    // the lengths of the node -> point lists
    __shared__ NodeCount<K> hc;
    for (int t = threadIdx.x; t < NodeCount<K>::kSlots; t += kKnnBlock) {
        hc.key[t] = -1;
        hc.cnt[t] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kKnnBlock + threadIdx.x;
    if (i < pts.n) knn_point<K>(pts, gv, wkind, sigma, idx_out, w_out, i, hc);
    __syncthreads();
    for (int t = threadIdx.x; t < NodeCount<K>::kSlots; t += kKnnBlock)
        if (hc.key[t] >= 0) atomicAdd(&list_cnt[hc.key[t]], hc.cnt[t]);
}

// ---------------------------------------------------------------- node -> point lists

__global__ void fill_u32_kernel(uint32_t *p, size_t n, uint32_t v) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
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

// One block per node: its list sorted by (sorted node set, point index).  A list of up to MISSLAM_MAX_LIST
// entries is bitonic-sorted in one piece; a longer one is sorted in pieces of MISSLAM_MAX_LIST, which are then
// merged pairwise in global memory through tmp (the same positions as the list), each merge split over the
// block's threads along the merge path.  The order is a total one (point indices are distinct), so the result
// does not depend on the way it was reached.
constexpr int kSortThreads = 256;

template <int K>
__device__ __forceinline__ bool entry_less(const int32_t *__restrict__ idx, int64_t n, uint32_t a, uint32_t b) {
    uint64_t ah, al, bh, bl;
    set_key<K>(idx, n, a, ah, al);
    set_key<K>(idx, n, b, bh, bl);
    return key_less(ah, K > 4 ? al : 0, a, bh, K > 4 ? bl : 0, b);
}

// Merges the sorted runs src[0, la) and src[la, la + lb) into dst[0, la + lb), split over the block's threads.
template <int K>
__device__ void merge_runs(const int32_t *__restrict__ idx, int64_t n, const int32_t *src, int la, int lb,
                           int32_t *dst) {
    const int T = la + lb;
    const int per = (T + kSortThreads - 1) / kSortThreads;
    const int d0 = min(T, (int)threadIdx.x * per), d1 = min(T, d0 + per);
    if (d0 >= d1) return;
    // merge path: the number of entries of run A among the first d0 of the output
    int lo = max(0, d0 - lb), hi = min(d0, la);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        // take A[mid] before B[d0 - mid - 1]?
        if (entry_less<K>(idx, n, (uint32_t)src[mid], (uint32_t)src[la + d0 - mid - 1]))
            lo = mid + 1;
        else
            hi = mid;
    }
    int ia = lo, ib = d0 - lo;
    for (int d = d0; d < d1; ++d) {
        bool take_a;
        if (ia >= la) take_a = false;
        else if (ib >= lb) take_a = true;
        else take_a = entry_less<K>(idx, n, (uint32_t)src[ia], (uint32_t)src[la + ib]);
        dst[d] = take_a ? src[ia++] : src[la + ib++];
    }
}

// A list entry's sort key: the sorted k-node set (l is 0 for k <= 4) and the point index.
struct SortKey {
    uint64_t h, l;
    uint32_t p;
};

__device__ __forceinline__ bool sk_less(const SortKey &a, const SortKey &b) {
    return key_less(a.h, a.l, a.p, b.h, b.l, b.p);
}

// The bitonic network over one piece of P = kSortThreads * E entries (padded with keys above every entry).
// Thread t holds entries t E .. t E + E - 1 in registers: a stage whose partner is in the same thread swaps
// registers, one whose partner is in the same wave exchanges with __shfl_xor, and only a stage whose partner
// is in another wave goes through LDS (3 of the 36-66 stages), with a barrier.
template <int K, int E, int S>
__device__ __forceinline__ void bitonic_in_thread(SortKey (&x)[E], int i0, int size) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if ((e & S) != 0 || e + S >= E) continue;
        const bool asc = ((i0 + e) & size) == 0;
        const SortKey a = x[e], b = x[e + S];
        const bool sw = sk_less(b, a) == asc;
        x[e] = sw ? b : a;
        x[e + S] = sw ? a : b;
    }
}

template <int K, int E>
__device__ __forceinline__ void sort_piece(const int32_t *__restrict__ idx, int64_t n, int32_t *__restrict__ lst,
                                           int c, uint64_t *kh, uint64_t *kl, uint32_t *kp) {
    constexpr int P = kSortThreads * E;
    const int i0 = (int)threadIdx.x * E;
    SortKey x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        x[e].h = ~0ull;
        x[e].l = K > 4 ? ~0ull : 0ull;
        x[e].p = 0xFFFFFFFFu;
        if (i0 + e < c) {
            x[e].p = (uint32_t)lst[i0 + e];
            uint64_t h, l;
            set_key<K>(idx, n, x[e].p, h, l);
            x[e].h = h;
            if (K > 4) x[e].l = l;
        }
    }
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < E) {   // partner in this thread
                if (stride == 4) bitonic_in_thread<K, E, 4>(x, i0, size);
                else if (stride == 2) bitonic_in_thread<K, E, 2>(x, i0, size);
                else bitonic_in_thread<K, E, 1>(x, i0, size);
            } else if (stride < kWave * E) {   // partner in this wave
                const int mask = stride / E;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    SortKey y;
                    y.h = __shfl_xor(x[e].h, mask, kWave);
                    y.l = K > 4 ? __shfl_xor(x[e].l, mask, kWave) : 0ull;
                    y.p = __shfl_xor(x[e].p, mask, kWave);
                    const int i = i0 + e;
                    const bool take_min = ((i & stride) == 0) == ((i & size) == 0);
                    if (sk_less(y, x[e]) == take_min) x[e] = y;
                }
            } else {   // partner in another wave: through LDS
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    kh[i0 + e] = x[e].h;
                    if (K > 4) kl[i0 + e] = x[e].l;
                    kp[i0 + e] = x[e].p;
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = i0 + e, o = i ^ stride;
                    SortKey y;
                    y.h = kh[o];
                    y.l = K > 4 ? kl[o] : 0ull;
                    y.p = kp[o];
                    const bool take_min = ((i & stride) == 0) == ((i & size) == 0);
                    if (sk_less(y, x[e]) == take_min) x[e] = y;
                }
                __syncthreads();
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (i0 + e < c) lst[i0 + e] = (int32_t)x[e].p;
}

template <int K>
__global__ void __launch_bounds__(kSortThreads) list_sort_kernel(const int32_t *__restrict__ idx, int64_t n,
                                                        const int32_t *__restrict__ ptr,
                                                        int32_t *__restrict__ list, int32_t *__restrict__ tmp) {
    __shared__ uint64_t kh[MISSLAM_MAX_LIST];
    __shared__ uint64_t kl[K > 4 ? MISSLAM_MAX_LIST : 1];
    __shared__ uint32_t kp[MISSLAM_MAX_LIST];
    const int j = blockIdx.x;
    const int b = ptr[j];
    const int call = ptr[j + 1] - b;
    for (int c0 = 0; c0 < call; c0 += MISSLAM_MAX_LIST) {   // one piece unless the list is long
        const int c = min(call - c0, MISSLAM_MAX_LIST);
        int32_t *lst = list + b + c0;
        if (c <= kSortThreads) sort_piece<K, 1>(idx, n, lst, c, kh, kl, kp);
        else if (c <= 2 * kSortThreads) sort_piece<K, 2>(idx, n, lst, c, kh, kl, kp);
        else if (c <= 4 * kSortThreads) sort_piece<K, 4>(idx, n, lst, c, kh, kl, kp);
        else sort_piece<K, 8>(idx, n, lst, c, kh, kl, kp);
        __syncthreads();
    }
    if (call <= MISSLAM_MAX_LIST) return;
    // pairwise merges of the sorted pieces, list -> tmp -> list ...
    int32_t *src = list + b, *dst = tmp + b;
    for (int run = MISSLAM_MAX_LIST; run < call; run *= 2) {
        for (int s0 = 0; s0 < call; s0 += 2 * run) {
            const int la = min(run, call - s0);
            const int lb = min(run, call - s0 - la);
            merge_runs<K>(idx, n, src + s0, la, lb, dst + s0);
        }
        __threadfence_block();
        __syncthreads();
        int32_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != list + b) {
        for (int t = threadIdx.x; t < call; t += kSortThreads) list[b + t] = src[t];
    }
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
    const int c = lptr[j + 1] - b;
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

hipError_t launch_normal_map_batched(const BatchItem *items, int count, int total_blocks, hipStream_t st) {
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(normal_map_batched_kernel, dim3(total_blocks), dim3(256), 0, st, items, count);
    return hipGetLastError();
}

template <int K>
static hipError_t graph_k(const PointsView &pts, const NodesView &nd, int wkind, float sigma, const GraphView &g,
                          const GraphScratch &s, hipStream_t st) {
    const int64_t n = pts.n;
    const int m = nd.m;
    int32_t *lcnt = s.cnt + m;
    if (n > 0) {   // the node grid's kernel also clears the counters and the graph's flags
        hipLaunchKernelGGL(node_grid_kernel, dim3(1), dim3(kGridThreads), 0, st, nd, s.grid, (uint32_t *)s.cnt,
                           (size_t)(2 * m + 8), (uint32_t *)g.info, (size_t)8);
        hipLaunchKernelGGL((knn_kernel<K>), dim3(nblk(n, kKnnBlock)), dim3(kKnnBlock), 0, st, pts, s.grid, wkind,
                           sigma, g.knn_idx, g.knn_w, lcnt);
    } else {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(nblk(2 * (int64_t)m + 8, 256)), dim3(256), 0, st, (uint32_t *)s.cnt,
                           (size_t)(2 * m + 8), 0u);
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)g.info, (size_t)8, 0u);
    }
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, lcnt, m, g.list_ptr, g.info, -1, 2,
                       0x7FFFFFFF, (int64_t)K * n);
    if (n > 0) {
        hipLaunchKernelGGL((list_fill_kernel<K>), dim3(nblk(n, 256)), dim3(256), 0, st, g.knn_idx, n, g.list_ptr,
                           s.cnt, g.list_pts);
        hipLaunchKernelGGL((list_sort_kernel<K>), dim3(m), dim3(kSortThreads), 0, st, g.knn_idx, n, g.list_ptr,
                           g.list_pts, s.ltmp);
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
