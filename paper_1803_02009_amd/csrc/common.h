// Internal device helpers shared by the gfx950 kernels of libmisslam.
//
// Built with -ffp-contract=off: every float64 decision below (projection,
// rounding, gates, nearest-node ordering) keeps the written operation order,
// and float32 arithmetic that should fuse says so with fmaf().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "misslam.h"

namespace msl {

constexpr int kWave = 64;

struct Cam {
    int W, H;
    float fx, fy, cx, cy;
};

struct Pose {
    float R[9];
    float T[3];
};

struct PointsView {
    const float *px, *py, *pz, *nx, *ny, *nz;
    int64_t n;
};

struct NodesView {
    const float *gx, *gy, *gz, *x;   // x: m x 12
    int m;
};

// ---------------------------------------------------------------- Eq.(1): ED warp of one point

// Blends the k node transforms of a point in kNN order (float32):
//   y = sum_s w_s [A_s (v - g_s) + g_s + t_s]
template <int K>
__device__ __forceinline__ void ed_blend(float vx, float vy, float vz, const int32_t *idx, const float *w,
                                         int64_t n, int64_t i, const NodesView &nd, float &ox, float &oy,
                                         float &oz) {
    ox = 0.f;
    oy = 0.f;
    oz = 0.f;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = idx[(int64_t)s * n + i];
        const float ws = w[(int64_t)s * n + i];
        const float gx = nd.gx[j], gy = nd.gy[j], gz = nd.gz[j];
        const float *x = nd.x + (size_t)j * 12;
        const float dx = vx - gx, dy = vy - gy, dz = vz - gz;
        // A d with A[:, c] = x[3c .. 3c+2]
        float ax = fmaf(x[6], dz, fmaf(x[3], dy, x[0] * dx));
        float ay = fmaf(x[7], dz, fmaf(x[4], dy, x[1] * dx));
        float az = fmaf(x[8], dz, fmaf(x[5], dy, x[2] * dx));
        ax = ax + gx + x[9];
        ay = ay + gy + x[10];
        az = az + gz + x[11];
        ox = fmaf(ws, ax, ox);
        oy = fmaf(ws, ay, oy);
        oz = fmaf(ws, az, oz);
    }
}

// Warped normal direction (unnormalised): sum_s w_s A_s^{-T} n, A^{-T} = cof(A) / det(A).
template <int K>
__device__ __forceinline__ void ed_blend_normal(float nx, float ny, float nz, const int32_t *idx, const float *w,
                                                int64_t n, int64_t i, const NodesView &nd, float &ox, float &oy,
                                                float &oz) {
    ox = 0.f;
    oy = 0.f;
    oz = 0.f;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int j = idx[(int64_t)s * n + i];
        const float ws = w[(int64_t)s * n + i];
        const float *x = nd.x + (size_t)j * 12;
        // A[a][c] = x[3c + a]
        const float a00 = x[0], a10 = x[1], a20 = x[2];
        const float a01 = x[3], a11 = x[4], a21 = x[5];
        const float a02 = x[6], a12 = x[7], a22 = x[8];
        // cofactor matrix C[a][c]; A^{-T} = C / det
        const float c00 = a11 * a22 - a12 * a21, c01 = a12 * a20 - a10 * a22, c02 = a10 * a21 - a11 * a20;
        const float c10 = a02 * a21 - a01 * a22, c11 = a00 * a22 - a02 * a20, c12 = a01 * a20 - a00 * a21;
        const float c20 = a01 * a12 - a02 * a11, c21 = a02 * a10 - a00 * a12, c22 = a00 * a11 - a01 * a10;
        const float det = a00 * c00 + a01 * c01 + a02 * c02;
        const float sc = ws / det;
        ox = fmaf(sc, c00 * nx + c01 * ny + c02 * nz, ox);
        oy = fmaf(sc, c10 * nx + c11 * ny + c12 * nz, oy);
        oz = fmaf(sc, c20 * nx + c21 * ny + c22 * nz, oz);
    }
}

// c . c - 1 for column a of A (c = (x[3a], x[3a+1], x[3a+2]), diagonal entry
// c[a]) without the cancellation of forming c . c near 1: (c[a] - 1) is exact
// for c[a] in [0.5, 2] and (c[a] - 1)(c[a] + 1) + the other squares keeps the
// residual's own relative precision (Eq.(5), its norm terms).
__device__ __forceinline__ float unit_residual(const float *c, int a) {
    const float d = c[a] - 1.f;
    const float o1 = c[(a + 1) % 3], o2 = c[(a + 2) % 3];
    return fmaf(d, c[a] + 1.f, fmaf(o2, o2, o1 * o1));
}

// Eq.(6) residual of the edge j -> l, A_j (g_l - g_j) + g_j + t_j - (g_l + t_l),
// evaluated as (A_j - I) e + (t_j - t_l) with e = g_l - g_j: the node
// positions cancel exactly instead of in float32 sums of millimetre-scale
// coordinates, so the residual keeps its own relative precision.
__device__ __forceinline__ void reg_residual(const float *xj, const float *xl, float ex, float ey, float ez, float &r0,
                                             float &r1, float &r2) {
    const float d0 = xj[0] - 1.f, d4 = xj[4] - 1.f, d8 = xj[8] - 1.f;   // diagonal of A_j - I, exact
    r0 = fmaf(xj[6], ez, fmaf(xj[3], ey, d0 * ex)) + (xj[9] - xl[9]);
    r1 = fmaf(xj[7], ez, fmaf(d4, ey, xj[1] * ex)) + (xj[10] - xl[10]);
    r2 = fmaf(d8, ez, fmaf(xj[5], ey, xj[2] * ex)) + (xj[11] - xl[11]);
}

__device__ __forceinline__ void apply_pose(const Pose &P, float &x, float &y, float &z) {
    const float X = x, Y = y, Z = z;
    x = fmaf(P.R[2], Z, fmaf(P.R[1], Y, P.R[0] * X)) + P.T[0];
    y = fmaf(P.R[5], Z, fmaf(P.R[4], Y, P.R[3] * X)) + P.T[1];
    z = fmaf(P.R[8], Z, fmaf(P.R[7], Y, P.R[6] * X)) + P.T[2];
}

__device__ __forceinline__ void rotate(const Pose &P, float &x, float &y, float &z) {
    const float X = x, Y = y, Z = z;
    x = fmaf(P.R[2], Z, fmaf(P.R[1], Y, P.R[0] * X));
    y = fmaf(P.R[5], Z, fmaf(P.R[4], Y, P.R[3] * X));
    z = fmaf(P.R[8], Z, fmaf(P.R[7], Y, P.R[6] * X));
}

__device__ __forceinline__ void normalize3(float &x, float &y, float &z) {
    const float s = sqrtf(x * x + y * y + z * z);
    const float inv = s > 0.f ? 1.0f / s : 0.f;
    x *= inv;
    y *= inv;
    z *= inv;
}

// ---------------------------------------------------------------- Eqs.(7)-(8): association

struct Match {
    int pix;        // v*W + u, or -1
    float r;        // point-to-plane residual N . (v~ - V)
    float Nx, Ny, Nz;
};

// Projects a warped camera-frame point to its nearest pixel and applies the
// visibility gates; every decision is float64 in a fixed order.
//   u_f = (x / z) fx + cx, u = floor(u_f + 0.5); likewise v
//   valid: z > 0, pixel inside, D > 0, normal present,
//          |v~ - V| < eps_d and n~ . N > cos_eps_n (both strict)
// nmap holds (Nx, Ny, Nz, D) per pixel.
__device__ __forceinline__ Match associate(float vx, float vy, float vz, float nx, float ny, float nz,
                                           const float4 *__restrict__ nmap, const Cam &cam, double eps_d,
                                           double cos_eps_n) {
    Match out{-1, 0.f, 0.f, 0.f, 0.f};
    const double x = vx, y = vy, z = vz;
    if (!(z > 0.0)) return out;
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    const double uf = (x / z) * fx + cx;
    const double vf = (y / z) * fy + cy;
    const double uu = floor(uf + 0.5);
    const double vv = floor(vf + 0.5);
    if (!(uu >= 0.0 && uu < (double)cam.W && vv >= 0.0 && vv < (double)cam.H)) return out;
    const int u = (int)uu, v = (int)vv;
    const float4 q = nmap[(size_t)v * cam.W + u];
    const double d = q.w;
    if (!(d > 0.0)) return out;
    if (q.x == 0.f && q.y == 0.f && q.z == 0.f) return out;
    const double Vx = d * (((double)u - cx) / fx);
    const double Vy = d * (((double)v - cy) / fy);
    const double Vz = d;
    const double dx = x - Vx, dy = y - Vy, dz = z - Vz;
    const double dist = sqrt((dx * dx + dy * dy) + dz * dz);
    const double Nx = q.x, Ny = q.y, Nz = q.z;
    const double nd = ((double)nx * Nx + (double)ny * Ny) + (double)nz * Nz;
    if (!(dist < eps_d && nd > cos_eps_n)) return out;
    out.pix = v * cam.W + u;
    out.r = (float)((Nx * dx + Ny * dy) + Nz * dz);
    out.Nx = q.x;
    out.Ny = q.y;
    out.Nz = q.z;
    return out;
}

// Residual against a given pixel (frozen correspondence): no gates are applied.
__device__ __forceinline__ Match match_fixed(float vx, float vy, float vz, int pix, const float4 *__restrict__ nmap,
                                             const Cam &cam) {
    Match out{-1, 0.f, 0.f, 0.f, 0.f};
    if (pix < 0 || pix >= cam.W * cam.H) return out;
    const float4 q = nmap[pix];
    const double d = q.w;
    if (!(d > 0.0) || (q.x == 0.f && q.y == 0.f && q.z == 0.f)) return out;
    const int u = pix % cam.W, v = pix / cam.W;
    const double Vx = d * (((double)u - (double)cam.cx) / (double)cam.fx);
    const double Vy = d * (((double)v - (double)cam.cy) / (double)cam.fy);
    const double dx = (double)vx - Vx, dy = (double)vy - Vy, dz = (double)vz - d;
    out.pix = pix;
    out.r = (float)(((double)q.x * dx + (double)q.y * dy) + (double)q.z * dz);
    out.Nx = q.x;
    out.Ny = q.y;
    out.Nz = q.z;
    return out;
}

// ---------------------------------------------------------------- deterministic block reductions

// Sum of one double per thread over a block of BS threads, fixed tree order.
// Every thread returns the total.  lds must hold BS doubles.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = BS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double t = lds[0];
    __syncthreads();
    return t;
}

// The same tree for N values at once (one barrier per level for all of them): each total keeps the bits of
// block_sum.  lds: N * BS doubles.
template <int BS, int N>
__device__ __forceinline__ void block_sums_tree(double (&v)[N], double *lds) {
#pragma unroll
    for (int q = 0; q < N; ++q) lds[q * BS + threadIdx.x] = v[q];
    __syncthreads();
#pragma unroll
    for (int s = BS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < N; ++q) lds[q * BS + threadIdx.x] += lds[q * BS + threadIdx.x + s];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = lds[q * BS];
    __syncthreads();
}

// ---------------------------------------------------------------- damped block inverse (block-Jacobi)

// Orders the LDS traffic of one wave (its lanes' writes before other lanes'
// reads); LDS operations of a wave complete in issue order.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// M = A^-1 for one SPD 12x12 block held in LDS as float64, by one wave (all
// 64 lanes call it).  A is overwritten by its Cholesky factor L (lower
// triangle); M = L^-T L^-1 goes to out (row-major 144 float32).  Returns false
// on every lane when a pivot is not positive, and M is then I.
__device__ __forceinline__ bool chol_inverse_wave(double (*A)[12], double (*Li)[12], float *out) {
    const int lane = threadIdx.x % 64;
    bool bad = false;
    for (int k = 0; k < 12; ++k) {
        const double d = A[k][k];
        bad = bad || !(d > 0.0);
        const double lkk = d > 0.0 ? sqrt(d) : 1.0;
        wave_sync();
        if (lane == 0) A[k][k] = lkk;
        if (lane > k && lane < 12) A[lane][k] = A[lane][k] / lkk;
        wave_sync();
        for (int t = lane; t < 144; t += 64) {
            const int i = t / 12, c = t % 12;
            if (c > k && c <= i) A[i][c] = A[i][c] - A[i][k] * A[c][k];
        }
        wave_sync();
    }
    if (lane < 12) {
        const int c = lane;
        for (int i = 0; i < 12; ++i) {
            if (i < c) {
                Li[i][c] = 0.0;
                continue;
            }
            double s = i == c ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= A[i][t] * Li[t][c];
            Li[i][c] = s / A[i][i];
        }
    }
    wave_sync();
    for (int t = lane; t < 144; t += 64) {
        const int i = t / 12, k = t % 12;
        double s = 0.0;
        for (int q = i > k ? i : k; q < 12; ++q) s += Li[q][i] * Li[q][k];
        out[t] = bad ? (i == k ? 1.f : 0.f) : (float)s;
    }
    return !bad;
}

// out = A^-1 (float32) for one SPD 12x12 block held in LDS as float64, by a
// whole workgroup of NT threads: Gauss-Jordan elimination on the diagonal
// pivots, each step reading row k and column k, then every thread rewriting
// its own entries.  Without pivoting the k-th pivot is the Schur complement
// d_k = det(A_1..k) / det(A_1..k-1), positive for every k exactly when A is
// SPD; a non-positive pivot marks the block non-SPD and the identity is
// written instead.  A is overwritten.  Every thread must call this.
template <int NT>
__device__ __forceinline__ bool gj_inverse_block(double (*A)[12], float *out) {
    constexpr int E = (144 + NT - 1) / NT;   // entries per thread
    const int tid = threadIdx.x;
    bool bad = false;
    for (int k = 0; k < 12; ++k) {
        const double p = A[k][k];
        double ark[E], akc[E], own[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = tid + e * NT;
            if (t < 144) {
                ark[e] = A[t / 12][k];
                akc[e] = A[k][t % 12];
                own[e] = A[t / 12][t % 12];
            }
        }
        __syncthreads();
        bad = bad || !(p > 0.0);
        const double ip = p > 0.0 ? 1.0 / p : 1.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = tid + e * NT;
            if (t < 144) {
                const int R = t / 12, C = t % 12;
                double v;
                if (R == k && C == k) v = ip;
                else if (R == k) v = akc[e] * ip;
                else if (C == k) v = -ark[e] * ip;
                else v = own[e] - ark[e] * (akc[e] * ip);
                A[R][C] = v;
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < 144; t += NT) out[t] = bad ? (t / 12 == t % 12 ? 1.f : 0.f) : (float)A[t / 12][t % 12];
    return !bad;
}

// Cross-lane partners for the wave butterfly without LDS traffic, on 32-bit words.  stage_pair<k32> returns
// the word and its partner lane's (xor 32, or xor 16) in an order that depends on the lane, by the gfx950 lane
// swaps (v_permlane32_swap / v_permlane16_swap with the word as both operands): their sum is the stage's sum.
// dpp_word<kCtrl> reads the word of another lane of the same 16-lane row: row_ror:8 / row_ror:4 give the xor-8 /
// xor-4 partner's value once the values repeat every 16 / 8 lanes (true after the larger stages), quad_perm
// [2,3,0,1] / [1,0,3,2] give the xor-2 / xor-1 partner exactly.
template <bool k32>
__device__ __forceinline__ void stage_pair(unsigned w, unsigned &a, unsigned &b) {
    if constexpr (k32) {
        const auto r = __builtin_amdgcn_permlane32_swap(w, w, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
        a = r[0];
        b = r[1];
    }
}
template <int kCtrl>
__device__ __forceinline__ unsigned dpp_word(unsigned w) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)w, kCtrl, 0xF, 0xF, false);
}
__device__ __forceinline__ float stage_sum32(float v, bool k32) {
    unsigned a, b;
    if (k32) stage_pair<true>(__float_as_uint(v), a, b);
    else stage_pair<false>(__float_as_uint(v), a, b);
    return __uint_as_float(a) + __uint_as_float(b);
}
__device__ __forceinline__ double stage_sum32(double v, bool k32) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(v);
    unsigned al, bl, ah, bh;
    if (k32) {
        stage_pair<true>((unsigned)x, al, bl);
        stage_pair<true>((unsigned)(x >> 32), ah, bh);
    } else {
        stage_pair<false>((unsigned)x, al, bl);
        stage_pair<false>((unsigned)(x >> 32), ah, bh);
    }
    return __longlong_as_double((long long)(((unsigned long long)ah << 32) | al)) +
           __longlong_as_double((long long)(((unsigned long long)bh << 32) | bl));
}
template <int kCtrl>
__device__ __forceinline__ float partner(float v) {
    return __uint_as_float(dpp_word<kCtrl>(__float_as_uint(v)));
}
template <int kCtrl>
__device__ __forceinline__ double partner(double v) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = dpp_word<kCtrl>((unsigned)x), hi = dpp_word<kCtrl>((unsigned)(x >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Butterfly sums of N values over the wave (xor partners 32, 16, ..., 1): every lane gets the totals, each
// value by the same additions as the textbook butterfly t += shfl_xor(t, off) (each stage adds a lane's value
// and its partner's; addition commutes).  Stage by stage over all N values, so their cross-lane moves overlap.
template <int N, typename T>
__device__ __forceinline__ void wave_sums(T (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = stage_sum32(v[q], true);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = stage_sum32(v[q], false);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += partner<0x128>(v[q]);   // row_ror:8
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += partner<0x124>(v[q]);   // row_ror:4
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += partner<0x4E>(v[q]);    // quad_perm [2,3,0,1]
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += partner<0xB1>(v[q]);    // quad_perm [1,0,3,2]
}

// A Gauss-Newton step's report, by one workgroup of 256 threads: the energies (the point pass's data partials,
// the assembly's node partials, the key points' energies) summed in a fixed order, n_valid, and the
// NONFINITE / FRAME_REJECT flags ORed into rep->flags; zero_words (zero_count words, if set) are cleared first.
__device__ __forceinline__ void energy_report_body(const double *__restrict__ pt_part, int npb,
                                                   const double *__restrict__ node_part, int m, misslam_report *rep,
                                                   float reject_thr, unsigned *__restrict__ zero_words,
                                                   int zero_count, const double *__restrict__ kp_energy = nullptr,
                                                   int kp_count = 0) {
    __shared__ double red[6][256 / kWave];
    if (zero_words)   // the next solve's sync area
        for (int t = threadIdx.x; t < zero_count / 4; t += 256)
            reinterpret_cast<uint4 *>(zero_words)[t] = make_uint4(0u, 0u, 0u, 0u);
    // thread t adds entries t, t + 256, ... in order; the loads of eight entries are issued before their adds
    constexpr int U = 8;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t0 = threadIdx.x; t0 < npb; t0 += U * 256) {
        double a[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + 256 * u, npb - 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) a[u][c] = pt_part[3 * t + c];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + 256 * u < npb) {
                v[0] += a[u][0];
                v[1] += a[u][1];
                v[2] += a[u][2];
            }
    }
    for (int t0 = threadIdx.x; t0 < m; t0 += U * 256) {
        double a[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + 256 * u, m - 1);
            a[u][0] = node_part[2 * t];
            a[u][1] = node_part[2 * t + 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + 256 * u < m) {
                v[3] += a[u][0];
                v[4] += a[u][1];
            }
    }
    for (int t0 = threadIdx.x; t0 < kp_count; t0 += U * 256) {
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = kp_energy[min(t0 + 256 * u, kp_count - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + 256 * u < kp_count) v[5] += a[u];
    }
    // wave butterflies, then the four waves in order: a fixed summation order
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    wave_sums(v);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) red[q][wave] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[6];
        for (int q = 0; q < 6; ++q) tot[q] = ((red[q][0] + red[q][1]) + red[q][2]) + red[q][3];
        const double ed = tot[0], nv = tot[1], sa = tot[2], er = tot[3], eg = tot[4];
        rep->e_data = ed;
        rep->e_rot = er;
        rep->e_reg = eg;
        rep->n_valid = (int32_t)nv;
        rep->e_corr = tot[5];
        int flags = 0;
        if (!isfinite(ed) || !isfinite(er) || !isfinite(eg) || !isfinite(tot[5])) flags |= MISSLAM_FLAG_NONFINITE;
        if (reject_thr > 0.f && nv > 0 && sa / nv > (double)reject_thr) flags |= MISSLAM_FLAG_FRAME_REJECT;
        rep->flags |= flags;
    }
}

// The value of v on lane l (l uniform), for float64.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same inverse as gj_inverse_block (the same operations in the same order, so the same bits), by one
// wave without LDS traffic or barriers: lane c < 12 holds column c of A in registers, and each elimination
// step reads the pivot column from lane k.  A (row-major float64 in LDS) is only read.  Returns false on
// every lane when a pivot is not positive, and out is then I.
__device__ __forceinline__ bool gj_inverse_lanes(const double (*A)[12], float *out) {
    const int lane = threadIdx.x % 64;
    const int c = lane < 12 ? lane : 0;
    double col[12];
#pragma unroll
    for (int R = 0; R < 12; ++R) col[R] = A[R][c];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        double ark[12];
#pragma unroll
        for (int R = 0; R < 12; ++R) ark[R] = readlane_f64(col[R], k);   // A[R][k]
        const double p = ark[k];
        bad = bad || !(p > 0.0);
        const double ip = p > 0.0 ? 1.0 / p : 1.0;
        const double akc = col[k];   // A[k][c]
        const bool ck = c == k;
#pragma unroll
        for (int R = 0; R < 12; ++R) {
            if (R == k) col[R] = ck ? ip : akc * ip;
            else col[R] = ck ? -ark[R] * ip : col[R] - ark[R] * (akc * ip);
        }
    }
    if (lane < 12) {
#pragma unroll
        for (int R = 0; R < 12; ++R) out[R * 12 + c] = bad ? (R == c ? 1.f : 0.f) : (float)col[R];
    }
    return !bad;
}

}  // namespace msl
