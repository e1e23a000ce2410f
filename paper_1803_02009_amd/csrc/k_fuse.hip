// Model update after registration (Sec. II-G): deform the model with the
// frame's final node parameters, build the point-to-pixel registration map
// (Alg. 2 step 2), test each winner against the depth (Alg. 1) and fuse the
// observation into it (Eqs.(12), (14), (15)).
#include "frame.h"

namespace msl {

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Projection of a camera-frame point to its nearest pixel with the float64
// rules of the association; -1 when behind the camera or outside the image.
__device__ __forceinline__ int project_pixel(float vx, float vy, float vz, const Cam &cam) {
    const double x = vx, y = vy, z = vz;
    if (!(z > 0.0)) return -1;
    const double uf = (x / z) * (double)cam.fx + (double)cam.cx;
    const double vf = (y / z) * (double)cam.fy + (double)cam.cy;
    const double uu = floor(uf + 0.5), vv = floor(vf + 0.5);
    if (!(uu >= 0.0 && uu < (double)cam.W && vv >= 0.0 && vv < (double)cam.H)) return -1;
    return (int)vv * cam.W + (int)uu;
}

// One thread per point: world-frame warp of point and normal (kept in tmp),
// camera projection, and a 64-bit z-buffer entry per pixel: (float32 depth
// bits, point index) min-combined, so the nearest point wins and equal depths
// go to the lower index (depths are positive: their bit patterns order as the values).
template <int K>
__global__ void __launch_bounds__(256) fuse_project_kernel(FuseArgs f) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = f.pts.n;
    if (i >= n) return;
    float x, y, z, a, b, c;
    ed_blend<K>(f.pts.px[i], f.pts.py[i], f.pts.pz[i], f.g.knn_idx, f.g.knn_w, n, i, f.nd, x, y, z);
    ed_blend_normal<K>(f.pts.nx[i], f.pts.ny[i], f.pts.nz[i], f.g.knn_idx, f.g.knn_w, n, i, f.nd, a, b, c);
    f.tmp[i] = x;
    f.tmp[n + i] = y;
    f.tmp[2 * n + i] = z;
    f.tmp[3 * n + i] = a;   // unnormalised; both frames normalise their own copy
    f.tmp[4 * n + i] = b;
    f.tmp[5 * n + i] = c;
    apply_pose(f.pose, x, y, z);
    const int pix = project_pixel(x, y, z, f.cam);
    f.pix[i] = pix;
    if (pix >= 0) {
        const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(uint32_t)i;
        atomicMin(&f.zbuf[pix], key);
    }
}

// One thread per point: registration test of Alg. 1 for the pixel's winner
// (depth present, |z~ - D| < tau, n~ . N > cos(delta), float64) and the fusion
// update p <- (w p~ + Gamma_w) / (w + 1), n likewise (renormalised),
// w <- min(w + 1, w_max), stamp <- frame; every other point takes its
// deformed position and normal.
__global__ void __launch_bounds__(256) fuse_update_kernel(FuseArgs f) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = f.pts.n;
    if (i >= n) return;
    float vx = f.tmp[i], vy = f.tmp[n + i], vz = f.tmp[2 * n + i];
    float ax = f.tmp[3 * n + i], ay = f.tmp[4 * n + i], az = f.tmp[5 * n + i];
    float cx = vx, cy = vy, cz = vz;
    apply_pose(f.pose, cx, cy, cz);
    float ncx = ax, ncy = ay, ncz = az;
    rotate(f.pose, ncx, ncy, ncz);
    normalize3(ncx, ncy, ncz);
    normalize3(ax, ay, az);                                  // world normal
    const int pix = f.pix[i];
    bool reg = false;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (pix >= 0 && (uint32_t)(f.zbuf[pix] & 0xFFFFFFFFull) == (uint32_t)i) {
        q = f.nmap[pix];
        const double d = q.w;
        const bool nvalid = !(q.x == 0.f && q.y == 0.f && q.z == 0.f);
        const double nd = ((double)ncx * (double)q.x + (double)ncy * (double)q.y) + (double)ncz * (double)q.z;
        reg = d > 0.0 && nvalid && fabs((double)cz - d) < f.tau && nd > f.cos_delta;
    }
    float w = f.w_in[i];
    int st = f.stamp_in[i];
    if (reg && f.color) {   // Eq.(13): the same weighted mean of the colour, with the weight before Eq.(15)
        const double om = w, den = om + 1.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float *cc = f.color + (size_t)c * f.color_stride + i;
            *cc = (float)((om * (double)*cc + (double)f.image[(size_t)pix * 3 + c]) / den);
        }
    }
    if (reg) {
        const int u = pix % f.cam.W, v = pix / f.cam.W;
        const double d = q.w;
        const double V[3] = {d * (((double)u - (double)f.cam.cx) / (double)f.cam.fx),
                             d * (((double)v - (double)f.cam.cy) / (double)f.cam.fy), d};
        const double *R = f.Rd;
        double G[3], Nw[3];
        const double dv[3] = {V[0] - f.Td[0], V[1] - f.Td[1], V[2] - f.Td[2]};
        const double Nc[3] = {q.x, q.y, q.z};
        for (int a = 0; a < 3; ++a) {   // R^T (V - T), R^T N
            G[a] = (R[a] * dv[0] + R[3 + a] * dv[1]) + R[6 + a] * dv[2];
            Nw[a] = (R[a] * Nc[0] + R[3 + a] * Nc[1]) + R[6 + a] * Nc[2];
        }
        const double om = w, den = om + 1.0;
        vx = (float)((om * vx + G[0]) / den);
        vy = (float)((om * vy + G[1]) / den);
        vz = (float)((om * vz + G[2]) / den);
        const double mx = (om * ax + Nw[0]) / den, my = (om * ay + Nw[1]) / den, mz = (om * az + Nw[2]) / den;
        const double mn = sqrt((mx * mx + my * my) + mz * mz);
        ax = (float)(mx / mn);
        ay = (float)(my / mn);
        az = (float)(mz / mn);
        w = fminf(w + 1.0f, f.w_max);
        st = f.frame;
    }
    f.out_px[i] = vx;
    f.out_py[i] = vy;
    f.out_pz[i] = vz;
    f.out_nx[i] = ax;
    f.out_ny[i] = ay;
    f.out_nz[i] = az;
    f.out_w[i] = w;
    f.out_stamp[i] = st;
    if (f.registered) f.registered[i] = reg ? 1 : 0;
}

__global__ void reg_map_kernel(const unsigned long long *__restrict__ zbuf, int64_t npx, int32_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= npx) return;
    const unsigned long long k = zbuf[t];
    out[t] = k == ~0ull ? -1 : (int32_t)(uint32_t)(k & 0xFFFFFFFFull);
}

// Nodes follow the deformation (g_j <- g_j + t_j) and the parameters restart at A = I, t = 0.
__global__ void fuse_nodes_kernel(float *gx, float *gy, float *gz, float *x, int m) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    float *p = x + (size_t)j * 12;
    gx[j] += p[9];
    gy[j] += p[10];
    gz[j] += p[11];
#pragma unroll
    for (int t = 0; t < 12; ++t) p[t] = (t == 0 || t == 4 || t == 8) ? 1.f : 0.f;
}

hipError_t launch_fuse(const FuseArgs &f, float *gx, float *gy, float *gz, float *params, int m, int32_t *reg_map,
                       hipStream_t st) {
    const int64_t n = f.pts.n;
    const int64_t npx = (int64_t)f.cam.W * f.cam.H;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(nblk(npx, 256)), dim3(256), 0, st, f.zbuf, npx, ~0ull);
    if (n > 0) {
        switch (f.g.k) {
#define MSL_FU_CASE(KK) \
    case KK: hipLaunchKernelGGL((fuse_project_kernel<KK>), dim3(nblk(n, 256)), dim3(256), 0, st, f); break;
            MSL_FU_CASE(1) MSL_FU_CASE(2) MSL_FU_CASE(3) MSL_FU_CASE(4)
            MSL_FU_CASE(5) MSL_FU_CASE(6) MSL_FU_CASE(7) MSL_FU_CASE(8)
#undef MSL_FU_CASE
            default: return hipErrorInvalidValue;
        }
        hipLaunchKernelGGL(fuse_update_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, f);
    }
    if (reg_map) hipLaunchKernelGGL(reg_map_kernel, dim3(nblk(npx, 256)), dim3(256), 0, st, f.zbuf, npx, reg_map);
    hipLaunchKernelGGL(fuse_nodes_kernel, dim3(nblk(m, 256)), dim3(256), 0, st, gx, gy, gz, params, m);
    return hipGetLastError();
}

}  // namespace msl
