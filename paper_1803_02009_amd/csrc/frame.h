// Internal declarations shared by the host layer and the kernel files of libmisslam.
#pragma once

#include "common.h"

namespace msl {

struct GraphView {
    int k, bsr_cap;
    int32_t *knn_idx;
    float *knn_w;
    int32_t *row_ptr, *col_idx, *list_ptr, *list_pts;
    uint32_t *list_key;   // 2 words per list entry
    int32_t *info;
};

struct GraphScratch {
    int32_t *tmp;     // m x MISSLAM_MAX_ROW row columns
    int32_t *cnt;     // 2m + 8
};

// Per-iteration scratch of the registration step.
struct StepScratch {
    float4 *nr;           // n: (R^T N of the matched pixel, point-to-plane residual); 0 when unmatched
    int32_t *corr;        // n
    double *pt_part;      // 3 per point block: sum r^2, count, sum |r|
    double *node_part;    // 2 per node: rot and reg energy of the node's terms
    float *minv;          // m x 144 block-Jacobi inverses
    int32_t *flags;       // 4 ints of device flags
};

struct PcgScratch {
    float *r, *z, *p, *q;  // 12m each
    double *part;          // (pcg_iters + 1) x 4 x nblk partial sums
    int32_t *status;       // 2 x (pcg_iters + 2): stop status, then per-iteration "updated" flags
    int nblk;              // workgroups of the multi-kernel path
    int nblk_max;          // partial slots per reduction (>= every path's workgroup count)
};

hipError_t launch_normal_map(const float *depth, const Cam &cam, float4 *out, hipStream_t st);
hipError_t launch_build_graph(const PointsView &pts, const NodesView &nd, int k, int wkind, float sigma,
                              const GraphView &g, const GraphScratch &s, hipStream_t st);
hipError_t launch_warp(const PointsView &pts, const NodesView &nd, const GraphView &g, const Pose *pose,
                       float *out_pos, float *out_nrm, hipStream_t st);

struct StepArgs {
    PointsView pts;
    NodesView nd;
    GraphView g;
    const float4 *nmap;
    Cam cam;
    Pose pose;
    double eps_d, cos_eps_n;
    float w_rot, w_reg, w_data, lambda;
    float *blocks;     // nnzb x 144
    float *gvec;       // 12 m
    int32_t *corr_out; // optional copy of correspondences
    const int32_t *corr_in;  // optional frozen correspondences (no association, no gates)
    float *minv;       // optional m x 144 block-Jacobi inverses computed with the assembly
    int32_t *flags;    // report flags (NONSPD_BLOCK) when minv is set
};

struct FuseArgs {
    PointsView pts;
    NodesView nd;
    GraphView g;
    const float4 *nmap;
    Cam cam;
    Pose pose;
    double Rd[9], Td[3];
    double tau, cos_delta;
    float w_max;
    int frame;
    const float *w_in;
    const int32_t *stamp_in;
    float *out_px, *out_py, *out_pz, *out_nx, *out_ny, *out_nz, *out_w;
    int32_t *out_stamp;
    int32_t *registered;           // optional, n
    float *tmp;                    // 6 x n: world warp and unnormalised warped normal
    int32_t *pix;                  // n
    unsigned long long *zbuf;      // H x W
};

hipError_t launch_fuse(const FuseArgs &f, float *gx, float *gy, float *gz, float *params, int m, int32_t *reg_map,
                       hipStream_t st);

hipError_t launch_point_pass(const StepArgs &a, const StepScratch &s, hipStream_t st);
hipError_t launch_assemble(const StepArgs &a, const StepScratch &s, hipStream_t st);
hipError_t launch_assemble_lp(const StepArgs &a, const StepScratch &s, int precision, float *rr_out,
                              hipStream_t st);
hipError_t launch_refine_rhs(const StepArgs &a, const StepScratch &s, const float *dx, const float *rr, const float *g,
                             float *jv, float *rhs, hipStream_t st);
hipError_t launch_axpy(float *y, const float *x, int count, hipStream_t st);
hipError_t launch_node_energy(const StepArgs &a, const StepScratch &s, hipStream_t st);
hipError_t launch_vjp_points(const StepArgs &a, const StepScratch &s, float sigma, const float *grad_e, float *out,
                             hipStream_t st);
hipError_t launch_grad_params(const float *g, int m, const float *grad_e, float *out, hipStream_t st);
hipError_t launch_energy_total(const misslam_report *rep, float w_data, float w_rot, float w_reg, double *out,
                               hipStream_t st);
hipError_t launch_energy_report(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                                hipStream_t st);
hipError_t launch_bjacobi(const GraphView &g, int m, const float *blocks, float lambda, float *minv,
                          int32_t *flags, hipStream_t st);
// PCG solve into delta; when params != nullptr also applies params += delta (the GN update).
hipError_t launch_pcg_update(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                             float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                             float *params, hipStream_t st);
hipError_t launch_report_init(misslam_report *rep, int count, hipStream_t st);
// Same solve as launch_pcg_update in one cooperative launch; *used = false when
// the device cannot co-schedule it (nothing launched, caller falls back).
hipError_t launch_pcg_persistent(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                                 float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                                 float *params, hipStream_t st, bool *used);
int pcg_blocks(int m);
hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st);

}  // namespace msl
