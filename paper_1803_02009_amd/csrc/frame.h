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

// Sync area of a persistent solve: 16 words (8 tagged 8-byte words) for each
// of at most MSL_TAG_WGS workgroups of one launch.  The words of the
// launch's workgroups must be zero when a solve starts.
constexpr int MSL_TAG_WGS = 1024;
constexpr int MSL_WG_WORDS = 16;
constexpr int MSL_BAR_WORDS = MSL_WG_WORDS * MSL_TAG_WGS;
constexpr int kJointTagWords = 16;   // 8-byte sync words per workgroup of the one-launch joint solve
constexpr int kJointMaxWgs = 2048;   // its workgroups at most (sync area: kJointTagWords * kJointMaxWgs words)
// 8-byte sync words the one-launch joint solve of m rows uses (at least MISSLAM_SOLVE_ROWS rows per workgroup).
inline int joint_sync_words(int m) {
    const int g = (m + MISSLAM_SOLVE_ROWS - 1) / MISSLAM_SOLVE_ROWS;
    return kJointTagWords * (g < 1 ? 1 : (g > kJointMaxWgs ? kJointMaxWgs : g));
}
// Sync words a persistent solve of m rows uses.
inline int msl_sync_words(int m) {
    const int g = (m + MISSLAM_SOLVE_ROWS - 1) / MISSLAM_SOLVE_ROWS;
    return g < 1 ? MSL_WG_WORDS : (g > MSL_TAG_WGS ? MSL_BAR_WORDS : MSL_WG_WORDS * g);
}

// Uniform grid of the nodes for the kNN search.
constexpr int MSL_GRID_CELLS = 1 << 18;
struct GridView {
    double *hdr;      // origin x, y, z, cell width
    int32_t *dims;    // cells per axis (0: no nodes)
    int32_t *start;   // MSL_GRID_CELLS + 1 cell offsets into nodes
    int32_t *cursor;  // MSL_GRID_CELLS fill cursors
    float4 *nodes;    // m: x, y, z, index bits, in cell order
};

struct GraphScratch {
    int32_t *tmp;     // m x MISSLAM_MAX_ROW row columns
    int32_t *ltmp;    // k n: merge buffer of the node lists longer than MISSLAM_MAX_LIST
    int32_t *cnt;     // 2m + 8
    GridView grid;
};

// Per-iteration scratch of the registration step.
struct StepScratch {
    float4 *nr;           // n: (R^T N of the matched pixel, point-to-plane residual); 0 when unmatched
    int32_t *corr;        // n
    double *pt_part;      // 3 per point block: sum r^2, count, sum |r|
    double *node_part;    // 2 per node: rot and reg energy of the node's terms
    float *minv;          // m x 144 block-Jacobi inverses
    int32_t *flags;       // 4 ints of device flags
    // per list entry of node j (point p), packed once per registration for the assembly:
    float4 *lpa;          // k n: (v_p - g_j, w_pj)
    float4 *lpw;          // k n x ceil(k/4): w_pj w_pq over the entry's nodes q in index order, zero-padded
    // joint pose form only:
    float4 *jp;           // 2 n: pose columns of the point's data row (v~ x N, N), 0 when unmatched
    double *pose_part;    // 27 per point block: upper triangle of sum Jp Jp^T (21), sum Jp r (6)
};

constexpr int kPosePart = 27;

// Key-point term scratch (at most n key points).
struct CorrScratch {
    int32_t *kp_nodes;    // k per key point: the carrying point's nodes (-1: skipped key point)
    float *kp_data;       // 3 + 4k per key point: R^T r, then per node w and v - g
    double *kp_energy;    // 1 per key point: |r|^2
};

struct PcgScratch {
    float *r, *z, *p, *q;  // 12m each
    double *part;          // (pcg_iters + 1) x 4 x nblk partial sums
    int32_t *status;       // 2 x (pcg_iters + 2): stop status, then per-iteration "updated" flags
    int nblk;              // workgroups of the multi-kernel path
    int nblk_max;          // partial slots per reduction (>= every path's workgroup count)
    unsigned *bar;         // MSL_BAR_WORDS words: sync area of the persistent solve
    double *halo;          // 2 x 12m: exchanged vectors of the pipelined one-launch solve
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
    const float *lambda_dev = nullptr;   // optional device damping, read in place of lambda
    const float *pose_dev = nullptr;     // optional device pose (R row-major, T), read in place of pose
    int asm_waves = 2;                   // assembly tile: waves per node row, 1 or 2
    unsigned *zero_words = nullptr;      // optional: words the assembly clears (the next solve's sync area)
    int zero_count = 0;                  // a multiple of 4
};

__device__ __forceinline__ Pose step_pose(const StepArgs &a) {
    if (!a.pose_dev) return a.pose;
    Pose P;
#pragma unroll
    for (int t = 0; t < 9; ++t) P.R[t] = a.pose_dev[t];
#pragma unroll
    for (int t = 0; t < 3; ++t) P.T[t] = a.pose_dev[9 + t];
    return P;
}

__device__ __forceinline__ float step_lambda(const StepArgs &a) { return a.lambda_dev ? *a.lambda_dev : a.lambda; }

// Key-point matches of the Eq.(9) correspondence term (device arrays).
struct KeyArgs {
    int count;
    float w_corr;
    const int32_t *point;    // carrying model point per key point (indices outside [0, n) are skipped)
    const float *target;     // 3 per key point, camera coordinates of the frame
};

template <int K>
constexpr int kp_stride() { return 9 + 4 * K; }   // per key point: R^T r, per node q: w_q, d_q (3); v~, r

// Eq.(9) at the current parameters for key point s: residual r = V~ - V (float32), R^T r, the k weights
// and d_q = v - g_q, the warped point V~ and r (camera coordinates) into kp_data, the energy |r|^2 (float64; 0
// for a skipped key point) into kp_energy.  The pose is the device pose when a.pose_dev is set.
template <int K>
__device__ __forceinline__ void kp_eval_body(const StepArgs &a, const KeyArgs &kp, float *kp_data,
                                             double *kp_energy, int s) {
    if (s >= kp.count) return;
    float *o = kp_data + (size_t)s * kp_stride<K>();
    const int64_t n = a.pts.n;
    const int p = kp.point[s];
    if (p < 0 || p >= n) {
        for (int t = 0; t < kp_stride<K>(); ++t) o[t] = 0.f;
        kp_energy[s] = 0.0;
        return;
    }
    const float vx = a.pts.px[p], vy = a.pts.py[p], vz = a.pts.pz[p];
    const Pose P = step_pose(a);
    float ox, oy, oz;
    ed_blend<K>(vx, vy, vz, a.g.knn_idx, a.g.knn_w, n, p, a.nd, ox, oy, oz);
    apply_pose(P, ox, oy, oz);
    const float rx = ox - kp.target[3 * (size_t)s], ry = oy - kp.target[3 * (size_t)s + 1],
                rz = oz - kp.target[3 * (size_t)s + 2];
    const float *R = P.R;
    o[0] = fmaf(R[6], rz, fmaf(R[3], ry, R[0] * rx));
    o[1] = fmaf(R[7], rz, fmaf(R[4], ry, R[1] * rx));
    o[2] = fmaf(R[8], rz, fmaf(R[5], ry, R[2] * rx));
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int l = a.g.knn_idx[(int64_t)q * n + p];
        o[3 + 4 * q] = a.g.knn_w[(int64_t)q * n + p];
        o[4 + 4 * q] = vx - a.nd.gx[l];
        o[5 + 4 * q] = vy - a.nd.gy[l];
        o[6 + 4 * q] = vz - a.nd.gz[l];
    }
    o[3 + 4 * K] = ox;
    o[4 + 4 * K] = oy;
    o[5 + 4 * K] = oz;
    o[6 + 4 * K] = rx;
    o[7 + 4 * K] = ry;
    o[8 + 4 * K] = rz;
    kp_energy[s] = ((double)rx * rx + (double)ry * ry) + (double)rz * rz;
}

struct PcgArgs {
    const int32_t *row_ptr, *col_idx;
    const float *blocks, *minv, *g;
    float lambda;
    const float *lambda_dev = nullptr;   // optional device damping, read in place of lambda
    int m, nblk, iters, cap;
    float *x, *r, *z, *p, *q;
    double *part;     // [(it * 4 + kind) * nblk + block], kind 0 = r.z, 1 = r.r, 2 = p.q, 3 = #non-finite x
    int32_t *status;  // [it]: 0 running, 2 stopped by breakdown (propagates)
    int32_t *done;    // [it]: 1 if iteration it updated x
    unsigned spin = 1u << 18;   // polls of one wait of the one-launch solves before they give up
    double *halo[2] = {nullptr, nullptr};   // 12 m each: the exchanged vector of the pipelined recurrence
    bool textbook = false;      // one-launch solve: the textbook recurrence instead of the pipelined one
};

// One registration problem of a batch solved side by side: its step and
// solve arguments (carved from its own slice of the batch workspace) and
// where its blocks start in each batched launch.
struct BatchItem {
    StepArgs a;          // minv set; flags come from rep[it]
    StepScratch s;
    PcgArgs p;
    misslam_report *rep; // gn_iters + 1 entries
    float *params;       // m x 12, updated in place
    const float *depth;
    float reject;
    int64_t pp0;         // first point-pass block
    int npb;             // point-pass blocks
    int nm0;             // first normal-map block
    int row0;            // first assembly workgroup
    int ne0;             // first node-energy block
    int wg0, wgs;        // persistent-solve workgroups
};

// Growth and maintenance after fusion: the model (in/out, up to its
// capacity), the fusion's registration outputs, the frame and the settings;
// stage* are the workspace copies of [survivors | lifted pixels].
struct GrowArgs {
    float *px, *py, *pz, *nx, *ny, *nz, *w;
    int32_t *stamp;
    int64_t n, capacity;
    float *gx, *gy, *gz, *params;
    int m, node_capacity;
    const int32_t *reg_map, *registered;
    const float4 *nmap;
    Cam cam;
    double Rd[9], Td[3];
    float voxel, node_spacing, tau_weight;
    int tau_time, frame;
    float *stage;             // 7 planes of stage_cap floats: p, n, w
    int32_t *stage_stamp;
    int64_t stage_cap;        // n + W H
    const int32_t *count;     // device: [0] staged points, [1] kept, [2] final, [3] new nodes
    // optional colour (Eq.(13)): the frame's H x W x 3 image, the point colours (planes r, g, b, color_stride
    // apart, capacity each) and 3 staging planes of stage_cap
    const float *image = nullptr;
    float *color = nullptr;
    int64_t color_stride = 0;
    float *stage_color = nullptr;
    // optional stability S_i (capacity flags) and its staging plane (stage_cap)
    uint8_t *stable = nullptr;
    uint8_t *stage_stable = nullptr;
};

struct GrowScratch {
    int32_t *flags, *alive, *bcount, *boffs, *bcount2, *boffs2, *count, *hist, *hoffs;
    unsigned long long *k0, *k1;
    uint32_t *v0, *v1;
    float *cent;
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
    const float *image = nullptr;  // optional H x W x 3 colour of the frame (Eq.(13))
    float *color = nullptr;        // optional point colours (planes r, g, b, color_stride apart), in/out
    int64_t color_stride = 0;
};

hipError_t launch_fuse(const FuseArgs &f, float *gx, float *gy, float *gz, float *params, int m, int32_t *reg_map,
                       hipStream_t st);

// With key points (kp, c), the same launch also evaluates them (kp_eval_body) in blocks of its own.
hipError_t launch_point_pass(const StepArgs &a, const StepScratch &s, hipStream_t st, const KeyArgs *kp = nullptr,
                             const CorrScratch *c = nullptr);
// Joint pose form: the point pass with the pose read from a.pose_dev, also writing s.jp and s.pose_part (and
// evaluating the key points (kp, c) at the device pose in blocks of its own).
hipError_t launch_point_pass_joint(const StepArgs &a, const StepScratch &s, hipStream_t st,
                                   const KeyArgs *kp = nullptr, const CorrScratch *c = nullptr);
int point_blocks(int64_t n);

// Joint pose + ED (Eq.(10)).
struct JointScratch {
    float *B;             // 72 m: the border, row 3c + a of node j, column k at B[j * 72 + (3c + a) * 6 + k]
    double *sys;          // 36 H_pp, 6 g_p, 36 (H_pp + lambda I)^-1
    double *jpart;        // (pcg_iters + 2) x 10 x nblk partial sums
    double *pst;          // (pcg_iters + 2) x 32: pose r, z, p, q, x per iteration
    unsigned long long *jbar;   // sync area of the one-launch joint solve (zeroed by launch_pose_setup)
};
struct PosePrior {
    float R0[9], T0[3];
    float w_r, w_p, w_data;
};
hipError_t launch_pose_init(const Pose &pose, float *pose_dev, hipStream_t st);
hipError_t launch_border_rows(const StepArgs &a, const StepScratch &s, float *B, hipStream_t st);
// Reduces the point pass's pose partials, adds the priors (energies into rep) and factors the damped block.
// jbar (optional): the joint solve's sync area for m node rows, zeroed on the way.  kp (optional): the key
// points' part of H_pp and g_p, from c.kp_data (carrying points outside [0, n) skipped).
hipError_t launch_pose_setup(const float *pose_dev, const PosePrior &pr, const double *pose_part, int nblk_pts,
                             float lambda, double *sys, misslam_report *rep, hipStream_t st,
                             unsigned long long *jbar = nullptr, int m = 0, const KeyArgs *kp = nullptr,
                             const CorrScratch *c = nullptr, int64_t n = 0, int k = 4);
// Joint PCG into delta (12 m) and the pose step; applies params += delta and the pose step unless non-finite
// or (one launch) a workgroup timed out.  One launch when every workgroup fits at once, else (or with kernels)
// one launch per phase: the same partition and reduction order, so the same bits.  spin: polls of one wait of
// the one-launch form (0: the default bound).
hipError_t launch_joint_pcg(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                            float lambda, int iters, float *delta, const PcgScratch &s, const JointScratch &js,
                            misslam_report *rep, float *params, float *pose_dev, hipStream_t st,
                            bool kernels = false, unsigned spin = 0);
// The list-entry packing the assembly reads; run once per registration (the graph, canonical points and node
// positions are fixed across its Gauss-Newton steps) before the first launch_assemble.
hipError_t launch_list_pack(const StepArgs &a, const StepScratch &s, hipStream_t st);
hipError_t launch_assemble(const StepArgs &a, const StepScratch &s, hipStream_t st);
// Eq.(9): adds the term to the blocks and gradient of every row it touches (after launch_assemble and
// launch_kp_eval) and re-inverts their damped diagonal blocks.
// With B (joint pose form), also adds the key points' part of the pose border B_j.
hipError_t launch_corr_rows(const StepArgs &a, const KeyArgs &kp, const CorrScratch &c, hipStream_t st,
                            float *B = nullptr);
// kp_nodes[s k + q] = node q of key point s's carrying point (-1 if its index is outside [0, n)); once per
// registration, before launch_corr_rows.
hipError_t launch_kp_nodes(const StepArgs &a, const KeyArgs &kp, int32_t *kp_nodes, hipStream_t st);
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
// zero_words (optional): zero_count words (a multiple of 4, 16-byte aligned) cleared on the way
// (the next persistent solve's sync area); kp_energy (optional): kp_count key-point energies summed into
// rep->e_corr
hipError_t launch_energy_report(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                                hipStream_t st, unsigned *zero_words = nullptr, int zero_count = 0,
                                const double *kp_energy = nullptr, int kp_count = 0);
struct ReportArgs;
// The same report's arguments, for a solve that forms it in an extra workgroup (launch_pcg_persistent), and
// the report kernel on them (when the solve does not).
void report_args(const StepScratch &s, int64_t n, int m, misslam_report *rep, float reject_thr,
                 const double *kp_energy, int kp_count, ReportArgs &out);
hipError_t launch_energy_report(const ReportArgs &ra, hipStream_t st);
hipError_t launch_bjacobi(const GraphView &g, int m, const float *blocks, float lambda, float *minv,
                          int32_t *flags, hipStream_t st);
// PCG solve into delta; when params != nullptr also applies params += delta (the GN update).  lambda_dev
// (optional): device damping read in place of lambda.
hipError_t launch_pcg_update(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                             float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                             float *params, hipStream_t st, const float *lambda_dev = nullptr);
// Adaptive damping (Sec. II-F): lambda slot := lambda0; x_trial = x + dx; then the decision on the
// trial point (objectives from rep_x and rep_t, weights w[4] = data, rot, reg, corr): x := x_trial when
// lower, the lambda slot updated, rep_x's lm_* fields written.
hipError_t launch_lm_init(float *lambda_slot, float lambda0, hipStream_t st);
hipError_t launch_lm_trial(const float *x, const float *dx, float *x_trial, int n, hipStream_t st);
hipError_t launch_lm_decide(misslam_report *rep_x, const misslam_report *rep_t, const misslam_lm_params &lm,
                            float w_data, float w_rot, float w_reg, float w_corr, float *x, const float *x_trial,
                            int n, float *lambda_slot, hipStream_t st);
// graph_info (optional): the graph's info words; a graph overflow (info[3]) starts every entry's flags.
hipError_t launch_report_init(misslam_report *rep, int count, hipStream_t st, const int32_t *graph_info = nullptr);
// Same solve as launch_pcg_update in one launch whose workgroups must all be
// resident (cooperative: guaranteed by the runtime; plain: no other work may
// hold the CUs); *used = false when the device cannot hold the grid at once
// (nothing launched, caller falls back).  params += delta is a separate launch
// after the solve (launch_step_commit), so a timeout discards the whole step.
// spin: polls of one wait before it gives up (0: the default bound).
hipError_t launch_pcg_persistent(const GraphView &g, int m, const float *blocks, const float *gvec, const float *minv,
                                 float lambda, int iters, float *delta, const PcgScratch &s, misslam_report *rep,
                                 float *params, hipStream_t st, bool *used, bool cooperative,
                                 int zeroed_words = 0, const float *lambda_dev = nullptr, unsigned spin = 0,
                                 bool textbook = false, const ReportArgs *report = nullptr);
// A step's energy report (energy_report_body) run by one extra workgroup of the one-launch solve: its inputs
// come from the kernels before the solve, and the step commit after it reads its flags.
struct ReportArgs {
    const double *pt_part = nullptr;
    int npb = 0;
    const double *node_part = nullptr;
    int m = 0;
    misslam_report *rep = nullptr;   // null: no report workgroup
    float reject = 0.f;
    const double *kp_energy = nullptr;
    int kp_count = 0;
};
// The pose columns of the joint system (pose + ED unknowns) for its one-launch solve.
struct JointExtra {
    const float *B = nullptr;      // the border: row 12 j + a, column k at B[j * 72 + a * 6 + k]
    const double *sys = nullptr;   // H_pp (36), g_p (6), (H_pp + lambda I)^-1 (36)
    double *xp_out = nullptr;      // the pose step (6), written by the first workgroup
};
// The joint system's one-launch solve (the tiled textbook recurrence with the pose part; base.part, x, z and the
// system as for launch_pcg_persistent).  bar: its sync area, of which zeroed_words 8-byte words are zero.  Sets
// *used = false and launches nothing when the grid does not fit (the per-phase joint kernels are used then).
hipError_t launch_joint_pcg_persistent(const PcgArgs &base, const JointExtra &jx, unsigned long long *bar,
                                       int zeroed_words, misslam_report *rep, hipStream_t st, bool *used);
// x += dx (n entries) unless rep's flags, ORed with extra's when given (and written back into rep), carry
// MISSLAM_FLAG_NONFINITE or MISSLAM_FLAG_SYNC_TIMEOUT: the whole step or nothing.
hipError_t launch_step_commit(float *x, const float *dx, int n, misslam_report *rep, hipStream_t st,
                              const misslam_report *extra = nullptr);
int pcg_blocks(int m);
// Batched launches: one grid covers every problem of items[0..count).
hipError_t launch_normal_map_batched(const BatchItem *items, int count, int total_blocks, hipStream_t st);
hipError_t launch_point_pass_batched(const BatchItem *items, int count, int k, int64_t total_blocks, int it,
                                     hipStream_t st);
hipError_t launch_list_pack_batched(const BatchItem *items, int count, int k, int total_rows, hipStream_t st);
hipError_t launch_assemble_batched(const BatchItem *items, int count, int k, int total_rows, int it, int waves,
                                   hipStream_t st);
hipError_t launch_energy_report_batched(const BatchItem *items, int count, int it, unsigned *zero_words,
                                        int zero_count, hipStream_t st);
hipError_t launch_node_energy_batched(const BatchItem *items, int count, int total_blocks, hipStream_t st);
hipError_t launch_report_init_batched(const BatchItem *items, int count, int per_problem, hipStream_t st);
// Side-by-side persistent solves: cooperative (co-residency checked by the
// runtime) unless capture is set, where the grid is checked against the
// occupancy instead.  *used = false: the shape does not fit; nothing launched.
// Each problem's params += dx follows in a second launch (skipped per problem on a non-finite value or a
// timeout in its report).
hipError_t launch_pcg_batched(const BatchItem *items, int count, int rows_per_wg, int total_wgs, int total_rows,
                              int it, unsigned *bar, bool cooperative, hipStream_t st, bool *used, bool textbook);
int pcg_batched_fits(int total_wgs, bool textbook);

hipError_t launch_grow(GrowArgs g, const GrowScratch &s, int64_t *counts_out, hipStream_t st);
int64_t grow_hist_entries(int64_t cap);

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st);

}  // namespace msl
