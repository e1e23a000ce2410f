/*
 * misslam.h - C ABI of a gfx950 (MI355X) library for the per-frame dense
 * deformable registration of MIS-SLAM (Song et al., arXiv:1803.02009):
 * Gauss-Newton registration of an embedded-deformation (ED) graph to a depth
 * map, and the fusion of the depth into the deformed point model.
 *
 * Conventions
 *  - Every array pointer is a DEVICE pointer owned by the caller unless marked
 *    (host).  Structs themselves are host structs passed by pointer.
 *  - Units are millimetres.  Model points, normals and nodes are SoA planes of
 *    float32.  Node parameters are m x 12 float32 rows x_j = (c1, c2, c3, t_j):
 *    A_j = [c1 c2 c3] column by column (the columns of the rotation term,
 *    Eq.(5)), x[3c + a] = A_j[a][c], x[9 + a] = t_j[a].
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream); outputs are valid once the stream is synchronised.  Argument
 *    checks happen on the host before anything is enqueued: a negative status
 *    means nothing was launched.  Numeric failures found on the device are not
 *    return codes; they set bits in misslam_report.flags.
 *  - Hot calls allocate no device memory: scratch comes from the caller's
 *    workspace `ws` of `ws_bytes` (query misslam_workspace_bytes).  Calls that
 *    share a workspace must not overlap in time.
 *  - Decision arithmetic (nearest nodes, pixel rounding, gates) is float64 with
 *    a fixed operation order and no contraction, so integer results are
 *    reproducible bit for bit by a float64 reference given the same inputs.
 *  - No floating-point atomics are used: results are bitwise deterministic.
 */
#ifndef MISSLAM_H
#define MISSLAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MISSLAM_OK = 0,
    MISSLAM_EINVAL = -1,       /* null pointer or out-of-range scalar */
    MISSLAM_ESHAPE = -2,       /* sizes inconsistent with each other */
    MISSLAM_EWORKSPACE = -3,   /* workspace too small */
    MISSLAM_EHIP = -4,         /* a HIP runtime call failed (see misslam_last_hip_error) */
    MISSLAM_ECAPACITY = -5,    /* a caller-provided capacity is too small */
    MISSLAM_EUNSUPPORTED = -6  /* valid request this build does not implement */
} misslam_status;

/* device-side failure bits in misslam_report.flags */
#define MISSLAM_FLAG_NONSPD_BLOCK   0x1   /* a damped diagonal block was not SPD; its preconditioner is I */
#define MISSLAM_FLAG_PCG_BREAKDOWN  0x2   /* p^T A p <= 0 in PCG; the solve stopped early */
#define MISSLAM_FLAG_NONFINITE      0x4   /* NaN/Inf met in an energy or the update; x left unchanged */
#define MISSLAM_FLAG_FRAME_REJECT   0x8   /* mean |r| above params.reject_threshold */
#define MISSLAM_FLAG_GRAPH_OVERFLOW 0x10  /* a per-frame graph capacity was exceeded */
#define MISSLAM_FLAG_SYNC_TIMEOUT   0x20  /* the persistent solve gave up waiting for another workgroup; discard the step */

#define MISSLAM_WEIGHT_GAUSS  0   /* w_j ~ exp(-|v-g_j|^2 / (2 sigma^2)), normalised over k */
#define MISSLAM_WEIGHT_LINEAR 1   /* Eq.(2): w_j ~ max(0, 1 - |v-g_j| / d_(k+1)), normalised */

/* The one-launch PCG needs all of its workgroups (at most one per CU) resident
 * at once, since they wait for each other's partials. */
#define MISSLAM_LAUNCH_PLAIN 0       /* an ordinary launch: all are resident when no other work holds the CUs
                                        (the usual case on the library's stream); a workgroup that waits too
                                        long sets MISSLAM_FLAG_SYNC_TIMEOUT */
#define MISSLAM_LAUNCH_COOPERATIVE 1 /* a cooperative launch: residency guaranteed by the runtime, at about
                                        15 us more per solve */
#define MISSLAM_LAUNCH_KERNELS 2     /* no one-launch solve: one launch per PCG phase, nothing depends on
                                        residency (the path taken anyway when the grid does not fit); the
                                        same results to rounding; not for batches (MISSLAM_EUNSUPPORTED) */

/* The recurrence of the one-launch solve (fixed pose; the joint pose form and
 * MISSLAM_LAUNCH_KERNELS always use the textbook one). */
#define MISSLAM_SOLVE_TEXTBOOK 0     /* the textbook recurrence: two exchanges per iteration, float32 vectors
                                        with float64 sums (default) */
#define MISSLAM_SOLVE_PIPELINED 1    /* pipelined preconditioned CG (Ghysels and Vanroose 2014): one exchange
                                        between workgroups per iteration, float64 vectors */

#define MISSLAM_PREC_FP32 0       /* plain float32 normal equations */
#define MISSLAM_PREC_BF16 1       /* data-term products in bfloat16 on the matrix cores, float32 accumulation */
#define MISSLAM_PREC_FP16 2       /* same with float16 inputs */

#define MISSLAM_MAX_K    8
#define MISSLAM_MAX_PCG  64
#define MISSLAM_MAX_ROW  32       /* max blocks per row of the normal matrix (node degree + 1) */
#define MISSLAM_MAX_LIST 2048     /* node lists up to this length are sorted in one LDS pass; longer ones are merged */
#define MISSLAM_NOALLOC_SCRATCH_BYTES 100663296   /* 96 MiB: scratch of misslam_gn_register_noalloc, per device */
#define MISSLAM_MAX_KEYPOINTS 16777216   /* max key points per registration (2^24) */
#define MISSLAM_SOLVE_ROWS 16     /* node rows per workgroup of the one-launch PCG of a single problem
                                     with at most 16 rows per CU (larger ones pack up to 21) */

/* (host) pinhole camera of the depth map: pixel (u, v) = (fx x/z + cx, fy y/z + cy) */
typedef struct { int32_t width, height; float fx, fy, cx, cy; } misslam_camera;

/* (host) rigid scope pose of the frame, camera = R * world + T, R row-major (Eq.(1)'s R, T) */
typedef struct { float R[9]; float T[3]; } misslam_pose;

/* model point cloud (Sec. II-A): coordinate, normal, fusion weight, time stamp, stability */
typedef struct {
    int64_t n, capacity;
    float *px, *py, *pz;      /* canonical coordinates, n (<= capacity) each */
    float *nx, *ny, *nz;      /* unit normals */
    float *w;                 /* fusion weight (Eq.(15)); may be NULL outside misslam_fuse */
    int32_t *stamp;           /* last registered frame; may be NULL outside misslam_fuse */
    uint8_t *stable;          /* stability S_i (Sec. II-G), 0 or 1; may be NULL; kept by misslam_grow */
} misslam_points;

/* ED nodes (Sec. II-D): positions g_j and parameters x_j */
typedef struct {
    int32_t m, capacity;
    float *gx, *gy, *gz;      /* m each */
    float *params;            /* m x 12 */
} misslam_nodes;

/*
 * Per-frame graph derived from the canonical points and nodes by
 * misslam_build_graph; read by every other call of the frame.
 *   knn_idx  k x n int32, slot-major (knn_idx[s*n + i]): the k nearest nodes of
 *            point i by (squared distance, node index)
 *   knn_w    k x n float32 normalised skinning weights (Eq.(2) / Gaussian)
 *   row_ptr  m+1, col_idx bsr_cap: block pattern of the normal matrix, row j =
 *            {j} U N(j) ascending, N(j) = nodes sharing a point with j (Eq.(6))
 *   list_ptr m+1, list_pts k*n: the points each node influences, ordered by
 *            (sorted k-node set, point index)
 *   list_key 2*k*n int32: per list entry of node j, the positions in row j of
 *            the entry's k nodes sorted by node index, 8 bits each (0xFF = cut
 *            from an overflowed row), nodes 0-3 in word 0, 4-7 in word 1
 *   info     8 int32 written by the device: [0] nnzb, [1] largest row,
 *            [2] largest list, [3] overflow flag (MISSLAM_FLAG_GRAPH_OVERFLOW)
 */
typedef struct {
    int32_t k, bsr_cap;
    int32_t *knn_idx;
    float *knn_w;
    int32_t *row_ptr, *col_idx;
    int32_t *list_ptr, *list_pts;
    int32_t *list_key;
    int32_t *info;
} misslam_graph;

/* (host) solver settings; defaults from the paper (Sec. III-B) via misslam_default_params */
typedef struct {
    int32_t k;                 /* nodes per point, 1..MISSLAM_MAX_K */
    int32_t weight_kind;       /* MISSLAM_WEIGHT_* */
    float sigma;               /* Gaussian width, mm */
    float w_rot, w_reg, w_data;/* 1000, 10000, 1 */
    double eps_d;              /* distance gate, Eq.(7): 15 mm */
    double cos_eps_n;          /* normal gate, Eq.(7): cos(10 deg) */
    float lambda;              /* damping added to the diagonal of H and of M */
    int32_t gn_iters;          /* Gauss-Newton iterations per frame */
    int32_t pcg_iters;         /* PCG iterations per Gauss-Newton step, <= MISSLAM_MAX_PCG */
    int32_t precision;         /* MISSLAM_PREC_* */
    int32_t refine_steps;      /* iterative-refinement steps for BF16/FP16 */
    float reject_threshold;    /* mean |r| above which FRAME_REJECT is set; <= 0 disables */
    int32_t solve_launch;      /* MISSLAM_LAUNCH_*: how the one-launch PCG is started */
    int32_t sync_spin_limit;   /* polls of one wait in the one-launch solves before they give up
                                  (MISSLAM_FLAG_SYNC_TIMEOUT, the step discarded); 0: 262144 */
    int32_t solve_form;        /* MISSLAM_SOLVE_*: recurrence of the one-launch solve */
    int32_t asm_waves;         /* assembly tile: waves per node row, 1 or 2; 0: 2 (a batch created with
                                  rows_per_wg 0 times both) */
} misslam_params;

/* one entry per Gauss-Newton iteration, plus a final entry at the returned parameters (device) */
typedef struct {
    double e_data, e_rot, e_reg;             /* unweighted sums of squares at the linearisation point */
    double pcg_resid[MISSLAM_MAX_PCG + 1];   /* |r_i| of the PCG residual, i = 0..pcg_iters_done */
    int32_t n_valid;                         /* points that passed the Eq.(7) gates */
    int32_t flags;                           /* MISSLAM_FLAG_* */
    int32_t pcg_iters_done;
    int32_t reserved;
    double e_corr;                           /* unweighted Eq.(9) key-point energy (0 without key points) */
    /* adaptive damping (misslam_lm_register; all 0 otherwise): the weighted objective at the step's
     * linearisation point and at the trial point x + dx, the damping the step was solved with, and
     * whether the trial point was taken */
    double lm_e, lm_e_trial;
    float lm_lambda;
    int32_t lm_accepted;
    /* joint pose (misslam_joint_register; 0 otherwise): unweighted Eq.(10) energies E_r = |log(R R0^T)|^2
     * and E_p = |C - C0|^2 at the step's pose, C = -R^T T the camera centre */
    double e_pose_r, e_pose_p;
} misslam_report;

/* (host) weights of the Eq.(10) global-pose terms, Sec. III-B: w_r = 1e6, w_p = 1e3 */
typedef struct {
    float w_r;
    float w_p;
} misslam_pose_weights;

/* (host) adaptive damping schedule of misslam_lm_register (Sec. II-F names Levenberg-Marquardt and no
 * schedule; this is the classical one): a step solved with damping lambda is taken when it lowers the
 * weighted Eq.(3) objective, and lambda then becomes max(lambda * down, lambda_min); otherwise the
 * parameters stay and lambda becomes min(lambda * up, lambda_max). */
typedef struct {
    float lambda0;             /* damping of the first step: 1e-3 */
    float up;                  /* 10 */
    float down;                /* 0.1 */
    float lambda_min;          /* 1e-6 */
    float lambda_max;          /* 1e6 */
} misslam_lm_params;

/* (host) key-point matches of the Eq.(9) correspondence term, Sec. II-E: each key point is carried by one
 * model point (its k nodes and skinning weights) and matched to a 3-D position in the frame's camera
 * coordinates (those of the depth map).  The term enters the least-squares objective as
 * w_corr * sum_s |V~_s - V_s|^2, V~_s the Eq.(1) warp of the carrying point with the pose applied. */
typedef struct {
    int32_t count;             /* key points, 0 <= count <= min(n, MISSLAM_MAX_KEYPOINTS) */
    float w_corr;              /* weight, Sec. III-B: 10 */
    const int32_t *point;      /* (device) count carrying point indices; indices outside [0, n) are skipped */
    const float *target;       /* (device) count x 3 matched positions (x, y, z), camera coordinates */
} misslam_keypoints;

/* (host) fusion settings (Alg. 1-2, Eqs.(12)-(15), Sec. III-B) */
typedef struct {
    double tau;                /* |z~ - D| gate of Alg. 1: 10 mm */
    double cos_delta;          /* normal angle gate of Alg. 1: cos(10 deg) */
    float w_max;               /* weight cap of Eq.(15): 20 */
    int32_t frame;             /* stamp written to registered points */
} misslam_fuse_params;

/* ------------------------------------------------------------------ utilities */

/* Fills *p with the paper's settings (Sec. III-B) and k = 4 Gaussian weights, sigma = 1. (host) */
void misslam_default_params(misslam_params *p);

/* Static description of a status code. */
const char *misslam_status_string(int32_t status);

/* The last hipError_t seen by a failing call on this thread (0 if none). */
int32_t misslam_last_hip_error(void);

/* Bytes of workspace needed by every call below for n points, m nodes and a
 * width x height depth map, or 0 if the sizes are invalid. */
size_t misslam_workspace_bytes(int64_t n, int32_t m, int32_t width, int32_t height,
                               const misslam_params *params);

/* ------------------------------------------------------------------ per-frame setup */

/*
 * Depth preprocessing for the data term (Eq.(8)).  out (height x width x 4
 * float32, pixel-major) receives (Nx, Ny, Nz, D) per pixel: the unit normal
 * N = normalize(b x a), a = V(u+1,v) - V(u-1,v), b = V(u,v+1) - V(u,v-1),
 * V(u,v) = D (u-cx)/fx, (v-cy)/fy, 1), computed in float64 and rounded; N = 0
 * on the border, next to an empty pixel or where b x a = 0.
 */
misslam_status misslam_normal_map(const float *depth, const misslam_camera *camera, float *out,
                                  void *stream);

/*
 * kNN sets, skinning weights (Eq.(2)), node graph N(j) (Eq.(6)), block pattern
 * and node -> point lists from the canonical points and nodes.  Capacities:
 * bsr_cap blocks; rows longer than MISSLAM_MAX_ROW (or a pattern beyond
 * bsr_cap) set graph->info[3] = MISSLAM_FLAG_GRAPH_OVERFLOW; every report of a
 * registration on that graph then carries the flag.  Node lists have no length
 * limit (info[2] holds the longest).
 */
misslam_status misslam_build_graph(const misslam_points *points, const misslam_nodes *nodes,
                                   const misslam_params *params, misslam_graph *graph, void *ws,
                                   size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ hot path */

/*
 * ED warp, Eq.(1): out_pos = R sum_j w_j [A_j (v - g_j) + g_j + t_j] + T and
 * out_nrm = normalize(R sum_j w_j A_j^-T n), both 3 x n float32 planes.
 * pose may be NULL (world coordinates).  out_nrm may be NULL.
 */
misslam_status misslam_warp(const misslam_points *points, const misslam_nodes *nodes,
                            const misslam_graph *graph, const misslam_pose *pose, float *out_pos,
                            float *out_nrm, void *stream);

/*
 * Linearisation of Eq.(3) (data, rotation and regularisation terms) at the
 * current node parameters: warp, projective association with the Eq.(7)
 * gates, point-to-plane residuals (Eq.(8)), and the normal equations
 * H = sum w J^T J (BSR, graph pattern, nnzb x 12 x 12 float32 row-major, both
 * triangles stored) and g = sum w J^T r (m x 12).  corr (n int32) receives
 * the matched pixel v*width+u or -1; it may be NULL.  rep (device, 1 entry)
 * receives the energies and n_valid.  nmap is the output of misslam_normal_map
 * for this depth map.
 */
misslam_status misslam_build_normal_eq(const misslam_points *points, const misslam_nodes *nodes,
                                       const misslam_graph *graph, const float *nmap,
                                       const misslam_camera *camera, const misslam_pose *pose,
                                       const misslam_params *params, float *blocks, float *g,
                                       int32_t *corr, misslam_report *rep, void *ws, size_t ws_bytes,
                                       void *stream);

/*
 * Block-Jacobi PCG for (H + lambda I) delta = -g on the graph pattern:
 * params->pcg_iters iterations from delta = 0, float32 products and float64
 * reductions.  delta: m x 12.  rep (device, 1 entry) receives the residual
 * norms, iterations done and flags.
 */
misslam_status misslam_pcg_solve(const misslam_graph *graph, int32_t m, const float *blocks,
                                 const float *g, const misslam_params *params, float *delta,
                                 misslam_report *rep, void *ws, size_t ws_bytes, void *stream);

/*
 * One frame of registration (Sec. II-E, II-F): params->gn_iters damped
 * Gauss-Newton steps on the node parameters (nodes->params in/out; the caller
 * initialises them, normally to A = I, t = 0), pose fixed.
 * With params->precision BF16 or FP16 (k <= 4) the data term of each step's
 * normal matrix is formed on the matrix cores from Jacobian rows rounded to
 * that type (float32 accumulation; regularisers, gradient and PCG as in the
 * float32 form), and params->refine_steps iterative-refinement steps win the
 * accuracy back: rho = -g - H32 dx with H32 dx evaluated matrix-free in
 * float32 from the points, then dx += (H_lo + lambda I)^-1 rho.  rep (device)
 * holds gn_iters + 1 entries: one per step at its linearisation point and a
 * final one at the returned parameters.  corr_hist, if not NULL, receives
 * the gn_iters x n correspondence arrays.  depth is height x width float32.
 */
misslam_status misslam_gn_register(const misslam_points *points, misslam_nodes *nodes,
                                   const misslam_graph *graph, const float *depth,
                                   const misslam_camera *camera, const misslam_pose *pose,
                                   const misslam_params *params, misslam_report *rep,
                                   int32_t *corr_hist, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory or pass a workspace: code
 * recorded under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The float32 form of misslam_gn_register (same kernels, same
 * arguments and results bit for bit) with its scratch in a file-scope device
 * array of MISSLAM_NOALLOC_SCRATCH_BYTES (96 MiB) that every device the library
 * runs on holds until the process ends.  It calls no hipMalloc or hipFree and
 * records no profiling events; on its first call on a device it looks up that
 * device's address of the array (hipGetSymbolAddress).
 * Errors: MISSLAM_EINVAL as misslam_gn_register; MISSLAM_EUNSUPPORTED unless
 * params->precision is FP32; MISSLAM_ECAPACITY when the frame's scratch (normal
 * map, point pass, packed node lists, normal matrix, solve vectors: about
 * 75 MB at 640x480, 250,000 points, 1,600 nodes, k = 4) exceeds the array.
 * Every size check runs before any HIP call.
 * All calls on one device share the one array and each leaves its contents
 * behind (the calls clear what must start at zero themselves): calls that
 * overlap on one device, on different streams or threads, race and must not
 * be issued.
 */
misslam_status misslam_gn_register_noalloc(const misslam_points *points, misslam_nodes *nodes,
                                           const misslam_graph *graph, const float *depth,
                                           const misslam_camera *camera, const misslam_pose *pose,
                                           const misslam_params *params, misslam_report *rep,
                                           int32_t *corr_hist, void *stream);

/*
 * misslam_gn_register with the key-point correspondence term of Eq.(3) added
 * (Eq.(9), Sec. II-E): each Gauss-Newton step adds, for every key point,
 * w_corr * w_j w_l (d_j d_l^T) (x) I3 to the blocks (j, l) of its carrying
 * point's k nodes and w_corr * w_j d_j (x) R^T r to g_j, with d_j = (v - g_j, 1)
 * and r the warped point minus its match, before the block-Jacobi inverses are
 * formed.  rep[i].e_corr holds the unweighted key-point energy.  keys must not
 * be NULL (count 0 runs exactly as misslam_gn_register); float32 form only
 * (MISSLAM_EUNSUPPORTED otherwise).
 */
misslam_status misslam_gn_register_keypoints(const misslam_points *points, misslam_nodes *nodes,
                                             const misslam_graph *graph, const float *depth,
                                             const misslam_camera *camera, const misslam_pose *pose,
                                             const misslam_params *params, const misslam_keypoints *keys,
                                             misslam_report *rep, int32_t *corr_hist, void *ws,
                                             size_t ws_bytes, void *stream);

/* (host) fills *lm with the defaults above */
void misslam_default_lm_params(misslam_lm_params *lm);

/*
 * Joint registration of the rigid pose and the ED graph (Eq.(3) with the
 * Eq.(10) pose terms; Sec. II-F: six more unknowns).  The pose *pose (the
 * front end's estimate) is the start and the prior: E_r = |log(R R0^T)|^2,
 * E_p = |C - C0|^2 with C = -R^T T the camera centre, weighted by *pw.  Each
 * Gauss-Newton step perturbs the pose by a rigid motion in camera coordinates
 * (R <- exp([dw]x) R, T <- exp([dw]x) T + dt), so the data rows gain pose
 * columns (v~ x N, N); the bordered system [[H, B], [B^T, H_pp]] is solved by
 * block-Jacobi PCG over the joint vector (params->pcg_iters iterations, the
 * damping params->lambda on the whole diagonal, the damped 6x6 pose block in
 * the preconditioner), then x += dx and the pose takes its step.
 * pose_out (device, 12 floats: R row-major, then T) receives the refined
 * pose; it is also the working pose during the call.  keys (may be NULL) adds
 * the Eq.(9) term as in misslam_gn_register_keypoints, its rows gaining the
 * pose columns [-[v~]x, I]: all six terms of Eq.(3) together.  rep as for
 * misslam_gn_register, with e_pose_r / e_pose_p (and e_corr) set.  Errors as
 * misslam_gn_register; MISSLAM_EINVAL for pw or pose_out NULL or a weight
 * that is negative or not finite; float32 form only (MISSLAM_EUNSUPPORTED
 * otherwise).
 */
misslam_status misslam_joint_register(const misslam_points *points, misslam_nodes *nodes,
                                      const misslam_graph *graph, const float *depth,
                                      const misslam_camera *camera, const misslam_pose *pose,
                                      const misslam_pose_weights *pw, const misslam_keypoints *keys,
                                      const misslam_params *params, float *pose_out, misslam_report *rep,
                                      int32_t *corr_hist, void *ws, size_t ws_bytes, void *stream);

/*
 * Registration with adaptive Levenberg-Marquardt damping (Sec. II-F): step i
 * linearises at x as misslam_gn_register does, solves (H + lambda_i I) dx = -g
 * with the same block-Jacobi PCG, evaluates the weighted objective
 * w_data E_data + w_rot E_rot + w_reg E_reg + w_corr E_corr at x + dx (the
 * correspondences re-decided there), and keeps x + dx only when that is lower
 * than at x; lambda follows *lm (params->lambda is not used).  keys may be
 * NULL (no key-point term) or as for misslam_gn_register_keypoints.  rep
 * (device) holds gn_iters + 1 entries as for misslam_gn_register, with the
 * lm_* fields of the first gn_iters set.  Errors as misslam_gn_register;
 * MISSLAM_EINVAL for lm NULL or a schedule outside 0 <= lambda_min <=
 * lambda0 <= lambda_max (finite), 1 <= up (finite), 0 < down <= 1; float32
 * form only (MISSLAM_EUNSUPPORTED otherwise).
 */
misslam_status misslam_lm_register(const misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                   const float *depth, const misslam_camera *camera, const misslam_pose *pose,
                                   const misslam_params *params, const misslam_keypoints *keys,
                                   const misslam_lm_params *lm, misslam_report *rep, int32_t *corr_hist, void *ws,
                                   size_t ws_bytes, void *stream);


/*
 * Model update after registration (Sec. II-G, Alg. 1-2, Eqs.(12), (14), (15)).
 * Deforms every point and normal with the frame's final node parameters
 * (world frame, Eq.(1) without the pose), projects them with the pose and
 * keeps per pixel the nearest point (float32 depth, ties to the lower index:
 * the registration map of Alg. 2 step 2).  A winner is registered when the
 * pixel has depth and a normal, |z~ - D| < tau and n~ . N > cos_delta
 * (float64, Alg. 1); it is fused: p <- (w p~ + R^T(V - T)) / (w + 1),
 * n <- normalize((w n~ + R^T N) / (w + 1)), w <- min(w + 1, w_max),
 * stamp <- frame.  All other points take their deformed position and normal.
 * points (in/out) must carry w and stamp.  nodes (in/out): g_j <- g_j + t_j,
 * params reset to A = I, t = 0.  nmap is misslam_normal_map of this depth.
 * reg_map (height x width int32, winner point or -1) and registered (n int32,
 * 1/0) are optional outputs.
 */
/*
 * misslam_fuse with the colour of Eq.(13) fused too: a registered point's
 * colour becomes (w c + I(p)) / (w + 1) per channel, with its weight before
 * the Eq.(15) update and I(p) the frame's colour at its pixel; other points
 * keep theirs.  image (device): height x width x 3 float32, interleaved;
 * color (device, in/out): the r, g and b planes of the point colours at color,
 * color + color_stride and color + 2 color_stride (color_stride >= n).
 * Everything else as misslam_fuse (bitwise the same outputs); MISSLAM_EINVAL
 * for a NULL image or color, or a short stride, when n > 0.
 */
misslam_status misslam_fuse_color(misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                  const float *nmap, const misslam_camera *camera, const misslam_pose *pose,
                                  const misslam_fuse_params *fp, const float *image, float *color,
                                  int64_t color_stride, int32_t *reg_map, int32_t *registered, void *ws,
                                  size_t ws_bytes, void *stream);

misslam_status misslam_fuse(misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                            const float *nmap, const misslam_camera *camera, const misslam_pose *pose,
                            const misslam_fuse_params *fp, int32_t *reg_map, int32_t *registered, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * Energy of Eq.(3) (data, rotation and regularisation terms) and its adjoint.
 * With corr_in == NULL the correspondences are found as in
 * misslam_build_normal_eq (Eq.(7) gates) and written to corr_out (optional);
 * with corr_in given they are held fixed (no gates; the Gauss-Newton
 * linearisation point).  Outputs (each optional, device):
 *   energy      1 double: w_data E_data + w_rot E_rot + w_reg E_reg
 *   grad_params m x 12: dE/dx = 2 sum w J^T r (twice the g of the normal equations)
 *   grad_points 3 x n: dE/dv with kNN sets fixed and the normalised Gaussian
 *               weights moving with the point (MISSLAM_WEIGHT_GAUSS only)
 *   rep         1 report entry (energies, n_valid)
 * Gradients are scaled by *grad_e (device float; NULL means 1).  The paper
 * has no gradient; this is the adjoint of its energy for learning-based or
 * differentiable uses of the registration.
 */
misslam_status misslam_energy_vjp(const misslam_points *points, const misslam_nodes *nodes,
                                  const misslam_graph *graph, const float *nmap, const misslam_camera *camera,
                                  const misslam_pose *pose, const misslam_params *params, const int32_t *corr_in,
                                  int32_t *corr_out, const float *grad_e, float *grad_params, float *grad_points,
                                  double *energy, misslam_report *rep, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ growth and maintenance */

/* (host) settings of the model's growth and maintenance (Alg. 2 steps 3-5, Alg. 3, Sec. III-B) */
typedef struct {
    float voxel;               /* down-sampling box edge: 0.22 mm */
    float node_spacing;        /* node regeneration voxel edge and minimum distance to a node, mm */
    float tau_weight;          /* removal weight bound (the paper gives none): 2 */
    int32_t tau_time;          /* removal age, frames: 10 */
    int32_t frame;             /* the frame's index: the stamp of registered and lifted points */
} misslam_grow_params;

/*
 * Growth and maintenance of the model after misslam_fuse for the same frame
 * (Alg. 2 steps 3-5, Alg. 3).  In order:
 *   1. removal: a point with frame - stamp > tau_time and w < tau_weight is dropped;
 *   2. Group 2: every pixel with depth and a depth normal (nmap, as from
 *      misslam_normal_map) whose reg_map winner is absent or was not
 *      registered (both outputs of misslam_fuse) becomes a point
 *      p = R^T (V - T), n = R^T N, w = 1, stamp = frame, appended in pixel order;
 *   3. down-sampling: voxels of edge voxel (origin 0); in every voxel that
 *      holds a point stamped with this frame and two or more points, the
 *      points merge into the lowest-index one: mean position, renormalised
 *      mean normal (float64, ascending index), largest w and stamp;
 *   4. node regeneration: for each voxel of edge node_spacing holding points,
 *      a node (identity parameters) is appended at their centroid when no
 *      node lies within node_spacing of it; new nodes in ascending
 *      (kz, ky, kx) voxel order.
 * The model is rewritten in place up to points->capacity / nodes->capacity
 * (positions and normals world-frame, as left by misslam_fuse); points->n and
 * nodes->m are the counts before the call and are NOT updated: the device
 * writes counts_out (7 int64): new n, new m, lifted, removed, merged away,
 * new nodes, overflow (1 if a capacity cut the model or the node list).
 * Read them after synchronising the stream and rebuild the graph
 * (misslam_build_graph) before the next registration.  points->w and
 * points->stamp are required.
 */
size_t misslam_grow_workspace_bytes(int64_t n, int32_t width, int32_t height);
misslam_status misslam_grow(misslam_points *points, misslam_nodes *nodes, const int32_t *reg_map,
                            const int32_t *registered, const float *nmap, const misslam_camera *camera,
                            const misslam_pose *pose, const misslam_grow_params *gp, int64_t *counts_out, void *ws,
                            size_t ws_bytes, void *stream);

/*
 * misslam_grow carrying the point colours of Eq.(13) along: survivors keep
 * theirs, a lifted point takes the frame's colour at its pixel, a merged
 * voxel the mean of its members' colours (float64, ascending index).  image
 * (device): height x width x 3 float32, interleaved; color (device, in/out):
 * the r, g, b planes at color, color + color_stride, color + 2 color_stride,
 * each of points->capacity entries (color_stride >= capacity).  Everything
 * else as misslam_grow (bitwise the same outputs); MISSLAM_EINVAL for a NULL
 * image or color or a short stride.
 */
misslam_status misslam_grow_color(misslam_points *points, misslam_nodes *nodes, const int32_t *reg_map,
                                  const int32_t *registered, const float *nmap, const misslam_camera *camera,
                                  const misslam_pose *pose, const misslam_grow_params *gp, const float *image,
                                  float *color, int64_t color_stride, int64_t *counts_out, void *ws, size_t ws_bytes,
                                  void *stream);

/* ------------------------------------------------------------------ uneven batches */

/*
 * Many independent registration problems of different sizes (each its own
 * frame, camera, pose, points, nodes and graph) registered together: every
 * phase of the per-frame loop of misslam_gn_register (normal map, then per
 * Gauss-Newton step the point pass, the row assembly, the energy report and
 * the persistent PCG solve with its update) runs as ONE launch over all
 * problems, and the whole frame is captured once into a hipGraph and
 * replayed by every later call.  Each problem's arithmetic, partition and
 * reduction order are those of misslam_gn_register with the same workgroup
 * tile, so with rows_per_wg = MISSLAM_SOLVE_ROWS every result is bitwise that
 * of calling misslam_gn_register once per problem; another tile changes only
 * the rounding order of the PCG reductions.
 *
 * misslam_problem: host structs holding device pointers, copied at
 *   creation; the pointed-to buffers (points, nodes and their params, graph,
 *   depth) may change contents between calls but not address.  report: device,
 *   params.gn_iters + 1 entries, filled as by misslam_gn_register.
 * misslam_batch_create: count in [1, 1024]; every problem valid for
 *   misslam_gn_register with params (float32 form, graph->k == params->k).
 *   rows_per_wg: the node rows each solve workgroup owns, 1..21, or 0 to let
 *   the first misslam_batch_register time the candidate tiles on the batch
 *   itself and keep the fastest (the tuning runs restore every problem's
 *   params, so results are as if only the final run happened).  Allocates
 *   host and device bookkeeping (released by misslam_batch_destroy).
 * misslam_batch_workspace_bytes: the caller-owned device workspace one call needs.
 * misslam_batch_register: runs the frame of every problem on stream; the
 *   first call (and a call with another workspace or stream) uploads the
 *   descriptors, tunes if asked and captures the graph, synchronising the
 *   stream; later calls only launch the graph and allocate nothing.  Errors
 *   as misslam_gn_register; MISSLAM_EUNSUPPORTED if the solves of the batch
 *   cannot all be resident at once with any tile.
 * misslam_batch_tile: the rows per workgroup in use (0 before the first call).
 * misslam_batch_asm_waves: the assembly tile in use, waves per node row (0
 *   before the first call).  With rows_per_wg 0 and params->asm_waves 0 the
 *   first call times both tiles with every solve tile.
 */
typedef struct {
    misslam_points points;
    misslam_nodes nodes;
    misslam_graph graph;
    const float *depth;
    misslam_camera camera;
    misslam_pose pose;
    misslam_report *report;
} misslam_problem;

typedef struct misslam_batch misslam_batch;

misslam_status misslam_batch_create(const misslam_problem *problems, int32_t count, const misslam_params *params,
                                    int32_t rows_per_wg, misslam_batch **out);
size_t misslam_batch_workspace_bytes(const misslam_batch *batch);
misslam_status misslam_batch_register(misslam_batch *batch, void *ws, size_t ws_bytes, void *stream);
int32_t misslam_batch_tile(const misslam_batch *batch);
int32_t misslam_batch_asm_waves(const misslam_batch *batch);
void misslam_batch_destroy(misslam_batch *batch);

/* ------------------------------------------------------------------ profiling */

/*
 * Phase timers for measurement.  While enabled, each call brackets the
 * launches of every phase it runs with HIP events on its own stream (not
 * allowed during stream capture).  Phases: "normal_map", "build_graph",
 * "point_pass", "assemble", "energy", "bjacobi", "pcg" (the whole PCG solve,
 * including the parameter update), "fuse", "refine" (the float32 matrix-free
 * residual of a low-precision step).  misslam_profile_get synchronises the
 * recorded events and returns the accumulated milliseconds and number of
 * bracketed launches since the last reset.  Returns the previous state.
 */
int32_t misslam_profile_enable(int32_t on);
misslam_status misslam_profile_get(const char *phase, double *total_ms, int64_t *launches);
void misslam_profile_reset(void);

/*
 * Calibration for measurement, not part of the registration: launches
 * `blocks` workgroups of four waves, each wave running eight independent
 * chains of `iters` bf16 16x16x32 matrix-core multiply-adds, on stream, and
 * returns the flops that launch performs in *flops (host).  Timing the launch
 * gives the device's achievable dense bf16 matrix-core rate.  sink (device,
 * blocks x 256 floats) receives the accumulators.  MISSLAM_EINVAL for iters or
 * blocks < 1 or a NULL pointer.
 */
misslam_status misslam_probe_mfma_bf16(int32_t iters, int32_t blocks, float *sink, int64_t *flops, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MISSLAM_H */
