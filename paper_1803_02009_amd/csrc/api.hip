// Host side of libmisslam: argument validation, workspace carving and the
// extern "C" entry points declared in include/misslam.h.  Nothing here
// computes; every step of the method runs in the gfx950 kernels.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "frame.h"

namespace {

// ---------------------------------------------------------------- phase timers (profiling only)

enum Phase {
    PH_NORMAL_MAP, PH_GRAPH, PH_POINT_PASS, PH_ASSEMBLE, PH_ENERGY, PH_BJACOBI, PH_PCG, PH_FUSE, PH_REFINE, PH_GROW,
    PH_LIST_PACK, PH_CORR, PH_LM, PH_POSE, PH_COUNT
};
const char *const kPhaseNames[PH_COUNT] = {"normal_map", "build_graph", "point_pass", "assemble",  "energy",
                                           "bjacobi",    "pcg",         "fuse",       "refine",    "grow",
                                           "list_pack",  "corr",        "lm_trial",  "pose_border"};

struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        int phase;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[PH_COUNT] = {};
    int64_t launches[PH_COUNT] = {};

    hipEvent_t get_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void collect() {
        for (auto &r : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                total_ms[r.phase] += ms;
                launches[r.phase] += 1;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
};

Profiler &prof() {
    static Profiler p;
    return p;
}

// Set while the allocation-free registration enqueues: it records no events
// (creating one can allocate).
thread_local bool tl_no_events = false;

// Brackets the launches of one phase with events on its stream when profiling is on.
struct Timed {
    hipStream_t st;
    int phase;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(int ph, hipStream_t s) : st(s), phase(ph) {
        if (tl_no_events) return;
        Profiler &p = prof();
        std::lock_guard<std::mutex> lk(p.mu);
        if (!p.on) return;
        a = p.get_event();
        b = p.get_event();
        if (a && b) (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a || !b) return;
        Profiler &p = prof();
        std::lock_guard<std::mutex> lk(p.mu);
        (void)hipEventRecord(b, st);
        p.pending.push_back({a, b, phase});
    }
};

thread_local int32_t g_last_hip = 0;

misslam_status hip_fail(hipError_t e) {
    g_last_hip = (int32_t)e;
    return MISSLAM_EHIP;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count) {
        off = align_up(off);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

struct Layout {
    msl::StepScratch step;
    msl::CorrScratch corr;
    float *lm_lambda;   // the adaptive damping of the next step (one float)
    msl::JointScratch joint;
    msl::PcgScratch pcg;
    msl::GraphScratch graph;
    float4 *nmap;
    float *fuse_tmp;
    int32_t *fuse_pix;
    unsigned long long *zbuf;
    misslam_report *rep;
    float *rr;          // regulariser + rotation blocks (low-precision refinement)
    float *jv;          // n: J dx of the matrix-free product
    float *rhs;         // 12m
    float *delta2;      // 12m
    float *blocks;
    float *gvec;
    float *delta;
    size_t bytes;
};

// Optional parts of the registration workspace.  Every entry point that takes a
// caller workspace carves all of them (WS_ALL), so its layout does not depend on
// the form it runs; the allocation-free registration carves the core only.
enum : unsigned {
    WS_CORE = 0,        // normal map, point pass, packed lists, system, solve
    WS_GRAPH = 1u << 0, // kNN grid and pattern scratch (graph setup)
    WS_FUSE = 1u << 1,  // fusion staging and z-buffer
    WS_LOWP = 1u << 2,  // bf16/fp16 form: fp32 regulariser blocks, matrix-free refinement vectors
    WS_KEYS = 1u << 3,  // key-point term
    WS_JOINT = 1u << 4, // joint pose form
    WS_LM = 1u << 5,    // adaptive damping: trial point and its report
    WS_ALL = 63u
};

Layout carve(void *ws, int64_t n, int32_t m, int32_t W, int32_t H, int pcg_iters, int k, unsigned parts = WS_ALL) {
    Carver c{static_cast<char *>(ws)};
    Layout L{};
    const bool graph = parts & WS_GRAPH, fuse = parts & WS_FUSE, lowp = parts & WS_LOWP, keys = parts & WS_KEYS,
               joint = parts & WS_JOINT, lm = parts & WS_LM;
    const int64_t npb = (n + 255) / 256 + 1;
    const int nblk = msl::pcg_blocks(m > 0 ? m : 1);
    const int nblk_max = nblk > 4096 ? nblk : 4096;
    L.nmap = c.take<float4>((size_t)W * H);
    L.step.nr = c.take<float4>((size_t)n);
    L.step.corr = c.take<int32_t>((size_t)n);
    L.step.pt_part = c.take<double>((size_t)3 * npb);
    L.step.node_part = c.take<double>((size_t)2 * m);
    L.step.minv = c.take<float>((size_t)144 * m);
    L.step.flags = c.take<int32_t>(4);
    L.blocks = c.take<float>((size_t)m * MISSLAM_MAX_ROW * 144);
    L.gvec = c.take<float>((size_t)12 * m);
    L.delta = c.take<float>((size_t)12 * m);
    L.pcg.r = c.take<float>((size_t)12 * m);
    L.pcg.z = c.take<float>((size_t)12 * m);
    L.pcg.p = c.take<float>((size_t)12 * m);
    L.pcg.q = c.take<float>((size_t)12 * m);
    L.pcg.part = c.take<double>((size_t)(pcg_iters + 2) * 4 * nblk_max);
    L.pcg.status = c.take<int32_t>((size_t)2 * (pcg_iters + 2));
    L.pcg.bar = c.take<unsigned>(msl::MSL_BAR_WORDS);
    L.pcg.halo = c.take<double>((size_t)24 * m);
    L.pcg.nblk = nblk;
    L.pcg.nblk_max = nblk_max;
    L.graph.tmp = graph ? c.take<int32_t>((size_t)m * MISSLAM_MAX_ROW) : nullptr;
    L.fuse_tmp = fuse ? c.take<float>((size_t)6 * n) : nullptr;
    L.fuse_pix = fuse ? c.take<int32_t>((size_t)n) : nullptr;
    L.zbuf = fuse ? c.take<unsigned long long>((size_t)W * H) : nullptr;
    L.rep = (lowp || lm) ? c.take<misslam_report>(1) : nullptr;
    L.rr = lowp ? c.take<float>((size_t)m * MISSLAM_MAX_ROW * 144) : nullptr;
    L.jv = lowp ? c.take<float>((size_t)n) : nullptr;
    L.rhs = lowp ? c.take<float>((size_t)12 * m) : nullptr;
    L.delta2 = (lowp || lm) ? c.take<float>((size_t)12 * m) : nullptr;
    if (graph) {
        L.graph.cnt = c.take<int32_t>((size_t)2 * m + 8);
        L.graph.grid.hdr = c.take<double>(4);
        L.graph.grid.dims = c.take<int32_t>(4);
        L.graph.grid.start = c.take<int32_t>((size_t)msl::MSL_GRID_CELLS + 1);
        L.graph.grid.cursor = c.take<int32_t>((size_t)msl::MSL_GRID_CELLS);
        L.graph.grid.nodes = c.take<float4>((size_t)m);
        L.graph.ltmp = c.take<int32_t>((size_t)k * n);
    }
    // last, so that every buffer above keeps its place whatever k is
    L.step.lpa = c.take<float4>((size_t)k * n);
    L.step.lpw = c.take<float4>((size_t)k * n * ((k + 3) / 4));
    if (keys) {
        L.corr.kp_nodes = c.take<int32_t>((size_t)k * n);
        L.corr.kp_data = c.take<float>((size_t)(9 + 4 * k) * n);
        L.corr.kp_energy = c.take<double>((size_t)n);
    }
    L.lm_lambda = lm ? c.take<float>(4) : nullptr;
    if (joint) {
        L.step.jp = c.take<float4>((size_t)2 * n);
        L.step.pose_part = c.take<double>((size_t)msl::kPosePart * msl::point_blocks(n));
        L.joint.B = c.take<float>((size_t)72 * m);
        L.joint.sys = c.take<double>(80);
        L.joint.jpart = c.take<double>((size_t)(pcg_iters + 2) * 10 * ((m + 20) / 21));
        L.joint.pst = c.take<double>((size_t)(pcg_iters + 2) * 32);
        L.joint.jbar = c.take<unsigned long long>((size_t)msl::kJointTagWords * msl::kJointMaxWgs);
    }
    L.bytes = align_up(c.off);
    return L;
}

bool valid_params(const misslam_params *p) {
    return p && p->k >= 1 && p->k <= MISSLAM_MAX_K &&
           (p->weight_kind == MISSLAM_WEIGHT_GAUSS || p->weight_kind == MISSLAM_WEIGHT_LINEAR) &&
           (p->weight_kind != MISSLAM_WEIGHT_GAUSS || p->sigma > 0.f) && p->gn_iters >= 0 && p->pcg_iters >= 0 &&
           p->pcg_iters <= MISSLAM_MAX_PCG && std::isfinite(p->lambda) && p->lambda >= 0.f &&
           std::isfinite(p->w_rot) && std::isfinite(p->w_reg) && std::isfinite(p->w_data) &&
           p->precision >= MISSLAM_PREC_FP32 && p->precision <= MISSLAM_PREC_FP16 && p->refine_steps >= 0 &&
           (p->solve_launch == MISSLAM_LAUNCH_PLAIN || p->solve_launch == MISSLAM_LAUNCH_COOPERATIVE ||
            p->solve_launch == MISSLAM_LAUNCH_KERNELS) &&
           p->sync_spin_limit >= 0 && (p->solve_form == MISSLAM_SOLVE_PIPELINED || p->solve_form == MISSLAM_SOLVE_TEXTBOOK) &&
           p->asm_waves >= 0 && p->asm_waves <= 2;
}

bool valid_points(const misslam_points *p) {
    return p && p->n >= 0 && p->n <= p->capacity && p->n < (int64_t)1 << 31 &&
           (p->n == 0 || (p->px && p->py && p->pz && p->nx && p->ny && p->nz));
}

bool valid_nodes(const misslam_nodes *nd) {
    return nd && nd->m >= 1 && nd->m <= nd->capacity && nd->m < 65535 && nd->gx && nd->gy && nd->gz && nd->params;
}

bool valid_graph(const misslam_graph *g, int64_t n) {
    return g && g->k >= 1 && g->k <= MISSLAM_MAX_K && g->bsr_cap >= 1 && g->row_ptr && g->col_idx && g->info &&
           g->list_ptr && (n == 0 || (g->knn_idx && g->knn_w && g->list_pts && g->list_key));
}

bool valid_camera(const misslam_camera *c) {
    return c && c->width >= 1 && c->height >= 1 && std::isfinite(c->fx) && std::isfinite(c->fy) && c->fx != 0.f &&
           c->fy != 0.f && std::isfinite(c->cx) && std::isfinite(c->cy);
}

msl::PointsView view(const misslam_points *p) {
    return msl::PointsView{p->px, p->py, p->pz, p->nx, p->ny, p->nz, p->n};
}
msl::NodesView view(const misslam_nodes *nd) { return msl::NodesView{nd->gx, nd->gy, nd->gz, nd->params, nd->m}; }
msl::GraphView view(const misslam_graph *g) {
    return msl::GraphView{g->k,        g->bsr_cap,  g->knn_idx,  g->knn_w, g->row_ptr,
                          g->col_idx,  g->list_ptr, g->list_pts, reinterpret_cast<uint32_t *>(g->list_key), g->info};
}
msl::Cam view(const misslam_camera *c) { return msl::Cam{c->width, c->height, c->fx, c->fy, c->cx, c->cy}; }
msl::Pose view(const misslam_pose *p) {
    msl::Pose P;
    std::memcpy(P.R, p->R, sizeof(P.R));
    std::memcpy(P.T, p->T, sizeof(P.T));
    return P;
}

hipStream_t stream_of(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

void misslam_default_params(misslam_params *p) {
    if (!p) return;
    p->k = 4;
    p->weight_kind = MISSLAM_WEIGHT_GAUSS;
    p->sigma = 1.0f;
    p->w_rot = 1000.0f;
    p->w_reg = 10000.0f;
    p->w_data = 1.0f;
    p->eps_d = 15.0;
    p->cos_eps_n = std::cos(10.0 * 3.14159265358979323846 / 180.0);
    p->lambda = 1e-3f;
    p->gn_iters = 10;
    p->pcg_iters = 10;
    p->precision = MISSLAM_PREC_FP32;
    p->refine_steps = 0;
    p->reject_threshold = 0.0f;
    p->solve_launch = MISSLAM_LAUNCH_PLAIN;
    p->sync_spin_limit = 0;
    p->solve_form = MISSLAM_SOLVE_TEXTBOOK;
    p->asm_waves = 0;
}

const char *misslam_status_string(int32_t s) {
    switch (s) {
        case MISSLAM_OK: return "ok";
        case MISSLAM_EINVAL: return "invalid argument";
        case MISSLAM_ESHAPE: return "inconsistent sizes";
        case MISSLAM_EWORKSPACE: return "workspace too small";
        case MISSLAM_EHIP: return "HIP runtime error";
        case MISSLAM_ECAPACITY: return "capacity too small";
        case MISSLAM_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

int32_t misslam_last_hip_error(void) { return g_last_hip; }

size_t misslam_workspace_bytes(int64_t n, int32_t m, int32_t width, int32_t height, const misslam_params *params) {
    if (n < 0 || m < 1 || width < 1 || height < 1 || !valid_params(params)) return 0;
    return carve(nullptr, n, m, width, height, params->pcg_iters, params->k).bytes;
}

misslam_status misslam_normal_map(const float *depth, const misslam_camera *camera, float *out, void *stream) {
    if (!depth || !out || !valid_camera(camera)) return MISSLAM_EINVAL;
    Timed t(PH_NORMAL_MAP, stream_of(stream));
    const hipError_t e = msl::launch_normal_map(depth, view(camera), reinterpret_cast<float4 *>(out), stream_of(stream));
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_build_graph(const misslam_points *points, const misslam_nodes *nodes,
                                   const misslam_params *params, misslam_graph *graph, void *ws, size_t ws_bytes,
                                   void *stream) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_params(params) || !valid_graph(graph, points->n) || !ws)
        return MISSLAM_EINVAL;
    if (graph->k != params->k || nodes->m < params->k) return MISSLAM_ESHAPE;
    const Layout L = carve(ws, points->n, nodes->m, 1, 1, params->pcg_iters, params->k);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    Timed t(PH_GRAPH, stream_of(stream));
    const hipError_t e = msl::launch_build_graph(view(points), view(nodes), params->k, params->weight_kind,
                                                 params->sigma, view(graph), L.graph, stream_of(stream));
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_warp(const misslam_points *points, const misslam_nodes *nodes, const misslam_graph *graph,
                            const misslam_pose *pose, float *out_pos, float *out_nrm, void *stream) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !out_pos)
        return MISSLAM_EINVAL;
    msl::Pose P{};
    if (pose) P = view(pose);
    const hipError_t e = msl::launch_warp(view(points), view(nodes), view(graph), pose ? &P : nullptr, out_pos,
                                          out_nrm, stream_of(stream));
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

// The point pass, the assembly (and the key-point rows), then the step's energy report.  With defer set the
// report is not launched: its arguments go to *defer for the solve that follows, which forms it in an extra
// workgroup (or launches it when it cannot), and the assembly clears the solve's sync area (zero_words).
static hipError_t linearize(const msl::StepArgs &a0, const msl::StepScratch &s, int64_t n, int m,
                            misslam_report *rep, float reject, hipStream_t st, unsigned *zero_words = nullptr,
                            int zero_count = 0, const msl::KeyArgs *kp = nullptr,
                            const msl::CorrScratch *corr = nullptr, msl::ReportArgs *defer = nullptr) {
    hipError_t e;
    const bool keys = kp && corr && kp->count > 0;
    msl::StepArgs a = a0;
    if (defer) {
        a.zero_words = zero_words;
        a.zero_count = zero_count;
    }
    {
        Timed t(PH_POINT_PASS, st);
        e = msl::launch_point_pass(a, s, st, keys ? kp : nullptr, keys ? corr : nullptr);
    }
    if (e == hipSuccess) {
        Timed t(PH_ASSEMBLE, st);
        e = msl::launch_assemble(a, s, st);
    }
    if (e == hipSuccess && keys) {
        Timed t(PH_CORR, st);
        e = msl::launch_corr_rows(a, *kp, *corr, st);
    }
    if (e == hipSuccess && defer) {
        msl::report_args(s, n, m, rep, reject, keys ? corr->kp_energy : nullptr, keys ? kp->count : 0, *defer);
        return e;
    }
    if (e == hipSuccess) {
        Timed t(PH_ENERGY, st);
        e = msl::launch_energy_report(s, n, m, rep, reject, st, zero_words, zero_count,
                                      keys ? corr->kp_energy : nullptr, keys ? kp->count : 0);
    }
    return e;
}

// The one-launch persistent solve where the device holds its grid, else the
// multi-kernel recurrence: the same arithmetic, with reductions added in a
// different (but in each path fixed) order, so the two agree to rounding.
static hipError_t solve_persistent(const msl::GraphView &g, int m, const float *blocks, const float *gvec,
                                   const float *minv, float lambda, int iters, float *delta, const msl::PcgScratch &s,
                                   misslam_report *rep, float *params, hipStream_t st, bool coop,
                                   int zeroed_words = 0, const float *lambda_dev = nullptr, bool kernels = false,
                                   unsigned spin = 0, bool textbook = false,
                                   const msl::ReportArgs *report = nullptr) {
    bool used = false;
    hipError_t e = kernels ? hipSuccess
                           : msl::launch_pcg_persistent(g, m, blocks, gvec, minv, lambda, iters, delta, s, rep,
                                                        params, st, &used, coop, zeroed_words, lambda_dev, spin,
                                                        textbook, report);
    if (e == hipSuccess && !used) {
        if (report && report->rep) e = msl::launch_energy_report(*report, st);   // not formed by a solve workgroup
        if (e == hipSuccess)
            e = msl::launch_pcg_update(g, m, blocks, gvec, minv, lambda, iters, delta, s, rep, params, st,
                                       lambda_dev);
    }
    return e;
}

static hipError_t solve(const msl::GraphView &g, int m, const float *blocks, const float *gvec, float *minv,
                        float lambda, int iters, float *delta, const msl::PcgScratch &s, misslam_report *rep,
                        float *params, hipStream_t st, bool coop, bool kernels = false, unsigned spin = 0,
                        bool textbook = false) {
    hipError_t e;
    {
        Timed t(PH_BJACOBI, st);
        e = msl::launch_bjacobi(g, m, blocks, lambda, minv, &rep->flags, st);
    }
    if (e == hipSuccess) {
        Timed t(PH_PCG, st);
        e = solve_persistent(g, m, blocks, gvec, minv, lambda, iters, delta, s, rep, params, st, coop, 0, nullptr,
                             kernels, spin, textbook);
    }
    return e;
}


static msl::StepArgs step_args(const misslam_points *points, const misslam_nodes *nodes, const misslam_graph *graph,
                               const float4 *nmap, const misslam_camera *camera, const misslam_pose *pose,
                               const misslam_params *params, float *blocks, float *g, int32_t *corr) {
    msl::StepArgs a;
    a.pts = view(points);
    a.nd = view(nodes);
    a.g = view(graph);
    a.nmap = nmap;
    a.cam = view(camera);
    a.pose = view(pose);
    a.eps_d = params->eps_d;
    a.cos_eps_n = params->cos_eps_n;
    a.w_rot = params->w_rot;
    a.w_reg = params->w_reg;
    a.w_data = params->w_data;
    a.lambda = params->lambda;
    a.blocks = blocks;
    a.gvec = g;
    a.corr_out = corr;
    a.corr_in = nullptr;
    a.minv = nullptr;
    a.flags = nullptr;
    a.asm_waves = params->asm_waves == 1 ? 1 : 2;
    return a;
}

misslam_status misslam_build_normal_eq(const misslam_points *points, const misslam_nodes *nodes,
                                       const misslam_graph *graph, const float *nmap, const misslam_camera *camera,
                                       const misslam_pose *pose, const misslam_params *params, float *blocks, float *g,
                                       int32_t *corr, misslam_report *rep, void *ws, size_t ws_bytes, void *stream) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !nmap ||
        !valid_camera(camera) || !pose || !valid_params(params) || !blocks || !g || !rep || !ws)
        return MISSLAM_EINVAL;
    if (graph->k != params->k) return MISSLAM_ESHAPE;
    if (params->precision != MISSLAM_PREC_FP32 && params->k > 4) return MISSLAM_EUNSUPPORTED;
    const Layout L = carve(ws, points->n, nodes->m, camera->width, camera->height, params->pcg_iters, params->k);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    const hipStream_t st = stream_of(stream);
    const msl::StepArgs a = step_args(points, nodes, graph, reinterpret_cast<const float4 *>(nmap), camera, pose,
                                      params, blocks, g, corr);
    hipError_t e = msl::launch_report_init(rep, 1, st);
    if (e == hipSuccess && params->precision != MISSLAM_PREC_FP32) {
        e = msl::launch_point_pass(a, L.step, st);
        if (e == hipSuccess) e = msl::launch_assemble_lp(a, L.step, params->precision, nullptr, st);
        if (e == hipSuccess) e = msl::launch_energy_report(L.step, points->n, nodes->m, rep, params->reject_threshold, st);
        return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
    }
    if (e == hipSuccess) e = msl::launch_list_pack(a, L.step, st);
    if (e == hipSuccess) e = linearize(a, L.step, points->n, nodes->m, rep, params->reject_threshold, st);
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_pcg_solve(const misslam_graph *graph, int32_t m, const float *blocks, const float *g,
                                 const misslam_params *params, float *delta, misslam_report *rep, void *ws,
                                 size_t ws_bytes, void *stream) {
    if (!graph || !graph->row_ptr || !graph->col_idx || m < 1 || m >= 65535 || !blocks || !g ||
        !valid_params(params) || !delta || !rep || !ws)
        return MISSLAM_EINVAL;
    const Layout L = carve(ws, 0, m, 1, 1, params->pcg_iters, params->k);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    const hipStream_t st = stream_of(stream);
    const msl::GraphView gv = view(graph);
    hipError_t e = msl::launch_report_init(rep, 1, st);
    if (e == hipSuccess)
        e = solve(gv, m, blocks, g, L.step.minv, params->lambda, params->pcg_iters, delta, L.pcg, rep, nullptr, st,
                  params->solve_launch == MISSLAM_LAUNCH_COOPERATIVE,
                  params->solve_launch == MISSLAM_LAUNCH_KERNELS, (unsigned)params->sync_spin_limit,
                  params->solve_form == MISSLAM_SOLVE_TEXTBOOK);
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

static misslam_status gn_register(const misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                  const float *depth, const misslam_camera *camera, const misslam_pose *pose,
                                  const misslam_params *params, const misslam_keypoints *keys,
                                  const misslam_lm_params *lm, misslam_report *rep, int32_t *corr_hist, void *ws,
                                  size_t ws_bytes, void *stream, const misslam_pose_weights *pw = nullptr,
                                  float *pose_out = nullptr, bool core_only = false) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !depth ||
        !valid_camera(camera) || !pose || !valid_params(params) || !rep || !ws)
        return MISSLAM_EINVAL;
    if (keys && (keys->count < 0 || keys->count > points->n || keys->count > MISSLAM_MAX_KEYPOINTS || (keys->count > 0 && (!keys->point || !keys->target)) ||
                 !std::isfinite(keys->w_corr) || keys->w_corr < 0.f))
        return MISSLAM_EINVAL;
    if (graph->k != params->k) return MISSLAM_ESHAPE;
    if (params->precision != MISSLAM_PREC_FP32 && params->k > 4) return MISSLAM_EUNSUPPORTED;
    if (params->precision != MISSLAM_PREC_FP32 && keys && keys->count > 0) return MISSLAM_EUNSUPPORTED;
    if (params->precision != MISSLAM_PREC_FP32 && lm) return MISSLAM_EUNSUPPORTED;
    if (pw && (params->precision != MISSLAM_PREC_FP32 || lm)) return MISSLAM_EUNSUPPORTED;
    msl::KeyArgs ka{};
    const msl::KeyArgs *kp = nullptr;
    if (keys && keys->count > 0) {
        ka.count = keys->count;
        ka.w_corr = keys->w_corr;
        ka.point = keys->point;
        ka.target = keys->target;
        kp = &ka;
    }
    if (core_only && (params->precision != MISSLAM_PREC_FP32 || kp || lm || pw)) return MISSLAM_EUNSUPPORTED;
    const Layout L = carve(ws, points->n, nodes->m, camera->width, camera->height, params->pcg_iters, params->k,
                           core_only ? WS_CORE : WS_ALL);
    if (ws_bytes < L.bytes) return core_only ? MISSLAM_ECAPACITY : MISSLAM_EWORKSPACE;
    if ((int64_t)graph->bsr_cap > (int64_t)nodes->m * MISSLAM_MAX_ROW) return MISSLAM_ECAPACITY;
    const bool lowp = params->precision != MISSLAM_PREC_FP32;
    const bool coop = params->solve_launch == MISSLAM_LAUNCH_COOPERATIVE;
    const bool kernels = params->solve_launch == MISSLAM_LAUNCH_KERNELS;
    const hipStream_t st = stream_of(stream);
    const int G = params->gn_iters;
    const int64_t n = points->n;
    const int m = nodes->m;
    const unsigned spin = (unsigned)params->sync_spin_limit;
    const bool textbook = params->solve_form == MISSLAM_SOLVE_TEXTBOOK;
    hipError_t e = msl::launch_report_init(rep, G + 1, st, graph->info);
    if (e == hipSuccess && lowp) e = msl::launch_report_init(L.rep, 1, st);
    if (e == hipSuccess && lm) e = msl::launch_lm_init(L.lm_lambda, lm->lambda0, st);
    if (e == hipSuccess && lm) e = msl::launch_report_init(L.rep, 1, st);
    msl::PosePrior prior{};
    if (pw) {
        for (int t = 0; t < 9; ++t) prior.R0[t] = pose->R[t];
        for (int t = 0; t < 3; ++t) prior.T0[t] = pose->T[t];
        prior.w_r = pw->w_r;
        prior.w_p = pw->w_p;
        prior.w_data = params->w_data;
        if (e == hipSuccess) e = msl::launch_pose_init(view(pose), pose_out, st);
    }
    if (e == hipSuccess) {
        Timed t(PH_NORMAL_MAP, st);
        e = msl::launch_normal_map(depth, view(camera), L.nmap, st);
    }
    if (e == hipSuccess && kp)
        e = msl::launch_kp_nodes(step_args(points, nodes, graph, L.nmap, camera, pose, params, L.blocks, L.gvec,
                                           nullptr),
                                 *kp, L.corr.kp_nodes, st);
    if (e == hipSuccess && !lowp && G > 0) {
        Timed t(PH_LIST_PACK, st);
        e = msl::launch_list_pack(step_args(points, nodes, graph, L.nmap, camera, pose, params, L.blocks, L.gvec,
                                            nullptr),
                                  L.step, st);
    }
    for (int it = 0; it <= G && e == hipSuccess; ++it) {
        int32_t *corr = (corr_hist && it < G) ? corr_hist + (size_t)it * n : nullptr;
        msl::StepArgs a = step_args(points, nodes, graph, L.nmap, camera, pose, params, L.blocks, L.gvec, corr);
        if (it < G) {
            a.minv = L.step.minv;     // block-Jacobi inverses come out of the assembly
            a.flags = &rep[it].flags;
        }
        if (pw) {   // joint pose + ED: the pose lives on the device
            a.pose_dev = pose_out;
            const bool keys = kp && kp->count > 0;
            {
                Timed t(PH_POINT_PASS, st);
                e = msl::launch_point_pass_joint(a, L.step, st, keys ? kp : nullptr, keys ? &L.corr : nullptr);
            }
            if (it == G) {
                if (e == hipSuccess) e = msl::launch_node_energy(a, L.step, st);
                if (e == hipSuccess)
                    e = msl::launch_energy_report(L.step, n, m, rep + it, params->reject_threshold, st, nullptr, 0,
                                                  keys ? L.corr.kp_energy : nullptr, keys ? kp->count : 0);
                if (e == hipSuccess)
                    e = msl::launch_pose_setup(pose_out, prior, L.step.pose_part, msl::point_blocks(n), params->lambda,
                                               nullptr, rep + it, st);
                break;
            }
            if (e == hipSuccess) {
                Timed t(PH_ASSEMBLE, st);
                e = msl::launch_assemble(a, L.step, st);
            }
            if (e == hipSuccess) {
                Timed t(PH_POSE, st);
                e = msl::launch_border_rows(a, L.step, L.joint.B, st);
            }
            if (e == hipSuccess && keys) {   // Eq.(9): ED rows and blocks, and its part of the border
                Timed t(PH_CORR, st);
                e = msl::launch_corr_rows(a, *kp, L.corr, st, L.joint.B);
            }
            if (e == hipSuccess)
                e = msl::launch_energy_report(L.step, n, m, rep + it, params->reject_threshold, st, nullptr, 0,
                                              keys ? L.corr.kp_energy : nullptr, keys ? kp->count : 0);
            if (e == hipSuccess)
                e = msl::launch_pose_setup(pose_out, prior, L.step.pose_part, msl::point_blocks(n), params->lambda,
                                           L.joint.sys, rep + it, st, L.joint.jbar, m, keys ? kp : nullptr,
                                           keys ? &L.corr : nullptr, n, params->k);
            if (e == hipSuccess) {
                Timed t(PH_PCG, st);
                e = msl::launch_joint_pcg(view(graph), m, L.blocks, L.gvec, L.step.minv, params->lambda,
                                          params->pcg_iters, L.delta, L.pcg, L.joint, rep + it, nodes->params,
                                          pose_out, st, kernels, spin);
            }
            continue;
        }
        if (it == G) {   // final entry: energies at the returned parameters, no system needed
            const bool keys = kp && kp->count > 0;
            {
                Timed t(PH_POINT_PASS, st);
                e = msl::launch_point_pass(a, L.step, st, keys ? kp : nullptr, keys ? &L.corr : nullptr);
            }
            if (e == hipSuccess) e = msl::launch_node_energy(a, L.step, st);
            if (e == hipSuccess)
                e = msl::launch_energy_report(L.step, n, m, rep + it, params->reject_threshold, st, nullptr, 0,
                                              keys ? L.corr.kp_energy : nullptr, keys ? kp->count : 0);
            break;
        }
        if (!lowp) {
            if (lm) a.lambda_dev = L.lm_lambda;
            msl::ReportArgs ra;   // the step's report, formed by the solve's extra workgroup
            e = linearize(a, L.step, n, m, rep + it, params->reject_threshold, st, L.pcg.bar, msl::msl_sync_words(m),
                          kp, &L.corr, &ra);
            if (e == hipSuccess) {
                Timed t(PH_PCG, st);
                e = solve_persistent(view(graph), m, L.blocks, L.gvec, L.step.minv, params->lambda, params->pcg_iters,
                                     L.delta, L.pcg, rep + it, lm ? nullptr : nodes->params, st, coop,
                                     msl::msl_sync_words(m), lm ? L.lm_lambda : nullptr, kernels, spin, textbook,
                                     &ra);
            }
            if (e == hipSuccess && lm) {
                // the trial point x + dx: its objective decides whether the step is taken
                Timed t(PH_LM, st);
                float *xt = L.delta2;
                const bool keys = kp && kp->count > 0;
                e = msl::launch_lm_trial(nodes->params, L.delta, xt, 12 * m, st);
                msl::StepArgs at = step_args(points, nodes, graph, L.nmap, camera, pose, params, L.blocks, L.gvec,
                                             nullptr);
                at.nd.x = xt;
                if (e == hipSuccess)
                    e = msl::launch_point_pass(at, L.step, st, keys ? kp : nullptr, keys ? &L.corr : nullptr);
                if (e == hipSuccess) e = msl::launch_node_energy(at, L.step, st);
                if (e == hipSuccess)
                    e = msl::launch_energy_report(L.step, n, m, L.rep, 0.f, st, nullptr, 0,
                                                  keys ? L.corr.kp_energy : nullptr, keys ? kp->count : 0);
                if (e == hipSuccess)
                    e = msl::launch_lm_decide(rep + it, L.rep, *lm, params->w_data, params->w_rot, params->w_reg,
                                              keys ? kp->w_corr : 0.f, nodes->params, xt, 12 * m, L.lm_lambda, st);
            }
            continue;
        }
        // low precision: H_lo from the matrix cores, then float32 refinement of the step.  The assembly and each
        // refinement's right-hand side clear the next solve's sync area, and the step's report is formed by the
        // first solve's extra workgroup (as in the float32 path).
        msl::StepArgs al = a;
        al.zero_words = L.pcg.bar;
        al.zero_count = msl::msl_sync_words(m);
        {
            Timed t(PH_POINT_PASS, st);
            e = msl::launch_point_pass(a, L.step, st);
        }
        if (e == hipSuccess) {
            Timed t(PH_ASSEMBLE, st);
            e = msl::launch_assemble_lp(al, L.step, params->precision, L.rr, st);
        }
        msl::ReportArgs ra;
        msl::report_args(L.step, n, m, rep + it, params->reject_threshold, nullptr, 0, ra);
        if (e == hipSuccess) {
            Timed t(PH_PCG, st);
            e = solve_persistent(view(graph), m, L.blocks, L.gvec, L.step.minv, params->lambda, params->pcg_iters,
                                 L.delta, L.pcg, rep + it, nullptr, st, coop, al.zero_count, nullptr, kernels, spin,
                                 textbook, &ra);
        }
        for (int r = 0; r < params->refine_steps && e == hipSuccess; ++r) {
            {
                Timed t(PH_REFINE, st);
                e = msl::launch_refine_rhs(al, L.step, L.delta, L.rr, L.gvec, L.jv, L.rhs, st);
            }
            if (e == hipSuccess) e = msl::launch_report_init(L.rep, 1, st);
            if (e == hipSuccess) {
                Timed t(PH_PCG, st);
                e = solve_persistent(view(graph), m, L.blocks, L.rhs, L.step.minv, params->lambda, params->pcg_iters,
                                     L.delta2, L.pcg, L.rep, nullptr, st, coop, al.zero_count, nullptr, kernels,
                                     spin, textbook);
            }
            // dx += the correction unless its solve failed; its flags join the step's report
            if (e == hipSuccess) e = msl::launch_step_commit(L.delta, L.delta2, 12 * m, L.rep, st, rep + it);
        }
        // x += dx unless the step's report (its own solve's flags and every refinement's) rules it out
        if (e == hipSuccess) e = msl::launch_step_commit(nodes->params, L.delta, 12 * m, rep + it, st);
    }
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_gn_register(const misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                   const float *depth, const misslam_camera *camera, const misslam_pose *pose,
                                   const misslam_params *params, misslam_report *rep, int32_t *corr_hist, void *ws,
                                   size_t ws_bytes, void *stream) {
    return gn_register(points, nodes, graph, depth, camera, pose, params, nullptr, nullptr, rep, corr_hist, ws,
                       ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free registration

namespace {

// Scratch of misslam_gn_register_noalloc.  Each device holds its own copy from
// the library's load until the process ends.  Host code never uses the name as
// an address: the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[MISSLAM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct ScratchTable {
    std::mutex mu;
    void *ptr[kMaxDevices] = {};
};

ScratchTable &scratch_table() {
    static ScratchTable t;
    return t;
}

// The current device's address of the scratch array, looked up on the first call on that device.
hipError_t scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        t.ptr[dev] = p;
    }
    *out = t.ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

misslam_status misslam_gn_register_noalloc(const misslam_points *points, misslam_nodes *nodes,
                                           const misslam_graph *graph, const float *depth,
                                           const misslam_camera *camera, const misslam_pose *pose,
                                           const misslam_params *params, misslam_report *rep, int32_t *corr_hist,
                                           void *stream) {
    // every size check first, before any HIP call
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !depth ||
        !valid_camera(camera) || !pose || !valid_params(params) || !rep)
        return MISSLAM_EINVAL;
    if (params->precision != MISSLAM_PREC_FP32) return MISSLAM_EUNSUPPORTED;
    if (carve(nullptr, points->n, nodes->m, camera->width, camera->height, params->pcg_iters, params->k, WS_CORE)
            .bytes > (size_t)MISSLAM_NOALLOC_SCRATCH_BYTES)
        return MISSLAM_ECAPACITY;
    void *ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return hip_fail(e);
    tl_no_events = true;
    const misslam_status st = gn_register(points, nodes, graph, depth, camera, pose, params, nullptr, nullptr, rep,
                                          corr_hist, ws, (size_t)MISSLAM_NOALLOC_SCRATCH_BYTES, stream, nullptr,
                                          nullptr, true);
    tl_no_events = false;
    return st;
}

misslam_status misslam_gn_register_keypoints(const misslam_points *points, misslam_nodes *nodes,
                                             const misslam_graph *graph, const float *depth,
                                             const misslam_camera *camera, const misslam_pose *pose,
                                             const misslam_params *params, const misslam_keypoints *keys,
                                             misslam_report *rep, int32_t *corr_hist, void *ws, size_t ws_bytes,
                                             void *stream) {
    if (!keys) return MISSLAM_EINVAL;
    return gn_register(points, nodes, graph, depth, camera, pose, params, keys, nullptr, rep, corr_hist, ws,
                       ws_bytes, stream);
}

void misslam_default_lm_params(misslam_lm_params *lm) {
    if (!lm) return;
    lm->lambda0 = 1e-3f;
    lm->up = 10.f;
    lm->down = 0.1f;
    lm->lambda_min = 1e-6f;
    lm->lambda_max = 1e6f;
}

misslam_status misslam_joint_register(const misslam_points *points, misslam_nodes *nodes,
                                      const misslam_graph *graph, const float *depth,
                                      const misslam_camera *camera, const misslam_pose *pose,
                                      const misslam_pose_weights *pw, const misslam_keypoints *keys,
                                      const misslam_params *params, float *pose_out, misslam_report *rep,
                                      int32_t *corr_hist, void *ws, size_t ws_bytes, void *stream) {
    if (!pw || !pose_out || !pose || !std::isfinite(pw->w_r) || !std::isfinite(pw->w_p) || !(pw->w_r >= 0.f) ||
        !(pw->w_p >= 0.f))
        return MISSLAM_EINVAL;
    return gn_register(points, nodes, graph, depth, camera, pose, params, keys, nullptr, rep, corr_hist, ws,
                       ws_bytes, stream, pw, pose_out);
}

misslam_status misslam_lm_register(const misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                   const float *depth, const misslam_camera *camera, const misslam_pose *pose,
                                   const misslam_params *params, const misslam_keypoints *keys,
                                   const misslam_lm_params *lm, misslam_report *rep, int32_t *corr_hist, void *ws,
                                   size_t ws_bytes, void *stream) {
    if (!lm || !std::isfinite(lm->lambda0) || !std::isfinite(lm->up) || !std::isfinite(lm->down) ||
        !std::isfinite(lm->lambda_min) || !std::isfinite(lm->lambda_max) || !(lm->lambda_min >= 0.f) ||
        !(lm->lambda0 >= lm->lambda_min) || !(lm->lambda_max >= lm->lambda0) || !(lm->up >= 1.f) ||
        !(lm->down > 0.f) || !(lm->down <= 1.f))
        return MISSLAM_EINVAL;
    return gn_register(points, nodes, graph, depth, camera, pose, params, keys, lm, rep, corr_hist, ws, ws_bytes,
                       stream);
}

static misslam_status fuse_impl(misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                const float *nmap, const misslam_camera *camera, const misslam_pose *pose,
                                const misslam_fuse_params *fp, const float *image, float *color,
                                int64_t color_stride, int32_t *reg_map, int32_t *registered, void *ws,
                                size_t ws_bytes, void *stream) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !nmap ||
        !valid_camera(camera) || !pose || !fp || !ws || (points->n > 0 && (!points->w || !points->stamp)) ||
        !std::isfinite(fp->tau) || !std::isfinite(fp->cos_delta) || !(fp->w_max > 0.f))
        return MISSLAM_EINVAL;
    misslam_params dp;
    misslam_default_params(&dp);
    const Layout L = carve(ws, points->n, nodes->m, camera->width, camera->height, dp.pcg_iters, graph->k);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    msl::FuseArgs f;
    f.pts = view(points);
    f.nd = view(nodes);
    f.g = view(graph);
    f.nmap = reinterpret_cast<const float4 *>(nmap);
    f.cam = view(camera);
    f.pose = view(pose);
    for (int t = 0; t < 9; ++t) f.Rd[t] = pose->R[t];
    for (int t = 0; t < 3; ++t) f.Td[t] = pose->T[t];
    f.tau = fp->tau;
    f.cos_delta = fp->cos_delta;
    f.w_max = fp->w_max;
    f.frame = fp->frame;
    f.w_in = points->w;
    f.stamp_in = points->stamp;
    f.out_px = points->px;
    f.out_py = points->py;
    f.out_pz = points->pz;
    f.out_nx = points->nx;
    f.out_ny = points->ny;
    f.out_nz = points->nz;
    f.out_w = points->w;
    f.out_stamp = points->stamp;
    f.registered = registered;
    f.tmp = L.fuse_tmp;
    f.pix = L.fuse_pix;
    f.zbuf = L.zbuf;
    f.image = image;
    f.color = color;
    f.color_stride = color_stride;
    Timed t(PH_FUSE, stream_of(stream));
    const hipError_t e = msl::launch_fuse(f, nodes->gx, nodes->gy, nodes->gz, nodes->params, nodes->m, reg_map,
                                          stream_of(stream));
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_fuse(misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                            const float *nmap, const misslam_camera *camera, const misslam_pose *pose,
                            const misslam_fuse_params *fp, int32_t *reg_map, int32_t *registered, void *ws,
                            size_t ws_bytes, void *stream) {
    return fuse_impl(points, nodes, graph, nmap, camera, pose, fp, nullptr, nullptr, 0, reg_map, registered, ws,
                     ws_bytes, stream);
}

misslam_status misslam_fuse_color(misslam_points *points, misslam_nodes *nodes, const misslam_graph *graph,
                                  const float *nmap, const misslam_camera *camera, const misslam_pose *pose,
                                  const misslam_fuse_params *fp, const float *image, float *color,
                                  int64_t color_stride, int32_t *reg_map, int32_t *registered, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (points && points->n > 0 && (!image || !color || color_stride < points->n)) return MISSLAM_EINVAL;
    return fuse_impl(points, nodes, graph, nmap, camera, pose, fp, image, color, color_stride, reg_map, registered,
                     ws, ws_bytes, stream);
}

misslam_status misslam_energy_vjp(const misslam_points *points, const misslam_nodes *nodes,
                                  const misslam_graph *graph, const float *nmap, const misslam_camera *camera,
                                  const misslam_pose *pose, const misslam_params *params, const int32_t *corr_in,
                                  int32_t *corr_out, const float *grad_e, float *grad_params, float *grad_points,
                                  double *energy, misslam_report *rep, void *ws, size_t ws_bytes, void *stream) {
    if (!valid_points(points) || !valid_nodes(nodes) || !valid_graph(graph, points->n) || !nmap ||
        !valid_camera(camera) || !pose || !valid_params(params) || !ws)
        return MISSLAM_EINVAL;
    if (graph->k != params->k) return MISSLAM_ESHAPE;
    if (grad_points && params->weight_kind != MISSLAM_WEIGHT_GAUSS) return MISSLAM_EUNSUPPORTED;
    const Layout L = carve(ws, points->n, nodes->m, camera->width, camera->height, params->pcg_iters, params->k);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    if ((int64_t)graph->bsr_cap > (int64_t)nodes->m * MISSLAM_MAX_ROW) return MISSLAM_ECAPACITY;
    const hipStream_t st = stream_of(stream);
    misslam_report *r = rep ? rep : L.rep;
    msl::StepArgs a = step_args(points, nodes, graph, reinterpret_cast<const float4 *>(nmap), camera, pose, params,
                                L.blocks, L.gvec, corr_out);
    a.corr_in = corr_in;
    hipError_t e = msl::launch_report_init(r, 1, st);
    if (e == hipSuccess) e = msl::launch_point_pass(a, L.step, st);
    if (e == hipSuccess && grad_params) e = msl::launch_list_pack(a, L.step, st);
    if (e == hipSuccess) e = grad_params ? msl::launch_assemble(a, L.step, st) : msl::launch_node_energy(a, L.step, st);
    if (e == hipSuccess) e = msl::launch_energy_report(L.step, points->n, nodes->m, r, params->reject_threshold, st);
    if (e == hipSuccess && energy)
        e = msl::launch_energy_total(r, params->w_data, params->w_rot, params->w_reg, energy, st);
    if (e == hipSuccess && grad_params) e = msl::launch_grad_params(L.gvec, nodes->m, grad_e, grad_params, st);
    if (e == hipSuccess && grad_points) e = msl::launch_vjp_points(a, L.step, params->sigma, grad_e, grad_points, st);
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

int32_t misslam_profile_enable(int32_t on) {
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    const int32_t was = p.on;
    p.on = on != 0;
    return was;
}

misslam_status misslam_profile_get(const char *phase, double *total_ms, int64_t *launches) {
    if (!phase || !total_ms || !launches) return MISSLAM_EINVAL;
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    for (int i = 0; i < PH_COUNT; ++i)
        if (std::strcmp(phase, kPhaseNames[i]) == 0) {
            p.collect();
            *total_ms = p.total_ms[i];
            *launches = p.launches[i];
            return MISSLAM_OK;
        }
    return MISSLAM_EINVAL;
}

void misslam_profile_reset(void) {
    Profiler &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    p.collect();
    for (int i = 0; i < PH_COUNT; ++i) {
        p.total_ms[i] = 0.0;
        p.launches[i] = 0;
    }
}

}  // extern "C"

// ------------------------------------------------------------------ growth and maintenance

namespace {

struct GrowLayout {
    msl::GrowScratch s;
    float *stage;
    int32_t *stage_stamp;
    float *stage_color;
    uint8_t *stage_stable;
    size_t bytes;
};

GrowLayout carve_grow(void *ws, int64_t n, int32_t W, int32_t H) {
    Carver c{static_cast<char *>(ws)};
    GrowLayout L{};
    const int64_t C = n + (int64_t)W * H;
    const int64_t Cb = C > 0 ? C : 1;
    const int64_t nb = (Cb + 255) / 256;
    L.stage = c.take<float>((size_t)7 * Cb);
    L.stage_stamp = c.take<int32_t>((size_t)Cb);
    L.s.flags = c.take<int32_t>((size_t)Cb);
    L.s.alive = c.take<int32_t>((size_t)Cb);
    L.s.bcount = c.take<int32_t>((size_t)nb);
    L.s.boffs = c.take<int32_t>((size_t)nb);
    L.s.bcount2 = c.take<int32_t>((size_t)nb);
    L.s.boffs2 = c.take<int32_t>((size_t)nb);
    L.s.count = c.take<int32_t>(8);
    L.s.hist = c.take<int32_t>((size_t)msl::grow_hist_entries(Cb));
    L.s.hoffs = c.take<int32_t>((size_t)msl::grow_hist_entries(Cb));
    L.s.k0 = c.take<unsigned long long>((size_t)Cb);
    L.s.k1 = c.take<unsigned long long>((size_t)Cb);
    L.s.v0 = c.take<uint32_t>((size_t)Cb);
    L.s.v1 = c.take<uint32_t>((size_t)Cb);
    L.s.cent = c.take<float>((size_t)3 * Cb);
    L.stage_color = c.take<float>((size_t)3 * Cb);
    L.stage_stable = c.take<uint8_t>((size_t)Cb);
    L.bytes = align_up(c.off);
    return L;
}

}  // namespace

extern "C" {

size_t misslam_grow_workspace_bytes(int64_t n, int32_t width, int32_t height) {
    if (n < 0 || width < 1 || height < 1) return 0;
    return carve_grow(nullptr, n, width, height).bytes;
}

static misslam_status grow_impl(misslam_points *points, misslam_nodes *nodes, const int32_t *reg_map,
                                const int32_t *registered, const float *nmap, const misslam_camera *camera,
                                const misslam_pose *pose, const misslam_grow_params *gp, const float *image,
                                float *color, int64_t color_stride, int64_t *counts_out, void *ws, size_t ws_bytes,
                                void *stream) {
    if (!points || points->n < 0 || points->n > points->capacity || !points->px || !points->py || !points->pz ||
        !points->nx || !points->ny || !points->nz || !points->w || !points->stamp || !nodes || nodes->m < 0 ||
        nodes->m > nodes->capacity || !nodes->gx || !nodes->gy || !nodes->gz || !nodes->params || !reg_map ||
        (points->n > 0 && !registered) || !nmap || !valid_camera(camera) || !pose || !gp || !counts_out || !ws)
        return MISSLAM_EINVAL;
    if (!(gp->voxel > 0.f) || !(gp->node_spacing > 0.f) || !std::isfinite(gp->tau_weight) || gp->tau_time < 0)
        return MISSLAM_EINVAL;
    const int64_t C = points->n + (int64_t)camera->width * camera->height;
    if (C >= (int64_t)1 << 31 || points->capacity >= (int64_t)1 << 31) return MISSLAM_ESHAPE;
    const GrowLayout L = carve_grow(ws, points->n, camera->width, camera->height);
    if (ws_bytes < L.bytes) return MISSLAM_EWORKSPACE;
    msl::GrowArgs g;
    g.px = points->px;
    g.py = points->py;
    g.pz = points->pz;
    g.nx = points->nx;
    g.ny = points->ny;
    g.nz = points->nz;
    g.w = points->w;
    g.stamp = points->stamp;
    g.n = points->n;
    g.capacity = points->capacity;
    g.gx = nodes->gx;
    g.gy = nodes->gy;
    g.gz = nodes->gz;
    g.params = nodes->params;
    g.m = nodes->m;
    g.node_capacity = nodes->capacity;
    g.reg_map = reg_map;
    g.registered = registered;
    g.nmap = reinterpret_cast<const float4 *>(nmap);
    g.cam = view(camera);
    for (int t = 0; t < 9; ++t) g.Rd[t] = pose->R[t];
    for (int t = 0; t < 3; ++t) g.Td[t] = pose->T[t];
    g.voxel = gp->voxel;
    g.node_spacing = gp->node_spacing;
    g.tau_weight = gp->tau_weight;
    g.tau_time = gp->tau_time;
    g.frame = gp->frame;
    g.stage = L.stage;
    g.stage_stamp = L.stage_stamp;
    g.stage_cap = C;
    g.count = L.s.count;
    g.image = image;
    g.color = color;
    g.color_stride = color_stride;
    g.stage_color = L.stage_color;
    g.stable = points->stable;
    g.stage_stable = L.stage_stable;
    const hipStream_t st = stream_of(stream);
    Timed t(PH_GROW, st);
    const hipError_t e = msl::launch_grow(g, L.s, counts_out, st);
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

misslam_status misslam_grow(misslam_points *points, misslam_nodes *nodes, const int32_t *reg_map,
                            const int32_t *registered, const float *nmap, const misslam_camera *camera,
                            const misslam_pose *pose, const misslam_grow_params *gp, int64_t *counts_out, void *ws,
                            size_t ws_bytes, void *stream) {
    return grow_impl(points, nodes, reg_map, registered, nmap, camera, pose, gp, nullptr, nullptr, 0, counts_out, ws,
                     ws_bytes, stream);
}

misslam_status misslam_grow_color(misslam_points *points, misslam_nodes *nodes, const int32_t *reg_map,
                                  const int32_t *registered, const float *nmap, const misslam_camera *camera,
                                  const misslam_pose *pose, const misslam_grow_params *gp, const float *image,
                                  float *color, int64_t color_stride, int64_t *counts_out, void *ws, size_t ws_bytes,
                                  void *stream) {
    if (!points || !image || !color || color_stride < points->capacity) return MISSLAM_EINVAL;
    return grow_impl(points, nodes, reg_map, registered, nmap, camera, pose, gp, image, color, color_stride,
                     counts_out, ws, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ uneven batches

struct misslam_batch {
    std::vector<misslam_problem> probs;
    misslam_params params;
    int count = 0;
    int req_rows = 0;          // 0: tune on the first call
    int rows = 0;              // tile in use
    int waves = 0;             // assembly tile in use (waves per node row)
    msl::BatchItem *d_items = nullptr;
    float *d_backup = nullptr; // params of every problem (tuning restores them)
    std::vector<size_t> param_off;
    std::vector<msl::BatchItem> items;
    void *items_ws = nullptr;  // workspace the items were carved from
    int items_rows = 0;
    int64_t total_pp = 0;
    int total_nm = 0, total_rows = 0, total_ne = 0, total_wgs = 0;
    unsigned *bar = nullptr;
    hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream, which cannot capture)
    hipGraphExec_t exec = nullptr;
    void *exec_ws = nullptr;
    int exec_rows = 0;
    int exec_waves = 0;
};

namespace {

size_t batch_bytes(const misslam_batch *b) {
    size_t off = align_up(msl::MSL_BAR_WORDS * sizeof(unsigned));
    for (const auto &p : b->probs)
        off += align_up(carve(nullptr, p.points.n, p.nodes.m, p.camera.width, p.camera.height, b->params.pcg_iters,
                              b->params.k).bytes);
    return off;
}

// Host descriptors of every problem for workspace ws and tile rows.
void batch_items(misslam_batch *b, void *ws, int rows) {
    char *base = static_cast<char *>(ws);
    b->bar = reinterpret_cast<unsigned *>(base);
    size_t off = align_up(msl::MSL_BAR_WORDS * sizeof(unsigned));
    b->items.assign(b->count, msl::BatchItem{});
    int64_t pp = 0;
    int nm = 0, row = 0, ne = 0, wg = 0;
    const int G = b->params.gn_iters;
    for (int i = 0; i < b->count; ++i) {
        const misslam_problem &p = b->probs[i];
        const Layout L = carve(base + off, p.points.n, p.nodes.m, p.camera.width, p.camera.height,
                               b->params.pcg_iters, b->params.k);
        off += align_up(L.bytes);
        msl::BatchItem &it = b->items[i];
        it.a = step_args(&p.points, &p.nodes, &p.graph, L.nmap, &p.camera, &p.pose, &b->params, L.blocks, L.gvec,
                         nullptr);
        it.a.minv = L.step.minv;
        it.s = L.step;
        const int m = p.nodes.m;
        const int wgs = (m + rows - 1) / rows;
        msl::PcgArgs &A = it.p;
        A.row_ptr = p.graph.row_ptr;
        A.col_idx = p.graph.col_idx;
        A.blocks = L.blocks;
        A.minv = L.step.minv;
        A.g = L.gvec;
        A.lambda = b->params.lambda;
        A.m = m;
        A.nblk = wgs;
        A.iters = b->params.pcg_iters;
        A.cap = p.graph.bsr_cap;
        A.x = L.delta;
        A.r = L.pcg.r;
        A.z = L.pcg.z;
        A.p = L.pcg.p;
        A.q = L.pcg.q;
        A.part = L.pcg.part;
        A.status = L.pcg.status;
        A.done = L.pcg.status + (b->params.pcg_iters + 2);
        if (b->params.sync_spin_limit > 0) A.spin = (unsigned)b->params.sync_spin_limit;
        A.halo[0] = L.pcg.halo;                       // the pipelined recurrence's exchanged vectors
        A.halo[1] = L.pcg.halo + (size_t)12 * m;
        A.textbook = b->params.solve_form == MISSLAM_SOLVE_TEXTBOOK;
        it.rep = p.report;
        it.params = p.nodes.params;
        it.depth = p.depth;
        it.reject = b->params.reject_threshold;
        const int64_t n = p.points.n;
        it.npb = (int)((n > 0 ? n + 255 : 256) / 256);   // as the single call: one block even for no points
        it.pp0 = pp;
        pp += it.npb;
        it.nm0 = nm;
        nm += (int)(((int64_t)p.camera.width * p.camera.height + 255) / 256);
        it.row0 = row;
        row += m;
        it.ne0 = ne;
        ne += (m + 255) / 256;
        it.wg0 = wg;
        it.wgs = wgs;
        wg += wgs;
        (void)G;
    }
    b->total_pp = pp;
    b->total_nm = nm;
    b->total_rows = row;
    b->total_ne = ne;
    b->total_wgs = wg;
}

// The frame of every problem, enqueued on st (eagerly or under capture).
hipError_t batch_enqueue(misslam_batch *b, hipStream_t st, bool cooperative) {
    const int G = b->params.gn_iters;
    const int count = b->count, k = b->params.k;
    const msl::BatchItem *d = b->d_items;
    hipError_t e = msl::launch_report_init_batched(d, count, G + 1, st);
    if (e == hipSuccess) e = msl::launch_normal_map_batched(d, count, b->total_nm, st);
    if (e == hipSuccess && G > 0) e = msl::launch_list_pack_batched(d, count, k, b->total_rows, st);
    for (int it = 0; it < G && e == hipSuccess; ++it) {
        e = msl::launch_point_pass_batched(d, count, k, b->total_pp, it, st);
        if (e == hipSuccess) e = msl::launch_assemble_batched(d, count, k, b->total_rows, it, b->waves, st);
        if (e == hipSuccess) e = msl::launch_energy_report_batched(d, count, it, b->bar,
                                                                   std::min(msl::MSL_WG_WORDS * b->total_wgs, msl::MSL_BAR_WORDS), st);
        bool used = false;
        if (e == hipSuccess)
            e = msl::launch_pcg_batched(d, count, b->rows, b->total_wgs, b->total_rows, it, b->bar,
                                        cooperative && b->params.solve_launch == MISSLAM_LAUNCH_COOPERATIVE, st, &used,
                                        b->params.solve_form == MISSLAM_SOLVE_TEXTBOOK);
        if (e == hipSuccess && !used) return hipErrorInvalidConfiguration;
    }
    if (e == hipSuccess) e = msl::launch_point_pass_batched(d, count, k, b->total_pp, G, st);
    if (e == hipSuccess) e = msl::launch_node_energy_batched(d, count, b->total_ne, st);
    if (e == hipSuccess) e = msl::launch_energy_report_batched(d, count, G, nullptr, 0, st);
    return e;
}

hipError_t batch_upload(misslam_batch *b, void *ws, int rows) {
    batch_items(b, ws, rows);
    b->items_ws = ws;
    b->items_rows = rows;
    return hipMemcpy(b->d_items, b->items.data(), sizeof(msl::BatchItem) * b->count, hipMemcpyHostToDevice);
}

hipError_t batch_save_params(misslam_batch *b, hipStream_t st, bool restore) {
    for (int i = 0; i < b->count; ++i) {
        const misslam_problem &p = b->probs[i];
        const size_t bytes = sizeof(float) * 12 * (size_t)p.nodes.m;
        float *dev = b->d_backup + b->param_off[i];
        const hipError_t e = restore ? hipMemcpyAsync(p.nodes.params, dev, bytes, hipMemcpyDeviceToDevice, st)
                                     : hipMemcpyAsync(dev, p.nodes.params, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Times one eager frame with tile rows (params restored afterwards); < 0 if the tile does not fit.
float batch_try(misslam_batch *b, void *ws, int rows, hipStream_t st) {
    int wgs = 0;
    for (const auto &p : b->probs) wgs += (p.nodes.m + rows - 1) / rows;
    if (!msl::pcg_batched_fits(wgs, b->params.solve_form == MISSLAM_SOLVE_TEXTBOOK)) return -1.f;
    // the descriptors are rewritten by a blocking copy: nothing queued on st may still read them
    if (hipStreamSynchronize(st) != hipSuccess) return -1.f;
    if (batch_upload(b, ws, rows) != hipSuccess) return -1.f;
    b->rows = rows;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = -1.f;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        bool ok = batch_enqueue(b, st, true) == hipSuccess;   // warm
        ok = ok && batch_save_params(b, st, true) == hipSuccess;
        ok = ok && hipEventRecord(e0, st) == hipSuccess;
        ok = ok && batch_enqueue(b, st, true) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess;
        ok = ok && batch_save_params(b, st, true) == hipSuccess;
        ok = ok && hipStreamSynchronize(st) == hipSuccess;
        if (ok && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.f;
        if (!ok) ms = -1.f;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return ms;
}

}  // namespace

extern "C" {

misslam_status misslam_batch_create(const misslam_problem *problems, int32_t count, const misslam_params *params,
                                    int32_t rows_per_wg, misslam_batch **out) {
    if (!problems || count < 1 || count > 1024 || !valid_params(params) || !out || rows_per_wg < 0 ||
        rows_per_wg > 21)
        return MISSLAM_EINVAL;
    if (params->precision != MISSLAM_PREC_FP32 || params->solve_launch == MISSLAM_LAUNCH_KERNELS)
        return MISSLAM_EUNSUPPORTED;
    for (int i = 0; i < count; ++i) {
        const misslam_problem &p = problems[i];
        if (!valid_points(&p.points) || !valid_nodes(&p.nodes) || !valid_graph(&p.graph, p.points.n) || !p.depth ||
            !valid_camera(&p.camera) || !p.report)
            return MISSLAM_EINVAL;
        if (p.graph.k != params->k) return MISSLAM_ESHAPE;
        if ((int64_t)p.graph.bsr_cap > (int64_t)p.nodes.m * MISSLAM_MAX_ROW) return MISSLAM_ECAPACITY;
    }
    misslam_batch *b = new misslam_batch();
    b->probs.assign(problems, problems + count);
    b->params = *params;
    b->count = count;
    b->req_rows = rows_per_wg;
    size_t poff = 0;
    for (int i = 0; i < count; ++i) {
        b->param_off.push_back(poff);
        poff += 12 * (size_t)problems[i].nodes.m;
    }
    hipError_t e = hipMalloc(&b->d_items, sizeof(msl::BatchItem) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_backup, sizeof(float) * (poff > 0 ? poff : 1));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        misslam_batch_destroy(b);
        return hip_fail(e);
    }
    *out = b;
    return MISSLAM_OK;
}

size_t misslam_batch_workspace_bytes(const misslam_batch *batch) { return batch ? batch_bytes(batch) : 0; }

int32_t misslam_batch_tile(const misslam_batch *batch) { return batch ? batch->rows : 0; }

int32_t misslam_batch_asm_waves(const misslam_batch *batch) { return batch && batch->rows ? batch->waves : 0; }

misslam_status misslam_batch_register(misslam_batch *b, void *ws, size_t ws_bytes, void *stream) {
    if (!b || !ws) return MISSLAM_EINVAL;
    if (ws_bytes < batch_bytes(b)) return MISSLAM_EWORKSPACE;
    const hipStream_t st = stream_of(stream);
    hipError_t e = hipSuccess;
    if (b->rows == 0) {
        const int req_waves = b->params.asm_waves;
        if (b->req_rows > 0) {
            int wgs = 0;
            for (const auto &p : b->probs) wgs += (p.nodes.m + b->req_rows - 1) / b->req_rows;
            if (!msl::pcg_batched_fits(wgs, b->params.solve_form == MISSLAM_SOLVE_TEXTBOOK))
                return MISSLAM_EUNSUPPORTED;
            b->rows = b->req_rows;
            b->waves = req_waves == 1 ? 1 : 2;
        } else {
            // the tiles: rows per solve workgroup and waves per assembly row, timed on this batch
            e = batch_save_params(b, st, false);
            float best = -1.f;
            int best_rows = 0, best_waves = 0;
            const int cand[4] = {21, 16, 12, 8};
            const int wcand[2] = {2, 1};
            for (int w = 0; w < 2 && e == hipSuccess; ++w) {
                if (req_waves != 0 && wcand[w] != req_waves) continue;
                b->waves = wcand[w];
                for (int c = 0; c < 4 && e == hipSuccess; ++c) {
                    const float ms = batch_try(b, ws, cand[c], st);
                    if (ms > 0.f && (best < 0.f || ms < best)) {
                        best = ms;
                        best_rows = cand[c];
                        best_waves = wcand[w];
                    }
                }
            }
            if (e != hipSuccess) return hip_fail(e);
            if (best_rows == 0) return MISSLAM_EUNSUPPORTED;
            b->rows = best_rows;
            b->waves = best_waves;
        }
    }
    if (b->items_ws != ws || b->items_rows != b->rows) {
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = batch_upload(b, ws, b->rows);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (!b->exec || b->exec_ws != ws || b->exec_rows != b->rows || b->exec_waves != b->waves) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        e = hipStreamSynchronize(st);
        hipGraph_t g = nullptr;
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t ee = batch_enqueue(b, b->cap, true);
            e = hipStreamEndCapture(b->cap, &g);
            if (ee != hipSuccess) e = ee;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return e == hipErrorInvalidConfiguration ? MISSLAM_EUNSUPPORTED : hip_fail(e);
        }
        b->exec_ws = ws;
        b->exec_rows = b->rows;
        b->exec_waves = b->waves;
    }
    e = hipGraphLaunch(b->exec, st);
    return e == hipSuccess ? MISSLAM_OK : hip_fail(e);
}

void misslam_batch_destroy(misslam_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_backup) (void)hipFree(b->d_backup);
    delete b;
}

}  // extern "C"
