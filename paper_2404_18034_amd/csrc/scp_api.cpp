// scp_api.cpp -- C ABI of the batched SCP solver: argument validation, workspace carving,
// handle state and error reporting.  All numerical work is in scp_kernels.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/scp_batch.h"
#include "scp_kernels.hpp"

namespace {

constexpr int KMAX_LIMIT = 50;  // 19 * k_max threads per subproblem workgroup must fit 1024
constexpr size_t ALIGN = 256;

thread_local std::string g_create_error;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    size_t blocks, what, dy, mup, mum, phi, th, step, sigma, stepsz, pipg_total, queue, bucket, order;
    size_t dblk, dwhat, tape, gstat, pbar;  // gradient scratch (when grad_pipg_steps > 0)
    size_t total;
};

bool settings_ok(const scp_settings *s, std::string &why)
{
    if (!s) { why = "settings is NULL"; return false; }
    if (s->dtype != SCP_F32 && s->dtype != SCP_F64) { why = "dtype must be SCP_F32 or SCP_F64"; return false; }
    if (s->k_max < 2 || s->k_max > KMAX_LIMIT) { why = "k_max must be in [2, 50]"; return false; }
    if (s->max_batch < 0) { why = "max_batch must be >= 0"; return false; }
    if (s->scp_iters_max < 1 || s->pipg_iters_max < 1 || s->rk4_substeps < 1 ||
        s->power_iters_max < 1) {
        why = "iteration counts and rk4_substeps must be >= 1";
        return false;
    }
    if (s->early_exit && s->pipg_check_every < 1) { why = "pipg_check_every must be >= 1"; return false; }
    if (s->mode < 0 || s->mode > 4) { why = "mode must be 0 (launches), 1 (graph), 2 (ordered), 3 (persistent) or 4 (K-bucketed)"; return false; }
    if (s->occupancy != 0 && (s->occupancy < 4 || s->occupancy > 6)) {
        why = "occupancy must be 0, 4, 5 or 6";
        return false;
    }
    if (s->grad_rk4_tangent != 0 && s->grad_rk4_tangent != 1) { why = "grad_rk4_tangent must be 0 or 1"; return false; }
    if (s->scalar_dilation != 0 && s->scalar_dilation != 1) { why = "scalar_dilation must be 0 or 1"; return false; }
    if (s->power_fp32 != 0 && s->power_fp32 != 1) { why = "power_fp32 must be 0 or 1"; return false; }
    if (s->n_u != 4 && s->n_u != 7) { why = "n_u must be 4 (thrust, dilation) or 7 (with the torque)"; return false; }
    if (!(s->w_prox > 0.0) || !(s->omega > 0.0) || !(s->rho > 0.0) || !(s->rho < 2.0) ||
        !(s->w_ep >= 0.0) || !isfinite(s->w_cost)) {
        why = "weights out of range (w_prox > 0, omega > 0, 0 < rho < 2, w_ep >= 0)";
        return false;
    }
    for (int i = 0; i < 15; ++i)
        if (!(s->px[i] > 0.0) || !isfinite(s->px[i])) { why = "px entries must be > 0"; return false; }
    for (int i = 0; i < s->n_u; ++i)
        if (!(s->pu[i] > 0.0) || !isfinite(s->pu[i])) { why = "pu entries must be > 0"; return false; }
    if (s->grad_pipg_steps < 0 ||
        (s->grad_pipg_steps > 0 &&
         (s->grad_ckpt_every < 1 || s->grad_ckpt_every > s->grad_pipg_steps))) {
        why = "grad_pipg_steps must be >= 0 and, when > 0, 1 <= grad_ckpt_every <= grad_pipg_steps";
        return false;
    }
    if (s->node_projections < 0 || s->node_projections > 31) {
        why = "node_projections is a bitmask in [0, 31]";
        return false;
    }
    if (s->node_projections &&
        (s->px[1] != s->px[2] || s->px[1] != s->px[3] || s->px[9] != s->px[10] ||
         s->px[11] != s->px[12] || s->px[11] != s->px[13] || s->pu[0] != s->pu[1] ||
         s->pu[0] != s->pu[2])) {
        why = "node projections need equal scales within r, (q2,q3), w and T";
        return false;
    }
    return true;
}

Layout layout_of(const scp_settings *s)
{
    const size_t rs = s->dtype == SCP_F64 ? 8 : 4;
    const size_t B = (size_t)s->max_batch, M = (size_t)(s->k_max - 1), K = (size_t)s->k_max;
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.blocks = take(B * M * (size_t)(15 + 2 * s->n_u) * 16 * rs);
    L.what = take(B * M * 16 * rs);
    L.dy = take(B * M * 8);
    L.mup = take(B * M * 16 * rs);
    L.mum = take(B * M * 16 * rs);
    L.phi = take(B * M * 16 * rs);
    L.th = take(B * K * rs);
    L.step = take(B * 8);
    L.sigma = take(B * 8);
    L.stepsz = take(B * 2 * rs);
    L.pipg_total = take(B * 4);
    L.queue = take((size_t)(s->scp_iters_max + 2) * 4);
    L.bucket = take((K + 1) * 4);
    L.order = take(B * 4);
    L.dblk = L.dwhat = L.tape = L.gstat = L.pbar = 0;
    if (s->grad_pipg_steps > 0) {
        const size_t n_ckpt = (size_t)((s->grad_pipg_steps + s->grad_ckpt_every - 1) / s->grad_ckpt_every);
        L.dblk = take(B * M * 2 * 23 * 16 * rs);
        L.dwhat = take(B * M * 2 * 16 * rs);
        L.tape = take(B * (n_ckpt + (size_t)s->grad_ckpt_every) * (size_t)scp::grad_state_len(s->k_max) * rs);
        L.gstat = take(B * 4);
        L.pbar = take(B * M * 2 * 8);
    }
    L.total = off == 0 ? ALIGN : off;
    return L;
}

}  // namespace

struct scp_batch_s {
    scp_settings st;
    int device;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Layout L;
    std::string err;
    // launch timing (scp_batch_profile)
    std::vector<hipEvent_t> events;
    std::vector<int> kinds;
    scp::LaunchTimer timer{nullptr, nullptr, 0, 0};
    bool profiling = false;
    int persistent_grid = 0;  // workgroups of the persistent subproblem kernel (0: not set)
    // graph replay (mode 1): the launch sequence of one solve, captured once per set of
    // arguments on a private stream and replayed on the handle's stream
    hipStream_t cap_stream = nullptr;
    hipStream_t aux_stream = nullptr;  // K-bucketed mode: the second subproblem launch
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void *graph_key[24] = {};
};

static void drop_graph(scp_batch h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    for (auto &k : h->graph_key) k = nullptr;
}

static void drop_events(scp_batch h)
{
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    h->kinds.clear();
    h->timer = scp::LaunchTimer{nullptr, nullptr, 0, 0};
    h->profiling = false;
}

static scp_status fail(scp_batch h, scp_status s, const std::string &msg)
{
    if (h) h->err = msg;
    return s;
}

extern "C" {

size_t scp_batch_workspace_bytes(const scp_settings *settings)
{
    std::string why;
    if (!settings_ok(settings, why)) return 0;
    return layout_of(settings).total;
}

const char *scp_batch_create_error(void) { return g_create_error.c_str(); }

scp_status scp_batch_create(const scp_settings *settings, int device, void *hip_stream,
                            void *workspace, size_t workspace_bytes, scp_batch *out)
{
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return SCP_ERR_ARG; }
    *out = nullptr;
    std::string why;
    if (!settings_ok(settings, why)) { g_create_error = why; return SCP_ERR_ARG; }
    if (settings->grad_pipg_steps > 0 &&
        scp::grad_smem_bytes(settings->dtype == SCP_F64 ? 1 : 0, settings->k_max) == 0) {
        g_create_error = "gradient state of this k_max and dtype does not fit one workgroup's LDS";
        return SCP_ERR_UNSUPPORTED;
    }
    if (settings->scalar_dilation && (settings->mode == 3 || settings->grad_pipg_steps > 0)) {
        g_create_error = "scalar_dilation is not implemented with mode 3 or with gradients";
        return SCP_ERR_UNSUPPORTED;
    }
    if (settings->n_u == 7 && (settings->scalar_dilation || settings->grad_pipg_steps > 0)) {
        g_create_error = "the torque input (n_u = 7) is not implemented with scalar_dilation or "
                         "with gradients";
        return SCP_ERR_UNSUPPORTED;
    }
    const Layout L = layout_of(settings);
    if (!workspace || workspace_bytes < L.total) {
        g_create_error = "workspace missing or smaller than scp_batch_workspace_bytes()";
        return SCP_ERR_WORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN != 0) {
        g_create_error = "workspace must be 256-byte aligned";
        return SCP_ERR_WORKSPACE;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) { g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e); return SCP_ERR_HIP; }
    if (device < 0 || device >= ndev) { g_create_error = "no such device"; return SCP_ERR_DEVICE; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { g_create_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e); return SCP_ERR_HIP; }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950";
        return SCP_ERR_DEVICE;
    }
    {
        const size_t need = scp::qp_smem_bytes(settings->k_max, settings->dtype == SCP_F64 ? 8 : 4);
        if (need > (size_t)prop.sharedMemPerBlock) {
            g_create_error = "subproblem workgroup needs " + std::to_string(need) +
                             " bytes of LDS, the device allows " +
                             std::to_string((size_t)prop.sharedMemPerBlock);
            return SCP_ERR_UNSUPPORTED;
        }
    }
    hipPointerAttribute_t attr;
    e = hipPointerGetAttributes(&attr, workspace);
    if (e != hipSuccess || attr.type != hipMemoryTypeDevice || attr.device != device) {
        (void)hipGetLastError();
        g_create_error = "workspace is not device memory of the requested device";
        return SCP_ERR_WORKSPACE;
    }
    scp_batch h = new (std::nothrow) scp_batch_s();
    if (!h) { g_create_error = "out of host memory"; return SCP_ERR_ARG; }
    h->st = *settings;
    h->device = device;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->ws = static_cast<char *>(workspace);
    h->ws_bytes = workspace_bytes;
    h->L = L;
    *out = h;
    return SCP_OK;
}

scp_status scp_batch_set_stream(scp_batch h, void *hip_stream)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    h->stream = static_cast<hipStream_t>(hip_stream);
    return SCP_OK;
}

const char *scp_batch_last_error(scp_batch h) { return h ? h->err.c_str() : "null handle"; }

static bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

static bool lastiter_ok(scp_batch h, const scp_lastiter *rec)
{
    const void *ptrs[] = {rec->xbar, rec->ubar, rec->mup, rec->mum, rec->phi, rec->th, rec->sigma};
    for (const void *p : ptrs)
        if (!p || !aligned16(p)) {
            h->err = "a last-iteration array is NULL or not 16-byte aligned";
            return false;
        }
    return true;
}

static void fill_config_from(const scp_settings &s, int batch, scp::Config &cfg)
{
    cfg.dtype = s.dtype == SCP_F64 ? 1 : 0;
    cfg.B = batch;
    cfg.kmax = s.k_max;
    cfg.scp_iters_max = s.scp_iters_max;
    cfg.pipg_iters_max = s.pipg_iters_max;
    cfg.pipg_check_every = s.pipg_check_every;
    cfg.rk4_substeps = s.rk4_substeps;
    cfg.power_iters_max = s.power_iters_max;
    cfg.early_exit = s.early_exit;
    cfg.node_projections = s.node_projections;
    cfg.persistent_blocks = 0;
    cfg.ordered = (s.mode == 2 || s.mode == 4) ? 1 : 0;
    cfg.bucketed = s.mode == 4 ? 1 : 0;
    cfg.aux_stream = nullptr;
    cfg.ev_fork = cfg.ev_join = nullptr;
    cfg.occupancy = s.occupancy;
    cfg.grad_rk4_tangent = s.grad_rk4_tangent;
    cfg.scalar_dilation = s.scalar_dilation;
    cfg.power_fp32 = s.power_fp32;
    cfg.nu = s.n_u;
    cfg.scp_tol = s.scp_tol;
    cfg.feas_tol = s.feas_tol;
    cfg.pipg_eps_abs = s.pipg_eps_abs;
    cfg.pipg_eps_rel = s.pipg_eps_rel;
    cfg.power_eps_abs = s.power_eps_abs;
    cfg.power_eps_rel = s.power_eps_rel;
    cfg.power_buff = s.power_buff;
    cfg.w_cost = s.w_cost;
    cfg.w_prox = s.w_prox;
    cfg.w_ep = s.w_ep;
    cfg.omega = s.omega;
    cfg.rho = s.rho;
    memcpy(cfg.px, s.px, sizeof(cfg.px));
    memcpy(cfg.pu, s.pu, sizeof(cfg.pu));
}

static void fill_config(scp_batch h, int batch, scp::Config &cfg)
{
    fill_config_from(h->st, batch, cfg);
}

static scp::Workspace workspace_at(char *ws, const Layout &L)
{
    scp::Workspace W;
    W.blocks = ws + L.blocks;
    W.what = ws + L.what;
    W.dy = reinterpret_cast<double *>(ws + L.dy);
    W.mup = ws + L.mup;
    W.mum = ws + L.mum;
    W.phi = ws + L.phi;
    W.th = ws + L.th;
    W.step = reinterpret_cast<double *>(ws + L.step);
    W.sigma = reinterpret_cast<double *>(ws + L.sigma);
    W.stepsz = ws + L.stepsz;
    W.pipg_total = reinterpret_cast<int32_t *>(ws + L.pipg_total);
    W.queue = reinterpret_cast<int32_t *>(ws + L.queue);
    W.bucket = reinterpret_cast<int32_t *>(ws + L.bucket);
    W.order = reinterpret_cast<int32_t *>(ws + L.order);
    return W;
}

static scp::Workspace workspace_of(scp_batch h) { return workspace_at(h->ws, h->L); }

static scp_status solve_impl(scp_batch h, const scp_problem *prob, scp_solution *sol,
                             const scp_lastiter *rec)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    if (!prob || !sol) return fail(h, SCP_ERR_ARG, "problem or solution is NULL");
    if (rec && !lastiter_ok(h, rec)) return SCP_ERR_ARG;
    if (prob->batch < 0 || prob->batch > h->st.max_batch)
        return fail(h, SCP_ERR_SHAPE, "batch must be in [0, max_batch]");
    if (prob->batch == 0) return SCP_OK;
    const void *in_ptrs[] = {prob->x0, prob->xf, prob->params, prob->K};
    for (const void *p : in_ptrs)
        if (!p) return fail(h, SCP_ERR_ARG, "a problem array is NULL");
    const void *out_ptrs[] = {sol->x, sol->u, sol->t_f, sol->m_f, sol->status,
                              sol->scp_iters, sol->pipg_iters, sol->defect_inf,
                              sol->ctcs_viol, sol->objective};
    for (const void *p : out_ptrs)
        if (!p) return fail(h, SCP_ERR_ARG, "a solution array is NULL");
    for (const void *p : in_ptrs)
        if (!aligned16(p)) return fail(h, SCP_ERR_ARG, "arrays must be 16-byte aligned");
    for (const void *p : out_ptrs)
        if (!aligned16(p)) return fail(h, SCP_ERR_ARG, "arrays must be 16-byte aligned");
    if ((prob->x_init && !aligned16(prob->x_init)) || (prob->u_init && !aligned16(prob->u_init)))
        return fail(h, SCP_ERR_ARG, "arrays must be 16-byte aligned");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != h->device) {
        e = hipSetDevice(h->device);
        if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }

    scp::Config cfg;
    fill_config(h, prob->batch, cfg);
    if (h->st.mode == 4 && h->st.k_max > 12) {
        // the second stream and the fork/join events of the K-bucketed launches (created once)
        if (!h->aux_stream) {
            e = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
            if (e != hipSuccess) {
                if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
                if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
                h->aux_stream = nullptr;
                h->ev_fork = nullptr;
                if (cur != h->device) (void)hipSetDevice(cur);
                return fail(h, SCP_ERR_HIP, std::string("auxiliary stream: ") + hipGetErrorString(e));
            }
        }
        cfg.aux_stream = h->aux_stream;
        cfg.ev_fork = h->ev_fork;
        cfg.ev_join = h->ev_join;
    }
    if (h->st.mode == 3) {
        if (h->persistent_grid == 0) {
            hipDeviceProp_t prop;
            e = hipGetDeviceProperties(&prop, h->device);
            if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
            h->persistent_grid =
                prop.multiProcessorCount * scp::qp_blocks_per_cu(cfg.dtype, h->st.k_max, h->st.n_u);
        }
        cfg.persistent_blocks = h->persistent_grid;
    }

    scp::Problem P{prob->x0, prob->xf, prob->params, prob->K, prob->x_init, prob->u_init};
    scp::Solution S{sol->x, sol->u, sol->t_f, sol->m_f, sol->status, sol->scp_iters,
                    sol->pipg_iters, sol->defect_inf, sol->ctcs_viol, sol->objective};
    const scp::Workspace W = workspace_of(h);
    scp::Record Rc{};
    if (rec) Rc = scp::Record{rec->xbar, rec->ubar, rec->mup, rec->mum, rec->phi, rec->th, rec->sigma};
    const scp::Record *RP = rec ? &Rc : nullptr;
    if (h->st.mode >= 1 && !h->profiling) {
        // replay a captured graph of the whole launch sequence when the arguments match
        const void *key[24] = {reinterpret_cast<const void *>((intptr_t)prob->batch), prob->x0,
                               prob->xf, prob->params, prob->K, sol->x, sol->u, sol->t_f,
                               sol->m_f, sol->status, sol->scp_iters, sol->pipg_iters,
                               sol->defect_inf, sol->ctcs_viol, sol->objective,
                               Rc.xbar, Rc.ubar, Rc.mup, Rc.mum, Rc.phi, Rc.th, Rc.sigma,
                               prob->x_init, prob->u_init};
        if (!h->graph_exec || memcmp(key, h->graph_key, sizeof(key)) != 0) {
            drop_graph(h);
            if (!h->cap_stream) {
                e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) {
                    h->cap_stream = nullptr;
                    if (cur != h->device) (void)hipSetDevice(cur);
                    return fail(h, SCP_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
                }
            }
            e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t el = scp::launch_solve(cfg, P, S, W, RP, h->cap_stream, nullptr);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(h->cap_stream, &g);
                if (el != hipSuccess) e = el;
                if (e == hipSuccess) {
                    h->graph = g;
                    e = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
                } else if (g) {
                    (void)hipGraphDestroy(g);
                }
            }
            if (e != hipSuccess) {
                drop_graph(h);
                if (cur != h->device) (void)hipSetDevice(cur);
                return fail(h, SCP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            }
            memcpy(h->graph_key, key, sizeof(key));
        }
        e = hipGraphLaunch(h->graph_exec, h->stream);
    } else {
        e = scp::launch_solve(cfg, P, S, W, RP, h->stream, h->profiling ? &h->timer : nullptr);
    }
    if (cur != h->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SCP_OK;
}

scp_status scp_batch_solve(scp_batch h, const scp_problem *prob, scp_solution *sol)
{
    return solve_impl(h, prob, sol, nullptr);
}

scp_status scp_batch_solve_record(scp_batch h, const scp_problem *prob, scp_solution *sol,
                                  const scp_lastiter *last)
{
    if (!h) return SCP_ERR_ARG;
    if (!last) {
        h->err = "last is NULL";
        return SCP_ERR_ARG;
    }
    return solve_impl(h, prob, sol, last);
}

scp_status scp_batch_grad(scp_batch h, const scp_problem *prob, const scp_lastiter *last,
                          const void *cotangent, void *grad, void *value)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    if (h->st.grad_pipg_steps <= 0)
        return fail(h, SCP_ERR_STATE, "the handle was created with grad_pipg_steps = 0");
    if (!prob || !last || !cotangent || !grad)
        return fail(h, SCP_ERR_ARG, "problem, last, cotangent or grad is NULL");
    if (!lastiter_ok(h, last)) return SCP_ERR_ARG;
    if (prob->batch < 0 || prob->batch > h->st.max_batch)
        return fail(h, SCP_ERR_SHAPE, "batch must be in [0, max_batch]");
    if (prob->batch == 0) return SCP_OK;
    const void *ptrs[] = {prob->x0, prob->xf, prob->params, prob->K, cotangent, grad};
    for (const void *p : ptrs)
        if (!p || !aligned16(p)) return fail(h, SCP_ERR_ARG, "arrays must be non-NULL and 16-byte aligned");
    if (value && !aligned16(value)) return fail(h, SCP_ERR_ARG, "arrays must be 16-byte aligned");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != h->device) {
        e = hipSetDevice(h->device);
        if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    scp::Config cfg;
    fill_config(h, prob->batch, cfg);
    const scp::Workspace W = workspace_of(h);
    scp::GradWorkspace G;
    G.dblk = h->ws + h->L.dblk;
    G.dwhat = h->ws + h->L.dwhat;
    G.tape = h->ws + h->L.tape;
    G.gstat = reinterpret_cast<int32_t *>(h->ws + h->L.gstat);
    G.pbar = reinterpret_cast<double *>(h->ws + h->L.pbar);
    const scp::Problem P{prob->x0, prob->xf, prob->params, prob->K};
    const scp::Record Rc{last->xbar, last->ubar, last->mup, last->mum, last->phi, last->th,
                         last->sigma};
    e = scp::launch_grad(cfg, h->st.grad_pipg_steps, h->st.grad_ckpt_every, P, Rc, cotangent,
                         grad, value, W, G, h->stream);
    if (cur != h->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SCP_OK;
}

scp_status scp_batch_profile(scp_batch h, int enable)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    if (!enable) {
        (void)hipStreamSynchronize(h->stream);
        drop_events(h);
        return SCP_OK;
    }
    if (h->profiling) return SCP_OK;
    const int cap = 1 + 3 * (h->st.scp_iters_max + 1);
    h->events.assign(2 * cap, nullptr);
    h->kinds.assign(cap, -1);
    for (auto &ev : h->events) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            drop_events(h);
            return fail(h, SCP_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
        }
    }
    h->timer = scp::LaunchTimer{h->events.data(), h->kinds.data(), cap, 0};
    h->profiling = true;
    return SCP_OK;
}

scp_status scp_batch_profile_read(scp_batch h, double *ms, int32_t *launches)
{
    if (!h || !ms || !launches) return SCP_ERR_ARG;
    h->err.clear();
    for (int k = 0; k < SCP_KERNEL_CLASSES; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    if (!h->profiling) return fail(h, SCP_ERR_STATE, "profiling is not enabled");
    const int n = h->timer.n_launches;
    if (n == 0) return SCP_OK;
    hipError_t e = hipEventSynchronize(h->events[2 * n - 1]);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    for (int i = 0; i < n; ++i) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, h->events[2 * i], h->events[2 * i + 1]);
        if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
        const int k = h->kinds[i];
        if (k >= 0 && k < SCP_KERNEL_CLASSES) {
            ms[k] += t;
            launches[k] += 1;
        }
    }
    return SCP_OK;
}

// ------------------------------------------------------------------------------------------
// Autotuner: time the dispatch modes on the caller's batch and keep the fastest.
// ------------------------------------------------------------------------------------------
static std::string tune_key(scp_batch h, int batch)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << ":kmax=" << h->st.k_max << ":dtype=" << (h->st.dtype == SCP_F64 ? "f64" : "f32")
      << ":early_exit=" << h->st.early_exit << ":proj=" << h->st.node_projections
      << ":sd=" << h->st.scalar_dilation << ":pw32=" << h->st.power_fp32 << ":nu=" << h->st.n_u
      << ":batch=" << batch;
    return k.str();
}

static const int TUNE_MODE[SCP_TUNE_VARIANTS] = {1, 2, 3, 1, 2, 1, 2, 4, 4, 4};
static const int TUNE_OCC[SCP_TUNE_VARIANTS] = {0, 0, 0, 5, 5, 6, 6, 0, 5, 6};

static int cache_lookup(const char *path, const std::string &key)
{
    if (!path) return -1;
    std::ifstream f(path);
    std::string line;
    int found = -1;
    const std::string pat = "\"key\": \"" + key + "\"";
    const std::string tag = "\"variant\": ";
    while (std::getline(f, line)) {
        if (line.find(pat) == std::string::npos) continue;
        const size_t m = line.find(tag);
        if (m != std::string::npos) found = atoi(line.c_str() + m + tag.size());
    }
    return (found >= 0 && found < SCP_TUNE_VARIANTS) ? found : -1;
}

static void set_variant(scp_batch h, int v)
{
    h->st.mode = TUNE_MODE[v];
    h->st.occupancy = TUNE_OCC[v];
    drop_graph(h);
}

scp_status scp_batch_autotune(scp_batch h, const scp_problem *prob, scp_solution *sol,
                              const char *cache_path, int32_t *variant_out, double *ms_out)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    if (!prob || !sol || !variant_out || !ms_out) return fail(h, SCP_ERR_ARG, "null argument");
    for (int v = 0; v < SCP_TUNE_VARIANTS; ++v) ms_out[v] = -1.0;
    const std::string key = tune_key(h, prob->batch);
    const int cached = cache_lookup(cache_path, key);
    if (cached >= 0) {
        set_variant(h, cached);
        *variant_out = cached;
        return SCP_OK;
    }
    if (h->profiling) return fail(h, SCP_ERR_STATE, "disable profiling before autotuning");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(h, SCP_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    const int saved_mode = h->st.mode, saved_occ = h->st.occupancy;
    int best = -1;
    double best_ms = 0.0;
    for (int m = 0; m < SCP_TUNE_VARIANTS; ++m) {
        // one dilation value: no persistent form, and one register budget whatever occupancy
        if (h->st.scalar_dilation && (TUNE_MODE[m] == 3 || TUNE_OCC[m] != 0)) continue;
        set_variant(h, m);
        scp_status st = scp_batch_solve(h, prob, sol);  // capture + warm-up
        if (st != SCP_OK) break;
        float t = 0.0f;
        e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess && scp_batch_solve(h, prob, sol) != SCP_OK) break;
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) break;
        ms_out[m] = t;
        if (best < 0 || t < best_ms) {
            best = m;
            best_ms = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) {
        h->st.mode = saved_mode;
        h->st.occupancy = saved_occ;
        drop_graph(h);
        if (h->err.empty()) h->err = std::string("autotune: ") + hipGetErrorString(e);
        return SCP_ERR_HIP;
    }
    set_variant(h, best);
    *variant_out = best;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << "{\"key\": \"" << key << "\", \"variant\": " << best << ", \"mode\": "
          << TUNE_MODE[best] << ", \"occupancy\": " << TUNE_OCC[best] << ", \"ms\": [";
        for (int v = 0; v < SCP_TUNE_VARIANTS; ++v) f << (v ? ", " : "") << ms_out[v];
        f << "]}\n";
    }
    return SCP_OK;
}

scp_status scp_batch_mode(scp_batch h, int32_t *mode_out, int32_t *occupancy_out)
{
    if (!h || !mode_out || !occupancy_out) return SCP_ERR_ARG;
    *mode_out = h->st.mode;
    *occupancy_out = h->st.occupancy;
    return SCP_OK;
}

scp_status scp_batch_select_best(scp_batch h, const scp_solution *sol, int32_t problems,
                                 int32_t starts, int32_t *best, scp_solution *out)
{
    if (!h) return SCP_ERR_ARG;
    h->err.clear();
    if (!sol || !out) return fail(h, SCP_ERR_ARG, "solution or out is NULL");
    if (problems < 0 || starts < 1)
        return fail(h, SCP_ERR_SHAPE, "problems must be >= 0 and starts >= 1");
    if ((int64_t)problems * starts > h->st.max_batch)
        return fail(h, SCP_ERR_SHAPE, "problems * starts must be <= max_batch");
    if (problems == 0) return SCP_OK;
    if (!best) return fail(h, SCP_ERR_ARG, "best is NULL");
    const size_t rs = h->st.dtype == SCP_F64 ? 8 : 4, km = (size_t)h->st.k_max;
    // every array with its extent in bytes per instance, for the solved batch and for out
    struct Arr { const void *p; size_t per; };
    const Arr in_a[] = {{sol->x, km * 15 * rs}, {sol->u, km * 4 * rs}, {sol->t_f, rs},
                        {sol->m_f, rs}, {sol->status, 4}, {sol->scp_iters, 4},
                        {sol->pipg_iters, 4}, {sol->defect_inf, 8}, {sol->ctcs_viol, 8},
                        {sol->objective, 8}};
    const Arr out_a[] = {{out->x, km * 15 * rs}, {out->u, km * 4 * rs}, {out->t_f, rs},
                         {out->m_f, rs}, {out->status, 4}, {out->scp_iters, 4},
                         {out->pipg_iters, 4}, {out->defect_inf, 8}, {out->ctcs_viol, 8},
                         {out->objective, 8}, {best, 4}};
    for (const Arr &a : in_a)
        if (!a.p || !aligned16(a.p)) return fail(h, SCP_ERR_ARG, "solution arrays must be non-NULL and 16-byte aligned");
    for (const Arr &a : out_a)
        if (!a.p || (a.p != best && !aligned16(a.p)))
            return fail(h, SCP_ERR_ARG, "out arrays must be non-NULL and 16-byte aligned");
    // the outputs (and best) may overlap neither the solved batch nor each other
    const size_t n_in = (size_t)problems * (size_t)starts, n_out = (size_t)problems;
    auto overlap = [](const void *a, size_t na, const void *b, size_t nb) {
        const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
        return x < y + nb && y < x + na;
    };
    for (size_t i = 0; i < sizeof(out_a) / sizeof(out_a[0]); ++i) {
        for (const Arr &a : in_a)
            if (overlap(out_a[i].p, out_a[i].per * n_out, a.p, a.per * n_in))
                return fail(h, SCP_ERR_ARG, "out and best must not overlap the solution");
        for (size_t j = 0; j < i; ++j)
            if (overlap(out_a[i].p, out_a[i].per * n_out, out_a[j].p, out_a[j].per * n_out))
                return fail(h, SCP_ERR_ARG, "out arrays and best must not overlap each other");
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != h->device) {
        e = hipSetDevice(h->device);
        if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    const scp::Solution S{sol->x, sol->u, sol->t_f, sol->m_f, sol->status, sol->scp_iters,
                          sol->pipg_iters, sol->defect_inf, sol->ctcs_viol, sol->objective};
    const scp::Solution O{out->x, out->u, out->t_f, out->m_f, out->status, out->scp_iters,
                          out->pipg_iters, out->defect_inf, out->ctcs_viol, out->objective};
    e = scp::launch_select_best(h->st.dtype == SCP_F64 ? 1 : 0, h->st.k_max, h->st.n_u, S, O,
                                problems, starts, best, h->stream);
    if (cur != h->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(h, SCP_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return SCP_OK;
}

// Allocation-free solve: the workspace is the library's fixed device scratch array.
static_assert(scp::SCRATCH_BYTES == SCP_NOALLOC_SCRATCH_BYTES, "scratch size of the header");
scp_status scp_batch_solve_noalloc(const scp_settings *settings, int device, void *hip_stream,
                                   const scp_problem *prob, scp_solution *sol)
{
    g_create_error.clear();
    std::string why;
    if (!settings_ok(settings, why)) { g_create_error = why; return SCP_ERR_ARG; }
    if (settings->n_u == 7 && settings->scalar_dilation) {
        g_create_error = "the torque input (n_u = 7) is not implemented with scalar_dilation";
        return SCP_ERR_UNSUPPORTED;
    }
    if (!prob || !sol) { g_create_error = "problem or solution is NULL"; return SCP_ERR_ARG; }
    if (prob->batch < 0 || prob->batch > settings->max_batch) {
        g_create_error = "batch must be in [0, max_batch]";
        return SCP_ERR_SHAPE;
    }
    if (prob->batch == 0) return SCP_OK;
    const void *in_ptrs[] = {prob->x0, prob->xf, prob->params, prob->K};
    const void *out_ptrs[] = {sol->x, sol->u, sol->t_f, sol->m_f, sol->status,
                              sol->scp_iters, sol->pipg_iters, sol->defect_inf,
                              sol->ctcs_viol, sol->objective};
    for (const void *p : in_ptrs)
        if (!p || !aligned16(p)) { g_create_error = "a problem array is NULL or not 16-byte aligned"; return SCP_ERR_ARG; }
    for (const void *p : out_ptrs)
        if (!p || !aligned16(p)) { g_create_error = "a solution array is NULL or not 16-byte aligned"; return SCP_ERR_ARG; }
    if ((prob->x_init && !aligned16(prob->x_init)) || (prob->u_init && !aligned16(prob->u_init))) {
        g_create_error = "x_init and u_init must be 16-byte aligned";
        return SCP_ERR_ARG;
    }
    // the workspace of this batch (no gradient scratch), carved from the fixed array
    scp_settings s = *settings;
    s.max_batch = prob->batch;
    s.grad_pipg_steps = 0;
    const Layout L = layout_of(&s);
    if (L.total > scp::SCRATCH_BYTES) {
        g_create_error = "this batch needs " + std::to_string(L.total) +
                         " bytes of workspace; the fixed scratch holds " +
                         std::to_string(scp::SCRATCH_BYTES);
        return SCP_ERR_WORKSPACE;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) { g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e); return SCP_ERR_HIP; }
    if (device < 0 || device >= ndev) { g_create_error = "no such device"; return SCP_ERR_DEVICE; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { g_create_error = std::string("hipGetDeviceProperties: ") + hipGetErrorString(e); return SCP_ERR_HIP; }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        g_create_error = std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950";
        return SCP_ERR_DEVICE;
    }
    if (scp::qp_smem_bytes(s.k_max, s.dtype == SCP_F64 ? 8 : 4) > (size_t)prop.sharedMemPerBlock) {
        g_create_error = "subproblem workgroup of this k_max does not fit the device's LDS";
        return SCP_ERR_UNSUPPORTED;
    }
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) { g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e); return SCP_ERR_HIP; }
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return SCP_ERR_HIP;
    }
    void *ws = nullptr;
    e = scp::scratch_address(device, &ws);
    if (e == hipSuccess) {
        scp::Config cfg;
        fill_config_from(s, prob->batch, cfg);
        // plain launches, workgroup b <-> instance b, whatever the mode setting
        cfg.ordered = 0;
        cfg.bucketed = 0;
        cfg.persistent_blocks = 0;
        const scp::Problem P{prob->x0, prob->xf, prob->params, prob->K, prob->x_init,
                             prob->u_init};
        const scp::Solution S{sol->x, sol->u, sol->t_f, sol->m_f, sol->status, sol->scp_iters,
                              sol->pipg_iters, sol->defect_inf, sol->ctcs_viol, sol->objective};
        e = scp::launch_solve(cfg, P, S, workspace_at(static_cast<char *>(ws), L), nullptr,
                              static_cast<hipStream_t>(hip_stream), nullptr);
        if (e != hipSuccess) g_create_error = std::string("kernel launch: ") + hipGetErrorString(e);
    } else {
        g_create_error = std::string("scratch address: ") + hipGetErrorString(e);
    }
    if (cur != device) (void)hipSetDevice(cur);
    return e == hipSuccess ? SCP_OK : SCP_ERR_HIP;
}

scp_status scp_batch_destroy(scp_batch h)
{
    if (!h) return SCP_ERR_ARG;
    hipError_t e = hipStreamSynchronize(h->stream);
    drop_events(h);
    drop_graph(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    delete h;
    return e == hipSuccess ? SCP_OK : SCP_ERR_HIP;
}

}  // extern "C"
