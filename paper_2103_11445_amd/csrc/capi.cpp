// capi.cpp -- the extern "C" boundary declared in include/sptrsv.h.
// Turns internal errors into status codes plus a thread-local message, and
// moves plans between host and device.
#include <hip/hip_runtime_api.h>

#include <climits>
#include <cstring>
#include <new>
#include <stdexcept>
#include <algorithm>
#include <cstddef>
#include <string>

#include "features.hpp"
#include "plan.hpp"

struct sptrsv_plan_s : sptrsv::Plan {};

namespace {
void drop_graph(sptrsv::Plan &p) {
    if (p.graph_exec) hipGraphExecDestroy(static_cast<hipGraphExec_t>(p.graph_exec));
    p.graph_exec = nullptr;
    p.graph_b = p.graph_x = nullptr;
}
}  // namespace

sptrsv::Plan::~Plan() {
    drop_graph(*this);
    if (capture_stream) hipStreamDestroy(static_cast<hipStream_t>(capture_stream));
}

namespace {
thread_local std::string g_err;

sptrsv_status set_err(sptrsv_status s, const std::string &m) {
    g_err = m;
    return s;
}

template <class F>
sptrsv_status guarded(F &&f) {
    try {
        g_err.clear();
        return f();
    } catch (const sptrsv::Error &e) {
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(SPTRSV_ERR_OOM, "out of host memory");
    } catch (const std::length_error &) {
        return set_err(SPTRSV_ERR_OOM, "out of host memory");
    }
}

sptrsv_status hip_err(hipError_t e, const char *what) {
    return set_err(SPTRSV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Waves of the cooperative solve grid.  Unless set by sptrsv_set_launch, the
// count follows the work per level: about two waves per CU for every CU's
// worth of tiles in an average level (1 to 8 per CU), because waves that
// run far ahead of the frontier only poll.
int launch_waves(const sptrsv::Plan &p) {
    int wpc = p.waves_per_cu;
    if (wpc <= 0) {
        const double per_level = p.nlev_rw > 0 ? (double)p.ntiles / p.nlev_rw : 0.0;
        const double want = 2.0 * per_level / std::max(1, p.cus);
        wpc = 1;
        while (wpc < 8 && wpc * 2 <= want) wpc *= 2;
        // a stage system's whole-stage segments each on a wave of their own
        if (p.comp_segs > 0)
            wpc = std::max<int>(wpc, (int)((p.comp_segs + std::max(1, p.cus) - 1) / std::max(1, p.cus)));
    }
    wpc = std::min({wpc, p.max_waves_per_cu, sptrsv::kMaxWavesPerCU});
    const int64_t w = std::min<int64_t>((int64_t)p.cus * wpc, p.ntiles);
    return (int)std::max<int64_t>(1, w);
}

// Launch shape: the waves above, split between the chain queue and the sink
// queue.  Unless set by sptrsv_set_chain_share, each queue gets the share of
// the waves its share of the work asks for (64-lane chunks of terms and rows
// packed), kept within [1/8, 7/8] so that neither queue is starved.
sptrsv::LaunchShape launch_shape(const sptrsv::Plan &p) {
    sptrsv::LaunchShape sh;
    sh.nitems = p.ntiles;
    sh.waves = launch_waves(p);
    if (p.nchain <= 0 || p.nchain >= p.ntiles || sh.waves < 2) {
        sh.nchain = p.ntiles;
        sh.chain_waves = sh.waves;
        return sh;
    }
    sh.nchain = p.nchain;
    double share = p.chain_share > 0 ? p.chain_share / 1000.0
                                     : (double)p.chain_work / (double)std::max<int64_t>(1, p.chain_work + p.sink_work);
    share = std::min(7.0 / 8.0, std::max(1.0 / 8.0, share));
    const int cw = (int)(share * sh.waves + 0.5);
    sh.chain_waves = std::min(std::max(cw, 1), sh.waves - 1);
    return sh;
}

// Launch shape of the stage system's solve (kRhsStage), else zeros.
sptrsv::LaunchShape sub_shape(const sptrsv::Plan &p) {
    if (!p.sub) return sptrsv::LaunchShape{};
    sptrsv::Plan &q = *p.sub;
    q.cus = p.cus;
    q.max_waves_per_cu = p.max_waves_per_cu;
    return launch_shape(q);
}

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bn && pb < pa + an;
}
}  // namespace

extern "C" {

void sptrsv_policy_default(sptrsv_policy *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->kind = SPTRSV_POLICY_THRESHOLD;
    p->max_width = 4;
    p->max_depth = 64;
    p->max_fill = 0.25;
    p->max_entries = INT32_MAX;
}

sptrsv_status sptrsv_analyse(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             const double *val, sptrsv_plan *out) {
    if (out) *out = nullptr;
    return guarded([&]() -> sptrsv_status {
        if (!out) return set_err(SPTRSV_ERR_ARG, "out is NULL");
        sptrsv_plan p = new sptrsv_plan_s();
        try {
            sptrsv::analyse(*p, n, row_ptr, col_idx, val);
            sptrsv_policy none{};
            none.kind = SPTRSV_POLICY_NONE;
            sptrsv::rewrite(*p, none);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_analyse_upper(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                   const double *val, sptrsv_plan *out) {
    if (out) *out = nullptr;
    return guarded([&]() -> sptrsv_status {
        if (!out) return set_err(SPTRSV_ERR_ARG, "out is NULL");
        sptrsv_plan p = new sptrsv_plan_s();
        try {
            sptrsv::analyse_upper(*p, n, row_ptr, col_idx, val);
            sptrsv_policy none{};
            none.kind = SPTRSV_POLICY_NONE;
            sptrsv::rewrite(*p, none);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_analyse_batch(int32_t count, const int32_t *n, const int32_t *const *row_ptr,
                                   const int32_t *const *col_idx, const double *const *val,
                                   const int32_t *k, sptrsv_plan *out) {
    if (out) *out = nullptr;
    return guarded([&]() -> sptrsv_status {
        if (!out) return set_err(SPTRSV_ERR_ARG, "out is NULL");
        sptrsv_plan p = new sptrsv_plan_s();
        try {
            sptrsv::analyse_batch(*p, count, n, row_ptr, col_idx, val, k);
            sptrsv_policy none{};
            none.kind = SPTRSV_POLICY_NONE;
            sptrsv::rewrite(*p, none);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_rewrite(sptrsv_plan plan, const sptrsv_policy *policy) {
    return guarded([&]() -> sptrsv_status {
        if (!plan || !policy) return set_err(SPTRSV_ERR_ARG, "null argument");
        sptrsv::validate_policy(*policy);
        plan->uploaded = false;
        drop_graph(*plan);
        try {
            sptrsv::rewrite(*plan, *policy);
        } catch (...) {
            // leave a consistent plan behind: the plain schedule
            sptrsv_policy none{};
            none.kind = SPTRSV_POLICY_NONE;
            try {
                sptrsv::rewrite(*plan, none);
            } catch (...) {
            }
            throw;
        }
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_device_bytes(sptrsv_plan plan, size_t *bytes) {
    if (!plan || !bytes) return set_err(SPTRSV_ERR_ARG, "null argument");
    *bytes = plan->layout.total;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_upload(sptrsv_plan plan, void *dev_buf, size_t bytes, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (!plan || !dev_buf) return set_err(SPTRSV_ERR_ARG, "null argument");
        if (bytes < plan->layout.total)
            return set_err(SPTRSV_ERR_ARG, "device buffer smaller than sptrsv_device_bytes");
        if (reinterpret_cast<uintptr_t>(dev_buf) % 256 != 0)
            return set_err(SPTRSV_ERR_ARG, "device buffer not 256-byte aligned");
        int cus = 0, maxw = 0;
        if (int e = sptrsv_device_limits(&cus, &maxw)) return hip_err((hipError_t)e, "device query");
        if (cus <= 0 || maxw <= 0) return set_err(SPTRSV_ERR_HIP, "solve kernel cannot be resident");
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = hipMemcpyAsync(dev_buf, plan->image.data(), plan->layout.total,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_err(e, "hipMemcpyAsync");
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "hipStreamSynchronize");
        drop_graph(*plan);
        plan->dev = dev_buf;
        plan->cus = cus;
        plan->max_waves_per_cu = maxw;
        plan->uploaded = true;
        return SPTRSV_OK;
    });
}

}  // extern "C"

namespace {
// Common checks of the solve entry points; 1 when there is nothing to do
// (n == 0), 0 when the solve may be enqueued.  Throws on a bad call.
int solve_args_ok(const sptrsv::Plan *plan, const void *b, const void *x, int precision, size_t elem) {
    if (!plan) throw sptrsv::Error{SPTRSV_ERR_ARG, "plan is NULL"};
    if (!plan->uploaded) throw sptrsv::Error{SPTRSV_ERR_STATE, "plan not uploaded (or rewritten since)"};
    if (plan->precision != precision)
        throw sptrsv::Error{SPTRSV_ERR_STATE, precision == 64
                                                  ? "plan is stored in FP32: use sptrsv_solve_fp32 or sptrsv_solve_refined"
                                                  : "plan is stored in FP64: set FP32 with sptrsv_set_precision"};
    const int32_t n = plan->n;
    if (n == 0) return 1;
    if (!b || !x) throw sptrsv::Error{SPTRSV_ERR_ARG, "null b or x"};
    const size_t nb = (size_t)n * elem;
    if (overlaps(b, nb, x, nb)) throw sptrsv::Error{SPTRSV_ERR_ARG, "b and x overlap"};
    if (overlaps(x, nb, plan->dev, plan->layout.total) || overlaps(b, nb, plan->dev, plan->layout.total))
        throw sptrsv::Error{SPTRSV_ERR_ARG, "b or x overlaps the plan buffer"};
    return 0;
}
}  // namespace

extern "C" {

sptrsv_status sptrsv_solve(sptrsv_plan plan, const double *b, double *x, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (solve_args_ok(plan, b, x, 64, sizeof(double))) return SPTRSV_OK;
        const sptrsv::LaunchShape sh = launch_shape(*plan), sub = sub_shape(*plan);
        const int e = sptrsv_launch_solve(static_cast<const unsigned char *>(plan->dev), &plan->layout, plan->n,
                                          &sh, &sub, plan->wait_limit, b, x, nullptr, 0, stream);
        if (e != 0) return hip_err((hipError_t)e, "kernel launch");
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_solve_fp32(sptrsv_plan plan, const float *b, float *x, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (solve_args_ok(plan, b, x, 32, sizeof(float))) return SPTRSV_OK;
        const sptrsv::LaunchShape sh = launch_shape(*plan), sub = sub_shape(*plan);
        const int e = sptrsv_launch_solve(static_cast<const unsigned char *>(plan->dev), &plan->layout, plan->n,
                                          &sh, &sub, plan->wait_limit, b, x, nullptr, 0, stream);
        if (e != 0) return hip_err((hipError_t)e, "kernel launch");
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_solve_refined(sptrsv_plan plan, const double *b, double *x, int32_t iterations,
                                   double tol, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (iterations < 1 || iterations > sptrsv::kMaxRefine)
            return set_err(SPTRSV_ERR_ARG, "iterations must be in [1, 16]");
        if (!(tol >= 0.0)) return set_err(SPTRSV_ERR_ARG, "tol must be >= 0");
        if (solve_args_ok(plan, b, x, 32, sizeof(double))) return SPTRSV_OK;
        const sptrsv::LaunchShape sh = launch_shape(*plan), sub = sub_shape(*plan);
        const int e = sptrsv_launch_refined(static_cast<const unsigned char *>(plan->dev), &plan->layout, plan->n,
                                            &sh, &sub, plan->wait_limit, b, x, iterations, tol, stream);
        if (e != 0) return hip_err((hipError_t)e, "kernel launch");
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_refine_stats(sptrsv_plan plan, void *stream, int32_t *iterations, double *correction) {
    return guarded([&]() -> sptrsv_status {
        if (!plan || !iterations || !correction) return set_err(SPTRSV_ERR_ARG, "null argument");
        if (!plan->uploaded) return set_err(SPTRSV_ERR_STATE, "plan not uploaded");
        if (plan->precision != 32) return set_err(SPTRSV_ERR_STATE, "plan is stored in FP64");
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_err(e, "hipStreamSynchronize");
        sptrsv::Workspace w;
        e = hipMemcpy(&w, static_cast<unsigned char *>(plan->dev) + plan->layout.workspace, sizeof(w),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_err(e, "hipMemcpy");
        *iterations = (int32_t)w.iters;
        double r = 0.0;
        if (w.iters > 0) std::memcpy(&r, &w.ratio[w.iters - 1], sizeof(r));
        *correction = w.iters > 0 ? r : 0.0;
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_set_precision(sptrsv_plan plan, int32_t bits) {
    return guarded([&]() -> sptrsv_status {
        if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
        if (bits != 32 && bits != 64) return set_err(SPTRSV_ERR_ARG, "bits must be 32 or 64");
        if (bits == plan->precision) return SPTRSV_OK;
        const int old = plan->precision;
        plan->precision = bits;
        plan->uploaded = false;
        drop_graph(*plan);
        try {
            sptrsv::pack(*plan);
        } catch (...) {
            plan->precision = old;
            sptrsv::pack(*plan);
            throw;
        }
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_set_tiling(sptrsv_plan plan, int32_t terms_per_lane) {
    return guarded([&]() -> sptrsv_status {
        if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
        if (terms_per_lane < 1 || terms_per_lane > 16 || (terms_per_lane & (terms_per_lane - 1)))
            return set_err(SPTRSV_ERR_ARG, "terms_per_lane must be 1, 2, 4, 8 or 16");
        if (terms_per_lane == plan->terms_per_lane) return SPTRSV_OK;
        const int old = plan->terms_per_lane;
        plan->terms_per_lane = terms_per_lane;
        plan->uploaded = false;
        drop_graph(*plan);
        try {
            sptrsv::pack(*plan);
        } catch (...) {
            plan->terms_per_lane = old;
            sptrsv::pack(*plan);
            throw;
        }
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_set_queues(sptrsv_plan plan, int32_t queues) {
    return guarded([&]() -> sptrsv_status {
        if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
        if (queues != 1 && queues != 2) return set_err(SPTRSV_ERR_ARG, "queues must be 1 or 2");
        if (queues == plan->queues) return SPTRSV_OK;
        const int old = plan->queues;
        plan->queues = queues;
        plan->uploaded = false;
        drop_graph(*plan);
        try {
            sptrsv::pack(*plan);
        } catch (...) {
            plan->queues = old;
            sptrsv::pack(*plan);
            throw;
        }
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_set_rhs_mode(sptrsv_plan plan, int32_t mode) {
    return guarded([&]() -> sptrsv_status {
        if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
        if (mode != SPTRSV_RHS_AUTO && mode != SPTRSV_RHS_MPASS && mode != SPTRSV_RHS_STAGE)
            return set_err(SPTRSV_ERR_ARG, "unknown right-hand-side mode");
        const int32_t req = mode == SPTRSV_RHS_AUTO ? -1 : mode;
        if (req == plan->rhs_request) return SPTRSV_OK;
        const int32_t old = plan->rhs_request;
        plan->rhs_request = req;
        plan->uploaded = false;
        drop_graph(*plan);
        try {
            sptrsv::pack(*plan);
        } catch (...) {
            plan->rhs_request = old;
            sptrsv::pack(*plan);
            throw;
        }
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_solve_graph(sptrsv_plan plan, const double *b, double *x, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (solve_args_ok(plan, b, x, 64, sizeof(double))) return SPTRSV_OK;
        const int32_t n = plan->n;
        const sptrsv::LaunchShape sh = launch_shape(*plan), sub = sub_shape(*plan);
        if (!plan->graph_exec || plan->graph_b != b || plan->graph_x != x || plan->graph_waves != sh.waves ||
            plan->graph_chain_waves != sh.chain_waves) {
            drop_graph(*plan);
            hipError_t e;
            if (!plan->capture_stream) {
                hipStream_t cs = nullptr;
                e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_err(e, "hipStreamCreateWithFlags");
                plan->capture_stream = cs;
            }
            hipStream_t cs = static_cast<hipStream_t>(plan->capture_stream);
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_err(e, "hipStreamBeginCapture");
            const int le = sptrsv_launch_solve(static_cast<const unsigned char *>(plan->dev), &plan->layout, n,
                                               &sh, &sub, plan->wait_limit, b, x, nullptr, 0, cs);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cs, &g);
            if (le != 0) {
                if (g) hipGraphDestroy(g);
                return hip_err((hipError_t)le, "kernel launch under capture");
            }
            if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
            hipGraphExec_t ge = nullptr;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (e != hipSuccess) return hip_err(e, "hipGraphInstantiate");
            plan->graph_exec = ge;
            plan->graph_b = b;
            plan->graph_x = x;
            plan->graph_waves = sh.waves;
            plan->graph_chain_waves = sh.chain_waves;
        }
        hipError_t e = hipGraphLaunch(static_cast<hipGraphExec_t>(plan->graph_exec), static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_check(sptrsv_plan plan, void *stream, int32_t *device_status) {
    return guarded([&]() -> sptrsv_status {
        if (!plan || !device_status) return set_err(SPTRSV_ERR_ARG, "null argument");
        if (!plan->uploaded) return set_err(SPTRSV_ERR_STATE, "plan not uploaded");
        hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(e, "hipStreamSynchronize");
        unsigned char *ws = static_cast<unsigned char *>(plan->dev) + plan->layout.workspace;
        unsigned int st = 0;
        e = hipMemcpy(&st, ws + offsetof(sptrsv::Workspace, status), sizeof(st), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_err(e, "hipMemcpy");
        const unsigned int zero = 0;
        e = hipMemcpy(ws + offsetof(sptrsv::Workspace, status), &zero, sizeof(zero), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_err(e, "hipMemcpy");
        *device_status = st ? SPTRSV_ERR_TIMEOUT : 0;
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_set_launch(sptrsv_plan plan, int32_t waves_per_cu) {
    if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
    if (waves_per_cu < 0) return set_err(SPTRSV_ERR_ARG, "waves_per_cu < 0");
    if (waves_per_cu > sptrsv::kMaxWavesPerCU)
        return set_err(SPTRSV_ERR_ARG, "waves_per_cu above 8: co-residency of the grid is not proven there");
    plan->waves_per_cu = waves_per_cu;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_set_chain_share(sptrsv_plan plan, int32_t per_mille) {
    if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
    if (per_mille < 0 || per_mille > 1000) return set_err(SPTRSV_ERR_ARG, "per_mille must be in [0, 1000]");
    plan->chain_share = per_mille;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_launch_shape(sptrsv_plan plan, int32_t *waves, int32_t *chain_waves) {
    if (!plan || !waves || !chain_waves) return set_err(SPTRSV_ERR_ARG, "null argument");
    if (!plan->uploaded) return set_err(SPTRSV_ERR_STATE, "plan not uploaded");
    const sptrsv::LaunchShape sh = launch_shape(*plan);
    *waves = sh.waves;
    *chain_waves = sh.chain_waves;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_set_wait_limit(sptrsv_plan plan, uint64_t ticks) {
    if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
    plan->wait_limit = ticks;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_info(sptrsv_plan plan, sptrsv_info *o) {
    if (!plan || !o) return set_err(SPTRSV_ERR_ARG, "null argument");
    const sptrsv::Plan &p = *plan;
    std::memset(o, 0, sizeof(*o));
    o->n = p.n;
    o->levels = p.nlev;
    o->stages = p.nstages;
    o->levels_rw = p.nlev_rw;
    o->nnz = p.n ? p.rp[(size_t)p.n] : 0;
    o->nnz_rw = p.lp_ptr.empty() ? 0 : p.lp_ptr.back();
    o->nnz_m = p.nnz_m();
    o->flops = 2 * (o->nnz - p.n) + p.n;
    o->flops_rw = 2 * (o->nnz_rw - p.n + o->nnz_m) + p.n;
    const int64_t vb = p.precision / 8;
    o->bytes = (4 + vb) * o->nnz + (8 + 2 * vb) * (int64_t)p.n;
    o->rhs_mode = p.layout.rhs_mode;
    o->nnz_rhs = p.layout.nnz_rhs;
    // the solve of L' plus the right-hand-side step: M entries and b, b' per
    // row (M pass), or a whole solve of L_B (stage solves)
    o->nnz_streamed = p.nnz_streamed;
    o->bytes_rw = (4 + vb) * (o->nnz_streamed + o->nnz_rhs) + (8 + 2 * vb) * (int64_t)p.n - 2 * p.nnz_col16;
    if (p.layout.rhs_mode == sptrsv::kRhsMPass) o->bytes_rw += 2 * vb * (int64_t)p.n;
    if (p.layout.rhs_mode == sptrsv::kRhsStage) o->bytes_rw += (8 + 2 * vb) * (int64_t)p.n;
    o->device_bytes = (int64_t)p.layout.total;
    o->tiles = p.ntiles;
    o->precision = p.precision;
    o->seg_tiles = p.nseg_tiles;
    o->rhs_segments = p.sub ? p.sub->comp_segs : 0;
    o->reg_chunks = p.layout.reg_chunks;
    o->segments = p.nseg;
    o->ring_segments = p.ring_segs;
    o->chain_items = p.nchain;
    o->m_stored = p.m_kept ? 1 : 0;
    o->compact_cols = p.layout.col16;
    o->compact_terms = p.nnz_col16;
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_levels(sptrsv_plan plan, int32_t which, int32_t *level) {
    if (!plan || (!level && plan->n > 0)) return set_err(SPTRSV_ERR_ARG, "null argument");
    if (which != 0 && which != 1) return set_err(SPTRSV_ERR_ARG, "which must be 0 or 1");
    const std::vector<int32_t> &v = which ? plan->level_rw : plan->level;
    std::copy(v.begin(), v.end(), level);
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_stages(sptrsv_plan plan, int32_t *stage_of_level, int64_t *delta_of_level) {
    if (!plan) return set_err(SPTRSV_ERR_ARG, "plan is NULL");
    if (stage_of_level) std::copy(plan->stage_of_level.begin(), plan->stage_of_level.end(), stage_of_level);
    if (delta_of_level) std::copy(plan->delta_of_level.begin(), plan->delta_of_level.end(), delta_of_level);
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_schedule(sptrsv_plan plan, int32_t *level_ptr, int32_t *rows) {
    if (!plan || !level_ptr || (!rows && plan->n > 0)) return set_err(SPTRSV_ERR_ARG, "null argument");
    std::copy(plan->sched_ptr.begin(), plan->sched_ptr.end(), level_ptr);
    std::copy(plan->sched_rows.begin(), plan->sched_rows.end(), rows);
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_export(sptrsv_plan plan, int64_t *lp_ptr, int32_t *lp_col, double *lp_val,
                                 int64_t *m_ptr, int32_t *m_col, double *m_val) {
    return guarded([&]() -> sptrsv_status {
        if (!plan || !lp_ptr) return set_err(SPTRSV_ERR_ARG, "null argument");
        sptrsv::Plan &p = *plan;
        if ((!lp_col || !lp_val) && !p.lp_col.empty()) return set_err(SPTRSV_ERR_ARG, "null L' arrays");
        if (m_ptr && (!m_col || !m_val) && p.nnz_m() > 0) return set_err(SPTRSV_ERR_ARG, "null M arrays");
        if (m_ptr) sptrsv::materialise_m(p);
        std::copy(p.lp_ptr.begin(), p.lp_ptr.end(), lp_ptr);
        std::copy(p.lp_col.begin(), p.lp_col.end(), lp_col);
        std::copy(p.lp_val.begin(), p.lp_val.end(), lp_val);
        if (!m_ptr) return SPTRSV_OK;  // L' only
        std::copy(p.m_ptr.begin(), p.m_ptr.end(), m_ptr);
        std::copy(p.m_col.begin(), p.m_col.end(), m_col);
        std::copy(p.m_val.begin(), p.m_val.end(), m_val);
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_solve_stamped(sptrsv_plan plan, const double *b, double *x, uint64_t *stamps, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (solve_args_ok(plan, b, x, 64, sizeof(double))) return SPTRSV_OK;
        if (!stamps) return set_err(SPTRSV_ERR_ARG, "stamps is NULL");
        const sptrsv::LaunchShape sh = launch_shape(*plan), sub = sub_shape(*plan);
        const int e = sptrsv_launch_solve(static_cast<const unsigned char *>(plan->dev), &plan->layout, plan->n,
                                          &sh, &sub, plan->wait_limit, b, x,
                                          reinterpret_cast<unsigned long long *>(stamps),
                                          plan->ntiles + plan->nseg_tiles, stream);
        if (e != 0) return hip_err((hipError_t)e, "kernel launch");
        return SPTRSV_OK;
    });
}

sptrsv_status sptrsv_plan_stamp_levels(sptrsv_plan plan, int32_t *level) {
    if (!plan || (!level && !plan->stamp_level.empty())) return set_err(SPTRSV_ERR_ARG, "null argument");
    std::copy(plan->stamp_level.begin(), plan->stamp_level.end(), level);
    return SPTRSV_OK;
}

sptrsv_status sptrsv_plan_level_features(sptrsv_plan plan, float *features) {
    if (!plan || (!features && plan->nlev_rw > 0)) return set_err(SPTRSV_ERR_ARG, "null argument");
    const sptrsv::Plan &p = *plan;
    for (int32_t l = 0; l < p.nlev_rw; ++l) {
        sptrsv::GroupShape g;
        int32_t lo = INT32_MAX, hi = -1;
        for (int32_t q = p.sched_ptr[(size_t)l]; q < p.sched_ptr[(size_t)l + 1]; ++q) {
            const int32_t i = p.sched_rows[(size_t)q];
            const int64_t len = (p.lp_ptr[(size_t)i + 1] - p.lp_ptr[(size_t)i]) +
                                (p.m_ptr[(size_t)i + 1] - p.m_ptr[(size_t)i]);
            ++g.rows;
            g.terms += len;
            g.orig += p.rp[(size_t)i + 1] - p.rp[(size_t)i];
            g.maxlen = std::max(g.maxlen, len);
            lo = std::min(lo, p.level[(size_t)i]);
            hi = std::max(hi, p.level[(size_t)i]);
        }
        g.span = hi >= lo ? hi - lo + 1 : 1;
        sptrsv::group_features(g, features + (size_t)l * sptrsv::kFeatures);
    }
    return SPTRSV_OK;
}

sptrsv_status sptrsv_mlp_forward(const float *params, const float *x, float *y, int32_t m, void *stream) {
    if (m < 0) return set_err(SPTRSV_ERR_ARG, "m < 0");
    if (m == 0) return SPTRSV_OK;
    if (!params || !x || !y) return set_err(SPTRSV_ERR_ARG, "null argument");
    const int e = sptrsv_launch_mlp_forward(params, x, y, m, stream);
    if (e != 0) return hip_err((hipError_t)e, "kernel launch");
    return SPTRSV_OK;
}

sptrsv_status sptrsv_mlp_grad_workspace(int32_t m, size_t *bytes) {
    if (m < 1 || !bytes) return set_err(SPTRSV_ERR_ARG, "m < 1 or bytes NULL");
    *bytes = sptrsv_launch_mlp_workspace(m);
    return SPTRSV_OK;
}

sptrsv_status sptrsv_mlp_grad(const float *params, const float *x, const float *t, int32_t m, float *grad,
                              float *loss, void *workspace, size_t workspace_bytes, void *stream) {
    if (m < 1) return set_err(SPTRSV_ERR_ARG, "m < 1");
    if (!params || !x || !t || !grad || !workspace) return set_err(SPTRSV_ERR_ARG, "null argument");
    if (workspace_bytes < sptrsv_launch_mlp_workspace(m)) return set_err(SPTRSV_ERR_ARG, "workspace too small");
    const int e = sptrsv_launch_mlp_grad(params, x, t, m, grad, loss, workspace, stream);
    if (e != 0) return hip_err((hipError_t)e, "kernel launch");
    return SPTRSV_OK;
}

sptrsv_status sptrsv_mlp_grad_noalloc(const float *params, const float *x, const float *t, int32_t m,
                                      float *grad, float *loss, void *stream) {
    if (m < 1) return set_err(SPTRSV_ERR_ARG, "m < 1");
    if (m > SPTRSV_MLP_NOALLOC_MAX_SAMPLES)
        return set_err(SPTRSV_ERR_ARG, "m above SPTRSV_MLP_NOALLOC_MAX_SAMPLES (8192): the static workspace "
                                       "is too small; use sptrsv_mlp_grad with a workspace");
    if (!params || !x || !t || !grad) return set_err(SPTRSV_ERR_ARG, "null argument");
    void *ws = nullptr;
    size_t bytes = 0;
    int e = sptrsv_mlp_static_workspace(&ws, &bytes);
    if (e != 0) return hip_err((hipError_t)e, "static workspace");
    if (bytes < sptrsv_launch_mlp_workspace(m)) return set_err(SPTRSV_ERR_ARG, "static workspace too small");
    e = sptrsv_launch_mlp_grad(params, x, t, m, grad, loss, ws, stream);
    if (e != 0) return hip_err((hipError_t)e, "kernel launch");
    return SPTRSV_OK;
}

sptrsv_status sptrsv_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step, float lr,
                              float beta1, float beta2, float eps, void *stream) {
    if (!params || !grad || !m1 || !m2) return set_err(SPTRSV_ERR_ARG, "null argument");
    if (step < 1) return set_err(SPTRSV_ERR_ARG, "step < 1");
    const int e = sptrsv_launch_mlp_adam(params, grad, m1, m2, step, lr, beta1, beta2, eps, stream);
    if (e != 0) return hip_err((hipError_t)e, "kernel launch");
    return SPTRSV_OK;
}

sptrsv_status sptrsv_probe_hop(int32_t hops, int32_t same_xcd, void *dev_scratch, size_t bytes,
                               double *ns_per_hop, void *stream) {
    return guarded([&]() -> sptrsv_status {
        if (!dev_scratch || !ns_per_hop) return set_err(SPTRSV_ERR_ARG, "null argument");
        if (bytes < 32) return set_err(SPTRSV_ERR_ARG, "scratch smaller than 32 bytes");
        if (reinterpret_cast<uintptr_t>(dev_scratch) % 8 != 0)
            return set_err(SPTRSV_ERR_ARG, "scratch not 8-byte aligned");
        if (hops < 2 || hops > (1 << 24)) return set_err(SPTRSV_ERR_ARG, "hops must be in [2, 2^24]");
        const int partner = same_xcd ? 8 : 1;
        // 100 ms per wait at 100 MHz: far above any hop, so only a lost
        // partner ends the probe early
        int e = sptrsv_launch_hop_probe(dev_scratch, hops, partner, 10000000ull, stream);
        if (e != 0) return hip_err((hipError_t)e, "hop probe launch");
        hipError_t he = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (he != hipSuccess) return hip_err(he, "hipStreamSynchronize");
        unsigned long long out[2] = {0, 0};
        he = hipMemcpy(out, static_cast<unsigned long long *>(dev_scratch) + 2, sizeof(out), hipMemcpyDeviceToHost);
        if (he != hipSuccess) return hip_err(he, "hipMemcpy");
        if (out[1]) return set_err(SPTRSV_ERR_TIMEOUT, "hop probe: a wait passed its limit");
        *ns_per_hop = (double)out[0] * 10.0 / hops;  // 100 MHz ticks
        return SPTRSV_OK;
    });
}

void sptrsv_plan_destroy(sptrsv_plan plan) { delete plan; }

const char *sptrsv_last_error(void) { return g_err.c_str(); }

}  // extern "C"
