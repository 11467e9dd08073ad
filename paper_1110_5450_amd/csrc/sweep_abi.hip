// sweep_abi.hip -- the C ABI declared in include/sweep.h: host-side
// validation, workspace layout and stream-ordered launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sweep.h"
#include "abi_internal.hpp"
#include "kernels.hpp"

namespace sweep {

// ----------------------------------------------------------------- trace

struct TraceState {
    int capacity = 0;   // calls still to record
    int used = 0;       // events in use
    hipEvent_t ev[3 * 4096];
    int calls = 0;
};
static TraceState g_trace;

static bool trace_active() { return g_trace.capacity > 0; }

// Records event k of the current call (k = 0 start, 1 frame done, 2 surface done).
static void trace_mark(int k, hipStream_t st)
{
    if (!trace_active()) return;
    const int idx = 3 * g_trace.calls + k;
    hipEventRecord(g_trace.ev[idx], st);
    if (k == 2) {
        ++g_trace.calls;
        --g_trace.capacity;
    }
}

// Parameter domain [U_p, U_n] of an open curve (given knots or [0, 1]).
static double domain_length(const sweep_curve* c)
{
    if (!c->knots) return 1.0;
    return c->knots[c->n_ctrl] - c->knots[c->degree];
}

// ----------------------------------------------------------------- tuning

// Shape class of a single sweep for the tuning table: output precision,
// n_v a multiple of 256, floor(log2 n_v), floor(log2 n_u*n_v).
static void single_class(int n_u, int n_v, int t64, int* cls)
{
    const int c[kTuneClassInts] = {t64, n_v % 256 == 0 ? 1 : 0, ilog2_ll(n_v), ilog2_ll((long long)n_u * n_v), 0};
    for (int k = 0; k < kTuneClassInts; ++k) cls[k] = c[k];
}

// Built-in rule (nontemporal stores measured 15-25 % faster for this
// write-once output): column tiles of one row when n_v fills whole
// 256-column tiles, otherwise the linear kernel with 4 vertices per lane.
static SurfaceConfig rule_surface_config(int n_v)
{
    if (n_v % 256 == 0) return SurfaceConfig{0, 1, 0, 1};
    return SurfaceConfig{1, 0, 1024, 1};
}

SurfaceConfig auto_surface_config(int n_u, int n_v, int t64)
{
    int cls[kTuneClassInts];
    single_class(n_u, n_v, t64, cls);
    const int c = tune_lookup("single", cls);
    return c >= 0 ? tile_config(c) : rule_surface_config(n_v);
}

// ---------------------------------------------------------- workspace plan

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct SingleLayout {
    size_t knots_path, knots_prof, trec, chunk_lv, chunk_tl, chunk_fix, fallback, agg, r_in, rows, prof_tab, knots_law;
    size_t arc_len, arc_cum, arc_u, arc_span, total;
};

// rl: values per row record (16, or kRowExt with a frame mode or law);
// nlk: knots of the law curve (0 without a law or with its default knots).
static SingleLayout single_layout(int np, int pp, int nq, int pq, int qclosed, int n_u, int n_v, size_t fsz, size_t tsz,
                                  int rl = 16, int nlk = 0, bool arclength = false)
{
    SingleLayout L{};
    const int nc = frame_chunks(n_u);
    size_t off = 0;
    L.knots_path = off; off = align_up(off + sizeof(double) * nknots(np, pp, 0));
    L.knots_prof = off; off = align_up(off + sizeof(double) * nknots(nq, pq, qclosed));
    L.trec = off;       off = align_up(off + sizeof(double) * kRunRec * (size_t)kBlock * (size_t)nc);
    L.chunk_lv = off;   off = align_up(off + sizeof(int) * (size_t)nc);
    L.chunk_tl = off;   off = align_up(off + sizeof(double) * 3 * (size_t)nc);
    L.chunk_fix = off;  off = align_up(off + sizeof(int) * (size_t)nc);
    L.fallback = off;   off = align_up(off + sizeof(double) * 3);
    L.agg = off;        off = align_up(off + fsz * 9 * (size_t)nc);
    L.r_in = off;       off = align_up(off + fsz * 3 * (size_t)nc);
    L.rows = off;       off = align_up(off + tsz * (size_t)rl * (size_t)n_u);
    L.prof_tab = off;   off = align_up(off + tsz * 8 * (size_t)n_v);
    L.knots_law = off;  off = align_up(off + sizeof(double) * (size_t)nlk);
    const size_t npc = arclength ? (size_t)(np - pp) * 32 : 0;   // pieces of the arc-length table
    L.arc_len = off;    off = align_up(off + sizeof(double) * npc);
    L.arc_cum = off;    off = align_up(off + sizeof(double) * (arclength ? npc + 1 : 0));
    L.arc_u = off;      off = align_up(off + sizeof(double) * (arclength ? (size_t)n_u : 0));
    L.arc_span = off;   off = align_up(off + sizeof(int) * (arclength ? (size_t)n_u : 0));
    L.total = off;
    return L;
}

static SingleLayout layout_for(const sweep_curve* path, const sweep_curve* prof, int n_u, int n_v,
                               const sweep_options* o)
{
    const size_t fsz = o->frame_precision == SWEEP_F64 ? 8 : 4;
    const size_t tsz = o->out_precision == SWEEP_F64 ? 8 : 4;
    const int nlk = (o->law && o->law->knots) ? nknots(o->law->n_ctrl, o->law->degree, 0) : 0;
    return single_layout(path->n_ctrl, path->degree, prof->n_ctrl, prof->degree, prof->closed, n_u, n_v, fsz, tsz,
                         options_ext(o) ? kRowExt : 16, nlk, o->u_sampling != SWEEP_U_PARAMETER);
}

static FrameWork frame_work(char* ws, const SingleLayout& L)
{
    return FrameWork{(double*)(ws + L.trec), (int*)(ws + L.chunk_lv), (double*)(ws + L.chunk_tl),
                     (int*)(ws + L.chunk_fix), (double*)(ws + L.fallback), ws + L.agg, ws + L.r_in};
}

// Copies given knots to the device (a blocking copy from pageable memory);
// default knots are computed on the fly by the kernels (dst unused).
sweep_status upload_knots(const double* host_knots, int n, int p, double* dst, hipStream_t st)
{
    if (!host_knots) return SWEEP_OK;
    hipError_t e = hipMemcpyAsync(dst, host_knots, sizeof(double) * nknots(n, p, 0), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "knots");
    return SWEEP_OK;
}

// Arc-length sampling: tabulates the path's sample parameters and spans in
// the workspace and points the curve at them.
static sweep_status setup_arclength(DCurve& dp, int n_u, const sweep_options* o, char* ws, const SingleLayout& L,
                                    hipStream_t st)
{
    if (o->u_sampling == SWEEP_U_PARAMETER) return SWEEP_OK;
    double* su = (double*)(ws + L.arc_u);
    int* ss = (int*)(ws + L.arc_span);
    const double lam = o->u_sampling == SWEEP_U_ADAPTIVE ? o->u_lambda : 0.0;
    hipError_t e = launch_arclength(dp, n_u, lam, (double*)(ws + L.arc_len), (double*)(ws + L.arc_cum), su, ss, st);
    if (e != hipSuccess) return hip_fail(e, "arc-length sampling");
    dp.su = su;
    dp.ss = ss;
    return SWEEP_OK;
}

// Frame stage only: knots, path samples and the frame scan into `rows`.
template <class F, class T>
static sweep_status run_frames(const sweep_curve* path, int n_u, const sweep_options* o, T* rows, char* ws,
                               const SingleLayout& L, hipStream_t st)
{
    double* Up = (double*)(ws + L.knots_path);
    sweep_status s = upload_knots(path->knots, path->n_ctrl, path->degree, Up, st);
    if (s != SWEEP_OK) return s;
    DCurve dp{path->ctrl, path->knots ? Up : nullptr, path->n_ctrl, path->degree, 0,
              nbasis(path->n_ctrl, path->degree, 0), path->weights};
    DCurve dq{nullptr, nullptr, 1, 1, 0, 1, nullptr};
    if ((s = setup_arclength(dp, n_u, o, ws, L, st)) != SWEEP_OK) return s;
    const FrameWork w = frame_work(ws, L);
    hipError_t e = launch_prep<F, T>(dp, n_u, dq, 0, w, (T*)nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "curve samples");
    InitialNormal n0{o->has_initial_normal, {o->initial_normal[0], o->initial_normal[1], o->initial_normal[2]}};
    e = launch_frame<F, T>(dp, n_u, w, n0, o->reorthonormalize, rows, st);
    if (e != hipSuccess) return hip_fail(e, "frame");
    return SWEEP_OK;
}

template <class F, class T>
static sweep_status run_single(const sweep_curve* path, const sweep_curve* prof, int n_u, int n_v,
                               const sweep_options* o, void* pos, void* nrm, char* ws, const SingleLayout& L,
                               hipStream_t st)
{
    double* Up = (double*)(ws + L.knots_path);
    double* Uq = (double*)(ws + L.knots_prof);
    sweep_status s = upload_knots(path->knots, path->n_ctrl, path->degree, Up, st);
    if (s != SWEEP_OK) return s;
    s = upload_knots(prof->knots, prof->n_ctrl, prof->degree, Uq, st);
    if (s != SWEEP_OK) return s;
    trace_mark(0, st);
    DCurve dp{path->ctrl, path->knots ? Up : nullptr, path->n_ctrl, path->degree, 0,
              nbasis(path->n_ctrl, path->degree, 0), path->weights};
    DCurve dq{prof->ctrl, prof->knots ? Uq : nullptr, prof->n_ctrl, prof->degree, prof->closed,
              nbasis(prof->n_ctrl, prof->degree, prof->closed), prof->weights};
    if ((s = setup_arclength(dp, n_u, o, ws, L, st)) != SWEEP_OK) return s;
    const FrameWork w = frame_work(ws, L);
    T* rows = (T*)(ws + L.rows);
    T* ptab = (T*)(ws + L.prof_tab);
    hipError_t e = launch_prep<F, T>(dp, n_u, dq, n_v, w, ptab, st);
    if (e != hipSuccess) return hip_fail(e, "curve samples");
    InitialNormal n0{o->has_initial_normal, {o->initial_normal[0], o->initial_normal[1], o->initial_normal[2]}};
    const bool ext = options_ext(o);
    FrameExt fx{};
    if (ext) {
        fx.frenet = o->frame_mode == SWEEP_FRAME_FRENET;
        if (o->law) {
            const sweep_curve* lc = o->law;
            double* Ul = (double*)(ws + L.knots_law);
            if ((s = upload_knots(lc->knots, lc->n_ctrl, lc->degree, Ul, st)) != SWEEP_OK) return s;
            fx.law = DCurve{lc->ctrl, lc->knots ? Ul : nullptr, lc->n_ctrl, lc->degree, 0,
                            nbasis(lc->n_ctrl, lc->degree, 0), lc->weights};
            fx.has_law = 1;
            fx.du_scale = domain_length(lc) / domain_length(path);
        }
    }
    e = launch_frame<F, T>(dp, n_u, w, n0, o->reorthonormalize, rows, st, ext ? &fx : nullptr);
    if (e != hipSuccess) return hip_fail(e, "frame");
    trace_mark(1, st);
    const SurfaceConfig cfg = o->tile_config >= 0 ? tile_config(o->tile_config)
                                                   : auto_surface_config(n_u, n_v, o->out_precision == SWEEP_F64);
    e = launch_surface<T>(rows, ptab, n_u, n_v, (T*)pos, (T*)nrm, cfg, st, ext);
    if (e != hipSuccess) return hip_fail(e, "surface");
    trace_mark(2, st);
    return SWEEP_OK;
}

}  // namespace sweep

using namespace sweep;

extern "C" {

size_t sweep_eval_workspace_size(const sweep_curve* path, const sweep_curve* profile, int32_t n_u, int32_t n_v,
                                 const sweep_options* opt)
{
    if (!path || !profile || !opt) return 0;
    if (check_curve_meta(path->n_ctrl, path->degree, path->closed, path->knots, "path", true) != SWEEP_OK) return 0;
    if (check_curve_meta(profile->n_ctrl, profile->degree, profile->closed, profile->knots, "profile", false) != SWEEP_OK) return 0;
    if (check_grid(n_u, n_v) != SWEEP_OK || check_options(opt) != SWEEP_OK) return 0;
    return layout_for(path, profile, n_u, n_v, opt).total;
}

sweep_status sweep_eval(const sweep_curve* path, const sweep_curve* profile, int32_t n_u, int32_t n_v,
                        const sweep_options* opt, void* pos, void* nrm, void* workspace, size_t ws_bytes,
                        void* stream)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    sweep_status s = check_options(opt);
    if (s != SWEEP_OK) return s;
    if ((s = check_curve(path, "path", true)) != SWEEP_OK) return s;
    if ((s = check_curve(profile, "profile", false)) != SWEEP_OK) return s;
    if ((s = check_grid(n_u, n_v)) != SWEEP_OK) return s;
    if (!pos) return fail(SWEEP_ERR_NULL_ARG, "pos is NULL");
    const SingleLayout L = layout_for(path, profile, n_u, n_v, opt);
    if (!workspace || ws_bytes < L.total)
        return fail(SWEEP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu required", workspace ? ws_bytes : (size_t)0, L.total);
    if (((uintptr_t)workspace) % 256 != 0) return fail(SWEEP_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    const bool f64 = opt->frame_precision == SWEEP_F64, t64 = opt->out_precision == SWEEP_F64;
    if (f64 && t64) return run_single<double, double>(path, profile, n_u, n_v, opt, pos, nrm, ws, L, st);
    if (f64) return run_single<double, float>(path, profile, n_u, n_v, opt, pos, nrm, ws, L, st);
    if (t64) return run_single<float, double>(path, profile, n_u, n_v, opt, pos, nrm, ws, L, st);
    return run_single<float, float>(path, profile, n_u, n_v, opt, pos, nrm, ws, L, st);
}

sweep_status sweep_trace_enable(int32_t max_calls)
{
    const int cap = (int)(sizeof g_trace.ev / sizeof g_trace.ev[0]) / 3;
    if (max_calls < 0 || max_calls > cap) return fail(SWEEP_ERR_BAD_OPTION, "trace length %d outside 0..%d", max_calls, cap);
    if (max_calls == 0) { g_trace.capacity = 0; return SWEEP_OK; }
    if (g_trace.calls != 0) return fail(SWEEP_ERR_BAD_OPTION, "read the previous trace first");
    for (int k = g_trace.used; k < 3 * max_calls; ++k) {
        // timing-only events: no system-scope fence (cache write-back) when
        // they complete, so tracing does not slow the traced work
        hipError_t e = hipEventCreateWithFlags(&g_trace.ev[k], hipEventDisableSystemFence);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        g_trace.used = k + 1;
    }
    g_trace.capacity = max_calls;
    return SWEEP_OK;
}

int32_t sweep_trace_read(int32_t* stage, float* ms, int32_t max)
{
    int n = 0;
    for (int c = 0; c < g_trace.calls; ++c) {
        for (int k = 0; k < 2; ++k) {
            hipError_t e = hipEventSynchronize(g_trace.ev[3 * c + k + 1]);
            if (e != hipSuccess) return hip_fail(e, "trace read");
            float t = 0.f;
            e = hipEventElapsedTime(&t, g_trace.ev[3 * c + k], g_trace.ev[3 * c + k + 1]);
            if (e != hipSuccess) return hip_fail(e, "trace read");
            if (n < max && stage && ms) { stage[n] = k; ms[n] = t; ++n; }
        }
    }
    g_trace.calls = 0;
    g_trace.capacity = 0;
    return n;
}

size_t sweep_frames_workspace_size(const sweep_curve* path, int32_t n_u, const sweep_options* opt)
{
    if (!path || !opt) return 0;
    if (check_curve_meta(path->n_ctrl, path->degree, path->closed, path->knots, "path", true) != SWEEP_OK) return 0;
    if (n_u < 2 || check_options(opt) != SWEEP_OK) return 0;
    const size_t fsz = opt->frame_precision == SWEEP_F64 ? 8 : 4;
    return single_layout(path->n_ctrl, path->degree, 4, 3, 1, n_u, 0, fsz, 0, 16, 0,
                         opt->u_sampling != SWEEP_U_PARAMETER).total;
}

sweep_status sweep_frames(const sweep_curve* path, int32_t n_u, const sweep_options* opt, void* frames,
                          void* workspace, size_t ws_bytes, void* stream)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    sweep_status s = check_options(opt);
    if (s != SWEEP_OK) return s;
    if ((s = check_curve(path, "path", true)) != SWEEP_OK) return s;
    if (options_ext(opt)) return fail(SWEEP_ERR_UNSUPPORTED, "sweep_frames: frame modes and laws are sweep_eval only");
    const bool arc = opt->u_sampling != SWEEP_U_PARAMETER;
    if (n_u < 2 || n_u >= (1 << 30)) return fail(SWEEP_ERR_BAD_GRID, "n_u %d outside 2..2^30-1", n_u);
    if (!frames) return fail(SWEEP_ERR_NULL_ARG, "frames is NULL");
    const size_t fsz = opt->frame_precision == SWEEP_F64 ? 8 : 4;
    const SingleLayout L = single_layout(path->n_ctrl, path->degree, 4, 3, 1, n_u, 0, fsz, 0, 16, 0, arc);
    if (!workspace || ws_bytes < L.total)
        return fail(SWEEP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu required", workspace ? ws_bytes : (size_t)0, L.total);
    if (((uintptr_t)workspace) % 256 != 0) return fail(SWEEP_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    const bool f64 = opt->frame_precision == SWEEP_F64, t64 = opt->out_precision == SWEEP_F64;
    if (f64 && t64) return run_frames<double, double>(path, n_u, opt, (double*)frames, ws, L, st);
    if (f64) return run_frames<double, float>(path, n_u, opt, (float*)frames, ws, L, st);
    if (t64) return run_frames<float, double>(path, n_u, opt, (double*)frames, ws, L, st);
    return run_frames<float, float>(path, n_u, opt, (float*)frames, ws, L, st);
}

sweep_status sweep_autotune(const sweep_curve* path, const sweep_curve* profile, int32_t n_u, int32_t n_v,
                            const sweep_options* opt, void* pos, void* nrm, void* workspace, size_t ws_bytes,
                            void* stream, int32_t* best_config, float* best_ms)
{
    sweep_options o;
    if (opt) o = *opt; else sweep_default_options(&o);
    o.tile_config = -1;
    sweep_status s = sweep_eval(path, profile, n_u, n_v, &o, pos, nrm, workspace, ws_bytes, stream);
    if (s != SWEEP_OK) return s;
    const SingleLayout L = layout_for(path, profile, n_u, n_v, &o);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev0, ev1;
    hipError_t e;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "autotune");
    if ((e = hipEventCreate(&ev1)) != hipSuccess) { hipEventDestroy(ev0); return hip_fail(e, "autotune"); }
    const bool t64 = o.out_precision == SWEEP_F64;
    const char* ws = (const char*)workspace;
    int best = -1;
    float best_t = 0.f;
    const int reps = 5;
    for (int c = 0; c < tile_config_count() && e == hipSuccess; ++c) {
        const SurfaceConfig& cfg = tile_config(c);
        auto run = [&]() -> hipError_t {
            return t64 ? launch_surface<double>((const double*)(ws + L.rows), (const double*)(ws + L.prof_tab), n_u,
                                                n_v, (double*)pos, (double*)nrm, cfg, st, options_ext(&o))
                       : launch_surface<float>((const float*)(ws + L.rows), (const float*)(ws + L.prof_tab), n_u, n_v,
                                               (float*)pos, (float*)nrm, cfg, st, options_ext(&o));
        };
        if ((e = run()) != hipSuccess) break;   // warm-up
        if ((e = hipEventRecord(ev0, st)) != hipSuccess) break;
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
        if (e != hipSuccess || (e = hipEventRecord(ev1, st)) != hipSuccess || (e = hipEventSynchronize(ev1)) != hipSuccess)
            break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) break;
        ms /= reps;
        if (best < 0 || ms < best_t) { best = c; best_t = ms; }
    }
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    {
        int cls[kTuneClassInts];
        single_class(n_u, n_v, t64, cls);
        tune_record("single", cls, best, best_t);
    }
    if (best_config) *best_config = best;
    if (best_ms) *best_ms = best_t;
    return SWEEP_OK;
}

int32_t sweep_surface_config_for(int32_t n_u, int32_t n_v, int32_t out_precision)
{
    const SurfaceConfig c = auto_surface_config(n_u, n_v, out_precision == SWEEP_F64);
    for (int k = 0; k < tile_config_count(); ++k) {
        const SurfaceConfig& t = tile_config(k);
        if (t.kind == c.kind && t.rows_per_block == c.rows_per_block && t.tile_vertices == c.tile_vertices &&
            t.nontemporal == c.nontemporal)
            return k;
    }
    return -1;
}

sweep_status sweep_triangles(int32_t n_u, int32_t n_v, int32_t closed_v, int32_t* tri, int64_t max_tri,
                             int64_t* n_tri, void* stream)
{
    if (closed_v != 0 && closed_v != 1) return fail(SWEEP_ERR_BAD_OPTION, "closed_v %d is not 0/1", closed_v);
    sweep_status s = check_grid(n_u, n_v);
    if (s != SWEEP_OK) return s;
    const long long nt = 2LL * (n_u - 1) * (closed_v ? n_v : n_v - 1);
    if (n_tri) *n_tri = nt;
    if (!tri) return fail(SWEEP_ERR_NULL_ARG, "tri is NULL");
    if (max_tri < nt) return fail(SWEEP_ERR_WORKSPACE, "tri holds %lld triangles, %lld needed", (long long)max_tri, nt);
    const hipError_t e = launch_triangles(n_u, n_v, closed_v, tri, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "triangles");
    return SWEEP_OK;
}

}  // extern "C"
