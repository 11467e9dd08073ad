// batched_abi.hip -- sweep_eval_batched and sweep_backward: plans keyed by
// batch shape, each holding the per-sweep descriptors, the per-degree sweep
// lists and the surface tile list in device memory, and a HIP graph
// (profile tables and one frame node per path degree, then the surface)
// that is replayed per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <vector>

#include "abi_internal.hpp"
#include "arclength.hpp"

namespace sweep {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }
static long long plane_stride(long long n) { return (n + kPlaneAlign - 1) / kPlaneAlign * kPlaneAlign; }

// Validated, flattened metadata of a batch plus the options that shape the
// kernels; equality of two keys means the same plan applies.
struct BatchKey {
    int device = 0;
    std::vector<int32_t> ints;     // per sweep: n_path p_path n_prof p_prof closed n_u n_v, then option ints
    std::vector<double> dbls;      // knots, initial normal
    bool operator==(const BatchKey& o) const { return device == o.device && ints == o.ints && dbls == o.dbls; }
};

struct BatchLayout {
    size_t rows, ptab, arc_len, arc_cum, arc_u, arc_s, total;
    long long n_rows = 0, n_vs = 0, n_vertices = 0, n_out = 0;
    long long n_rowpart = 0, n_colpart = 0, n_units = 0, n_uchunks = 0;
    long long n_arc = 0;           // arc-length pieces of all paths
};

// Workspace of sweep_backward (FP64 frame recomputation and adjoint buffers).
struct BackwardLayout {
    size_t rows, ptab, rowpart, colpart, rowacc, colacc, rho, ctot, sgrad, spans_u, qgrad, spans_v;
    size_t xstash, recu, recv, total;
};

static BackwardLayout backward_layout(const BatchLayout& L)
{
    BackwardLayout B{};
    size_t off = 0;
    auto seg = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    B.rows = seg(8 * 16 * (size_t)L.n_rows);
    B.ptab = seg(8 * 8 * (size_t)L.n_vs);
    // sized for the normal terms (the longer partial records)
    B.rowpart = seg(8 * kRowPartNrm * (size_t)L.n_rowpart);
    B.colpart = seg(8 * kColPartNrm * (size_t)L.n_colpart);
    B.rowacc = seg(8 * kRowPartNrm * (size_t)L.n_rows);
    B.colacc = seg(8 * kColPartNrm * (size_t)L.n_vs);
    B.rho = seg(8 * 3 * (size_t)L.n_rows);
    B.ctot = seg(8 * 3 * (size_t)L.n_uchunks);
    B.sgrad = seg(8 * 24 * (size_t)L.n_rows);
    B.spans_u = seg(4 * (size_t)L.n_rows);
    B.qgrad = seg(8 * 24 * (size_t)L.n_vs);
    B.spans_v = seg(4 * (size_t)L.n_vs);
    // knot and weight gradients: per-sample adjoints and records
    B.xstash = seg(8 * 9 * (size_t)L.n_rows);
    B.recu = seg(8 * 24 * (size_t)L.n_rows);
    B.recv = seg(8 * 24 * (size_t)L.n_vs);
    B.total = off;
    return B;
}

static sweep_status check_batch(const sweep_batch* b, const sweep_options* o, BatchKey* key, BatchLayout* lay,
                                std::vector<BatchDesc>* descs, std::vector<double>* knots)
{
    if (!b) return fail(SWEEP_ERR_NULL_ARG, "batch is NULL");
    if (!o) return fail(SWEEP_ERR_NULL_ARG, "options are NULL");
    sweep_status st = check_options(o);
    if (st != SWEEP_OK) return st;
    const bool arc = o->u_sampling != SWEEP_U_PARAMETER;
    if (arc && (options_ext(o) || o->frame_precision != SWEEP_F64))
        return fail(SWEEP_ERR_UNSUPPORTED, "arc-length sampling in a batch needs the FP64 frame, without a frame mode or law");
    if (options_ext(o) && o->frame_precision != SWEEP_F64)
        return fail(SWEEP_ERR_UNSUPPORTED, "frame modes and laws in a batch need the FP64 frame");
    if (b->n_sweeps < 1) return fail(SWEEP_ERR_BAD_COUNT, "n_sweeps %d < 1", b->n_sweeps);
    if (o->batch_stages < 0 || o->batch_stages > 4)
        return fail(SWEEP_ERR_BAD_OPTION, "batch_stages %d outside 0..4", o->batch_stages);
    if (!b->path_n || !b->path_degree || !b->prof_n || !b->prof_degree || !b->n_u || !b->n_v)
        return fail(SWEEP_ERR_NULL_ARG, "a per-sweep array is NULL");
    const size_t tsz = o->out_precision == SWEEP_F64 ? 8 : 4;
    long long path_off = 0, prof_off = 0, pk_off = 0, qk_off = 0;
    BatchLayout L{};
    if (key) key->ints.reserve(7 * (size_t)b->n_sweeps + 8);
    for (int k = 0; k < b->n_sweeps; ++k) {
        const int np = b->path_n[k], pp = b->path_degree[k], nq = b->prof_n[k], pq = b->prof_degree[k];
        const int qc = b->prof_closed ? b->prof_closed[k] : 1;
        const int nu = b->n_u[k], nv = b->n_v[k];
        // (the sweep index is added to the message on the error path only:
        // this runs for every sweep on every call)
        const double* pk = b->path_knots ? b->path_knots + pk_off : nullptr;
        if ((st = check_curve_meta(np, pp, 0, pk, "path", true)) != SWEEP_OK)
            return fail(st, "sweep %d %s", k, sweep_last_error());
        const double* qk = (b->prof_knots && !qc) ? b->prof_knots + qk_off : nullptr;
        if ((st = check_curve_meta(nq, pq, qc, qk, "profile", false)) != SWEEP_OK)
            return fail(st, "sweep %d %s", k, sweep_last_error());
        if ((st = check_grid(nu, nv)) != SWEEP_OK) {
            return fail(st, "sweep %d: %s", k, sweep_last_error());
        }
        const int nseg = (nv + 63) / 64;
        const int G = bw_unit_rows_for(o->out_precision == SWEEP_F64);
        const int ngroup = (nu + G - 1) / G;
        if (descs) {
            BatchDesc d{};
            d.n_path = np; d.p_path = pp; d.n_prof = nq; d.p_prof = pq;
            d.closed_prof = qc; d.n_u = nu; d.n_v = nv;
            fastdiv_constants(nv, &d.fd_m, &d.fd_shift);
            d.path_ctrl_off = path_off; d.prof_ctrl_off = prof_off;
            d.path_knot_off = pk ? (long long)knots->size() : -1;
            if (pk) knots->insert(knots->end(), pk, pk + np + pp + 1);
            d.prof_knot_off = qk ? (long long)knots->size() : -1;
            if (qk) knots->insert(knots->end(), qk, qk + nq + pq + 1);
            d.out_off = L.n_out;
            d.plane = plane_stride((long long)nu * nv);
            d.row_off = L.n_rows; d.ptab_off = L.n_vs;
            d.rowpart_off = L.n_rowpart; d.colpart_off = L.n_colpart; d.nseg = nseg; d.ngroup = ngroup;
            d.path_kuser_off = pk ? pk_off : -1;
            d.prof_kuser_off = qk ? qk_off : -1;
            d.ctot_off = L.n_uchunks;
            d.arc_off = L.n_arc;
            descs->push_back(d);
        }
        if (key) {
            const int32_t v[7] = {np, pp, nq, pq, qc, nu, nv};
            key->ints.insert(key->ints.end(), v, v + 7);
            if (pk) key->dbls.insert(key->dbls.end(), pk, pk + np + pp + 1);
            if (qk) key->dbls.insert(key->dbls.end(), qk, qk + nq + pq + 1);
        }
        if (b->path_knots) pk_off += np + pp + 1;
        if (b->prof_knots && !qc) qk_off += nq + pq + 1;
        path_off += np; prof_off += nq;
        L.n_vertices += (long long)nu * nv;
        L.n_out += 3 * plane_stride((long long)nu * nv);
        L.n_rows += nu; L.n_vs += nv;
        L.n_rowpart += (long long)nseg * nu; L.n_colpart += (long long)ngroup * nv;
        L.n_units += (long long)nseg * ngroup;
        L.n_uchunks += (nu + kBlock - 1) / kBlock;
        if (arc) L.n_arc += arc_piece_count(np, pp);
    }
    if (!b->path_ctrl || !b->prof_ctrl) return fail(SWEEP_ERR_NULL_ARG, "control point buffer is NULL");
    size_t off = 0;
    const size_t rl = options_ext(o) ? kRowExt : 16;   // row record length
    L.rows = off; off = align_up(off + tsz * rl * (size_t)L.n_rows);
    L.ptab = off; off = align_up(off + tsz * 8 * (size_t)L.n_vs);
    // arc-length tables: piece lengths, cumulative tables (one entry more
    // per sweep), sample parameters and spans (per u-row)
    L.arc_len = off; off = align_up(off + sizeof(double) * (size_t)L.n_arc);
    L.arc_cum = off; off = align_up(off + sizeof(double) * (arc ? (size_t)(L.n_arc + b->n_sweeps) : 0));
    L.arc_u = off; off = align_up(off + sizeof(double) * (arc ? (size_t)L.n_rows : 0));
    L.arc_s = off; off = align_up(off + sizeof(int) * (arc ? (size_t)L.n_rows : 0));
    L.total = off;
    if (lay) *lay = L;
    if (key) {
        // (rational paths stage their weights in the frame kernel's LDS: the
        // sweeps routed to the chunk-walking kernel depend on it)
        const int32_t v[8] = {o->out_precision, o->frame_precision, o->reorthonormalize, o->has_initial_normal,
                              o->tile_config, o->batch_stages, b->path_weights ? 1 : 0, b->prof_weights ? 1 : 0};
        key->ints.insert(key->ints.end(), v, v + 8);
        // the frame mode and the law's shape (its control points are a call
        // argument, its knots are uploaded with the plan)
        const sweep_curve* lw = o->law;
        const int32_t x[6] = {o->frame_mode, lw ? 1 : 0, lw ? lw->n_ctrl : 0, lw ? lw->degree : 0,
                              lw && lw->knots ? 1 : 0, o->u_sampling};
        key->ints.insert(key->ints.end(), x, x + 6);
        if (arc) key->dbls.push_back(o->u_sampling == SWEEP_U_ADAPTIVE ? o->u_lambda : 0.0);
        if (lw && lw->knots) key->dbls.insert(key->dbls.end(), lw->knots, lw->knots + lw->n_ctrl + lw->degree + 1);
        if (o->has_initial_normal) key->dbls.insert(key->dbls.end(), o->initial_normal, o->initial_normal + 3);
    }
    return SWEEP_OK;
}

// Argument values of one graph node; its parameter array points into this
// block.  `sweeps` is a frame node's own sweep list.
struct NodeArgs {
    const BatchDesc* descs;
    const int* sweeps;
    const int2* vchunks;
    const int2* tiles;
    const double* path_ctrl;
    const double* prof_ctrl;
    const double* path_w;
    const double* prof_w;
    const double* knots;
    InitialNormal n0;
    int reorth;
    void* rows;
    void* ptab;
    void* pos;
    void* nrm;
    BatchFrameExt fx;
    // arc-length sampling
    const int2* apch;              // (sweep, first span index) per block
    const int2* asch;              // (sweep, first u-sample) per block
    double lam;                    // adaptive sampling weight (0: arc length)
    double* arc_len;
    double* arc_cum;
    double* arc_u;
    int* arc_s;
};

enum NodeKind { kProfile, kFrame, kSurface, kArcPieces, kArcCumsum, kArcParams };

struct GNode {
    NodeKind kind;
    int deg;
    hipGraphNode_t node = nullptr;
    hipKernelNodeParams prm{};
    NodeArgs a{};
    void* ptrs[9];
};

// Parameter array of a node kind (pointers into n.a).
static int node_args(GNode& n)
{
    NodeArgs& A = n.a;
    void** q = n.ptrs;
    switch (n.kind) {
    case kProfile: { void* v[] = {&A.descs, &A.vchunks, &A.prof_ctrl, &A.prof_w, &A.knots, &A.ptab}; std::memcpy(q, v, sizeof v); return 6; }
    case kFrame: { void* v[] = {&A.descs, &A.sweeps, &A.path_ctrl, &A.path_w, &A.knots, &A.n0, &A.reorth, &A.rows, &A.fx}; std::memcpy(q, v, sizeof v); return 9; }
    case kArcPieces: { void* v[] = {&A.descs, &A.apch, &A.path_ctrl, &A.path_w, &A.knots, &A.lam, &A.arc_len}; std::memcpy(q, v, sizeof v); return 7; }
    case kArcCumsum: { void* v[] = {&A.descs, &A.arc_len, &A.arc_cum}; std::memcpy(q, v, sizeof v); return 3; }
    case kArcParams: { void* v[] = {&A.descs, &A.asch, &A.path_ctrl, &A.path_w, &A.knots, &A.lam, &A.arc_cum, &A.arc_u, &A.arc_s}; std::memcpy(q, v, sizeof v); return 9; }
    default: { void* v[] = {&A.descs, &A.tiles, &A.rows, &A.ptab, &A.pos, &A.nrm}; std::memcpy(q, v, sizeof v); return 6; }
    }
}

struct Plan {
    BatchKey key;
    BatchLayout lay;
    int n_sweeps = 0;
    int n_tiles = 0;
    bool with_nrm = false;
    BatchDesc* d_descs = nullptr;
    int2* d_tiles = nullptr;
    int4* d_units = nullptr;       // adjoint reduction units, built on the first backward call
    int n_units = 0;
    int2* d_uchunks_all = nullptr; // (sweep, chunk) of every path chunk, built on the first backward call
    int n_uchunks_all = 0;
    double* d_knots = nullptr;
    double* d_law_knots = nullptr;  // the law's given knots
    int2* d_arc_pch = nullptr;      // arc-length sampling: (sweep, first span index) per block
    int2* d_arc_sch = nullptr;      // (sweep, first u-sample) per block
    int arc_pr[9] = {}, arc_sr[9] = {};   // both lists by path degree: degree p at [r[p], r[p+1])
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int* d_sweeps[8] = {};         // sweeps by path degree: by stage and frame kernel, longest n_u first
    int n_deg[8] = {};
    // Frame launches: a range of d_sweeps[deg], all of one stage and one
    // frame kernel: chunk-walking (longer than one frame chunk, or a path too
    // large to stage in LDS), one-chunk block, or one wave per sweep.
    enum { kWalkFrame = 0, kBlockFrame = 1, kWaveFrame = 2 };
    struct FrameRange {
        int deg, first, grid, stage, kind;   // list entries [first, first + grid * (kWaves if wave kind else 1))
    };
    std::vector<FrameRange> franges;
    int n_stages = 1;
    std::vector<int> stage_tiles;  // first surface tile of each stage, and the total
    int2* d_vchunks = nullptr;     // (sweep, chunk) of every profile chunk
    int n_vchunks = 0;
    NodeArgs a{};                  // values shared by all nodes
    std::vector<std::unique_ptr<GNode>> nodes;
    // Completion markers of the plan's launches, one event per stream the
    // plan was launched on, recorded after every launch (graph replay or
    // adjoint kernels).  They are waited on before the graph's parameters
    // change and before the plan is destroyed (evicted or released), so
    // that no launch still in flight reads a kernel-argument block, a
    // descriptor array or a graph executable that is being replaced.
    std::vector<std::pair<hipStream_t, hipEvent_t>> done;
    void wait_launches()
    {
        for (auto& d : done) hipEventSynchronize(d.second);
    }
    hipError_t mark_launched(hipStream_t s)
    {
        for (auto& d : done)
            if (d.first == s) return hipEventRecord(d.second, s);
        if (done.size() >= kMaxStreamsTracked) {
            // more streams than tracked: retire the markers of the others
            wait_launches();
            for (auto& d : done) hipEventDestroy(d.second);
            done.clear();
        }
        hipEvent_t e = nullptr;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) return r;
        done.emplace_back(s, e);
        return hipEventRecord(e, s);
    }
    static constexpr size_t kMaxStreamsTracked = 8;
    ~Plan()
    {
        wait_launches();
        for (auto& d : done) hipEventDestroy(d.second);
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (d_descs) hipFree(d_descs);
        if (d_tiles) hipFree(d_tiles);
        if (d_units) hipFree(d_units);
        if (d_uchunks_all) hipFree(d_uchunks_all);
        for (int p = 0; p < 8; ++p)
            if (d_sweeps[p]) hipFree(d_sweeps[p]);
        if (d_vchunks) hipFree(d_vchunks);
        if (d_knots) hipFree(d_knots);
        if (d_law_knots) hipFree(d_law_knots);
        if (d_arc_pch) hipFree(d_arc_pch);
        if (d_arc_sch) hipFree(d_arc_sch);
    }
};

// Shape class of a batch for the tuning table: output precision, normals
// written, floor(log2) of the sweep count, of the total vertex count and of
// the mean n_v.
static void batch_class(const sweep_batch* b, const sweep_options* o, bool with_nrm, int* cls)
{
    long long verts = 0, rows = 0;
    for (int k = 0; k < b->n_sweeps; ++k) {
        verts += (long long)b->n_u[k] * b->n_v[k];
        rows += b->n_u[k];
    }
    const int c[kTuneClassInts] = {o->out_precision == SWEEP_F64 ? 1 : 0, with_nrm ? 1 : 0, ilog2_ll(b->n_sweeps),
                                   ilog2_ll(verts), ilog2_ll(rows > 0 ? verts / rows : 1)};
    for (int k = 0; k < kTuneClassInts; ++k) cls[k] = c[k];
}

// Built-in batched surface configuration: linear tiles of 1024 vertices with
// nontemporal stores (tile_config index kBatchDefaultConfig).
constexpr int kBatchDefaultConfig = 14;

// Configuration index for tile_config = -1: the tuned one for the batch's
// shape class if sweep_autotune_batched recorded one, else the built-in.
static int batched_auto_config(const sweep_batch* b, const sweep_options* o, bool with_nrm)
{
    int cls[kTuneClassInts];
    batch_class(b, o, with_nrm, cls);
    const int c = tune_lookup("batch", cls);
    return c >= 0 && tile_config(c).kind == 1 ? c : kBatchDefaultConfig;
}

// The options a plan is keyed and built with: tile_config = -1 resolved to
// the configuration it selects, so that a tuned choice maps to the plan of
// that configuration.
static sweep_options resolved_options(const sweep_batch* b, const sweep_options* o, bool with_nrm)
{
    sweep_options r = *o;
    if (r.tile_config < 0) r.tile_config = batched_auto_config(b, o, with_nrm);
    return r;
}

// Surface tiles of tv consecutive vertices: (sweep, first local vertex) in
// sweep order.
static std::vector<int2> surface_tiles(const sweep_batch* b, int tv)
{
    std::vector<int2> tiles;
    for (int k = 0; k < b->n_sweeps; ++k) {
        const long long N = (long long)b->n_u[k] * b->n_v[k];
        for (long long v = 0; v < N; v += tv) tiles.push_back(make_int2(k, (int)v));
    }
    return tiles;
}

// Pipeline stages of a batch schedule.  A sweep's frame level is log2 of its
// run length K (the smallest power of two up to kMaxRun with kBlock*K >= n_u),
// or kMaxRunLog + 1 for a sweep longer than one frame chunk; the level range
// is cut into S equal parts, shortest paths first.  Stage s's frame launches
// wait for those of stage s-1, and stage s's surface launch waits only for
// its own frames: the surfaces of the earlier stages are written while the
// later stages' frames are formed.
constexpr int kMaxStages = 4;
constexpr int kDefaultStages = 1;
static int frame_level(int n_u)
{
    if (n_u > kBlock * kMaxRun) return 5;
    int K = 1, l = 0;
    while (K < kMaxRun && kBlock * K < n_u) { K *= 2; ++l; }
    return l;
}
static int frame_stage(int n_u, int S) { return frame_level(n_u) * S / 6; }
static int resolved_stages(const sweep_options* o) { return o->batch_stages > 0 ? o->batch_stages : kDefaultStages; }
static_assert(kMaxStages == 4, "batch_stages is validated as 0..4");

// The frame mode and law of a batch as the frame kernels take them (every
// field set, so that argument blocks compare bytewise).
static void set_frame_ext(BatchFrameExt& fx, const sweep_options* o, const double* d_law_knots,
                          const double* su = nullptr, const int* ss = nullptr)
{
    std::memset(&fx, 0, sizeof fx);
    fx.su = su;
    fx.ss = ss;
    fx.frenet = o->frame_mode == SWEEP_FRAME_FRENET;
    if (const sweep_curve* lw = o->law) {
        fx.has_law = 1;
        fx.law_len = lw->knots ? lw->knots[lw->n_ctrl] - lw->knots[lw->degree] : 1.0;
        DCurve c{};
        c.ctrl = lw->ctrl;
        c.knots = lw->knots ? d_law_knots : nullptr;
        c.n = lw->n_ctrl;
        c.p = lw->degree;
        c.closed = 0;
        c.nb = nbasis(lw->n_ctrl, lw->degree, 0);
        c.w = lw->weights;
        fx.law = c;
    }
}

static std::mutex g_mu;
static std::list<std::unique_ptr<Plan>> g_plans;   // most recently used first
static const size_t kMaxPlans = 16;

static sweep_status build_plan(const sweep_batch* b, const sweep_options* o, bool with_nrm, BatchKey&& key,
                               std::unique_ptr<Plan>& out)
{
    std::unique_ptr<Plan> P(new Plan());
    std::vector<BatchDesc> descs;
    std::vector<double> knots;
    sweep_status st = check_batch(b, o, nullptr, &P->lay, &descs, &knots);
    if (st != SWEEP_OK) return st;
    P->key = std::move(key);
    P->n_sweeps = b->n_sweeps;
    P->with_nrm = with_nrm;
    // surface tiles: (sweep, first local vertex) in sweep order; sweeps by
    // path degree, longest first (the frame blocks' work is proportional to
    // n_u); profile chunks: (sweep, chunk) of every 256 v-samples
    const SurfaceConfig cfg = tile_config(o->tile_config);   // resolved by the caller
    // column-tile configurations map to one-row-sized linear tiles
    const int tv = cfg.kind == 1 ? cfg.tile_vertices : kBlock;
    const int S = resolved_stages(o);
    P->n_stages = S;
    // surface tiles grouped by stage (sweep order inside a stage)
    std::vector<int2> tiles;
    {
        const std::vector<int2> all = surface_tiles(b, tv);
        for (int st = 0; st < S; ++st) {
            P->stage_tiles.push_back((int)tiles.size());
            for (const int2& t : all)
                if (frame_stage(b->n_u[t.x], S) == st) tiles.push_back(t);
        }
        P->stage_tiles.push_back((int)tiles.size());
    }
    std::vector<int2> vchunks;
    std::vector<int> sweeps[8];
    for (int k = 0; k < b->n_sweeps; ++k) {
        sweeps[b->path_degree[k]].push_back(k);
        for (int c = 0; c * kBlock < b->n_v[k]; ++c) vchunks.push_back(make_int2(k, c));
    }
    // frame kernel of a sweep: one wave per sweep up to kWaveMaxU
    // u-samples; the one-chunk block kernel up to kBlock*kMaxRun if the path
    // fits its LDS; else the chunk-walking kernel
    const bool rat = b->path_weights != nullptr;
    const bool arc = o->u_sampling != SWEEP_U_PARAMETER;
    auto fkind = [&](int k) -> int {
        if (b->n_u[k] <= kWaveMaxU) return Plan::kWaveFrame;
        if (b->n_u[k] <= kBlock * kMaxRun && lds_path_doubles(b->path_n[k], b->path_degree[k], rat) <= kLdsPathDoubles)
            return Plan::kBlockFrame;
        return Plan::kWalkFrame;
    };
    for (auto& l : sweeps)
        std::stable_sort(l.begin(), l.end(), [&](int x, int y) {
            const int sx = frame_stage(b->n_u[x], S), sy = frame_stage(b->n_u[y], S);
            if (sx != sy) return sx < sy;
            if (fkind(x) != fkind(y)) return fkind(x) < fkind(y);
            return b->n_u[x] > b->n_u[y];
        });
    // device lists: the sorted sweeps, each wave-kernel range padded with -1
    // to whole blocks of kWaves sweeps
    std::vector<int> lists[8];
    for (int p = 1; p <= SWEEP_MAX_DEGREE; ++p) {
        const std::vector<int>& l = sweeps[p];
        size_t i = 0;
        while (i < l.size()) {
            const int st = frame_stage(b->n_u[l[i]], S);
            const int kind = fkind(l[i]);
            size_t j = i;
            while (j < l.size() && frame_stage(b->n_u[l[j]], S) == st && fkind(l[j]) == kind) ++j;
            const int first = (int)lists[p].size();
            lists[p].insert(lists[p].end(), l.begin() + i, l.begin() + j);
            int grid = (int)(j - i);
            if (kind == Plan::kWaveFrame) {
                while ((lists[p].size() - first) % kWaves) lists[p].push_back(-1);
                grid = ((int)lists[p].size() - first) / kWaves;
            }
            P->franges.push_back(Plan::FrameRange{p, first, grid, st, kind});
            i = j;
        }
    }
    if (tiles.size() > 0x7fffffffull || vchunks.size() > 0x7fffffffull)
        return fail(SWEEP_ERR_BAD_COUNT, "batch needs too many blocks");
    P->n_tiles = (int)tiles.size();
    P->n_vchunks = (int)vchunks.size();
    hipError_t e;
    auto upload = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t r = hipMalloc(dst, bytes);
        if (r != hipSuccess) return r;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    if ((e = upload((void**)&P->d_descs, descs.data(), sizeof(BatchDesc) * descs.size())) != hipSuccess ||
        (e = upload((void**)&P->d_tiles, tiles.data(), sizeof(int2) * tiles.size())) != hipSuccess ||
        (e = upload((void**)&P->d_vchunks, vchunks.data(), sizeof(int2) * vchunks.size())) != hipSuccess)
        return hip_fail(e, "plan upload");
    for (int p = 1; p <= SWEEP_MAX_DEGREE; ++p) {
        P->n_deg[p] = (int)sweeps[p].size();
        if (!lists[p].empty() &&
            (e = upload((void**)&P->d_sweeps[p], lists[p].data(), sizeof(int) * lists[p].size())) != hipSuccess)
            return hip_fail(e, "plan upload");
    }
    if (!knots.empty() && (e = upload((void**)&P->d_knots, knots.data(), sizeof(double) * knots.size())) != hipSuccess)
        return hip_fail(e, "plan upload");

    const bool ext = options_ext(o);
    const bool adaptive = o->u_sampling == SWEEP_U_ADAPTIVE && o->u_lambda != 0.0;
    const BatchedKernels K = batched_kernels(o->frame_precision == SWEEP_F64, o->out_precision == SWEEP_F64,
                                             with_nrm, cfg.nontemporal != 0, tv, ext, arc, adaptive,
                                             b->path_weights != nullptr);
    if (arc) {
        // work lists of the arc-length kernels, by path degree (a launch
        // each): kWaves spans (a wave each) and 32 u-samples (eight lanes
        // each) per block
        std::vector<int2> pch, sch;
        for (int p = 1; p <= SWEEP_MAX_DEGREE; ++p) {
            P->arc_pr[p] = (int)pch.size();
            P->arc_sr[p] = (int)sch.size();
            for (int k = 0; k < b->n_sweeps; ++k) {
                if (b->path_degree[k] != p) continue;
                const int nspan = b->path_n[k] - p;
                for (int q = 0; q < nspan; q += kWaves) pch.push_back(make_int2(k, q));
                for (int i = 0; i < b->n_u[k]; i += kBlock / kArcLanes) sch.push_back(make_int2(k, i));
            }
        }
        P->arc_pr[SWEEP_MAX_DEGREE + 1] = (int)pch.size();
        P->arc_sr[SWEEP_MAX_DEGREE + 1] = (int)sch.size();
        if ((e = upload((void**)&P->d_arc_pch, pch.data(), sizeof(int2) * pch.size())) != hipSuccess ||
            (e = upload((void**)&P->d_arc_sch, sch.data(), sizeof(int2) * sch.size())) != hipSuccess)
            return hip_fail(e, "plan upload");
    }
    if (o->law && o->law->knots) {
        const sweep_curve* lw = o->law;
        if ((e = upload((void**)&P->d_law_knots, lw->knots, sizeof(double) * (lw->n_ctrl + lw->degree + 1))) !=
            hipSuccess)
            return hip_fail(e, "plan upload");
    }
    // argument blocks are compared bytewise on every call: clear the padding
    std::memset(&P->a, 0, sizeof P->a);
    NodeArgs& A = P->a;
    A.descs = P->d_descs;
    A.vchunks = P->d_vchunks;
    A.tiles = P->d_tiles;
    A.knots = P->d_knots;
    A.n0.enabled = o->has_initial_normal;
    for (int c = 0; c < 3; ++c) A.n0.v[c] = o->initial_normal[c];
    A.reorth = o->reorthonormalize;
    set_frame_ext(A.fx, o, P->d_law_knots);
    A.apch = P->d_arc_pch;
    A.asch = P->d_arc_sch;
    A.lam = adaptive ? o->u_lambda : 0.0;
    if ((e = hipGraphCreate(&P->graph, 0)) != hipSuccess) return hip_fail(e, "graph");
    // frame nodes: sweeps [first, first + grid) of the degree's list;
    // surface nodes: tiles [first, first + grid)
    auto add = [&](NodeKind kind, int deg, const void* fn, unsigned grid,
                   const std::vector<hipGraphNode_t>& deps, int first = 0, unsigned lds = 0,
                   unsigned block = kBlock) -> hipError_t {
        std::unique_ptr<GNode> n(new GNode());
        n->kind = kind;
        n->deg = deg;
        std::memcpy(&n->a, &P->a, sizeof n->a);
        if (kind == kFrame) n->a.sweeps = P->d_sweeps[deg] + first;
        if (kind == kSurface) n->a.tiles = P->d_tiles + first;
        if (kind == kArcPieces) n->a.apch = P->d_arc_pch + first;
        if (kind == kArcParams) n->a.asch = P->d_arc_sch + first;
        node_args(*n);
        n->prm.func = const_cast<void*>(fn);
        n->prm.gridDim = dim3(grid);
        n->prm.blockDim = dim3(block);
        n->prm.sharedMemBytes = lds;
        n->prm.kernelParams = n->ptrs;
        n->prm.extra = nullptr;
        hipError_t r = hipGraphAddKernelNode(&n->node, P->graph, deps.empty() ? nullptr : deps.data(), deps.size(),
                                             &n->prm);
        P->nodes.push_back(std::move(n));
        return r;
    };
    if ((e = add(kProfile, 0, K.profile, (unsigned)P->n_vchunks, {})) != hipSuccess) return hip_fail(e, "graph node");
    const hipGraphNode_t profile_node = P->nodes.back()->node;
    std::vector<hipGraphNode_t> prev_frames;
    if (arc) {
        // arc-length samples of every path before any frame: the pieces of
        // each path degree, one scan per sweep, the samples of each degree
        std::vector<hipGraphNode_t> pieces;
        for (int p = 1; p <= SWEEP_MAX_DEGREE; ++p) {
            const int n = P->arc_pr[p + 1] - P->arc_pr[p];
            if (n == 0) continue;
            if ((e = add(kArcPieces, p, K.arc_pieces[p], (unsigned)n, {}, P->arc_pr[p])) != hipSuccess)
                return hip_fail(e, "graph node");
            pieces.push_back(P->nodes.back()->node);
        }
        if ((e = add(kArcCumsum, 0, K.arc_cumsum, (unsigned)b->n_sweeps, pieces, 0, 0, kScanThreads)) != hipSuccess)
            return hip_fail(e, "graph node");
        const hipGraphNode_t cums = P->nodes.back()->node;
        for (int p = 1; p <= SWEEP_MAX_DEGREE; ++p) {
            const int n = P->arc_sr[p + 1] - P->arc_sr[p];
            if (n == 0) continue;
            if ((e = add(kArcParams, p, K.arc_params[p], (unsigned)n, {cums}, P->arc_sr[p])) != hipSuccess)
                return hip_fail(e, "graph node");
            prev_frames.push_back(P->nodes.back()->node);
        }
    }
    for (int st = 0; st < S; ++st) {
        std::vector<hipGraphNode_t> frames;
        for (const Plan::FrameRange& r : P->franges) {
            if (r.stage != st) continue;
            const void* fn = r.kind == Plan::kWalkFrame    ? K.frame_long[r.deg]
                             : r.kind == Plan::kBlockFrame ? K.frame[r.deg]
                                                           : K.frame_wave[r.deg];
            const unsigned lds = r.kind == Plan::kBlockFrame ? (unsigned)(sizeof(double) * kLdsPathDoubles) : 0u;
            if ((e = add(kFrame, r.deg, fn, (unsigned)r.grid, prev_frames, r.first, lds)) != hipSuccess)
                return fail(SWEEP_ERR_HIP, "graph node (frame kernel %d, degree %d, %d blocks, %u B LDS): %s", r.kind,
                            r.deg, r.grid, lds, hipGetErrorString(e));
            frames.push_back(P->nodes.back()->node);
        }
        const int t0 = P->stage_tiles[st], nt = P->stage_tiles[st + 1] - t0;
        if (nt > 0) {
            std::vector<hipGraphNode_t> deps = frames;
            deps.push_back(profile_node);
            if ((e = add(kSurface, 0, K.surface, (unsigned)nt, deps, t0)) != hipSuccess)
                return hip_fail(e, "graph node");
        }
        if (!frames.empty()) prev_frames = frames;
    }
    if ((e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "graph instantiate");
    out = std::move(P);
    return SWEEP_OK;
}

// Finds or builds the plan of this batch shape (caller holds g_mu).
static sweep_status get_plan(const sweep_batch* b, const sweep_options* o, bool with_nrm, BatchKey&& key, Plan** out)
{
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
        if ((*it)->key == key) {
            g_plans.splice(g_plans.begin(), g_plans, it);
            *out = g_plans.front().get();
            return SWEEP_OK;
        }
    }
    std::unique_ptr<Plan> np;
    sweep_status st = build_plan(b, o, with_nrm, std::move(key), np);
    if (st != SWEEP_OK) return st;
    g_plans.push_front(std::move(np));
    while (g_plans.size() > kMaxPlans) g_plans.pop_back();
    *out = g_plans.front().get();
    return SWEEP_OK;
}

static size_t batched_ws_size(const sweep_batch* b, const sweep_options* o)
{
    BatchLayout L;
    if (check_batch(b, o, nullptr, &L, nullptr, nullptr) != SWEEP_OK) return 0;
    return L.total;
}

}  // namespace sweep

using namespace sweep;

extern "C" {

int64_t sweep_batched_output_elems(const sweep_batch* batch)
{
    if (!batch || batch->n_sweeps < 1 || !batch->n_u || !batch->n_v) return 0;
    long long n = 0;
    for (int k = 0; k < batch->n_sweeps; ++k) {
        if (batch->n_u[k] < 0 || batch->n_v[k] < 0) return 0;
        n += 3 * plane_stride((long long)batch->n_u[k] * batch->n_v[k]);
    }
    return n;
}

size_t sweep_batched_workspace_size(const sweep_batch* batch, const sweep_options* opt)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    return batched_ws_size(batch, opt);
}

sweep_status sweep_eval_batched(const sweep_batch* batch, const sweep_options* opt, void* pos, void* nrm,
                                void* workspace, size_t ws_bytes, void* stream)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    BatchKey key;
    BatchLayout L;
    sweep_status st = check_batch(batch, opt, nullptr, nullptr, nullptr, nullptr);
    if (st != SWEEP_OK) return st;
    const sweep_options ro = resolved_options(batch, opt, nrm != nullptr);
    opt = &ro;
    if ((st = check_batch(batch, opt, &key, &L, nullptr, nullptr)) != SWEEP_OK) return st;
    if (!pos) return fail(SWEEP_ERR_NULL_ARG, "pos is NULL");
    if (!workspace || ws_bytes < L.total)
        return fail(SWEEP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu required", workspace ? ws_bytes : (size_t)0, L.total);
    if (((uintptr_t)workspace) % 256 != 0) return fail(SWEEP_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    hipError_t e = hipGetDevice(&key.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    key.ints.push_back(nrm ? 1 : 0);

    std::lock_guard<std::mutex> lock(g_mu);
    Plan* P = nullptr;
    if ((st = get_plan(batch, opt, nrm != nullptr, std::move(key), &P)) != SWEEP_OK) return st;
    char* ws = (char*)workspace;
    NodeArgs A;
    std::memcpy(&A, &P->a, sizeof A);
    A.path_ctrl = batch->path_ctrl;
    A.prof_ctrl = batch->prof_ctrl;
    A.path_w = batch->path_weights;
    A.prof_w = batch->prof_weights;
    A.rows = ws + L.rows;
    A.ptab = ws + L.ptab;
    A.pos = pos;
    A.nrm = nrm;
    if (opt->u_sampling != SWEEP_U_PARAMETER) {
        A.arc_len = (double*)(ws + L.arc_len);
        A.arc_cum = (double*)(ws + L.arc_cum);
        A.arc_u = (double*)(ws + L.arc_u);
        A.arc_s = (int*)(ws + L.arc_s);
    }
    // the law's control points are a call argument; the sample tables live
    // in the caller's workspace
    set_frame_ext(A.fx, opt, P->d_law_knots, A.arc_u, A.arc_s);
    if (std::memcmp(&A, &P->a, sizeof A) != 0) {
        // a replay of this graph may still be in flight on some stream:
        // let it finish before its node parameters are rewritten
        P->wait_launches();
        P->a = A;
        for (auto& n : P->nodes) {
            // each node's own slice of the work lists stays
            const int* own = n->a.sweeps;
            const int2* own_tiles = n->a.tiles;
            const int2* own_apch = n->a.apch;
            const int2* own_asch = n->a.asch;
            std::memcpy(&n->a, &A, sizeof A);
            n->a.sweeps = own;
            n->a.tiles = own_tiles;
            n->a.apch = own_apch;
            n->a.asch = own_asch;
            if ((e = hipGraphExecKernelNodeSetParams(P->exec, n->node, &n->prm)) != hipSuccess)
                return hip_fail(e, "graph update");
        }
    }
    if ((e = hipGraphLaunch(P->exec, (hipStream_t)stream)) != hipSuccess) return hip_fail(e, "graph launch");
    if ((e = P->mark_launched((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "launch marker");
    return SWEEP_OK;
}

size_t sweep_backward_workspace_size(const sweep_batch* batch, const sweep_options* opt)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    BatchLayout L;
    if (options_ext(opt) || opt->u_sampling != SWEEP_U_PARAMETER ||
        check_batch(batch, opt, nullptr, &L, nullptr, nullptr) != SWEEP_OK)
        return 0;
    return backward_layout(L).total;
}

sweep_status sweep_backward(const sweep_batch* batch, const sweep_options* opt, const void* grad_pos,
                            double* grad_path_ctrl, double* grad_prof_ctrl, void* workspace, size_t ws_bytes,
                            void* stream)
{
    if (!grad_pos) return fail(SWEEP_ERR_NULL_ARG, "grad_pos is NULL");
    return sweep_backward_ex(batch, opt, grad_pos, nullptr, grad_path_ctrl, grad_prof_ctrl, nullptr, workspace,
                             ws_bytes, stream);
}

sweep_status sweep_backward_ex(const sweep_batch* batch, const sweep_options* opt, const void* grad_pos,
                               const void* grad_nrm, double* grad_path_ctrl, double* grad_prof_ctrl,
                               const sweep_param_grads* params, void* workspace, size_t ws_bytes, void* stream)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    BatchKey key;
    BatchLayout L;
    sweep_status st = check_batch(batch, opt, nullptr, nullptr, nullptr, nullptr);
    if (st != SWEEP_OK) return st;
    if (options_ext(opt) || opt->u_sampling != SWEEP_U_PARAMETER)
        return fail(SWEEP_ERR_UNSUPPORTED,
                    "the adjoint differentiates rotation-minimizing frames of uniform samples without a law only");
    const sweep_options ro = resolved_options(batch, opt, true);
    opt = &ro;
    if ((st = check_batch(batch, opt, &key, &L, nullptr, nullptr)) != SWEEP_OK) return st;
    if (!grad_pos && !grad_nrm) return fail(SWEEP_ERR_NULL_ARG, "grad_pos and grad_nrm are both NULL");
    if (!grad_path_ctrl || !grad_prof_ctrl) return fail(SWEEP_ERR_NULL_ARG, "a gradient buffer is NULL");
    const int nrm = grad_nrm != nullptr;
    sweep_param_grads pg{};
    if (params) pg = *params;
    if (pg.path_knots && !batch->path_knots) return fail(SWEEP_ERR_BAD_OPTION, "path knot gradients need given path knots");
    if (pg.prof_knots && !batch->prof_knots) return fail(SWEEP_ERR_BAD_OPTION, "profile knot gradients need given profile knots");
    if (pg.path_weights && !batch->path_weights) return fail(SWEEP_ERR_BAD_OPTION, "path weight gradients need path weights");
    if (pg.prof_weights && !batch->prof_weights) return fail(SWEEP_ERR_BAD_OPTION, "profile weight gradients need profile weights");
    const bool want_params = pg.path_knots || pg.prof_knots || pg.path_weights || pg.prof_weights;
    const BackwardLayout B = backward_layout(L);
    if (!workspace || ws_bytes < B.total)
        return fail(SWEEP_ERR_WORKSPACE, "workspace of %zu bytes given, %zu required", workspace ? ws_bytes : (size_t)0, B.total);
    if (((uintptr_t)workspace) % 256 != 0) return fail(SWEEP_ERR_WORKSPACE, "workspace is not 256-byte aligned");
    hipError_t e = hipGetDevice(&key.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    key.ints.push_back(1);   // plans are shared with the forward call that writes normals

    std::lock_guard<std::mutex> lock(g_mu);
    Plan* P = nullptr;
    if ((st = get_plan(batch, opt, true, std::move(key), &P)) != SWEEP_OK) return st;
    if (!P->d_units) {
        std::vector<int4> units;
        units.reserve((size_t)L.n_units);
        for (int k = 0; k < batch->n_sweeps; ++k) {
            const int G = bw_unit_rows_for(opt->out_precision == SWEEP_F64);
            const int ng = (batch->n_u[k] + G - 1) / G, ns = (batch->n_v[k] + 63) / 64;
            for (int g = 0; g < ng; ++g)
                for (int sg = 0; sg < ns; ++sg) units.push_back(make_int4(k, g, sg, 0));
        }
        if ((e = hipMalloc(&P->d_units, sizeof(int4) * units.size())) != hipSuccess) return hip_fail(e, "plan alloc");
        if ((e = hipMemcpy(P->d_units, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "plan upload");
        P->n_units = (int)units.size();
    }
    hipStream_t sm = (hipStream_t)stream;
    char* ws = (char*)workspace;
    // every exit after the first launch records the plan's completion marker
    struct MarkOnExit {
        Plan* P;
        hipStream_t s;
        ~MarkOnExit() { P->mark_launched(s); }
    } marker{P, sm};
    const BatchedKernels FK = batched_kernels(true, true, false, false, kBlock, false, false, false, false);
    const BackwardKernels BK = backward_kernels(opt->out_precision == SWEEP_F64, nrm);
    {
        // FP64 frame recomputation with re-orthonormalisation: profile tables, frames
        GNode n;
        std::memcpy(&n.a, &P->a, sizeof n.a);
        n.a.path_ctrl = batch->path_ctrl;
        n.a.prof_ctrl = batch->prof_ctrl;
        n.a.path_w = batch->path_weights;
        n.a.prof_w = batch->prof_weights;
        n.a.reorth = 1;
        n.a.rows = ws + B.rows;
        n.a.ptab = ws + B.ptab;
        auto launch = [&](NodeKind kind, int deg, const void* fn, unsigned grid, int first = 0,
                          size_t lds = 0) -> hipError_t {
            n.kind = kind;
            n.a.sweeps = kind == kFrame ? P->d_sweeps[deg] + first : nullptr;
            node_args(n);
            return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), n.ptrs, lds, sm);
        };
        if ((e = launch(kProfile, 0, FK.profile, (unsigned)P->n_vchunks)) != hipSuccess)
            return hip_fail(e, "backward frames");
        for (const Plan::FrameRange& r : P->franges) {
            const void* fn = r.kind == Plan::kWalkFrame    ? FK.frame_long[r.deg]
                             : r.kind == Plan::kBlockFrame ? FK.frame[r.deg]
                                                           : FK.frame_wave[r.deg];
            const size_t lds = r.kind == Plan::kBlockFrame ? sizeof(double) * kLdsPathDoubles : 0;
            if ((e = launch(kFrame, r.deg, fn, (unsigned)r.grid, r.first, lds)) != hipSuccess)
                return hip_fail(e, "backward frames");
        }
    }
    {
        const BatchDesc* descs = P->d_descs;
        const int4* units = P->d_units;
        int n_units = P->n_units;
        const void* g = grad_pos;
        const void* gn = grad_nrm;
        const void* rows = ws + B.rows;
        const void* ptab = ws + B.ptab;
        void* rowpart = ws + B.rowpart;
        void* colpart = ws + B.colpart;
        void* args[9] = {&descs, &units, &n_units, &g, &gn, &rows, &ptab, &rowpart, &colpart};
        const unsigned grid = (unsigned)n_units;   // one block per unit
        if ((e = hipLaunchKernel(BK.reduce, dim3(grid), dim3(kBlock), args, 0, sm)) != hipSuccess)
            return hip_fail(e, "backward reduce");
    }
    if (!P->d_uchunks_all) {
        // (sweep, chunk) of every path chunk of kBlock u-samples
        std::vector<int2> ch;
        for (int k = 0; k < batch->n_sweeps; ++k)
            for (int c = 0; c * kBlock < batch->n_u[k]; ++c) ch.push_back(make_int2(k, c));
        if ((e = hipMalloc(&P->d_uchunks_all, sizeof(int2) * ch.size())) != hipSuccess) return hip_fail(e, "plan alloc");
        if ((e = hipMemcpy(P->d_uchunks_all, ch.data(), sizeof(int2) * ch.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "plan upload");
        P->n_uchunks_all = (int)ch.size();
    }
    {
        const BatchDesc* descs = P->d_descs;
        const int2* uch = P->d_uchunks_all;
        const double* pc = batch->path_ctrl;
        const double* qc = batch->prof_ctrl;
        const double* pw = batch->path_weights;
        const double* qw = batch->prof_weights;
        const double* kn = P->d_knots;
        InitialNormal n0 = P->a.n0;
        const void* rows = ws + B.rows;
        const void* rowpart = ws + B.rowpart;
        const void* colpart = ws + B.colpart;
        void* rowacc = ws + B.rowacc;
        void* colacc = ws + B.colacc;
        void* sfx = ws + B.rho;
        void* ctot = ws + B.ctot;
        void* sgrad = ws + B.sgrad;
        void* spans_u = ws + B.spans_u;
        void* qgrad = ws + B.qgrad;
        void* spans_v = ws + B.spans_v;
        double* gp = grad_path_ctrl;
        double* gq = grad_prof_ctrl;
        int nrm_arg = nrm;
        void* xstash = want_params ? ws + B.xstash : nullptr;
        const unsigned nch = (unsigned)P->n_uchunks_all;
        void* rargs[11] = {&descs, &uch, &pc, &pw, &kn, &rows, &rowpart, &rowacc, &sfx, &ctot, &nrm_arg};
        if ((e = hipLaunchKernel(BK.rows, dim3(nch), dim3(kBlock), rargs, 0, sm)) != hipSuccess)
            return hip_fail(e, "backward rows");
        void* sargs[14] = {&descs, &uch, &pc, &pw, &kn, &n0, &rows, &rowacc, &sfx, &ctot, &sgrad, &spans_u, &nrm_arg,
                           &xstash};
        if ((e = hipLaunchKernel(BK.samples, dim3(nch), dim3(kBlock), sargs, 0, sm)) != hipSuccess)
            return hip_fail(e, "backward samples");
        void* fargs[15] = {&descs, &pc, &qc, &pw, &qw, &kn, &colpart, &colacc, &sgrad, &spans_u, &qgrad, &spans_v,
                           &gp, &gq, &nrm_arg};
        if ((e = hipLaunchKernel(BK.final_, dim3(batch->n_sweeps), dim3(kBlock), fargs, 0, sm)) != hipSuccess)
            return hip_fail(e, "backward gathers");
        if (want_params) {
            const void* xs = xstash;
            const void* ca = colacc;
            const void* su = spans_u;
            const void* sv = spans_v;
            void* recu = ws + B.recu;
            void* recv = ws + B.recv;
            double* gpk = pg.path_knots;
            double* gqk = pg.prof_knots;
            double* gpw = pg.path_weights;
            double* gqw = pg.prof_weights;
            // per-sample records (all samples of all sweeps in parallel), then the gathers per sweep
            for (int prof_side = 0; prof_side < 2; ++prof_side) {
                int wk = prof_side ? pg.prof_knots != nullptr : pg.path_knots != nullptr;
                int ww = prof_side ? pg.prof_weights != nullptr : pg.path_weights != nullptr;
                if (!wk && !ww) continue;
                const int2* chunks = prof_side ? P->d_vchunks : P->d_uchunks_all;
                const unsigned grid = (unsigned)(prof_side ? P->n_vchunks : P->n_uchunks_all);
                void* rargs[17] = {&descs, &chunks, &pc, &qc, &pw, &qw, &kn, &xs, &ca, &su, &sv, &recu, &recv,
                                   &nrm_arg, &wk, &ww};
                if ((e = hipLaunchKernel(prof_side ? BK.param_rec_prof : BK.param_rec_path, dim3(grid), dim3(kBlock),
                                         rargs, 0, sm)) != hipSuccess)
                    return hip_fail(e, "backward knot and weight records");
            }
            void* pargs[14] = {&descs, &pc, &qc, &pw, &qw, &kn, &su, &sv, &recu, &recv, &gpk, &gqk, &gpw, &gqw};
            if ((e = hipLaunchKernel(BK.params, dim3(batch->n_sweeps), dim3(kBlock), pargs, 0, sm)) != hipSuccess)
                return hip_fail(e, "backward knot and weight gradients");
        }
    }
    return SWEEP_OK;
}

int32_t sweep_batched_config_for(const sweep_batch* batch, const sweep_options* opt, int32_t with_normals)
{
    sweep_options def;
    if (!opt) { sweep_default_options(&def); opt = &def; }
    if (check_batch(batch, opt, nullptr, nullptr, nullptr, nullptr) != SWEEP_OK) return -1;
    if (opt->tile_config >= 0) return tile_config(opt->tile_config).kind == 1 ? opt->tile_config : -1;
    return batched_auto_config(batch, opt, with_normals != 0);
}

sweep_status sweep_autotune_batched(const sweep_batch* batch, const sweep_options* opt, void* pos, void* nrm,
                                    void* workspace, size_t ws_bytes, void* stream, int32_t* best_config,
                                    float* best_ms)
{
    sweep_options o;
    if (opt) o = *opt; else sweep_default_options(&o);
    o.tile_config = -1;
    // validates everything, builds (or finds) the automatic plan and leaves
    // the row and profile tables in the workspace
    sweep_status st = sweep_eval_batched(batch, &o, pos, nrm, workspace, ws_bytes, stream);
    if (st != SWEEP_OK) return st;
    BatchLayout L;
    if ((st = check_batch(batch, &o, nullptr, &L, nullptr, nullptr)) != SWEEP_OK) return st;
    const sweep_options ro = resolved_options(batch, &o, nrm != nullptr);
    BatchKey key;
    if ((st = check_batch(batch, &ro, &key, nullptr, nullptr, nullptr)) != SWEEP_OK) return st;
    hipError_t e = hipGetDevice(&key.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    key.ints.push_back(nrm ? 1 : 0);
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = ro.frame_precision == SWEEP_F64, t64 = ro.out_precision == SWEEP_F64;
    char* ws = (char*)workspace;
    const void* rows = ws + L.rows;
    const void* ptab = ws + L.ptab;
    // Every linear surface configuration is timed on the plan's descriptors
    // and tables with a tile list of its own (the surface kernel alone: the
    // profile and frame stages do not depend on the tile).
    std::lock_guard<std::mutex> lock(g_mu);
    Plan* P = nullptr;
    if ((st = get_plan(batch, &ro, nrm != nullptr, std::move(key), &P)) != SWEEP_OK) return st;
    const BatchDesc* descs = P->d_descs;
    const bool ext = options_ext(&ro);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int2* d_tiles = nullptr;
    int best = -1;
    float best_t = 0.f;
    const int reps = 5;
    if ((e = hipEventCreate(&ev0)) == hipSuccess && (e = hipEventCreate(&ev1)) == hipSuccess) {
        for (int c = 0; c < tile_config_count() && e == hipSuccess; ++c) {
            const SurfaceConfig& cfg = tile_config(c);
            if (cfg.kind != 1) continue;   // a batch has linear tiles only
            const std::vector<int2> tiles = surface_tiles(batch, cfg.tile_vertices);
            if ((e = hipMalloc(&d_tiles, sizeof(int2) * tiles.size())) != hipSuccess) break;
            if ((e = hipMemcpy(d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice)) != hipSuccess)
                break;
            const BatchedKernels K = batched_kernels(f64, t64, nrm != nullptr, cfg.nontemporal != 0, cfg.tile_vertices,
                                                     ext, false, false, false);
            const int2* tl = d_tiles;
            void* pp = pos;
            void* np = nrm;
            void* args[6] = {&descs, &tl, &rows, &ptab, &pp, &np};
            auto run = [&]() { return hipLaunchKernel(K.surface, dim3((unsigned)tiles.size()), dim3(kBlock), args, 0, s); };
            if ((e = run()) != hipSuccess) break;   // warm-up
            if ((e = hipEventRecord(ev0, s)) != hipSuccess) break;
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
            if (e != hipSuccess || (e = hipEventRecord(ev1, s)) != hipSuccess || (e = hipEventSynchronize(ev1)) != hipSuccess)
                break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) break;
            ms /= reps;
            if (best < 0 || ms < best_t) { best = c; best_t = ms; }
            // the launches have completed (the event after them was waited on)
            hipFree(d_tiles);
            d_tiles = nullptr;
        }
    }
    if (d_tiles) {
        hipStreamSynchronize(s);
        hipFree(d_tiles);
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    if (e != hipSuccess) return hip_fail(e, "batched autotune");
    int cls[kTuneClassInts];
    batch_class(batch, &o, nrm != nullptr, cls);
    tune_record("batch", cls, best, best_t);
    if (best_config) *best_config = best;
    if (best_ms) *best_ms = best_t;
    return SWEEP_OK;
}

void sweep_release_caches(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_plans.clear();
}

}  // extern "C"
