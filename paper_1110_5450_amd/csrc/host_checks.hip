// host_checks.hip -- host-only parts of the C ABI shared by the entry
// points: the thread-local error text, validation of curves, options and
// grids, the table of fixed surface configurations, and the default options.
// No kernel code: this file and batched_abi.hip also build against a CPU
// stand-in of the HIP runtime, which the plan tests use.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/sweep.h"
#include "abi_internal.hpp"

namespace sweep {

static thread_local std::string g_last_error;

sweep_status fail(sweep_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

sweep_status hip_fail(hipError_t e, const char* where)
{
    return fail(SWEEP_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// ---------------------------------------------------------------- checks

sweep_status check_curve_meta(int n, int p, int closed, const double* knots, const char* what, bool is_path)
{
    if (p < 1 || p > SWEEP_MAX_DEGREE) return fail(SWEEP_ERR_BAD_DEGREE, "%s: degree %d outside 1..%d", what, p, SWEEP_MAX_DEGREE);
    if (closed != 0 && closed != 1) return fail(SWEEP_ERR_BAD_OPTION, "%s: closed flag %d is not 0/1", what, closed);
    if (closed && is_path) return fail(SWEEP_ERR_UNSUPPORTED, "%s: closed paths are not supported", what);
    if (n < p + 1) return fail(SWEEP_ERR_BAD_COUNT, "%s: %d control points for degree %d (need >= %d)", what, n, p, p + 1);
    if (n > (1 << 24)) return fail(SWEEP_ERR_BAD_COUNT, "%s: %d control points (max 2^24)", what, n);
    if (closed && knots) return fail(SWEEP_ERR_UNSUPPORTED, "%s: knots must be NULL for a closed curve", what);
    if (knots) {
        const int nk = n + p + 1;
        for (int k = 0; k < nk; ++k) {
            if (!std::isfinite(knots[k])) return fail(SWEEP_ERR_BAD_KNOTS, "%s: knot %d is not finite", what, k);
            if (k > 0 && knots[k] < knots[k - 1]) return fail(SWEEP_ERR_BAD_KNOTS, "%s: knots decrease at %d", what, k);
        }
        // multiplicities: interior knots at most p, end knots at most p+1,
        // and a non-empty first and last span.
        int run = 1;
        for (int k = 1; k <= nk; ++k) {
            if (k < nk && knots[k] == knots[k - 1]) { ++run; continue; }
            const int first = k - run, last = k - 1;
            const bool interior = first > 0 && last < nk - 1;
            if (interior && run > p) return fail(SWEEP_ERR_BAD_KNOTS, "%s: interior knot %g has multiplicity %d > degree", what, knots[last], run);
            if (run > p + 1) return fail(SWEEP_ERR_BAD_KNOTS, "%s: knot %g has multiplicity %d > degree+1", what, knots[last], run);
            run = 1;
        }
        if (!(knots[p] < knots[p + 1]) || !(knots[n - 1] < knots[n]))
            return fail(SWEEP_ERR_BAD_KNOTS, "%s: first or last span of the domain is empty", what);
    }
    return SWEEP_OK;
}

sweep_status check_curve(const sweep_curve* c, const char* what, bool is_path)
{
    if (!c) return fail(SWEEP_ERR_NULL_ARG, "%s is NULL", what);
    sweep_status st = check_curve_meta(c->n_ctrl, c->degree, c->closed, c->knots, what, is_path);
    if (st != SWEEP_OK) return st;
    if (!c->ctrl) return fail(SWEEP_ERR_NULL_ARG, "%s: ctrl is NULL", what);
    return SWEEP_OK;
}

sweep_status check_options(const sweep_options* o)
{
    if (o->out_precision != SWEEP_F32 && o->out_precision != SWEEP_F64)
        return fail(SWEEP_ERR_BAD_PRECISION, "out_precision %d", o->out_precision);
    if (o->frame_precision != SWEEP_F32 && o->frame_precision != SWEEP_F64)
        return fail(SWEEP_ERR_BAD_PRECISION, "frame_precision %d", o->frame_precision);
    if (o->reorthonormalize != 0 && o->reorthonormalize != 1)
        return fail(SWEEP_ERR_BAD_OPTION, "reorthonormalize %d is not 0/1", o->reorthonormalize);
    if (o->has_initial_normal != 0 && o->has_initial_normal != 1)
        return fail(SWEEP_ERR_BAD_OPTION, "has_initial_normal %d is not 0/1", o->has_initial_normal);
    if (o->has_initial_normal)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(o->initial_normal[k])) return fail(SWEEP_ERR_BAD_OPTION, "initial_normal not finite");
    if (o->tile_config < -1 || o->tile_config >= tile_config_count())
        return fail(SWEEP_ERR_BAD_OPTION, "tile_config %d outside -1..%d", o->tile_config, tile_config_count() - 1);
    if (o->frame_mode != SWEEP_FRAME_RMF && o->frame_mode != SWEEP_FRAME_FRENET)
        return fail(SWEEP_ERR_BAD_OPTION, "frame_mode %d is not RMF (0) or FRENET (1)", o->frame_mode);
    if (o->u_sampling != SWEEP_U_PARAMETER && o->u_sampling != SWEEP_U_ARCLENGTH && o->u_sampling != SWEEP_U_ADAPTIVE)
        return fail(SWEEP_ERR_BAD_OPTION, "u_sampling %d is not PARAMETER (0), ARCLENGTH (1) or ADAPTIVE (2)",
                    o->u_sampling);
    if (o->u_sampling == SWEEP_U_ADAPTIVE && !(std::isfinite(o->u_lambda) && o->u_lambda >= 0.0))
        return fail(SWEEP_ERR_BAD_OPTION, "u_lambda %g is not a finite value >= 0", o->u_lambda);
    if (o->u_sampling != SWEEP_U_PARAMETER && o->law)
        return fail(SWEEP_ERR_UNSUPPORTED, "arc-length or adaptive sampling with a sweep law");
    if (o->law) {
        if (o->law->closed) return fail(SWEEP_ERR_UNSUPPORTED, "law: the law curve must be open");
        sweep_status st = check_curve(o->law, "law", true);
        if (st != SWEEP_OK) return st;
    }
    return SWEEP_OK;
}

// Options that need the extended row records (Frenet frame or a law).
bool options_ext(const sweep_options* o) { return o->frame_mode != SWEEP_FRAME_RMF || o->law != nullptr; }

// Options supported by sweep_eval (and, without frame modes and laws,
// sweep_frames) only.
bool options_single_only(const sweep_options* o) { return options_ext(o) || o->u_sampling != SWEEP_U_PARAMETER; }

sweep_status check_grid(int n_u, int n_v)
{
    if (n_u < 2 || n_v < 3) return fail(SWEEP_ERR_BAD_GRID, "grid %d x %d (need n_u >= 2, n_v >= 3)", n_u, n_v);
    if ((long long)n_u * (long long)n_v >= (1LL << 31))
        return fail(SWEEP_ERR_BAD_GRID, "grid %d x %d has 2^31 or more vertices", n_u, n_v);
    return SWEEP_OK;
}

int nbasis(int n, int p, int closed) { return closed ? n + p : n; }
int nknots(int n, int p, int closed) { return nbasis(n, p, closed) + p + 1; }

// -------------------------------------------------------------- tile table

// Fixed surface configurations (tile_config >= 0); -1 picks automatically.
static const SurfaceConfig kTiles[] = {
    {0, 1, 0, 0}, {0, 2, 0, 0}, {0, 4, 0, 0}, {0, 8, 0, 0},
    {0, 1, 0, 1}, {0, 2, 0, 1}, {0, 4, 0, 1}, {0, 8, 0, 1},
    {1, 0, 256, 0}, {1, 0, 512, 0}, {1, 0, 1024, 0}, {1, 0, 2048, 0},
    {1, 0, 256, 1}, {1, 0, 512, 1}, {1, 0, 1024, 1}, {1, 0, 2048, 1},
};

int tile_config_count() { return (int)(sizeof kTiles / sizeof kTiles[0]); }

const SurfaceConfig& tile_config(int k) { return kTiles[k]; }

}  // namespace sweep

using namespace sweep;

extern "C" {

void sweep_default_options(sweep_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->out_precision = SWEEP_F32;
    opt->frame_precision = SWEEP_F64;
    opt->reorthonormalize = 1;
    opt->has_initial_normal = 0;
    opt->tile_config = -1;
}

int32_t sweep_tile_config_count(void) { return tile_config_count(); }

sweep_status sweep_tile_config_info(int32_t k, int32_t* info)
{
    if (!info) return fail(SWEEP_ERR_NULL_ARG, "info is NULL");
    if (k < 0 || k >= tile_config_count()) return fail(SWEEP_ERR_BAD_OPTION, "tile_config %d outside 0..%d", k, tile_config_count() - 1);
    const SurfaceConfig& c = tile_config(k);
    info[0] = c.kind;
    info[1] = c.rows_per_block;
    info[2] = c.tile_vertices;
    info[3] = c.nontemporal;
    return SWEEP_OK;
}

const char* sweep_last_error(void) { return g_last_error.c_str(); }

int32_t sweep_version(void) { return SWEEP_VERSION; }

}  // extern "C"
