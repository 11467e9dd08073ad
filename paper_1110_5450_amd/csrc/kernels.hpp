// kernels.hpp -- launchers of the sweep kernels (internal to libsweep).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device_math.hpp"

namespace sweep {

struct InitialNormal {
    int enabled;
    double v[3];
};

// Frame of a single sweep: runs of K consecutive u-samples per thread,
// chunks of kBlock runs (K and the chunk count for n_u samples).  The fused
// frame kernel takes up to kBlock*kFusedGroup chunks (kFusedGroup per thread
// in its carry).
constexpr int kFusedGroup = 2;
int frame_run_length(int n_u);
int frame_chunks(int n_u);

// Workspace of the single-sweep frame: per-run records (kRunRec doubles),
// per-chunk last sample with C' != 0, its tangent (3 doubles), flag, product
// (9 values of the frame precision) and entering normal (3 values), and the
// fallback tangent (3 doubles).
// Per-run record between the passes: the run's product of step rotations
// (9 values) and its resolved first tangent (3), as doubles.
constexpr int kRunRec = 12;
struct FrameWork {
    double* trec;
    int* chunk_lv;
    double* chunk_tl;
    int* chunk_fix;
    double* fallback_t;
    void* agg;
    void* r_in;
};

// Run records, chunk products and flags of the path, and the profile table.
template <class F, class T>
hipError_t launch_prep(const DCurve& path, int n_u, const DCurve& prof, int n_v, const FrameWork& w, T* ptab,
                       hipStream_t st);
// Arc-length sampling of an open curve (lam = 0), or curvature-adaptive
// sampling with density |C'| (1 + lam kappa): piece integrals (len,
// arc_pieces(c) values), their cumulative table (cum, one more), sample
// parameters su and spans ss (ns each).
int arc_pieces(const DCurve& c);
hipError_t launch_arclength(const DCurve& c, int ns, double lam, double* len, double* cum, double* su, int* ss,
                            hipStream_t st);
// Triangle list of the n_u x n_v grid (6 ints per quad).
hipError_t launch_triangles(int n_u, int n_v, int closed_v, int* tri, hipStream_t st);

// Values per extended row record (frame modes, sweep laws).
constexpr int kRowExt = 32;

// Frenet frame mode and sweep law of a single sweep (extended row records).
struct FrameExt {
    int frenet;        // 1: Frenet frame
    DCurve law;        // law curve (sigma, theta, -), valid when has_law
    int has_law;
    double du_scale;   // d(law parameter)/du
};

// Chunk carry and row table: 16 values per u-row, or 32 (extended records)
// when ext is given.
template <class F, class T>
hipError_t launch_frame(const DCurve& path, int n_u, const FrameWork& w, InitialNormal n0, int reorth, T* rows,
                        hipStream_t st, const FrameExt* ext = nullptr);

// Surface write of one sweep from its row table (16 values per u-row) and
// profile table (8 values per v-sample).
struct SurfaceConfig {
    int kind;           // 0: column tiles (n_v >= 256), 1: linear with LDS-staged rows (any shape)
    int rows_per_block; // kind 0: rows R per block
    int tile_vertices;  // kind 1: vertices per block, 256*K with K in {1, 2, 4, 8}
    int nontemporal;    // nontemporal stores
};

// ext: row records of 32 values (frame modes, laws) instead of 16.
template <class T>
hipError_t launch_surface(const T* rows, const T* prof, int n_u, int n_v, T* pos, T* nrm,
                          const SurfaceConfig& cfg, hipStream_t st, bool ext = false);


// ----------------------------------------------------------------- batched

// Per-sweep descriptor of a batch (device array, filled on the host).
struct BatchDesc {
    int n_path, p_path, n_prof, p_prof;
    int closed_prof, n_u, n_v, fd_shift;
    unsigned long long fd_m;       // floor(v / n_v) = (v * fd_m) >> fd_shift for v < 2^31
    long long path_ctrl_off;       // in points
    long long prof_ctrl_off;
    long long path_knot_off;       // into the batch knot array, -1 = default knots
    long long prof_knot_off;
    long long out_off;             // element offset of the sweep's output block (3 planes)
    long long plane;               // plane stride: n_u*n_v rounded up to kPlaneAlign
    long long row_off;             // first row record
    long long ptab_off;            // first profile record
    long long rowpart_off;         // adjoint: first per-segment row partial (12 doubles each)
    long long colpart_off;         // adjoint: first per-group column partial (3 doubles each)
    int nseg, ngroup;              // adjoint: 64-column segments, row groups
    long long path_kuser_off;      // adjoint: offset of the path's knots in the caller's packing, -1 = none
    long long prof_kuser_off;      // adjoint: the same for an open profile's knots
    long long ctot_off;            // adjoint: first per-chunk total (chunks of kBlock u-samples)
    long long arc_off;             // arc-length sampling: first piece length (its cumulative table at arc_off + k)
};

// Batched output planes start on multiples of this many elements (256 B in
// FP32): nontemporal stores into planes that start mid-cache-line write
// partial lines and ran at half the bandwidth on MI355X.
constexpr int kPlaneAlign = 64;

// Rows per reduction group in the adjoint's streaming read of dL/dX (the
// LDS tile of a wave holds G x 65 values per plane).
template <class T>
constexpr int bw_row_group() { return sizeof(T) == 8 ? 4 : 8; }
// Rows per reduction unit: one block, one group of G rows per wave, one
// column partial per unit (the column partials' row groups).
inline int bw_unit_rows_for(bool t64) { return (t64 ? 4 : 8) * kWaves; }

struct BackwardKernels {
    const void* reduce;
    const void* rows;            // row sums, direct terms and their suffix sums per chunk
    const void* samples;         // per-sample adjoint and basis contributions per chunk
    const void* final_;          // column sums, profile samples and the gathers per sweep
    const void* params;          // knot and weight gradients: gathers per sweep
    const void* param_rec_path;  // per-sample records, path chunks
    const void* param_rec_prof;  // per-sample records, profile chunks
};
// nrm: the reduction also takes dL/dN (normal terms, longer partial records).
BackwardKernels backward_kernels(bool t64, bool nrm);

// Partial-sum record lengths of the adjoint (doubles per row / per column).
constexpr int kRowPart = 12, kRowPartNrm = 24;
constexpr int kColPart = 3, kColPartNrm = 6;

// Fast division constants for 0 <= v < 2^31.
void fastdiv_constants(int d, unsigned long long* m, int* shift);

// Longest batched sweep whose frame is one chunk: kBlock runs of up to
// kMaxRun u-samples (longer sweeps take the chunk-walking frame kernel).
constexpr int kMaxRun = 16;
// Dynamic LDS of the one-chunk batched frame kernel (the staged path:
// lds_path_doubles of the path must not exceed it; other sweeps take the
// chunk-walking kernel).  44 KB: two blocks per CU with the static LDS.
constexpr int kLdsPathDoubles = 5632;
// Sweeps of at most this many u-samples are framed by one wave each (four
// per block, no block barriers).  Short sweeps spend most of a block's time
// in its fixed steps; longer runs per lane than 4 lengthen a wave's serial
// walk more than they save (measured on the 4096-sweep batch).
constexpr int kWaveMaxU = 256;
// LDS doubles an open path of n control points and degree p needs when
// staged: knots, control points, weights (rational), per-span reciprocals.
constexpr long long lds_path_doubles(int n, int p, bool rat)
{
    return (long long)(n + p + 1) + 3LL * n + (rat ? n : 0) + (long long)(n - p) * (p * (p + 1) / 2);
}

struct BatchedKernels {
    const void* profile;
    const void* frame[8];        // by path degree (index 0 unused): sweeps of n_u <= kBlock*kMaxRun
    const void* frame_long[8];   // longer sweeps, or paths too large for the LDS staging
    const void* frame_wave[8];   // sweeps of n_u <= kWaveMaxU, one wave each
    const void* arc_pieces[8];   // arc-length tables (arc-length or adaptive sampling), by path degree
    const void* arc_cumsum;
    const void* arc_params[8];
    const void* surface;
};
// Kernel entry points for a precision combination (host stubs usable as
// graph kernel-node functions).
// tile_vertices = vertices per surface block: 256, 512, 1024 or 2048.
// ext: extended row records (a frame mode or law); arc: arc-length or
// adaptive u-sampling (lam != 0: adaptive), FP64 frame only; rat: the paths
// carry weights.
BatchedKernels batched_kernels(bool f64, bool t64, bool nrm, bool nontemporal, int tile_vertices, bool ext, bool arc,
                               bool adaptive, bool rat);

// Frame mode and sweep law of a batch (every sweep of the batch takes the
// batch's options): Frenet frames and/or one law for all sweeps, written as
// extended row records (kRowExt values).  law_len is the law's parameter
// domain length; a sweep's dl/du is law_len over its path's domain length.
struct BatchFrameExt {
    int frenet;
    int has_law;
    double law_len;
    DCurve law;
    const double* su;   // arc-length sampling: every sweep's sample parameters (at its row offset), else null
    const int* ss;      // and their spans
};

}  // namespace sweep
