/*
 * sweep.h -- C ABI of libsweep, dense evaluation of swept surfaces on
 * AMD Instinct MI355X (gfx950).
 *
 * A profile curve S(v) is swept along a path curve C(u); both are B-splines
 * given by control points, a knot vector (or the clamped / periodic uniform
 * default) and a degree, and the caller asks for n_u x n_v samples.  For
 * every (u_i, v_j) the library writes the vertex position
 *     X_ij = C(u_i) + S_x(v_j) r_i + S_y(v_j) s_i + S_z(v_j) t_i
 * and the unit normal N_ij = (X_v x X_u)/|X_v x X_u|, where (r_i, s_i, t_i) is
 * the rotation-minimizing frame of the path at u_i computed by the
 * double-reflection method (Wang, Juettler, Zheng & Liu, ACM TOG 27(1), 2008)
 * as a parallel prefix product of 3x3 rotations.
 *
 * The framing paper (arXiv 1110.5450) only introduces the notation: a path C,
 * a profile S and the tangent / normal / binormal of a curve.  It defines no
 * sweep, frame or B-spline evaluation; every operation below follows the
 * published method named at its entry point.
 *
 * Definitions (shared with the library's FP64 reference):
 *   knots   open curves: clamped uniform U = (0^{p+1}, 1/(n-p), ...,
 *           (n-p-1)/(n-p), 1^{p+1}) when no knots are given, else the given
 *           vector (non-decreasing, finite, interior multiplicity <= p,
 *           end multiplicity <= p+1); closed curves: periodic uniform
 *           U_k = k over the control polygon wrapped by p points.
 *   rational with weights w_k (NURBS, Piegl & Tiller, The NURBS Book ch. 4):
 *           C(u) = sum_k N_k(u) w_k P_k / sum_k N_k(u) w_k, derivatives from
 *           the homogeneous curve (w P, w) by the quotient rule; a closed
 *           curve wraps its weights with its control points.
 *   samples open: u_i = U_p + (U_n - U_p) * (i/(n_s-1)), both ends included;
 *           closed: t_j = p + (m*j)/n_s, the seam not repeated.
 *   span    U_k <= u < U_{k+1}; the last span at the right end of the domain.
 *   tangent t_i = C'(u_i)/|C'(u_i)|; where C'(u_i) = 0 the previous sample's
 *           tangent; at i = 0 the first nonzero control-polygon leg.
 *   r_0     the given initial normal projected onto the plane normal to t_0
 *           (if it is not parallel to t_0), else e_a projected, a = argmin |t_0[a]|
 *           (ties to the smaller index); s_i = t_i x r_i.
 *   step    M_i = H2 H1, H1 the reflection swapping x_i, x_{i+1}, H2 the one
 *           then taking H1 t_i to t_{i+1}; when |t_{i+1} - H1 t_i|^2 <= 1e-24
 *           (tangent reversal) the smallest rotation taking t_i to t_{i+1}
 *           (rotation by pi about the axis-rule direction of t_i if they are
 *           opposite); r_{i+1} = M_i r_i, re-projected and normalised.
 *   normal  X_v = R S'(v), X_u = (|C'| - S_x a - S_y b) t + S_z t', with
 *           a = r.C''/|C'|, b = s.C''/|C'|, t' = (C'' - (C''.t) t)/|C'| (the
 *           derivative of the continuous rotation-minimizing frame);
 *           N = 0 where the cross product is 0 or not finite.
 *
 * Memory: every buffer is allocated and owned by the caller.  Control points
 * and outputs are DEVICE pointers; knot vectors, counts and options are HOST
 * memory read before the call returns.  Positions and normals are written as
 * structure-of-arrays planes: element (c, i, j) of a sweep with N = n_u*n_v
 * vertices is at [c*N + i*n_v + j], c = x, y, z, in the output precision.
 * The batched calls concatenate per-sweep blocks whose planes are padded:
 * sweep k has plane stride P_k = n_u[k]*n_v[k] rounded up to a multiple of
 * 64 elements, its block starts at element off_k = 3 * sum_{k'<k} P_{k'},
 * and element (c, i, j) is at [off_k + c*P_k + i*n_v[k] + j].  The padding
 * elements are written as 0 by sweep_eval_batched and ignored by
 * sweep_backward.  (With 256-byte aligned buffers every plane then starts
 * on a cache-line boundary; see sweep_batched_output_elems.)
 *
 * Streams and errors: work is enqueued on the given stream (a hipStream_t,
 * NULL for the default stream) and the call returns without waiting for it.
 * Metadata is validated on the host before anything is enqueued; a non-OK
 * status means nothing was enqueued (except SWEEP_ERR_HIP, which reports a
 * failed launch).  Faults inside kernels surface at the caller's next
 * synchronisation.  sweep_last_error() returns a thread-local message for the
 * last non-OK status.  No call aborts or exits the process.
 */
#ifndef SWEEP_H
#define SWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWEEP_VERSION 105  /* major*100 + minor */
#define SWEEP_MAX_DEGREE 7

typedef enum {
    SWEEP_OK = 0,
    SWEEP_ERR_NULL_ARG = -1,      /* a required pointer is NULL */
    SWEEP_ERR_BAD_COUNT = -2,     /* n_ctrl < degree+1, or sizes overflow */
    SWEEP_ERR_BAD_DEGREE = -3,    /* degree outside 1..SWEEP_MAX_DEGREE */
    SWEEP_ERR_BAD_KNOTS = -4,     /* wrong ordering, NaN, bad multiplicity */
    SWEEP_ERR_BAD_GRID = -5,      /* n_u < 2, n_v < 3, or n_u*n_v >= 2^31 */
    SWEEP_ERR_BAD_PRECISION = -6, /* precision not SWEEP_F32 / SWEEP_F64 */
    SWEEP_ERR_WORKSPACE = -7,     /* workspace NULL or smaller than required */
    SWEEP_ERR_UNSUPPORTED = -8,   /* valid but not implemented (e.g. closed path) */
    SWEEP_ERR_HIP = -9,           /* a HIP runtime call or launch failed */
    SWEEP_ERR_BAD_OPTION = -10    /* an option field out of range */
} sweep_status;

typedef enum { SWEEP_F32 = 0, SWEEP_F64 = 1 } sweep_precision;

/*
 * Frame modes.  SWEEP_FRAME_RMF: the rotation-minimizing frame above.
 * SWEEP_FRAME_FRENET: the Frenet frame of the path, pointwise: r = the
 * principal normal normalize(C'' - (C''.t) t), s = t x r (the binormal);
 * where |C'' - (C''.t) t| <= 1e-8 |C''| (straight pieces, inflections) r is
 * the axis-rule vector of t.  The surface normal then uses the Frenet frame's
 * derivative: the frame turns about t at the rate omega = |C'| tau relative
 * to a rotation-minimizing frame, with the torsion
 * tau = det(C', C'', C3)/|C' x C''|^2 (C3 the third derivative; omega = 0
 * where the axis rule was used).
 *
 * Sweep law (sweep_options.law): an open B-spline L(l) whose control points
 * hold (sigma, theta, unused), sampled like the path (sample i of n_u on its
 * own domain).  At u-sample i the profile point S becomes
 *     sigma (cos th S_x - sin th S_y, sin th S_x + cos th S_y, S_z),
 * i.e. the cross-section is scaled by sigma and turned about t by theta
 * (radians); the surface normal includes d(sigma)/du and d(theta)/du.
 * Frame modes and laws are supported by sweep_eval (and sweep_autotune) and
 * by sweep_eval_batched (and sweep_autotune_batched), where the options'
 * frame mode and law apply to every sweep of the batch (the law sampled on
 * each sweep's own u-samples; FP64 frame precision only, else
 * SWEEP_ERR_UNSUPPORTED); sweep_frames and the adjoint entry points return
 * SWEEP_ERR_UNSUPPORTED for them.
 */
typedef enum { SWEEP_FRAME_RMF = 0, SWEEP_FRAME_FRENET = 1 } sweep_frame_mode;

/*
 * Path sampling.  SWEEP_U_PARAMETER: the uniform parameter samples above.
 * SWEEP_U_ARCLENGTH: u_i with s(u_i) = (i/(n_u-1)) s(U_n), s(u) the arc
 * length from the start of the domain (u_0 and u_{n_u-1} the domain ends).
 * Every non-empty knot span is cut into 32 equal pieces integrated by
 * 8-point Gauss-Legendre (a cumulative table); inside the piece holding a
 * target, Newton's method on s(u) - target kept in a bisection bracket, to
 * |du| <= 4 eps max(1, |u|).  SWEEP_U_ADAPTIVE: the same with the density
 * |C'| (1 + u_lambda kappa) in place of |C'| (kappa the path's curvature):
 * equal steps of arc length plus u_lambda times the tangent's turning angle,
 * so samples crowd where the path bends (u_lambda = 0 is arc length).
 * Supported by sweep_eval (not with a law), sweep_frames and
 * sweep_eval_batched (every sweep of the batch, FP64 frame, not with a frame
 * mode or law); otherwise, and in the adjoint entry points, the call returns
 * SWEEP_ERR_UNSUPPORTED.
 */
typedef enum { SWEEP_U_PARAMETER = 0, SWEEP_U_ARCLENGTH = 1, SWEEP_U_ADAPTIVE = 2 } sweep_u_sampling;

/* A B-spline curve. */
typedef struct sweep_curve_s {
    int32_t n_ctrl;      /* control points (for a closed curve: the m distinct ones) */
    int32_t degree;      /* 1..SWEEP_MAX_DEGREE */
    int32_t closed;      /* 0 open, 1 closed periodic uniform (profiles only) */
    int32_t reserved;
    const double *ctrl;  /* DEVICE, n_ctrl x 3 FP64, row-major (x, y, z) */
    const double *knots; /* HOST, n_ctrl+degree+1 FP64, or NULL for the default
                            knots; must be NULL for a closed curve */
    const double *weights; /* DEVICE, n_ctrl FP64 weights (a rational curve, see
                              "rational" above), or NULL (polynomial B-spline);
                              weights must be positive and finite -- they are
                              device data and not checked */
} sweep_curve;

/* Options; sweep_default_options() fills the defaults noted here. */
typedef struct {
    int32_t out_precision;    /* SWEEP_F32 (default) or SWEEP_F64: type of pos/nrm */
    int32_t frame_precision;  /* SWEEP_F64 (default) or SWEEP_F32: precision of the
                                 step matrices, the frame scan and re-orthonormalisation */
    int32_t reorthonormalize; /* 1 (default): r_i projected onto t_i^perp and
                                 normalised, s_i = t_i x r_i; 0: r_i = P_i r_0 raw
                                 (precision study) */
    int32_t has_initial_normal;  /* 0 (default): axis rule; 1: use initial_normal */
    double initial_normal[3];
    int32_t tile_config;      /* -1 (default): tuned/automatic; >= 0 a fixed
                                 surface-kernel configuration (sweep_tile_config_count) */
    int32_t frame_mode;       /* SWEEP_FRAME_RMF (default) or SWEEP_FRAME_FRENET, see above */
    const struct sweep_curve_s *law; /* NULL (default) or a sweep law, see above */
    int32_t u_sampling;       /* SWEEP_U_PARAMETER (default), SWEEP_U_ARCLENGTH or
                                 SWEEP_U_ADAPTIVE, see above */
    int32_t batch_stages;     /* sweep_eval_batched: 0 (default) automatic, else 1-4
                                 pipeline stages of the frame/surface schedule
                                 (sweeps grouped by path length; the surface of a
                                 stage is written while the next stage's frames
                                 are formed) */
    double u_lambda;          /* SWEEP_U_ADAPTIVE: length weight of the turning angle (>= 0, finite) */
} sweep_options;

/* A batch of independent sweeps.  Per-sweep arrays are HOST memory with
 * n_sweeps entries; control points of all paths (profiles) are packed in one
 * DEVICE buffer, sweep k's starting at point offset sum_{k'<k} path_n[k'].
 * Knot vectors, if given, are concatenated per sweep in HOST memory. */
typedef struct {
    int32_t n_sweeps;
    int32_t reserved;
    const int32_t *path_n;       /* control points per path */
    const int32_t *path_degree;
    const int32_t *prof_n;       /* control points per profile */
    const int32_t *prof_degree;
    const int32_t *prof_closed;  /* NULL: every profile closed */
    const int32_t *n_u;
    const int32_t *n_v;
    const double *path_knots;    /* NULL: clamped uniform; else path_n[k]+path_degree[k]+1 per sweep */
    const double *prof_knots;    /* NULL: default; else one vector per OPEN profile, in sweep order */
    const double *path_ctrl;     /* DEVICE, sum(path_n) x 3 FP64 */
    const double *prof_ctrl;     /* DEVICE, sum(prof_n) x 3 FP64 */
    const double *path_weights;  /* DEVICE, sum(path_n) FP64 packed like path_ctrl, or NULL
                                    (every path polynomial) */
    const double *prof_weights;  /* DEVICE, sum(prof_n) FP64, or NULL */
} sweep_batch;

void sweep_default_options(sweep_options *opt);

/*
 * Evaluate one sweep: positions (and normals if nrm != NULL) on the
 * n_u x n_v grid.  pos/nrm: DEVICE, 3*n_u*n_v elements of the output
 * precision.  workspace: DEVICE, at least sweep_eval_workspace_size() bytes,
 * 256-byte aligned; it holds knots, curve samples, step-matrix carries, the
 * per-row frame table and the profile table, and may be reused once the
 * stream has passed this call.  With user knots the knot copy to the device
 * is a blocking copy from pageable memory.
 */
sweep_status sweep_eval(const sweep_curve *path, const sweep_curve *profile,
                        int32_t n_u, int32_t n_v, const sweep_options *opt,
                        void *pos, void *nrm, void *workspace, size_t ws_bytes,
                        void *stream);
size_t sweep_eval_workspace_size(const sweep_curve *path, const sweep_curve *profile,
                                 int32_t n_u, int32_t n_v, const sweep_options *opt);

/*
 * sweep_eval without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  The workspace is a static device array
 * of SWEEP_NOALLOC_WORKSPACE_BYTES bytes that the library's code object holds
 * on every GPU it runs on, from load until the process ends; the call itself
 * allocates and frees nothing.  Arguments, output layout and results are
 * those of sweep_eval.  A sweep whose sweep_eval_workspace_size() exceeds
 * the array is rejected with SWEEP_ERR_WORKSPACE before anything is
 * enqueued (at FP32 output and FP64 frame: above about 490,000 u-samples).
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (nothing in it needs to start at zero): calls on one
 * stream are ordered, but calls that can overlap on one GPU (different
 * streams, or threads without ordering between them) race on the array and
 * give undefined results.
 */
#define SWEEP_NOALLOC_WORKSPACE_BYTES (64u << 20)
sweep_status sweep_eval_noalloc(const sweep_curve *path, const sweep_curve *profile,
                                int32_t n_u, int32_t n_v, const sweep_options *opt,
                                void *pos, void *nrm, void *stream);

/*
 * The moving frame alone: for each u-sample i of the path, write the 16-value
 * row record (x_i[3], r_i[3], s_i[3], t_i[3], |C'(u_i)|, a_i, b_i, 0) with
 * a = r.C''/|C'|, b = s.C''/|C'|, in the output precision, to frames (DEVICE,
 * 16*n_u elements).  Same kernels and options as sweep_eval (frame
 * precision, re-orthonormalisation, initial normal).
 */
sweep_status sweep_frames(const sweep_curve *path, int32_t n_u, const sweep_options *opt, void *frames,
                          void *workspace, size_t ws_bytes, void *stream);
size_t sweep_frames_workspace_size(const sweep_curve *path, int32_t n_u, const sweep_options *opt);

/*
 * Evaluate a batch of independent sweeps in one frame launch and one
 * persistent surface launch, replayed from a HIP graph.  The first call with
 * a new batch shape (all per-sweep host arrays, knots and options) validates
 * it, uploads per-sweep descriptors with a blocking copy, picks the surface
 * schedule and builds the graph; later calls with the same shape only update
 * the graph's pointer arguments and launch it.  Sweep k's output equals
 * sweep_eval's for that sweep (same kernels, same arithmetic).
 * pos/nrm: DEVICE, sweep_batched_output_elems(batch) elements in the padded
 * batched layout, best 256-byte aligned.
 */
sweep_status sweep_eval_batched(const sweep_batch *batch, const sweep_options *opt,
                                void *pos, void *nrm, void *workspace, size_t ws_bytes,
                                void *stream);
size_t sweep_batched_workspace_size(const sweep_batch *batch, const sweep_options *opt);
/* Elements of one batched output buffer: 3 * sum_k P_k (padded layout
 * above); 0 if batch, n_u or n_v is NULL, n_sweeps < 1 or a count is
 * negative.  Counts are not otherwise validated. */
int64_t sweep_batched_output_elems(const sweep_batch *batch);

/*
 * Adjoint of the positions: given grad_pos = dL/dpos (DEVICE, same layout and
 * precision as the batched pos output), accumulate nothing but WRITE
 * grad_path_ctrl (DEVICE, sum(path_n) x 3 FP64) and grad_prof_ctrl (DEVICE,
 * sum(prof_n) x 3 FP64), the gradients of L with respect to the control
 * points.  The frame is recomputed in FP64; reductions accumulate in FP64 in
 * a fixed order (deterministic).  Knots and weights are held fixed here;
 * sweep_backward_ex also gives their gradients.
 * At tangent reversals the step rotation is treated as locally constant.
 * sweep_backward(..., grad_pos, ...) is sweep_backward_ex with
 * grad_nrm = NULL.
 *
 * sweep_backward_ex also takes grad_nrm = dL/dnrm (DEVICE, same layout and
 * precision as the batched nrm output, or NULL); grad_pos may be NULL when
 * grad_nrm is not (both NULL is SWEEP_ERR_NULL_ARG), and params (or NULL)
 * asks for gradients with respect to knots and weights, see below.  The normal is
 * N = (X_v x X_u)/|X_v x X_u| with X_u from the continuous frame's derivative
 * (its dependence on C'' through the frame's rate of turn is included);
 * where the cross product is 0 or not finite the normal is the constant 0
 * and passes no gradient.  Samples with C' = 0 pass none through a, b, |C'|.
 * The workspace size covers both entry points.
 */
sweep_status sweep_backward(const sweep_batch *batch, const sweep_options *opt,
                            const void *grad_pos, double *grad_path_ctrl,
                            double *grad_prof_ctrl, void *workspace, size_t ws_bytes,
                            void *stream);

/*
 * Knot and weight gradients of sweep_backward_ex (each pointer NULL to skip).
 * path_knots: DEVICE, packed like batch->path_knots (which must be given),
 * dL/dU_m for every entry; prof_knots: the same for the open profiles' given
 * knots (closed profiles have none).  The sample parameters follow the
 * domain ends U_p and U_n, so those two entries also carry the samples'
 * motion.  An entry inside a run of equal knots gets the partial derivative
 * of the evaluation formula with the run's other entries held; the sum over
 * the run is the derivative for moving the run as a whole (the first and last
 * knots of a vector never enter the curve: 0).  path_weights / prof_weights:
 * DEVICE, packed like batch->path_weights / prof_weights (which must be
 * given), dL/dw_k.  A request without the matching batch field is
 * SWEEP_ERR_BAD_OPTION.
 */
typedef struct {
    double *path_knots;
    double *prof_knots;
    double *path_weights;
    double *prof_weights;
} sweep_param_grads;

sweep_status sweep_backward_ex(const sweep_batch *batch, const sweep_options *opt,
                               const void *grad_pos, const void *grad_nrm,
                               double *grad_path_ctrl, double *grad_prof_ctrl,
                               const sweep_param_grads *params,
                               void *workspace, size_t ws_bytes, void *stream);
size_t sweep_backward_workspace_size(const sweep_batch *batch, const sweep_options *opt);

/*
 * Launch timing for profiling.  sweep_trace_enable(n), n > 0, makes the next
 * n sweep_eval calls record HIP events on their stream around the frame
 * stage (knots, curve samples, profile table, frame scan) and the surface
 * stage; n = 0 stops recording.  sweep_trace_read waits for the recorded
 * events, writes up to max (stage, milliseconds) pairs -- stage 0 frame,
 * stage 1 surface -- in call order, clears the record and returns the number
 * written (or a negative status).  Events are created by the enable call, so
 * enable outside any graph capture.
 */
sweep_status sweep_trace_enable(int32_t max_calls);
int32_t sweep_trace_read(int32_t *stage, float *ms, int32_t max);

/*
 * Surface-kernel autotuner.  Evaluates the sweep once, then times every fixed
 * surface configuration on it with HIP events on `stream` (the call waits for
 * the stream), using the caller's buffers, and records the fastest under the
 * shape class (device architecture and CU count, output precision,
 * n_v % 256 == 0, floor(log2 n_v), floor(log2 n_u*n_v)).  Later calls with
 * tile_config = -1 in the same class use the recorded configuration.  When
 * the environment variable SWEEP_TUNE_CACHE names a file, the table is read
 * from it on first use and rewritten (to a temporary file, then renamed)
 * after each tuning, one entry per line: kind (single / batch), architecture,
 * CU count, the five class integers, configuration, milliseconds.
 * best_config / best_ms may be NULL.
 */
sweep_status sweep_autotune(const sweep_curve *path, const sweep_curve *profile, int32_t n_u, int32_t n_v,
                            const sweep_options *opt, void *pos, void *nrm, void *workspace, size_t ws_bytes,
                            void *stream, int32_t *best_config, float *best_ms);

/* The surface configuration tile_config = -1 selects for this shape and
 * output precision (the tuned one if recorded, else the built-in rule). */
int32_t sweep_surface_config_for(int32_t n_u, int32_t n_v, int32_t out_precision);

/*
 * Batched autotuner.  Evaluates the batch once with tile_config = -1, then
 * times the surface kernel of every linear tile configuration (256, 512,
 * 1024 and 2048 consecutive vertices per block, plain and nontemporal
 * stores; a batch has no column tiles) on that evaluation's row and profile
 * tables, five launches each with HIP events on `stream` (the call waits for
 * the stream; the outputs are rewritten with the same values), and records
 * the fastest under the batch's shape class: device architecture and CU
 * count, output precision, whether normals are written, floor(log2) of the
 * sweep count, of the total vertex count and of the mean n_v.  Later
 * sweep_eval_batched calls with tile_config = -1 in that class use it (the
 * plan of that configuration is built on the next call).  The table is the
 * one sweep_autotune keeps, persisted through SWEEP_TUNE_CACHE.  Arguments
 * as sweep_eval_batched; best_config / best_ms may be NULL.
 */
sweep_status sweep_autotune_batched(const sweep_batch *batch, const sweep_options *opt, void *pos, void *nrm,
                                    void *workspace, size_t ws_bytes, void *stream, int32_t *best_config,
                                    float *best_ms);

/* The tile_config index sweep_eval_batched uses for this batch and options
 * (the tuned one for tile_config = -1 if recorded, else linear tiles of 1024
 * vertices with nontemporal stores); -1 for an invalid batch. */
int32_t sweep_batched_config_for(const sweep_batch *batch, const sweep_options *opt, int32_t with_normals);

/*
 * Triangle list of an n_u x n_v grid (vertex (i, j) has index i*n_v + j, the
 * single-sweep layout): every quad (i, j), (i+1, j), (i, j+1), (i+1, j+1),
 * j+1 taken modulo n_v when closed_v (a closed profile), gives the triangles
 *     (i,j) (i,j+1) (i+1,j)   and   (i+1,j) (i,j+1) (i+1,j+1),
 * counter-clockwise seen from the side the normal X_v x X_u points to.
 * tri: DEVICE, 3 int32 per triangle, quads in row-major order; n_tri (HOST,
 * may be NULL) receives 2 (n_u-1) (closed_v ? n_v : n_v-1).  max_tri is the
 * capacity of tri in triangles; a smaller capacity is an error
 * (SWEEP_ERR_WORKSPACE) and nothing is written.
 */
sweep_status sweep_triangles(int32_t n_u, int32_t n_v, int32_t closed_v, int32_t *tri, int64_t max_tri,
                             int64_t *n_tri, void *stream);

/* Number of fixed surface-kernel configurations accepted in tile_config. */
int32_t sweep_tile_config_count(void);
/* Configuration k: info (HOST, 4 int32) receives its kind (0 column tiles of
 * 256 columns, 1 linear tiles), rows per block (kind 0), vertices per block
 * (kind 1) and whether the stores are nontemporal. */
sweep_status sweep_tile_config_info(int32_t k, int32_t *info);

/* Thread-local text describing the last non-OK status on this thread. */
const char *sweep_last_error(void);

int32_t sweep_version(void);

/* Free cached batch plans and HIP graphs (library-owned device memory). */
void sweep_release_caches(void);

#ifdef __cplusplus
}
#endif

#endif /* SWEEP_H */
