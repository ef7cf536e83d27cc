/*
 * fif.h -- C ABI of the MI355X Fisher Information Field library (libfif.so).
 *
 * Method: Zhang & Scaramuzza, "Fisher Information Field: an Efficient and
 * Differentiable Map for Perception-aware Planning", arXiv 2008.03324.
 *
 * Memory and ownership
 *   Every array argument is a DEVICE pointer (HBM of the current HIP device)
 *   unless its comment says "host".  Struct arguments (fif_grid, fif_vis,
 *   fif_pinhole, fif_field) are host structs passed by pointer.  The caller
 *   owns every buffer; the library never allocates or frees device memory.
 *
 * Streams and errors
 *   Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *   asynchronous.  Argument errors are detected on the host before anything is
 *   enqueued and return FIF_EINVAL; a failed launch returns FIF_EDEVICE and
 *   fif_last_error() (thread-local) holds the HIP message.  Nothing throws
 *   across the ABI.  NaN inputs give NaN outputs, not errors.
 *
 * Sizes
 *   Pose counts, landmark counts and voxel-id counts may be up to 2^40, sweep
 *   positions up to 2^31 - 1 (FIF_EINVAL beyond).  A call whose input is
 *   longer than one dispatch can cover (2^30 work-items) is split into several
 *   launches on the same stream; the results are the same as in one launch.
 *   fif_build and fif_update cover the grid with one launch of the build
 *   kernel (after the landmark sort when given a workspace) and return
 *   FIF_EUNSUPPORTED for grids with nx > 134,217,720, ny > 524,280 or
 *   nz > 262,140.
 *
 * Conventions
 *   Pose T_wc = {R_wc, t}: t is the camera position in the world, R_wc = R(q)
 *   with q = (w, x, y, z) Hamilton (need not be unit: the library normalises).
 *   The camera optical axis is e3, so z = R_wc e3 (Sec. V-B).  Perturbations
 *   are global (left) se(3) about the world origin (Sec. V-A, eq:deriv_se3
 *   first form, eq:jac_pose_global); so(3) gradients are w.r.t. phi in
 *   R <- exp([phi]x) R.
 *   Grid: voxel (i, j, k) has its centre at origin + (i, j, k) h; linear index
 *   i + nx (j + ny k) (x fastest).
 *   Landmark membership V_t (Sec. V, first step): a landmark p counts for a
 *   position t iff max(r_min^2, 1e-12) <= n^2 <= r_max^2, n^2 evaluated in FP32
 *   as fma(dz, dz, fma(dy, dy, dx*dx)) with d = fl32(p) - fl32(t), bounds
 *   rounded to FP32 (r_max = INFINITY keeps every landmark, as in Sec. VII-A).
 *   Visibility: the quadratic model of eq:quad_vis_approx with coefficients
 *   fixed by eq:quadratic_conditions from (half_fov, v_alpha).
 *   Noise: sigma_bearing is the bearing noise in radians (1 px at f = 300 px
 *   is 1/300); I_i = J^T J / sigma^2 (eq:fim_gaussian).
 */
#ifndef FIF_H
#define FIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fif_status;
#define FIF_OK 0
#define FIF_EINVAL (-1)       /* bad argument (checked on the host, nothing enqueued) */
#define FIF_ENOMEM (-2)       /* workspace too small */
#define FIF_EDEVICE (-3)      /* HIP runtime or launch error, see fif_last_error() */
#define FIF_EUNSUPPORTED (-4) /* valid but not implemented combination */

/* Precision of a field or of a point-cloud sum. */
#define FIF_FP32_NAIVE 0 /* FP32 arithmetic, FP32 accumulation */
#define FIF_FP32_COMP 1  /* FP32 arithmetic, compensated (two-level TwoSum) accumulation */
#define FIF_FP64 2       /* FP64 throughout */

/* Field kinds. */
#define FIF_KIND_INFO 0  /* positional information factor C_I (eq:general_info_pif) */
#define FIF_KIND_TRACE 1 /* positional trace factor C_Tr (eq:general_trace_pif) */
/* The trace factor stored per cell: each voxel holds the 10 factors of the 8
 * corners of the cell whose lowest corner it is (320 B in FP32, 6.7x the
 * FIF_KIND_TRACE field), so that a trilinear query reads one contiguous block
 * (3 lines of 128 B) instead of 8 scattered records.  Same values, same
 * results as FIF_KIND_TRACE, bit for bit; trades memory for query traffic. */
#define FIF_KIND_TRACE_CELLS 2

/* Metric mask; output columns follow this bit order.  FIF_FIM21 appends the 21
 * upper-triangle entries (row-major) of the 6x6 FIM. */
#define FIF_TRACE 1u
#define FIF_LMIN 2u
#define FIF_LOGDET 4u
#define FIF_FIM21 8u

/* Interpolation of the factors (Sec. VI-A: nearest neighbour or interpolation). */
#define FIF_TRILINEAR 0 /* over the 8 surrounding voxel centres */
#define FIF_NEAREST 1   /* round-half-up voxel */

/* Per-query flags (not errors). */
#define FIF_FLAG_CLAMPED 1u  /* position outside the hull of voxel centres, clamped */
#define FIF_FLAG_NOT_PD 2u   /* FIM not positive definite: logdet is NaN */
#define FIF_FLAG_LMIN_TIE 4u /* smallest eigenvalue within 1e-8 lambda_max of the next */

typedef struct {
  double origin[3]; /* centre of voxel (0, 0, 0), metres */
  double h;         /* voxel edge, metres */
  int32_t nx, ny, nz;
  int32_t reserved; /* must be 0 */
} fif_grid;

typedef struct {
  double half_fov;      /* alpha, radians (pi/4 for a 90 deg FoV) */
  double v_alpha;       /* quadratic visibility at the FoV boundary */
  double sigma_bearing; /* radians */
  double r_min, r_max;  /* V_t range predicate, metres; r_max may be INFINITY */
} fif_vis;

typedef struct {
  double fx, fy, cx, cy; /* pixels */
  int32_t width, height; /* image bounds: 0 <= u < width, 0 <= v < height */
} fif_pinhole;

typedef struct {
  fif_grid grid;
  fif_vis vis;
  int32_t prec; /* FIF_FP32_NAIVE | FIF_FP32_COMP | FIF_FP64 */
  int32_t kind; /* FIF_KIND_INFO | FIF_KIND_TRACE */
  void* data;   /* device buffer of fif_field_bytes(&grid, prec, kind) bytes, 256-B aligned */
} fif_field;

/* Bytes of the device buffer of a field.  The layout is private to the
 * library; fif_field_export recovers the paper's blocks from it.  Returns 0 for
 * an invalid grid, precision or kind. */
size_t fif_field_bytes(const fif_grid* grid, int32_t prec, int32_t kind);

/* Bytes of the optional fif_build / fif_update workspace for n_landmarks
 * landmarks (0 when n_landmarks <= 0 or the grid/precision is invalid).  With
 * it, fif_build first orders the landmarks
 * spatially (Morton keys, stable radix sort) and skips, per voxel tile, every
 * batch of landmarks whose bounding box is out of range; with a NULL workspace
 * every (voxel, landmark) pair is tested in input order.  Both orders give the
 * same field up to rounding, each deterministic.  The sort (rocPRIM radix sort)
 * enqueues a hipMemsetAsync: keep calls given a workspace out of captured HIP
 * graphs (pass NULL there). */
size_t fif_workspace_bytes(const fif_grid* grid, int64_t n_landmarks, int32_t prec);

/* Build a field (Sec. VI-A): for every voxel centre t_v,
 *   C_I(t_v) = sum_{i in V_{t_v}} diag6(vp(u_i)) I_i      (eq:general_info_pif)
 * or, for FIF_KIND_TRACE, C_Tr(t_v) = sum vp(u_i) Tr(I_i)  (eq:general_trace_pif).
 * landmarks: double[n_landmarks][3], world coordinates.  field->data is
 * overwritten.  workspace: NULL, or 256-B aligned device memory of at least
 * fif_workspace_bytes() bytes (FIF_ENOMEM if smaller); it is scratch only.
 * Deterministic: the summation order is fixed. */
fif_status fif_build(const double* landmarks, int64_t n_landmarks, fif_field* field,
                     void* workspace, size_t workspace_bytes, void* stream);

/* fif_build without a workspace argument and without allocating: for callers
 * that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc).  The landmarks are ordered
 * spatially and batch-culled exactly as fif_build does with a workspace (the
 * same sort, the same summation order: the field equals fif_build's bit for
 * bit), but the sort's scratch lives in a static device array of
 * FIF_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends.  The call makes no hipMalloc/hipFree and no
 * allocating library call.  Nothing in the scratch needs to start at zero:
 * every byte the build reads is written earlier in the same call.
 * Limits and errors: as fif_build, plus FIF_EINVAL (before anything is
 * enqueued) when fif_workspace_bytes(grid, n_landmarks, prec) exceeds
 * FIF_NOALLOC_SCRATCH_BYTES (about 1.19 million landmarks: the sort takes
 * 56 bytes per landmark).  All calls on one
 * device share that device's scratch: calls that overlap in time on one
 * device (different streams or threads without ordering) race and must not be
 * made.  Like fif_build with a workspace, the sort enqueues a
 * hipMemsetAsync, so keep the call out of captured HIP graphs. */
#define FIF_NOALLOC_SCRATCH_BYTES (64u << 20)
fif_status fif_build_noalloc(const double* landmarks, int64_t n_landmarks, fif_field* field,
                             void* stream);

/* Incremental update (Sec. VI-A, "Offline Processing vs. Online Update"): add
 * (sign = +1) or remove (sign = -1) the contribution of the given landmarks to
 * every voxel whose centre has them in range.  Same landmark layout and
 * workspace as fif_build (fif_workspace_bytes() for n_landmarks): with a
 * workspace the added landmarks are ordered spatially and voxel tiles out of
 * range of a whole batch of them skip it; with NULL every voxel tests every
 * added landmark.  Both give the same sums up to rounding order. */
fif_status fif_update(const double* landmarks, int64_t n_landmarks, int32_t sign,
                      fif_field* field, void* workspace, size_t workspace_bytes, void* stream);

/* Batched pose query (Sec. VI-A, eq:fim_separation): F = V_I(R) C_I(t) with
 * C_I(t) interpolated from the voxel centres, reduced to the requested metrics
 * (eq:cost_info: trace, smallest eigenvalue, log-det; the latter two in FP64).
 * t: [m][3], q: [m][4]; float for FP32 fields, double for FP64 fields.
 * out: double[m][ncols], ncols = popcount(metrics & 7) + (metrics & FIF_FIM21 ? 21 : 0).
 * flags: uint8[m] or NULL.  For trace fields (FIF_KIND_TRACE, FIF_KIND_TRACE_CELLS)
 * only FIF_TRACE is valid.
 * m = 0 is allowed (nothing is enqueued). */
fif_status fif_query(const fif_field* field, const void* t, const void* q, int64_t m,
                     uint32_t metrics, int32_t interp, double* out, uint8_t* flags,
                     void* stream);

/* Gradient of L = sum_r sum_c dL_dout[r][c] s_c(pose_r) w.r.t. each pose
 * (a metric whose dL_dout is 0 is left out of L: a FIM that is not positive
 * definite gives NaN gradients only where its log-det weight is nonzero):
 *   dL_dt[m][3]   through the trilinear weights,
 *   dL_dphi[m][3] w.r.t. the left so(3) perturbation of R_wc.
 * metrics: subset of FIF_TRACE | FIF_LMIN | FIF_LOGDET (dL_dout has that many
 * columns, in bit order).  dL_dt/dL_dphi have the type of t (float or double).
 * out (double[m][popcount], or NULL) receives the forward metrics as well,
 * bit for bit those of fif_query on the same field, poses and metrics.
 * Trilinear interpolation only; the derivative is one-sided on cell faces. */
fif_status fif_query_grad(const fif_field* field, const void* t, const void* q, int64_t m,
                          uint32_t metrics, const double* dL_dout, void* dL_dt, void* dL_dphi,
                          double* out, void* stream);

/* Bytes of the optional pc_query workspace for n_landmarks landmarks and m
 * poses (0 for non-positive sizes, an invalid precision or n_landmarks >=
 * 2^32).  Poses are ordered in passes of at most 2^26, so the size stops
 * growing with m there. */
size_t pc_workspace_bytes(int64_t n_landmarks, int64_t m, int32_t prec);

/* Point-cloud brute force (eq:cost_info, eq:vis_fim): F = sum_{i in V_t} v_i I_i
 * for each pose, with v_i the quadratic visibility of z.u_i (cam == NULL,
 * eq:quad_vis_approx, unclamped) or the exact pinhole test (eq:exact_vis_func:
 * in front of the camera and inside [0, width) x [0, height)).
 * t, q: float for FP32 precisions, double for FIF_FP64.  out as fif_query.
 * workspace: NULL, or 256-B aligned device memory of at least
 * pc_workspace_bytes() bytes (FIF_ENOMEM if smaller; scratch only).  With a
 * workspace and a finite r_max, landmarks and poses are first ordered by the
 * Morton code of their cell (edge r_max / 32; cell index floor(x * 32 / r_max)
 * per axis taken modulo 1024, codes sorted stably), and each group of 256
 * consecutive ordered poses skips every batch of 256 ordered landmarks whose
 * bounding box is out of range of the group's box.  A skipped batch holds no
 * landmark in range of those poses, and each pose sums its landmarks in the
 * ordered sequence, so the results equal those of the call without a
 * workspace given the landmarks in that order, bit for bit; results are
 * written in the caller's pose order.  With NULL (or r_max = INFINITY) every
 * pair is tested in input order.  The sort enqueues hipMemsetAsync: keep calls
 * given a workspace out of captured HIP graphs. */
fif_status pc_query(const double* landmarks, int64_t n_landmarks, const fif_vis* vis,
                    const fif_pinhole* cam, int32_t prec, const void* t, const void* q,
                    int64_t m, uint32_t metrics, double* out, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Optimal-view sweep (Sec. VII-A "Relative Measures": the optimal view at a
 * position is the rotation that maximises the metric).  Under the smooth
 * visibility models the FIM at a position depends on the rotation only through
 * the optical axis z (eq:quad_vis_component), so the sweep runs over candidate
 * axes: for each position the factor blocks are interpolated once and
 * contracted with vr(z) (eq:fim_separation) for every axis.
 * t: [n_pos][3] (float for FP32 fields, double for FP64 fields).
 * dirs: double[n_dir][3] unit optical axes (device).  metric: exactly one of
 * FIF_TRACE, FIF_LMIN, FIF_LOGDET.  values: double[n_pos][n_dir] or NULL;
 * best: int64[n_pos] or NULL, the index of the largest value (lowest index
 * among equal values; NaN values never win; -1 when every value is NaN).
 * Information fields only. */
fif_status fif_view_sweep(const fif_field* field, const void* t, int64_t n_pos,
                          const double* dirs, int64_t n_dir, uint32_t metric, int32_t interp,
                          double* values, int64_t* best, void* stream);

/* The paper's positional information factor of the listed voxels, recovered
 * from the field: blocks[n][10][21] (double), block k = sum_i vp_k(u_i) I_i in
 * world coordinates (eq:general_info_pif), 21 = upper triangle row-major.
 * For trace fields: blocks[n][10] = C_Tr.  voxel_ids: int64[n]. */
fif_status fif_field_export(const fif_field* field, const int64_t* voxel_ids, int64_t n,
                            double* blocks, void* stream);

/* ------------------------------------------------------------------------
 * GP visibility fields (Sec. V-B "GP Regression"; G-I-N_s / G-T-N_s of Sec.
 * VII-A).  The visibility of a landmark with bearing u seen along optical axis
 * z is the GP posterior mean
 *   v_gp(z, u) = K_z (K^s + noise I)^-1 v^s(u),
 *   K_z[g] = k(z, z_g),  K^s[g][h] = k(z_g, z_h),  k(a, b) = exp(-|a - b|^2 / (2 l^2)),
 *   v^s_g(u) = 1 / (1 + exp(-k_s (z_g . u - cos alpha)))      (eq:sigmoid_vis_func)
 * over N_s sample axes z_g.  eq:gp_vis_approx prints K_z K^s v^s; the inverse
 * of the posterior mean is the reading taken here.  So vr = K_z and
 * vp = (K^s + noise I)^-1 v^s in eq:fim_separation, N_v = N_s.
 *
 * The device buffer stores, per voxel and sample axis, the sums of v^s_g(u_i)
 * times the camera-frame terms of I_i (information fields) or of v^s_g(u_i)
 * Tr(I_i) (trace fields); the inverse is applied on the query side.  The field
 * therefore depends on the axes, k_s, alpha, the range bounds and the
 * precision, but not on l or the noise.  fif_gp_export recovers the paper's
 * factors C_g = sum_i vp_g(u_i) I_i.
 * ---------------------------------------------------------------------- */

#define FIF_GP_MAX_NS 160 /* largest N_s (the paper uses 30..150) */

typedef struct {
  int32_t n_s;        /* number of sample axes, 1..FIF_GP_MAX_NS */
  int32_t reserved;   /* must be 0 */
  double k_s;         /* sigmoid slope (15 in the paper) */
  double length;      /* SE length scale l > 0 */
  double noise;       /* variance added to the diagonal of K^s (1e-10 in the paper) */
  const double* axes; /* device double[n_s][3], unit sample axes */
  double* kinv;       /* device double[n_s][n_s]: (K^s + noise I)^-1, filled by fif_gp_setup */
} fif_gp;

typedef struct {
  fif_grid grid;
  fif_vis vis;  /* half_fov = alpha of the sigmoid, sigma_bearing, r_min, r_max (v_alpha unused) */
  fif_gp gp;
  int32_t prec; /* FIF_FP32_NAIVE | FIF_FP32_COMP | FIF_FP64 */
  int32_t kind; /* FIF_KIND_INFO | FIF_KIND_TRACE */
  void* data;   /* device buffer of fif_gp_field_bytes() bytes, 256-B aligned */
} fif_gp_field;

/* Bytes of the device buffer of a GP field; 0 for invalid arguments. */
size_t fif_gp_field_bytes(const fif_grid* grid, int32_t n_s, int32_t prec, int32_t kind);

/* (K^s + noise I)^-1 of the model into gp->kinv (FP64 Cholesky on the device).
 * FIF_EINVAL for n_s out of range, NULL pointers or l <= 0.  A matrix that is
 * not positive definite gives NaN in kinv (no error: detected on the device). */
fif_status fif_gp_setup(const fif_gp* gp, void* stream);

/* Log marginal likelihood of each candidate length scale (Sec. V-B: l is
 * chosen by maximising it), for training outputs y_t[g] = v^s_g(u_t) at the
 * training bearings u_t (unit, device double[n_train][3]):
 *   sum_t -1/2 y_t^T K_y^-1 y_t - n_train/2 log|K_y| - n_train n_s/2 log 2 pi,
 * K_y = K^s(l) + noise I.  lengths: device double[n_len]; lml: device
 * double[n_len] (-inf where K_y is not positive definite).  gp->length and
 * gp->kinv are not used. */
fif_status fif_gp_evidence(const fif_gp* gp, double half_fov, const double* train_u,
                           int32_t n_train, const double* lengths, int32_t n_len, double* lml,
                           void* stream);

/* Build a GP field (eq:general_info_pif / eq:general_trace_pif with the GP vp)
 * at every voxel centre from the landmarks in range (same V_t predicate as
 * fif_build).  workspace: NULL or fif_workspace_bytes(grid, n_landmarks, prec)
 * bytes (spatial ordering and batch culling, as fif_build).  field->gp.axes
 * must be set; kinv is not used by the build. */
fif_status fif_gp_build(const double* landmarks, int64_t n_landmarks, fif_gp_field* field,
                        void* workspace, size_t workspace_bytes, void* stream);

/* Batched pose query of a GP field: F = sum_g K_z[g] Cbar_g with the factors
 * interpolated at t (eq:fim_separation), metrics and layouts as fif_query
 * (trace fields: FIF_TRACE only).  field->gp.kinv must hold fif_gp_setup's
 * result for field->gp. */
fif_status fif_gp_query(const fif_gp_field* field, const void* t, const void* q, int64_t m,
                        uint32_t metrics, int32_t interp, double* out, uint8_t* flags,
                        void* stream);

/* The paper's GP factors of the listed voxels: information fields
 * blocks[n][n_s][21] = C_g = sum_i vp_g(u_i) I_i in world coordinates (upper
 * triangle row-major); trace fields blocks[n][n_s].  Needs kinv. */
fif_status fif_gp_export(const fif_gp_field* field, const int64_t* voxel_ids, int64_t n,
                         double* blocks, void* stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching over resident fields.  (Not a step of the paper's
 * method: its planners re-evaluate pose FIMs many times across samples,
 * iterations and sessions, Sec. I and Sec. VII, which is what a resident field
 * serves.)  fif_serve_run serves a list of requests on the calling thread:
 *   - a request is seen at its arrival time (realtime) or at once;
 *   - requests are admitted in arrival order while fewer than max_inflight
 *     are in flight and their buffers fit hbm_budget (FIF_SERVE_PLAN:
 *     m x 24 B, FIF_SERVE_OPT: m x 96 B);
 *   - admitted requests for the same field and kind are packed into one
 *     launch (co_batch; up to max_batch poses and FIF_SERVE_MAX_PACK
 *     requests): one kernel gathers their poses into a stream's batch
 *     buffers, the query or query + gradient kernels run, one kernel scatters
 *     the results to the requests' buffers;
 *   - batches go round-robin over n_streams HIP streams created for the run
 *     (default priority) and destroyed before it returns;
 *   - a request is done when the event recorded after its batch is observed
 *     complete.  admitted and done are written in seconds from the start of
 *     the run; *elapsed is the run's length.
 * Each request's results equal those of fif_query (metrics FIF_TRACE |
 * FIF_LMIN | FIF_LOGDET, trilinear) or fif_query_grad (the same metrics,
 * dL/dout = the request's weights for every pose) on that request alone: a
 * pose's arithmetic does not depend on the other poses of a launch.  The
 * request buffers must be ready on the device before the call and stay
 * allocated until it returns; the call
 * returns after all work has completed.  The run uses the current device
 * (where the fields, requests and workspace must live); the workspace holds
 * the streams' batch buffers for the whole call, so calls that overlap in time
 * need workspaces of their own.
 * Errors: FIF_EINVAL (before anything is enqueued) for invalid fields,
 * requests (field index, kind, m < 1, NULL or misaligned buffers, weights
 * not finite, a request larger than hbm_budget or max_batch) or
 * configuration; FIF_ENOMEM for a workspace smaller than
 * fif_serve_workspace_bytes(cfg); FIF_EDEVICE for a
 * HIP error during the run (the remaining requests keep done = NaN). */
#define FIF_SERVE_PLAN 0
#define FIF_SERVE_OPT 1
#define FIF_SERVE_MAX_PACK 32
#define FIF_SERVE_MAX_STREAMS 16

typedef struct {
  double arrival;  /* host: seconds from the start of the run */
  int32_t field;   /* index into fields[] */
  int32_t kind;    /* FIF_SERVE_PLAN | FIF_SERVE_OPT */
  int64_t m;       /* poses, >= 1 */
  const void* t;   /* device [m][3], float (FP32 fields) or double (FP64) */
  const void* q;   /* device [m][4], (w, x, y, z) */
  double* out;     /* device [m][3]: trace, lambda_min, log-det */
  void* grad_t;    /* device [m][3] (FIF_SERVE_OPT; pose precision) */
  void* grad_phi;  /* device [m][3] (FIF_SERVE_OPT; left so(3)) */
  double weights[3]; /* host (FIF_SERVE_OPT): dL/dout of every pose for trace,
                        lambda_min, log-det; 0 leaves a metric out of L */
  double admitted; /* written by fif_serve_run */
  double done;     /* written by fif_serve_run */
} fif_serve_request;

typedef struct {
  int32_t n_streams;    /* 1 .. FIF_SERVE_MAX_STREAMS */
  int32_t max_inflight; /* requests in flight, >= 1 */
  int64_t hbm_budget;   /* bytes of request buffers in flight, >= 1 */
  int64_t max_batch;    /* poses per launch, 1 .. 2^24 */
  int32_t co_batch;     /* nonzero: pack requests of one field and kind */
  int32_t realtime;     /* nonzero: a request is not seen before its arrival */
} fif_serve_config;

/* Bytes of the device workspace of fif_serve_run (per stream: the batch's
 * poses, outputs, upstream ones and gradients for max_batch poses); 0 for an
 * invalid configuration. */
size_t fif_serve_workspace_bytes(const fif_serve_config* cfg);

fif_status fif_serve_run(const fif_field* fields, int32_t n_fields, fif_serve_request* reqs,
                         int64_t n_req, const fif_serve_config* cfg, void* workspace,
                         size_t workspace_bytes, double* elapsed);

/* Static string for a status code. */
const char* fif_status_string(fif_status status);

/* Thread-local text of the last FIF_EDEVICE / FIF_EINVAL of this thread. */
const char* fif_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIF_H */
