/*
 * cvo.h - C ABI of the MI355X continuous sensor registration library.
 *
 * Method: Ghaffari, Clark, Bloch, Eustice, Grizzle, "Continuous Direct Sparse
 * Visual Odometry from RGB-D Images".  Two labelled point clouds X (source)
 * and Z (target) become functions in a reproducing kernel Hilbert space; the
 * registration maximises their inner product (Section III, Problem 1)
 *
 *     F = sum_ij c_ij k_ij,   c_ij = s_f <l_i, m_j>,
 *     k_ij = sigma^2 exp(-|x_i - z~_j|^2 / (2 ell^2)),   z~_j = T z_j,
 *
 * (eq. scalar; squared-exponential kernel of Section IV; label inner product
 * of the Section VII-B remark, scaled by s_f) by the gradient flow on SE(3):
 *
 *     omega = 1/(a^2 ell^2) sum_ij c_ij k_ij (x_i x z~_j)
 *     v     = 1/(b^2 ell^2) sum_ij c_ij k_ij (z~_j - x_i)          (eq. 3_gradient)
 *
 * integrated with the closed-form exponential map (eq. step, eq. newstep).
 *
 * Conventions
 *   - T is a row-major 4x4 FP64 rigid transform that acts on TARGET points
 *     (z~ = R z + t).  The paper's pose h is T^-1; the update h <- h exp(tau xi)
 *     is applied here as T <- Exp(-tau (omega, v)) T.
 *   - v carries the sign obtained by differentiating the kernel (z~ - x); the
 *     paper prints the opposite sign in eq. 3_gradient while its own
 *     differential and Taylor coefficients imply this one.
 *   - Step length, by params->step_rule:
 *     CVO_STEP_FIXED    tau = eta * ell^2 / F (a project rule);
 *     CVO_STEP_QUARTIC  the paper's rule (Sec. VI-B, eq. fourth): tau is the
 *       t > 0 that maximises the fourth-order Taylor model
 *       P(t) = F + A1 t + A2 t^2 + A3 t^3 + A4 t^4 of G(t) = F(h exp(t xi))
 *       along the gradient xi = (omega, v) (the local maximum with the
 *       largest P when there are two) within the interval where the
 *       expansion describes G: t <= t_max = 3 ell / (|xi_w| rho + |xi_v|),
 *       the step that moves a typical target by three length-scales (rho =
 *       the targets' root mean square norm plus |t| of the pose); when P
 *       has no maximum on (0, t_max] the fixed rule's tau is taken.  A second pass over the same pairs sums
 *       A_k = sigma^2 s_f sum_ij <l_i, m_j> e^alpha_ij g^k_ij with the
 *       exponent's exact Taylor coefficients (alpha .. eps of the moving
 *       target exp(-t Xi) z~; the printed gamma, delta, eps omit the
 *       exponential's factorials and signs) and the paper's g^1..g^4.
 *     CVO_STEP_CONJUGATE  the paper's line search of CVO_STEP_QUARTIC taken
 *       along conjugate directions instead of the gradient itself (a project
 *       rule): d = g + beta d_prev with the Polak-Ribiere
 *       beta = max(0, <g, g - g_prev> / <g_prev, g_prev>), inner products in
 *       the metric a^2 omega.eta + b^2 v.u (Sec. IV-B), g the gradient in the
 *       subgroup dof_mask selects; d restarts from g at the first iteration
 *       of every length-scale stage, every 6 steps and whenever
 *       <g, d> <= 0.  The pose moves by Exp(-tau d); the trace and result
 *       still report the gradient.  The gradient flow's fixed step contracts
 *       the slowest direction of the RGB-D workloads by ~1% per iteration;
 *       conjugate directions reach |tau d| < 1e-5 within a stage.
 *   - With cutoff_mult = kappa > 0 a pair contributes only if
 *     |x_i - z~_j| <= kappa * ell (the paper sparsifies small kernel values,
 *     Section VII-B; here in distance form); kappa = 0 sums all pairs.
 *
 * Ownership and threading
 *   - Host inputs (on_device = 0) are copied before the call returns (or
 *     before cvo_submit returns).
 *   - Device inputs (on_device = 1) must be device pointers on the context's
 *     device.  cvo_eval / cvo_register read them on the context's stream (see
 *     cvo_set_stream), ordered after the work already queued there; they are
 *     borrowed until the call returns.  cvo_submit reads them later on the
 *     scheduler's own stream, with no ordering against any caller stream: the
 *     data must be complete when cvo_submit is called (synchronize the stream
 *     that wrote them first), and stay valid and unmodified until cvo_poll
 *     reports a terminal status for the ticket.
 *   - All outputs go to caller buffers; the context owns all device state.
 *   - cvo_eval / cvo_register serialise on the context.  cvo_submit and
 *     cvo_poll are thread-safe.
 *   - No C++ exception crosses this boundary.
 *
 * Return codes: 0 success, CVO_PENDING (>0) from cvo_poll, negative on error.
 */
#ifndef CVO_H_
#define CVO_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cvo_ctx cvo_ctx;

enum {
  CVO_OK = 0,
  CVO_PENDING = 1,       /* cvo_poll: the request has not finished */
  CVO_EINVAL = -1,       /* bad argument: n <= 0, feat_dim outside [1,8], non-finite input, bad schedule */
  CVO_ENOMEM = -2,       /* one request needs more device memory than the context budget */
  CVO_EBUSY = -3,        /* the submission queue is full */
  CVO_ENOOVERLAP = -4,   /* F <= 1e-300 at some iteration: no pair within reach */
  CVO_EDEVICE = -5,      /* HIP runtime error (see cvo_strerror / cvo_last_error) */
  CVO_ENOTFOUND = -6     /* unknown ticket */
};

enum { CVO_FP32_KAHAN = 0, CVO_FP64 = 1 };
enum { CVO_STEP_FIXED = 0, CVO_STEP_QUARTIC = 1, CVO_STEP_CONJUGATE = 2 };

/* One labelled point cloud (Section III-A: points x_i with labels l(x_i) in R^feat_dim). */
typedef struct {
  int32_t n;           /* number of points, 1 .. 16,000,000 */
  int32_t feat_dim;    /* label channels, 1..8 (both clouds must match) */
  const float* xyz;    /* [n][3] row-major, finite */
  const float* feat;   /* [n][feat_dim] row-major, finite */
  int32_t on_device;   /* 0: host pointers; 1: device pointers on the context's device */
} cvo_cloud;

/* Registration parameters (Section IV kernel; Table 1 lists the paper's values). */
typedef struct {
  double sigma;             /* kernel signal parameter; the prefactor is sigma^2 (> 0) */
  double feat_scale;        /* s_f in c_ij = s_f <l_i, m_j> (> 0) */
  double a2;                /* rotational metric weight a^2; <= 0 selects mean |x_i|^2 of the source
                               (a source whose points all lie at the origin then gives a^2 = 0: EINVAL) */
  double b2;                /* translational metric weight b^2 (> 0) */
  double eta;               /* step rule tau = eta ell^2 / F (> 0) */
  double cutoff_mult;       /* kappa >= 0; 0 = every pair (brute force) */
  int32_t n_stages;         /* length-scale stages, 1..8 */
  const int32_t* stage_iters; /* [n_stages-1] iterations spent in each stage but the last (>= 1) */
  const double* stage_ell;  /* [n_stages] length-scale of each stage (> 0) */
  int32_t max_iters;        /* iteration cap, >= 1 */
  double tol;               /* stop once the last stage is reached and the applied twist
                               |tau d|_2 < tol (d = (omega, v), or the conjugate direction) */
  int32_t precision;        /* CVO_FP32_KAHAN (FP32 pair terms, Kahan FP32 partials, FP64
                               reduction and step) or CVO_FP64 (every pair term in FP64) */
  int32_t trace;            /* 1: keep the per-iteration trace (cvo_trace) */
  int32_t step_rule;        /* CVO_STEP_FIXED, CVO_STEP_QUARTIC or CVO_STEP_CONJUGATE (see the step
                               length above) */
  double grad_tol;          /* also stop once the last stage is reached and |(omega, v)|_2 < grad_tol
                               (Table 1's gradient-norm threshold; 0: off) */
  double kernel_floor;      /* > 0: sparsify by kernel value as in the TUM experiment (Table 1):
                               pairs with sigma^2 exp(-r^2/(2 ell^2)) < kernel_floor are dropped,
                               i.e. the cutoff r <= ell sqrt(2 ln(sigma^2 / kernel_floor)); needs
                               cutoff_mult = 0 and sigma^2 > kernel_floor.  0: cutoff_mult applies */
  int32_t dof_mask;         /* the subgroup of SE(3) the registration runs on: bit q set = the flow moves
                               along generator q (bits 0-2: rotation about x, y, z; 3-5: translation
                               along x, y, z); the step uses the gradient's components in the mask
                               (its orthogonal projection under the metric a^2, b^2).  0 or 0x3F: SE(3);
                               0x1C: planar motion SE(2) (rotation about z, translation in x, y);
                               0x07: SO(3); 0x38: translations.  The trace and result report the full
                               gradient. */
  double stage_tol;         /* > 0: a length-scale stage also ends as soon as its applied twist
                               |tau d|_2 < stage_tol (the stage's own convergence; stage_iters then
                               bounds each stage); 0: stages last stage_iters iterations */
  int32_t work_item_min;    /* work items: a target cluster's candidate sources are cut into items of at
                               least this many sources (8 .. 2^20); 0: the context's tuning table */
  int32_t work_items_max;   /* ... and at most this many items per cluster (1 .. 256); 0: the table.
                               The sizing changes only how the pair terms are grouped into compensated
                               FP32 partials and FP64 sums (results agree to that rounding); it depends
                               on the request alone, so a request gives the same result alone and in a
                               batch. */
} cvo_params;

/* One organised RGB-D frame (the input of the front end, Sec. VII-B). */
typedef struct {
  int32_t width, height;    /* pixels, 1..16384 each, width * height <= 16,777,216 */
  const float* depth;       /* [height][width] depth along the optical axis (m); a pixel whose depth is
                               not finite or outside [dmin, dmax] gives no point */
  const float* rgb;         /* [height][width][3] colour, finite (EINVAL otherwise) */
  double fx, fy, cx, cy;    /* pinhole intrinsics in pixels (fx, fy > 0) */
  double dmin, dmax;        /* valid depth range (m), dmin <= dmax */
  int32_t on_device;        /* 1: depth, rgb and the outputs are device pointers on the context's device */
} cvo_rgbd_frame;

typedef struct {
  int32_t status;           /* 0 or a negative code */
  int32_t iters;            /* iterations performed */
  int32_t converged;        /* 1 if the tolerance test stopped the flow */
  int32_t reserved;
  double F, omega[3], v[3]; /* at the last evaluated pose */
  double gpu_ms;            /* device time of the request (event-timed, register path) */
  double wall_ms;           /* host time from call (or submission) to completion */
  uint64_t pairs_within;    /* pairs inside the cutoff, summed over iterations */
  uint64_t pairs_examined;  /* candidate pairs tested, summed over iterations */
  uint64_t device_bytes;    /* device memory the request held (set-up and iteration buffers) */
} cvo_result;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory of concurrently admitted requests (0: 80% of free memory); max_slots
 * bounds concurrently active requests of the batched path (1..4096). */
int cvo_create(int device, uint64_t hbm_budget_bytes, int max_slots, cvo_ctx** out);

/* Wait for outstanding requests, free every device buffer, destroy the context. */
int cvo_destroy(cvo_ctx* ctx);

/* Run subsequent eval/register work on this hipStream_t (e.g. torch's current
 * stream).  NULL selects the context's own stream. */
int cvo_set_stream(cvo_ctx* ctx, void* hip_stream);

/* One evaluation of F, omega, v at pose T (Section VI-C, eq. 3_gradient) with
 * ell = params->stage_ell[0]; no step is taken. */
int cvo_eval(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
             const double T[16], double* F, double omega[3], double v[3]);

/* cvo_eval for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation and kernels, with every device buffer taken from a 64 MiB array
 * that the library holds per device for the life of the process (no
 * hipMalloc, hipFree or pinned host allocation during the call; the context
 * must exist beforehand).  Limits: at most 65,536 points per cloud, and the
 * request's set-up and per-cluster buffers must fit the array (spatially
 * coherent 30k-point clouds need about 25 MiB); otherwise CVO_ENOMEM with the
 * reason in cvo_last_error.  Calls on one device share the array: the library
 * serialises them within the process (calls that overlap on one GPU would
 * race), and each call overwrites what the previous one left.  Inputs and
 * outputs as for cvo_eval. */
int cvo_eval_static(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
                    const double T[16], double* F, double omega[3], double v[3]);

/* The fourth-order model of the line G(t) = F(h exp(t xi)) at pose T along
 * xi = (omega, v) (Sec. VI-B, eq. fourth; h = T^-1), ell = params->stage_ell[0]:
 * coef = F, A1, A2, A3, A4 with G(t) = coef . (1, t, t^2, t^3, t^4) + O(t^5),
 * over the pairs inside the cutoff at t = 0.  Along the gradient
 * A1 = a^2 |omega|^2 + b^2 |v|^2.  omega and v must be finite. */
int cvo_quartic(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
                const double T[16], const double omega[3], const double v[3], double coef[5]);

/* RGB-D front end (Sec. VII-B: the semi-dense cloud of high-gradient pixels
 * taken from the organised depth image, one point per pixel, the pixel's
 * colour as label).  Every step that decides the selection is FP32 in this
 * order, without fused multiply-adds:
 *   I = ((r + g) + b) / 3;  gu = (I[v][u+1] - I[v][u-1]) / 2 (one-sided
 *   differences at the border: I[v][1] - I[v][0], I[v][W-1] - I[v][W-2]),
 *   gv likewise along rows;  s = gu*gu + gv*gv;
 * the k valid pixels of largest s are kept (ties to the smaller pixel index
 * p = v * width + u; all valid pixels when there are at most k), in increasing
 * pixel order.  Point p: (rx d, ry d, d) with rx = (float)((u - cx) / fx),
 * ry = (float)((v - cy) / fy) (FP64 ray, one rounding, one FP32 product);
 * label: (r, g, b, 0.5 + 0.5 tanh(gu / 0.05), 0.5 + 0.5 tanh(gv / 0.05)).
 * xyz [k][3] and feat [k][5] receive the first *n_out rows (caller buffers,
 * on the device when frame->on_device).  Synchronous. */
int cvo_frontend(cvo_ctx* ctx, const cvo_rgbd_frame* frame, int32_t k, float* xyz, float* feat, int32_t* n_out);

/* The step of CVO_STEP_QUARTIC for given coefficients (host code, the same
 * rule the step kernel applies): returns 1 and *t = the maximiser over t > 0
 * of A1 t + A2 t^2 + A3 t^3 + A4 t^4 (coef[1..4]), 0 when it has no local
 * maximum on t > 0, CVO_EINVAL for null or non-finite input. */
int cvo_quartic_step(const double coef[5], double* t);
/* The same with the trusted interval (0, tmax] of the step kernel: only
 * local maxima at t <= tmax count (tmax > 0, may be +inf). */
int cvo_quartic_step_bounded(const double coef[5], double tmax, double* t);

/* Per-target terms of the same double sum: for each selected original target
 * index sel[k] (0 <= sel[k] < tgt->n), out[7k..7k+6] = (F_j, omega_j, v_j),
 * the sums over sources i of the terms of eq. scalar and eq. 3_gradient.
 * nsel = 0 with sel = NULL returns all targets in original order. */
int cvo_eval_targets(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
                     const double T[16], int32_t nsel, const int32_t* sel, double* out);

/* Full registration: from T0, iterate the gradient flow (Section VI) through
 * the length-scale stages until max_iters or the tolerance; T_out receives the
 * final pose, res the summary.  Synchronous. */
int cvo_register(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
                 const double T0[16], double T_out[16], cvo_result* res);

/* Asynchronous registration through the continuous-batching scheduler:
 * requests are admitted while device memory and slots allow and run together,
 * one launch per iteration for all active requests.  Returns a ticket. */
int cvo_submit(cvo_ctx* ctx, const cvo_cloud* src, const cvo_cloud* tgt, const cvo_params* params,
               const double T0[16], uint64_t* ticket);

/* Wait up to wait_us microseconds (0: do not wait, <0: wait forever) for the
 * ticket.  Returns CVO_PENDING if unfinished; otherwise the request's status,
 * with T_out and res filled, and the ticket is released. */
int cvo_poll(cvo_ctx* ctx, uint64_t ticket, int32_t wait_us, double T_out[16], cvo_result* res);

/* Serving counters of the batched path (cvo_submit / cvo_poll). */
typedef struct {
  int64_t pending;          /* submitted, not yet admitted */
  int64_t active;           /* admitted and iterating */
  int64_t completed;        /* finished since cvo_create (any status) */
  int64_t failed;           /* of those, finished with a negative status */
  uint64_t hbm_in_use;      /* device bytes held by admitted requests */
  uint64_t hbm_budget;      /* the admission budget (bytes) */
  uint64_t hbm_peak;        /* the largest hbm_in_use since cvo_create */
  int64_t graph_chunks;     /* scheduler chunks replayed from a captured graph (cvo_set_graphs) */
} cvo_serving_counters;
int cvo_serving_stats(cvo_ctx* ctx, cvo_serving_counters* out);

/* Bound the submission queue (requests submitted and not yet admitted):
 * cvo_submit returns CVO_EBUSY while max_pending requests wait.  Default
 * 65536; 0 refuses every submission.  Admission itself is bounded by the
 * context's slots and its device-memory budget: a request is charged its set-up
 * buffers exactly and its iteration buffers by estimate until its ingest has
 * counted its target clusters, then exactly; one that no longer fits beside
 * the running requests returns to the head of the queue. */
int cvo_set_queue_limit(cvo_ctx* ctx, int64_t max_pending);

/* Copy a per-iteration trace into buf[iters][26]: F, omega[3], v[3], tau,
 * ell, pairs within the cutoff, then the pose T (row-major 4x4) after that
 * iteration's step (with params->trace = 1).  ticket 0: the last cvo_register
 * call.  A batched ticket: its trace once the request has finished, before
 * and after cvo_poll (the traces of the 1024 most recently polled tickets are
 * kept); CVO_PENDING while it runs.  Returns the number of rows written
 * (<= cap), CVO_PENDING, or a negative code (CVO_ENOTFOUND: unknown ticket,
 * or a ticket polled long ago). */
int cvo_trace(cvo_ctx* ctx, uint64_t ticket, double* buf, int32_t cap);

/* Launch mode of the iteration loops: 0 (default) launches each iteration's
 * kernels on the stream; 1 captures a chunk of iterations as a HIP graph once
 * per launch layout and replays it per chunk (the kernels read the requests'
 * state on the device and return at once after a request has stopped).
 * cvo_register's chunk is the whole registration, or 16 iterations when a
 * stopping tolerance is set; it needs a stream other than the legacy null
 * stream, and with profiling on, or on the null stream, iterations are
 * launched directly.  The batched scheduler's chunk is its 8 iterations for
 * all active requests, captured again whenever the set of active requests
 * (and so the launches' grids and arguments) changes.  Results are the same
 * in either mode, bit for bit. */
int cvo_set_graphs(cvo_ctx* ctx, int32_t enable);

/* Event timing of the kernels of each iteration (the per-cluster
 * candidate-list kernel, the pair kernel and, with the quartic rule, the pair
 * kernel's second pass): when enabled, every iteration of cvo_register
 * brackets them with HIP events on the launch stream. */
int cvo_set_profiling(cvo_ctx* ctx, int32_t enable);
/* Totals since the last reset: iterations timed, summed device milliseconds of
 * the pair kernel (gradient pass), of the candidate-list kernel and of the
 * quartic pass, and the pairs within the cutoff evaluated (gradient pass). */
int cvo_kernel_stats(cvo_ctx* ctx, int32_t reset, int64_t* iterations, double* pair_ms, double* prepare_ms,
                     double* quartic_ms, uint64_t* pairs);

/* The work-item sizing the context gives a request of n sources, m targets,
 * with (cutoff = 1) or without a cutoff when its parameters leave it at 0:
 * the first class of the tuning table that matches, else 256 sources per item
 * and 64 items per cluster.  The table is read by cvo_create from the file
 * named by the CVO_TUNING_FILE environment variable, else from tuning.json
 * one directory above the library file: {"classes": [{"cutoff": 0|1,
 * "max_points": N, "work_item_min": N, "work_items_max": N}, ...]} (classes
 * in order; a request matches the first of its kind with max(n, m) <=
 * max_points).  *table_classes receives the classes loaded (0: none). */
int cvo_tuning(cvo_ctx* ctx, int32_t n, int32_t m, int32_t cutoff, int32_t* work_item_min, int32_t* work_items_max,
               int32_t* table_classes);

/* Static text for a return code; cvo_last_error gives the last HIP message. */
const char* cvo_strerror(int code);
const char* cvo_last_error(cvo_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CVO_H_ */
