/*
 * pat.h — C ABI of the MI355X (gfx950) photoacoustic forward / adjoint library.
 *
 * The library evaluates, for K initial-pressure datasets that share one sound
 * speed, the forward map of eq. (2) (a k-space pseudospectral solution of the
 * lossless wave problem, eq. (1), sampled at point sensors), the data misfit of
 * eq. (4), the exact gradient of that misfit with respect to every p0_i and c
 * (eqs. (5)-(9), as the gradient of the discrete objective), and the vector
 * pieces of the projected L-BFGS reconstruction (eq. (10), eq. (11), Alg. 1)
 * and of the multigrid continuation (Sec. 3.1, Sec. 4.1.2).
 *
 * Conventions (all entry points):
 *  - Array arguments are DEVICE pointers unless marked "host".  The caller owns
 *    every array; the library never frees caller memory.
 *  - Fields are float32, row-major [ny][nx] (x fastest); K fields are stacked
 *    [K][ny][nx]; sensor traces are [K][nt][m].
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *    default stream) and is asynchronous; results are valid once the stream has
 *    reached that point.  Results are deterministic: the same inputs give the
 *    same bits (no floating-point atomics).
 *  - Every call returns a status: PAT_OK (0) or a negative PAT_E* code; a
 *    failing call enqueues nothing.  pat_status_string() names a code.
 *  - A plan and its internal scratch belong to one stream at a time: calls on
 *    one plan that overlap on different streams race.
 *  - Environment: PAT_NO_GRAPHS (any value) launches every pass directly
 *    instead of replaying captured step graphs (same bits);
 *    PAT_GENERIC_KERNELS (any value, read by pat_plan_create) selects the
 *    any-radix LDS kernels also for power-of-two grids (same results to
 *    float32 rounding); PAT_CHECK_FINITE (any value, read by pat_plan_create)
 *    turns on the check mode of the plan: pat_forward and
 *    pat_adjoint_gradient then scan their outputs, synchronize the stream and
 *    return PAT_ENONFINITE if any value is NaN or infinite (a debugging aid:
 *    the synchronisation makes these calls unusable under graph capture).
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PAT_OK            0
#define PAT_EINVAL       -1  /* null pointer, non-positive or inconsistent size   */
#define PAT_EUNSUPPORTED -2  /* grid length without a compiled FFT plan, K > 64   */
#define PAT_EWORKSPACE   -3  /* workspace too small, or not filled by pat_forward */
#define PAT_EHIP         -4  /* HIP runtime error (launch or allocation)          */
#define PAT_ENONFINITE   -5  /* an output holds NaN or Inf (check mode only)       */

/* One computational grid.  nx, ny include the PML.  The time axis holds nt
 * samples t_n = n*dt, n = 0..nt-1 (nt-1 updates).  c_ref is the fixed speed of
 * the k-space correction kappa = sinc(c_ref |k| dt / 2); rho0 the constant
 * ambient density; pml_alpha the PML absorption at its outer edge in nepers per
 * grid point, profile alpha(d) = pml_alpha * (c_ref/dx) * (d/pml)^4 over the
 * `pml` outermost points of every side.  Pixel i of an axis of length n sits at
 * (i + 1/2 - n/2) * dx. */
typedef struct pat_grid {
  int32_t nx, ny;
  int32_t nt;
  int32_t pml;
  double dx;
  double dt;
  double c_ref;
  double rho0;
  double pml_alpha;
} pat_grid;

typedef struct pat_plan pat_plan;

/* Create a plan for K datasets on grid `g` with m point sensors at physical
 * positions `sensor_xy` (HOST, [m][2] metres, (x, y), origin at the grid
 * centre).  Sec. 2.2: the pressure at a sensor is the bilinear interpolation
 * of its four surrounding pixels; the adjoint injects with the transpose.
 * Pixel i of an axis with n points is centred at (i + 1/2 - n/2) dx; a sensor
 * is inside the interpolation range when its fractional pixel index
 * x / dx + n/2 - 1/2 lies in [0, n - 1) on both axes (the last pixel centre
 * itself is outside: its upper neighbour would be off the grid).
 * Supported axis lengths: 32 36 40 48 64 81 84 96 125 128 160 175 192 243 256
 * 375 384 512 768 (products of 2, 3, 5, 7 with a compiled radix plan).
 * Errors: PAT_EINVAL (sizes, sensor outside the interpolation range),
 * PAT_EUNSUPPORTED (axis length, K > 64), PAT_EHIP (table upload).
 * The plan owns small device tables (twiddles, PML profiles, sensor taps,
 * kappa); release it with pat_plan_destroy. */
int pat_plan_create(const pat_grid* g, int32_t K, int32_t m, const double* sensor_xy,
                    pat_plan** plan);
int pat_plan_destroy(pat_plan* plan);

/* Workspace bytes for pat_forward / pat_adjoint_gradient.  ckpt_every = 0
 * stores the whole pressure history (nt fields of K*ny*nx floats);
 * ckpt_every = s > 0 stores the solver state every s steps and recomputes
 * s-step segments during the adjoint (gradients are bit-identical either way). */
int pat_workspace_size(const pat_plan* plan, int32_t ckpt_every, size_t* bytes);

/* Forward map f of eq. (2) for all K datasets: data[k][n][:] = S p_k^n.
 * c [ny][nx] (> 0), p0 [K][ny][nx], data [K][nt][m].
 * record != 0 keeps what pat_adjoint_gradient needs in `ws` (the pressure
 * history or the checkpoints, per ckpt_every); record == 0 (line-search
 * trials) only needs the state part of the workspace and leaves the recorded
 * part untouched.  ws must hold pat_workspace_size(plan, ckpt_every) bytes. */
int pat_forward(pat_plan* plan, const float* c, const float* p0, float* data,
                void* ws, size_t ws_bytes, int32_t ckpt_every, int32_t record, void* stream);

/* The recorded pressure field p^n (eq. (1) solved as in Sec. 2.1; n = 0 is
 * p0) of all K datasets, [K][ny][nx] float32, inside a workspace that the last
 * recording pat_forward of this plan filled with the whole history
 * (ckpt_every = 0).  *field receives a DEVICE address inside ws (read-only,
 * valid until the next pat_forward on that workspace); no work is enqueued.
 * PAT_EINVAL for n outside [0, nt) or null arguments; PAT_EWORKSPACE if ws
 * holds no store-all recording of this plan. */
int pat_history_field(const pat_plan* plan, const void* ws, int32_t n, const float** field);

/* Data term of eq. (4) with W_i = w[i] (w: DEVICE array of K weights 1/sigma_i):
 * resid = w^2 (data - y) (the adjoint source, eq. (6) with the sign folded
 * in) and J = 1/2 sum w^2 (data - y)^2 accumulated in float64 into the DEVICE
 * scalar *J.  data, y, resid: [K][nt][m]; resid may alias data. */
int pat_misfit(pat_plan* plan, const float* data, const float* y, const float* w,
               float* resid, double* J, void* stream);

/* Exact gradient of J with respect to every p0_k and the shared c (eqs. (5)-(9)
 * for the discrete forward map): the adjoint field is driven backwards in time
 * by `resid` [K][nt][m] (dJ/d data) injected at the sensors.
 * g_p0 [K][ny][nx]; g_c [ny][nx] = sum over the K datasets (eq. (8)).
 * Requires that the last pat_forward on this plan ran with record != 0 on the
 * same ws, c and p0 (else PAT_EWORKSPACE). */
int pat_adjoint_gradient(pat_plan* plan, const float* c, const float* p0, const float* resid,
                         float* g_p0, float* g_c, void* ws, size_t ws_bytes, void* stream);

/* Eq. (10)-(11): x <- P(x - alpha d), P the element-wise clamp to [L, U].
 * Bounds per element (lo, hi DEVICE arrays of n) or, where an array pointer is
 * NULL, the scalar lo_s / hi_s (hi_s = +INFINITY allowed: no upper bound).
 * lo == hi pins an element. */
int pat_project_update(int64_t n, float* x, const float* d, float alpha,
                       const float* lo, const float* hi, float lo_s, float hi_s, void* stream);

/* Eq. (10)-(11): the free part of a vector for a projected step at x with
 * gradient g: out_i = 0 where x_i sits on a bound with g pointing out of the
 * box (x_i <= lo_i and g_i > 0, or x_i >= hi_i and g_i < 0), else v_i.  All
 * arrays DEVICE [n]; out may alias v (not x or g). */
int pat_free_part(int64_t n, const float* x, const float* g, const float* lo, const float* hi, const float* v,
                  float* out, void* stream);

/* Vector updates of the optimiser around Alg. 1 (step differences s = x+ - x,
 * y = g+ - g, scaling): out = a x + b y (y may be NULL: out = a x), and
 * out = x * s element-wise.  DEVICE arrays of n floats; out may alias the
 * inputs. */
int pat_axpby(int64_t n, float a, const float* x, float b, const float* y, float* out, void* stream);
int pat_mul(int64_t n, const float* x, const float* s, float* out, void* stream);

/* Sec. 3.1: bilinear interpolation of nchan coarse fields [nchan][nyc][nxc]
 * onto a finer grid [nchan][nyf][nxf] covering the same physical square
 * (cell-centred pixels), clamped at the border.  Each fine value is a convex
 * combination of at most four coarse values.  Sizes are given x first. */
int pat_prolong(int32_t nchan, const float* coarse, int32_t nxc, int32_t nyc,
                float* fine, int32_t nxf, int32_t nyf, void* stream);

/* Sec. 3.1 for levels of different physical extent (Table 1's grids carry PML
 * layers of different widths): bilinear interpolation of nchan coarse fields
 * [nchan][nyc][nxc] with pixel spacing dxc (metres) onto [nchan][nyf][nxf]
 * with spacing dxf, both grids centred on the origin (pixel i at
 * (i + 1/2 - n/2) * dx), each fine value taken at its own physical position
 * and clamped to the coarse grid.  Equals pat_prolong when nxc * dxc ==
 * nxf * dxf.  PAT_EINVAL for null arrays, non-positive sizes or spacings. */
int pat_prolong_phys(int32_t nchan, const float* coarse, int32_t nxc, int32_t nyc, double dxc,
                     float* fine, int32_t nxf, int32_t nyf, double dxf, void* stream);

/* Sec. 4.1.2: linear interpolation in time of traces y [nlead][nt_src][m]
 * sampled at n*dt_src onto out [nlead][nt_dst][m] at n*dt_dst (held at the
 * last sample beyond the end). */
int pat_time_interp(int32_t nlead, int32_t nt_src, int32_t m, const float* y, double dt_src,
                    float* out, int32_t nt_dst, double dt_dst, void* stream);

/* Alg. 1 (two-loop recursion): d = H g for the L-BFGS inverse Hessian built
 * from `npairs` pairs s_j = x_{j+1} - x_j, y_j = g_{j+1} - g_j given oldest
 * first (s, y: HOST arrays of npairs DEVICE pointers to n floats), with
 * H^0 = (s^T y / y^T y) I of the newest pair.  Dot products accumulate in
 * float64.  npairs = 0 gives d = g.  `scratch`: DEVICE buffer of at least
 * pat_lbfgs_scratch_bytes(npairs) bytes.  d may alias g. */
size_t pat_lbfgs_scratch_bytes(int32_t npairs);
int pat_lbfgs_direction(int64_t n, const float* g, int32_t npairs, const float* const* s,
                        const float* const* y, float* d, void* scratch, void* stream);

/* Alg. 1 as pat_lbfgs_direction, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): no scratch argument and no allocation of any kind; the
 * library keeps the scratch in one static device array per GPU, sized for at
 * most PAT_LBFGS_NOALLOC_MAX_PAIRS pairs (5.1 KB), held until the process
 * ends.  Same arguments, results bit-identical to pat_lbfgs_direction.
 * PAT_EUNSUPPORTED if npairs > PAT_LBFGS_NOALLOC_MAX_PAIRS; PAT_EINVAL as for
 * pat_lbfgs_direction; PAT_EHIP if the array's device address cannot be
 * obtained.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (different streams or host threads) race. */
#define PAT_LBFGS_NOALLOC_MAX_PAIRS 64
int pat_lbfgs_direction_noalloc(int64_t n, const float* g, int32_t npairs, const float* const* s,
                                const float* const* y, float* d, void* stream);

/* Float64 dot product a . b of n floats into the DEVICE scalar *out
 * (deterministic two-level reduction; `scratch` as for pat_lbfgs_direction
 * with npairs = 0). */
int pat_dot(int64_t n, const float* a, const float* b, double* out, void* scratch, void* stream);

/* max_i |x_i| of n floats into the DEVICE double *out (the steepest-descent
 * normalisation of the first step; `scratch` as for pat_dot). */
int pat_absmax(int64_t n, const float* x, double* out, void* scratch, void* stream);

/* Column-pass tile width of a plan (power-of-two grids): 0 = the default for
 * the transform length, 8 = eight adjacent columns per block.  A tuning knob
 * (results are identical); captured step graphs of the plan are discarded
 * when it changes.  PAT_EINVAL for other values. */
int pat_plan_set_tile(pat_plan* plan, int32_t col_tile);

/* Column-pass transform order of a plan (power-of-two grids): 0 = the two
 * transforms a thread holds advance stage by stage together (shared
 * barriers; the default), 1 = one after the other (the first array's loads
 * issued first, so its transform starts while the second array's loads land,
 * and its result is stored while the second is transformed), 2 = the two
 * arrays of a pass on the two halves of a block of twice the threads (one
 * transform per thread, twice the waves per launch; always the default
 * column tile).  A tuning knob (results are identical); captured step graphs
 * of the plan are discarded when it changes.  PAT_EINVAL for other values. */
int pat_plan_set_col_order(pat_plan* plan, int32_t order);

/* One independent problem of a batch: everything a forward + misfit +
 * adjoint evaluation needs (as for pat_forward / pat_misfit /
 * pat_adjoint_gradient with store-all history, ckpt_every = 0). */
typedef struct pat_problem {
  pat_plan* plan;
  const float* c;      /* [ny][nx] */
  const float* p0;     /* [K][ny][nx] */
  const float* y;      /* [K][nt][m] observed traces */
  const float* w;      /* [K] weights 1/sigma_i */
  float* data;         /* [K][nt][m] out: f(p0, c) */
  float* resid;        /* [K][nt][m] out: w^2 (f - y) */
  double* J;           /* device scalar out: eq. (4) data term */
  float* g_p0;         /* [K][ny][nx] out */
  float* g_c;          /* [ny][nx] out */
  void* ws;            /* workspace of pat_workspace_size(plan, 0) bytes */
  size_t ws_bytes;
} pat_problem;

/* Destroy the library's internal batch streams (created by the first
 * pat_batch_gradient and kept for later batches) once the work queued on them
 * has finished.  The next batch creates them again.  Not to be called while
 * a batch is being enqueued from another thread. */
int pat_batch_release(void);

/* Objective and gradient (eqs. (4)-(9)) of `nprob` independent problems of
 * any sizes at once: the problems are spread over `nstreams` (1..16) internal
 * streams (longest first, onto the least-loaded stream) and advanced in
 * interleaved runs of time steps, each replayed from the problem's captured
 * step graphs, so that small problems share the GPU.  Ordered after the work
 * queued on `stream`; `stream` waits for all of it.  Every problem gets
 * exactly the bits that it gets alone.  Each problem needs its own plan and
 * workspace (PAT_EINVAL otherwise). */
int pat_batch_gradient(int32_t nprob, const pat_problem* probs, int32_t nstreams, void* stream);

/* Eq. (4) prior terms with the Ornstein-Uhlenbeck covariance of Sec. 4.1.2:
 * Gamma_z = sigma_z^2 Xi, Xi_ij = exp(-|r_i - r_j| / tau), over the pixels
 * r_i (spacing dx, metres) of the reconstruction domain given by a host mask
 * [ny][nx] (nonzero = in the domain; NULL = the whole grid).  An opaque object
 * holds the operator: products with Xi are exact (FFT convolution on a
 * periodic embedding of the mask's bounding box, L >= 2 * box side - 1 from
 * the supported transform lengths); Xi^{-1} is applied by preconditioned
 * conjugate gradients.  PAT_EUNSUPPORTED when the box needs L > 512;
 * PAT_EINVAL for an empty mask or non-positive sizes.  Vectors are device
 * arrays [nvec][ny][nx]; entries outside the mask are ignored on input and
 * written as zero. */
typedef struct pat_ou pat_ou;
int pat_ou_create(int32_t ny, int32_t nx, double dx, double tau, const uint8_t* mask, pat_ou** out);
int pat_ou_destroy(pat_ou* ou);
/* bytes of caller-owned device scratch for nvec vectors */
int pat_ou_scratch_bytes(const pat_ou* ou, int32_t nvec, size_t* bytes);
/* out = Xi v on the mask (the exact product; for tests and diagnostics) */
int pat_ou_apply(pat_ou* ou, int32_t nvec, const float* v, float* out, void* scratch, size_t scratch_bytes,
                 void* stream);
/* For every vector z_v with mean eta[v] and 1/sigma_v^2 = inv_var[v] (device
 * float arrays [nvec]): grad_v = inv_var[v] Xi^{-1} (z_v - eta[v]) and
 * *J (device double) = sum_v 1/2 inv_var[v] (z_v - eta[v])^T Xi^{-1} (z_v - eta[v]).
 * Conjugate gradients stop when every residual is below tol times its
 * right-hand side (checked every 8 iterations) or after maxit iterations;
 * *iters (host, may be NULL) receives the count.  Synchronizes the stream. */
int pat_ou_prior(pat_ou* ou, int32_t nvec, const float* z, const float* eta, const float* inv_var, float* grad,
                 double* J, double tol, int32_t maxit, void* scratch, size_t scratch_bytes, int32_t* iters,
                 void* stream);

/* Kernel timing (diagnostics).  Kinds of fused pass, in time-step order:
 * forward column GRAD, row U, column DIV, row RHO; adjoint column SUMM, row
 * RHO, column GRAD, row U. */
#define PAT_PASS_FWD_COL_GRAD 0
#define PAT_PASS_FWD_ROW_U    1
#define PAT_PASS_FWD_COL_DIV  2
#define PAT_PASS_FWD_ROW_RHO  3
#define PAT_PASS_ADJ_COL_SUMM 4
#define PAT_PASS_ADJ_ROW_RHO  5
#define PAT_PASS_ADJ_COL_GRAD 6
#define PAT_PASS_ADJ_ROW_U    7
#define PAT_PASS_KINDS        8
/* pat_trace_start(every): from now on every `every`-th launch of each pass
 * kind carries two HIP events as the start and stop events of its own
 * dispatch on the stream it is launched on, so their elapsed time is the
 * kernel's execution (at most 1024 launches per kind; the events are created
 * here, on the current device).  pat_trace_stop() stops recording.  pat_trace_read(kind,
 * &count, &total_ms): once those streams have drained, the number of timed
 * launches of `kind` and their summed duration in milliseconds.  Process-wide
 * state: not for concurrent use from several threads. */
int pat_trace_start(int32_t every);
int pat_trace_stop(void);
int pat_trace_read(int32_t kind, int64_t* count, double* total_ms);

const char* pat_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PAT_H */
