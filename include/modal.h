/*
 * modal.h -- C ABI of the MI355X modal time-stepping library (libmodal.so).
 *
 * The library steps batches of independent modal systems, one audio sample
 * per step, each mode a damped oscillator driven by an external force and a
 * nonlinear modal force (paper: Sec. 3.2, modal oscillator equation
 *   q'' + 2 gamma q' + omega^2 q = f_ext - f_nl ).
 * Nonlinear forces (paper: Sec. 3.1):
 *   MODAL_KIND_TENSION  tension-modulated string / membrane (modal
 *                       string-membrane equation with normalised modes):
 *                       f_k = kappa lambda_k q_k sum_j lambda_j q_j^2
 *   MODAL_KIND_VK       von Karman plate (nonlinear plate equation with the
 *                       scaled coupling tensor Ht[n][k][j], symmetric in k, j):
 *                       eta_n = sum_kj Ht[n][k][j] q_k q_j,
 *                       f_k   = sum_{n,j} Ht[n][k][j] q_j eta_n
 *   MODAL_KIND_LINEAR   f_nl = 0.
 * Schemes (paper: Sec. 3.2): Stormer-Verlet (modal oscillator update) and the
 * impulse-invariant transfer-function recursion (df update), both written as
 *   q^{n+1} = g q^n + p q^{n-1} + r (f_ext^n - f_nl^n).
 *
 * Conventions for every entry point:
 *  - Return value: MODAL_OK (0) or a negative modal_status.  Nothing throws
 *    across the ABI.  modal_last_error() gives a message for the last failure
 *    of the calling thread.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory of the current device.  Streams are hipStream_t passed as void*
 *    (NULL = the default stream).
 *  - modal_init deep-copies every input; the caller may free its arrays as
 *    soon as it returns.  A context owns all device memory it allocates and
 *    frees it in modal_destroy.  A context is not thread safe: use one
 *    context per stream.
 */
#ifndef MODAL_H
#define MODAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct modal_ctx modal_ctx;

typedef enum {
  MODAL_OK = 0,
  MODAL_EINVAL = -1,     /* invalid argument or inconsistent sizes            */
  MODAL_EUNSTABLE = -2,  /* a mode's recursion has a root outside |z| <= 1    */
  MODAL_ENOMEM = -3,     /* device or host allocation failed                  */
  MODAL_EHIP = -4,       /* a HIP runtime call failed                         */
  MODAL_ENONFINITE = -5, /* a state became Inf/NaN during the run (sticky
                            until modal_reset)                                */
  MODAL_ESTATE = -6,     /* call not valid in the context's current state     */
  MODAL_EHANG = -7       /* a per-instance step barrier timed out; the run
                            was abandoned and the state is undefined          */
} modal_status;

enum { MODAL_KIND_LINEAR = 0, MODAL_KIND_TENSION = 1, MODAL_KIND_VK = 2 };
enum { MODAL_SCHEME_SV = 0, MODAL_SCHEME_TF = 1 };

/* modal_desc.flags */
enum {
  MODAL_FLAG_ASYNC = 1, /* modal_run does not wait for completion nor read
                           the status flags; call modal_check afterwards     */
  MODAL_FLAG_GRAPH = 2, /* modal_run records its launches into a hipGraph
                           on first use for a given (n_steps, y, y_stride)
                           and replays it afterwards                          */
  MODAL_FLAG_GRAD = 4,  /* plan the work so that modal_grad can run (its
                           reverse kernel needs more LDS per workgroup)       */
  MODAL_FLAG_SPLIT_ANY = 8, /* cut VK instances into row slabs whenever
                           workgroups are free (tests, tuning); by default
                           instances below 4 MB of tensor stay whole and a
                           slab must pay for its per-step exchange          */
  MODAL_FLAG_NO_SHARED = 16, /* never use the shared-tensor (MFMA) path     */
  MODAL_FLAG_NO_BLOCK = 32, /* ignore mode_class: store every tensor dense  */
  MODAL_FLAG_RECURSE = 64   /* step linear batches through the recursion too */
};

/* One modal system.  All arrays are host memory. */
typedef struct {
  int32_t kind;          /* MODAL_KIND_*                                      */
  int32_t n_t;           /* number of time-stepped modes, 1..1024             */
  int32_t n_in;          /* VK: number of in-plane modes (>= 1); else 0       */
  int32_t reserved;      /* must be 0                                         */
  const double *omega;   /* [n_t] angular frequencies omega_k (rad/s)         */
  const double *gamma;   /* [n_t] decay rates gamma_k >= 0 (1/s)              */
  const double *lambda;  /* TENSION: [n_t] Laplacian eigenvalues; else NULL   */
  double kappa;          /* TENSION: tau / rho_s; else ignored                */
  const float *H;        /* VK: [n_in][n_t][n_t] scaled coupling tensor Ht,
                            row-major, symmetric in the last two indices to
                            1e-6 of its largest entry; host or device memory */
  const double *x0;      /* [n_t] initial state q^0                           */
  const double *xm1;     /* [n_t] initial state q^-1                          */
  const double *b_ext;   /* [n_t] modal force weights, or NULL (no forcing)   */
  const float *e_ext;    /* [n_exc] force signal: f_ext^n = b_ext e_ext[n]
                            for n < n_exc (absolute step index), else 0       */
  int64_t n_exc;
  const double *c_out;   /* [n_t] output weights: y^n = sum_k c_k q_k^n       */
  const double *h_row_scale; /* VK, optional [n_in]: the instance's tensor is
                            h_row_scale[n] * H[n][k][j] (NULL = 1).  Instances
                            that pass the same H pointer (and n_t, n_in) share
                            one tensor up to these scales; see modal_init.   */
  const uint8_t *mode_class; /* VK, optional [n_t] values 0..3: a partition of
                            the modes (e.g. the parities of a plate mode's
                            two indices).  When H is host memory and, for
                            every in-plane row n and class i, the entries
                            H[n][k][j] with class(k) = i vanish exactly
                            outside a single class of j, the tensor is stored
                            as one dense block per (n, i) and only those
                            blocks are streamed (about a quarter of the bytes
                            for plate parity classes).  Otherwise, and with
                            MODAL_FLAG_GRAD or MODAL_FLAG_NO_BLOCK, ignored.  */
} modal_instance;

typedef struct {
  int32_t batch;                /* number of instances, >= 1                  */
  int32_t scheme;               /* MODAL_SCHEME_*                             */
  const modal_instance *inst;   /* [batch]                                    */
  double fs;                    /* sampling rate (Hz), T = 1/fs               */
  int32_t flags;                /* MODAL_FLAG_*                               */
  int32_t max_workgroups;       /* 0 = default (at most 6 workgroups per CU,
                                   and never more than fit co-resident); else
                                   an upper bound, capped by co-residency     */
  int32_t chunk_steps;          /* steps per kernel launch; 0 = whole run     */
  int32_t waves;                /* waves (64 lanes) per workgroup sharing a
                                   work unit's rows: 1, 4 or 8, or 0 = default
                                   (8 for a batch of at most one instance per
                                   CU whose tensors are all small, when its
                                   reduction space fits the LDS; else 4).
                                   The reverse kernel takes fewer waves when
                                   its larger reduction space does not fit.  */
  int32_t barrier_us;           /* limit of each wait for the other slabs of
                                   a split instance, in microseconds (0 =
                                   4 s); past it the run is abandoned, every
                                   workgroup leaves, and modal_run or
                                   modal_grad returns MODAL_EHANG           */
  const char *tune_cache;       /* optional path of a JSON file written by
                                   the autotuner (paper_2505_05940_amd/
                                   tune.py): {"<key>": {"waves": W,
                                   "max_workgroups": M, ...}, ...}.  With
                                   waves and max_workgroups 0, a batch whose
                                   key (modal_tune_key) is listed takes that
                                   launch shape; a missing file or key
                                   leaves the defaults.  NULL = none.  An
                                   entry's optional "split_cost_kb" applies
                                   when split_cost_kb below is 0.           */
  int32_t split_cost_kb;        /* the per-step cost the planner charges each
                                   slab of a split instance for its exchange,
                                   in KiB of streamed tensor (0 = default, 32;
                                   at most 2^20).  It shifts which instances
                                   are cut and how units are packed; the
                                   autotuner searches it.                    */
} modal_desc;

/* Validates the description (before any device work), computes the per-mode
 * recursion coefficients in FP64 (paper: Sec. 3.2, the Stormer-Verlet and
 * transfer-function updates of each modal oscillator) and stores them as
 * float-float pairs,
 * partitions the batch into per-workgroup work, allocates device memory and
 * uploads the coupling tensors and initial states on `stream`.
 * Shared-tensor path: when every instance is VK with n_t <= 64 and
 * n_in <= 64, the
 * instances pass at most batch/16 distinct H pointers (so the tensors are
 * shared by 16 instances on average) and neither MODAL_FLAG_GRAD nor
 * MODAL_FLAG_NO_SHARED is set, each distinct tensor is stored once and the
 * force is evaluated as a dense FP32 matrix product over the instances that
 * share it (MFMA); otherwise every instance streams its own (scaled) copy.
 * Both paths compute the same recursion; they differ only in the FP32
 * rounding inside the force (order of sums, where the row scale is applied).
 * Linear path: when every instance is MODAL_KIND_LINEAR (and neither
 * MODAL_FLAG_GRAD nor MODAL_FLAG_RECURSE is set), each mode's recursion is
 * solved in closed form from the roots of its characteristic polynomial
 * (FP64 on the host) and modal_run evaluates the outputs of all requested
 * steps in parallel in float-float arithmetic (free response plus the
 * excitation convolved with the impulse response); MODAL_FLAG_GRAPH has no
 * effect there.  A mode with a double root keeps the batch on the recursion.
 * On-chip path (paper: Sec. 4.2, the single small plate stepped in real
 * time): a latency-bound batch (below) without MODAL_FLAG_GRAD whose
 * instances all have n_t <= 64 and whose widest tensor fits one workgroup's
 * registers (ceil(n_in / 8) rows per wave times the column width, n_t
 * rounded up to 16, 32, 40, 48 or 64, at most 200: 40/40 and 64/24 fit)
 * steps each instance in one workgroup of 8 waves that loads its tensor
 * into registers at the start of each launch; no memory traffic between
 * workgroups, two workgroup barriers per step.  A batch with no tensor at
 * all (MODAL_KIND_TENSION and MODAL_KIND_LINEAR instances of n_t <= 256)
 * steps each instance in one wave instead, ceil(n_t / 64) modes per lane,
 * with no barrier.
 * Streaming path plans: a latency-bound batch (at most one instance per CU,
 * dense tensors under 64 MB per step, waves and max_workgroups 0, no
 * MODAL_FLAG_SPLIT_ANY) keeps its tensors dense, takes 8 waves per
 * workgroup and, in batches of at most 16 instances, cuts each instance
 * into slabs of about 8 in-plane rows, one per workgroup.  Any other batch
 * is packed onto the co-resident workgroups by streamed bytes, with
 * tensors whose mode_class hint holds stored parity-blocked (forward
 * only).
 * Errors: EINVAL (NULL/size/kind/finite/symmetry), EUNSTABLE (a mode's
 * characteristic roots outside the unit circle; also gamma <= 0 or, for TF,
 * omega <= gamma), ENOMEM, EHIP.  On error *out is NULL. */
int modal_init(modal_ctx **out, const modal_desc *d, void *stream);

/* Advances every instance by n_steps samples from its current state (paper:
 * Sec. 3.2, one update per sample with the nonlinear modal force of Sec. 3.1
 * evaluated at q^n) and writes y[b * y_stride + i] = output of instance b at
 * step (current + i), the modal-to-physical transform at the pickup
 * (Sec. 4.1),
 * i < n_steps.  y is device memory of at least batch * y_stride floats,
 * y_stride >= n_steps.  Launches on `stream`.  Unless MODAL_FLAG_ASYNC, waits
 * for completion and returns ENONFINITE / EHANG if raised.  Steps already
 * taken persist: two calls of a and b steps equal one call of a + b. */
int modal_run(modal_ctx *c, int64_t n_steps, float *y, int64_t y_stride,
              void *stream);

/* modal_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launches and results as modal_run (bit for bit), with the arrival
 * words and partial forces of split instances taken from a scratch
 * array of 16 MiB that the library holds on each GPU until the process ends
 * (its address resolved once per device by modal_init), and no hipMalloc,
 * hipFree, graph creation or checkpoint recording.  A small kernel first sets
 * the scratch arrival words to this context's step count, so calls of different
 * contexts may follow each other in any order; calls that overlap on one GPU
 * (two streams at once) race on the scratch and must not be issued.
 * y, y_stride and the return values as modal_run; the launches go straight
 * to `stream` (MODAL_FLAG_GRAPH is not used here; a caller may capture them
 * itself, with MODAL_FLAG_ASYNC so that no status read-back is made).
 * Errors: EINVAL when the batch's arrival words (4 bytes per slab, rounded
 * up to 256) and partial forces (4 bytes per float of 2 x slabs x padded
 * modes per split instance) need more than the 16 MiB; ESTATE on the linear
 * closed-form and shared-tensor paths, or when the current device is not the
 * context's. */
int modal_run_noalloc(modal_ctx *c, int64_t n_steps, float *y, int64_t y_stride,
                      void *stream);

/* Waits for `stream` and reports ENONFINITE / EHANG raised since init/reset. */
int modal_check(modal_ctx *c, void *stream);

/* Restores q^0, q^-1 (the initial conditions of Sec. 3.2's two-step
 * recursion) and the step counter to their values at init. */
int modal_reset(modal_ctx *c, void *stream);

/* Copies the current state of every instance (the modal displacements of
 * Sec. 3.2's recursion, recombined from their float-float pairs) to host
 * FP64 arrays laid out as the concatenation of the instances' modes:
 * x = q^n, xm1 = q^{n-1}
 * (each [sum n_t]).  Waits for `stream`. */
int modal_get_state(modal_ctx *c, double *x, double *xm1, void *stream);

/* Partition and sizes, for tests and measurement:
 * info[0] workgroups launched, [1] work units, [2] split instances,
 * [3] coupling bytes read per step (sum over VK instances of
 * 4 n_in n_t n_t), [4] bytes of the padded device layout streamed per step,
 * [5] steps taken so far, [6] dynamic LDS bytes per workgroup,
 * [7] co-resident workgroups per CU used for the plan, [8] planned cost of
 * the most loaded workgroup and [9] the mean planned cost per co-resident
 * workgroup (both in streamed-byte units), [10] the path: 0 persistent
 * recursion, 1 shared tensor (then [1] is the number of instance columns
 * and [2], [8], [9] are 0), 2 linear closed form, 3 on-chip recursion
 * (one workgroup of 8 waves, or of one wave without tensors, per instance,
 * [6] 0),
 * [11] FP32 operations of the force per step (sum over VK instances of
 * 2 n_in n_t^2 + 4 n_in n_t), [12] instances stored parity-blocked,
 * [13] dense-equivalent tensor bytes per step (sum of 4 n_in n_t^2),
 * [14] floats per LDS-resident array when every workgroup owns one unit and
 * keeps its state and coefficients in LDS for a whole launch (latency-bound
 * plans), else 0.
 * [3] counts the entries of the stored representation: for a blocked
 * instance, 4 bytes per entry of its stored blocks without padding. */
int modal_info(const modal_ctx *c, int64_t info[15]);

void modal_destroy(modal_ctx *c);

/* Tangent tensor of instance `inst` (VK only): Hd = dHt/dtheta for one
 * scalar parameter theta, [n_in][n_t][n_t] like H, host or device memory,
 * copied.  modal_grad then also returns dL/dtheta through the tensor. */
int modal_set_tangent(modal_ctx *c, int32_t inst, const float *Hd, void *stream);

/* Reverse-mode gradient of a loss L(y) over the first n_steps outputs of
 * every instance, run from the initial state (paper: Sec. 4.3, fitting by
 * propagating gradients through the time integrator).  dL_dy is device
 * memory [batch][y_stride] (FP32).  The forward pass is recomputed from
 * float-float checkpoints taken every ckpt_every steps (0 = 512); each
 * segment is re-run, recorded, and swept backwards by the adjoint kernel.
 * Outputs (host, FP64, modes concatenated over instances; NULL to skip):
 *   g_omega, g_gamma  dL/d omega_k, dL/d gamma_k (through the scheme's
 *                     coefficients, differentiated exactly on the host)
 *   g_c               dL/d c_k
 *   g_x0, g_xm1       dL/d q^0_k, dL/d q^-1_k
 *   g_scale [batch]   dL/d log s for a factor s on the nonlinear force
 *   g_theta [batch]   dL/d theta through the tangent tensor (0 without one)
 *   g_row             dL/d log s_n for a factor s_n on row n of the scaled
 *                     tensor, per in-plane row of every VK instance in batch
 *                     order ([sum of n_in over VK instances])
 *   g_H [batch]       host array of device pointers, one per instance (NULL
 *                     entries to skip; non-NULL only for VK instances): the
 *                     gradient with respect to every entry of the tensor the
 *                     dynamics uses (the scaled tensor, row scales included),
 *                     each entry an independent parameter (paper: Sec. 4.3,
 *                     fitting the coupling coefficients H):
 *                       g_H[b][n][i][j] = -sum over steps of
 *                                         ((V_n . u) q_i + eta_n u_i) q_j,
 *                     FP32 device memory [n_in][n_t][n_t], overwritten (the
 *                     caller owns it).  Per checkpoint segment, one product
 *                     over the segment's steps per in-plane row.
 * A context created with MODAL_FLAG_GRAD (and without MODAL_FLAG_GRAPH)
 * records these checkpoints, every 512 steps, while modal_run steps it
 * forward from step 0; with ckpt_every 0 or 512, modal_grad then reuses them
 * for the first n_steps if they cover them, and skips its own forward pass
 * (same result, bit for bit).  While it fits 2 GB, such a run also records
 * the whole trajectory, and modal_grad then skips the segment recomputes
 * too.  modal_set_tensor voids both.
 * Needs a context created with MODAL_FLAG_GRAD (else ESTATE).  Leaves the
 * context reset to its initial state.  Errors: EINVAL, ENOMEM, EHIP,
 * ENONFINITE, EHANG. */
int modal_grad(modal_ctx *c, int64_t n_steps, const float *dL_dy, int64_t y_stride,
               int32_t ckpt_every, double *g_omega, double *g_gamma, double *g_c,
               double *g_x0, double *g_xm1, double *g_scale, double *g_theta,
               double *g_row, float *const *g_H, void *stream);

/* Replaces the coupling tensor of VK instance `inst` by H ([n_in][n_t][n_t],
 * FP32, host or device memory, copied): the tensor the dynamics uses, row
 * scales given at init not applied again (paper: Sec. 4.3, fitting the
 * coupling coefficients H, where the tensor itself is the parameter).  H must
 * be exactly symmetric in its last two indices, as the coupling coefficients
 * are (checked; the kernels contract rows by that symmetry); a fit keeps it
 * so by stepping with the symmetric part of g_H.  The state is left as it
 * is.  ESTATE on the shared-tensor and linear paths and for parity-blocked
 * instances (MODAL_FLAG_GRAD keeps tensors dense); EINVAL for a bad index or
 * an asymmetric tensor (the stored tensor is then unchanged). */
int modal_set_tensor(modal_ctx *c, int32_t inst, const float *H, void *stream);

/* Transfer-function response of linear modal systems (paper: Sec. 3.2,
 * impulse-invariant transfer function; Sec. 4.3, linear string fits on a
 * Bark-sampled magnitude response, with a second numerator coefficient and
 * free output weights per mode):
 *   H[b][k] = sum over modes mu of instance b of
 *             w_mu (b1_mu z + b2_mu) / (z^2 + a1_mu z + a2_mu),  z = e^{i omega[k]}.
 * All pointers are host memory, FP64: coef [modes][5] = (a1, a2, b1, b2, w),
 * modes of instance b at [mode_off[b], mode_off[b+1]) (int32 [batch + 1],
 * non-decreasing); omega [n_freq] in radians per sample; H [batch][n_freq][2]
 * (real, imaginary) written.  The device evaluates the sums in float-float
 * arithmetic (FP32 pairs, about 48 bits) from the split inputs, and the host
 * adds the pairs back into FP64; near a lightly damped pole the relative
 * error grows like 2^-48 / (gamma T).  Synchronous on `stream` (device
 * buffers are allocated and freed within the call).  EINVAL for NULL
 * pointers, batch outside [1, 65535], n_freq < 1 or a decreasing mode_off. */
int modal_tf_response(const double *coef, const int32_t *mode_off, int32_t batch,
                      const double *omega, int32_t n_freq, double *H, void *stream);

/* Gradient of L = sum_{b,k} Re(conj(g[b][k]) H[b][k]) with g = dL_dH
 * [batch][n_freq][2] (dL/dRe H, dL/dIm H), host memory, with respect to
 * every mode's (a1, a2, b1, b2, w): g_coef [modes][5] (host, written; modes
 * outside every instance's range are left as they are).  max_modes: at
 * least the largest mode count of an instance.  Same layout, arithmetic and
 * errors as modal_tf_response. */
int modal_tf_grad(const double *coef, const int32_t *mode_off, int32_t batch, int32_t max_modes,
                  const double *omega, int32_t n_freq, const double *dL_dH, double *g_coef,
                  void *stream);

/* Host-only preview of the byte-balanced work partition modal_init makes
 * for `d` with n_workgroups co-resident workgroups (validates d like
 * modal_init; no device calls): out[0] work units, [1] workgroups used, [2]
 * planned cost of the most loaded workgroup, [3] mean cost per workgroup
 * (streamed-byte units).  A latency-bound batch (at most one instance per
 * CU, dense tensors under 64 MB per step, default waves and workgroups, no
 * MODAL_FLAG_SPLIT_ANY) is planned by modal_init with one slab per
 * workgroup instead, which this preview does not show.  EINVAL if the batch
 * cannot be partitioned. */
int modal_plan(const modal_desc *d, int32_t n_workgroups, int64_t out[4]);

/* The autotuner's key of a batch: 16 hexadecimal digits of a hash of the
 * device name, the scheme, the planning flags and every instance's kind,
 * mode counts and block-structure hint (no tensor values).  out: host
 * memory of at least 17 chars.  EINVAL for a description modal_init would
 * reject, or len < 17. */
int modal_tune_key(const modal_desc *d, char *out, int32_t len);

/* Message for the last failure on the calling thread ("" if none). */
const char *modal_last_error(void);

/* Host FP64 builder of the scaled coupling tensor for the sine in-plane
 * family (paper: Sec. 3.1, coupling-coefficient equations; modes
 * Phi_i = 2/sqrt(Lx Ly) sin(m_i pi x/Lx) sin(q_i pi y/Ly), Psi_n likewise
 * with (a_n, b_n)):
 *   out[n][i][j] = scale_n * int Psi_n L(Phi_i, Phi_j) dS
 * with the integral exact when nx = ny = 0, else the midpoint rule on an
 * nx x ny grid.  scale_n is given per in-plane mode (sqrt(E/2rho)/zeta_n^2
 * for the scaled tensor).  out is host memory [n_in][n_t][n_t] (FP32),
 * exactly symmetric in i, j.  Runs on `threads` host threads (0 = all). */
int modal_vk_coupling_sine(double Lx, double Ly, int32_t n_t, const int32_t *m,
                           const int32_t *q, int32_t n_in, const int32_t *a,
                           const int32_t *b, int32_t nx, int32_t ny,
                           const double *scale_n, float *out, int32_t threads);

#ifdef __cplusplus
}
#endif
#endif /* MODAL_H */
