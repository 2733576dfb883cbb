/*
 * pf.h - C ABI of the MI355X (gfx950) FFT phase-field twin-propagation step.
 *
 * One call of pf_step advances the twin volume fractions f_alpha of one
 * periodic grid by one time step of the phase-field model of twinning of
 * Zhang, Ma & Llorca (Sec. 2.2 and Sec. 3 of the paper):
 *   1. micro-elastic equilibrium at f^n for the eigenstrain
 *      eps* = eps_p + sum_a h(f_a) eps0_a and the mixture stiffness
 *      C(x) = C_g + sum_a h(f_a) (C_twin^a - C_g) (eq. (5)), solved by a
 *      Moulinec-Suquet fixed point with a Fourier-space Green's operator
 *      under a mixed mean strain/stress condition;
 *   2. the driving forces of eq. (17): double well (eq. (13)), gradient
 *      (eq. (14)) and elastic (eq. (15)) terms;
 *   3. the linearised semi-implicit update of eqs. (19)-(20), solved in
 *      Fourier space (Table 1):
 *      f^{n+1} = IFFT[FFT(f^n - L dt (chem - mech)) / (1 + 2 L dt kappa |xi|^2)];
 *   4. FP64 reductions: energies (eq. (12)), mean stress and strain, mean f.
 * The plastic strain eps_p is the per-voxel input handed over by the crystal
 * plasticity side, and f goes back to it (Table 1).
 *
 * Conventions
 *   Grid fields are float32, component-major, [comp][z][y][x] with x
 *   contiguous. Symmetric tensors use 6 tensor-Voigt components in the order
 *   xx, yy, zz, yz, xz, xy with TENSOR (not engineering) shear. 6x6 stiffness
 *   matrices are Voigt matrices in the engineering convention
 *   (sigma_I = C_IJ gamma_J, gamma = (e_xx, e_yy, e_zz, 2e_yz, 2e_xz, 2e_xy)),
 *   row-major, in Pa. Spectra are [comp][z][y][x/2+1] complex float32
 *   (interleaved re, im), unnormalised forward transform.
 *
 * Two paths compute the equilibrium of a step. The general one is the
 * fixed point above. When an instance has one stiffness everywhere
 * (n_grains == 1 and every C_var equal to C_grain), linear h, n_var <= 3 and
 * no plastic strain, the equilibrium stress of each wavevector is known in
 * closed form (the microelasticity of a homogeneous body, as used for
 * phase-field models with Fourier solvers): sigma_hat : eps0_a =
 * -sum_b B_ab(n) f_hat_b with B_ab(n) = eps0_a:C:eps0_b - (C:eps0_a n) .
 * K(n)^{-1} (C:eps0_b n), K(n) = C n n, and the mean strain follows from the
 * mixed condition. That is the exact solution the fixed point converges to
 * (the iteration is not needed), so the library takes it by itself; it keeps
 * no strain field, and PF_STEP_SAVE_STRESS or PF_STEP_FIXED_POINT select the
 * fixed point for a step.
 *
 * Batches
 *   pf_batch_init takes n_inst independent problems (e.g. an ensemble of
 *   representative volume elements of several sizes). Instances of one grid
 *   size are stacked along z in the workspace and every pass over them is
 *   one launch; a step of the whole batch that needs no host decision is
 *   captured once in a HIP graph and replayed. Batched instances are one
 *   grain each and share n_var, h_kind, A, kappa, L, dt, dx, ms_tol,
 *   ms_max_iter and bc_stress_mask; each has its own material, reference
 *   medium, eta0 and load. The instances of one grid size hold fewer than
 *   2^30 voxels together (PF_EINVAL otherwise).
 *
 * Memory and streams
 *   Every device buffer is owned by the caller. pf_init receives one device
 *   workspace of at least pf_workspace_size() bytes and keeps pointers into
 *   it; the library allocates only a small block of pinned host memory for
 *   the convergence status (freed by pf_destroy). All work is enqueued on
 *   the HIP stream given to pf_init (NULL = the default stream).
 *
 * Errors
 *   Every int-returning call returns PF_OK (0) or a negative PF_E* code and
 *   never throws. Argument errors are detected before any work is enqueued.
 *   Device-side conditions (non-finite fields, fixed point not converged)
 *   surface at the end of the pf_step call that met them. pf_last_error()
 *   gives a text description of the last failure on that context.
 */
#ifndef PF_TWIN_H
#define PF_TWIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_OK             0
#define PF_EINVAL        -1   /* bad argument or unsupported size          */
#define PF_ENOMEM        -2   /* workspace too small                        */
#define PF_EDEVICE       -3   /* HIP runtime error                          */
#define PF_ENOCONV       -4   /* equilibrium fixed point did not converge   */
#define PF_ENONFINITE    -5   /* NaN/Inf met in the order parameter         */
#define PF_EUNSUPPORTED  -6   /* valid request this build does not support  */

#define PF_H_LINEAR   0       /* h(f) = f                                   */
#define PF_H_QUINTIC  1       /* h(f) = f^3 (6 f^2 - 15 f + 10)             */

/* pf_step flags */
#define PF_STEP_SAVE_STRESS  1u  /* keep the equilibrium stress of the step  */
#define PF_STEP_FIXED_POINT  2u  /* use the fixed-point path even where the
                                    homogeneous spectral path applies        */

/* pf_fields selectors */
#define PF_FIELD_ETA     0    /* [n_var][nz][ny][nx]  order parameters       */
#define PF_FIELD_STRAIN  1    /* [6][nz][ny][nx]      total strain (state)   */
#define PF_FIELD_STRESS  2    /* [6][nz][ny][nx]      stress of the last step
                                 run with PF_STEP_SAVE_STRESS (get only)     */

typedef struct pf_ctx pf_ctx;

/* Problem fixed over a run. Supported sizes: nx, ny, nz each in
 * {32, 48, 64, 96, 128, 192, 256, 384, 512}; n_var in 1..6; n_grains in
 * 1..255. */
typedef struct {
  int32_t nx, ny, nz;
  double dx;               /* voxel edge, m                                 */
  int32_t n_var;           /* twin variants carried per voxel               */
  double A;                /* double-well height c1 (eq. (13)), J/m^3       */
  double kappa;            /* gradient coefficient c2 (eq. (14)), J/m       */
  double L;                /* mobility (c3 of eq. (16)), m^3/(J s)          */
  double dt;               /* time step, s                                  */
  int32_t h_kind;          /* PF_H_LINEAR or PF_H_QUINTIC                   */
  int32_t n_grains;
  const double *C_grain;   /* host [n_grains][6][6] parent stiffness        */
  const double *C_var;     /* host [n_grains][n_var][6][6] twin stiffness   */
  const double *eps0;      /* host [n_grains][n_var][6] twin eigenstrain    */
  const double *grain_rot; /* optional host [n_grains][3][3] crystal->sample
                              rotations (row-major). When given, C_grain,
                              C_var and eps0 are read for index 0 only, as
                              the crystal-frame material every grain shares;
                              grain g uses it turned by its rotation.       */
  const uint8_t *grain_id; /* device [nz][ny][nx], or NULL if n_grains == 1;
                              every value below n_grains (read once by
                              pf_init: PF_EINVAL otherwise); must stay
                              valid until pf_destroy                        */
  const float *eta0;       /* device [n_var][nz][ny][nx] initial f          */
  double C_ref[36];        /* reference medium of the fixed point (6x6)     */
  int32_t C_ref_auto;      /* 1: use the mean of all C_grain and C_var      */
  double ms_tol;           /* ||eps^{k+1}-eps^k|| <= tol ||eps^{k+1}||      */
  int32_t ms_max_iter;     /* >= 1; a problem with one stiffness everywhere
                              and C_ref equal to it needs exactly one       */
  uint32_t bc_stress_mask; /* bit i set: mean stress component i prescribed,
                              clear: mean strain component i prescribed     */
  const double *kappa_var; /* optional host [n_var][6]: anisotropic gradient
                              energy, one symmetric tensor K_a per variant
                              (tensor-Voigt xx yy zz yz xz xy, J/m, sample
                              frame) in place of kappa I: the gradient term
                              of f_a is grad f_a . K_a . grad f_a and its
                              implicit symbol xi . K_a . xi (Table 5 gives c2
                              along the twin-plane normal and the shear
                              direction; pf_mg_twin_gradient builds K_a). A
                              component at its Nyquist index enters only the
                              diagonal term. NULL: isotropic kappa. Needs
                              n_grains == 1 (PF_EUNSUPPORTED otherwise: a
                              spatially varying K is not solved exactly by
                              the spectral implicit step; kappa_grain takes
                              one tensor per grain). Copied at init.        */
  const float *mobility;   /* optional device [nz][ny][nx]: relative mobility
                              m in [0, 1] of each cell, L(x) = L m (the pad
                              layer of very low mobility around a specimen,
                              Sec. 4). The gradient term is split with L
                              implicit and L (m - 1) explicit, stable for any
                              m in [0, 1] (values outside are the caller's
                              responsibility); m = 1 is the plain step, m = 0
                              freezes f. Steps take the generic path. Needs a
                              one-instance context (PF_EUNSUPPORTED in a
                              batch); not for pf_macro_residual. Must stay
                              valid until pf_destroy. NULL: m = 1.         */
  double pf_tol;           /* ERR_f of Table 1 (see pf_max_iter)            */
  int32_t pf_max_iter;     /* solves of the fixed point i of Table 1 per step
                              (eqs. (19)-(20)): the guess is f^n, each further
                              solve re-evaluates the chemical (double-well)
                              force at the latest iterate with the gradient
                              term implicit and the mechanical force that of
                              f^n; the step ends when max |f^i - f^{i-1}| <=
                              pf_tol, checked after every solve (one stream
                              wait each), else PF_ENOCONV after pf_max_iter
                              solves, f left at the last iterate. 0 or 1: one
                              solve, the plain semi-implicit step. > 1 needs
                              a one-instance context (PF_EUNSUPPORTED in a
                              batch) and takes the generic path. With
                              f_M = 1 - sum f the conservation check of
                              Table 1 holds identically.                    */
  const double *kappa_grain; /* optional host [n_grains][n_var][6]: per-grain
                              anisotropic gradient tensors K_a^g of a
                              polycrystal (tensor-Voigt, J/m, sample frame;
                              pf_mg_twin_gradient builds them from the grain
                              rotations; Table 5, Sec. 4.3). The gradient
                              force -2 div(K_a(x) grad f_a) is split: kbar_a I
                              implicit, kbar_a the largest eigenvalue of K_a^g
                              over the grains, and the remainder
                              2 div((K_a(x) - kbar_a I) grad f_a) explicit at
                              f^n through spectral first derivatives (zero at
                              a Nyquist index), three more spectral passes
                              over 3 n_var components per step. Stable at any
                              dt (kbar_a I - K_a(x) is positive semidefinite).
                              G_gd reports the energy of the same operator.
                              Not with kappa_var (PF_EINVAL); not with a
                              mobility field, pf_max_iter > 1 or in a batch
                              (PF_EUNSUPPORTED). Copied at init.            */
} pf_problem;

/* Load of one pf_step call. */
typedef struct {
  double eps_bar[6];       /* prescribed mean strain (strain-controlled)    */
  double sig_bar[6];       /* prescribed mean stress (stress-controlled), Pa */
  const float *eps_p;      /* device [6][nz][ny][nx] plastic strain; NULL
                              keeps the previous one (zero at first). The
                              buffer must stay valid while steps use it.    */
  uint32_t flags;          /* PF_STEP_* */
} pf_load;

/* Reductions of the state a step started from (FP64 on the device). */
typedef struct {
  int64_t step;            /* steps completed                               */
  double G_dw, G_gd, G_me; /* energies of eqs. (13)-(15) over the grid, J   */
  double sig_mean[6];      /* volume-averaged stress, Pa                    */
  double eps_mean[6];      /* volume-averaged strain                        */
  double eta_mean[6];      /* volume-averaged f per variant                 */
  double eta_min, eta_max; /* over all variants and voxels                  */
  int32_t ms_iters;        /* fixed-point iterations of the last step       */
  double ms_residual;      /* last relative strain change                   */
  int32_t pf_iters;        /* solves of the update in the last step (1
                              unless pf_max_iter > 1)                       */
  double pf_change;        /* max |f^i - f^{i-1}| of its last solve (0
                              unless pf_max_iter > 1)                       */
  int64_t steps_replayed;  /* steps of the context run as one replayed graph
                              whose fixed point converged on the device     */
} pf_stats;

/* Workspace bytes for a problem (only the sizes, n_var and n_grains are read). */
int pf_workspace_size(const pf_problem *prob, size_t *bytes);

/* Validate, carve the workspace, upload tables, copy eta0 in, set the strain
 * to the mean load later given by the first pf_step. hip_stream: hipStream_t
 * or NULL. On success *out receives a new context. */
int pf_init(const pf_problem *prob, void *workspace, size_t ws_bytes,
            void *hip_stream, pf_ctx **out);

/* Advance n_steps steps under one load. Work is enqueued on the context's
 * stream. A step that needs no decision on the host (the homogeneous spectral
 * path, or one exact fixed-point iteration) is replayed from a captured graph.
 * A fixed-point step whose first iterate is extrapolated from four converged
 * steps (the fifth step on) is also replayed as one graph: as many
 * iterations as the last step took, each returning at once on the device
 * once its instance has converged, then the update, which runs only if every
 * instance of its group converged; the call reads the convergence flags once
 * per step and, if a group needs more iterations, continues them (one status
 * read per iteration) and then updates it. Other fixed-point steps (the first
 * four, after pf_fields sets a field, with profiling, PF_STEP_SAVE_STRESS or
 * pf_max_iter > 1) read the flags after every iteration. Either way the
 * kernels and their order are the same, so the results are identical. */
int pf_step(pf_ctx *ctx, int32_t n_steps, const pf_load *load);

/* Copy a field between the context and a caller device buffer of the same
 * layout (set = 0: context -> buf, set = 1: buf -> context), on the stream.
 * Setting the order parameters or the strain restarts the extrapolation of
 * the next step's first fixed-point iterate from the field set; setting the
 * strain also takes its mean (FP64, on the stream) as the mean strain of the
 * state. A checkpoint is the order parameters and the strain read back; set
 * into a context of the same problem they continue the run (to the fixed
 * point's tolerance, since the extrapolation history is not part of it; bit
 * for bit on the homogeneous spectral path, whose state is f alone).
 * Errors: PF_EINVAL for an unknown selector, a null buffer, a set of the
 * stress, or a get of the strain that the spectral path did not form. */
int pf_fields(pf_ctx *ctx, int32_t which, int32_t set, float *buf);

/* Synchronise the stream and return the reductions of the last step. */
int pf_stats_get(pf_ctx *ctx, pf_stats *out);

/* 3D transforms with the context's plan, for checking the FFT passes.
 * direction +1: real[ncomp][nz][ny][nx] -> spec[ncomp][nz][ny][nx/2+1]
 * (unnormalised). direction -1: spec -> real with the 1/(nx ny nz) factor;
 * spec is overwritten. ncomp in 1..6. */
int pf_fft(pf_ctx *ctx, int32_t direction, int32_t ncomp, float *real, void *spec);

/* Launch plan of a group of same-size instances: for each column pass the
 * FFT plan variant (radix split and elements per thread, see pf_fft_plan)
 * and the column tile (pencils of consecutive kx per block).
 *   ytile, yplan:       y passes (tile 8 or 16, variant 0, 1 or 2)
 *   ztile_ms, zplan_ms: Green z pass of the fixed point (8 or 16; 0 or 1)
 *   zplan_ac:           z pass of the Allen-Cahn update (16 columns; 0, 1, 2)
 *   ztile_kh, zplan_kh: z pass of the homogeneous spectral path (8 or 16; 0, 1)
 * A plan whose block would exceed 1024 threads does not exist. */
typedef struct {
  int32_t ytile, yplan;
  int32_t ztile_ms, zplan_ms;
  int32_t zplan_ac;
  int32_t ztile_kh, zplan_kh;
} pf_plan;

/* Autotuner (the FFT plans and tiles of the column passes picked by timing on
 * the device; Sec. 3 solves in Fourier space, the plans are this
 * implementation's): for every group of same-size instances, each pass's
 * candidates (y: 3 plan variants x 2 tiles; Green z: 2 x 2; Allen-Cahn z: 3;
 * spectral z: 2 x 2; those that fit a block) are timed within the passes a
 * step runs around that pass (x forward, y forward, z, y inverse of a
 * fixed-point iteration, an Allen-Cahn update or a spectral step), on the
 * group's own fields and spectral buffer (zeroed first; it holds nothing
 * between steps; no state field is written and the instances' FP64 state is
 * kept), best of two alternating rounds of 10 sequences. Plans differ in rounding only (each is
 * the same transform), so a tuned context matches an untuned one to FP32
 * round-off. cache_path (may be NULL): a text file of one JSON object per
 * line, keyed by the device's architecture name and compute-unit count and by
 * the group's grid, instance count, n_var and path, holding the plan and every
 * candidate's time; an entry found there is applied without timing (unless
 * flags has PF_TUNE_RETIME) and each timed group is appended. Synchronises
 * the stream; not during graph capture; call between steps. *n_timed (may be
 * NULL) receives the number of groups timed. */
#define PF_TUNE_RETIME 1u
int pf_autotune(pf_ctx *ctx, const char *cache_path, uint32_t flags, int32_t *n_timed);

/* Plan of the group holding instance inst (the defaults until tuned or set). */
int pf_batch_plan(pf_ctx *ctx, int32_t inst, pf_plan *out);

/* Set the plan of the group holding instance inst (e.g. one read from a
 * cache); PF_EINVAL if a pass has no such plan for the group's grid. */
int pf_batch_set_plan(pf_ctx *ctx, int32_t inst, const pf_plan *plan);

/* FFT plan variant of an axis length n: elements per thread, radix of each
 * Stockham stage (radices[8]) and the stage count. PF_EINVAL for an
 * unsupported length or variant (0, 1, 2). */
int pf_fft_plan(int32_t n, int32_t variant, int32_t *elems_per_thread, int32_t *radices,
                int32_t *n_stages);

/* Spectral convolution of the learned stepper for training (the layers
 * v_l = GELU(W v + b + K v) of a Fourier neural operator; K v keeps 2m x 2m x m
 * modes: kx < m, ky and kz in [0, m) u [n - m, n), positive then negative).
 * Batches of B samples with C channels, channel-first FP32 device arrays:
 * v, y, dy, dv [B][C][nz][ny][nx]; S, M, G [B][C][2m][2m][m] complex64
 * (re, im interleaved); R, dR [C][C][2m][2m][m] complex64, [out][in][kz'][ky'][kx].
 *   forward:  S = kept modes of rfftn(v), M = R S per mode,
 *             y = irfftn(M placed on the kept modes) = K v;
 *   backward: G = c(kx)/N kept modes of rfftn(dy) (c = 1 on kx = 0, else 2),
 *             dR = sum_b G conj(S) (dL/dRe R + i dL/dIm R for L with
 *             dL/dy = dy), M = R^H G, dv = sum over kept modes
 *             Re[M e^{+i k.x}] (= dL/dv), given S from the forward call.
 * Sizes: 1 <= B <= 64, 1 <= C <= 256, axes 4..256, 2m < nx, 2m <= ny, nz.
 * work: pf_specconv_workspace_size bytes of device memory. Enqueued on
 * hip_stream (NULL: the null stream); PF_EINVAL for bad sizes or NULL
 * pointers, PF_ENOMEM for a short work buffer. */
int pf_specconv_workspace_size(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m,
                               size_t *bytes);
int pf_specconv_forward(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m,
                        const float *v, const float *R, float *S, float *M, float *y, void *work,
                        size_t work_bytes, void *hip_stream);
int pf_specconv_backward(int32_t B, int32_t C, int32_t nx, int32_t ny, int32_t nz, int32_t m,
                         const float *dy, const float *R, const float *S, float *G, float *M, float *dv,
                         float *dR, void *work, size_t work_bytes, void *hip_stream);

/* Pointwise parts of the learned stepper's training and its optimiser (FP32,
 * channel-first device arrays [B][channels][nvox], nvox = nz ny nx; C in
 * {4, 8, 16, 32, 64}, H <= 128; the network of the stepper: v_0 = P [f, c] + p
 * with 7 conditioning values c per sample, v_l = GELU(u_l), u_l = W_l v + b_l
 * + K_l v, f~ = f + Q2 GELU(Q1 v_L + q1) + q2). Parameters as the stepper
 * holds them: P [C][8], W [C][C] (out, in), Q1 [H][C], Q2 [H]. All enqueued on
 * stream (NULL: the null stream); PF_EINVAL for bad sizes or NULL pointers.
 *   pf_nt_lift:            v0 = P [f, cond] + p
 *   pf_nt_layer_forward:   u = W v + bias + kv, vout = GELU(u)
 *   pf_nt_project_forward: z = Q1 v + q1 (kept), out = f + Q2 GELU(z) + q2
 *   pf_nt_project_backward: for the loss sum of (out - target)^2 times
 *       scale / 2, g = scale (out - target), dz = g Q2 GELU'(z), hg = GELU(z),
 *       dv = Q1^T dz
 *   pf_nt_gelu_backward:   du = dvout GELU'(u) over n values
 *   pf_nt_layer_input_grad: dv = W^T du + dvs
 *   pf_nt_outer_sum:       out[a][c] (+)= sum over samples and voxels of
 *       X[b][a][i] Y[b][c][i] (Y NULL: 1), a < MA, c < MC; work of
 *       pf_nt_outer_workspace bytes (per-chunk partials, added in a fixed order)
 *   pf_nt_cond_grad:       dP[c][1 + j] = sum_b dK[b][c] cond[b][j],
 *       dp[c] = sum_b dK[b][c] (dK: per-sample channel sums of dv0)
 *   pf_nt_adam:            Adam with bias correction, step >= 1 */
int pf_nt_lift(int32_t B, int32_t C, int64_t nvox, const float *P, const float *p, const float *f,
               const float *cond, float *v0, void *stream);
int pf_nt_layer_forward(int32_t B, int32_t C, int64_t nvox, const float *W, const float *bias,
                        const float *v, const float *kv, float *u, float *vout, void *stream);
int pf_nt_project_forward(int32_t B, int32_t C, int32_t H, int64_t nvox, const float *Q1,
                          const float *q1, const float *Q2, float q2, const float *v, const float *f,
                          float *z, float *out, void *stream);
int pf_nt_project_backward(int32_t B, int32_t C, int32_t H, int64_t nvox, const float *Q1,
                           const float *Q2, const float *z, const float *out, const float *target,
                           float scale, float *g, float *dz, float *hg, float *dv, void *stream);
int pf_nt_gelu_backward(int64_t n, const float *dvout, const float *u, float *du, void *stream);
int pf_nt_layer_input_grad(int32_t B, int32_t C, int64_t nvox, const float *W, const float *du,
                           const float *dvs, float *dv, void *stream);
int pf_nt_outer_workspace(int32_t B, int32_t MA, int32_t MC, int64_t nvox, size_t *bytes);
int pf_nt_outer_sum(int32_t B, int32_t MA, int32_t MC, int64_t nvox, const float *X, const float *Y,
                    float *out, int32_t accumulate, float *work, size_t work_bytes, void *stream);
/* pf_nt_outer_sum without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, bit for bit, with the
 * per-chunk partials in a fixed array of the library (16 MiB on each GPU it
 * runs on, kept until the process ends; its address is looked up on the
 * first call on a device). The call allocates nothing. PF_ENOMEM when the
 * partials (pf_nt_outer_workspace bytes) exceed 16 MiB, PF_EINVAL as
 * pf_nt_outer_sum, PF_EDEVICE when the stream's device cannot be resolved.
 * Every call on one GPU shares the array: calls that overlap on a GPU (two
 * streams, two threads) race; calls in order on one stream do not. */
int pf_nt_outer_sum_noalloc(int32_t B, int32_t MA, int32_t MC, int64_t nvox, const float *X,
                            const float *Y, float *out, int32_t accumulate, void *stream);
int pf_nt_cond_grad(int32_t B, int32_t C, const float *dK, const float *cond, float *dP, float *dp,
                    void *stream);
int pf_nt_adam(int64_t n, float *w, const float *g, float *m, float *v, float lr, float beta1,
               float beta2, float eps, int32_t step, void *stream);

/* Per-kernel timing with HIP events on the context's stream: enable (1) or
 * disable (0) and reset; read returns up to max_n entries of name, launch
 * count and total milliseconds, the number of entries in *n. */
int pf_profile_enable(pf_ctx *ctx, int32_t on);
int pf_profile_read(pf_ctx *ctx, int32_t max_n, char (*names)[64],
                    int64_t *counts, double *total_ms, int32_t *n);
/* Time only the launches of the named stage (e.g. "ms_x_forward"); NULL or
 * "" times every launch. The name is copied. */
int pf_profile_select(pf_ctx *ctx, const char *name);

int pf_destroy(pf_ctx *ctx);
const char *pf_last_error(const pf_ctx *ctx);

/* FE <-> FFT mapping by nearest Gauss point (the mapping of Sec. 3 that
 * Sec. 5 compares with interpolation and keeps; Table 1 starts each step by
 * mapping the finite-element data to the FFT cells and ends by mapping the
 * volume fractions back). The Gauss points seed a Voronoi tessellation of
 * the grid: every cell takes the data of the point nearest to its centre,
 * every point takes the mean over the cells of its domain (the cell that
 * contains it, clamped to the grid, when the domain holds no cell centre).
 * Cell (i, j, k), x fastest, has its centre at ((i+1/2) dx, (j+1/2) dx,
 * (k+1/2) dx) in the frame of the points; distances are Euclidean and not
 * periodic; the squared distance is (px-cx)^2 + (py-cy)^2 + (pz-cz)^2 in
 * FP64, summed in that order without fused multiply-adds, and ties go to the
 * lower point index, so the map is exact and reproducible. Any grid with
 * nx, ny, nz >= 1 and fewer than 2^31 cells; 1 <= n_points <= 2^28.
 * All arrays are device memory owned by the caller; work goes on the given
 * HIP stream (NULL = default). */

/* Workspace bytes for a grid and n_points. The workspace holds scratch of
 * the build and then each point's list of cells, which pf_vmap_to_points
 * reads: keep it, unchanged, between the two. */
int pf_vmap_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t n_points,
                           size_t *bytes);

/* Nearest point of every cell: points [n_points][3] (m, FP64), out
 * cell_point [nz][ny][nx] point indices; also fills the workspace's per-
 * point cell lists. Waits on the stream once (the bounding box sizes the
 * bins); PF_EINVAL on a non-finite coordinate, PF_ENOMEM if ws_bytes is
 * short. */
int pf_vmap_build(int32_t nx, int32_t ny, int32_t nz, double dx,
                  int32_t n_points, const double *points,
                  void *workspace, size_t ws_bytes, void *hip_stream,
                  int32_t *cell_point);

/* Point data to the cells: cell_values[c][cell] =
 * point_values[c][cell_point[cell]] for ncomp components (FP32). */
int pf_vmap_to_cells(int64_t n_cells, const int32_t *cell_point,
                     int32_t n_points, int32_t ncomp,
                     const float *point_values, float *cell_values,
                     void *hip_stream);

/* Cell data back to the points: the mean over each point's domain (FP64
 * sum in ascending cell order, then one division, rounded to FP32: exact
 * and reproducible), or the cell that contains the point. cell_values
 * [ncomp][nz][ny][nx], point_values [ncomp][n_points]; cell_point, points
 * and the workspace as left by pf_vmap_build. */
int pf_vmap_to_points(int32_t nx, int32_t ny, int32_t nz, double dx,
                      const int32_t *cell_point, int32_t n_points,
                      const double *points, int32_t ncomp,
                      const float *cell_values, float *point_values,
                      const void *workspace, size_t ws_bytes, void *hip_stream);

/* Batches of independent instances (see "Batches" above). The single-instance
 * calls are these with n_inst = 1; pf_step, pf_fields and pf_stats_get act on
 * instance 0 of a one-instance context only.
 *   pf_batch_workspace_size: bytes for the whole batch (validates it).
 *   pf_batch_init: as pf_init for probs[0..n_inst-1].
 *   pf_batch_step: loads[n_inst], one per instance. A given eps_p is copied
 *     into the batch's own plastic-strain field (zero until first given).
 *     The flags of all loads are or-ed.
 *   pf_batch_fields, pf_batch_stats: as pf_fields, pf_stats_get for
 *     instance inst (0-based, in the order of probs). */
int pf_batch_workspace_size(const pf_problem *probs, int32_t n_inst, size_t *bytes);
int pf_batch_init(const pf_problem *probs, int32_t n_inst, void *workspace,
                  size_t ws_bytes, void *hip_stream, pf_ctx **out);
int pf_batch_step(pf_ctx *ctx, int32_t n_steps, const pf_load *loads);
int pf_batch_fields(pf_ctx *ctx, int32_t inst, int32_t which, int32_t set,
                    float *buf);
int pf_batch_stats(pf_ctx *ctx, int32_t inst, pf_stats *out);
int pf_batch_size(const pf_ctx *ctx);  /* number of instances, 0 for NULL */

/* ------------------------------------------------------------ surrogate
 * A Fourier neural operator (Li et al. 2021) standing in for S plain steps of
 * a one-variant homogeneous context (a learned macro stepper; the paper has
 * none: its Sec. 3 notes that small PF time steps dominate the cost):
 *   v_0 = P [f, c] + p;  v_l = GELU(W_l v + b_l + K_l v), l = 1..4;
 *   f~  = f + Q_2 GELU(Q_1 v_4 + q_1) + q_2,
 * K v = inverse real 3D transform of R(k) times the transform of v on the
 * kept modes kx < m, ky, kz in [0, m) u [n - m, n) (ordered positive, then
 * negative), zero elsewhere; forward transform unnormalised, inverse with
 * 1 / (nx ny nz); GELU(x) = x Phi(x). c: 7 constant conditioning values
 * (sample-frame eps0 / gamma_tw in tensor-Voigt order, applied strain /
 * 5e-3). The forward pass runs with BF16 activations and weights and FP32
 * accumulation (matrix cores for the channel mixing and the projection).
 *
 * The prediction is accepted when the residual of the macro step of S plain
 * steps from f^n to f~ (the summed plain steps with both sums by the
 * end-corrected trapezoid rule; see pf_macro_residual) is <= tol; otherwise
 * the context falls back to S plain steps from f^n. Supported: a single-instance
 * context, n_var = 1, the homogeneous spectral path (one stiffness, linear h,
 * no plastic strain), nx a multiple of 32, every axis <= 128, modes <= 16. */
typedef struct pf_fno pf_fno;

typedef struct {
  int32_t width, modes, hidden, n_layers, n_cond;  /* 32, m, 128, 4, 7        */
  const float *P;    /* host [width][1 + n_cond] lift (column 0: f)          */
  const float *p;    /* host [width]                                        */
  const float *W;    /* host [n_layers][width][width] (out, in)             */
  const float *b;    /* host [n_layers][width]                              */
  const float *R;    /* host [n_layers][width out][width in][2m kz][2m ky][m kx][2]
                        complex (re, im), kz / ky in kept order              */
  const float *Q1;   /* host [hidden][width]                                */
  const float *q1;   /* host [hidden]                                       */
  const float *Q2;   /* host [hidden]                                       */
  float q2;
} pf_fno_weights;

typedef struct {     /* accumulated by pf_fno_advance (zero it first)       */
  int32_t accepted, rejected;
  double rho_max_accepted, rho_min_rejected, last_rho;
} pf_fno_report;

/* Device workspace bytes of a stepper on this context with m modes. */
int pf_fno_workspace_size(const pf_ctx *ctx, int32_t modes, size_t *bytes);
/* Convert (BF16) and upload the weights into the caller's workspace. */
int pf_fno_init(pf_ctx *ctx, const pf_fno_weights *w, void *workspace,
                size_t ws_bytes, pf_fno **out);
/* eta_out = f~(eta_in) for conditioning cond[7]; device buffers
 * [nz][ny][nx], not aliased; on the context's stream. */
int pf_fno_forward(pf_fno *fno, const double *cond, const float *eta_in,
                   float *eta_out);
/* n_calls macro steps of steps_per_call plain steps each on the context's
 * order parameter: predict, check rho <= tol (one wait on the stream per
 * call), else fall back to plain steps under load. */
int pf_fno_advance(pf_fno *fno, int32_t n_calls, int32_t steps_per_call,
                   const double *cond, const pf_load *load, double tol,
                   pf_fno_report *report);
int pf_fno_destroy(pf_fno *fno);

/* Residual of a macro step of n = n_steps plain steps from eta_prev (device
 * [nz][ny][nx]) to the context's current order parameter f, under load.
 * The n plain steps summed (Sec. 3, eqs. (19)-(20): local force chem - mech
 * at the old state, gradient force G f = -2 kappa lap f at the new one) with
 * both sums taken by the trapezoid rule with the end correction of a left
 * (right) Riemann sum, p = (n+1)/2, m = (n-1)/2:
 *   r = f - eta_prev + L dt [p dF/df(eta_prev) + m dF/df(f) + G (f - eta_prev)],
 * dF/df = chem + G f - mech at the equilibrium of each state; *rho = max |r|.
 * Zero up to rounding when f is one exact plain step from eta_prev (n = 1),
 * second order in n dt over n exact steps. Homogeneous single-instance
 * contexts (the spectral path: one stiffness, linear h, n_var <= 3, no
 * plastic strain, uniform mobility), else PF_EUNSUPPORTED; uses the
 * context's spectral buffer; waits on the stream. */
int pf_macro_residual(pf_ctx *ctx, const float *eta_prev, int32_t n_steps,
                      const pf_load *load, double *rho);

/* Streaming device copy of bytes (a multiple of 16, both pointers 16-byte
 * aligned, else PF_EINVAL; PF_EDEVICE if the launch fails) on hip_stream:
 * 16 bytes per lane with the nontemporal hint on both sides, grid-stride.
 * Not part of the method: the attainable HBM rate of a kernel that only
 * moves bytes, measured beside the passes as the reference for their rates
 * (the roofline's peak stays the 8 TB/s datasheet figure). Asynchronous. */
int pf_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Host helper: sample-frame tables of Mg tension twins for n_grains grains.
 * Crystal frame x || [10-10], y || [-12-10], z || [0001]; c_over_a and
 * gamma_tw as in Sec. 2.1 (1.633, 0.129); C_hex = {C11, C12, C13, C33, C44}
 * in Pa (Table 2); rotations [n_grains][3][3] map crystal to sample vectors;
 * variant_ids[n_var] pick among the six {10-12}<-1011> variants (0-based);
 * the twin stiffness is the parent one turned by Q = 2 m m^T - I.
 * Outputs: C_grain [n_grains][6][6], C_var [n_grains][n_var][6][6],
 * eps0 [n_grains][n_var][6] (tensor-Voigt). Host memory, caller-owned. */
int pf_mg_twin_tables(const double C_hex[5], double c_over_a, double gamma_tw,
                      int32_t n_grains, const double *rotations,
                      int32_t n_var, const int32_t *variant_ids,
                      double *C_grain, double *C_var, double *eps0);

/* Host helper: anisotropic gradient tensors of Mg tension-twin variants,
 * K_a = c2n m m + c2s s s + c2t t t (m the twin-plane normal, s the shear
 * direction, t = m x s; Table 5 gives c2n = 2.81e-7 N and c2s = 2.81e-6 N,
 * nothing along t), turned to the sample frame by the rotations
 * [n_grains][3][3]. Output kappa_var [n_grains][n_var][6] (tensor-Voigt),
 * host memory, caller-owned. PF_EINVAL on a bad variant id or a negative
 * coefficient. */
int pf_mg_twin_gradient(double c_over_a, double c2n, double c2s, double c2t,
                        int32_t n_grains, const double *rotations,
                        int32_t n_var, const int32_t *variant_ids,
                        double *kappa_var);

#ifdef __cplusplus
}
#endif
#endif /* PF_TWIN_H */
