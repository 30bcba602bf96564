/*
 * delimit.h -- C ABI of libdelimit.so, an MI355X (gfx950) implementation of
 * the DELIMIT diffusion-imaging layers (Koppers & Merhof, arXiv:1808.01517):
 * Signal2SH and SH2Signal (Sec. 2.2) and the local spherical convolution
 * with cyclic kernels, single- and multi-shell (Sec. 2.3 and 2.3.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Plain C: no C++ or torch types.  Voxel counts are int64_t.  A stream
 *   is a hipStream_t passed as void* (NULL = the default stream).
 * - Pointers documented "device" must point to device memory of the current
 *   HIP device; "host" pointers are ordinary CPU memory.  Device data at the
 *   ABI is row-major float32, except LSC activations passed to the _io
 *   calls as bfloat16 (dlm_io_flags); the caller owns every activation,
 *   gradient, weight and workspace buffer.  Plans own their device tables.
 * - Compute calls are asynchronous on the given stream and never allocate;
 *   they validate every argument on the host before any launch and return a
 *   dlm_status.  No C++ exception crosses the ABI.  On error nothing has been
 *   launched and dlm_last_error() describes the problem (thread-local).
 * - Results are deterministic: no floating-point atomics; reductions run in
 *   a fixed order for a given (V, workspace size).
 * - Real even-order SH of order L (even, 0..16) have K = (L+1)(L+2)/2
 *   coefficients, index j = l(l+1)/2 + m; m<0 uses sqrt2 N P_l^|m| cos(|m|phi),
 *   m=0 N P_l, m>0 sqrt2 N P_l^m sin(m phi), Condon-Shortley phase included.
 */
#ifndef DELIMIT_H
#define DELIMIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DLM_OK = 0,
  DLM_EINVAL = 1,      /* invalid argument: NULL pointer, size, order, NaN   */
  DLM_ESINGULAR = 2,   /* a fit's normal matrix is not positive definite     */
  DLM_ENOMEM = 3,      /* allocation failed (plan creation only)             */
  DLM_EDEVICE = 4,     /* HIP runtime error (no device, launch, copy)        */
  DLM_EWORKSPACE = 5   /* workspace smaller than the minimum                 */
} dlm_status;

/* Arithmetic form.  DLM_FP32: float32 inputs and products, float32
 * accumulation.  DLM_BF16: matrix-core inputs rounded to bfloat16 (round to
 * nearest even) with float32 accumulation; tables are formed in float64 and
 * rounded once.  Storage at the ABI is float32 in both forms. */
typedef enum { DLM_FP32 = 0, DLM_BF16 = 1 } dlm_precision;

const char *dlm_status_str(dlm_status s);
/* Last error message of the calling thread ("" if none). */
const char *dlm_last_error(void);
/* Library ABI version, currently 1. */
int dlm_version(void);

/* ------------------------------------------------------------------------
 * Host-only float64 tables (no device needed; for inspection and tests).
 * ------------------------------------------------------------------------ */

/* SH basis B[i][j] = Y_j(dir_i), dirs host [n][3] (normalised internally),
 * B host [n][K].  Sec. 2.2 (the layers' spherical-harmonic representation). */
dlm_status dlm_sh_basis(int sh_order, const double *dirs, int64_t n, double *B);

/* Regularised least-squares fit P = (B^T B + lambda L)^{-1} B^T with
 * L = diag(l^2 (l+1)^2) (Laplace-Beltrami penalty, Signal2SH's lb_lambda,
 * Sec. 2.2).  dirs host [n][3]; P host [K][n].  DLM_ESINGULAR when the
 * normal matrix is not positive definite (e.g. lambda = 0 with n < K). */
dlm_status dlm_sh_fit_matrix(int sh_order, const double *dirs, int64_t n, double lb_lambda, double *P);

/* Cyclic-kernel points (Sec. 2.3, Fig. 3): for every direction g_i the
 * centre g_i followed by ring r = 1..R of kernel_sizes[r-1] points at
 * angular distance r * angular_distance / R (radians), azimuth 2 pi b / n_r
 * measured from e_theta toward e_phi.  g host [m][3]; points host [m][T][3],
 * T = 1 + sum(kernel_sizes). */
dlm_status dlm_lsc_kernel_points(const double *g, int64_t m, const int *kernel_sizes, int n_rings,
                                 double angular_distance, double *points);

/* ------------------------------------------------------------------------
 * SH plan: one gradient table (Signal2SH / SH2Signal parameters, Sec. 2.2)
 * ------------------------------------------------------------------------ */
typedef struct dlm_sh_plan dlm_sh_plan;

/* Build the per-shell basis B_s [N_s][K] and fit P_s [K][N_s] in float64 on
 * the host and upload float32 and bfloat16 copies to the current device.
 * bvecs host [n][3], bvals host [n].  Volumes with b < b0_max are b=0
 * volumes and are dropped (the layers take b0-normalised signal); the rest
 * are grouped into shells (b within shell_rel_tol of a shell's mean b),
 * ordered by increasing b, volumes within a shell in table order.
 * Signal arrays at the ABI are shell-major: [V][N_dw] = shell 0's N_0
 * values, then shell 1's ...  *out receives the plan (free with
 * dlm_sh_plan_destroy).
 * SH2Signal evaluates the basis on any table (Sec. 2.2: signals on N
 * resampled directions), so a shell whose regularised normal matrix
 * B_s^T B_s + lambda L is singular (e.g. fewer directions than K at
 * lambda = 0) does not fail creation: the plan then evaluates only
 * (dlm_sh2signal_fwd/bwd, dlm_sh2signal_mse_fwd_bwd), and every call that
 * needs P_s (dlm_signal2sh_fwd/bwd, dlm_signal2sh_fwd_raw, P copies of
 * dlm_sh_plan_matrices) returns DLM_ESINGULAR. */
dlm_status dlm_sh_plan_create(const double *bvecs, const double *bvals, int64_t n, int sh_order,
                              double lb_lambda, double b0_max, double shell_rel_tol, dlm_sh_plan **out);
/* n_shells, K and total diffusion-weighted count N_dw (any may be NULL). */
dlm_status dlm_sh_plan_info(const dlm_sh_plan *plan, int *n_shells, int *K, int64_t *n_dw);
/* Shell s: direction count, mean b, and (if volume_index != NULL) the
 * index into the creation table of each of its n_dirs volumes. */
dlm_status dlm_sh_plan_shell(const dlm_sh_plan *plan, int shell, int64_t *n_dirs, double *b,
                             int64_t *volume_index);
/* Host float64 copies of B_s [N_s][K] and P_s [K][N_s] (either may be NULL;
 * B is copied before P is refused on a plan without a fit). */
dlm_status dlm_sh_plan_matrices(const dlm_sh_plan *plan, int shell, double *B, double *P);
/* DLM_OK when every shell has its fit P_s (Signal2SH is available),
 * DLM_ESINGULAR (message names the first singular shell) when the plan
 * evaluates only. */
dlm_status dlm_sh_plan_fit_status(const dlm_sh_plan *plan);
/* Replace the directions (same n and b-values as at creation, e.g. a fresh
 * per-scan distortion) and rebuild every table in float64; the upload is
 * ordered on `stream`, so calls already queued on it use the old tables.
 * A plan with a fit keeps one: if the new table's fit is singular the call
 * returns DLM_ESINGULAR and leaves the plan unchanged. */
dlm_status dlm_sh_plan_update_gradients(dlm_sh_plan *plan, const double *bvecs, void *stream);
void dlm_sh_plan_destroy(dlm_sh_plan *plan);

/* Signal2SH (Sec. 2.2): c[v][s][:] = P_s x[v][s-block].
 * x device [V][N_dw] (b0-normalised), c device [V][S][K]. */
dlm_status dlm_signal2sh_fwd(const dlm_sh_plan *plan, const float *x, float *c, int64_t V,
                             dlm_precision prec, void *stream);
/* Adjoint of Signal2SH: dx[v][s-block] = P_s^T dc[v][s][:]. */
dlm_status dlm_signal2sh_bwd(const dlm_sh_plan *plan, const float *dc, float *dx, int64_t V,
                             dlm_precision prec, void *stream);
/* SH2Signal (Sec. 2.2): x[v][s-block] = B_s c[v][s][:].
 * c device [V][S][K], x device [V][N_dw]. */
dlm_status dlm_sh2signal_fwd(const dlm_sh_plan *plan, const float *c, float *x, int64_t V,
                             dlm_precision prec, void *stream);
/* Adjoint of SH2Signal: dc[v][s][:] = B_s^T dx[v][s-block]. */
dlm_status dlm_sh2signal_bwd(const dlm_sh_plan *plan, const float *dx, float *dc, int64_t V,
                             dlm_precision prec, void *stream);

/* The q-space loss head of training (Sec. 1: the network's SH output is
 * taken back to q-space by SH2Signal, Sec. 2.2, and compared there), fused
 * into one pass so that neither the predicted signal nor its gradient has
 * to go through device memory:
 *   xhat[v][s-block] = B_s c[v][s][:]
 *   loss             = mean over V * N_dw of (xhat - target)^2   (device scalar)
 *   dc[v][s][:]      = B_s^T (2 (xhat - target) / (V N_dw))[v][s-block]
 * c device [V][S][K]; target, xhat device [V][N_dw] (xhat may be NULL, then
 * it is not written); dc device [V][S][K] (must not alias c).  Same result as
 * dlm_sh2signal_fwd, dlm_mse_fwd_bwd and dlm_sh2signal_bwd in a row.
 * Supported when every shell has at most 96 directions and K <= 64 (sh
 * order <= 8); dlm_sh2signal_mse_supported says whether a plan qualifies,
 * otherwise the call returns DLM_EINVAL.  ws: device workspace of at least
 * dlm_sh2signal_mse_workspace_bytes(plan, V) bytes (per-wave partial sums). */
int dlm_sh2signal_mse_supported(const dlm_sh_plan *plan);
size_t dlm_sh2signal_mse_workspace_bytes(const dlm_sh_plan *plan, int64_t V);
dlm_status dlm_sh2signal_mse_fwd_bwd(const dlm_sh_plan *plan, const float *c, const float *target, int64_t V,
                                     float *loss, float *dc, float *xhat, void *ws, size_t ws_bytes,
                                     dlm_precision prec, void *stream);
/* dlm_sh2signal_mse_fwd_bwd without a workspace, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation).  The partial sums live in a static
 * device array of dlm_sh2signal_mse_static_scratch_bytes() bytes (4 MiB),
 * one per device, held until the process ends; calls whose
 * dlm_sh2signal_mse_workspace_bytes(plan, V) exceeds it return
 * DLM_EWORKSPACE (about 5.59 M voxels of a three-shell table fit).  The
 * call allocates nothing (with timing off, the default): its first call on
 * a device only looks up that device's array address.  Every call on one
 * device shares the array and leaves its contents behind; nothing in it
 * needs clearing, but calls that overlap on one device (other streams,
 * unordered host threads) race.  Results are those of
 * dlm_sh2signal_mse_fwd_bwd, bit for bit. */
size_t dlm_sh2signal_mse_static_scratch_bytes(void);
dlm_status dlm_sh2signal_mse_fwd_bwd_noalloc(const dlm_sh_plan *plan, const float *c, const float *target, int64_t V,
                                             float *loss, float *dc, float *xhat, dlm_precision prec, void *stream);

/* Signal2SH straight from raw acquisitions, with the b=0 normalisation the
 * layer requires of its input (Sec. 2.2) fused into the load:
 *   c[v][s][:] = P_s (raw[v][dw volumes of shell s] / mean_b0(raw[v]))
 * raw device [V][n] in the creation table's volume order (n = the table
 * size given to dlm_sh_plan_create, b0 volumes included); the plan must have
 * at least one b0 volume (DLM_EINVAL otherwise).  ws: device workspace of at
 * least dlm_signal2sh_raw_workspace_bytes(V) bytes (per-voxel 1/mean_b0). */
size_t dlm_signal2sh_raw_workspace_bytes(int64_t V);
dlm_status dlm_signal2sh_fwd_raw(const dlm_sh_plan *plan, const float *raw, float *c, int64_t V, void *ws,
                                 size_t ws_bytes, dlm_precision prec, void *stream);

/* ------------------------------------------------------------------------
 * Local spherical convolution (Sec. 2.3, multi-b-value form Sec. 2.3.1)
 * ------------------------------------------------------------------------ */
typedef struct dlm_lsc_plan dlm_lsc_plan;

/* How an LSC call evaluates the layer.  Both forms compute the same linear
 * map (up to float rounding order):
 *  DLM_LSC_RESAMPLE -- the paper's order (Sec. 2.3, Fig. 4): resample the
 *    neighbourhood matrices X into the workspace, row-dot them with the
 *    cyclic kernel, refit.  Workspace grows with the voxels per pass.
 *  DLM_LSC_FOLDED -- by linearity of resample, row dot and refit, the layer
 *    is a_out[o] = sum_c T_oc a_in[c] + bias[o] P_m 1 with
 *    T_oc = sum_t W[o][c][t] (P_m B_t), B_t the resampling rows of tap t;
 *    the small (P_m B_t) tables are built in float64 with the plan, T is
 *    formed on the device from W on every call, and the layer is one matrix
 *    product over voxels.  Workspace is independent of V. */
typedef enum { DLM_LSC_RESAMPLE = 0, DLM_LSC_FOLDED = 1 } dlm_lsc_form;

/* Geometry of one LSC layer: m sampled directions (sampled_gradients host
 * [m][3]), input order sh_order_in, output order sh_order_out, cyclic
 * kernel rings kernel_sizes[n_rings] (points per ring), outer-ring angular
 * distance (radians), refit penalty lb_lambda.  Builds in float64 and
 * uploads: the resampling basis B_nb [m*T][K_in] (SH interpolation at every
 * kernel point) and the refit P_m [K_out][m]. */
dlm_status dlm_lsc_plan_create(const double *sampled_gradients, int64_t m, int sh_order_in,
                               int sh_order_out, const int *kernel_sizes, int n_rings,
                               double angular_distance, double lb_lambda, dlm_lsc_plan **out);
/* T = kernel taps, K_in, K_out, m (any may be NULL). */
dlm_status dlm_lsc_plan_info(const dlm_lsc_plan *plan, int *T, int *K_in, int *K_out, int64_t *m);
/* Host float64 tables: points [m][T][3], B_nb [m*T][K_in], P_m [K_out][m]
 * (any may be NULL). */
dlm_status dlm_lsc_plan_tables(const dlm_lsc_plan *plan, double *points, double *B_nb, double *P_m);
void dlm_lsc_plan_destroy(dlm_lsc_plan *plan);

/* Workspace bytes that dlm_lsc_fwd / dlm_lsc_bwd need for C input and O
 * output channels.  DLM_LSC_RESAMPLE: for `V_chunk` voxels per pass; a call
 * given fewer bytes than needed for its V processes the voxels in several
 * passes, the minimum being one 64-voxel pass (less -> DLM_EWORKSPACE).
 * DLM_LSC_FOLDED: independent of V_chunk. */
dlm_status dlm_lsc_workspace_bytes(const dlm_lsc_plan *plan, int C, int O, int64_t V_chunk,
                                   dlm_lsc_form form, dlm_precision prec, size_t *bytes);

/* LSC forward in the paper's order (Sec. 2.3, Fig. 4):
 *   X[v][c][i*T+t] = sum_j B_nb[i*T+t][j] a_in[v][c][j]   (neighbourhood resampling)
 *   y[v][o][i]     = bias[o] + sum_c sum_t W[o][c][t] X[v][c][i*T+t]
 *                    (kernel row dot, a cross-correlation; channels = b-values)
 *   a_out[v][o][:] = P_m y[v][o][:]                        (refit)
 *   optional ReLU: a_out = max(a_out, 0) when fuse_relu != 0.
 * a_in device [V][C][K_in]; W device [O][C][T]; bias device [O] or NULL;
 * a_out device [V][O][K_out]; ws device workspace of ws_bytes. */
dlm_status dlm_lsc_fwd(const dlm_lsc_plan *plan, const float *a_in, int C, const float *W,
                       const float *bias, int O, float *a_out, int64_t V, int fuse_relu,
                       dlm_lsc_form form, void *ws, size_t ws_bytes, dlm_precision prec, void *stream);

/* ReLU handling of dlm_lsc_bwd (bit flags, 0 = no ReLU):
 * DLM_RELU_OUT: this layer's forward fused a ReLU into a_out, and da_out is
 *   the gradient of the ReLU's output: it is masked by a_out > 0 (a_out is
 *   needed).
 * DLM_RELU_IN: a_in is the output of the previous layer's fused ReLU; da_in
 *   is written already masked by a_in > 0, i.e. as the gradient of that
 *   layer's pre-activation, so the previous layer's dlm_lsc_bwd is then
 *   called without DLM_RELU_OUT.  In a stack of layers this reads each ReLU
 *   mask once (in the epilogue that writes da_in) instead of twice. */
typedef enum { DLM_RELU_OUT = 1, DLM_RELU_IN = 2 } dlm_relu_flags;

/* Adjoint of dlm_lsc_fwd.  da_out device [V][O][K_out] is the gradient of the
 * layer output (masked by a_out > 0 under DLM_RELU_OUT, a_out device
 * [V][O][K_out] the forward's output).  Outputs (each may be NULL to skip):
 *   da_in device [V][C][K_in]   = B_nb^T (sum_o W dy),  dy = P_m^T da
 *                                 (times [a_in > 0] under DLM_RELU_IN)
 *   dW    device [O][C][T]      = sum_{v,i} dy[v][o][i] X[v][c][i*T+t] (overwritten)
 *   dbias device [O]            = sum_{v,i} dy[v][o][i]                (overwritten)
 * relu_flags: a combination of dlm_relu_flags (other bits: DLM_EINVAL).
 * Resample form: the neighbourhood matrices X are recomputed from a_in, not
 * stored.  Folded form: dW comes from dT_oc = sum_v da_out[v][o] a_in[v][c]^T
 * contracted with each tap's (P_m B_t). */
dlm_status dlm_lsc_bwd(const dlm_lsc_plan *plan, const float *a_in, int C, const float *W, int O,
                       const float *a_out, const float *da_out, float *da_in, float *dW, float *dbias,
                       int64_t V, int relu_flags, dlm_lsc_form form, void *ws, size_t ws_bytes,
                       dlm_precision prec, void *stream);

/* Storage of LSC activations in bfloat16 (bit flags, 0 = float32 as above).
 * Every BF16 contraction rounds its operands to bfloat16 (RNE) as it loads
 * them, so storing an activation rounded once instead changes no value the
 * contraction sees (a positive float32 below 2^-133 that rounds to zero
 * would flip a ReLU mask; nothing else differs) and halves its traffic:
 * DLM_IO_IN_BF16:  a_in (and da_in) are bfloat16;
 * DLM_IO_OUT_BF16: a_out (and da_out) are bfloat16.
 * Needs DLM_BF16, the folded form, rows of a multiple of 8 entries (C*K_in
 * for IN, O*K_out for OUT) and 16-byte aligned tensors (DLM_EINVAL
 * otherwise).  In the backward, DLM_RELU_OUT is not available with these
 * flags: the ReLU of a stacked layer is applied by the next layer's adjoint
 * (DLM_RELU_IN). */
typedef enum { DLM_IO_IN_BF16 = 1, DLM_IO_OUT_BF16 = 2 } dlm_io_flags;

/* ReLU bits: a stacked layer's ReLU needs, in the backward, only the sign
 * pattern of its output, one bit per element instead of the 2- or 4-byte
 * activation.  relu_bits is a device array [V][N/16] of uint16, N the row
 * length (O*K_out in the forward, C*K_in in the backward, a multiple of 16);
 * bit (n mod 16) of word [v][n/16] is 1 iff the stored activation a[v][n] is
 * > 0 (after its bfloat16 rounding when stored in bfloat16).  Caller-owned,
 * written whole by the forward, read by the backward; NULL = not used.
 * Needs the folded form (DLM_EINVAL otherwise). */

/* dlm_lsc_fwd with activation storage chosen by io_flags (void pointers to
 * float32 or bfloat16 data as the flags say); io_flags = 0 is dlm_lsc_fwd.
 * relu_bits (NULL or as above, needs fuse_relu) receives the output's ReLU
 * bits beside a_out. */
dlm_status dlm_lsc_fwd_io(const dlm_lsc_plan *plan, const void *a_in, int C, const float *W,
                          const float *bias, int O, void *a_out, int64_t V, int fuse_relu,
                          int io_flags, uint16_t *relu_bits, dlm_lsc_form form, void *ws,
                          size_t ws_bytes, dlm_precision prec, void *stream);
/* dlm_lsc_bwd with activation storage chosen by io_flags; dW and dbias stay
 * float32.  io_flags = 0 and relu_bits = NULL is dlm_lsc_bwd.  relu_bits
 * (NULL or as above, needs DLM_RELU_IN, excludes DLM_RELU_OUT) replaces
 * a_in as the source of the DLM_RELU_IN mask, with identical results; a_in
 * is still read for dW. */
dlm_status dlm_lsc_bwd_io(const dlm_lsc_plan *plan, const void *a_in, int C, const float *W, int O,
                          const void *a_out, const void *da_out, void *da_in, float *dW, float *dbias,
                          int64_t V, int relu_flags, int io_flags, const uint16_t *relu_bits,
                          dlm_lsc_form form, void *ws, size_t ws_bytes, dlm_precision prec,
                          void *stream);

/* ------------------------------------------------------------------------
 * Training helpers (q-space loss, Sec. 1; optimiser)
 * ------------------------------------------------------------------------ */

/* Bytes of workspace dlm_mse_fwd_bwd needs for n elements. */
size_t dlm_mse_workspace_bytes(int64_t n);
/* loss (device scalar) = mean((pred - target)^2) over n elements;
 * dpred device [n] = 2 (pred - target) / n (NULL to skip). */
dlm_status dlm_mse_fwd_bwd(const float *pred, const float *target, int64_t n, float *loss, float *dpred,
                           void *ws, size_t ws_bytes, void *stream);

/* A relative q-space loss (Sec. 1: once back in q-space, losses that
 * measure the error relative to the signal become usable): loss (device
 * scalar) = mean(((pred - target) / (|target| + eps))^2) over n elements;
 * dpred = 2 (pred - target) / ((|target| + eps)^2 n) (NULL to skip).
 * eps >= 0 guards near-zero targets.  Workspace as dlm_mse_fwd_bwd. */
dlm_status dlm_relmse_fwd_bwd(const float *pred, const float *target, int64_t n, float eps, float *loss,
                              float *dpred, void *ws, size_t ws_bytes, void *stream);

/* One Adam step on n parameters (device w, g, m, v), bias-corrected with the
 * 1-based step count. */
dlm_status dlm_adam_step(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int64_t step, void *stream);

/* ------------------------------------------------------------------------
 * Measurement support (not part of the layers)
 * ------------------------------------------------------------------------
 * While enabled, every kernel the library launches is bracketed by a pair of
 * HIP events recorded on its launch stream and filed under an operation tag
 * ("lsc_resample", "signal2sh_fwd", ...) together with the algorithmic bytes
 * and flops of that launch (input + output bytes and multiply-adds x 2 of the
 * operation as defined, excluding padding and workspace re-reads).
 * dlm_timing_count waits for every recorded event and returns the number of
 * tags; dlm_timing_entry reads tag i (tag copied into a caller buffer of
 * tag_len bytes).  Event recording adds small gaps between kernels, so time
 * whole steps with timing disabled. */
dlm_status dlm_timing_enable(int on);
dlm_status dlm_timing_reset(void);
int dlm_timing_count(void);
dlm_status dlm_timing_entry(int i, char *tag, size_t tag_len, double *total_ms, int64_t *launches,
                            double *alg_bytes, double *alg_flops);

/* Reference kernels for the roofline, measured on the same GPU as the
 * layers (the rates a streaming kernel and the matrix cores deliver there,
 * next to the spec-sheet peaks).
 * dlm_peak_copy: device-to-device copy of `bytes` (a multiple of 4; both
 * buffers 16-byte aligned, not overlapping); it moves 2 * bytes through
 * HBM.  dlm_peak_mfma: `blocks` workgroups of four waves each run `iters`
 * rounds of independent MFMAs (sixteen v_mfma_f32_16x16x4_f32 for DLM_FP32,
 * eight v_mfma_f32_32x32x16_bf16 for DLM_BF16) and write one float per lane to
 * out (device, dlm_peak_mfma_out_floats(blocks) floats); the work done is
 * dlm_peak_mfma_flops(prec, blocks, iters) flops. */
dlm_status dlm_peak_copy(const void *src, void *dst, size_t bytes, void *stream);
size_t dlm_peak_mfma_out_floats(int blocks);
double dlm_peak_mfma_flops(dlm_precision prec, int blocks, int iters);
dlm_status dlm_peak_mfma(dlm_precision prec, int blocks, int iters, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DELIMIT_H */
