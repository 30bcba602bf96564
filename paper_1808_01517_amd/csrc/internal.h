// Internal declarations of libdelimit (not part of the public ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/delimit.h"

namespace dlm {

constexpr int kMaxShOrder = 16;
constexpr int kMaxChannels = 256;
constexpr int kMaxTaps = 256;

// ---------------------------------------------------------------- host fp64
int sh_num_coeffs(int L);
bool sh_order_ok(int L);
bool unit_dir(const double *in, double *out);
void sh_row(int L, const double *u, double *row);
void sh_basis_unit(int L, const double *u, int64_t n, double *B);
bool fit_from_basis(int L, const double *B, int64_t n, double lambda, double *P);
void group_shells(const double *bvals, int64_t n, double b0_max, double rel_tol,
                  std::vector<std::vector<int64_t>> &members, std::vector<double> &centres);
void kernel_points_unit(const double *g, int64_t m, const int *ks, int R, double alpha, double *pts);
uint16_t f32_to_bf16_rne(float f);
uint16_t f64_to_bf16_rne(double d);

// ------------------------------------------------------------ device tables
// A row-major matrix [rows][cols] uploaded once as float32 and bfloat16.
struct DevMat {
  int rows = 0, cols = 0;
  float *f32 = nullptr;
  uint16_t *bf16 = nullptr;
};

// ------------------------------------------------------------------ kernels
// Every operation gets its own kernel symbol (template argument) so that
// profilers report each one separately.
enum KernelOp : int {
  kOpS2shFwd = 0,
  kOpS2shBwd,
  kOpSh2sFwd,
  kOpSh2sBwd,
  kOpResample,
  kOpResampleBwd,
  kOpRefit,
  kOpRefitBwd,
  kOpContractFwd,
  kOpContractBwdData,
  kOpContractBwdWeight,
  kOpFoldMake,
  kOpFoldFwd,
  kOpFoldBwdData,
  kOpFoldGrad,
  kOpS2shRaw,
};

// C[r][n] = sum_k A[r][k] * B[n][k] over one group g:
//   A row r of group g at A + r*lda + g*a_gs, mask (same indexing) optional:
//     A is replaced by A * (mask > 0);
//   B (float32 or bf16 table, [N][K] row-major) at B + g*b_gs;
//   C at C + r*ldc + g*c_gs, plus bias_n[n] if given, optional ReLU.
struct TableGemm {
  const float *A = nullptr;
  const float *mask = nullptr;
  int64_t lda = 0, a_gs = 0;
  const float *Bf = nullptr;
  const uint16_t *Bh = nullptr;
  int64_t b_gs = 0;
  int64_t ldb_f = 0;  // row stride of the float32 table (0: K)
  int64_t ldb_h = 0;  // row stride of the bfloat16 table (0: K)
  float *C = nullptr;
  const float *bias_n = nullptr;
  const float *out_mask = nullptr;  // C zeroed where out_mask (indexed as C) <= 0
  int64_t ldc = 0, c_gs = 0;
  int64_t M = 0;
  int N = 0, K = 0, groups = 1;
  int relu = 0;
  KernelOp op = kOpS2shFwd;
  // bfloat16 activations (BF16, streaming core only): A as Ah, C as Ch, the
  // output mask as out_mask_h (with Ch); the float32 pointer is then null
  const uint16_t *Ah = nullptr;
  uint16_t *Ch = nullptr;
  const uint16_t *out_mask_h = nullptr;
  // ReLU bit masks (streaming core; N a multiple of 16): the forward writes
  // bit (output > 0) of every output, one uint16 per 16 columns
  // ([M][N / 16]); the input gradient masks by them instead of out_mask
  uint16_t *relu_bits_out = nullptr;
  const uint16_t *relu_bits_in = nullptr;
};
int launch_table_gemm(const TableGemm &g, dlm_precision prec, void *stream);

// Streaming core (operands DMA'd into an LDS ring).  Table form: one group,
// no operand mask, the precision's table (float32 Bf / bfloat16 Bh) with row
// stride ldb_f / ldb_h a multiple of 32 and zeros in columns K .. stride-1.
bool stream_table_ok(const TableGemm &g, dlm_precision prec);
int launch_stream_table(const TableGemm &g, dlm_precision prec, void *stream);
// Weight-gradient form of launch_lsc_fold_grad (no mask), ksplit a multiple of 32.
// whether launch_stream_grad takes these sizes (ksplit: voxels per split)
bool stream_grad_ok(int M, int CK, int ksplit);
// g / a as float32, or (BF16 only) as bfloat16 gh / ah (M, CK multiples of 8,
// 16-byte aligned); the other pointer of each pair is null.
bool stream_grad_bf16_ok(const uint16_t *gh, const uint16_t *ah, int M, int CK);
int launch_stream_grad(const float *g, const uint16_t *gh, const float *a, const uint16_t *ah, int64_t V, int M,
                       int CK, int splits, int ksplit, float *partial, dlm_precision prec, void *stream);
// Per-shell SH contraction, one wave per 16 voxels x one shell (groups
// shells of equal size in one launch):
//   C[v][g*c_gs + n] = sum_k A[v][g*a_gs + k] * Bt_g[n][k],  n < ncol, k < nred
// with Bt_g given in MFMA fragment order (shell_frag_tables), frag_gs_* the
// per-shell stride of the fragment tables in bytes.  nred <= 128.
struct ShellGemm {
  const float *A = nullptr;
  int64_t lda = 0, a_gs = 0;
  float *C = nullptr;
  int64_t ldc = 0, c_gs = 0;
  const float *frag_f = nullptr;
  const uint16_t *frag_h = nullptr;
  int64_t frag_gs_f = 0, frag_gs_h = 0;
  int ncol = 0, nred = 0, groups = 1;
  int64_t V = 0;
  KernelOp op = kOpS2shFwd;
};
bool shell_gemm_ok(int ncol, int nred);
int launch_shell_gemm(const ShellGemm &g, dlm_precision prec, void *stream);
// Whether launch_shell_gemm runs g (a Signal2SH contraction) in the
// table-resident FP32 form: FP32, nred <= 128 and a batch large enough.
bool shell_s2sh_resident(const ShellGemm &g, dlm_precision prec);
// BF16 reduction over 65..96 directions on a batch large enough for the
// per-shell kernel's two-block waves (otherwise the tiled core runs it)
bool shell_long_bf16(const ShellGemm &t, dlm_precision prec);
size_t shell_frag_floats(int ncol, int nred);
size_t shell_frag_halves(int ncol, int nred);
void shell_frag_tables(const double *t, int ncol, int nred, float *f, uint16_t *h);
// bf16 fragment table of Bt [ncol][nred] with the reduction index in the
// accumulator order of sh2s_mse_kernel's second contraction
void shell_frag_halves_acc(const double *t, int ncol, int nred, uint16_t *h);

// Fused SH2Signal -> MSE -> SH2Signal adjoint over `groups` shells of N
// directions each (c [V][ldcoef], shell g at g*K; target/xhat [V][ldsig],
// shell g at g*N).  fragB_*: fragment tables of B [N][K]; fragBt_f: of
// B^T [K][N]; fragBt_h: shell_frag_halves_acc of B^T.  gs*: per-shell
// strides in bytes.  Writes one squared-error sum per wave to partials
// (sh2s_mse_partials of them), dc = B^T (scale (x^ - target)), and x^ when
// xhat is not null.
struct Sh2sMse {
  const float *c = nullptr;
  int64_t ldcoef = 0;
  int K = 0;
  const float *target = nullptr;
  int64_t ldsig = 0;
  int N = 0;
  float *dc = nullptr, *xhat = nullptr;
  const float *fragB_f = nullptr, *fragBt_f = nullptr;
  const uint16_t *fragB_h = nullptr, *fragBt_h = nullptr;
  int64_t gsB_f = 0, gsBt_f = 0, gsB_h = 0, gsBt_h = 0;
  int groups = 1;
  int64_t V = 0;
  float scale = 0.0f;
  float *partials = nullptr;
};
bool sh2s_mse_ok(int N, int K);
int64_t sh2s_mse_partials(int64_t V, int groups);
int launch_sh2s_mse(const Sh2sMse &t, dlm_precision prec, void *stream);
// *out = scale * sum(partials[0..n)) in a fixed summation order; beyond 4096
// partials, two passes through scratch[kSumBlocks]
constexpr int kSumBlocks = 256;
int launch_sum_scaled(const float *partials, int64_t n, float *out, float scale, float *scratch, void *stream);

// fill `bytes` (a multiple of 4) at p with zeros
int launch_zero(void *p, size_t bytes, void *stream);
// zero bytes [c0_bytes, ld_bytes) of each of `rows` rows ld_bytes apart (even sizes)
int launch_zero_cols(void *p, int64_t rows, int64_t c0_bytes, int64_t ld_bytes, void *stream);

// y[v][o][i] = bias[o] + sum_{c,t} W[o][c][t] X[v][c][i*T+t]
int launch_lsc_contract_fwd(const float *X, const float *W, const uint16_t *Wh, const float *bias, float *y,
                            int64_t V, int C, int O, int m, int T, dlm_precision prec, void *stream);
// dX[v][c][i*T+t] = sum_o W[o][c][t] dy[v][o][i]   (Wt = W transposed [C*T][O])
int launch_lsc_contract_bwd_data(const float *dy, const float *Wt, const uint16_t *Wth, float *dX, int64_t V,
                                 int C, int O, int m, int T, dlm_precision prec, void *stream);
// partial[s][(c*T+t)][o] and partial[s][C*T][o] (bias row) over voxel split s.
int launch_lsc_contract_bwd_weight(const float *X, const float *dy, float *partial, int64_t V, int C, int O, int m,
                                   int T, int splits, dlm_precision prec, void *stream);
// dW[o][c][t] (+)= sum_s partial[s][c*T+t][o]; db[o] (+)= sum_s partial[s][C*T][o]
int launch_reduce_weight_partials(const float *partial, int splits, float *dW, float *db, int C, int O, int T,
                                  int accumulate, void *stream);
// Wt[(c*T+t)][o] = W[o][c][t] (+ bf16 copies of W and Wt when requested)
int launch_prepare_weights(const float *W, float *Wt, uint16_t *Wh, uint16_t *Wth, int C, int O, int T,
                           void *stream);
int launch_mse(const float *pred, const float *target, int64_t n, float *loss, float *dpred, float *partials,
               int nblocks, void *stream);
// relative form: errors weighted by 1 / (|target| + eps)
int launch_relmse(const float *pred, const float *target, int64_t n, float eps, float *loss, float *dpred,
                  float *partials, int nblocks, void *stream);
// inv[v] = n_b0 / sum_i raw[v*ld + b0idx[i]]
int launch_b0_inverse_mean(const float *raw, int64_t ld, const int32_t *b0idx, int nb0, int64_t V, float *inv,
                           void *stream);
// Signal2SH on raw data: A(r, k) = raw[r*ld + dwidx[g*N + k]] * inv[r] for group (shell) g
int launch_s2sh_raw(const float *raw, int64_t ld, const int32_t *dwidx, const float *inv, const float *Pf,
                    const uint16_t *Ph, float *c, int64_t ldc, int64_t V, int S, int N, int K, dlm_precision prec,
                    void *stream);
int mse_blocks(int64_t n);
int launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, void *stream);

// ----------------------------------------------------- folded LSC form
// Tw[(o*Ko+k)][(c*Ki+j)] = sum_t W[o][c][t] Q[t][k][j]  (and the transpose
// TwT[(c*Ki+j)][(o*Ko+k)]), float32 always, bfloat16 copies when non-null;
// rows of Tw / Twh have stride ld, rows of TwT / TwTh stride ldt.
int launch_lsc_fold(const float *W, const float *Q, int C, int O, int T, int Ki, int Ko, float *Tw, float *TwT,
                    uint16_t *Twh, uint16_t *TwTh, int64_t ld, int64_t ldt, void *stream);
int fold_grad_split_len(int64_t V, int splits);
// bvec[o*Ko+k] = bias[o] * pm1[k]  (zero when bias is null)
int launch_lsc_bias_vec(const float *bias, const float *pm1, int O, int Ko, float *bvec, void *stream);
// partial[s][m][n] over voxel slice s: m = (o,k) of g = da_out (masked by
// a_out > 0 when mask != null), n = (c,j) of a_in plus one ones-column.
int launch_lsc_fold_grad(const float *da_out, const float *mask, const float *a_in, int64_t V, int M, int CK,
                         int splits, float *partial, dlm_precision prec, void *stream);
int fold_grad_splits(int64_t V, int M, int N1);
// out[i] = sum_s part[s*n + i]
int launch_sum_partials(const float *part, int splits, int64_t n, float *out, void *stream);
// dW[(o*C+c)][t] = sum_{k,j} dTw[(o*Ko+k)][c*Ki+j] Q[t][k][j];  db[o] = sum_k dTw[(o*Ko+k)][C*Ki] pm1[k]
int launch_lsc_unfold(const float *dTw, const float *Q, const float *pm1, int C, int O, int T, int Ki, int Ko,
                      float *dW, float *db, void *stream);

// ----------------------------------------------------------- status text
// Set the thread's dlm_last_error() text and return s (for library sources
// other than the C ABI file).
dlm_status report(dlm_status s, const char *fmt, ...);

// ------------------------------------------------------- timing support
// When enabled, TimedScope brackets a launch with a HIP event pair on its
// stream and files it under `tag` with its algorithmic bytes and flops.
void timing_begin(const char *tag, void *stream);
void timing_end(void *stream, double alg_bytes, double alg_flops);
bool timing_on();

struct TimedScope {
  void *st;
  double bytes, flops;
  bool on;
  TimedScope(const char *tag, void *stream, double b, double f) : st(stream), bytes(b), flops(f), on(timing_on()) {
    if (on) timing_begin(tag, st);
  }
  ~TimedScope() {
    if (on) timing_end(st, bytes, flops);
  }
};

}  // namespace dlm
