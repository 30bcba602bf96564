// Per-shell SH contractions (Sec. 2.2: Signal2SH c = P_s x, SH2Signal
// x = B_s c, and their adjoints) for one MI355X, and the q-space loss head
// that fuses SH2Signal, the MSE and the SH2Signal adjoint (sh2s_mse_kernel).
//
// Each is, per voxel v and shell g,
//   C[v][g*c_gs + n] = sum_k A[v][g*a_gs + k] * Bt_g[n][k],   n < ncol, k < nred,
// with ncol, nred <= 96 for the workloads here (K = 45 coefficients, 90
// directions per shell).  Such a contraction is a stream: 15 flop per byte
// against a bf16 ridge near 300, so the design keeps the loads flowing and
// nothing else in the way:
// * one wave computes 16 voxels x one shell (BF16 contractions over the
//   coefficients: two such blocks of the same shell, sharing each table
//   fragment); its A fragments are loaded straight from HBM into registers
//   (16-byte loads along the voxel's row, all issued before the first
//   MFMA), so there is no LDS staging and no barrier, and many resident
//   waves hide the latency;
// * the table Bt_g arrives pre-arranged on the host in MFMA fragment order,
//   one 16-byte load per lane per fragment (it stays in L1/L2).  The FP32
//   loss head on large batches runs as persistent 1024-thread blocks that
//   first copy every shell's two fragment tables into LDS and then loop
//   over wave items: its waves re-read ~36 KB of tables per 16 voxels x
//   shell, more than 3x the voxels' own HBM traffic, and from L1/L2 that
//   bound the FP32 MFMAs (1.00 -> 0.70 ms on the three-shell batch).  The
//   same resident form measured slower for the BF16 head and for the
//   contractions over the coefficients, which are bound by memory latency
//   instead, so those keep the short blocks.  FP32 Signal2SH (the
//   reduction over a shell's directions) gains from it when each wave
//   also fetches its next item's rows ahead (0.575 -> 0.528 ms); it runs
//   on the tiled core otherwise;
// * BF16: v_mfma_f32_16x16x32_bf16, lane (q16, g4) holds k = 32 s + 8 g4 .. + 7;
//   FP32: v_mfma_f32_16x16x4_f32 over 16-k groups, lane (q16, g4) holds
//   k = 16 h + 4 g4 .. + 3 and MFMA e takes k = 16 h + 4 g4 + e;
// * the B fragment goes first, so each accumulator is the transposed 16 x 16
//   tile and a lane stores four consecutive columns of one voxel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "gemm_common.h"
#include "internal.h"

namespace dlm {
namespace shellk {

constexpr int kMaxRed = 128;  // reduction length handled (FP32: 8 groups of 16, BF16: 4 steps of 32)
constexpr int kColChunk = 6;  // output tiles of 16 per pass over A (96 columns)

// 4 consecutive floats of row a from k, zero where k + e >= kend or the row is absent
__device__ __forceinline__ floatx4 load_run(const float *a, int k, int kend, bool row) {
  if (row && k + 3 < kend) return ld4(a + k);
  floatx4 v{0.f, 0.f, 0.f, 0.f};
  if (row)
    for (int e = 0; e < 4; ++e)
      if (k + e < kend) v[e] = a[k + e];
  return v;
}

template <int OP, bool F32, int MAXRED, int IT>
__global__ __launch_bounds__(256) void shell_gemm_kernel(const float *A, int64_t lda, int64_t a_gs, float *C,
                                                         int64_t ldc, int64_t c_gs, const void *frag,
                                                         int64_t frag_gs, int ncol, int nred, int groups, int64_t V,
                                                         int64_t nwaves) {
  // IT row blocks of 16 voxels of one shell per wave: every block's loads
  // are issued before the first MFMA and each table fragment serves all of
  // them.  MAXRED bounds the reduction (registers for A are sized by it).
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwaves) return;  // whole waves only; no barriers in this kernel
  const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
  const int64_t rb = w / groups;
  const int g = (int)(w - rb * groups);
  const float *a[IT];
  float *c[IT];
  bool row[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int64_t r = (rb * IT + it) * 16 + q16;
    row[it] = r < V;
    a[it] = A + r * lda + (int64_t)g * a_gs;
    c[it] = C + r * ldc + (int64_t)g * c_gs;
  }
  const int NT = (ncol + 15) / 16;
  auto store = [&](int it, int j0, int nt, const floatx4 (&acc)[kColChunk]) {
    if (!row[it]) return;
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      if (j >= nt) break;
      const int n = 16 * (j0 + j) + 4 * g4;
      if (n + 3 < ncol) __builtin_memcpy(c[it] + n, &acc[j], 16);
      else
        for (int e = 0; e < 4; ++e)
          if (n + e < ncol) c[it][n + e] = acc[j][e];
    }
  };
  if constexpr (F32) {
    constexpr int HM = MAXRED / 16;
    const int H = (nred + 15) / 16;
    const floatx4 *fr = reinterpret_cast<const floatx4 *>(frag) + (int64_t)g * frag_gs / 16;
    floatx4 av[IT][HM];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
      for (int h = 0; h < HM; ++h)
        av[it][h] = h < H ? load_run(a[it], 16 * h + 4 * g4, nred, row[it]) : floatx4{0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < NT; j0 += kColChunk) {
      const int nt = min(kColChunk, NT - j0);
      floatx4 acc[IT][kColChunk];
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int j = 0; j < kColChunk; ++j) acc[it][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int h = 0; h < HM; ++h) {
        if (h >= H) break;
#pragma unroll
        for (int j = 0; j < kColChunk; ++j) {
          if (j >= nt) break;
          const floatx4 b = fr[((int64_t)(j0 + j) * H + h) * 64 + lane];
#pragma unroll
          for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              acc[it][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], av[it][h][e], acc[it][j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) store(it, j0, nt, acc[it]);
    }
  } else {
    constexpr int SM = MAXRED / 32;
    const int S = (nred + 31) / 32;
    const bf16x8 *fr = reinterpret_cast<const bf16x8 *>(frag) + (int64_t)g * frag_gs / 16;
    floatx4 lo[IT][SM], hi[IT][SM];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        lo[it][s] = s < S ? load_run(a[it], 32 * s + 8 * g4, nred, row[it]) : floatx4{0.f, 0.f, 0.f, 0.f};
        hi[it][s] = s < S ? load_run(a[it], 32 * s + 8 * g4 + 4, nred, row[it]) : floatx4{0.f, 0.f, 0.f, 0.f};
      }
    bf16x8 av[IT][SM];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
      for (int s = 0; s < SM; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          av[it][s][e] = (__bf16)lo[it][s][e];
          av[it][s][4 + e] = (__bf16)hi[it][s][e];
        }
    for (int j0 = 0; j0 < NT; j0 += kColChunk) {
      const int nt = min(kColChunk, NT - j0);
      floatx4 acc[IT][kColChunk];
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int j = 0; j < kColChunk; ++j) acc[it][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        if (s >= S) break;
#pragma unroll
        for (int j = 0; j < kColChunk; ++j) {
          if (j >= nt) break;
          const bf16x8 b = fr[((int64_t)(j0 + j) * S + s) * 64 + lane];
#pragma unroll
          for (int it = 0; it < IT; ++it)
            acc[it][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, av[it][s], acc[it][j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) store(it, j0, nt, acc[it]);
    }
  }
}

// Reductions of at most 64 entries (every contraction over a shell's
// coefficients up to order 12) size A's registers for 64.  BF16 takes two
// row blocks per wave, FP32 one (measured on the three-shell Signal2SH
// adjoint at 1M voxels: BF16 0.448 -> 0.419 ms with two, 0.481 with one;
// FP32 0.559 -> 0.554 ms with one, 0.559 with two).
// DLM_SHELL_PAIRS=0 in the environment gives these BF16 contractions one
// 16-voxel block per wave instead of two (the same results bit for bit;
// read at every call, for tests).  The loss head keeps one block per wave:
// with two it measured 0.646 -> 0.869 ms.
inline bool bf16_pairs() {
  const char *e = std::getenv("DLM_SHELL_PAIRS");
  return !(e && e[0] == '0');
}

template <int OP, bool F32, int MAXRED, int IT>
int launch_op_t(const ShellGemm &t, const void *frag, int64_t frag_gs, hipStream_t st) {
  const int64_t nwaves = ((t.V + 15) / 16 + IT - 1) / IT * t.groups;
  const int64_t blocks = (nwaves + 3) / 4;
  if (blocks > 0x7fffffff) return -4;
  hipLaunchKernelGGL((shell_gemm_kernel<OP, F32, MAXRED, IT>), dim3((unsigned)blocks), dim3(256), 0, st, t.A, t.lda,
                     t.a_gs, t.C, t.ldc, t.c_gs, frag, frag_gs, t.ncol, t.nred, t.groups, t.V, nwaves);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int OP>
int launch_op(const ShellGemm &t, dlm_precision prec, hipStream_t st) {
  const bool bf = prec == DLM_BF16;
  const void *frag = bf ? (const void *)t.frag_h : (const void *)t.frag_f;
  const int64_t gs = bf ? t.frag_gs_h : t.frag_gs_f;
  if (t.nred <= 64) {
    if (bf) return bf16_pairs() ? launch_op_t<OP, false, 64, 2>(t, frag, gs, st)
                                : launch_op_t<OP, false, 64, 1>(t, frag, gs, st);
    return launch_op_t<OP, true, 64, 1>(t, frag, gs, st);
  }
  if (bf && t.nred <= 96)  // see shell_long_bf16
    return bf16_pairs() ? launch_op_t<OP, false, 96, 2>(t, frag, gs, st)
                        : launch_op_t<OP, false, 96, 1>(t, frag, gs, st);
  if (bf) return launch_op_t<OP, false, kMaxRed, 1>(t, frag, gs, st);
  return launch_op_t<OP, true, kMaxRed, 1>(t, frag, gs, st);
}

// SH2Signal -> q-space MSE -> SH2Signal adjoint for 16 voxels x one shell
// per wave (the tail of a training step, Sec. 1: the loss is taken back in
// q-space):
//   x^[n]  = sum_k B[n][k] c[k]                 (GEMM 1, n < N, k < K)
//   loss  += (x^[n] - t[n])^2                   (one partial per wave)
//   d[n]   = scale (x^[n] - t[n]),  scale = 2 / (V n_dw)
//   dc[k]  = sum_n B[n][k] d[n]                 (GEMM 2)
// GEMM 2 takes d straight from GEMM 1's accumulators: lane (q16, g4) holds
// d at n = 16 j + 4 g4 + e, which is exactly the FP32 fragment order of the
// 16-k groups (so the standard fragment table of B^T serves), and in BF16
// a 32-k step takes tiles 2s and 2s+1 (its table is built in that order,
// shell_frag_halves_acc).  N <= 96, K <= 64.
template <bool F32>
__global__ __launch_bounds__(256) void sh2s_mse_kernel(const float *c, int64_t ldcoef, int K, const float *tgt,
                                                       int64_t ldsig, int N, float *dc, float *xhat,
                                                       const void *fragB, const void *fragBt, int64_t gsB,
                                                       int64_t gsBt, int groups, int64_t V, int64_t nwaves,
                                                       float scale, float *partials) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwaves) return;  // whole waves only; no barriers in this kernel
  const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
  const int64_t rb = w / groups;
  const int g = (int)(w - rb * groups);
  const int64_t r = rb * 16 + q16;
  const bool row = r < V;
  const float *a = c + r * ldcoef + (int64_t)g * K;
  const float *t = tgt + r * ldsig + (int64_t)g * N;
  const int NT1 = (N + 15) / 16, NT2 = (K + 15) / 16;
  floatx4 acc[kColChunk], acc2[4];
#pragma unroll
  for (int j = 0; j < kColChunk; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 4; ++j) acc2[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // target values of this lane's accumulator positions, loaded up front
  floatx4 tv[kColChunk];
#pragma unroll
  for (int j = 0; j < kColChunk; ++j)
    tv[j] = j < NT1 ? load_run(t, 16 * j + 4 * g4, N, row) : floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (F32) {
    const floatx4 *f1 = reinterpret_cast<const floatx4 *>(fragB) + (int64_t)g * gsB / 16;
    const floatx4 *f2 = reinterpret_cast<const floatx4 *>(fragBt) + (int64_t)g * gsBt / 16;
    const int H = (K + 15) / 16;
    floatx4 av[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) av[h] = h < H ? load_run(a, 16 * h + 4 * g4, K, row) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if (h >= H) break;
#pragma unroll
      for (int j = 0; j < kColChunk; ++j) {
        if (j >= NT1) break;
        const floatx4 b = f1[((int64_t)j * H + h) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], av[h][e], acc[j], 0, 0, 0);
      }
    }
    float lsum = 0.0f;
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      if (j >= NT1) break;
      const int n = 16 * j + 4 * g4;
      if (xhat && row) {
        float *xo = xhat + r * ldsig + (int64_t)g * N;
        if (n + 3 < N) __builtin_memcpy(xo + n, &acc[j], 16);
        else
          for (int e = 0; e < 4; ++e)
            if (n + e < N) xo[n + e] = acc[j][e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float diff = row && n + e < N ? acc[j][e] - tv[j][e] : 0.0f;
        lsum += diff * diff;
        acc[j][e] = diff * scale;  // now d
      }
    }
    // GEMM 2 over n: group h of 16 n = accumulator tile h
#pragma unroll
    for (int h = 0; h < kColChunk; ++h) {
      if (h >= NT1) break;
#pragma unroll
      for (int j2 = 0; j2 < 4; ++j2) {
        if (j2 >= NT2) break;
        const floatx4 b = f2[((int64_t)j2 * NT1 + h) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc2[j2] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], acc[h][e], acc2[j2], 0, 0, 0);
      }
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) partials[w] = lsum;
  } else {
    const bf16x8 *f1 = reinterpret_cast<const bf16x8 *>(fragB) + (int64_t)g * gsB / 16;
    const bf16x8 *f2 = reinterpret_cast<const bf16x8 *>(fragBt) + (int64_t)g * gsBt / 16;
    const int S = (K + 31) / 32;
    bf16x8 av[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const floatx4 lo = s < S ? load_run(a, 32 * s + 8 * g4, K, row) : floatx4{0.f, 0.f, 0.f, 0.f};
      const floatx4 hi = s < S ? load_run(a, 32 * s + 8 * g4 + 4, K, row) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        av[s][e] = (__bf16)lo[e];
        av[s][4 + e] = (__bf16)hi[e];
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= S) break;
#pragma unroll
      for (int j = 0; j < kColChunk; ++j) {
        if (j >= NT1) break;
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f1[((int64_t)j * S + s) * 64 + lane], av[s], acc[j], 0, 0, 0);
      }
    }
    float lsum = 0.0f;
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      if (j >= NT1) break;
      const int n = 16 * j + 4 * g4;
      if (xhat && row) {
        float *xo = xhat + r * ldsig + (int64_t)g * N;
        if (n + 3 < N) __builtin_memcpy(xo + n, &acc[j], 16);
        else
          for (int e = 0; e < 4; ++e)
            if (n + e < N) xo[n + e] = acc[j][e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float diff = row && n + e < N ? acc[j][e] - tv[j][e] : 0.0f;
        lsum += diff * diff;
        acc[j][e] = diff * scale;
      }
    }
    // GEMM 2: a 32-n step s takes the lane's d of tiles 2s (slots 0-3) and 2s+1 (slots 4-7)
    const int S2 = (NT1 + 1) / 2;
#pragma unroll
    for (int s = 0; s < kColChunk / 2; ++s) {
      if (s >= S2) break;
      bf16x8 dv;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        dv[e] = (__bf16)acc[2 * s][e];
        dv[4 + e] = (__bf16)(2 * s + 1 < NT1 ? acc[2 * s + 1][e] : 0.0f);
      }
#pragma unroll
      for (int j2 = 0; j2 < 4; ++j2) {
        if (j2 >= NT2) break;
        acc2[j2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f2[((int64_t)j2 * S2 + s) * 64 + lane], dv, acc2[j2], 0, 0, 0);
      }
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) partials[w] = lsum;
  }
  if (row) {
    float *o = dc + r * ldcoef + (int64_t)g * K;
#pragma unroll
    for (int j2 = 0; j2 < 4; ++j2) {
      if (j2 >= NT2) break;
      const int k = 16 * j2 + 4 * g4;
      if (k + 3 < K) __builtin_memcpy(o + k, &acc2[j2], 16);
      else
        for (int e = 0; e < 4; ++e)
          if (k + e < K) o[k + e] = acc2[j2][e];
    }
  }
}


// One FP32 wave item of the loss head (w = rb * groups + g), the FP32 branch
// of sh2s_mse_kernel with the fragment tables in the block's LDS copy.
__device__ __forceinline__ void sh2s_mse_item_f32(const float *c, int64_t ldcoef, int K, const float *tgt,
                                                  int64_t ldsig, int N, float *dc, float *xhat, const char *fragB,
                                                  const char *fragBt, int64_t gsB, int64_t gsBt, int groups, int64_t V,
                                                  int64_t w, float scale, float *partials) {
  const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
  const int64_t rb = w / groups;
  const int g = (int)(w - rb * groups);
  const int64_t r = rb * 16 + q16;
  const bool row = r < V;
  const float *a = c + r * ldcoef + (int64_t)g * K;
  const float *t = tgt + r * ldsig + (int64_t)g * N;
  const int NT1 = (N + 15) / 16, NT2 = (K + 15) / 16;
  floatx4 acc[kColChunk], acc2[4];
#pragma unroll
  for (int j = 0; j < kColChunk; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < 4; ++j) acc2[j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // target values of this lane's accumulator positions, loaded up front
  floatx4 tv[kColChunk];
#pragma unroll
  for (int j = 0; j < kColChunk; ++j)
    tv[j] = j < NT1 ? load_run(t, 16 * j + 4 * g4, N, row) : floatx4{0.f, 0.f, 0.f, 0.f};
  {
    const floatx4 *f1 = reinterpret_cast<const floatx4 *>(fragB + (int64_t)g * gsB);
    const floatx4 *f2 = reinterpret_cast<const floatx4 *>(fragBt + (int64_t)g * gsBt);
    const int H = (K + 15) / 16;
    floatx4 av[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) av[h] = h < H ? load_run(a, 16 * h + 4 * g4, K, row) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      if (h >= H) break;
#pragma unroll
      for (int j = 0; j < kColChunk; ++j) {
        if (j >= NT1) break;
        const floatx4 b = f1[((int64_t)j * H + h) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], av[h][e], acc[j], 0, 0, 0);
      }
    }
    float lsum = 0.0f;
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      if (j >= NT1) break;
      const int n = 16 * j + 4 * g4;
      if (xhat && row) {
        float *xo = xhat + r * ldsig + (int64_t)g * N;
        if (n + 3 < N) __builtin_memcpy(xo + n, &acc[j], 16);
        else
          for (int e = 0; e < 4; ++e)
            if (n + e < N) xo[n + e] = acc[j][e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float diff = row && n + e < N ? acc[j][e] - tv[j][e] : 0.0f;
        lsum += diff * diff;
        acc[j][e] = diff * scale;  // now d
      }
    }
    // GEMM 2 over n: group h of 16 n = accumulator tile h
#pragma unroll
    for (int h = 0; h < kColChunk; ++h) {
      if (h >= NT1) break;
#pragma unroll
      for (int j2 = 0; j2 < 4; ++j2) {
        if (j2 >= NT2) break;
        const floatx4 b = f2[((int64_t)j2 * NT1 + h) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc2[j2] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], acc[h][e], acc2[j2], 0, 0, 0);
      }
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) partials[w] = lsum;
  }
  if (row) {
    float *o = dc + r * ldcoef + (int64_t)g * K;
#pragma unroll
    for (int j2 = 0; j2 < 4; ++j2) {
      if (j2 >= NT2) break;
      const int k = 16 * j2 + 4 * g4;
      if (k + 3 < K) __builtin_memcpy(o + k, &acc2[j2], 16);
      else
        for (int e = 0; e < 4; ++e)
          if (k + e < K) o[k + e] = acc2[j2][e];
    }
  }
}


// Table-resident form: kResWaves waves per block; the block copies the
// fragment tables (a multiple of 16 bytes) into LDS, then each wave takes
// items w = blockIdx.x * kResWaves + wave, stepping by the grid.
constexpr int kResWaves = 16;

__device__ __forceinline__ void copy_to_lds(char *dst, const void *src, int64_t bytes) {
  const uint4 *s4 = static_cast<const uint4 *>(src);
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  for (int64_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d4[i] = s4[i];
}

// Compute units of the current device (cached per device).
int device_cus() {
  static int cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (!cus[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cus[dev] = n;
  }
  return cus[dev];
}

// LDS the table-resident blocks may take, and the least number of wave
// items per block for them to pay (below it the short-block form runs).
constexpr int64_t kResLdsMax = 150 * 1024;
constexpr int64_t kResMinItems = 4 * kResWaves;

// Grid of the table-resident form for nwaves items and tab_bytes of tables:
// as many blocks as fit on every compute unit at once (registers and LDS
// decide), or 0 when the short-block form should run.
// DLM_SHELL_RESIDENT=0 in the environment (read at each launch) selects the
// short-block form everywhere, so that tests can compare the two.  The LDS
// limit and the occupancy query are done once per device, kernel and table
// size and then cached, so later launches make no such host calls.
struct ResFit {
  int dev = -1;
  const void *kernel = nullptr;
  int64_t bytes = 0;
  int per_cu = 0;  // 0: does not fit
};
struct ResLimit {  // the dynamic-LDS limit set for a kernel on a device: only ever raised
  int dev = -1;
  const void *kernel = nullptr;
  int64_t bytes = 0;
};

template <class KERNEL>
int res_grid(KERNEL kernel, int64_t nwaves, int64_t tab_bytes) {
  const char *env = std::getenv("DLM_SHELL_RESIDENT");
  if (env && env[0] == '0') return 0;
  if (tab_bytes > kResLdsMax || tab_bytes % 16 != 0) return 0;
  const int cus = device_cus();
  if (cus <= 0 || nwaves < kResMinItems * cus) return 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const void *k = reinterpret_cast<const void *>(kernel);
  static std::mutex mu;
  static ResFit fits[32];
  static ResLimit limits[16];
  static int nfits = 0, nlimits = 0;
  std::lock_guard<std::mutex> lk(mu);
  int per_cu = -1;
  for (int i = 0; i < nfits; ++i)
    if (fits[i].dev == dev && fits[i].kernel == k && fits[i].bytes == tab_bytes) per_cu = fits[i].per_cu;
  if (per_cu < 0) {
    if (nfits == 32) return 0;  // more table sizes than the cache holds: short blocks
    bool ok = true;
    if (tab_bytes > 64 * 1024) {
      int li = -1;
      for (int i = 0; i < nlimits; ++i)
        if (limits[i].dev == dev && limits[i].kernel == k) li = i;
      if (li < 0 && nlimits < 16) {
        li = nlimits++;
        limits[li] = ResLimit{dev, k, 64 * 1024};
      }
      if (li < 0) return 0;
      if (limits[li].bytes < tab_bytes) {
        ok = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tab_bytes) == hipSuccess;
        if (ok) limits[li].bytes = tab_bytes;
      }
    }
    per_cu = 0;
    if (ok && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * kResWaves, (size_t)tab_bytes) !=
                   hipSuccess ||
               per_cu < 0))
      per_cu = 0;
    if (!ok || per_cu == 0) (void)hipGetLastError();
    fits[nfits++] = ResFit{dev, k, tab_bytes, per_cu};
  }
  if (per_cu <= 0) return 0;
  if (nwaves < kResMinItems * cus * per_cu) per_cu = 1;
  return cus * per_cu;
}

// Table-resident FP32 loss head: both tables of every shell in LDS, B's
// first (groups * gsB bytes), then B^T's.
__global__ __launch_bounds__(1024) void sh2s_mse_res_kernel(const float *c, int64_t ldcoef, int K, const float *tgt,
                                                            int64_t ldsig, int N, float *dc, float *xhat,
                                                            const void *fragB, const void *fragBt, int64_t gsB,
                                                            int64_t gsBt, int groups, int64_t V, int64_t nwaves,
                                                            float scale, float *partials) {
  extern __shared__ __attribute__((aligned(16))) char tab[];
  copy_to_lds(tab, fragB, gsB * groups);
  copy_to_lds(tab + gsB * groups, fragBt, gsBt * groups);
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * kResWaves;
  for (int64_t w = (int64_t)blockIdx.x * kResWaves + (threadIdx.x >> 6); w < nwaves; w += step)
    sh2s_mse_item_f32(c, ldcoef, K, tgt, ldsig, N, dc, xhat, tab, tab + gsB * groups, gsB, gsBt, groups, V, w, scale,
                      partials);
}

// Table-resident FP32 Signal2SH, the reduction over a shell's directions
// (nred <= kMaxRed): persistent blocks as the resident loss head, and each
// wave keeps one item ahead, issuing the next item's A loads before this
// item's MFMAs.  The item arithmetic is shell_gemm_kernel's FP32 branch.
// Where this form does not apply Signal2SH runs on the tiled core, whose
// summation order differs: results agree to rounding, not bit for bit.
struct RowsF32 {
  floatx4 v[kMaxRed / 16];  // lane (q16, g4): k = 16 h + 4 g4 .. + 3 of its row
};

__device__ __forceinline__ void s2sh_load(RowsF32 &x, const float *A, int64_t lda, int64_t a_gs, int nred, int groups,
                                          int64_t V, int64_t w) {
  const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
  const int64_t rb = w / groups;
  const int g = (int)(w - rb * groups);
  const int64_t r = rb * 16 + q16;
  const float *a = A + r * lda + (int64_t)g * a_gs;
  const int H = (nred + 15) / 16;
#pragma unroll
  for (int h = 0; h < kMaxRed / 16; ++h)
    x.v[h] = h < H ? load_run(a, 16 * h + 4 * g4, nred, r < V) : floatx4{0.f, 0.f, 0.f, 0.f};
}

__device__ __forceinline__ void s2sh_compute(const RowsF32 &x, float *C, int64_t ldc, int64_t c_gs, const char *frag,
                                             int64_t frag_gs, int ncol, int nred, int groups, int64_t V, int64_t w) {
  const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
  const int64_t rb = w / groups;
  const int g = (int)(w - rb * groups);
  const int64_t r = rb * 16 + q16;
  float *c = C + r * ldc + (int64_t)g * c_gs;
  const int NT = (ncol + 15) / 16, H = (nred + 15) / 16;
  const floatx4 *fr = reinterpret_cast<const floatx4 *>(frag + (int64_t)g * frag_gs);
  for (int j0 = 0; j0 < NT; j0 += kColChunk) {
    const int nt = min(kColChunk, NT - j0);
    floatx4 acc[kColChunk];
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < kMaxRed / 16; ++h) {
      if (h >= H) break;
#pragma unroll
      for (int j = 0; j < kColChunk; ++j) {
        if (j >= nt) break;
        const floatx4 b = fr[((int64_t)(j0 + j) * H + h) * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[e], x.v[h][e], acc[j], 0, 0, 0);
      }
    }
    if (r < V) {
#pragma unroll
      for (int j = 0; j < kColChunk; ++j) {
        if (j >= nt) break;
        const int n = 16 * (j0 + j) + 4 * g4;
        if (n + 3 < ncol) __builtin_memcpy(c + n, &acc[j], 16);
        else
          for (int e = 0; e < 4; ++e)
            if (n + e < ncol) c[n + e] = acc[j][e];
      }
    }
  }
}

__global__ __launch_bounds__(1024) void s2sh_res_kernel(const float *A, int64_t lda, int64_t a_gs, float *C,
                                                        int64_t ldc, int64_t c_gs, const void *frag, int64_t frag_gs,
                                                        int ncol, int nred, int groups, int64_t V, int64_t nwaves) {
  extern __shared__ __attribute__((aligned(16))) char tab[];
  copy_to_lds(tab, frag, frag_gs * groups);
  __syncthreads();
  const int64_t step = (int64_t)gridDim.x * kResWaves;
  int64_t w = (int64_t)blockIdx.x * kResWaves + (threadIdx.x >> 6);
  if (w >= nwaves) return;  // no barrier follows
  RowsF32 cur;
  s2sh_load(cur, A, lda, a_gs, nred, groups, V, w);
  for (; w < nwaves; w += step) {
    RowsF32 nxt;
    if (w + step < nwaves) s2sh_load(nxt, A, lda, a_gs, nred, groups, V, w + step);
    s2sh_compute(cur, C, ldc, c_gs, tab, frag_gs, ncol, nred, groups, V, w);
    cur = nxt;
  }
}

// Grid of the resident FP32 Signal2SH for t, 0 when it does not apply.
int s2sh_res_grid(const ShellGemm &t) {
  const int64_t nwaves = (t.V + 15) / 16 * t.groups;
  return res_grid(s2sh_res_kernel, nwaves, t.frag_gs_f * t.groups);
}

}  // namespace shellk

bool shell_s2sh_resident(const ShellGemm &t, dlm_precision prec) {
  return prec != DLM_BF16 && t.op == kOpS2shFwd && shell_gemm_ok(t.ncol, t.nred) && t.V > 0 &&
         shellk::s2sh_res_grid(t) > 0;
}

bool sh2s_mse_ok(int N, int K) { return N > 0 && N <= 16 * shellk::kColChunk && K > 0 && K <= 64; }

int64_t sh2s_mse_partials(int64_t V, int groups) { return (V + 15) / 16 * groups; }

int launch_sh2s_mse(const Sh2sMse &t, dlm_precision prec, void *stream) {
  if (!sh2s_mse_ok(t.N, t.K)) return -3;
  if (t.V <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nwaves = sh2s_mse_partials(t.V, t.groups);
  const int64_t blocks = (nwaves + 3) / 4;
  if (blocks > 0x7fffffff) return -4;
  if (prec == DLM_BF16) {
    hipLaunchKernelGGL((shellk::sh2s_mse_kernel<false>), dim3((unsigned)blocks), dim3(256), 0, st, t.c, t.ldcoef, t.K,
                       t.target, t.ldsig, t.N, t.dc, t.xhat, (const void *)t.fragB_h, (const void *)t.fragBt_h,
                       t.gsB_h, t.gsBt_h, t.groups, t.V, nwaves, t.scale, t.partials);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const int64_t tab = (t.gsB_f + t.gsBt_f) * t.groups;
  const int grid = shellk::res_grid(shellk::sh2s_mse_res_kernel, nwaves, tab);
  if (grid > 0)
    hipLaunchKernelGGL((shellk::sh2s_mse_res_kernel), dim3(grid), dim3(64 * shellk::kResWaves), tab, st, t.c,
                       t.ldcoef, t.K, t.target, t.ldsig, t.N, t.dc, t.xhat, (const void *)t.fragB_f,
                       (const void *)t.fragBt_f, t.gsB_f, t.gsBt_f, t.groups, t.V, nwaves, t.scale, t.partials);
  else
    hipLaunchKernelGGL((shellk::sh2s_mse_kernel<true>), dim3((unsigned)blocks), dim3(256), 0, st, t.c, t.ldcoef, t.K,
                       t.target, t.ldsig, t.N, t.dc, t.xhat, (const void *)t.fragB_f, (const void *)t.fragBt_f,
                       t.gsB_f, t.gsBt_f, t.groups, t.V, nwaves, t.scale, t.partials);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool shell_gemm_ok(int ncol, int nred) { return ncol > 0 && nred > 0 && nred <= shellk::kMaxRed; }

// BF16 reductions over 65..96 directions run here with two voxel blocks per
// wave once the batch gives at least 4096 such waves (16 per CU): three-shell
// Signal2SH at 1M voxels 0.488 -> 0.432 ms against the tiled core, which
// keeps smaller batches (it has 64-voxel tiles).
bool shell_long_bf16(const ShellGemm &t, dlm_precision prec) {
  if (prec != DLM_BF16 || t.nred <= 64 || t.nred > 96 || t.V <= 0) return false;
  return ((t.V + 15) / 16 + 1) / 2 * t.groups >= 4096;
}

int launch_shell_gemm(const ShellGemm &t, dlm_precision prec, void *stream) {
  if (!shell_gemm_ok(t.ncol, t.nred)) return -3;
  if (t.V <= 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  switch (t.op) {
    case kOpS2shFwd:
      if (shell_s2sh_resident(t, prec)) {
        const int grid = shellk::s2sh_res_grid(t);
        const int64_t nwaves = (t.V + 15) / 16 * t.groups;
        hipLaunchKernelGGL(shellk::s2sh_res_kernel, dim3(grid), dim3(64 * shellk::kResWaves), t.frag_gs_f * t.groups,
                           st, t.A, t.lda, t.a_gs, t.C, t.ldc, t.c_gs, (const void *)t.frag_f, t.frag_gs_f, t.ncol,
                           t.nred, t.groups, t.V, nwaves);
        return hipGetLastError() == hipSuccess ? 0 : -1;
      }
      return shellk::launch_op<kOpS2shFwd>(t, prec, st);
    case kOpS2shBwd: return shellk::launch_op<kOpS2shBwd>(t, prec, st);
    case kOpSh2sFwd: return shellk::launch_op<kOpSh2sFwd>(t, prec, st);
    case kOpSh2sBwd: return shellk::launch_op<kOpSh2sBwd>(t, prec, st);
    default: return -3;
  }
}

// Fragment order of a [ncol][nred] table: float32 entry ((j*H + h)*64 + lane)*4 + e
// holds Bt[16 j + lane % 16][16 h + 4 (lane / 16) + e]; bfloat16 entry
// ((j*S + s)*64 + lane)*8 + e holds Bt[16 j + lane % 16][32 s + 8 (lane / 16) + e];
// zero outside the table.
size_t shell_frag_floats(int ncol, int nred) { return size_t((ncol + 15) / 16) * ((nred + 15) / 16) * 256; }
size_t shell_frag_halves(int ncol, int nred) { return size_t((ncol + 15) / 16) * ((nred + 31) / 32) * 512; }

void shell_frag_tables(const double *t, int ncol, int nred, float *f, uint16_t *h) {
  const int NT = (ncol + 15) / 16, H = (nred + 15) / 16, S = (nred + 31) / 32;
  for (int j = 0; j < NT; ++j)
    for (int lane = 0; lane < 64; ++lane) {
      const int col = 16 * j + (lane & 15), g4 = lane >> 4;
      for (int hh = 0; hh < H; ++hh)
        for (int e = 0; e < 4; ++e) {
          const int red = 16 * hh + 4 * g4 + e;
          f[((size_t(j) * H + hh) * 64 + lane) * 4 + e] =
              col < ncol && red < nred ? float(t[size_t(col) * nred + red]) : 0.0f;
        }
      for (int s = 0; s < S; ++s)
        for (int e = 0; e < 8; ++e) {
          const int red = 32 * s + 8 * g4 + e;
          h[((size_t(j) * S + s) * 64 + lane) * 8 + e] =
              col < ncol && red < nred ? f64_to_bf16_rne(t[size_t(col) * nred + red]) : uint16_t(0);
        }
    }
}

// bfloat16 table in the accumulator order of the fused loss head: entry
// ((j*S + s)*64 + lane)*8 + e holds Bt[16 j + lane % 16][n(s, e)] with
// n = 32 s + 4 (lane / 16) + e for e < 4 and 32 s + 16 + 4 (lane / 16) + e - 4
// for e >= 4 (zero outside).  Same size as shell_frag_halves.
void shell_frag_halves_acc(const double *t, int ncol, int nred, uint16_t *h) {
  const int NT = (ncol + 15) / 16, S = (nred + 31) / 32;
  for (int j = 0; j < NT; ++j)
    for (int lane = 0; lane < 64; ++lane) {
      const int col = 16 * j + (lane & 15), g4 = lane >> 4;
      for (int s = 0; s < S; ++s)
        for (int e = 0; e < 8; ++e) {
          const int red = 32 * s + (e < 4 ? 4 * g4 + e : 16 + 4 * g4 + e - 4);
          h[((size_t(j) * S + s) * 64 + lane) * 8 + e] =
              col < ncol && red < nred ? f64_to_bf16_rne(t[size_t(col) * nred + red]) : uint16_t(0);
        }
    }
}

}  // namespace dlm
