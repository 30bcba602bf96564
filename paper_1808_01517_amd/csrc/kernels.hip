// HIP kernels for gfx950 (MI355X): the register-staged matrix-core GEMM
// core, whose operand addressing is a policy type, and the small kernels
// (fold/unfold of the kernel tensor, losses, Adam, reductions).  The SH
// reductions over a shell's directions (Sec. 2.2), the LSC neighbourhood
// resampling, cyclic-kernel row dot and refit in the paper's order
// (Sec. 2.3), the fold of the kernel tensor and the masked LSC GEMMs share
// this tiled MFMA pipeline (the folded LSC GEMMs run on the streaming core,
// stream.hip; the per-shell SH contractions over the coefficients and the
// loss head on shell.hip):
//
//   C[r][n] = sum_k A(r, k) * B(n, k)
//
// FP32 form: v_mfma_f32_16x16x4_f32 (float32 products and accumulation).
// BF16 form: v_mfma_f32_16x16x32_bf16 with operands rounded to bfloat16
// (round to nearest even) as they are staged into LDS, float32 accumulation.
//
// Block = 256 threads (4 wave64s).  A block computes a BM x BN tile; each
// wave owns TM x TN MFMA tiles of 16 x 16.  K is walked in BK slices staged
// through LDS with the next slice prefetched into registers while the
// current one is multiplied.  Ragged M/N/K are zero-filled at load and
// masked at store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gemm_common.h"
#include "internal.h"

namespace dlm {


template <int BM_, int BN_, int WAVES_M_, int WAVES_N_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WAVES_M_, WN = WAVES_N_;
  static constexpr int TM = BM / (WM * 16), TN = BN / (WN * 16);
  static_assert(WM * WN == 4, "four waves per block");
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
};
using Cfg96 = Cfg<128, 96, 2, 2>;    // N = 1440, 2880 (15/30 tiles exactly)
using Cfg144 = Cfg<128, 144, 4, 1>;  // 96 < N <= 144 (N = 135)
using Cfg48 = Cfg<64, 48, 4, 1>;     // N <= 96 (N = 45, 90)
using Cfg16 = Cfg<128, 16, 4, 1>;    // N <= 16
using Cfg64 = Cfg<64, 64, 2, 2>;     // everything else

// Row stride (32-bit words) of a k-major LDS tile whose rows hold B row
// entries: padded so that the four k-rows one MFMA operand read touches
// start 16 banks apart (conflict-free for 32 and 64 banks).
constexpr int lds_stride(int B) {
  return (B % 64 == 16 || B % 64 == 48) ? B : B + ((B % 64) < 16 ? 16 - B % 64 : (B % 64) < 48 ? 48 - B % 64 : 80 - B % 64);
}



// Operand staging.  An operand is "k-contiguous" (kContig) or contiguous
// along its row index.  Threads move runs of 4 elements along the
// contiguous dimension: op.load4(row, k, g) for a run that lies inside the
// matrix, element-wise op(row, k, g) with zero fill at ragged edges.  The
// load phase only issues loads into registers; masking (op.kMask: element
// kept where op.mask4 / op.maskv > 0) and any conversion happen when the
// registers are written to LDS, after the current slice's MFMAs, so the
// prefetch latency overlaps the math.
template <class OPND, int ROWS, int BK>
struct Runs {
  static constexpr bool KC = OPND::kContig;
  static constexpr int NRUN = ROWS * BK / 4;               // runs per tile
  static constexpr int PER = (NRUN + 255) / 256;            // runs per thread
  __device__ static void coord(int e, int &row, int &k) {
    if constexpr (KC) { k = 4 * (e % (BK / 4)); row = e / (BK / 4); } else { row = 4 * (e % (ROWS / 4)); k = e / (ROWS / 4); }
  }
  // raw values (and mask values when the operand has one) of run (r, k)
  __device__ static void fetch(const OPND &op, int64_t r, int k, int64_t rows, int kend, int g, floatx4 &v, floatx4 &m) {
    const bool full = KC ? (r < rows && k + 3 < kend) : (r + 3 < rows && k < kend);
    if (full) {
      v = op.load4(r, k, g);
      if constexpr (OPND::kMask) m = op.mask4(r, k, g);
    } else {
      v = floatx4{0.f, 0.f, 0.f, 0.f};
      m = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int i = 0; i < 4; ++i) {
        const int64_t ri = KC ? r : r + i;
        const int ki = KC ? k + i : k;
        if (ri < rows && ki < kend) {
          v[i] = op(ri, ki, g);
          if constexpr (OPND::kMask) m[i] = op.maskv(ri, ki, g);
        }
      }
    }
  }
  __device__ static floatx4 finish(floatx4 v, floatx4 m) {
    if constexpr (OPND::kMask)
      for (int i = 0; i < 4; ++i) v[i] = m[i] > 0.0f ? v[i] : 0.0f;
    return v;
  }
};

// ------------------------------------------------------------- FP32 core
// LDS: a k-contiguous operand is stored row-major with k contiguous (row
// stride BK+4 words) and each lane reads 4 consecutive k with one 128-bit
// LDS load; a row-contiguous operand is stored k-major (rows contiguous)
// and read one word per MFMA.  Both use the same k order inside a 16-wide
// slice: MFMA j of 4 takes k = 4*(lane/16) + j, which is a permutation of
// the reduction index applied identically to A and B.
template <int OP, class CF, class AL, class BL, class CS>
__global__ __launch_bounds__(256) void gemm_f32_kernel(AL al, BL bl, CS cs, int64_t M, int N, int K, int ksplit,
                                                       int nbM, int nbN, int nz) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = 16;
  constexpr bool AK = AL::kContig, BKC = BL::kContig;
  constexpr int SA = AK ? BK + 4 : lds_stride(BM);
  constexpr int SB = BKC ? BK + 4 : lds_stride(BN);
  constexpr int AE = AK ? BM * SA : BK * SA;
  constexpr int BE = BKC ? BN * SB : BK * SB;
  using RA = Runs<AL, BM, BK>;
  using RB = Runs<BL, BN, BK>;
  __shared__ __attribute__((aligned(16))) float As[2][AE];
  __shared__ __attribute__((aligned(16))) float Bs[2][BE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const int q16 = lane & 15, g4 = lane >> 4;
  const TileMap tm(blockIdx.x, nbM, nbN, nz, ksplit > 0);
  const int64_t m0 = (int64_t)tm.mt * BM;
  const int n0 = tm.nt * BN;
  const int g = tm.z;
  int kbeg = 0, kend = K;
  if (ksplit > 0) {
    kbeg = g * ksplit;
    kend = min(K, kbeg + ksplit);
  }
  floatx4 ra[RA::PER], rb[RB::PER], ma[RA::PER], mb[RB::PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < RA::PER; ++p) {
      const int e = tid + p * 256;
      int row, kk;
      RA::coord(e, row, kk);
      if (e < RA::NRUN) RA::fetch(al, m0 + row, k0 + kk, M, kend, g, ra[p], ma[p]);
    }
#pragma unroll
    for (int p = 0; p < RB::PER; ++p) {
      const int e = tid + p * 256;
      int col, kk;
      RB::coord(e, col, kk);
      if (e < RB::NRUN) RB::fetch(bl, n0 + col, k0 + kk, N, kend, g, rb[p], mb[p]);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < RA::PER; ++p) {
      const int e = tid + p * 256;
      int row, kk;
      RA::coord(e, row, kk);
      if (e < RA::NRUN) {
        const floatx4 v = RA::finish(ra[p], ma[p]);
        if constexpr (AK) *reinterpret_cast<floatx4 *>(&As[buf][row * SA + kk]) = v;
        else *reinterpret_cast<floatx4 *>(&As[buf][kk * SA + row]) = v;
      }
    }
#pragma unroll
    for (int p = 0; p < RB::PER; ++p) {
      const int e = tid + p * 256;
      int col, kk;
      RB::coord(e, col, kk);
      if (e < RB::NRUN) {
        const floatx4 v = RB::finish(rb[p], mb[p]);
        if constexpr (BKC) *reinterpret_cast<floatx4 *>(&Bs[buf][col * SB + kk]) = v;
        else *reinterpret_cast<floatx4 *>(&Bs[buf][kk * SB + col]) = v;
      }
    }
  };
  floatx4 acc[CF::TM][CF::TN];
#pragma unroll
  for (int i = 0; i < CF::TM; ++i)
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int niter = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (niter > 0) {
    load(kbeg);
    stash(0);
    __syncthreads();
  }
  for (int it = 0; it < niter; ++it) {
    const int cur = it & 1;
    if (it + 1 < niter) load(kbeg + (it + 1) * BK);
    const float *Ac = As[cur];
    const float *Bc = Bs[cur];
    floatx4 a[CF::TM], b[CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i) {
      const int row = (wm * CF::TM + i) * 16 + q16;
      if constexpr (AK) a[i] = *reinterpret_cast<const floatx4 *>(&Ac[row * SA + 4 * g4]);
      else
        for (int j = 0; j < 4; ++j) a[i][j] = Ac[(4 * g4 + j) * SA + row];
    }
#pragma unroll
    for (int jn = 0; jn < CF::TN; ++jn) {
      const int col = (wn * CF::TN + jn) * 16 + q16;
      if constexpr (BKC) b[jn] = *reinterpret_cast<const floatx4 *>(&Bc[col * SB + 4 * g4]);
      else
        for (int j = 0; j < 4; ++j) b[jn][j] = Bc[(4 * g4 + j) * SB + col];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int jn = 0; jn < CF::TN; ++jn)
          acc[i][jn] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[jn][j], a[i][j], acc[i][jn], 0, 0, 0);
    if (it + 1 < niter) stash(cur ^ 1);
    __syncthreads();
  }
  // The MFMAs take the B fragment as their first operand, so each 16 x 16
  // accumulator is the transposed tile: lane l holds row m = l % 16 and the
  // four consecutive columns 4 (l / 16) .. +3, stored as one 16-byte run.
#pragma unroll
  for (int i = 0; i < CF::TM; ++i) {
    const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) {
      const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
      if (n + 3 < N) {
        cs.store4(r, n, g, acc[i][j]);
      } else {
        for (int q = 0; q < 4; ++q)
          if (n + q < N) cs(r, n + q, g, acc[i][j][q]);
      }
    }
  }
}

// ------------------------------------------------------------- BF16 core
// LDS holds both operands row-major with BK bfloat16 per row (k
// contiguous, row stride BK+8) so each lane reads its 8 consecutive k with
// one 128-bit load.  The 16-byte chunk c of row r is stored at chunk
// c ^ ((r >> 4) & 3), which keeps both the staging stores and the MFMA
// reads free of bank conflicts.  Every operand moves as 16-byte runs of 4
// floats (k-contiguous: 4 k of one row; row-contiguous: 4 rows of one k);
// conversion to bfloat16 (round to nearest even) happens when a run is
// written to LDS.  bfloat16 tables arrive as 8-byte runs of 4 k.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return (uint32_t)to_bf16_bits(lo) | ((uint32_t)to_bf16_bits(hi) << 16);
}

template <int OP, class CF, class AL, class BL, class CS>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(AL al, BL bl, CS cs, int64_t M, int N, int K, int ksplit,
                                                        int nbM, int nbN, int nz) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = 32, LD = BK + 8;
  constexpr bool AK = AL::kContig, BKC = BL::kContig;
  constexpr bool BT = std::is_same<typename BL::type, uint16_t>::value;
  static_assert(!BT || BKC, "bfloat16 tables are k-contiguous");
  using RA = Runs<AL, BM, BK>;
  using RB = Runs<BL, BN, BK>;
  // row-contiguous runs are grouped in 4 consecutive k (4 rows x 4 k per item)
  constexpr int NA = AK ? RA::NRUN : RA::NRUN / 4;
  constexpr int NB = BKC ? RB::NRUN : RB::NRUN / 4;
  constexpr int PA = (NA + 255) / 256, PB = (NB + 255) / 256;
  constexpr int QA = AK ? 1 : 4, QB = BKC ? 1 : 4;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const int q16 = lane & 15, g4 = lane >> 4;
  const TileMap tm(blockIdx.x, nbM, nbN, nz, ksplit > 0);
  const int64_t m0 = (int64_t)tm.mt * BM;
  const int n0 = tm.nt * BN;
  const int g = tm.z;
  int kbeg = 0, kend = K;
  if (ksplit > 0) {
    kbeg = g * ksplit;
    kend = min(K, kbeg + ksplit);
  }
  floatx4 ra[PA][QA], ma[PA][QA], rb[PB][QB], mb[PB][QB];
  uint2 rt[BT ? PB : 1];
  auto coordA = [&](int e, int &row, int &kk) {
    if constexpr (AK) { kk = 4 * (e % (BK / 4)); row = e / (BK / 4); } else { row = 4 * (e % (BM / 4)); kk = 4 * (e / (BM / 4)); }
  };
  auto coordB = [&](int e, int &col, int &kk) {
    if constexpr (BKC) { kk = 4 * (e % (BK / 4)); col = e / (BK / 4); } else { col = 4 * (e % (BN / 4)); kk = 4 * (e / (BN / 4)); }
  };
  auto sw = [&](int row, int k) { return row * LD + 8 * ((k >> 3) ^ ((row >> 4) & 3)) + (k & 7); };
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int e = tid + p * 256;
      if (e >= NA) continue;
      int row, kk;
      coordA(e, row, kk);
      for (int q = 0; q < QA; ++q) RA::fetch(al, m0 + row, k0 + kk + q, M, kend, g, ra[p][q], ma[p][q]);
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int e = tid + p * 256;
      if (e >= NB) continue;
      int col, kk;
      coordB(e, col, kk);
      const int n = n0 + col;
      const int k = k0 + kk;
      if constexpr (BT) {
        if (n < N && k + 3 < kend) {
          rt[p] = bl.load4h(n, k, g);
        } else {
          uint32_t h[4] = {0u, 0u, 0u, 0u};
          if (n < N)
            for (int i = 0; i < 4; ++i)
              if (k + i < kend) h[i] = bl(n, k + i, g);
          rt[p] = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        }
      } else {
        for (int q = 0; q < QB; ++q) RB::fetch(bl, n, k + q, N, kend, g, rb[p][q], mb[p][q]);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int e = tid + p * 256;
      if (e >= NA) continue;
      int row, kk;
      coordA(e, row, kk);
      if constexpr (AK) {
        const floatx4 v = RA::finish(ra[p][0], ma[p][0]);
        *reinterpret_cast<uint2 *>(&As[buf][sw(row, kk)]) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
      } else {
        floatx4 v[4];
        for (int q = 0; q < 4; ++q) v[q] = RA::finish(ra[p][q], ma[p][q]);
        for (int i = 0; i < 4; ++i)
          *reinterpret_cast<uint2 *>(&As[buf][sw(row + i, kk)]) =
              make_uint2(pack_bf16(v[0][i], v[1][i]), pack_bf16(v[2][i], v[3][i]));
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int e = tid + p * 256;
      if (e >= NB) continue;
      int col, kk;
      coordB(e, col, kk);
      if constexpr (BT) {
        *reinterpret_cast<uint2 *>(&Bs[buf][sw(col, kk)]) = rt[p];
      } else if constexpr (BKC) {
        const floatx4 v = RB::finish(rb[p][0], mb[p][0]);
        *reinterpret_cast<uint2 *>(&Bs[buf][sw(col, kk)]) = make_uint2(pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]));
      } else {
        floatx4 v[4];
        for (int q = 0; q < 4; ++q) v[q] = RB::finish(rb[p][q], mb[p][q]);
        for (int i = 0; i < 4; ++i)
          *reinterpret_cast<uint2 *>(&Bs[buf][sw(col + i, kk)]) =
              make_uint2(pack_bf16(v[0][i], v[1][i]), pack_bf16(v[2][i], v[3][i]));
      }
    }
  };
  floatx4 acc[CF::TM][CF::TN];
#pragma unroll
  for (int i = 0; i < CF::TM; ++i)
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int niter = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (niter > 0) {
    load(kbeg);
    stash(0);
    __syncthreads();
  }
  for (int it = 0; it < niter; ++it) {
    const int cur = it & 1;
    if (it + 1 < niter) load(kbeg + (it + 1) * BK);
    bf16x8 a[CF::TM], b[CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
      a[i] = *reinterpret_cast<const bf16x8 *>(&As[cur][sw((wm * CF::TM + i) * 16 + q16, 8 * g4)]);
#pragma unroll
    for (int j = 0; j < CF::TN; ++j)
      b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][sw((wn * CF::TN + j) * 16 + q16, 8 * g4)]);
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
    if (it + 1 < niter) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CF::TM; ++i) {
    const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
    if (r >= M) continue;
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) {
      const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
      if (n + 3 < N) {
        cs.store4(r, n, g, acc[i][j]);
      } else {
        for (int q = 0; q < 4; ++q)
          if (n + q < N) cs(r, n + q, g, acc[i][j][q]);
      }
    }
  }
}

// ------------------------------------------------------------- launching
enum class Shape { S96, S144, S48, S16, S64 };

static Shape pick_shape(int N) {
  if (N <= 16) return Shape::S16;
  if (N <= 96) return Shape::S48;
  if (N <= 144) return Shape::S144;
  const int p96 = (N + 95) / 96 * 96, p64 = (N + 63) / 64 * 64;
  return p96 <= p64 ? Shape::S96 : Shape::S64;
}

// Launch only the kernel of the requested precision (BF16 = true).
template <int OP, bool BF16, class AL, class BL, class CS>
static int run_gemm_p(AL al, BL bl, CS cs, int64_t M, int N, int K, int Z, int ksplit, hipStream_t st, Shape shape) {
  if (M <= 0 || N <= 0 || Z <= 0) return 0;
#define DLM_LAUNCH(CFG)                                                                                          \
  do {                                                                                                           \
    const int64_t nbM = (M + CFG::BM - 1) / CFG::BM;                                                             \
    const int nbN = (N + CFG::BN - 1) / CFG::BN;                                                                 \
    if (nbM * nbN * Z > 0x7fffffff) return -4;                                                                   \
    dim3 grid((unsigned)(nbM * nbN * Z));                                                                        \
    if constexpr (BF16)                                                                                          \
      hipLaunchKernelGGL((gemm_bf16_kernel<OP, CFG, AL, BL, CS>), grid, dim3(256), 0, st, al, bl, cs, M, N, K,    \
                         ksplit, (int)nbM, nbN, Z);                                                              \
    else                                                                                                         \
      hipLaunchKernelGGL((gemm_f32_kernel<OP, CFG, AL, BL, CS>), grid, dim3(256), 0, st, al, bl, cs, M, N, K,     \
                         ksplit, (int)nbM, nbN, Z);                                                              \
  } while (0)
  switch (shape) {
    case Shape::S96: DLM_LAUNCH(Cfg96); break;
    case Shape::S144: DLM_LAUNCH(Cfg144); break;
    case Shape::S48: DLM_LAUNCH(Cfg48); break;
    case Shape::S16: DLM_LAUNCH(Cfg16); break;
    default: DLM_LAUNCH(Cfg64); break;
  }
#undef DLM_LAUNCH
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int OP, class AL, class BL, class CS>
static int run_gemm(AL al, BL bl, CS cs, int64_t M, int N, int K, int Z, int ksplit, dlm_precision prec,
                    hipStream_t st, Shape shape) {
  if (prec == DLM_BF16) return run_gemm_p<OP, true>(al, bl, cs, M, N, K, Z, ksplit, st, shape);
  return run_gemm_p<OP, false>(al, bl, cs, M, N, K, Z, ksplit, st, shape);
}

// ------------------------------------------------------- operand policies
template <bool MASK>
struct ARowMajorT {
  static constexpr bool kContig = true;
  static constexpr bool kMask = MASK;
  const float *A, *mask;
  int64_t lda, gs;
  __device__ float operator()(int64_t r, int k, int g) const { return A[r * lda + (int64_t)g * gs + k]; }
  __device__ floatx4 load4(int64_t r, int k, int g) const { return ld4(A + r * lda + (int64_t)g * gs + k); }
  __device__ float maskv(int64_t r, int k, int g) const { return mask[r * lda + (int64_t)g * gs + k]; }
  __device__ floatx4 mask4(int64_t r, int k, int g) const { return ld4(mask + r * lda + (int64_t)g * gs + k); }
};
using ARowMajor = ARowMajorT<false>;

struct BTableF {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  using type = float;
  const float *B;
  int64_t gs;
  int64_t ld;  // row stride (>= K)
  __device__ float operator()(int n, int k, int g) const { return B[(int64_t)g * gs + (int64_t)n * ld + k]; }
  __device__ floatx4 load4(int n, int k, int g) const { return ld4(B + (int64_t)g * gs + (int64_t)n * ld + k); }
};

struct BTableH {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  using type = uint16_t;
  const uint16_t *B;
  int64_t gs;
  int64_t ld;  // row stride (>= K)
  __device__ uint16_t operator()(int n, int k, int g) const { return B[(int64_t)g * gs + (int64_t)n * ld + k]; }
  __device__ uint2 load4h(int n, int k, int g) const {
    uint2 v;
    __builtin_memcpy(&v, B + (int64_t)g * gs + (int64_t)n * ld + k, 8);
    return v;
  }
};


template <int OP, bool MASK>
static int table_gemm_m(const TableGemm &t, dlm_precision prec, hipStream_t st) {
  const Shape sh = pick_shape(t.N);
  CRowMajor cs{t.C, t.ldc, t.c_gs, t.relu, t.bias_n, t.out_mask};
  ARowMajorT<MASK> al{t.A, t.mask, t.lda, t.a_gs};
  if (prec == DLM_BF16)
    return run_gemm_p<OP, true>(al, BTableH{t.Bh, t.b_gs, t.ldb_h ? t.ldb_h : t.K}, cs, t.M, t.N, t.K, t.groups, 0, st,
                                sh);
  return run_gemm_p<OP, false>(al, BTableF{t.Bf, t.b_gs, t.ldb_f ? t.ldb_f : t.K}, cs, t.M, t.N, t.K, t.groups, 0,
                               st, sh);
}

template <int OP>
static int table_gemm_op(const TableGemm &t, dlm_precision prec, hipStream_t st) {
  return t.mask ? table_gemm_m<OP, true>(t, prec, st) : table_gemm_m<OP, false>(t, prec, st);
}

int launch_table_gemm(const TableGemm &t, dlm_precision prec, void *stream) {
  if (stream_table_ok(t, prec)) return launch_stream_table(t, prec, stream);
  if (t.Ah || t.Ch || t.out_mask_h || t.relu_bits_out || t.relu_bits_in)
    return -3;  // bfloat16 activations and ReLU bits: streaming core only
  hipStream_t st = (hipStream_t)stream;
  switch (t.op) {
    case kOpS2shFwd: return table_gemm_op<kOpS2shFwd>(t, prec, st);
    case kOpS2shBwd: return table_gemm_op<kOpS2shBwd>(t, prec, st);
    case kOpSh2sFwd: return table_gemm_op<kOpSh2sFwd>(t, prec, st);
    case kOpSh2sBwd: return table_gemm_op<kOpSh2sBwd>(t, prec, st);
    case kOpResample: return table_gemm_op<kOpResample>(t, prec, st);
    case kOpResampleBwd: return table_gemm_op<kOpResampleBwd>(t, prec, st);
    case kOpRefit: return table_gemm_op<kOpRefit>(t, prec, st);
    case kOpRefitBwd: return table_gemm_op<kOpRefitBwd>(t, prec, st);
    case kOpFoldFwd: return table_gemm_op<kOpFoldFwd>(t, prec, st);
    case kOpFoldBwdData: return table_gemm_op<kOpFoldBwdData>(t, prec, st);
    default: return -3;
  }
}

// --------------------------------------------- LSC neighbourhood contraction
// Index arithmetic of the paper-order form: the neighbourhood matrices X
// are [v][c][i][t] (m rows of T taps per voxel and channel), row-major, so
// the contractions address them through (v, i) = divmod(r, m) and
// (c, t) = divmod(k, T).  FastDiv divides by such a divisor with one 64-bit
// multiply and a shift (the round-up reciprocal mul = ceil(2^(32+s) / d),
// s = ceil(log2 d), exact for every dividend below 2^31 because 2^s >= d;
// the launchers keep row and reduction counts below 2^31).  Runs of 4
// entries that lie inside one T-tap segment (or inside one voxel's m rows)
// move as one 16-byte access; only runs across a boundary go entry by entry.
struct FastDiv {
  uint64_t mul = uint64_t(1) << 32;
  int shift = 32;
  int d = 1;
  static FastDiv make(int d) {
    FastDiv f;
    int s = 0;
    while ((int64_t(1) << s) < d) ++s;
    f.d = d;
    f.shift = 32 + s;
    f.mul = ((uint64_t(1) << f.shift) + uint64_t(d) - 1) / uint64_t(d);
    return f;
  }
  __device__ int div(int n) const { return (int)(((uint64_t)(uint32_t)n * mul) >> shift); }
};

__device__ __forceinline__ void st4(float *p, floatx4 v) {
  __builtin_memcpy(p, &v, 16);  // dword-aligned 16-byte store
}

// Row r = (v, i) of the neighbourhood matrix; column k = (c, t).
struct ANbhd {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  const float *X;
  int m, T, C;
  FastDiv fm, fT;
  __device__ const float *row(int64_t r, int c, int t) const {
    const int v = fm.div((int)r), i = (int)r - v * m;
    return X + ((int64_t)v * C + c) * ((int64_t)m * T) + (int64_t)i * T + t;
  }
  __device__ float operator()(int64_t r, int k, int) const {
    const int c = fT.div(k), t = k - c * T;
    return *row(r, c, t);
  }
  __device__ floatx4 load4(int64_t r, int k, int) const {
    const int c = fT.div(k), t = k - c * T;
    const float *p = row(r, c, t);
    if (t + 3 < T) return ld4(p);
    // the run crosses into channel c + 1 (k + 3 < C T is the caller's range)
    const int64_t next = (int64_t)m * T - T;  // from (c, T) to (c + 1, 0) in the same row i
    floatx4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = t + e < T ? p[e] : p[e + next];
    return v;
  }
};

struct BWeightF {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  using type = float;
  const float *W;
  int ld;
  __device__ float operator()(int n, int k, int) const { return W[(int64_t)n * ld + k]; }
  __device__ floatx4 load4(int n, int k, int) const { return ld4(W + (int64_t)n * ld + k); }
};

struct BWeightH {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  using type = uint16_t;
  const uint16_t *W;
  int ld;
  __device__ uint16_t operator()(int n, int k, int) const { return W[(int64_t)n * ld + k]; }
  __device__ uint2 load4h(int n, int k, int) const {
    uint2 v;
    __builtin_memcpy(&v, W + (int64_t)n * ld + k, 8);
    return v;
  }
};

// y[v][o][i] for row r = (v, i), column o: four columns are m apart (the
// lanes of a wave hold consecutive rows, so each store is coalesced).
struct CSignalY {
  float *y;
  const float *bias;
  int m, O;
  FastDiv fm;
  __device__ void operator()(int64_t r, int o, int, float v) const {
    const int vx = fm.div((int)r), i = (int)r - vx * m;
    if (bias) v += bias[o];
    y[((int64_t)vx * O + o) * m + i] = v;
  }
  __device__ void store4(int64_t r, int n, int, floatx4 v) const {
    const int vx = fm.div((int)r), i = (int)r - vx * m;
    float *p = y + ((int64_t)vx * O + n) * m + i;
#pragma unroll
    for (int q = 0; q < 4; ++q) p[(int64_t)q * m] = v[q] + (bias ? bias[n + q] : 0.0f);
  }
};

int launch_lsc_contract_fwd(const float *X, const float *W, const uint16_t *Wh, const float *bias, float *y,
                            int64_t V, int C, int O, int m, int T, dlm_precision prec, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t M = V * m;
  const int K = C * T;
  if (M >= (int64_t(1) << 31)) return -4;
  ANbhd al{X, m, T, C, FastDiv::make(m), FastDiv::make(T)};
  CSignalY cs{y, bias, m, O, FastDiv::make(m)};
  const Shape sh = pick_shape(O);
  if (prec == DLM_BF16) return run_gemm_p<kOpContractFwd, true>(al, BWeightH{Wh, K}, cs, M, O, K, 1, 0, st, sh);
  return run_gemm_p<kOpContractFwd, false>(al, BWeightF{W, K}, cs, M, O, K, 1, 0, st, sh);
}

// dy as the A operand: row r = (v, i), column k = o; consecutive rows are
// consecutive in memory.
struct ADy {
  static constexpr bool kContig = false;
  static constexpr bool kMask = false;
  const float *dy;
  int m, O;
  FastDiv fm;
  __device__ float operator()(int64_t r, int o, int) const {
    const int v = fm.div((int)r), i = (int)r - v * m;
    return dy[((int64_t)v * O + o) * m + i];
  }
  __device__ floatx4 load4(int64_t r, int o, int g) const {
    const int v = fm.div((int)r), i = (int)r - v * m;
    if (i + 3 < m) return ld4(dy + ((int64_t)v * O + o) * m + i);  // four rows of one voxel
    return floatx4{(*this)(r, o, g), (*this)(r + 1, o, g), (*this)(r + 2, o, g), (*this)(r + 3, o, g)};
  }
};

struct CNbhd {
  float *dX;
  int m, T, C;
  FastDiv fm, fT;
  __device__ float *at(int64_t r, int n) const {
    const int v = fm.div((int)r), i = (int)r - v * m;
    const int c = fT.div(n), t = n - c * T;
    return dX + ((int64_t)v * C + c) * ((int64_t)m * T) + (int64_t)i * T + t;
  }
  __device__ void operator()(int64_t r, int n, int, float val) const { *at(r, n) = val; }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    const int t = n - fT.div(n) * T;
    if (t + 3 < T) {
      st4(at(r, n), v);
    } else {
      for (int q = 0; q < 4; ++q) (*this)(r, n + q, g, v[q]);
    }
  }
};

int launch_lsc_contract_bwd_data(const float *dy, const float *Wt, const uint16_t *Wth, float *dX, int64_t V, int C,
                                 int O, int m, int T, dlm_precision prec, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t M = V * m;
  const int N = C * T;
  if (M >= (int64_t(1) << 31)) return -4;
  ADy al{dy, m, O, FastDiv::make(m)};
  CNbhd cs{dX, m, T, C, FastDiv::make(m), FastDiv::make(T)};
  const Shape sh = pick_shape(N);
  if (prec == DLM_BF16) return run_gemm_p<kOpContractBwdData, true>(al, BWeightH{Wth, O}, cs, M, N, O, 1, 0, st, sh);
  return run_gemm_p<kOpContractBwdData, false>(al, BWeightF{Wt, O}, cs, M, N, O, 1, 0, st, sh);
}

// Weight gradient: rows r = (c, t) plus one bias row (r = C*T, value 1),
// columns n = o, reduction k = (v, i) split into `splits` slices.
struct AXt {
  static constexpr bool kContig = false;
  static constexpr bool kMask = false;
  const float *X;
  int m, T, C;
  FastDiv fm, fT;
  __device__ float operator()(int64_t r, int k, int) const {
    const int CT = C * T;
    if (r == CT) return 1.0f;
    const int v = fm.div(k), i = k - v * m;
    const int c = fT.div((int)r), t = (int)r - c * T;
    return X[((int64_t)v * C + c) * ((int64_t)m * T) + (int64_t)i * T + t];
  }
  __device__ floatx4 load4(int64_t r, int k, int g) const {
    // four consecutive taps (c, t .. t+3) of one row i: contiguous inside a
    // segment; the bias row r = C T and segment crossings go entry by entry
    const int c = fT.div((int)r), t = (int)r - c * T;
    if (t + 3 < T) {
      const int v = fm.div(k), i = k - v * m;
      return ld4(X + ((int64_t)v * C + c) * ((int64_t)m * T) + (int64_t)i * T + t);
    }
    return floatx4{(*this)(r, k, g), (*this)(r + 1, k, g), (*this)(r + 2, k, g), (*this)(r + 3, k, g)};
  }
};

struct BDyT {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  using type = float;
  const float *dy;
  int m, O;
  FastDiv fm;
  __device__ float operator()(int o, int k, int) const {
    const int v = fm.div(k), i = k - v * m;
    return dy[((int64_t)v * O + o) * m + i];
  }
  __device__ floatx4 load4(int o, int k, int g) const {
    const int v = fm.div(k), i = k - v * m;
    if (i + 3 < m) return ld4(dy + ((int64_t)v * O + o) * m + i);  // four rows of one voxel
    return floatx4{(*this)(o, k, g), (*this)(o, k + 1, g), (*this)(o, k + 2, g), (*this)(o, k + 3, g)};
  }
};

struct CPartial {
  float *part;
  int rows, O;
  __device__ void operator()(int64_t r, int o, int s, float v) const {
    part[((int64_t)s * rows + r) * O + o] = v;
  }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    st4(part + ((int64_t)g * rows + r) * O + n, v);  // n + 3 < O: four adjacent columns
  }
};

int launch_lsc_contract_bwd_weight(const float *X, const float *dy, float *partial, int64_t V, int C, int O, int m,
                                   int T, int splits, dlm_precision prec, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int rows = C * T + 1;
  const int64_t Kfull = V * m;
  const int bk = 32;  // a multiple of both cores' K slice
  int ksplit = (int)((Kfull + splits - 1) / splits);
  ksplit = (ksplit + bk - 1) / bk * bk;
  const int used = (int)((Kfull + ksplit - 1) / ksplit);
  // splits beyond `used` would see an empty range; the caller sizes `splits`
  // so that every slice is non-empty and reduces exactly `splits` partials.
  if (used != splits) return -2;
  if (Kfull >= (int64_t(1) << 31)) return -4;
  return run_gemm<kOpContractBwdWeight>(AXt{X, m, T, C, FastDiv::make(m), FastDiv::make(T)},
                                        BDyT{dy, m, O, FastDiv::make(m)}, CPartial{partial, rows, O}, rows, O,
                                        (int)Kfull, splits, ksplit, prec, st, pick_shape(O));
}

int lsc_weight_splits(int64_t V, int m, int target) {
  const int64_t Kfull = V * m;
  const int bk = 32;
  int s = target;
  while (s > 1) {
    int ksplit = (int)((Kfull + s - 1) / s);
    ksplit = (ksplit + bk - 1) / bk * bk;
    if ((Kfull + ksplit - 1) / ksplit == s) break;
    --s;
  }
  return s < 1 ? 1 : s;
}

// ------------------------------------------------------- folded LSC form
// B(n = (k,j), t) = Q[t][k][j]: consecutive n are consecutive in memory.
struct BQt {
  static constexpr bool kContig = false;
  static constexpr bool kMask = false;
  using type = float;
  const float *Q;
  int KK;
  __device__ float operator()(int n, int t, int) const { return Q[(int64_t)t * KK + n]; }
  __device__ floatx4 load4(int n, int t, int) const { return ld4(Q + (int64_t)t * KK + n); }
};

struct CFold {
  float *Tw, *TwT;
  uint16_t *Twh, *TwTh;
  int C, Ki, Ko, O;
  int64_t ld, ldt;
  __device__ void operator()(int64_t r, int n, int, float v) const {
    const int o = (int)r / C, c = (int)r - o * C;
    const int k = n / Ki, j = n - k * Ki;
    const int64_t row = (int64_t)o * Ko + k, col = (int64_t)c * Ki + j;
    const int64_t a = row * ld + col, b = col * ldt + row;
    if (Tw) Tw[a] = v;
    if (TwT) TwT[b] = v;
    if (Twh) Twh[a] = to_bf16_bits(v);
    if (TwTh) TwTh[b] = to_bf16_bits(v);
  }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    for (int q = 0; q < 4; ++q) (*this)(r, n + q, g, v[q]);
  }
};

int launch_lsc_fold(const float *W, const float *Q, int C, int O, int T, int Ki, int Ko, float *Tw, float *TwT,
                    uint16_t *Twh, uint16_t *TwTh, int64_t ld, int64_t ldt, void *stream) {
  const int KK = Ko * Ki;
  return run_gemm<kOpFoldMake>(ARowMajor{W, nullptr, T, 0}, BQt{Q, KK},
                               CFold{Tw, TwT, Twh, TwTh, C, Ki, Ko, O, ld, ldt}, (int64_t)O * C, KK, T, 1, 0,
                               DLM_FP32, (hipStream_t)stream, pick_shape(KK));
}

__global__ void zero_kernel(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int launch_zero(void *p, size_t bytes, void *stream) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return 0;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<uint32_t *>(p), n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// zero bytes [c0, ld) of each of `rows` rows of ld bytes (c0, ld even)
__global__ void zero_cols_kernel(uint16_t *p, int64_t rows, int64_t c0, int64_t ld) {
  const int64_t w = (ld - c0) / 2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * w) return;
  const int64_t r = i / w;
  p[(r * ld + c0) / 2 + (i - r * w)] = 0;
}

int launch_zero_cols(void *p, int64_t rows, int64_t c0_bytes, int64_t ld_bytes, void *stream) {
  if (rows <= 0 || ld_bytes <= c0_bytes) return 0;
  if ((c0_bytes | ld_bytes) & 1) return -3;
  const int64_t n = rows * ((ld_bytes - c0_bytes) / 2);
  hipLaunchKernelGGL(zero_cols_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     static_cast<uint16_t *>(p), rows, c0_bytes, ld_bytes);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void bias_vec_kernel(const float *bias, const float *pm1, int O, int Ko, float *bvec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= O * Ko) return;
  const int o = i / Ko, k = i - o * Ko;
  bvec[i] = bias ? bias[o] * pm1[k] : 0.0f;
}

int launch_lsc_bias_vec(const float *bias, const float *pm1, int O, int Ko, float *bvec, void *stream) {
  hipLaunchKernelGGL(bias_vec_kernel, dim3((O * Ko + 255) / 256), dim3(256), 0, (hipStream_t)stream, bias, pm1, O,
                     Ko, bvec);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Weight-gradient reduction dT[m][n] = sum_v g[v][m] * act[v][n] over voxel
// slices (split K).  g = da_out masked by a_out > 0 (m = (o,k)); act = a_in
// plus a ones column (n = (c,j) or n = CK, giving the bias term).  Both
// operands are contiguous along their row index, so the voxel index is the
// strided one.  The larger of M and N1 is put on the GEMM's row side.
template <bool MASK>
struct AGradT {
  static constexpr bool kContig = false;
  static constexpr bool kMask = MASK;
  const float *g, *mask;
  int M;
  __device__ float operator()(int64_t m, int v, int) const { return g[(int64_t)v * M + m]; }
  __device__ floatx4 load4(int64_t m, int v, int) const { return ld4(g + (int64_t)v * M + m); }
  __device__ float maskv(int64_t m, int v, int) const { return mask[(int64_t)v * M + m]; }
  __device__ floatx4 mask4(int64_t m, int v, int) const { return ld4(mask + (int64_t)v * M + m); }
};

struct BActT {
  static constexpr bool kContig = false;
  static constexpr bool kMask = false;
  using type = float;
  const float *a;
  int CK;
  __device__ float operator()(int n, int v, int) const { return n < CK ? a[(int64_t)v * CK + n] : 1.0f; }
  __device__ floatx4 load4(int n, int v, int g) const {
    if (n + 3 < CK) return ld4(a + (int64_t)v * CK + n);
    return floatx4{(*this)(n, v, g), (*this)(n + 1, v, g), (*this)(n + 2, v, g), (*this)(n + 3, v, g)};
  }
};

// transposed orientation: activations on the row side, gradient on the column side
struct AActT {
  static constexpr bool kContig = false;
  static constexpr bool kMask = false;
  const float *a;
  int CK;
  __device__ float operator()(int64_t n, int v, int) const { return n < CK ? a[(int64_t)v * CK + n] : 1.0f; }
  __device__ floatx4 load4(int64_t n, int v, int g) const {
    if (n + 3 < CK) return ld4(a + (int64_t)v * CK + n);
    return floatx4{(*this)(n, v, g), (*this)(n + 1, v, g), (*this)(n + 2, v, g), (*this)(n + 3, v, g)};
  }
};

template <bool MASK>
struct BGradT {
  static constexpr bool kContig = false;
  static constexpr bool kMask = MASK;
  using type = float;
  const float *g, *mask;
  int M;
  __device__ float operator()(int m, int v, int) const { return g[(int64_t)v * M + m]; }
  __device__ floatx4 load4(int m, int v, int) const { return ld4(g + (int64_t)v * M + m); }
  __device__ float maskv(int m, int v, int) const { return mask[(int64_t)v * M + m]; }
  __device__ floatx4 mask4(int m, int v, int) const { return ld4(mask + (int64_t)v * M + m); }
};


static int split_len(int64_t K, int splits) {
  const int bk = 32;
  int ks = (int)((K + splits - 1) / splits);
  return (ks + bk - 1) / bk * bk;
}

int fold_grad_split_len(int64_t V, int splits) { return split_len(V, splits); }

static Shape grad_shape(int M, int N1) {
  // the smaller side (135/136 for the three-shell layers) fits one 144-wide
  // tile, so the larger operand is read once; otherwise 64 x 64
  return std::min(M, N1) <= 144 ? Shape::S144 : Shape::S64;
}

int fold_grad_splits(int64_t V, int M, int N1) {
  const int big = std::max(M, N1), small = std::min(M, N1);
  const int64_t tiles = grad_shape(M, N1) == Shape::S144 ? (big + 127) / 128 : ((big + 63) / 64) * ((small + 63) / 64);
  int s = (int)std::min<int64_t>(128, std::max<int64_t>(1, (2048 + tiles - 1) / tiles));
  s = (int)std::min<int64_t>(s, std::max<int64_t>(1, V / 512));
  while (s > 1 && (V + split_len(V, s) - 1) / split_len(V, s) != s) --s;
  return s;
}

int launch_lsc_fold_grad(const float *da_out, const float *mask, const float *a_in, int64_t V, int M, int CK,
                         int splits, float *partial, dlm_precision prec, void *stream) {
  const int N1 = CK + 1;
  const int ks = split_len(V, splits);
  if ((V + ks - 1) / ks != splits) return -2;
  if (!mask && stream_grad_ok(M, CK, ks))
    return launch_stream_grad(da_out, nullptr, a_in, nullptr, V, M, CK, splits, ks, partial, prec, stream);
  hipStream_t st = (hipStream_t)stream;
  const Shape sh = grad_shape(M, N1);
  if (M >= N1) {
    if (mask)
      return run_gemm<kOpFoldGrad>(AGradT<true>{da_out, mask, M}, BActT{a_in, CK}, CPartial2<false>{partial, M, N1}, M,
                                   N1, (int)V, splits, ks, prec, st, sh);
    return run_gemm<kOpFoldGrad>(AGradT<false>{da_out, nullptr, M}, BActT{a_in, CK}, CPartial2<false>{partial, M, N1},
                                 M, N1, (int)V, splits, ks, prec, st, sh);
  }
  if (mask)
    return run_gemm<kOpFoldGrad>(AActT{a_in, CK}, BGradT<true>{da_out, mask, M}, CPartial2<true>{partial, M, N1}, N1, M,
                                 (int)V, splits, ks, prec, st, sh);
  return run_gemm<kOpFoldGrad>(AActT{a_in, CK}, BGradT<false>{da_out, nullptr, M}, CPartial2<true>{partial, M, N1}, N1,
                               M, (int)V, splits, ks, prec, st, sh);
}

__global__ void sum_partials_kernel(const float *part, int splits, int64_t n, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int p = 0; p < splits; ++p) s += part[(int64_t)p * n + i];
  out[i] = s;
}

int launch_sum_partials(const float *part, int splits, int64_t n, float *out, void *stream) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, part,
                     splits, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// dW[(o*C+c)][t] = sum_{kk,j} dTw[(o*Ko+kk)][c*Ki+j] Q[t][kk][j]: one wave
// per output (O*C*T of them), lanes striding the Ko*Ki-long reduction in a
// fixed order, then a butterfly sum.  (A GEMM here has a 96 x 17 output and
// a 2025-deep reduction: two blocks, all latency.)
__global__ __launch_bounds__(256) void unfold_kernel(const float *dTw, const float *Q, int C, int T, int Ki, int Ko,
                                                     int N1, int nout, float *dW) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (w >= nout) return;  // whole waves only
  const int t = w % T, oc = w / T, o = oc / C, c = oc - o * C;
  const int KK = Ko * Ki;
  const float *q = Q + (int64_t)t * KK;
  const float *g = dTw + (int64_t)o * Ko * N1 + (int64_t)c * Ki;
  float s = 0.0f;
  for (int e = lane; e < KK; e += 64) {
    const int kk = e / Ki, j = e - kk * Ki;
    s += g[(int64_t)kk * N1 + j] * q[e];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) dW[(int64_t)oc * T + t] = s;
}

__global__ void bias_grad_kernel(const float *dTw, const float *pm1, int O, int Ko, int N1, int CK, float *db) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= O) return;
  float s = 0.0f;
  for (int k = 0; k < Ko; ++k) s += dTw[((int64_t)o * Ko + k) * N1 + CK] * pm1[k];
  db[o] = s;
}

int launch_lsc_unfold(const float *dTw, const float *Q, const float *pm1, int C, int O, int T, int Ki, int Ko,
                      float *dW, float *db, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int N1 = C * Ki + 1;
  const int nout = O * C * T;
  hipLaunchKernelGGL(unfold_kernel, dim3((unsigned)((nout + 3) / 4)), dim3(256), 0, st, dTw, Q, C, T, Ki, Ko, N1, nout,
                     dW);
  if (hipGetLastError() != hipSuccess) return -1;
  if (!db) return 0;
  hipLaunchKernelGGL(bias_grad_kernel, dim3((O + 63) / 64), dim3(64), 0, st, dTw, pm1, O, Ko, N1, C * Ki, db);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// --------------------------------------------------------- small kernels
__global__ void reduce_weight_partials_kernel(const float *part, int splits, float *dW, float *db, int C, int O,
                                              int T, int accumulate) {
  const int CT = C * T, rows = CT + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * O) return;
  const int r = idx / O, o = idx - r * O;
  float s = 0.0f;
  for (int p = 0; p < splits; ++p) s += part[((int64_t)p * rows + r) * O + o];
  if (r < CT) {
    float *dst = dW + (int64_t)o * CT + r;
    *dst = accumulate ? *dst + s : s;
  } else if (db) {
    db[o] = accumulate ? db[o] + s : s;
  }
}

int launch_reduce_weight_partials(const float *partial, int splits, float *dW, float *db, int C, int O, int T,
                                  int accumulate, void *stream) {
  const int n = (C * T + 1) * O;
  hipLaunchKernelGGL(reduce_weight_partials_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     partial, splits, dW, db, C, O, T, accumulate);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void prepare_weights_kernel(const float *W, float *Wt, uint16_t *Wh, uint16_t *Wth, int C, int O, int T) {
  const int CT = C * T;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= O * CT) return;
  const int o = idx / CT, ct = idx - o * CT;
  const float w = W[idx];
  Wt[(int64_t)ct * O + o] = w;
  if (Wh) Wh[idx] = to_bf16_bits(w);
  if (Wth) Wth[(int64_t)ct * O + o] = to_bf16_bits(w);
}

int launch_prepare_weights(const float *W, float *Wt, uint16_t *Wh, uint16_t *Wth, int C, int O, int T,
                           void *stream) {
  const int n = O * C * T;
  hipLaunchKernelGGL(prepare_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, W, Wt, Wh,
                     Wth, C, O, T);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// MSE: each block sums its grid-stride share in a fixed order and writes one
// partial; a single block then adds the partials in index order.  REL
// weights every error by 1 / (|target| + eps).
template <bool REL>
__global__ __launch_bounds__(256) void mse_partial_kernel(const float *pred, const float *target, int64_t n,
                                                          float *dpred, float *partials, float scale, float eps) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float t = target[i];
    const float w = REL ? 1.0f / (fabsf(t) + eps) : 1.0f;
    const float d = (pred[i] - t) * w;
    s += d * d;
    if (dpred) dpred[i] = scale * d * w;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void mse_final_kernel(const float *partials, int nb, float *loss, float inv_n) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < nb; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

int mse_blocks(int64_t n) {
  int64_t b = (n + 256 * 8 - 1) / (256 * 8);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

int launch_mse(const float *pred, const float *target, int64_t n, float *loss, float *dpred, float *partials,
               int nblocks, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(mse_partial_kernel<false>, dim3(nblocks), dim3(256), 0, st, pred, target, n, dpred, partials,
                     (float)(2.0 / (double)n), 0.0f);
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, loss, (float)(1.0 / (double)n));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// sums[b] = sum of partials[b*chunk .. min(n, (b+1)*chunk)), one block each
__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *partials, int64_t n, int64_t chunk,
                                                         float *sums) {
  __shared__ float red[256];
  const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  float s = 0.0f;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

int launch_sum_scaled(const float *partials, int64_t n, float *out, float scale, float *scratch, void *stream) {
  if (n <= 0 || n > 0x7fffffff) return -3;
  hipStream_t st = (hipStream_t)stream;
  if (n <= 4096) {
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, partials, (int)n, out, scale);
  } else {
    // two passes in a fixed order: kSumBlocks chunk sums, then one block
    const int64_t chunk = (n + kSumBlocks - 1) / kSumBlocks;
    const int nb = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(nb), dim3(256), 0, st, partials, n, chunk, scratch);
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, scratch, nb, out, scale);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_relmse(const float *pred, const float *target, int64_t n, float eps, float *loss, float *dpred,
                  float *partials, int nblocks, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(mse_partial_kernel<true>, dim3(nblocks), dim3(256), 0, st, pred, target, n, dpred, partials,
                     (float)(2.0 / (double)n), eps);
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, loss, (float)(1.0 / (double)n));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------- Signal2SH on raw acquisitions
__global__ void b0_inverse_mean_kernel(const float *raw, int64_t ld, const int32_t *b0idx, int nb0, int64_t V,
                                       float *inv) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  float s = 0.0f;
  for (int i = 0; i < nb0; ++i) s += raw[v * ld + b0idx[i]];
  inv[v] = (float)nb0 / s;
}

int launch_b0_inverse_mean(const float *raw, int64_t ld, const int32_t *b0idx, int nb0, int64_t V, float *inv,
                           void *stream) {
  hipLaunchKernelGGL(b0_inverse_mean_kernel, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     raw, ld, b0idx, nb0, V, inv);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

struct ARawNorm {
  static constexpr bool kContig = true;
  static constexpr bool kMask = false;
  const float *raw;
  int64_t ld;
  const int32_t *dwidx;
  const float *inv;
  int N;
  __device__ float operator()(int64_t r, int k, int g) const { return raw[r * ld + dwidx[g * N + k]] * inv[r]; }
  __device__ floatx4 load4(int64_t r, int k, int g) const {
    return floatx4{(*this)(r, k, g), (*this)(r, k + 1, g), (*this)(r, k + 2, g), (*this)(r, k + 3, g)};
  }
};

int launch_s2sh_raw(const float *raw, int64_t ld, const int32_t *dwidx, const float *inv, const float *Pf,
                    const uint16_t *Ph, float *c, int64_t ldc, int64_t V, int S, int N, int K, dlm_precision prec,
                    void *stream) {
  hipStream_t st = (hipStream_t)stream;
  ARawNorm al{raw, ld, dwidx, inv, N};
  CRowMajor cs{c, ldc, K, 0, nullptr};
  const Shape sh = pick_shape(K);
  if (prec == DLM_BF16) return run_gemm_p<kOpS2shRaw, true>(al, BTableH{Ph, (int64_t)N * K, N}, cs, V, K, N, S, 0, st, sh);
  return run_gemm_p<kOpS2shRaw, false>(al, BTableF{Pf, (int64_t)N * K, N}, cs, V, K, N, S, 0, st, sh);
}

__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, void *stream) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                     n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace dlm
