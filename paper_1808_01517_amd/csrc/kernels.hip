// HIP kernels for gfx950 (MI355X): every contraction of the DELIMIT layers
// runs through one matrix-core GEMM core whose operand addressing is a
// policy type, so the SH transforms (Sec. 2.2), the LSC neighbourhood
// resampling, the cyclic-kernel row dot and the refit (Sec. 2.3) and all
// their adjoints share the same tiled MFMA pipeline:
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

#include "internal.h"

namespace dlm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
  __bf16 h = (__bf16)f;  // hardware round-to-nearest-even conversion
  return __builtin_bit_cast(uint16_t, h);
}

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

// Row stride (in 32-bit words) of a k-major LDS tile whose rows hold B
// entries: padded so that the four k-rows one MFMA operand read touches
// start 16 banks apart (conflict-free for 32 and 64 banks).
constexpr int lds_stride(int B) {
  return (B % 64 == 16 || B % 64 == 48) ? B : B + ((B % 64) < 16 ? 16 - B % 64 : (B % 64) < 48 ? 48 - B % 64 : 80 - B % 64);
}

// Block index -> (M tile, N tile).  Workgroups are dispatched round-robin
// over the 8 XCDs; consecutive logical tiles are gathered onto one XCD so
// the N tiles that share an A row-block run together and hit the same L2.
struct TileMap {
  int mt, nt;
  __device__ TileMap(int b, int nbM, int nbN) {
    const int total = nbM * nbN;
    const int q = total >> 3, r = total & 7;
    const int xcd = b & 7, local = b >> 3;
    const int L = xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
    mt = L / nbN;
    nt = L - mt * nbN;
  }
};

// ------------------------------------------------------------- FP32 core
template <int OP, class CF, class AL, class BL, class CS>
__global__ __launch_bounds__(256) void gemm_f32_kernel(AL al, BL bl, CS cs, int64_t M, int N, int K, int ksplit,
                                                       int nbM, int nbN) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = 16;
  constexpr int SA = lds_stride(BM), SB = lds_stride(BN);
  constexpr int APT = BM * BK / 256, BPT = (BN * BK + 255) / 256;
  __shared__ float As[2][BK * SA];
  __shared__ float Bs[2][BK * SB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const TileMap tm(blockIdx.x, nbM, nbN);
  const int64_t m0 = (int64_t)tm.mt * BM;
  const int n0 = tm.nt * BN;
  const int g = blockIdx.z;
  int kbeg = 0, kend = K;
  if (ksplit > 0) {
    kbeg = g * ksplit;
    kend = min(K, kbeg + ksplit);
  }
  float ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int e = tid + p * 256;
      int mm, kk;
      if constexpr (AL::kContig) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      const int64_t r = m0 + mm;
      const int k = k0 + kk;
      ra[p] = (r < M && k < kend) ? al(r, k, g) : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int e = tid + p * 256;
      int nn, kk;
      if constexpr (BL::kContig) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
      const int n = n0 + nn;
      const int k = k0 + kk;
      rb[p] = (e < BN * BK && n < N && k < kend) ? bl(n, k, g) : 0.0f;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int e = tid + p * 256;
      int mm, kk;
      if constexpr (AL::kContig) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      As[buf][kk * SA + mm] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BPT; ++p) {
      const int e = tid + p * 256;
      int nn, kk;
      if constexpr (BL::kContig) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
      if (e < BN * BK) Bs[buf][kk * SB + nn] = rb[p];
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
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float a[CF::TM], b[CF::TN];
      const int row = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < CF::TM; ++i) a[i] = Ac[row * SA + (wm * CF::TM + i) * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) b[j] = Bc[row * SB + (wn * CF::TN + j) * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < CF::TM; ++i)
#pragma unroll
        for (int j = 0; j < CF::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (it + 1 < niter) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CF::TM; ++i)
#pragma unroll
    for (int j = 0; j < CF::TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = m0 + (wm * CF::TM + i) * 16 + 4 * (lane >> 4) + q;
        const int n = n0 + (wn * CF::TN + j) * 16 + (lane & 15);
        if (r < M && n < N) cs(r, n, g, acc[i][j][q]);
      }
}

// ------------------------------------------------------------- BF16 core
// LDS holds m-major rows of BK bfloat16 (k contiguous) so that each lane
// reads its 8 consecutive k as one 16-byte load.
template <int OP, class CF, class AL, class BL, class CS>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(AL al, BL bl, CS cs, int64_t M, int N, int K, int ksplit,
                                                        int nbM, int nbN) {
  constexpr int BM = CF::BM, BN = CF::BN, BK = 32, LD = BK + 8;
  constexpr int APT = BM * BK / 256, BPT = (BN * BK + 255) / 256;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const TileMap tm(blockIdx.x, nbM, nbN);
  const int64_t m0 = (int64_t)tm.mt * BM;
  const int n0 = tm.nt * BN;
  const int g = blockIdx.z;
  int kbeg = 0, kend = K;
  if (ksplit > 0) {
    kbeg = g * ksplit;
    kend = min(K, kbeg + ksplit);
  }
  // K-contiguous operands: each thread converts pairs of consecutive k and
  // stores them as one 32-bit word.
  uint32_t ra[APT], rb[BPT];
  // Every thread converts pairs of consecutive k and stores them as one
  // 32-bit LDS word; for m/n-contiguous operands the pair's two loads are
  // each coalesced across the consecutive m (n) of neighbouring threads.
  auto ida = [&](int e, int &mm, int &kk) {
    if constexpr (AL::kContig) { kk = 2 * (e % (BK / 2)); mm = e / (BK / 2); } else { mm = e % BM; kk = 2 * (e / BM); }
  };
  auto idb = [&](int e, int &nn, int &kk) {
    if constexpr (BL::kContig) { kk = 2 * (e % (BK / 2)); nn = e / (BK / 2); } else { nn = e % BN; kk = 2 * (e / BN); }
  };
  constexpr int AITEMS = APT / 2;
  constexpr int BITEMS = (BPT + 1) / 2;
  constexpr int BTOTAL = BN * BK / 2;
  auto cvt = [&](float f) -> uint32_t { return (uint32_t)to_bf16_bits(f); };
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AITEMS; ++p) {
      const int e = tid + p * 256;
      int mm, kk;
      ida(e, mm, kk);
      const int64_t r = m0 + mm;
      const int k = k0 + kk;
      const uint32_t lo = (r < M && k < kend) ? cvt(al(r, k, g)) : 0u;
      const uint32_t hi = (r < M && k + 1 < kend) ? cvt(al(r, k + 1, g)) : 0u;
      ra[p] = lo | (hi << 16);
    }
#pragma unroll
    for (int p = 0; p < BITEMS; ++p) {
      const int e = tid + p * 256;
      int nn, kk;
      idb(e, nn, kk);
      const int n = n0 + nn;
      const int k = k0 + kk;
      const bool okn = e < BTOTAL && n < N;
      uint32_t lo = 0u, hi = 0u;
      if constexpr (std::is_same<typename BL::type, float>::value) {
        lo = (okn && k < kend) ? cvt(bl(n, k, g)) : 0u;
        hi = (okn && k + 1 < kend) ? cvt(bl(n, k + 1, g)) : 0u;
      } else {
        lo = (okn && k < kend) ? (uint32_t)bl(n, k, g) : 0u;
        hi = (okn && k + 1 < kend) ? (uint32_t)bl(n, k + 1, g) : 0u;
      }
      rb[p] = lo | (hi << 16);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < AITEMS; ++p) {
      const int e = tid + p * 256;
      int mm, kk;
      ida(e, mm, kk);
      *reinterpret_cast<uint32_t *>(&As[buf][mm * LD + kk]) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BITEMS; ++p) {
      const int e = tid + p * 256;
      int nn, kk;
      idb(e, nn, kk);
      if (e < BTOTAL) *reinterpret_cast<uint32_t *>(&Bs[buf][nn * LD + kk]) = rb[p];
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
      a[i] = *reinterpret_cast<const bf16x8 *>(&As[cur][((wm * CF::TM + i) * 16 + (lane & 15)) * LD + 8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < CF::TN; ++j)
      b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][((wn * CF::TN + j) * 16 + (lane & 15)) * LD + 8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (it + 1 < niter) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CF::TM; ++i)
#pragma unroll
    for (int j = 0; j < CF::TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = m0 + (wm * CF::TM + i) * 16 + 4 * (lane >> 4) + q;
        const int n = n0 + (wn * CF::TN + j) * 16 + (lane & 15);
        if (r < M && n < N) cs(r, n, g, acc[i][j][q]);
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

template <int OP, class AL, class BL, class CS>
static int run_gemm(AL al, BL bl, CS cs, int64_t M, int N, int K, int Z, int ksplit, dlm_precision prec,
                    hipStream_t st, Shape shape) {
  if (M <= 0 || N <= 0 || Z <= 0) return 0;
#define DLM_LAUNCH(CFG)                                                                                           \
  do {                                                                                                            \
    const int64_t nbM = (M + CFG::BM - 1) / CFG::BM;                                                              \
    const int nbN = (N + CFG::BN - 1) / CFG::BN;                                                                  \
    if (nbM * nbN > 0x7fffffff) return -4;                                                                        \
    dim3 grid((unsigned)(nbM * nbN), 1, (unsigned)Z);                                                             \
    if (prec == DLM_BF16)                                                                                         \
      hipLaunchKernelGGL((gemm_bf16_kernel<OP, CFG, AL, BL, CS>), grid, dim3(256), 0, st, al, bl, cs, M, N, K,     \
                         ksplit, (int)nbM, nbN);                                                                  \
    else                                                                                                          \
      hipLaunchKernelGGL((gemm_f32_kernel<OP, CFG, AL, BL, CS>), grid, dim3(256), 0, st, al, bl, cs, M, N, K,      \
                         ksplit, (int)nbM, nbN);                                                                  \
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

// ------------------------------------------------------- operand policies
struct ARowMajor {
  static constexpr bool kContig = true;
  const float *A, *mask;
  int64_t lda, gs;
  __device__ float operator()(int64_t r, int k, int g) const {
    const int64_t o = r * lda + (int64_t)g * gs + k;
    float v = A[o];
    if (mask) v = mask[o] > 0.0f ? v : 0.0f;
    return v;
  }
};

struct BTableF {
  static constexpr bool kContig = true;
  using type = float;
  const float *B;
  int64_t gs;
  int K;
  __device__ float operator()(int n, int k, int g) const { return B[(int64_t)g * gs + (int64_t)n * K + k]; }
};

struct BTableH {
  static constexpr bool kContig = true;
  using type = uint16_t;
  const uint16_t *B;
  int64_t gs;
  int K;
  __device__ uint16_t operator()(int n, int k, int g) const { return B[(int64_t)g * gs + (int64_t)n * K + k]; }
};

struct CRowMajor {
  float *C;
  int64_t ldc, gs;
  int relu;
  const float *bias_n;
  __device__ void operator()(int64_t r, int n, int g, float v) const {
    if (bias_n) v += bias_n[n];
    if (relu) v = fmaxf(v, 0.0f);
    C[r * ldc + (int64_t)g * gs + n] = v;
  }
};

template <int OP>
static int table_gemm_op(const TableGemm &t, dlm_precision prec, hipStream_t st) {
  const Shape sh = pick_shape(t.N);
  CRowMajor cs{t.C, t.ldc, t.c_gs, t.relu, t.bias_n};
  ARowMajor al{t.A, t.mask, t.lda, t.a_gs};
  if (prec == DLM_BF16) return run_gemm<OP>(al, BTableH{t.Bh, t.b_gs, t.K}, cs, t.M, t.N, t.K, t.groups, 0, prec, st, sh);
  return run_gemm<OP>(al, BTableF{t.Bf, t.b_gs, t.K}, cs, t.M, t.N, t.K, t.groups, 0, prec, st, sh);
}

int launch_table_gemm(const TableGemm &t, dlm_precision prec, void *stream) {
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
// Row r = (v, i) of the neighbourhood matrix; column k = (c, t).
struct ANbhd {
  static constexpr bool kContig = true;
  const float *X;
  int m, T, C;
  __device__ float operator()(int64_t r, int k, int) const {
    const int64_t v = r / m;
    const int i = (int)(r - v * m);
    const int c = k / T, t = k - c * T;
    const int64_t P = (int64_t)m * T;
    return X[(v * C + c) * P + (int64_t)i * T + t];
  }
};

struct BWeightF {
  static constexpr bool kContig = true;
  using type = float;
  const float *W;
  int ld;
  __device__ float operator()(int n, int k, int) const { return W[(int64_t)n * ld + k]; }
};

struct BWeightH {
  static constexpr bool kContig = true;
  using type = uint16_t;
  const uint16_t *W;
  int ld;
  __device__ uint16_t operator()(int n, int k, int) const { return W[(int64_t)n * ld + k]; }
};

struct CSignalY {
  float *y;
  const float *bias;
  int m, O;
  __device__ void operator()(int64_t r, int o, int, float v) const {
    const int64_t vx = r / m;
    const int i = (int)(r - vx * m);
    if (bias) v += bias[o];
    y[(vx * O + o) * m + i] = v;
  }
};

int launch_lsc_contract_fwd(const float *X, const float *W, const uint16_t *Wh, const float *bias, float *y,
                            int64_t V, int C, int O, int m, int T, dlm_precision prec, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t M = V * m;
  const int K = C * T;
  ANbhd al{X, m, T, C};
  CSignalY cs{y, bias, m, O};
  const Shape sh = pick_shape(O);
  if (prec == DLM_BF16) return run_gemm<kOpContractFwd>(al, BWeightH{Wh, K}, cs, M, O, K, 1, 0, prec, st, sh);
  return run_gemm<kOpContractFwd>(al, BWeightF{W, K}, cs, M, O, K, 1, 0, prec, st, sh);
}

// dy as the A operand: row r = (v, i), column k = o; consecutive rows are
// consecutive in memory.
struct ADy {
  static constexpr bool kContig = false;
  const float *dy;
  int m, O;
  __device__ float operator()(int64_t r, int o, int) const {
    const int64_t v = r / m;
    const int i = (int)(r - v * m);
    return dy[(v * O + o) * m + i];
  }
};

struct CNbhd {
  float *dX;
  int m, T, C;
  __device__ void operator()(int64_t r, int n, int, float val) const {
    const int64_t v = r / m;
    const int i = (int)(r - v * m);
    const int c = n / T, t = n - c * T;
    const int64_t P = (int64_t)m * T;
    dX[(v * C + c) * P + (int64_t)i * T + t] = val;
  }
};

int launch_lsc_contract_bwd_data(const float *dy, const float *Wt, const uint16_t *Wth, float *dX, int64_t V, int C,
                                 int O, int m, int T, dlm_precision prec, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t M = V * m;
  const int N = C * T;
  ADy al{dy, m, O};
  CNbhd cs{dX, m, T, C};
  const Shape sh = pick_shape(N);
  if (prec == DLM_BF16) return run_gemm<kOpContractBwdData>(al, BWeightH{Wth, O}, cs, M, N, O, 1, 0, prec, st, sh);
  return run_gemm<kOpContractBwdData>(al, BWeightF{Wt, O}, cs, M, N, O, 1, 0, prec, st, sh);
}

// Weight gradient: rows r = (c, t) plus one bias row (r = C*T, value 1),
// columns n = o, reduction k = (v, i) split into `splits` slices.
struct AXt {
  static constexpr bool kContig = false;
  const float *X;
  int m, T, C;
  __device__ float operator()(int64_t r, int k, int) const {
    const int CT = C * T;
    if (r == CT) return 1.0f;
    const int v = k / m, i = k - v * m;
    const int c = (int)r / T, t = (int)r - c * T;
    const int64_t P = (int64_t)m * T;
    return X[((int64_t)v * C + c) * P + (int64_t)i * T + t];
  }
};

struct BDyT {
  static constexpr bool kContig = true;
  using type = float;
  const float *dy;
  int m, O;
  __device__ float operator()(int o, int k, int) const {
    const int v = k / m, i = k - v * m;
    return dy[((int64_t)v * O + o) * m + i];
  }
};

struct CPartial {
  float *part;
  int rows, O;
  __device__ void operator()(int64_t r, int o, int s, float v) const {
    part[((int64_t)s * rows + r) * O + o] = v;
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
  return run_gemm<kOpContractBwdWeight>(AXt{X, m, T, C}, BDyT{dy, m, O}, CPartial{partial, rows, O}, rows, O, (int)Kfull, splits, ksplit,
                  prec, st, pick_shape(O));
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
  using type = float;
  const float *Q;
  int KK;
  __device__ float operator()(int n, int t, int) const { return Q[(int64_t)t * KK + n]; }
};

struct CFold {
  float *Tw, *TwT;
  uint16_t *Twh, *TwTh;
  int C, Ki, Ko, O;
  __device__ void operator()(int64_t r, int n, int, float v) const {
    const int o = (int)r / C, c = (int)r - o * C;
    const int k = n / Ki, j = n - k * Ki;
    const int64_t row = (int64_t)o * Ko + k, col = (int64_t)c * Ki + j;
    const int64_t a = row * ((int64_t)C * Ki) + col, b = col * ((int64_t)O * Ko) + row;
    Tw[a] = v;
    TwT[b] = v;
    if (Twh) Twh[a] = to_bf16_bits(v);
    if (TwTh) TwTh[b] = to_bf16_bits(v);
  }
};

int launch_lsc_fold(const float *W, const float *Q, int C, int O, int T, int Ki, int Ko, float *Tw, float *TwT,
                    uint16_t *Twh, uint16_t *TwTh, void *stream) {
  const int KK = Ko * Ki;
  return run_gemm<kOpFoldMake>(ARowMajor{W, nullptr, T, 0}, BQt{Q, KK}, CFold{Tw, TwT, Twh, TwTh, C, Ki, Ko, O},
                               (int64_t)O * C, KK, T, 1, 0, DLM_FP32, (hipStream_t)stream, pick_shape(KK));
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
struct AGradT {
  static constexpr bool kContig = false;
  const float *g, *mask;
  int M;
  __device__ float operator()(int64_t m, int v, int) const {
    const int64_t o = (int64_t)v * M + m;
    float x = g[o];
    if (mask) x = mask[o] > 0.0f ? x : 0.0f;
    return x;
  }
};

struct BActT {
  static constexpr bool kContig = false;
  using type = float;
  const float *a;
  int CK;
  __device__ float operator()(int n, int v, int) const { return n < CK ? a[(int64_t)v * CK + n] : 1.0f; }
};

// transposed orientation: activations on the row side, gradient on the column side
struct AActT {
  static constexpr bool kContig = false;
  const float *a;
  int CK;
  __device__ float operator()(int64_t n, int v, int) const { return n < CK ? a[(int64_t)v * CK + n] : 1.0f; }
};

struct BGradT {
  static constexpr bool kContig = false;
  using type = float;
  const float *g, *mask;
  int M;
  __device__ float operator()(int m, int v, int) const {
    const int64_t o = (int64_t)v * M + m;
    float x = g[o];
    if (mask) x = mask[o] > 0.0f ? x : 0.0f;
    return x;
  }
};

template <bool TRANS>
struct CPartial2 {
  float *part;
  int M, N1;
  __device__ void operator()(int64_t r, int c, int s, float v) const {
    if constexpr (TRANS)
      part[((int64_t)s * M + c) * N1 + r] = v;
    else
      part[((int64_t)s * M + r) * N1 + c] = v;
  }
};

static int split_len(int64_t K, int splits) {
  const int bk = 32;
  int ks = (int)((K + splits - 1) / splits);
  return (ks + bk - 1) / bk * bk;
}

int fold_grad_splits(int64_t V, int M, int N1) {
  const int64_t tiles = ((std::max(M, N1) + 63) / 64) * ((std::min(M, N1) + 63) / 64);
  int s = (int)std::min<int64_t>(64, std::max<int64_t>(1, (4096 + tiles - 1) / tiles));
  s = (int)std::min<int64_t>(s, std::max<int64_t>(1, V / 512));
  while (s > 1 && (V + split_len(V, s) - 1) / split_len(V, s) != s) --s;
  return s;
}

int launch_lsc_fold_grad(const float *da_out, const float *mask, const float *a_in, int64_t V, int M, int CK,
                         int splits, float *partial, dlm_precision prec, void *stream) {
  const int N1 = CK + 1;
  const int ks = split_len(V, splits);
  if ((V + ks - 1) / ks != splits) return -2;
  hipStream_t st = (hipStream_t)stream;
  if (M >= N1)
    return run_gemm<kOpFoldGrad>(AGradT{da_out, mask, M}, BActT{a_in, CK}, CPartial2<false>{partial, M, N1}, M, N1,
                                 (int)V, splits, ks, prec, st, Shape::S64);
  return run_gemm<kOpFoldGrad>(AActT{a_in, CK}, BGradT{da_out, mask, M}, CPartial2<true>{partial, M, N1}, N1, M,
                               (int)V, splits, ks, prec, st, Shape::S64);
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

// dTw viewed per (o,c): row r = (o,c), column k = (kk,j) of the Ko x Ki block.
struct AUnfold {
  static constexpr bool kContig = true;
  const float *dTw;
  int C, Ki, Ko, N1;
  __device__ float operator()(int64_t r, int k, int) const {
    const int o = (int)r / C, c = (int)r - o * C;
    const int kk = k / Ki, j = k - kk * Ki;
    return dTw[((int64_t)o * Ko + kk) * N1 + (int64_t)c * Ki + j];
  }
};

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
  int rc = run_gemm<kOpFoldUnfold>(AUnfold{dTw, C, Ki, Ko, N1}, BTableF{Q, 0, Ko * Ki}, CRowMajor{dW, T, 0, 0, nullptr},
                                   (int64_t)O * C, T, Ko * Ki, 1, 0, DLM_FP32, st, pick_shape(T));
  if (rc != 0 || !db) return rc;
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
// partial; a single block then adds the partials in index order.
__global__ __launch_bounds__(256) void mse_partial_kernel(const float *pred, const float *target, int64_t n,
                                                          float *dpred, float *partials, float scale) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = pred[i] - target[i];
    s += d * d;
    if (dpred) dpred[i] = scale * d;
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
  hipLaunchKernelGGL(mse_partial_kernel, dim3(nblocks), dim3(256), 0, st, pred, target, n, dpred, partials,
                     (float)(2.0 / (double)n));
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, loss, (float)(1.0 / (double)n));
  return hipGetLastError() == hipSuccess ? 0 : -1;
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
