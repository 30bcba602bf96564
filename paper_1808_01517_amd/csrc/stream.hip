// Streaming GEMM core for the large contractions of the folded LSC layer
// (Sec. 2.3: resampling, cyclic-kernel dot and refit composed into one
// matrix per layer) and its adjoints.
//
// These contractions do 15-60 flop per HBM byte: far below the bf16
// matrix-core ridge (~300 flop/B), so the BF16 form is bandwidth-bound,
// and above the fp32 ridge (~20 flop/B), so the FP32 form is bound by the
// fp32 MFMA rate.  Both want the operand traffic off the register file and
// out of the way of the matrix cores:
//
// * Operands travel from global memory straight into LDS with
//   global_load_lds_dword / _dwordx4 (no register staging), through a ring of
//   NS stages, so NS-1 slices of 32 k are in flight while one is multiplied.
// * Float32 operands stay float32 in LDS and are rounded to bfloat16 (RNE)
//   when a wave reads its MFMA fragment; bfloat16 tables and activations
//   stored in bfloat16 are copied as is (the same values either way).
//   A stage wholly inside the reduction range copies from one wave-uniform
//   base address plus per-lane 32-bit offsets computed once per block, so
//   the loop spends a scalar add and one instruction per copy.  In the one
//   stage where the range ends, lanes at or beyond the end copy zeros from a
//   4 KB zero buffer (spread over lanes, so no single cache line is hot).
//   LDS thus holds the exact operands and fragment reads need no
//   conditionals.  Rows beyond the matrix are clamped to valid rows (their
//   outputs are never stored).  The weight gradient's ones row (its bias
//   term) is one of them: in FP32 the wave whose tiles hold it sums the
//   other operand's fragments as they pass, and the epilogue stores those
//   sums in place of the row's MFMA results; BF16 sets the row's fragments
//   to ones in registers.
// * Every LDS layout is swizzled so that fragment reads avoid bank
//   conflicts while each DMA instruction still fills 64 consecutive slots
//   (the hardware writes lane i of an instruction to base + i * size).
// * Waits are explicit: s_waitcnt vmcnt(n) for the slice about to be used,
//   then a barrier.  A slot is refilled only after the barrier that follows
//   its last read by every wave.
// * The epilogue's side inputs (bias, ReLU mask) are loaded behind the last
//   DMA, after the second-to-last stage's wait, when they fit in registers;
//   only the last stage's wait then covers them.
//
// MFMA, B fragment first, so each accumulator is the transposed 16 x 16
// tile (a lane holds four consecutive output columns of one row), the same
// epilogue as the register-staged cores:
//   BF16: v_mfma_f32_16x16x32_bf16, lane (q16, g4) holds k = 8 g4 .. 8 g4 + 7;
//   FP32: v_mfma_f32_16x16x4_f32 over each 16-k group: lane (q16, g4) reads
//         k = 4 g4 .. 4 g4 + 3 of the group at once and MFMA j takes k = 4 g4
//         + j (a permutation of the reduction index, the same for A and B).
// The ring is three stages deep in BF16 (latency-bound) and two in FP32
// (one stage of fp32 MFMA work outlasts a load).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "gemm_common.h"
#include "internal.h"

namespace dlm {
namespace streaming {

constexpr int SBK = 32;  // reduction entries per stage (one MFMA deep)

#ifndef DLM_ASTAT
#define DLM_ASTAT 1  // the short-reduction kernel below (0: tiled core only)
#endif

#define DLM_LDS(p) ((__attribute__((address_space(3))) void *)(p))

// Source of the DMA lanes that fill padding (zero-initialised, never written).
__device__ __attribute__((aligned(16))) float kZeros[1024];
__device__ __forceinline__ const float *zeros_for(int s) { return kZeros + ((s & 255) << 2); }

// Wait until at most N vector-memory operations of this wave are pending and
// its LDS operations are complete, then join the workgroup barrier.
template <int N>
__device__ __forceinline__ void wait_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// One DMA lane copy of SIZE bytes from global memory into LDS; the LDS
// address of lane i is lds + i * SIZE (lds must be wave-uniform).  The
// builtin is only legal in the gfx950 device pass (the 16-byte form is a
// gfx950 instruction), so the host pass sees an empty body.
template <int SIZE>
__device__ __forceinline__ void dma_to_lds(const void *src, void *lds) {
  static_assert(SIZE == 4 || SIZE == 16, "DMA lane size");
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (SIZE == 16) __builtin_amdgcn_global_load_lds(src, DLM_LDS(lds), 16, 0, 0);
  else __builtin_amdgcn_global_load_lds(src, DLM_LDS(lds), 4, 0, 0);
#endif
}

__device__ __forceinline__ bf16x8 to_bf16x8(floatx4 lo, floatx4 hi) {
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = (__bf16)lo[e];
    r[4 + e] = (__bf16)hi[e];
  }
  return r;
}

// ------------------------------------------------------ streamed operands
// Each operand type gives, for a tile of BR rows and one stage of SBK
// reduction entries: bytes() of LDS, slots() DMA lanes of kUnit bytes,
// base(r0, k0) + lane_off(slot, r0) the global address slot `slot` copies,
// k_of(slot) its reduction index within the stage (for zero padding), and
// frag() the bfloat16 MFMA fragment of 16 rows (row group rg) x 8 k for lane
// (q16, g4): row rg*16 + q16, k = 8*g4 .. 8*g4 + 7.

// k-contiguous float32: element (r, k) at p[r * ld + k], valid for r < rows,
// k < kend.  LDS: [BR][32] floats, 4-float chunk c of row r stored at chunk
// c ^ (r & 7).  VEC (16-byte lanes) needs 16-byte aligned rows and kend % 4
// == 0, so a chunk lies wholly inside or wholly beyond the range.
template <bool VEC>
struct SKc {
  const float *p;
  int64_t ld, rows;
  static constexpr int kUnit = VEC ? 16 : 4;
  static constexpr bool kOnes = false;
  template <int BR>
  static constexpr int bytes() { return BR * SBK * 4; }
  template <int BR>
  static constexpr int slots() { return bytes<BR>() / kUnit; }
  // Stage with every k inside the range: lane s copies from
  // base(r0, k0) + lane_off(s, r0) bytes.
  __device__ const char *base(int64_t r0, int k0) const {
    return reinterpret_cast<const char *>(p + r0 * ld + k0);
  }
  template <int BR>
  __device__ uint32_t lane_off(int s, int64_t r0) const {
    int r, k;
    if constexpr (VEC) {
      r = s >> 3;
      k = ((s & 7) ^ (r & 7)) << 2;
    } else {
      r = s >> 5;
      k = ((((s >> 2) & 7) ^ (r & 7)) << 2) | (s & 3);
    }
    const int64_t gr = r0 + r < rows ? r0 + r : rows - 1;
    return (uint32_t)(((gr - r0) * ld + k) * 4);
  }
  // reduction index (within the stage) of slot s: its first, for 16-byte lanes
  template <int BR>
  __device__ static int k_of(int s) {
    if constexpr (VEC) return ((s & 7) ^ ((s >> 3) & 7)) << 2;
    else return ((((s >> 2) & 7) ^ ((s >> 5) & 7)) << 2) | (s & 3);
  }
  __device__ void bind(int64_t) {}
  template <int BR>
  __device__ bf16x8 frag(const char *lds, int rg, int q16, int g4) const {
    const int r = rg * 16 + q16;
    const float *row = reinterpret_cast<const float *>(lds) + r * SBK;
    const floatx4 lo = *reinterpret_cast<const floatx4 *>(row + (((2 * g4) ^ (r & 7)) << 2));
    const floatx4 hi = *reinterpret_cast<const floatx4 *>(row + (((2 * g4 + 1) ^ (r & 7)) << 2));
    return to_bf16x8(lo, hi);
  }
  // float32 values k = 16 h + 4 g4 .. + 3 of the stage for row rg*16 + q16
  template <int BR>
  __device__ floatx4 frag4(const char *lds, int rg, int q16, int g4, int h) const {
    const int r = rg * 16 + q16;
    const float *row = reinterpret_cast<const float *>(lds) + r * SBK;
    return *reinterpret_cast<const floatx4 *>(row + (((4 * h + g4) ^ (r & 7)) << 2));
  }
};

// Row-contiguous float32: element (r, k) at p[k * ld + r], valid for
// r < rows, k < kend; with ONES, row `ones` (if >= 0) stands for a row of
// ones (bind() locates it in the block's tile).  VEC needs 16-byte aligned k-lines and rows % 4 == 0.
// LDS: a stage (32 k x BR rows) in windows of 16 rows of one k (64 bytes).
// With k = 16 h + 4 q + j (h = bit 4, q = bits 2-3, j = bits 0-1) and
// NG = BR / 16 row groups, window (k, rg) sits at window index
// 4 ((4 h + j) NG + rg) + c(k), c(k) = (bit2 ^ bit3) + 2 (bit3 ^ bit4).
// The four k of one fragment read (FP32: 16 h + 4 g4 + j over g4; BF16:
// 8 g4 + e over g4) have four different c, so a 32-bit read covers 64
// banks once; and the two k of each half-wave (g4 = 0, 1 and 2, 3) have c
// of different parity, so each half-wave also covers 32 banks once.  (A
// 32-bit LDS read behaves as 32 banks per half-wave here: with c = 2 bit3
// + (bit2 ^ bit4), conflict-free over 64 banks, the BF16 reads measured
// 2.3e8 conflict cycles per weight gradient.)  A DMA instruction fills
// whole windows: 4 k x 16 rows (4-byte lanes) or 4 k x 64 rows (16-byte
// lanes).
template <bool VEC, bool ONES>
struct SRc {
  const float *p;
  int64_t ld, rows, ones;
  int orel = -1;  // row `ones` relative to the bound tile, -1 if outside
  static constexpr int kUnit = VEC ? 16 : 4;
  static constexpr bool kOnes = ONES;  // the operand may hold the ones row
  template <int BR>
  static constexpr int bytes() { return BR * SBK * 4; }
  template <int BR>
  static constexpr int slots() { return bytes<BR>() / kUnit; }
  // rows beyond the matrix (the ones row among them) copy the last row, or
  // for 16-byte lanes the last chunk
  static constexpr int kLast = VEC ? 4 : 1;
  __device__ int64_t clamp(int64_t gr) const { return gr < rows ? gr : rows - kLast; }
  // A tile may start at or past the last row (the ones row is row `rows`),
  // so full-stage addresses are taken relative to the clamped tile start,
  // never above any clamped row: offsets stay non-negative.
  __device__ int64_t rbase(int64_t r0) const { return r0 < rows - kLast ? r0 : rows - kLast; }
  __device__ const char *base(int64_t r0, int k0) const {
    return reinterpret_cast<const char *>(p + (int64_t)k0 * ld + rbase(r0));
  }
  // (k, first row) within the stage and tile of slot s
  template <int BR>
  __device__ static void slot_kr(int s, int &k, int &r) {
    static_assert(BR % 16 == 0, "row tile");
    constexpr int NG = BR / 16;
    const int w = VEC ? s >> 2 : s >> 4;
    const int t = VEC ? (s & 3) << 2 : s & 15;
    const int idx = w >> 2, c = w & 3;
    const int hj = idx / NG, rg = idx - hj * NG;
    const int h = hj >> 2, j = hj & 3;
    const int b3 = (c >> 1) ^ h, b2 = (c & 1) ^ b3;  // c = (b2 ^ b3) + 2 (b3 ^ h)
    k = 16 * h + 8 * b3 + 4 * b2 + j;
    r = 16 * rg + t;
  }
  template <int BR>
  __device__ uint32_t lane_off(int s, int64_t r0) const {
    int k, r;
    slot_kr<BR>(s, k, r);
    return (uint32_t)(((int64_t)k * ld + (clamp(r0 + r) - rbase(r0))) * 4);
  }
  template <int BR>
  __device__ static int k_of(int s) {
    int k, r;
    slot_kr<BR>(s, k, r);
    return k;
  }
  __device__ void bind(int64_t r0) {
    const int64_t ro = ones - r0;
    orel = ones >= 0 && ro >= 0 && ro < 1 << 20 ? (int)ro : -1;
  }
  // Element (k = 16 h + 4 q + j, row 16 rg + q16) sits at float
  // 64 ((4 h + j) NG + rg) + 16 c(k) + q16: a per-lane part (h, c, q16), a
  // wave-uniform part (rg) and a constant (j), added in that order so that
  // the constant stays an instruction offset.
  // BF16 fragments of the ones row are set to ones here (FP32 sums instead)
  __device__ bool ones_lane(int rg, int q16) const { return ONES && orel >= 0 && orel == 16 * rg + q16; }
  template <int BR>
  __device__ bf16x8 frag(const char *lds, int rg, int q16, int g4) const {
    constexpr int NG = BR / 16;
    const float *t = reinterpret_cast<const float *>(lds) + 64 * rg;
    // k = 8 g4 + e: h = g4 >> 1, bit 3 = g4 & 1, bit 2 = 0 (lo) or 1 (hi)
    const int h = g4 >> 1, b3 = g4 & 1, c2 = 2 * (b3 ^ h);
    const float *lo_p = t + (256 * NG * h + 16 * (b3 + c2) + q16);
    const float *hi_p = t + (256 * NG * h + 16 * ((1 ^ b3) + c2) + q16);
    floatx4 lo, hi;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lo[e] = lo_p[64 * NG * e];
      hi[e] = hi_p[64 * NG * e];
    }
    bf16x8 v = to_bf16x8(lo, hi);
    if (ones_lane(rg, q16))
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)1.0f;
    return v;
  }
  template <int BR>
  __device__ floatx4 frag4(const char *lds, int rg, int q16, int g4, int h) const {
    constexpr int NG = BR / 16;
    // k = 16 h + 4 g4 + j: bit 2 = g4 & 1, bit 3 = g4 >> 1
    const int c = ((g4 & 1) ^ (g4 >> 1)) + 2 * ((g4 >> 1) ^ h);
    const float *p0 = reinterpret_cast<const float *>(lds) + 64 * rg + (256 * NG * h + 16 * c + q16);
    floatx4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = p0[64 * NG * j];
    return v;
  }
};

// bfloat16 table: element (r, k) at p[r * ldp + k], ldp a multiple of 32,
// entries k >= K stored as zeros.  LDS: [BR][32] bf16, 16-byte chunk c
// (8 k) of row r stored at chunk c ^ ((r >> 1) & 3).
struct SKh {
  const uint16_t *p;
  int64_t ldp, rows;
  static constexpr int kUnit = 16;
  static constexpr bool kOnes = false;
  template <int BR>
  static constexpr int bytes() { return BR * SBK * 2; }
  template <int BR>
  static constexpr int slots() { return bytes<BR>() / kUnit; }
  __device__ const char *base(int64_t r0, int k0) const {
    return reinterpret_cast<const char *>(p + r0 * ldp + k0);
  }
  template <int BR>
  __device__ uint32_t lane_off(int s, int64_t r0) const {
    const int r = s >> 2, c = (s & 3) ^ ((r >> 1) & 3);
    const int64_t gr = r0 + r < rows ? r0 + r : rows - 1;
    return (uint32_t)(((gr - r0) * ldp + 8 * c) * 2);
  }
  // the table is zero-padded to a whole stage: no copy lies beyond the range
  template <int BR>
  __device__ static int k_of(int) { return 0; }
  __device__ void bind(int64_t) {}
  template <int BR>
  __device__ bf16x8 frag(const char *lds, int rg, int q16, int g4) const {
    const int r = rg * 16 + q16;
    return *reinterpret_cast<const bf16x8 *>(lds + r * 64 + ((g4 ^ ((r >> 1) & 3)) << 4));
  }
};

// bfloat16 k-contiguous rows (activations stored in bfloat16): element
// (r, k) at p[r * ldp + k], valid for r < rows, k < kend; ldp a multiple of 8
// with 16-byte aligned rows and kend a multiple of 8, so a 16-byte chunk
// (8 k) lies wholly inside or wholly beyond the range.  LDS as SKh.
struct SKb : SKh {
  template <int BR>
  __device__ static int k_of(int s) {
    const int r = s >> 2;
    return 8 * ((s & 3) ^ ((r >> 1) & 3));
  }
};

// bfloat16 row-contiguous (activations stored in bfloat16, reduced over
// voxels): element (r, k) at p[k * ld + r], valid for r < rows, k < kend;
// with ONES, row `ones` (if >= 0) stands for a row of ones, as in SRc.  A 16-byte
// lane copies 8 consecutive rows of one k, so ld and rows are multiples of 8
// and k-lines are 16-byte aligned.  LDS: [32][BR] bf16; the 8-row chunk c of
// k-line k sits at chunk (c + 2 g(k)) mod (BR / 8), g(k) = (k >> 3) & 3, so
// the four k of one fragment read (8 g4 + e, g4 = 0..3) land 32 bytes apart.
template <bool ONES>
struct SRb {
  const uint16_t *p;
  int64_t ld, rows, ones;
  int orel = -1;
  static constexpr int kUnit = 16;
  static constexpr bool kOnes = ONES;
  template <int BR>
  static constexpr int bytes() { return BR * SBK * 2; }
  template <int BR>
  static constexpr int slots() { return bytes<BR>() / kUnit; }
  __device__ static int rot(int k) { return 2 * ((k >> 3) & 3); }
  // rows beyond the matrix copy its last 8-row chunk (never stored)
  __device__ int64_t clamp(int64_t gr) const { return gr < rows ? gr : rows - 8; }
  __device__ int64_t rbase(int64_t r0) const { return r0 < rows - 8 ? r0 : rows - 8; }
  __device__ const char *base(int64_t r0, int k0) const {
    return reinterpret_cast<const char *>(p + (int64_t)k0 * ld + rbase(r0));
  }
  template <int BR>
  __device__ uint32_t lane_off(int s, int64_t r0) const {
    static_assert(BR % 16 == 0 && BR / 8 > 6, "row tile");
    constexpr int NC = BR / 8;
    const int k = s / NC;
    int c = s - k * NC - rot(k);
    if (c < 0) c += NC;
    return (uint32_t)(((int64_t)k * ld + (clamp(r0 + 8 * c) - rbase(r0))) * 2);
  }
  template <int BR>
  __device__ static int k_of(int s) { return s / (BR / 8); }
  __device__ void bind(int64_t r0) {
    const int64_t ro = ones - r0;
    orel = ones >= 0 && ro >= 0 && ro < 1 << 20 ? (int)ro : -1;
  }
  // Lane (q16, g4) needs row r at k = 8 g4 .. + 7, eight k-lines apart.  It
  // reads the whole dword holding rows r & ~1 and r | 1 of each k-line (the
  // lanes of rows 2i and 2i + 1 read the same dword: a broadcast) and keeps
  // its half with one byte permute per pair of k-lines, in place of sixteen
  // 16-bit reads into register halves (measured: 4% faster weight gradient).
  template <int BR>
  __device__ bf16x8 frag(const char *lds, int rg, int q16, int g4) const {
    constexpr int NC = BR / 8;
    const uint32_t *t = reinterpret_cast<const uint32_t *>(lds);
    const int r = rg * 16 + q16, c = r >> 3, w = r & 7;
    int pc = c + 2 * g4;  // rot(8 g4 + e) = 2 g4 for every e
    if (pc >= NC) pc -= NC;
    const uint32_t *p = t + ((8 * g4) * BR + pc * 8 + (w & ~1)) / 2;
    // bytes of the lane's half from two dwords (lo halves, or hi halves)
    const uint32_t sel = (w & 1) ? 0x07060302u : 0x05040100u;
    uint32_t d[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) d[e] = p[e * (BR / 2)];
    uint32_t u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = __builtin_amdgcn_perm(d[2 * i + 1], d[2 * i], sel);
    bf16x8 v = __builtin_bit_cast(bf16x8, u);
    if (ONES && orel >= 0 && orel == r)  // the ones row (a BF16 fragment: set here)
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)1.0f;
    return v;
  }
};

// ------------------------------------------------------------------ core
template <int BM_, int BN_, int WM_, int WN_, int NS_>
struct SCfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, NS = NS_;
  static constexpr int TM = BM / (WM * 16), TN = BN / (WN * 16);
  static_assert(WM * WN == 4, "four waves per block");
  static_assert(TM * WM * 16 == BM && TN * WN * 16 == BN, "tile shape");
  static_assert(NS >= 2 && NS <= 4, "ring depth");
};

// Sums standing in for the weight gradient's ones row in FP32.  The MFMAs
// read that row's slots as copied (a clamped row), so the wave whose tiles
// hold the row adds up the other operand's fragments instead: rs[i] the
// k-sums of its A rows (ones row in B: an output column), cs[j] those of
// its B rows (ones row in A: an output row), per lane over the lane's k;
// the epilogue finishes the sums across lanes and stores them in place of
// the row's MFMA results.  Flags are wave-uniform.  (Setting the row's
// fragments to ones instead costs a select per fragment value: 44 per 72
// MFMAs in the 128 x 144 tile.  BF16, bound by memory rather than by the
// matrix cores, keeps those selects, which measured faster there than the
// sums.)
template <class CF>
struct OnesSum {
  bool a_on = false, b_on = false;  // ones row in this wave's A / B tiles
  int rel = 0;                      // its row, relative to the wave's first row on that side
  float rs[CF::TM], cs[CF::TN];
};

__device__ __forceinline__ float sum4(floatx4 v) { return (v[0] + v[1]) + (v[2] + v[3]); }

// One stage (32 k) of MFMAs for a wave's TM x TN tiles.  FP32 runs the
// stage's nh (1 or 2) groups of 16 k through one MFMA sequence (a last stage
// ending within its first group needs one); BF16 ignores nh.
template <class CF, bool F32, class AO, class BO>
__device__ __forceinline__ void mma_stage(const AO &ao, const BO &bo, const char *sa, const char *sb, int wm, int wn,
                                          int q16, int g4, int nh, floatx4 (&acc)[CF::TM][CF::TN],
                                          OnesSum<CF> &os) {
  constexpr int BM = CF::BM, BN = CF::BN;
  if constexpr (F32) {
#pragma unroll 1
    for (int h = 0; h < nh; ++h) {
      floatx4 a[CF::TM], b[CF::TN];
#pragma unroll
      for (int i = 0; i < CF::TM; ++i) a[i] = ao.template frag4<BM>(sa, wm * CF::TM + i, q16, g4, h);
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) b[j] = bo.template frag4<BN>(sb, wn * CF::TN + j, q16, g4, h);
      if constexpr (BO::kOnes)  // every wave of a tile with the ones column: no branch
#pragma unroll
        for (int i = 0; i < CF::TM; ++i) os.rs[i] += sum4(a[i]);
      if constexpr (AO::kOnes)
        if (os.a_on)
#pragma unroll
          for (int j = 0; j < CF::TN; ++j) os.cs[j] += sum4(b[j]);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
#pragma unroll
          for (int j = 0; j < CF::TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j][jj], a[i][jj], acc[i][j], 0, 0, 0);
    }
  } else {
    bf16x8 a[CF::TM], b[CF::TN];
#pragma unroll
    for (int i = 0; i < CF::TM; ++i) a[i] = ao.template frag<BM>(sa, wm * CF::TM + i, q16, g4);
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) b[j] = bo.template frag<BN>(sb, wn * CF::TN + j, q16, g4);
#pragma unroll
    for (int i = 0; i < CF::TM; ++i)
#pragma unroll
      for (int j = 0; j < CF::TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
  }
}

// Start the ones-row sums of a wave: locate the row in its A or B tiles.
template <class CF, class AO, class BO>
__device__ __forceinline__ void ones_begin(const AO &aw, const BO &bw, int wm, int wn, OnesSum<CF> &os) {
  static_assert(!(AO::kOnes && BO::kOnes), "one operand with a ones row");
  if constexpr (AO::kOnes) {
    os.rel = aw.orel - wm * CF::TM * 16;
    os.a_on = aw.orel >= 0 && os.rel >= 0 && os.rel < CF::TM * 16;
  }
  if constexpr (BO::kOnes) {
    os.rel = bw.orel - wn * CF::TN * 16;
    os.b_on = bw.orel >= 0 && os.rel >= 0 && os.rel < CF::TN * 16;
  }
#pragma unroll
  for (int i = 0; i < CF::TM; ++i) os.rs[i] = 0.f;
#pragma unroll
  for (int j = 0; j < CF::TN; ++j) os.cs[j] = 0.f;
}

// Finish the sums across the four lanes of a row (lanes q16 + 16 g4 hold
// disjoint k) and store them in place of the ones row's MFMA results: a
// ones row in B is output column `rel` (lane (q16, g4) holds columns
// 4 g4 .. 4 g4 + 3 of each 16-column tile), a ones row in A is output row
// `rel`, whose column n of tile j is the sum lane q16 = n holds.
template <class CF>
__device__ __forceinline__ void ones_end(OnesSum<CF> &os, floatx4 (&acc)[CF::TM][CF::TN], int q16, int g4) {
  if (os.b_on) {
    const int jo = os.rel >> 4, go = (os.rel & 15) >> 2, eo = os.rel & 3;
#pragma unroll
    for (int i = 0; i < CF::TM; ++i) {
      float r = os.rs[i];
      r += __shfl_xor(r, 16);
      r += __shfl_xor(r, 32);
#pragma unroll
      for (int j = 0; j < CF::TN; ++j)
        if (j == jo && g4 == go)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (e == eo) acc[i][j][e] = r;
    }
  }
  if (os.a_on) {
    const int io = os.rel >> 4, qo = os.rel & 15;
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) {
      float c = os.cs[j];
      c += __shfl_xor(c, 16);
      c += __shfl_xor(c, 32);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = __shfl(c, 4 * g4 + e);
#pragma unroll
        for (int i = 0; i < CF::TM; ++i)
          if (i == io && q16 == qo) acc[i][j][e] = v;
      }
    }
  }
}

// Side inputs (bias of the lane's columns, mask of its elements) of a
// wave's tiles, loaded ahead of the epilogue when they fit in registers
// (at most 12 tiles per wave).
template <class CF, class CS>
struct SidePre {
  static constexpr bool kOn = CS::kSide && CF::TM * CF::TN <= 12;
  floatx4 cb[CF::TN];
  floatx4 em[CF::TM][CF::TN];
};

template <class CF, class CS>
__device__ __forceinline__ void load_side(const CS &cs, SidePre<CF, CS> &sp, int64_t M, int N, int64_t m0, int n0,
                                          int wm, int wn, int q16, int g4, int z) {
#pragma unroll
  for (int j = 0; j < CF::TN; ++j) {
    const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
    sp.cb[j] = n + 3 < N ? cs.colside(n) : floatx4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int i = 0; i < CF::TM; ++i) {
    const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) {
      const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
      sp.em[i][j] = r < M && n + 3 < N ? cs.elside(r, n, z) : floatx4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// Store a consumer wave's tiles: lane (q16, g4) holds row m0 + (wm*TM+i)*16
// + q16 and columns n0 + (wn*TN+j)*16 + 4 g4 .. + 3 of tile (i, j).
template <class CF, class CS>
__device__ __forceinline__ void store_tiles(const CS &cs, const floatx4 (&acc)[CF::TM][CF::TN], int64_t M, int N,
                                            int64_t m0, int n0, int wm, int wn, int q16, int g4, int z,
                                            const SidePre<CF, CS> &sp) {
  if constexpr (SidePre<CF, CS>::kOn) {
#pragma unroll
    for (int i = 0; i < CF::TM; ++i) {
      const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
      if (r >= M) continue;
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) {
        const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
        if (n + 3 < N) {
          cs.store4s(r, n, z, acc[i][j], sp.cb[j], sp.em[i][j]);
        } else {
          for (int q = 0; q < 4; ++q)
            if (n + q < N) cs(r, n + q, z, acc[i][j][q]);
        }
      }
    }
  } else if constexpr (CS::kSide) {
    // side inputs (bias, mask) of a chunk of tiles first, then its stores;
    // chunks of RG tile rows keep the prefetched values within ~12 tiles
    constexpr int RG = CF::TN >= 12 ? 1 : (12 / CF::TN < CF::TM ? 12 / CF::TN : CF::TM);
    floatx4 cb[CF::TN];
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) {
      const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
      cb[j] = n + 3 < N ? cs.colside(n) : floatx4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int i0 = 0; i0 < CF::TM; i0 += RG) {
      floatx4 em[RG][CF::TN];
#pragma unroll
      for (int ii = 0; ii < RG; ++ii) {
        const int64_t r = m0 + (wm * CF::TM + i0 + ii) * 16 + q16;
#pragma unroll
        for (int j = 0; j < CF::TN; ++j) {
          const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
          em[ii][j] = i0 + ii < CF::TM && r < M && n + 3 < N ? cs.elside(r, n, z) : floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }
      // Let the side loads land before the first store.  Without this the
      // compiler may find one of them still pending at the next stage (on a
      // path that stores nothing, e.g. rows beyond M) and wait there for every
      // outstanding store too.  (vmcnt(0), expcnt and lgkmcnt untouched.)
      __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
      for (int ii = 0; ii < RG; ++ii) {
        const int i = i0 + ii;
        if (i >= CF::TM) break;
        const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
        if (r >= M) continue;
        auto one = [&](int j) {
          const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
          if (n + 3 < N) {
            cs.store4s(r, n, z, acc[i][j], cb[j], em[ii][j]);
          } else {
            for (int q = 0; q < 4; ++q)
              if (n + q < N) cs(r, n + q, z, acc[i][j][q]);
          }
        };
        if constexpr (CS::kPair) {
          // two adjacent tiles per 16-byte store when both lie inside N
          // (a condition uniform over the wave, so every lane swaps)
#pragma unroll
          for (int jp = 0; jp < CF::TN / 2; ++jp) {
            const int j = 2 * jp;
            const int nt = n0 + (wn * CF::TN + j) * 16;
            if (nt + 32 <= N) {
              cs.store_pair(r, nt, g4, acc[i][j], cb[j], em[ii][j], acc[i][j + 1], cb[j + 1], em[ii][j + 1]);
            } else {
              one(j);
              one(j + 1);
            }
          }
          if constexpr (CF::TN % 2 != 0) one(CF::TN - 1);
        } else {
#pragma unroll
          for (int j = 0; j < CF::TN; ++j) one(j);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < CF::TM; ++i) {
      const int64_t r = m0 + (wm * CF::TM + i) * 16 + q16;
      if (r >= M) continue;
#pragma unroll
      for (int j = 0; j < CF::TN; ++j) {
        const int n = n0 + (wn * CF::TN + j) * 16 + 4 * g4;
        if (n + 3 < N) {
          cs.store4(r, n, z, acc[i][j]);
        } else {
          for (int q = 0; q < 4; ++q)
            if (n + q < N) cs(r, n + q, z, acc[i][j][q]);
        }
      }
    }
  }
}

// The stage where the range ends (krem = kend - k0 < SBK reduction entries
// left): lanes whose entries lie beyond it copy zeros instead.
template <int BR, class OPND, int STEP, int NW>
__device__ __forceinline__ void dma_stage_tail(const char *base, const uint32_t (&off)[NW], char *dst, int first,
                                               int lane, int krem) {
  constexpr int NSL = OPND::template slots<BR>();
  constexpr int NI = (NSL + 63) / 64;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int inst = first + STEP * i;
    const int s = inst * 64 + lane;
    if ((NI % STEP == 0 || inst < NI) && (NSL % 64 == 0 || s < NSL)) {
      const void *src = OPND::template k_of<BR>(s) < krem ? (const void *)(base + off[i]) : (const void *)zeros_for(s);
      dma_to_lds<OPND::kUnit>(src, dst + inst * 64 * OPND::kUnit);
    }
  }
}

// Number of DMA instructions of an operand that wave `first` (of `step`)
// issues per stage, at most.
template <int BR, class OPND>
constexpr int dma_per_wave(int step) {
  return ((OPND::template slots<BR>() + 63) / 64 + step - 1) / step;
}

// Byte offsets of the lane's DMA copies within a full stage (loop-invariant).
template <int BR, class OPND, int NW>
__device__ __forceinline__ void dma_offsets(const OPND &op, uint32_t (&off)[NW], int first, int step, int lane,
                                            int64_t r0) {
  constexpr int NSL = OPND::template slots<BR>();
  constexpr int NI = (NSL + 63) / 64;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int inst = first + step * i;
    const int s = inst * 64 + lane;
    off[i] = inst < NI && s < NSL ? op.template lane_off<BR>(s, r0) : 0u;
  }
}

// A full stage: every lane copies from the stage's wave-uniform base plus
// its precomputed offset.  The offset passes through an empty asm inside the
// loop so that its zero extension stays next to the add and the copy is
// selected in the scalar-base + 32-bit vector-offset form (a hoisted 64-bit
// offset would cost a 64-bit add and two registers per copy).
template <int BR, class OPND, int STEP, int NW>
__device__ __forceinline__ void dma_stage_full(const char *base, const uint32_t (&off)[NW], char *dst, int first,
                                               int lane) {
  constexpr int NSL = OPND::template slots<BR>();
  constexpr int NI = (NSL + 63) / 64;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int inst = first + STEP * i;
    if ((NI % STEP == 0 || inst < NI) && (NSL % 64 == 0 || inst * 64 + lane < NSL)) {
      uint32_t o = off[i];
      asm volatile("" : "+v"(o));
      dma_to_lds<OPND::kUnit>(base + o, dst + inst * 64 * OPND::kUnit);
    }
  }
}

// One output tile (and one split-K slice) per block; all four waves issue
// their share of every stage's DMA and compute.  Several blocks per CU keep
// loads in flight while another block multiplies or stores.
template <int OP, class CF, bool F32, class AO, class BO, class CS>
__global__ __launch_bounds__(256) void gemm_stream_kernel(AO ao, BO bo, CS cs, int64_t M, int N, int K, int ksplit,
                                                          int nbM, int nbN, int nz) {
  constexpr int BM = CF::BM, BN = CF::BN;
  constexpr int AB = AO::template bytes<BM>(), BB = BO::template bytes<BN>(), SB = AB + BB;
  constexpr int NIA = (AO::template slots<BM>() + 63) / 64, NIB = (BO::template slots<BN>() + 63) / 64;
  // DMA instructions every wave issues per stage, at least (wave w issues
  // instructions w, w + 4, ...); waits use this count, so a wave with more
  // waits for slightly more than it needs.
  constexpr int NIW = NIA / 4 + NIB / 4;
  // ring depth: two stages in FP32; in BF16 as configured while the pending
  // count fits vmcnt (6 bits)
  constexpr int NS = F32 ? 2 : ((CF::NS - 2) * NIW < 64 ? CF::NS : 2), D = NS - 1;
  __shared__ __attribute__((aligned(16))) char lds[NS * SB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % CF::WM, wn = wave / CF::WM;
  const int q16 = lane & 15, g4 = lane >> 4;
  const TileMap tm(blockIdx.x, nbM, nbN, nz, ksplit > 0);
  const int64_t m0 = (int64_t)tm.mt * BM;
  const int n0 = tm.nt * BN;
  const int z = tm.z;
  int kbeg = 0, kend = K;
  if (ksplit > 0) {
    kbeg = z * ksplit;
    kend = min(K, kbeg + ksplit);
  }
  const int niter = kend > kbeg ? (kend - kbeg + SBK - 1) / SBK : 0;

  AO aw = ao;
  BO bw = bo;
  aw.bind(m0);
  bw.bind(n0);
  OnesSum<CF> os;
  if constexpr (F32 && (AO::kOnes || BO::kOnes)) ones_begin<CF>(aw, bw, wm, wn, os);
  constexpr int NWA = dma_per_wave<BM, AO>(4), NWB = dma_per_wave<BN, BO>(4);
  uint32_t offa[NWA], offb[NWB];
  dma_offsets<BM>(ao, offa, wave, 4, lane, m0);
  dma_offsets<BN>(bo, offb, wave, 4, lane, n0);
  auto issue = [&](int it) {
    char *sa = lds + (it % NS) * SB;
    const int k0 = kbeg + it * SBK;
    if (k0 + SBK <= kend) {
      dma_stage_full<BM, AO, 4>(ao.base(m0, k0), offa, sa, wave, lane);
      dma_stage_full<BN, BO, 4>(bo.base(n0, k0), offb, sa + AB, wave, lane);
    } else {  // the range ends inside this stage: zeros beyond it
      dma_stage_tail<BM, AO, 4>(ao.base(m0, k0), offa, sa, wave, lane, kend - k0);
      dma_stage_tail<BN, BO, 4>(bo.base(n0, k0), offb, sa + AB, wave, lane, kend - k0);
    }
  };

  floatx4 acc[CF::TM][CF::TN];
#pragma unroll
  for (int i = 0; i < CF::TM; ++i)
#pragma unroll
    for (int j = 0; j < CF::TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int s = 0; s < D; ++s)
    if (s < niter) issue(s);
  auto wait_issue = [&](int it) {
    const int after = min(D - 1, niter - 1 - it);  // stages issued after this one
    if constexpr (D >= 3) {
      if (after >= 2) wait_barrier<2 * NIW>();
      else if (after == 1) wait_barrier<NIW>();
      else wait_barrier<0>();
    } else if constexpr (D == 2) {
      if (after == 1) wait_barrier<NIW>();
      else wait_barrier<0>();
    } else {
      wait_barrier<0>();
    }
    if (it + D < niter) issue(it + D);
  };
  // Side inputs of the epilogue go out after the wait of the second-to-last
  // stage (behind every DMA, so no stage wait has to cover them except the
  // last, which waits for everything): their latency overlaps the last two
  // stages instead of stalling the stores.
  SidePre<CF, CS> sp;
  const int side_it = niter >= 2 ? niter - 2 : 0;
  for (int it = 0; it < niter; ++it) {
    wait_issue(it);
    if constexpr (SidePre<CF, CS>::kOn)
      if (it == side_it) load_side<CF>(cs, sp, M, N, m0, n0, wm, wn, q16, g4, z);
    const char *sa = lds + (it % NS) * SB;
    const int nh = kend - (kbeg + it * SBK) > 16 ? 2 : 1;
    mma_stage<CF, F32>(aw, bw, sa, sa + AB, wm, wn, q16, g4, nh, acc, os);
  }
  if constexpr (F32 && (AO::kOnes || BO::kOnes)) ones_end<CF>(os, acc, q16, g4);
  if constexpr (SidePre<CF, CS>::kOn)
    if (niter == 0) load_side<CF>(cs, sp, M, N, m0, n0, wm, wn, q16, g4, z);
  store_tiles<CF>(cs, acc, M, N, m0, n0, wm, wn, q16, g4, z, sp);
}

template <int OP, class CF, bool F32, class AO, class BO, class CS>
int run_stream(AO ao, BO bo, CS cs, int64_t M, int N, int K, int Z, int ksplit, hipStream_t st) {
  if (M <= 0 || N <= 0 || Z <= 0) return 0;
  const int64_t nbM = (M + CF::BM - 1) / CF::BM;
  const int nbN = (N + CF::BN - 1) / CF::BN;
  if (nbM * nbN * Z > 0x7fffffff) return -4;
  hipLaunchKernelGGL((gemm_stream_kernel<OP, CF, F32, AO, BO, CS>), dim3((unsigned)(nbM * nbN * Z)), dim3(256), 0, st,
                     ao, bo, cs, M, N, K, ksplit, (int)nbM, nbN, Z);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Row-major output with compile-time side inputs: BIAS adds bias_n[n], MASK
// zeroes entries where omask (indexed as C) <= 0; optional ReLU in between.
// ReLU bit masks (BM): 1 = write bit (stored value > 0) of every output to
// obits, 2 = take the mask (MASK) from mbits instead of omask.  Bit c % 16 of
// word r * ldm + c / 16 belongs to element (r, c); N is a multiple of 16, so
// a 16-column tile is one word, held four bits per lane by the four lanes
// (q16, g4) of one row.
__device__ __forceinline__ floatx4 bits_mask(const uint16_t *mbits, int64_t ldm, int64_t r, int n) {
  const unsigned w = (unsigned)mbits[r * ldm + n / 16] >> (n & 15);
  return floatx4{(float)(w & 1u), (float)((w >> 1) & 1u), (float)((w >> 2) & 1u), (float)((w >> 3) & 1u)};
}
__device__ __forceinline__ void bits_store(uint16_t *obits, int64_t ldm, int64_t r, int n, unsigned nib) {
  // OR the nibbles of the four lanes of this row (lanes q16 + 16 g4): the
  // row swaps exchange lane l with l ^ 16, then with l ^ 32, in registers
  unsigned w = nib << (n & 15);
  const auto s16 = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  w = s16[0] | s16[1];
  const auto s32 = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  w = s32[0] | s32[1];
  if ((n & 15) == 0) obits[r * ldm + n / 16] = (uint16_t)w;
}

// Row-major output with compile-time side inputs: BIAS adds bias_n[n], MASK
// zeroes entries where omask (indexed as C) <= 0, or where the ReLU bit is
// clear (BM = 2); optional ReLU in between; BM = 1 also writes the ReLU bits.
template <bool BIAS, bool MASK, int BM = 0>
struct CRowSide {
  static constexpr bool kSide = BIAS || MASK;
  static constexpr bool kPair = false;
  static constexpr bool kBias = BIAS, kMask = MASK, kHalf = false;
  static constexpr int kBits = BM;
  float *C;
  int64_t ldc;
  int relu;
  const float *bias_n, *omask;
  const uint16_t *mbits = nullptr;
  uint16_t *obits = nullptr;
  int64_t ldm = 0;
  __device__ void operator()(int64_t r, int n, int, float v) const {
    const int64_t o = r * ldc + n;
    if constexpr (BIAS) v += bias_n[n];
    if (relu) v = fmaxf(v, 0.0f);
    if constexpr (MASK) {
      if constexpr (BM == 2) v = (mbits[r * ldm + n / 16] >> (n & 15)) & 1u ? v : 0.0f;
      else v = omask[o] > 0.0f ? v : 0.0f;
    }
    C[o] = v;
  }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    for (int q = 0; q < 4; ++q) (*this)(r, n + q, g, v[q]);
  }
  __device__ floatx4 colside(int n) const {
    if constexpr (BIAS) return ld4(bias_n + n);
    else return floatx4{0.f, 0.f, 0.f, 0.f};
  }
  __device__ floatx4 elside(int64_t r, int n, int) const {
    if constexpr (MASK && BM == 2) return bits_mask(mbits, ldm, r, n);
    else if constexpr (MASK) return ld4(omask + r * ldc + n);
    else return floatx4{1.f, 1.f, 1.f, 1.f};
  }
  __device__ void store4s(int64_t r, int n, int, floatx4 v, floatx4 cb, floatx4 em) const {
    unsigned nib = 0;
    for (int q = 0; q < 4; ++q) {
      if constexpr (BIAS) v[q] += cb[q];
      if (relu) v[q] = fmaxf(v[q], 0.0f);
      if constexpr (MASK) v[q] = em[q] > 0.0f ? v[q] : 0.0f;
      nib |= (v[q] > 0.0f ? 1u : 0u) << q;
    }
    __builtin_memcpy(C + r * ldc + n, &v, 16);
    if constexpr (BM == 1) bits_store(obits, ldm, r, n, nib);
  }
};

// The same with a bfloat16 output (RNE) and a bfloat16 mask: activations and
// their gradients stored in bfloat16.  ldc a multiple of 4, 8-byte aligned rows.
// ReLU bits (BM = 1) describe the stored (rounded) values.
template <bool BIAS, bool MASK, int BM = 0>
struct CRowSideH {
  static constexpr bool kSide = BIAS || MASK;
  static constexpr bool kPair = true;
  static constexpr bool kBias = BIAS, kMask = MASK, kHalf = true;
  static constexpr int kBits = BM;
  uint16_t *C;
  int64_t ldc;
  int relu;
  const float *bias_n;
  const uint16_t *omask;
  const uint16_t *mbits = nullptr;
  uint16_t *obits = nullptr;
  int64_t ldm = 0;
  __device__ static float widen(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }
  __device__ void operator()(int64_t r, int n, int, float v) const {
    const int64_t o = r * ldc + n;
    if constexpr (BIAS) v += bias_n[n];
    if (relu) v = fmaxf(v, 0.0f);
    if constexpr (MASK) {
      if constexpr (BM == 2) v = (mbits[r * ldm + n / 16] >> (n & 15)) & 1u ? v : 0.0f;
      else v = widen(omask[o]) > 0.0f ? v : 0.0f;
    }
    C[o] = to_bf16_bits(v);
  }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    for (int q = 0; q < 4; ++q) (*this)(r, n + q, g, v[q]);
  }
  __device__ floatx4 colside(int n) const {
    if constexpr (BIAS) return ld4(bias_n + n);
    else return floatx4{0.f, 0.f, 0.f, 0.f};
  }
  __device__ floatx4 elside(int64_t r, int n, int) const {
    if constexpr (MASK && BM == 2) {
      return bits_mask(mbits, ldm, r, n);
    } else if constexpr (MASK) {
      uint16_t h[4];
      __builtin_memcpy(h, omask + r * ldc + n, 8);
      return floatx4{widen(h[0]), widen(h[1]), widen(h[2]), widen(h[3])};
    } else {
      return floatx4{1.f, 1.f, 1.f, 1.f};
    }
  }
  __device__ void store4s(int64_t r, int n, int, floatx4 v, floatx4 cb, floatx4 em) const {
    uint16_t h[4];
    unsigned nib = 0;
    for (int q = 0; q < 4; ++q) {
      if constexpr (BIAS) v[q] += cb[q];
      if (relu) v[q] = fmaxf(v[q], 0.0f);
      if constexpr (MASK) v[q] = em[q] > 0.0f ? v[q] : 0.0f;
      h[q] = to_bf16_bits(v[q]);
      nib |= (widen(h[q]) > 0.0f ? 1u : 0u) << q;
    }
    __builtin_memcpy(C + r * ldc + n, h, 8);
    if constexpr (BM == 1) bits_store(obits, ldm, r, n, nib);
  }
  // Tiles j (columns nt..nt+15) and j+1 (nt+16..nt+31) of one row: lane g4
  // holds columns 4 g4..4 g4+3 of both.  A row swap (lane l with l ^ 16,
  // i.e. g4 with g4 ^ 1) hands each even lane its neighbour's half of tile
  // j and each odd lane its neighbour's half of tile j+1, so every lane
  // stores 8 contiguous columns (16 bytes) with one instruction.
  __device__ void store_pair(int64_t r, int nt, int g4, floatx4 v0, floatx4 cb0, floatx4 em0, floatx4 v1,
                             floatx4 cb1, floatx4 em1) const {
    uint32_t w0[2], w1[2];
    unsigned nib0 = 0, nib1 = 0;
    for (int q = 0; q < 4; ++q) {
      if constexpr (BIAS) {
        v0[q] += cb0[q];
        v1[q] += cb1[q];
      }
      if (relu) {
        v0[q] = fmaxf(v0[q], 0.0f);
        v1[q] = fmaxf(v1[q], 0.0f);
      }
      if constexpr (MASK) {
        v0[q] = em0[q] > 0.0f ? v0[q] : 0.0f;
        v1[q] = em1[q] > 0.0f ? v1[q] : 0.0f;
      }
    }
    for (int q = 0; q < 2; ++q) {
      const uint16_t a = to_bf16_bits(v0[2 * q]), b = to_bf16_bits(v0[2 * q + 1]);
      const uint16_t c = to_bf16_bits(v1[2 * q]), d = to_bf16_bits(v1[2 * q + 1]);
      w0[q] = (uint32_t)a | ((uint32_t)b << 16);
      w1[q] = (uint32_t)c | ((uint32_t)d << 16);
      if constexpr (BM == 1) {
        nib0 |= ((widen(a) > 0.0f ? 1u : 0u) | (widen(b) > 0.0f ? 2u : 0u)) << (2 * q);
        nib1 |= ((widen(c) > 0.0f ? 1u : 0u) | (widen(d) > 0.0f ? 2u : 0u)) << (2 * q);
      }
    }
    if constexpr (BM == 1) {
      bits_store(obits, ldm, r, nt + 4 * g4, nib0);
      bits_store(obits, ldm, r, nt + 16 + 4 * g4, nib1);
    }
    const bool odd = g4 & 1;
    uint32_t out[4];
    for (int q = 0; q < 2; ++q) {
      const uint32_t mine = odd ? w0[q] : w1[q];  // the half the partner stores
      const auto x = __builtin_amdgcn_permlane16_swap(mine, mine, false, false);
      // one of the two results is this lane's own value, the other the partner's
      const uint32_t theirs = x[0] ^ x[1] ^ mine;
      if (odd) {
        out[q] = theirs;
        out[2 + q] = w1[q];
      } else {
        out[q] = w0[q];
        out[2 + q] = theirs;
      }
    }
    const int col = odd ? nt + 16 + 4 * (g4 - 1) : nt + 4 * g4;
    __builtin_memcpy(C + r * ldc + col, out, 16);
  }
};

// --------------------------------------------- short-reduction kernel
// C[M][N] = A[M][K] B[N][K]^T for 128 < K <= 160 and N <= 1440: the folded
// forward of a layer with three input channels and the input gradient of a
// layer with three output channels (K = 135, N = 1440 in the three-shell
// stack).  With five k-slices per tile, a block of the tiled core above
// spends most of its life waiting for the loads of its first slices.  Here
// a block keeps its rows of A in registers, loaded once, and sweeps every
// column tile of the table, which streams through an LDS ring by DMA (the
// table stays in L2).  The stores of one tile are in flight while the next
// tiles are loaded and multiplied.
//
// Waits count vector-memory operations in issue order: the DMA of tile t
// is waited for with s_waitcnt vmcnt(n), n = a lower bound of the
// operations the wave issued after it (the stores of the tiles in between,
// the DMA of later tiles).  The block holding the last rows skips the
// stores of rows beyond M, so there the store count is taken as zero.
//
// Side data stay in LDS for the block's whole life: the bias of every
// column (forward), the ReLU bit words of the block's rows (the input
// gradient's mask), or the bit words the forward produces for the block's
// rows, which go to memory once, as one contiguous run, when the block ends.
// Per element the epilogue is the tiled core's (bias, ReLU, mask, RNE
// rounding, bits of the stored value) with the ReLU chosen at compile time;
// the accumulation order is also the tiled core's (k-slices in order; FP32:
// within a slice, k groups of 16, then the four MFMAs of a group), so with
// one accumulator set the results are bitwise the same.
namespace astat {

#ifndef DLM_ASTAT_TM
#define DLM_ASTAT_TM 2
#endif
#ifndef DLM_ASTAT_BN_BF16
#define DLM_ASTAT_BN_BF16 32
#endif
#ifndef DLM_ASTAT_BN_F32
#define DLM_ASTAT_BN_F32 32
#endif
#ifndef DLM_ASTAT_NACC
#define DLM_ASTAT_NACC 1
#endif
#ifndef DLM_ASTAT_D_BF16
#define DLM_ASTAT_D_BF16 3
#endif
#ifndef DLM_ASTAT_D_F32
#define DLM_ASTAT_D_F32 1
#endif

constexpr int TM = DLM_ASTAT_TM;  // 16-row groups per wave
constexpr int BM = 64 * TM;       // rows per block: four waves
constexpr int KS = 5;             // 32-k slices (128 < K <= 160)
constexpr int kMaxN = 1440;       // columns whose side data fit in LDS

// BF16: lane (q16, g4) holds A[row][32 s + 8 g4 .. + 7] rounded to bfloat16;
// FP32: A[row][16 g + 4 g4 .. + 3], g < 2 KS (row = 16 i + q16 of the wave).
template <bool F32>
struct AFrag {
  bf16x8 v[TM][KS];
};
template <>
struct AFrag<true> {
  floatx4 v[TM][2 * KS];
};

// NV consecutive values of a row from k0 on, zeros at and beyond K.
template <int NV>
__device__ __forceinline__ void load_run(const float *row, int k0, int K, float (&out)[NV]) {
  if (k0 + NV <= K) {
#pragma unroll
    for (int q = 0; q < NV / 4; ++q) {
      const floatx4 t = ld4(row + k0 + 4 * q);
#pragma unroll
      for (int e = 0; e < 4; ++e) out[4 * q + e] = t[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < NV; ++e) out[e] = k0 + e < K ? row[k0 + e] : 0.0f;
  }
}

template <bool F32>
__device__ __forceinline__ void load_a(const float *A, int64_t lda, int64_t M, int K, int64_t r0, int q16, int g4,
                                       AFrag<F32> &a) {
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    int64_t r = r0 + i * 16 + q16;
    if (r >= M) r = M - 1;  // rows beyond M read a valid row and are never stored
    const float *row = A + r * lda;
    if constexpr (F32) {
#pragma unroll
      for (int g = 0; g < 2 * KS; ++g) {
        float t[4];
        load_run<4>(row, 16 * g + 4 * g4, K, t);
        a.v[i][g] = floatx4{t[0], t[1], t[2], t[3]};
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        float t[8];
        load_run<8>(row, 32 * s + 8 * g4, K, t);
#pragma unroll
        for (int e = 0; e < 8; ++e) a.v[i][s][e] = (__bf16)t[e];
      }
    }
  }
}

template <class CS>
constexpr int bias_bytes() {
  return CS::kBias ? kMaxN * 4 : 0;
}
template <class CS>
constexpr int side_bytes() {
  constexpr int b = bias_bytes<CS>() + ((CS::kMask || CS::kBits == 1) ? BM * (kMaxN / 16) * 2 : 0);
  return b > 0 ? b : 16;
}

// Two floats rounded to bfloat16 (nearest even) and packed, lo in the low
// half: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pack2_bf16(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 h2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{lo, hi}, h2));
}

// The 16-bit ReLU word of one row's 16-column tile: each of the row's four
// lanes (q16, g4) holds the nibble of its four columns; two row swaps OR
// them together in every lane.
__device__ __forceinline__ unsigned bits_word(unsigned nib, int g4) {
  unsigned w = nib << (4 * g4);
  const auto s16 = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  w = s16[0] | s16[1];
  const auto s32 = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return s32[0] | s32[1];
}

// Two adjacent 16-column tiles of one row in bfloat16 (lane g4 holds
// columns 4 g4 .. 4 g4 + 3 of both, two packed words each): a row swap
// hands each lane 8 contiguous columns, stored with one 16-byte store.
__device__ __forceinline__ void store_pair_bf16(uint16_t *C, int64_t ldc, int64_t r, int nt, int g4,
                                                const uint32_t (&w0)[2], const uint32_t (&w1)[2]) {
  const bool odd = g4 & 1;
  uint32_t out[4];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t mine = odd ? w0[q] : w1[q];  // the half the partner stores
    const auto x = __builtin_amdgcn_permlane16_swap(mine, mine, false, false);
    const uint32_t theirs = x[0] ^ x[1] ^ mine;  // one result is this lane's own value
    if (odd) {
      out[q] = theirs;
      out[2 + q] = w1[q];
    } else {
      out[q] = w0[q];
      out[2 + q] = theirs;
    }
  }
  const int col = odd ? nt + 16 + 4 * (g4 - 1) : nt + 4 * g4;
  __builtin_memcpy(C + r * ldc + col, out, 16);
}

template <bool F32, int BN, int D, int NACC, bool RELU, class BO, class CS>
__global__ __launch_bounds__(256) void astat_kernel(const float *A, int64_t lda, int64_t M, int K, BO bo, CS cs,
                                                    int N) {
  constexpr int TN = BN / 16, NS = D + 1;
  constexpr bool kHalf = CS::kHalf, kMaskIn = CS::kMask, kBitsOut = CS::kBits == 1;
  static_assert(!CS::kMask || CS::kBits == 2, "masks from ReLU bits only");
  constexpr int SLAB = BO::template bytes<BN>();  // one 32-k slice of a column tile
  constexpr int TILE = KS * SLAB;
  constexpr int NSL = BO::template slots<BN>();
  static_assert(BO::kUnit == 16 && NSL % 64 == 0, "whole 16-byte DMA instructions per slice");
  constexpr int NI = NSL / 64;        // DMA instructions per slice
  constexpr int NIT = KS * NI;        // per tile, dealt round-robin to the four waves
  constexpr int KW = (NIT + 3) / 4;   // per wave per tile, at most
  constexpr int IW = NIT / 4;         // and at least
  constexpr int KB = BO::template bytes<1>() / SBK;  // bytes per table entry
  // stores per wave per tile, at least: one per pair of bfloat16 tiles (and
  // per odd tile), or one per float32 tile
  constexpr int SW = TM * (kHalf ? (TN + 1) / 2 : TN);
  static_assert(D >= 1 && D <= 3 && D * SW + (D - 1) * IW < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) char lds[NS * TILE + side_bytes<CS>()];
  static_assert((NS * TILE + bias_bytes<CS>()) % 16 == 0, "16-byte aligned bit words in LDS");
  float *sbias = reinterpret_cast<float *>(lds + NS * TILE);
  uint16_t *sbits = reinterpret_cast<uint16_t *>(lds + NS * TILE + bias_bytes<CS>());

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q16 = lane & 15, g4 = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * BM;
  const int64_t r0 = m0 + wave * 16 * TM;
  const int NT = N / BN;
  const int wpr = N / 16;  // ReLU-bit words per row
  const bool full = m0 + BM <= M;

  // The wave's DMA instructions of a tile (q = wave + 4k: slice q / NI,
  // instruction q % NI of it): per-lane byte offsets from the tile's first
  // table row, and LDS offsets in the slot (the same for every tile: N is a
  // multiple of BN, so no row is clamped).
  uint32_t voff[KW];
  int loff[KW];
  const int nq = (NIT - wave + 3) / 4;
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int q = wave + 4 * k, sl = q / NI, ins = q - sl * NI;
    voff[k] = q < NIT ? bo.template lane_off<BN>(ins * 64 + lane, 0) + uint32_t(sl * SBK * KB) : 0u;
    loff[k] = sl * SLAB + ins * 64 * 16;
  }
  const char *gtab = bo.base(0, 0);
  const int64_t tstride = bo.base(BN, 0) - gtab;  // bytes between column tiles
  auto issue = [&](int t) {
    const char *src = gtab + (int64_t)t * tstride;
    char *dst = lds + (t % NS) * TILE;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      if (k < nq) {
        uint32_t o = voff[k];
        asm volatile("" : "+v"(o));
        dma_to_lds<16>(src + o, dst + loff[k]);
      }
    }
  };

  // prologue: A into registers, the first tiles and the side data into LDS
  AFrag<F32> a;
  load_a<F32>(A, lda, M, K, r0, q16, g4, a);
#pragma unroll
  for (int t = 0; t < D; ++t)
    if (t < NT) issue(t);
  if constexpr (CS::kBias)
    for (int c = tid; c < N; c += 256) sbias[c] = cs.bias_n[c];
  if constexpr (kMaskIn) {
    // the block's bit words are one run of memory: 16-byte copies when it
    // is whole and aligned (LDS side: the tiles and the bias are multiples
    // of 16 bytes), else word by word with rows clamped
    const uint16_t *src = cs.mbits + m0 * wpr;
    if (full && (BM * wpr) % 8 == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
      for (int c = tid; c < BM * wpr / 8; c += 256)
        __builtin_memcpy(reinterpret_cast<uint4 *>(sbits) + c, reinterpret_cast<const uint4 *>(src) + c, 16);
    } else {
      for (int c = tid; c < BM * wpr; c += 256) {
        const int rr = c / wpr;
        int64_t r = m0 + rr;
        if (r >= M) r = M - 1;
        sbits[c] = cs.mbits[r * wpr + (c - rr * wpr)];
      }
    }
  }
  wait_barrier<0>();

  for (int t = 0; t < NT; ++t) {
    if (t >= D) {
      // after the DMA of tile t this wave issued: the stores of tiles
      // t-D .. t-1 and the DMA of tiles t+1 .. t+D-1 (those that exist)
      const int later = min(D - 1, NT - 1 - t);
      if constexpr (D == 1) {
        if (full) wait_barrier<SW>();
        else wait_barrier<0>();
      } else if constexpr (D == 2) {
        if (full) {
          if (later) wait_barrier<2 * SW + IW>();
          else wait_barrier<2 * SW>();
        } else {
          if (later) wait_barrier<IW>();
          else wait_barrier<0>();
        }
      } else {
        if (full) {
          if (later == 2) wait_barrier<3 * SW + 2 * IW>();
          else if (later == 1) wait_barrier<3 * SW + IW>();
          else wait_barrier<3 * SW>();
        } else {
          if (later == 2) wait_barrier<2 * IW>();
          else if (later == 1) wait_barrier<IW>();
          else wait_barrier<0>();
        }
      }
    } else if (t > 0) {
      // every wave is done reading the slot refilled next (tiles t < D
      // arrived before the prologue's barrier)
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }
    if (t + D < NT) issue(t + D);

    const char *tile = lds + (t % NS) * TILE;
    floatx4 acc[NACC][TM][TN];
#pragma unroll
    for (int u = 0; u < NACC; ++u)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[u][i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
      const char *sb = tile + sl * SLAB;
      if constexpr (F32) {
        const int nh = K - SBK * sl > 16 ? 2 : 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h < nh) {
            floatx4 b[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = bo.template frag4<BN>(sb, j, q16, g4, h);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
              for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                  acc[jj % NACC][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j][jj], a.v[i][2 * sl + h][jj],
                                                                              acc[jj % NACC][i][j], 0, 0, 0);
          }
        }
      } else {
        bf16x8 b[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = bo.template frag<BN>(sb, j, q16, g4);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a.v[i][sl], acc[0][i][j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 1; u < NACC; ++u)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[0][i][j] += acc[u][i][j];

    // epilogue: bias, ReLU, mask, rounding, bits; then the stores
    const int n0 = t * BN;
    floatx4 cbv[TN];
    if constexpr (CS::kBias) {
#pragma unroll
      for (int j = 0; j < TN; ++j) cbv[j] = *reinterpret_cast<const floatx4 *>(sbias + n0 + 16 * j + 4 * g4);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int rr = wave * 16 * TM + i * 16 + q16;
      const int64_t r = m0 + rr;
      floatx4 v[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        v[j] = acc[0][i][j];
        unsigned mnib = 15u;
        if constexpr (kMaskIn) mnib = (unsigned)sbits[rr * wpr + n0 / 16 + j] >> (4 * g4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (CS::kBias) v[j][q] += cbv[j][q];
          if constexpr (RELU) v[j][q] = fmaxf(v[j][q], 0.0f);
          if constexpr (kMaskIn) v[j][q] = (mnib >> q) & 1u ? v[j][q] : 0.0f;
        }
      }
      if constexpr (kHalf) {
        uint32_t h2[TN][2];
        unsigned nib[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          nib[j] = 0;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            // both values rounded (RNE) by one packed conversion
            const uint32_t w = pack2_bf16(v[j][2 * q], v[j][2 * q + 1]);
            h2[j][q] = w;
            if constexpr (kBitsOut)  // the stored (rounded) value is > 0
              nib[j] |= ((__builtin_bit_cast(float, w << 16) > 0.0f ? 1u : 0u) |
                         (__builtin_bit_cast(float, w & 0xffff0000u) > 0.0f ? 2u : 0u))
                        << (2 * q);
          }
        }
        if constexpr (kBitsOut) {
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const unsigned w = bits_word(nib[j], g4);
            if (g4 == 0) sbits[rr * wpr + n0 / 16 + j] = (uint16_t)w;
          }
        }
        if (r >= M) continue;
#pragma unroll
        for (int jp = 0; jp < TN / 2; ++jp)
          store_pair_bf16(cs.C, cs.ldc, r, n0 + 32 * jp, g4, h2[2 * jp], h2[2 * jp + 1]);
        if constexpr (TN % 2 != 0) __builtin_memcpy(cs.C + r * cs.ldc + n0 + 16 * (TN - 1) + 4 * g4, h2[TN - 1], 8);
      } else {
        if constexpr (kBitsOut) {
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            unsigned nib = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) nib |= (v[j][q] > 0.0f ? 1u : 0u) << q;
            const unsigned w = bits_word(nib, g4);
            if (g4 == 0) sbits[rr * wpr + n0 / 16 + j] = (uint16_t)w;
          }
        }
        if (r >= M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) __builtin_memcpy(cs.C + r * cs.ldc + n0 + 16 * j + 4 * g4, &v[j], 16);
      }
    }
  }

  if constexpr (kBitsOut) {
    // the block's bit words, rows m0 .. m0 + BM - 1 (those below M): one
    // contiguous run of memory
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    const int64_t rows = min((int64_t)BM, M - m0);
    const int64_t nw = rows * wpr;
    uint16_t *dst = cs.obits + m0 * wpr;
    if (((reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
      const int64_t n16 = nw / 8;
      for (int64_t c = tid; c < n16; c += 256)
        __builtin_memcpy(dst + 8 * c, reinterpret_cast<const uint4 *>(sbits) + c, 16);
      for (int64_t c = 8 * n16 + tid; c < nw; c += 256) dst[c] = sbits[c];
    } else {
      for (int64_t c = tid; c < nw; c += 256) dst[c] = sbits[c];
    }
  }
}

// Which output policies the kernel takes: bias or none, or the ReLU mask
// from bit words (an activation mask would be as large as the output).
template <class CS>
constexpr bool takes() {
  return !CS::kMask || CS::kBits == 2;
}

// DLM_TILED_ONLY=1 in the environment sends these GEMMs to the tiled core
// instead (the same results bit for bit; read at every call, for tests).
inline bool tiled_only() {
  const char *e = std::getenv("DLM_TILED_ONLY");
  return e && e[0] == '1';
}

template <bool F32>
bool ok(const TableGemm &t) {
  constexpr int BN = F32 ? DLM_ASTAT_BN_F32 : DLM_ASTAT_BN_BF16;
  return DLM_ASTAT != 0 && !tiled_only() && t.A != nullptr && t.Ah == nullptr && t.K > SBK * (KS - 1) && t.K <= SBK * KS &&
         t.N % BN == 0 && t.N <= kMaxN && t.N % 16 == 0 && t.M > 0 && (t.M + BM - 1) / BM <= 0x7fffffff;
}

template <bool F32, class BO, class CS>
int run(const TableGemm &t, BO bo, CS cs, hipStream_t st) {
  constexpr int BN = F32 ? DLM_ASTAT_BN_F32 : DLM_ASTAT_BN_BF16;
  constexpr int D = F32 ? DLM_ASTAT_D_F32 : DLM_ASTAT_D_BF16;
  constexpr int NACC = F32 ? DLM_ASTAT_NACC : 1;
  const unsigned blocks = (unsigned)((t.M + BM - 1) / BM);
  if constexpr (CS::kBias) {  // the forward: ReLU fused or not
    if (t.relu)
      hipLaunchKernelGGL((astat_kernel<F32, BN, D, NACC, true, BO, CS>), dim3(blocks), dim3(256), 0, st, t.A, t.lda,
                         t.M, t.K, bo, cs, t.N);
    else
      hipLaunchKernelGGL((astat_kernel<F32, BN, D, NACC, false, BO, CS>), dim3(blocks), dim3(256), 0, st, t.A, t.lda,
                         t.M, t.K, bo, cs, t.N);
  } else {
    if (t.relu) return -3;  // an input gradient never fuses a ReLU
    hipLaunchKernelGGL((astat_kernel<F32, BN, D, NACC, false, BO, CS>), dim3(blocks), dim3(256), 0, st, t.A, t.lda,
                       t.M, t.K, bo, cs, t.N);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace astat

// BF16, N > 96 (N = 135/136, and 1440/2880 = 10/20 tiles exactly): one
// configuration; for the K = 135 GEMMs it also amortises a block's fixed
// cost (DMA offsets, first loads, epilogue) over 1.5x the output of 128 x 96
using SCfgNarrow = SCfg<128, 144, 4, 1, 3>;
// FP32, N > 144 (two-stage ring): 64-row tiles hold four blocks per CU, which
// keeps the matrix cores fed through the short (K = 135) reduction and the
// epilogue
using SCfgWideF32 = SCfg<64, 96, 2, 2, 2>;
using SCfgSmall = SCfg<128, 48, 4, 1, 3>;   // N <= 96
// weight gradient: two float32 operands per stage (34 KB); a two-stage ring
// keeps two blocks per CU
using SCfgGrad = SCfg<128, 144, 4, 1, 2>;

template <int OP, bool F32, class AO, class BO, class CS>
int stream_table_c(AO ao, BO bo, CS cs, const TableGemm &t, hipStream_t st) {
  if constexpr (astat::takes<CS>())
    if (astat::ok<F32>(t)) return astat::run<F32>(t, bo, cs, st);
  if (t.N <= 96) return run_stream<OP, SCfgSmall, F32>(ao, bo, cs, t.M, t.N, t.K, 1, 0, st);
  if constexpr (F32)
    if (t.N > 144) return run_stream<OP, SCfgWideF32, F32>(ao, bo, cs, t.M, t.N, t.K, 1, 0, st);
  return run_stream<OP, SCfgNarrow, F32>(ao, bo, cs, t.M, t.N, t.K, 1, 0, st);
}

// the forward GEMM adds the folded bias; the input-gradient GEMM may mask
template <int OP, bool F32, class AO, class BO>
int stream_table(AO ao, BO bo, const TableGemm &t, hipStream_t st) {
  const int64_t ldm = t.N / 16;  // ReLU-bit words per row
  if constexpr (!F32) {
    if (t.Ch) {  // bfloat16 output (and mask)
      if constexpr (OP == kOpFoldFwd) {
        if (t.relu_bits_out)
          return stream_table_c<OP, F32>(
              ao, bo, CRowSideH<true, false, 1>{t.Ch, t.ldc, t.relu, t.bias_n, nullptr, nullptr, t.relu_bits_out, ldm},
              t, st);
        return stream_table_c<OP, F32>(ao, bo, CRowSideH<true, false>{t.Ch, t.ldc, t.relu, t.bias_n, nullptr}, t, st);
      } else {
        if (t.relu_bits_in)
          return stream_table_c<OP, F32>(
              ao, bo, CRowSideH<false, true, 2>{t.Ch, t.ldc, t.relu, nullptr, nullptr, t.relu_bits_in, nullptr, ldm},
              t, st);
        if (t.out_mask_h)
          return stream_table_c<OP, F32>(ao, bo, CRowSideH<false, true>{t.Ch, t.ldc, t.relu, nullptr, t.out_mask_h},
                                         t, st);
        return stream_table_c<OP, F32>(ao, bo, CRowSideH<false, false>{t.Ch, t.ldc, t.relu, nullptr, nullptr}, t, st);
      }
    }
  }
  if constexpr (OP == kOpFoldFwd) {
    if (t.relu_bits_out)
      return stream_table_c<OP, F32>(
          ao, bo, CRowSide<true, false, 1>{t.C, t.ldc, t.relu, t.bias_n, nullptr, nullptr, t.relu_bits_out, ldm}, t,
          st);
    return stream_table_c<OP, F32>(ao, bo, CRowSide<true, false>{t.C, t.ldc, t.relu, t.bias_n, nullptr}, t, st);
  } else {
    if (t.relu_bits_in)
      return stream_table_c<OP, F32>(
          ao, bo, CRowSide<false, true, 2>{t.C, t.ldc, t.relu, nullptr, nullptr, t.relu_bits_in, nullptr, ldm}, t, st);
    if (t.out_mask)
      return stream_table_c<OP, F32>(ao, bo, CRowSide<false, true>{t.C, t.ldc, t.relu, nullptr, t.out_mask}, t, st);
    return stream_table_c<OP, F32>(ao, bo, CRowSide<false, false>{t.C, t.ldc, t.relu, nullptr, nullptr}, t, st);
  }
}

template <int OP, bool F32, class AO>
int stream_table_b(AO ao, const TableGemm &t, hipStream_t st) {
  // float32 tables are read as k-contiguous float32 rows of stride ldb_f
  if constexpr (F32) return stream_table<OP, true>(ao, SKc<true>{t.Bf, t.ldb_f, t.N}, t, st);
  else return stream_table<OP, false>(ao, SKh{t.Bh, t.ldb_h, t.N}, t, st);
}

template <int OP, bool F32>
int stream_table_op(const TableGemm &t, hipStream_t st) {
  if constexpr (!F32)
    if (t.Ah) return stream_table_b<OP, F32>(SKb{{t.Ah, t.lda, t.M}}, t, st);
  const bool vec = t.lda % 4 == 0 && t.K % 4 == 0 && aligned16(t.A);
  if (vec) return stream_table_b<OP, F32>(SKc<true>{t.A, t.lda, t.M}, t, st);
  return stream_table_b<OP, F32>(SKc<false>{t.A, t.lda, t.M}, t, st);
}

template <bool F32, class AO, class BO, class CS>
int stream_grad(AO ao, BO bo, CS cs, int64_t rows, int cols, int64_t V, int splits, int ks, hipStream_t st) {
  return run_stream<kOpFoldGrad, SCfgGrad, F32>(ao, bo, cs, rows, cols, (int)V, splits, ks, st);
}

}  // namespace streaming

using namespace streaming;

// Full-stage DMA offsets are 32-bit: a tile's rows must span < 4 GiB.
constexpr int64_t kMaxStreamLd = int64_t(1) << 22;

bool stream_table_ok(const TableGemm &t, dlm_precision prec) {
  if (t.groups != 1 || t.mask != nullptr || (t.op != kOpFoldFwd && t.op != kOpFoldBwdData)) return false;
  if (t.relu_bits_out || t.relu_bits_in) {  // ReLU bits: one word per 16 columns
    if (t.N % 16 != 0) return false;
    if (t.relu_bits_out && (t.op != kOpFoldFwd || !t.relu)) return false;
    if (t.relu_bits_in && (t.op != kOpFoldBwdData || t.out_mask || t.out_mask_h)) return false;
  }
  if (t.Ah || t.Ch || t.out_mask_h) {  // bfloat16 activations: BF16 only, 16-byte rows
    if (prec != DLM_BF16) return false;
    if (t.Ah && (t.A || t.lda % 8 != 0 || t.K % 8 != 0 || !aligned16(t.Ah))) return false;
    if (t.Ch && (t.C || t.ldc % 8 != 0 || !aligned16(t.Ch))) return false;
    if (t.out_mask_h && (!t.Ch || t.out_mask || !aligned16(t.out_mask_h))) return false;
  }
  if (t.lda >= kMaxStreamLd || t.ldb_f >= kMaxStreamLd || t.ldb_h >= kMaxStreamLd) return false;
  if (t.op == kOpFoldFwd ? (t.bias_n == nullptr || t.out_mask != nullptr) : t.bias_n != nullptr) return false;
  if (prec == DLM_BF16)
    return t.Bh != nullptr && t.ldb_h > 0 && t.ldb_h % SBK == 0 && t.ldb_h >= t.K && aligned16(t.Bh);
  return t.Bf != nullptr && t.ldb_f > 0 && t.ldb_f % SBK == 0 && t.ldb_f >= t.K && aligned16(t.Bf);
}

int launch_stream_table(const TableGemm &t, dlm_precision prec, void *stream) {
  if (!stream_table_ok(t, prec)) return -3;
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = prec != DLM_BF16;
  switch (t.op) {
    case kOpFoldFwd: return f32 ? stream_table_op<kOpFoldFwd, true>(t, st) : stream_table_op<kOpFoldFwd, false>(t, st);
    case kOpFoldBwdData:
      return f32 ? stream_table_op<kOpFoldBwdData, true>(t, st) : stream_table_op<kOpFoldBwdData, false>(t, st);
    default: return -3;
  }
}

// dT[m][n] = sum_v g[v][m] * act[v][n] over voxel slices, act with a ones
// column at n = CK (the bias term); the larger of M and CK + 1 on the row side.
// g and act each come as float32 (g, a) or, in BF16, bfloat16 (gh, ah).
struct GradArgs {
  int64_t V;
  int M, CK, splits, ksplit;
  float *partial;
  hipStream_t st;
};

template <bool F32, class GO, class AOp>
static int grad_orient(GO go, AOp aop, const GradArgs &x) {
  const int N1 = x.CK + 1;
  if (x.M >= N1)
    return stream_grad<F32>(go, aop, CPartial2<false>{x.partial, x.M, N1}, x.M, N1, x.V, x.splits, x.ksplit, x.st);
  return stream_grad<F32>(aop, go, CPartial2<true>{x.partial, x.M, N1}, N1, x.M, x.V, x.splits, x.ksplit, x.st);
}

template <bool F32, class GO>
static int grad_act(GO go, const float *a, const uint16_t *ah, const GradArgs &x) {
  const int CK = x.CK;
  if constexpr (!F32)
    if (ah) return grad_orient<F32>(go, SRb<true>{ah, CK, CK, CK}, x);
  if (CK % 4 == 0 && aligned16(a)) return grad_orient<F32>(go, SRc<true, true>{a, CK, CK, CK}, x);
  return grad_orient<F32>(go, SRc<false, true>{a, CK, CK, CK}, x);
}

template <bool F32>
static int stream_grad_p(const float *g, const uint16_t *gh, const float *a, const uint16_t *ah, const GradArgs &x) {
  const int M = x.M;
  if constexpr (!F32)
    if (gh) return grad_act<F32>(SRb<false>{gh, M, M, -1}, a, ah, x);
  if (M % 4 == 0 && aligned16(g)) return grad_act<F32>(SRc<true, false>{g, M, M, -1}, a, ah, x);
  return grad_act<F32>(SRc<false, false>{g, M, M, -1}, a, ah, x);
}

bool stream_grad_ok(int M, int CK, int ksplit) {
  return ksplit % SBK == 0 && M < kMaxStreamLd && CK < kMaxStreamLd;
}

bool stream_grad_bf16_ok(const uint16_t *gh, const uint16_t *ah, int M, int CK) {
  return (!gh || (M % 8 == 0 && aligned16(gh))) && (!ah || (CK % 8 == 0 && aligned16(ah)));
}

int launch_stream_grad(const float *g, const uint16_t *gh, const float *a, const uint16_t *ah, int64_t V, int M,
                       int CK, int splits, int ksplit, float *partial, dlm_precision prec, void *stream) {
  if (!stream_grad_ok(M, CK, ksplit)) return -2;
  if ((gh || ah) && (prec != DLM_BF16 || !stream_grad_bf16_ok(gh, ah, M, CK))) return -3;
  const GradArgs x{V, M, CK, splits, ksplit, partial, (hipStream_t)stream};
  if (prec == DLM_BF16) return stream_grad_p<false>(g, gh, a, ah, x);
  return stream_grad_p<true>(g, nullptr, a, nullptr, x);
}

}  // namespace dlm
