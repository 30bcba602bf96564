// Device-side building blocks shared by the GEMM cores: vector types,
// bfloat16 rounding, 16-byte loads, the XCD-aware block map and the output
// (epilogue) policies.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dlm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16_bits(float f) {
  __bf16 h = (__bf16)f;  // hardware round-to-nearest-even conversion
  return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ floatx4 ld4(const float *p) {
  floatx4 v;
  __builtin_memcpy(&v, p, 16);  // dword-aligned 16-byte load (global_load_dwordx4)
  return v;
}

// Block index -> (group / split z, M tile, N tile).  The grid is 1-D over
// nbM * nbN * Z blocks, dispatched round-robin over the 8 XCDs; the block
// index is remapped so that consecutive logical tiles land on one XCD and
// share its L2.  Logical order: split-K (ZOUTER) puts all tiles of one voxel
// slice together (they stream the same activation rows); grouped GEMMs put
// the groups of one row-block together, then their N tiles.
struct TileMap {
  int mt, nt, z;
  __device__ TileMap(int b, int nbM, int nbN, int Z, bool zouter) {
    const int total = nbM * nbN * Z;
    const int q = total >> 3, r = total & 7;
    const int xcd = b & 7, local = b >> 3;
    const int L = xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
    if (zouter) {
      z = L / (nbM * nbN);
      const int t = L - z * nbM * nbN;
      mt = t / nbN;
      nt = t - mt * nbN;
    } else {
      nt = L % nbN;
      z = (L / nbN) % Z;
      mt = L / (nbN * Z);
    }
  }
};

// C[r][n] (row stride ldc, group stride gs) = acc + bias_n[n], then an
// optional ReLU, then (if omask) zeroed where omask (same indexing as C) <= 0.
// Side inputs: colside (bias, per column) and elside (mask, per element) let
// an epilogue load every tile's side values before its first store, so their
// latency is paid once instead of once per store.
struct CRowMajor {
  static constexpr bool kSide = true;
  float *C;
  int64_t ldc, gs;
  int relu;
  const float *bias_n;
  const float *omask = nullptr;
  __device__ floatx4 colside(int n) const { return bias_n ? ld4(bias_n + n) : floatx4{0.f, 0.f, 0.f, 0.f}; }
  __device__ floatx4 elside(int64_t r, int n, int g) const {
    return omask ? ld4(omask + r * ldc + (int64_t)g * gs + n) : floatx4{1.f, 1.f, 1.f, 1.f};
  }
  __device__ void store4s(int64_t r, int n, int g, floatx4 v, floatx4 cb, floatx4 em) const {
    for (int q = 0; q < 4; ++q) {
      v[q] += cb[q];
      if (relu) v[q] = fmaxf(v[q], 0.0f);
      v[q] = em[q] > 0.0f ? v[q] : 0.0f;
    }
    __builtin_memcpy(C + r * ldc + (int64_t)g * gs + n, &v, 16);
  }
  __device__ void operator()(int64_t r, int n, int g, float v) const {
    const int64_t o = r * ldc + (int64_t)g * gs + n;
    if (bias_n) v += bias_n[n];
    if (relu) v = fmaxf(v, 0.0f);
    if (omask && !(omask[o] > 0.0f)) v = 0.0f;
    C[o] = v;
  }
  __device__ void store4(int64_t r, int n, int g, floatx4 v) const {
    const int64_t o = r * ldc + (int64_t)g * gs + n;
    if (bias_n) {
      const floatx4 b = ld4(bias_n + n);
      for (int q = 0; q < 4; ++q) v[q] += b[q];
    }
    if (relu)
      for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q], 0.0f);
    if (omask) {
      const floatx4 m = ld4(omask + o);
      for (int q = 0; q < 4; ++q) v[q] = m[q] > 0.0f ? v[q] : 0.0f;
    }
    __builtin_memcpy(C + o, &v, 16);
  }
};


template <bool TRANS>
struct CPartial2 {
  static constexpr bool kSide = false;
  float *part;
  int M, N1;
  __device__ void operator()(int64_t r, int c, int s, float v) const {
    if constexpr (TRANS)
      part[((int64_t)s * M + c) * N1 + r] = v;
    else
      part[((int64_t)s * M + r) * N1 + c] = v;
  }
  __device__ void store4(int64_t r, int c, int s, floatx4 v) const {
    if constexpr (TRANS) {
      for (int q = 0; q < 4; ++q) part[((int64_t)s * M + c + q) * N1 + r] = v[q];
    } else {
      __builtin_memcpy(part + ((int64_t)s * M + r) * N1 + c, &v, 16);
    }
  }
};


}  // namespace dlm
