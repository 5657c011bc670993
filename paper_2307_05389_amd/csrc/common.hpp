// common.hpp -- device-side building blocks shared by the gfx950 kernels of
// libtsds: element traits for the 11 dtypes, order-preserving 64-bit keys,
// and DPP wave64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsds.h"

namespace tsds {

constexpr int kWave = 64;

// Per-chunk partial result of a bin that straddles chunk boundaries: the
// ordered keys of the running minimum / maximum and their first indices.
struct Partial {
  uint64_t kmin;
  int64_t imin;
  uint64_t kmax;
  int64_t imax;
};

// ---------------------------------------------------------------- elements
//
// Elem<T>: T is the storage type.  C is the type compared in registers
// (f16 compares natively as _Float16).  `lowest`/`highest` are the neutral
// elements of max/min (NaN is excluded by precondition, so +-inf work for
// floats).  key() maps a value to a uint64 whose unsigned order equals the
// numeric order of the value, with -0 folded onto +0 (IEEE equality), so
// partial results from different chunks merge by plain integer compares.

template <typename T> struct Elem;

template <> struct Elem<int8_t> {
  using C = int32_t;
  static __device__ __host__ C lowest() { return -128; }
  static __device__ __host__ C highest() { return 127; }
  static __device__ C load(const int8_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return (uint64_t)(int64_t)v ^ 0x8000000000000000ull; }
};
template <> struct Elem<uint8_t> {
  using C = uint32_t;
  static __device__ __host__ C lowest() { return 0; }
  static __device__ __host__ C highest() { return 255; }
  static __device__ C load(const uint8_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return v; }
};
template <> struct Elem<int16_t> {
  using C = int32_t;
  static __device__ __host__ C lowest() { return -32768; }
  static __device__ __host__ C highest() { return 32767; }
  static __device__ C load(const int16_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return (uint64_t)(int64_t)v ^ 0x8000000000000000ull; }
};
template <> struct Elem<uint16_t> {
  using C = uint32_t;
  static __device__ __host__ C lowest() { return 0; }
  static __device__ __host__ C highest() { return 65535; }
  static __device__ C load(const uint16_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return v; }
};
template <> struct Elem<int32_t> {
  using C = int32_t;
  static __device__ __host__ C lowest() { return INT32_MIN; }
  static __device__ __host__ C highest() { return INT32_MAX; }
  static __device__ C load(const int32_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return (uint64_t)(int64_t)v ^ 0x8000000000000000ull; }
};
template <> struct Elem<uint32_t> {
  using C = uint32_t;
  static __device__ __host__ C lowest() { return 0; }
  static __device__ __host__ C highest() { return UINT32_MAX; }
  static __device__ C load(const uint32_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return v; }
};
template <> struct Elem<int64_t> {
  using C = int64_t;
  static __device__ __host__ C lowest() { return INT64_MIN; }
  static __device__ __host__ C highest() { return INT64_MAX; }
  static __device__ C load(const int64_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return (uint64_t)v ^ 0x8000000000000000ull; }
};
template <> struct Elem<uint64_t> {
  using C = uint64_t;
  static __device__ __host__ C lowest() { return 0; }
  static __device__ __host__ C highest() { return UINT64_MAX; }
  static __device__ C load(const uint64_t *p) { return *p; }
  static __device__ uint64_t key(C v) { return v; }
};

// Sign-magnitude float bits -> unsigned order: negative values get all bits
// flipped, non-negative values get the sign bit set.
__device__ inline uint64_t float_bits_key32(uint32_t u) {
  uint32_t k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return k;
}
__device__ inline uint64_t float_bits_key64(uint64_t u) {
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// binary16 is stored as uint16_t so that host code never needs the type.
struct half_t {
  uint16_t bits;
};

template <> struct Elem<half_t> {
  using C = _Float16;
  static __device__ C lowest() { return __builtin_bit_cast(_Float16, (uint16_t)0xFC00); }
  static __device__ C highest() { return __builtin_bit_cast(_Float16, (uint16_t)0x7C00); }
  static __device__ C load(const half_t *p) { return __builtin_bit_cast(_Float16, p->bits); }
  static __device__ uint64_t key(C v) {
    float f = (float)v;  // exact widening
    if (f == 0.0f) f = 0.0f;
    return float_bits_key32(__builtin_bit_cast(uint32_t, f));
  }
};
template <> struct Elem<float> {
  using C = float;
  static __device__ C lowest() { return -__builtin_huge_valf(); }
  static __device__ C highest() { return __builtin_huge_valf(); }
  static __device__ C load(const float *p) { return *p; }
  static __device__ uint64_t key(C v) {
    if (v == 0.0f) v = 0.0f;
    return float_bits_key32(__builtin_bit_cast(uint32_t, v));
  }
};
template <> struct Elem<double> {
  using C = double;
  static __device__ C lowest() { return -__builtin_huge_val(); }
  static __device__ C highest() { return __builtin_huge_val(); }
  static __device__ C load(const double *p) { return *p; }
  static __device__ uint64_t key(C v) {
    if (v == 0.0) v = 0.0;
    return float_bits_key64(__builtin_bit_cast(uint64_t, v));
  }
};

// min / max that map to single VALU instructions (no NaN by precondition).
template <typename C> __device__ inline C vmin(C a, C b) { return b < a ? b : a; }
template <typename C> __device__ inline C vmax(C a, C b) { return a < b ? b : a; }
template <> __device__ inline float vmin(float a, float b) { return __builtin_fminf(a, b); }
template <> __device__ inline float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
template <> __device__ inline double vmin(double a, double b) { return __builtin_fmin(a, b); }
template <> __device__ inline double vmax(double a, double b) { return __builtin_fmax(a, b); }

// ---------------------------------------------------------------- wave64

__device__ inline int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// DPP move of a 32-bit word; rows outside ROW_MASK keep their own value.
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK, typename C>
__device__ inline C dpp_any(C v) {
  if constexpr (sizeof(C) == 8) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)u);
    uint32_t hi = dpp32<CTRL, ROW_MASK>((uint32_t)(u >> 32));
    return __builtin_bit_cast(C, ((uint64_t)hi << 32) | lo);
  } else if constexpr (sizeof(C) == 4) {
    return __builtin_bit_cast(C, dpp32<CTRL, ROW_MASK>(__builtin_bit_cast(uint32_t, v)));
  } else {
    static_assert(sizeof(C) == 2, "2, 4 or 8 byte values");
    uint32_t w = __builtin_bit_cast(uint16_t, v);
    return __builtin_bit_cast(C, (uint16_t)dpp32<CTRL, ROW_MASK>(w));
  }
}

template <typename C>
__device__ inline C readlane63(C v) {
  if constexpr (sizeof(C) == 8) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(C, ((uint64_t)hi << 32) | lo);
  } else if constexpr (sizeof(C) == 4) {
    return __builtin_bit_cast(C, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), 63));
  } else {
    uint32_t w = __builtin_bit_cast(uint16_t, v);
    return __builtin_bit_cast(C, (uint16_t)__builtin_amdgcn_readlane((int)w, 63));
  }
}

// Full-wave reduction with a commutative, associative `op`; the result is
// returned wave-uniform.  Steps: xor 1 and xor 2 inside quads, half-row and
// row mirrors (row of 16 reduced in every lane), then the row broadcasts of
// lanes 15 and 31 fold the four rows into lane 63.  All 64 lanes must be
// active and hold a value (inactive contributions must be the neutral
// element of `op`).
template <typename C, typename Op>
__device__ inline C wave_reduce(C x, Op op) {
  x = op(x, dpp_any<0xB1, 0xf>(x));   // quad_perm [1,0,3,2]
  x = op(x, dpp_any<0x4E, 0xf>(x));   // quad_perm [2,3,0,1]
  x = op(x, dpp_any<0x141, 0xf>(x));  // row_half_mirror
  x = op(x, dpp_any<0x140, 0xf>(x));  // row_mirror
  x = op(x, dpp_any<0x142, 0xa>(x));  // row_bcast:15 into rows 1 and 3
  x = op(x, dpp_any<0x143, 0xc>(x));  // row_bcast:31 into rows 2 and 3
  return readlane63(x);
}

template <typename C> __device__ inline C wave_min(C x) {
  return wave_reduce(x, [](C a, C b) { return vmin(a, b); });
}
template <typename C> __device__ inline C wave_max(C x) {
  return wave_reduce(x, [](C a, C b) { return vmax(a, b); });
}

__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Mark a value wave-uniform (it is kept in scalar registers from then on).
template <typename V>
__device__ inline V uniform(V v) {
  static_assert(sizeof(V) == 4 || sizeof(V) == 8, "4 or 8 byte values");
  if constexpr (sizeof(V) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(V, (uint32_t)__builtin_amdgcn_readfirstlane((int)__builtin_bit_cast(uint32_t, v)));
  }
}

template <typename C>
__device__ inline C readlane(C v, int lane) {
  if constexpr (sizeof(C) == 8) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(C, ((uint64_t)hi << 32) | lo);
  } else {
    static_assert(sizeof(C) == 4, "4 or 8 byte values");
    return __builtin_bit_cast(C, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), lane));
  }
}

// Lexicographic (key, index) merge of two results; smaller key wins, equal
// keys keep the smaller index (first occurrence).
__device__ inline void lex_min(uint64_t &k, int64_t &i, uint64_t k2, int64_t i2) {
  if (k2 < k || (k2 == k && i2 < i)) { k = k2; i = i2; }
}
__device__ inline void lex_max(uint64_t &k, int64_t &i, uint64_t k2, int64_t i2) {
  if (k2 > k || (k2 == k && i2 < i)) { k = k2; i = i2; }
}

}  // namespace tsds
