// Device-side building blocks: complex arithmetic, the storage formats of
// spinor and link fields, and SU(3) reconstruction from 12 reals.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "wd_internal.h"

namespace wd {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i^N * z
template <int N, typename R>
__device__ __forceinline__ cx<R> iph(cx<R> z) {
  constexpr int n = ((N % 4) + 4) % 4;
  if constexpr (n == 0) return z;
  else if constexpr (n == 1) return {-z.im, z.re};
  else if constexpr (n == 2) return {-z.re, -z.im};
  else return {z.im, -z.re};
}

// ---- storage formats ---------------------------------------------------------------
// Tag types for the four storage precisions; `real` is the arithmetic type.
struct SF64 { using real = double; static constexpr wd_prec prec = WD_FP64; static constexpr int NCH = 12; };
struct SF32 { using real = float;  static constexpr wd_prec prec = WD_FP32; static constexpr int NCH = 6; };
struct SI16 { using real = float;  static constexpr wd_prec prec = WD_HALF_I16; static constexpr int NCH = 3; };
struct SF16 { using real = float;  static constexpr wd_prec prec = WD_HALF_F16; static constexpr int NCH = 3; };

template <class S>
constexpr bool kHalf = (S::prec == WD_HALF_I16 || S::prec == WD_HALF_F16);

// Spinor of one site: 4 spins x 3 colours.
template <typename R>
struct Spinor {
  cx<R> v[4][3];
};

struct FieldView {
  char* ptr;
  int64_t stride;
  int nrhs;
};

template <class S>
__device__ __forceinline__ const char* chunk_base(const FieldView& f, int r, int k) {
  return f.ptr + ((int64_t)(r * S::NCH + k) * f.stride) * 16;
}
__device__ __forceinline__ float* norm_base(const FieldView& f, int r) {
  return reinterpret_cast<float*>(f.ptr + (int64_t)f.nrhs * 3 * f.stride * 16) + (int64_t)r * f.stride;
}

// 16-bit helpers.  Fixed point: value = q * (norm / 32767).  binary16: value = h * norm.
__device__ __forceinline__ float h16_to_f(uint16_t bits) {
  return __half2float(__ushort_as_half(bits));
}
__device__ __forceinline__ uint16_t f_to_h16(float v) {
  return __half_as_ushort(__float2half_rn(v));
}
// Pins a binary32 value in a register as computed.  Without it the compiler
// fuses a multiply feeding a binary16 conversion into one mixed-precision FMA,
// or folds a double -> binary32 -> binary16 chain into one direct rounding;
// both round differently from "round to binary32, then to binary16", which is
// how the 16-bit formats are defined.  (Empty asm, no memory access.)
__device__ __forceinline__ float pin_f32(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <class S>
__device__ __forceinline__ void load_spinor(const FieldView& f, int r, int64_t i,
                                            Spinor<typename S::real>& s) {
  using R = typename S::real;
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 c = reinterpret_cast<const double2*>(chunk_base<S>(f, r, k))[i];
      s.v[k / 3][k % 3] = {c.x, c.y};
    }
  } else if constexpr (S::prec == WD_FP32) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 c = reinterpret_cast<const float4*>(chunk_base<S>(f, r, k))[i];
      s.v[(2 * k) / 3][(2 * k) % 3] = {c.x, c.y};
      s.v[(2 * k + 1) / 3][(2 * k + 1) % 3] = {c.z, c.w};
    }
  } else {
    const float nm = norm_base(f, r)[i];
    const float sc = (S::prec == WD_HALF_I16) ? nm / 32767.0f : nm;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 c = reinterpret_cast<const uint4*>(chunk_base<S>(f, r, k))[i];
      uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {  // complex number 4k + j
        uint16_t lo = (uint16_t)(w[j] & 0xffffu), hi = (uint16_t)(w[j] >> 16);
        float re, im;
        if constexpr (S::prec == WD_HALF_I16) {
          re = (float)(int16_t)lo * sc;
          im = (float)(int16_t)hi * sc;
        } else {
          re = h16_to_f(lo) * sc;
          im = h16_to_f(hi) * sc;
        }
        const int n = 4 * k + j;
        s.v[n / 3][n % 3] = {re, im};
      }
    }
  }
  (void)sizeof(R);
}

// Same as load_spinor, but 16-bit values come back in units of the site's
// norm (no multiply) with the factor returned in `scale`; for FP32/FP64
// fields scale is 1.
template <class S>
__device__ __forceinline__ void load_spinor_raw(const FieldView& f, int r, int64_t i,
                                                Spinor<typename S::real>& s, typename S::real& scale) {
  if constexpr (S::prec == WD_FP64 || S::prec == WD_FP32) {
    load_spinor<S>(f, r, i, s);
    scale = typename S::real(1);
  } else {
    const float nm = norm_base(f, r)[i];
    scale = (S::prec == WD_HALF_I16) ? nm / 32767.0f : nm;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 c = reinterpret_cast<const uint4*>(chunk_base<S>(f, r, k))[i];
      uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint16_t lo = (uint16_t)(w[j] & 0xffffu), hi = (uint16_t)(w[j] >> 16);
        const int n = 4 * k + j;
        if constexpr (S::prec == WD_HALF_I16) s.v[n / 3][n % 3] = {(float)(int16_t)lo, (float)(int16_t)hi};
        else s.v[n / 3][n % 3] = {h16_to_f(lo), h16_to_f(hi)};
      }
    }
  }
}

// 16-byte store; NT marks it streaming (not kept in L2).
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef uint32_t uvec4 __attribute__((ext_vector_type(4)));
template <bool NT, typename V>
__device__ __forceinline__ void st16(V* p, V v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Encode 24 reals of the arithmetic type into one site of the field.
template <class S, bool NT = false>
__device__ __forceinline__ void store_spinor(const FieldView& f, int r, int64_t i,
                                             const Spinor<typename S::real>& s) {
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cx<double> z = s.v[k / 3][k % 3];
      st16<NT>(reinterpret_cast<dvec2*>(const_cast<char*>(chunk_base<S>(f, r, k))) + i, dvec2{z.re, z.im});
    }
  } else if constexpr (S::prec == WD_FP32) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cx<float> a = s.v[(2 * k) / 3][(2 * k) % 3], b = s.v[(2 * k + 1) / 3][(2 * k + 1) % 3];
      st16<NT>(reinterpret_cast<fvec4*>(const_cast<char*>(chunk_base<S>(f, r, k))) + i,
               fvec4{a.re, a.im, b.re, b.im});
    }
  } else {
    float nm = 0.0f;
#pragma unroll
    for (int n = 0; n < 12; ++n) {
      nm = fmaxf(nm, fabsf(s.v[n / 3][n % 3].re));
      nm = fmaxf(nm, fabsf(s.v[n / 3][n % 3].im));
    }
    // A site whose norm is below 2^-100 is stored as zero: 32767/norm and
    // 1/norm must stay finite in binary32.
    if (!(nm >= 0x1p-100f)) nm = 0.0f;
    norm_base(f, r)[i] = nm;
    float sc;
    if constexpr (S::prec == WD_HALF_I16) sc = (nm > 0.0f) ? 32767.0f / nm : 0.0f;
    else sc = (nm > 0.0f) ? 1.0f / nm : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 4 * k + j;
        cx<float> z = s.v[n / 3][n % 3];
        uint16_t lo, hi;
        if constexpr (S::prec == WD_HALF_I16) {
          float a = fminf(fmaxf(rintf(z.re * sc), -32767.0f), 32767.0f);
          float b = fminf(fmaxf(rintf(z.im * sc), -32767.0f), 32767.0f);
          lo = (uint16_t)(int16_t)a;
          hi = (uint16_t)(int16_t)b;
        } else {
          lo = f_to_h16(pin_f32(z.re * sc));
          hi = f_to_h16(pin_f32(z.im * sc));
        }
        w[j] = (uint32_t)lo | ((uint32_t)hi << 16);
      }
      st16<NT>(reinterpret_cast<uvec4*>(const_cast<char*>(chunk_base<S>(f, r, k))) + i,
               uvec4{w[0], w[1], w[2], w[3]});
    }
  }
}

// ---- links ---------------------------------------------------------------------
// Link field of one precision: [parity][mu][chunk][site]; FP64 has 6 double2
// chunks, FP32 3 float4 chunks, 16-bit 3 chunks of 8 bytes (4 x 16 bit).
template <class S>
struct LinkChunks {
  static constexpr int N = (S::prec == WD_FP64) ? 6 : 3;
  static constexpr int BYTES = (S::prec == WD_FP64 || S::prec == WD_FP32) ? 16 : 8;
};

template <typename R>
struct Link {
  cx<R> u[3][3];
};

template <class S>
__device__ __forceinline__ const char* link_chunk(const char* base, int64_t stride, int par, int mu,
                                                  int k) {
  return base + ((int64_t)((par * 4 + mu) * LinkChunks<S>::N + k) * stride) * LinkChunks<S>::BYTES;
}

}  // namespace wd
