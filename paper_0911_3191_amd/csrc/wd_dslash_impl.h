// Wilson-Dirac hopping term on one parity (Section 3, Eq. 1), for the
// storage formats FP64, FP32, int16 + norm and binary16 + norm: kernel
// templates and launch logic, instantiated once per storage format by
// wd_dslash_<format>.hip so the formats compile in parallel.
//
// One thread computes one output site of parity p for NR right-hand sides:
// for each direction mu it loads and rebuilds the link once (12 reals ->
// 3x3, Appendix A.1), then for each of its RHS gathers the neighbour of the
// opposite parity, projects it onto its rank-2 spin subspace (6 complex
// numbers), multiplies by U (forward) or U^dagger (backward), expands back to
// 4 spins and accumulates.  The t-boundary sign is applied to the hop, never
// folded into the stored link.
//
// Spin projection in the DeGrand-Rossi basis (Appendix B): every gamma_mu is
// off-diagonal in 2x2 blocks, gamma_mu = [[0, A_mu], [A_mu^dag, 0]], so
//   (1 + s gamma_mu) psi = [ h ; s A_mu^dag h ],  h = psi_up + s A_mu psi_down,
// with s = -1 on the forward hop and s = +1 on the backward hop of D (the
// adjoint swaps them).  Each A_mu has one entry per row, a power of i:
//   A_x = [[0, i], [i, 0]],  A_y = [[0, -1], [1, 0]],
//   A_z = [[i, 0], [0, -i]], A_t = [[1, 0], [0, 1]].
//
// 16-bit neighbours are projected and multiplied in units of their own site
// norm; the norm enters once, in the accumulating FMA.
//
// Work distribution (XCD-aware): the 8 XCDs of the chip each own one z-slab
// of the lattice and sweep it with t slowest, so the two t-neighbour slices a
// site needs were fetched by the same XCD shortly before (its own L2 holds
// them for single-RHS FP32/FP64).  Hardware assigns workgroup b to XCD b % 8;
// within an XCD, consecutive workgroups take consecutive slab positions, and
// the RHS groups of one site block are adjacent so their link loads hit L2.
// Lattices with Lz not divisible by 8 fall back to one contiguous
// checkerboard range per XCD.
#pragma once

#include <algorithm>

#include "wd_device.h"
#include "wd_reduce.h"

namespace wd {

// Row k of A_mu has its entry in column P_k with value i^PH_k.
template <int MU>
struct Gamma;
template <> struct Gamma<0> { static constexpr int P0 = 1, P1 = 0, PH0 = 1, PH1 = 1; };
template <> struct Gamma<1> { static constexpr int P0 = 1, P1 = 0, PH0 = 2, PH1 = 0; };
template <> struct Gamma<2> { static constexpr int P0 = 0, P1 = 1, PH0 = 1, PH1 = 3; };
template <> struct Gamma<3> { static constexpr int P0 = 0, P1 = 1, PH0 = 0, PH1 = 0; };

// Spin bases of the fields a launch works on (Appendix B).  In the UKQCD
// ("non-relativistic") basis psi' = S psi with
//   S = [[0, 1, 0, 1], [-1, 0, -1, 0], [0, 1, 0, -1], [-1, 0, 1, 0]] / sqrt(2),
// gamma_x and gamma_z are those of the DeGrand-Rossi basis, gamma_y changes
// sign (A_y = [[0, 1], [-1, 0]]) and gamma_t = diag(1, 1, -1, -1): the
// temporal projectors 1 +- gamma_t keep only the upper or only the lower two
// spins (times 2), so a temporal hop loads half a spinor.
template <int MU, int BASIS>
struct GammaB : Gamma<MU> {};
template <> struct GammaB<1, kBasisUK> { static constexpr int P0 = 1, P1 = 0, PH0 = 0, PH1 = 2; };

// n / d for n < 2^31 with a precomputed multiplier (round-up method).
struct FastDiv {
  uint32_t m, s;
};
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  return (__umulhi(n, f.m) + n) >> f.s;
}
static FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  const uint64_t m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
  return FastDiv{static_cast<uint32_t>(m), s};
}

struct DslashGeom {
  int L[4];
  int Lxh, Vh, tap;
  int64_t stride;       // chunk stride of every field and of the links
  FastDiv div_lxh;      // / Lxh
  FastDiv div_ly;       // / Ly
  FastDiv div_lz;       // / Lz
  int slab;             // 1: z-slab mapping, 0: contiguous range per XCD
  int nsub;             // y-sub-slabs per XCD slab, swept one after the other
  int sub_sites;        // sites of one parity in one sub-slab (all t)
  int sub_t_sites;      // ... at fixed t: Lxh * (Ly / nsub) * (Lz / 8)
  int sub_plane;        // Lxh * (Ly / nsub)
  FastDiv div_sub;      // / sub_sites
  FastDiv div_sub_t;    // / sub_t_sites
  FastDiv div_sub_plane;  // / sub_plane
  int site_blocks;      // site blocks per XCD (slab) or in total (contiguous)
  int ngroups;          // RHS groups
  int nrhs;             // RHS the launch covers (entries of the RHS list when mapped)
  int mapped;           // 1: `sel` lists the RHS indices to process; 0: it is an active mask (or null)
  int gslow;            // 1: an XCD sweeps its slab once per RHS group (group slowest)
  int link_nt;          // 1: link loads are marked streaming (read once per launch)
  int out_nt;           // 1: output stores are marked streaming
  int tgauge;           // 1: temporal links are the unit matrix off the last time slice
  // staging of x/y neighbours in LDS (16-bit formats, slab mapping)
  int lds_cap;          // staged sites per RHS slot (rows of Lxh sites)
  int slab_rows;        // rows (Lxh sites each) in one XCD's slab
  int suby;             // Ly / nsub
  FastDiv div_suby;     // / (Ly / nsub)
  FastDiv div_zl;       // / (Lz / 8)
  FastDiv div_lt;       // / Lt
};

// ---- buffer loads --------------------------------------------------------------
// Gathers use raw buffer loads: a per-RHS descriptor (base in SGPRs), the
// site offset as a 32-bit VGPR and the chunk offset as an SGPR, which keeps
// 64-bit address arithmetic out of the hot loop.  Out-of-range offsets read
// zero instead of faulting.
constexpr int kBufWord3 = 0x00020000;  // raw, untyped buffer (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}

template <class S>
struct SpinorBuf {
  __amdgpu_buffer_rsrc_t chunks;  // [chunk][site] of one RHS
  __amdgpu_buffer_rsrc_t norms;   // [site] of one RHS (16-bit formats)
  uint32_t chunk_bytes;           // stride * 16
};

// on = false gives an empty buffer (every load from it reads zero and moves
// no data), so a thread's RHS slots need no branches.
template <class S>
__device__ __forceinline__ SpinorBuf<S> spinor_buf(const FieldView& f, int r, bool on = true) {
  SpinorBuf<S> b;
  b.chunk_bytes = (uint32_t)(f.stride * 16);
  b.chunks = make_rsrc(chunk_base<S>(f, r, 0), on ? b.chunk_bytes * S::NCH : 0u);
  if constexpr (kHalf<S>) b.norms = make_rsrc(norm_base(f, r), on ? (uint32_t)(f.stride * 4) : 0u);
  else b.norms = b.chunks;
  return b;
}

// AUX is the load's cache policy: 0 default, kStream (nt) marks data read
// once so that it is evicted first and neighbour spinors stay in L2.
constexpr int kStream = 2;
template <int AUX = 0>
__device__ __forceinline__ uint4 bload16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ uint2 bload8(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

// Neighbour spinor of one RHS (FP64 / FP32 storage).
template <class S>
__device__ __forceinline__ void gather_spinor(const SpinorBuf<S>& b, int i, Spinor<typename S::real>& s) {
  const uint32_t vo = (uint32_t)i * 16u;
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double2 c = __builtin_bit_cast(double2, bload16(b.chunks, vo, k * b.chunk_bytes));
      s.v[k / 3][k % 3] = {c.x, c.y};
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 c = __builtin_bit_cast(float4, bload16(b.chunks, vo, k * b.chunk_bytes));
      s.v[(2 * k) / 3][(2 * k) % 3] = {c.x, c.y};
      s.v[(2 * k + 1) / 3][(2 * k + 1) % 3] = {c.z, c.w};
    }
  }
}

// Neighbour spinor of one RHS in a 16-bit format, left packed: word n holds
// complex component n = 3 spin + colour as (re | im << 16).  scale = the
// factor that turns stored values into reals (norm, or norm / 32767).
struct Raw16 {
  uint32_t w[12];
};
template <class S>
__device__ __forceinline__ void gather_spinor16(const SpinorBuf<S>& b, int i, Raw16& s, float& scale) {
  const uint32_t vo = (uint32_t)i * 16u;
  const float nm = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.norms, (uint32_t)i * 4u, 0, 0));
  scale = (S::prec == WD_HALF_I16) ? nm * (1.0f / 32767.0f) : nm;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 c = bload16(b.chunks, vo, k * b.chunk_bytes);
    s.w[4 * k] = c.x;
    s.w[4 * k + 1] = c.y;
    s.w[4 * k + 2] = c.z;
    s.w[4 * k + 3] = c.w;
  }
}

// Halves of a packed word as binary32 (exact).
__device__ __forceinline__ float half_lo(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// a + i^N b for two packed components, result in binary32.  Binary16: each
// real is one mixed-precision FMA b * one + a on the stored halves (`one` is
// 1.0 kept opaque so the multiply is not folded away); both halves convert
// exactly, so this equals the binary32 sum of the decoded values.  int16: the
// sum is formed exactly in integers and converted once.
template <int N, class S>
__device__ __forceinline__ cx<float> proj16(uint32_t a, uint32_t b, float one) {
  constexpr int n = ((N % 4) + 4) % 4;
  if constexpr (S::prec == WD_HALF_F16) {
    const float ar = half_lo(a), ai = half_hi(a), br = half_lo(b), bi = half_hi(b);
    if constexpr (n == 0) return {__builtin_fmaf(br, one, ar), __builtin_fmaf(bi, one, ai)};
    else if constexpr (n == 1) return {__builtin_fmaf(-bi, one, ar), __builtin_fmaf(br, one, ai)};
    else if constexpr (n == 2) return {__builtin_fmaf(-br, one, ar), __builtin_fmaf(-bi, one, ai)};
    else return {__builtin_fmaf(bi, one, ar), __builtin_fmaf(-br, one, ai)};
  } else {
    const int ar = (int16_t)(a & 0xffffu), ai = (int16_t)(a >> 16);
    const int br = (int16_t)(b & 0xffffu), bi = (int16_t)(b >> 16);
    if constexpr (n == 0) return {(float)(ar + br), (float)(ai + bi)};
    else if constexpr (n == 1) return {(float)(ar - bi), (float)(ai + br)};
    else if constexpr (n == 2) return {(float)(ar - br), (float)(ai - bi)};
    else return {(float)(ar + bi), (float)(ai - br)};
  }
}

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Third row c_j = conj(a_j1 b_j2 - a_j2 b_j1) of a 12-real link from its
// rows a and b (Appendix A.1).  In binary32 each real part is one chain of
// four FMAs; in FP64 the two products are formed side by side and subtracted
// (one instruction more, a shorter dependency chain: measured faster there).
template <typename R>
__device__ __forceinline__ void third_row(const cx<R> (&a)[3], const cx<R> (&b)[3], cx<R> (&c)[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    const cx<R> p = a[j1], q = b[j2], u = a[j2], v = b[j1];
    if constexpr (sizeof(R) == 8) {
      c[j] = conj(p * q - u * v);
    } else {
      c[j].re = fmar(p.re, q.re, fmar(-p.im, q.im, fmar(-u.re, v.re, u.im * v.im)));
      c[j].im = fmar(u.re, v.im, fmar(u.im, v.re, fmar(-p.re, q.im, -(p.im * q.re))));
    }
  }
}

// Rows a, b of link (par, mu) at site i, third row rebuilt as (a x b)^*.
template <class S, int AUX>
__device__ __forceinline__ void gather_link_aux(const char* links, int64_t stride, int par, int mu, int i,
                                                Link<typename S::real>& L) {
  using R = typename S::real;
  constexpr int N = LinkChunks<S>::N, B = LinkChunks<S>::BYTES;
  const uint32_t cbytes = (uint32_t)(stride * B);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(link_chunk<S>(links, stride, par, mu, 0), cbytes * N);
  const uint32_t vo = (uint32_t)i * (uint32_t)B;
  cx<R> e[6];
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2 c = __builtin_bit_cast(double2, bload16<AUX>(rs, vo, k * cbytes));
      e[k] = {c.x, c.y};
    }
  } else if constexpr (S::prec == WD_FP32) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 c = __builtin_bit_cast(float4, bload16<AUX>(rs, vo, k * cbytes));
      e[2 * k] = {c.x, c.y};
      e[2 * k + 1] = {c.z, c.w};
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint2 c = bload8<AUX>(rs, vo, k * cbytes);
      const uint32_t w[2] = {c.x, c.y};
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint16_t lo = (uint16_t)(w[j] & 0xffffu), hi = (uint16_t)(w[j] >> 16);
        if constexpr (S::prec == WD_HALF_I16)
          e[2 * k + j] = {(float)(int16_t)lo * (1.0f / 32767.0f), (float)(int16_t)hi * (1.0f / 32767.0f)};
        else
          e[2 * k + j] = {h16_to_f(lo), h16_to_f(hi)};
      }
    }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    L.u[0][b] = e[b];
    L.u[1][b] = e[3 + b];
  }
  third_row(L.u[0], L.u[1], L.u[2]);
}

__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }

// Link of (par, mu) at site i stored as 8 reals (Appendix A.2): a2, a3, b1 and
// the phases of a1 and c1 (16-bit formats: phases / pi).  Rebuilt with
// |a1| = sqrt(1 - |a2|^2 - |a3|^2), |c1| = sqrt(1 - |a1|^2 - |b1|^2) (negative
// arguments taken as zero), N = sqrt(|a2|^2 + |a3|^2), the plane vectors
// b' = (0, -a3*, a2*) / N and c' = (N, -a1* a2 / N, -a1* a3 / N), and the
// rotation b = p1 b' + p2 c', c = -p2* b' + p1* c' with p1 = c1* / N,
// p2 = b1 / N.
template <class S, int AUX>
__device__ __forceinline__ void gather_link8(const char* links, int64_t stride, int par, int mu, int i,
                                          Link<typename S::real>& L) {
  using R = typename S::real;
  constexpr int N8 = (S::prec == WD_FP64) ? 4 : (S::prec == WD_FP32 ? 2 : 1);  // 16-byte chunks
  const uint32_t cbytes = (uint32_t)(stride * 16);
  const __amdgpu_buffer_rsrc_t rs =
      make_rsrc(links + (int64_t)((par * 4 + mu) * N8) * stride * 16, cbytes * N8);
  const uint32_t vo = (uint32_t)i * 16u;
  R v[8];
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double2 c = __builtin_bit_cast(double2, bload16<AUX>(rs, vo, k * cbytes));
      v[2 * k] = c.x;
      v[2 * k + 1] = c.y;
    }
  } else if constexpr (S::prec == WD_FP32) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float4 c = __builtin_bit_cast(float4, bload16<AUX>(rs, vo, k * cbytes));
      v[4 * k] = c.x;
      v[4 * k + 1] = c.y;
      v[4 * k + 2] = c.z;
      v[4 * k + 3] = c.w;
    }
  } else {
    const uint4 c = bload16<AUX>(rs, vo, 0);
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (S::prec == WD_HALF_I16) {
        v[2 * j] = (float)(int16_t)(w[j] & 0xffffu) * (1.0f / 32767.0f);
        v[2 * j + 1] = (float)(int16_t)(w[j] >> 16) * (1.0f / 32767.0f);
      } else {
        v[2 * j] = half_lo(w[j]);
        v[2 * j + 1] = half_hi(w[j]);
      }
    }
    v[6] *= 3.14159265358979323846f;
    v[7] *= 3.14159265358979323846f;
  }
  const cx<R> a2 = {v[0], v[1]}, a3 = {v[2], v[3]}, b1 = {v[4], v[5]};
  const R n2 = a2.re * a2.re + a2.im * a2.im + a3.re * a3.re + a3.im * a3.im;
  R t = R(1) - n2;
  const R ma1 = t > R(0) ? sqrt(t) : R(0);
  t = R(1) - (ma1 * ma1 + (b1.re * b1.re + b1.im * b1.im));
  const R mc1 = t > R(0) ? sqrt(t) : R(0);
  R s1, c1c, s2, c2c;
  sincos_r(v[6], &s1, &c1c);
  sincos_r(v[7], &s2, &c2c);
  const cx<R> a1 = {ma1 * c1c, ma1 * s1}, c1 = {mc1 * c2c, mc1 * s2};
  const R nn = sqrt(n2);
  const R rn = R(1) / nn;
  // plane vectors b' (first entry 0) and c'
  const cx<R> bp1 = {-a3.re * rn, a3.im * rn}, bp2 = {a2.re * rn, -a2.im * rn};
  const cx<R> a1c = conj(a1);
  const cx<R> cp1 = (-rn) * (a1c * a2), cp2 = (-rn) * (a1c * a3);
  const cx<R> p1 = rn * conj(c1), p2 = rn * b1;
  const cx<R> p1c = conj(p1), p2c = conj(p2);
  L.u[0][0] = a1;
  L.u[0][1] = a2;
  L.u[0][2] = a3;
  L.u[1][0] = nn * p2;
  L.u[1][1] = p1 * bp1 + p2 * cp1;
  L.u[1][2] = p1 * bp2 + p2 * cp2;
  L.u[2][0] = nn * p1c;
  L.u[2][1] = p1c * cp1 - p2c * bp1;
  L.u[2][2] = p1c * cp2 - p2c * bp2;
}

template <typename R>
__device__ __forceinline__ void unit_link(Link<R>& L) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) L.u[a][b] = {a == b ? R(1) : R(0), R(0)};
}

// Link of (par, mu) at site i in the handle's format.  AUX is the cache
// policy, fixed per kernel (a run-time choice would put a branch in every
// hop, which splits the scheduling regions): one-slot kernels mark links
// streaming, since a single RHS group reads each link exactly once.
template <class S, int RECON, int AUX>
__device__ __forceinline__ void gather_link(const DslashGeom& g, const char* links, int par, int mu, int i,
                                            Link<typename S::real>& L) {
  if constexpr (RECON == 8) gather_link8<S, AUX>(links, g.stride, par, mu, i, L);
  else gather_link_aux<S, AUX>(links, g.stride, par, mu, i, L);
}

// acc + a * b and acc + conj(a) * b as four FMAs
template <typename R>
__device__ __forceinline__ cx<R> cmac(cx<R> acc, cx<R> a, cx<R> b) {
  return {fmar(-a.im, b.im, fmar(a.re, b.re, acc.re)), fmar(a.im, b.re, fmar(a.re, b.im, acc.im))};
}
template <typename R>
__device__ __forceinline__ cx<R> cmacc(cx<R> acc, cx<R> a, cx<R> b) {
  return {fmar(a.im, b.im, fmar(a.re, b.re, acc.re)), fmar(-a.im, b.re, fmar(a.re, b.im, acc.im))};
}

// Multiply the projected half spinor h by W = U or U^dagger, expand to four
// spins and accumulate: acc += scale * (1 + s gamma_mu) (W psi), where scale
// carries the 16-bit norm and the t-boundary sign.
template <int MU, int S, bool DAG_LINK, int BASIS, typename R>
__device__ __forceinline__ void mul_acc(Spinor<R>& acc, const cx<R> (&h)[2][3], const Link<R>& U, R scale) {
  using G = GammaB<MU, BASIS>;
  constexpr int sh = (S < 0) ? 2 : 0;  // multiplying by s = -1 is a factor i^2
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int lo = 2 + (k == 0 ? G::P0 : G::P1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> w = {R(0), R(0)};
      if constexpr (!DAG_LINK) {
        w = cmac(w, U.u[a][0], h[k][0]);
        w = cmac(w, U.u[a][1], h[k][1]);
        w = cmac(w, U.u[a][2], h[k][2]);
      } else {
        w = cmacc(w, U.u[0][a], h[k][0]);
        w = cmacc(w, U.u[1][a], h[k][1]);
        w = cmacc(w, U.u[2][a], h[k][2]);
      }
      // upper spin k gets w; lower spin P_k gets s conj(A[k][P_k]) w = i^(sh - PH_k) w
      acc.v[k][a] = acc.v[k][a] + scale * w;
      const cx<R> wl = (k == 0) ? iph<sh - G::PH0 + 4>(w) : iph<sh - G::PH1 + 4>(w);
      acc.v[lo][a] = acc.v[lo][a] + scale * wl;
    }
  }
}

// One hop from a decoded neighbour (FP64 / FP32 storage).
template <int MU, int S, bool DAG_LINK, int BASIS, typename R>
__device__ __forceinline__ void hop(Spinor<R>& acc, const Spinor<R>& psi, const Link<R>& U, R scale) {
  using G = GammaB<MU, BASIS>;
  constexpr int sh = (S < 0) ? 2 : 0;
  cx<R> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = psi.v[0][c] + iph<G::PH0 + sh>(psi.v[2 + G::P0][c]);
    h[1][c] = psi.v[1][c] + iph<G::PH1 + sh>(psi.v[2 + G::P1][c]);
  }
  mul_acc<MU, S, DAG_LINK, BASIS>(acc, h, U, scale);
}

// One hop from a packed 16-bit neighbour: the projection reads the stored
// values directly (see proj16), in units of the neighbour's norm.
template <int MU, int S, bool DAG_LINK, class SF, int BASIS>
__device__ __forceinline__ void hop16(Spinor<float>& acc, const Raw16& psi, const Link<float>& U, float scale,
                                      float one) {
  using G = GammaB<MU, BASIS>;
  constexpr int sh = (S < 0) ? 2 : 0;
  cx<float> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = proj16<G::PH0 + sh, SF>(psi.w[c], psi.w[3 * (2 + G::P0) + c], one);
    h[1][c] = proj16<G::PH1 + sh, SF>(psi.w[3 + c], psi.w[3 * (2 + G::P1) + c], one);
  }
  mul_acc<MU, S, DAG_LINK, BASIS>(acc, h, U, scale);
}

// ---- temporal hop in the UKQCD basis ---------------------------------------------
// acc[BASE + k] += scale * W psi[BASE + k] for the two spins the projector keeps
// (BASE = 0: 1 + gamma_t; BASE = 2: 1 - gamma_t); the factor 2 is in scale.
template <bool DAG_LINK, int BASE, typename R>
__device__ __forceinline__ void mul_acc_half(Spinor<R>& acc, const cx<R> (&h)[2][3], const Link<R>& U, R scale) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> w = {R(0), R(0)};
      if constexpr (!DAG_LINK) {
        w = cmac(w, U.u[a][0], h[k][0]);
        w = cmac(w, U.u[a][1], h[k][1]);
        w = cmac(w, U.u[a][2], h[k][2]);
      } else {
        w = cmacc(w, U.u[0][a], h[k][0]);
        w = cmacc(w, U.u[1][a], h[k][1]);
        w = cmacc(w, U.u[2][a], h[k][2]);
      }
      acc.v[BASE + k][a] = acc.v[BASE + k][a] + scale * w;
    }
}

// Spins BASE, BASE + 1 of a neighbour (FP64 / FP32): chunks of one complex
// (FP64) or two (FP32) hold them contiguously.
template <class S, int BASE>
__device__ __forceinline__ void gather_half(const SpinorBuf<S>& b, int i, cx<typename S::real> (&h)[2][3]) {
  const uint32_t vo = (uint32_t)i * 16u;
  if constexpr (S::prec == WD_FP64) {
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      const double2 c = __builtin_bit_cast(double2, bload16(b.chunks, vo, (3 * BASE + n) * b.chunk_bytes));
      h[n / 3][n % 3] = {c.x, c.y};
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float4 c = __builtin_bit_cast(float4, bload16(b.chunks, vo, (3 * BASE / 2 + q) * b.chunk_bytes));
      h[(2 * q) / 3][(2 * q) % 3] = {c.x, c.y};
      h[(2 * q + 1) / 3][(2 * q + 1) % 3] = {c.z, c.w};
    }
  }
}

// Spins BASE, BASE + 1 of a 16-bit neighbour: 6 packed words (upper: chunk 0
// and the first half of chunk 1; lower: the second half of chunk 1 and chunk 2).
template <class S, int BASE>
__device__ __forceinline__ void gather_half16(const SpinorBuf<S>& b, int i, cx<float> (&h)[2][3], float& scale) {
  const uint32_t vo = (uint32_t)i * 16u;
  const float nm = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.norms, (uint32_t)i * 4u, 0, 0));
  scale = (S::prec == WD_HALF_I16) ? nm * (1.0f / 32767.0f) : nm;
  uint32_t w[6];
  if constexpr (BASE == 0) {
    const uint4 c0 = bload16(b.chunks, vo, 0);
    const uint2 c1 = bload8(b.chunks, vo, b.chunk_bytes);
    w[0] = c0.x; w[1] = c0.y; w[2] = c0.z; w[3] = c0.w; w[4] = c1.x; w[5] = c1.y;
  } else {
    const uint2 c1 = bload8(b.chunks, vo + 8u, b.chunk_bytes);
    const uint4 c2 = bload16(b.chunks, vo, 2 * b.chunk_bytes);
    w[0] = c1.x; w[1] = c1.y; w[2] = c2.x; w[3] = c2.y; w[4] = c2.z; w[5] = c2.w;
  }
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    if constexpr (S::prec == WD_HALF_I16) h[n / 3][n % 3] = {(float)(int16_t)(w[n] & 0xffffu), (float)(int16_t)(w[n] >> 16)};
    else h[n / 3][n % 3] = {half_lo(w[n]), half_hi(w[n])};
  }
}

// ---- binary16 fields: SU(3) products as packed dot products -------------------
// For binary16 storage the link rows a, b are binary16 (re, im) pairs as
// stored, the third row is formed in binary32 from them and rounded once to
// binary16, and the projected half spinor h = psi_up + i^n psi_dn is formed
// with one packed binary16 add per complex number (one rounding).  Each real
// part of U h is then a chain of three v_dot2_f32_f16: two exact binary16
// products per instruction, summed in binary32:
//   (U h).re     = sum_b dot2(u_ab, conj(h_b)),  (U h).im     = sum_b dot2(u_ab, swap(h_b)),
//   (U^dag h).re = sum_b dot2(u_ba, h_b),        (U^dag h).im = sum_b dot2(u_ba, -i h_b),
// with swap(h) = (h.im, h.re).  The link is used exactly as stored; each of
// the two forms of h a hop needs is one packed add whose operand modifiers
// carry the phase i^n and the form.  The neighbour's norm and the boundary
// sign enter in the binary32 accumulation, as for the other formats.
// Complex numbers are handled as 32-bit words (re in the low half).  The
// packed adds and the first product of each chain are written out as
// instructions so that each form is one instruction (the compiler would
// otherwise share a + i^n b between the forms and fix it up afterwards) and a
// chain needs no zeroed accumulator.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 as_h2(uint32_t w) { return __builtin_bit_cast(h2, w); }
__device__ __forceinline__ uint32_t wswap(uint32_t w) { return (w >> 16) | (w << 16); }
__device__ __forceinline__ uint32_t wconj(uint32_t w) { return w ^ 0x80000000u; }
__device__ __forceinline__ uint32_t pack_w(float re, float im) {
  return __builtin_bit_cast(uint32_t, h2{(_Float16)re, (_Float16)im});
}
// c + a.lo b.lo + a.hi b.hi in binary32; dot2z: the same with c = 0
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2(as_h2(a), as_h2(b), c, false);
}
__device__ __forceinline__ float dot2z(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// -i w = (w.im, -w.re)
__device__ __forceinline__ uint32_t wmi(uint32_t w) {
  uint32_t r;
  asm("v_pk_add_f16 %0, %1, 0 op_sel:[1,0] op_sel_hi:[0,0] neg_lo:[0,0] neg_hi:[1,0]" : "=v"(r) : "v"(w));
  return r;
}

// Forms of h = a + i^N b, one packed add each: F = 0: h, 1: conj(h),
// 2: swap(h), 3: -i h.
constexpr int kFormId = 0, kFormConj = 1, kFormSwap = 2, kFormMi = 3;
template <int F, int N>
__device__ __forceinline__ uint32_t pk_form(uint32_t a, uint32_t b) {
  constexpr int n = ((N % 4) + 4) % 4;
  uint32_t r;
  if constexpr (F == 0 && n == 0)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,0] neg_hi:[0,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 0 && n == 1)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[0,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 0 && n == 2)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,1] neg_hi:[0,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 0 && n == 3)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,0] neg_hi:[0,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 1 && n == 0)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,0] neg_hi:[1,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 1 && n == 1)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,1] neg_hi:[1,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 1 && n == 2)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,0] op_sel_hi:[1,1] neg_lo:[0,1] neg_hi:[1,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 1 && n == 3)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[0,1] op_sel_hi:[1,0] neg_lo:[0,0] neg_hi:[1,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 2 && n == 0)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,0] neg_hi:[0,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 2 && n == 1)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,0] neg_hi:[0,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 2 && n == 2)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[0,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 2 && n == 3)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[0,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 3 && n == 0)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,0] neg_hi:[1,1]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 3 && n == 1)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,0] neg_hi:[1,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 3 && n == 2)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[0,1] neg_hi:[1,0]" : "=v"(r) : "v"(a), "v"(b));
  else if constexpr (F == 3 && n == 3)
    asm("v_pk_add_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1] neg_lo:[0,1] neg_hi:[1,1]" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

struct Link16 {
  uint32_t u[3][3];  // (re, im) binary16 pairs
};

// Rows a, b of a binary16 12-real link as stored; third row c = (a x b)^*
// in binary32 from the stored values, rounded once to binary16.
template <int AUX>
__device__ __forceinline__ void gather_link16(const char* links, int64_t stride, int par, int mu, int i,
                                              Link16& L) {
  const uint32_t cbytes = (uint32_t)(stride * 8);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(links + ((int64_t)(par * 4 + mu) * 3) * stride * 8, cbytes * 3);
  const uint32_t vo = (uint32_t)i * 8u;
  uint32_t w[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint2 c = bload8<AUX>(rs, vo, k * cbytes);
    w[2 * k] = c.x;
    w[2 * k + 1] = c.y;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    L.u[0][j] = w[j];
    L.u[1][j] = w[3 + j];
  }
  // c_j = conj(a_j1 b_j2 - a_j2 b_j1): binary32 products of binary16 values
  // (mixed-precision FMAs read the halves in place)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const h2 p = as_h2(w[(j + 1) % 3]), q = as_h2(w[3 + (j + 2) % 3]);
    const h2 u = as_h2(w[(j + 2) % 3]), v = as_h2(w[3 + (j + 1) % 3]);
    const float re = fmar((float)p.x, (float)q.x, fmar(-(float)p.y, (float)q.y,
                          fmar(-(float)u.x, (float)v.x, (float)u.y * (float)v.y)));
    const float im = fmar((float)u.x, (float)v.y, fmar((float)u.y, (float)v.x,
                          fmar(-(float)p.x, (float)q.y, -((float)p.y * (float)q.x))));
    L.u[2][j] = pack_w(re, im);
  }
}

// A binary32 link (8-real rebuild, unit matrix) in the binary16 operand form.
__device__ __forceinline__ void link16_from(const Link<float>& U, Link16& L) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) L.u[a][b] = pack_w(U.u[a][b].re, U.u[a][b].im);
}

// Row a of W h for W = U (DAG_LINK false; forms f1 = conj(h), f2 = swap(h))
// or W = U^dagger (forms f1 = h, f2 = -i h).
template <bool DAG_LINK>
__device__ __forceinline__ cx<float> su3_row16(const Link16& U, int a, const uint32_t (&f1)[3],
                                               const uint32_t (&f2)[3]) {
  cx<float> w;
  if constexpr (!DAG_LINK) {
    w.re = dot2(U.u[a][2], f1[2], dot2(U.u[a][1], f1[1], dot2z(U.u[a][0], f1[0])));
    w.im = dot2(U.u[a][2], f2[2], dot2(U.u[a][1], f2[1], dot2z(U.u[a][0], f2[0])));
  } else {
    w.re = dot2(U.u[2][a], f1[2], dot2(U.u[1][a], f1[1], dot2z(U.u[0][a], f1[0])));
    w.im = dot2(U.u[2][a], f2[2], dot2(U.u[1][a], f2[1], dot2z(U.u[0][a], f2[0])));
  }
  return w;
}

// One hop from a packed binary16 neighbour (in units of its norm): project,
// multiply by W, expand to four spins and accumulate (as hop16 / mul_acc).
template <int MU, int S, bool DAG_LINK, int BASIS>
__device__ __forceinline__ void hop16d(Spinor<float>& acc, const Raw16& psi, const Link16& U, float scale) {
  using G = GammaB<MU, BASIS>;
  constexpr int sh = (S < 0) ? 2 : 0;
  constexpr int F1 = DAG_LINK ? kFormId : kFormConj, F2 = DAG_LINK ? kFormMi : kFormSwap;
  uint32_t f1[2][3], f2[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint32_t a0 = psi.w[c], b0 = psi.w[3 * (2 + G::P0) + c];
    const uint32_t a1 = psi.w[3 + c], b1 = psi.w[3 * (2 + G::P1) + c];
    f1[0][c] = pk_form<F1, G::PH0 + sh>(a0, b0);
    f2[0][c] = pk_form<F2, G::PH0 + sh>(a0, b0);
    f1[1][c] = pk_form<F1, G::PH1 + sh>(a1, b1);
    f2[1][c] = pk_form<F2, G::PH1 + sh>(a1, b1);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int lo = 2 + (k == 0 ? G::P0 : G::P1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const cx<float> w = su3_row16<DAG_LINK>(U, a, f1[k], f2[k]);
      acc.v[k][a] = acc.v[k][a] + scale * w;
      const cx<float> wl = (k == 0) ? iph<sh - G::PH0 + 4>(w) : iph<sh - G::PH1 + 4>(w);
      acc.v[lo][a] = acc.v[lo][a] + scale * wl;
    }
  }
}

// Temporal hop in the UKQCD basis on binary16 fields: the two spins the
// projector keeps (BASE, BASE + 1; packed words w) times W, added to those
// spins; the factor 2 is in scale.
template <bool DAG_LINK, int BASE>
__device__ __forceinline__ void mul_acc_half16(Spinor<float>& acc, const uint32_t (&w)[6], const Link16& U,
                                               float scale) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint32_t f1[3], f2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t h = w[3 * k + c];
      f1[c] = DAG_LINK ? h : wconj(h);
      f2[c] = DAG_LINK ? wmi(h) : wswap(h);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) acc.v[BASE + k][a] = acc.v[BASE + k][a] + scale * su3_row16<DAG_LINK>(U, a, f1, f2);
  }
}

// Spins BASE, BASE + 1 of a binary16 neighbour as packed words (see
// gather_half16), with the factor that turns stored values into reals.
template <int BASE>
__device__ __forceinline__ void gather_half16w(const SpinorBuf<SF16>& b, int i, uint32_t (&w)[6], float& scale) {
  const uint32_t vo = (uint32_t)i * 16u;
  scale = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.norms, (uint32_t)i * 4u, 0, 0));
  if constexpr (BASE == 0) {
    const uint4 c0 = bload16(b.chunks, vo, 0);
    const uint2 c1 = bload8(b.chunks, vo, b.chunk_bytes);
    w[0] = c0.x; w[1] = c0.y; w[2] = c0.z; w[3] = c0.w; w[4] = c1.x; w[5] = c1.y;
  } else {
    const uint2 c1 = bload8(b.chunks, vo + 8u, b.chunk_bytes);
    const uint4 c2 = bload16(b.chunks, vo, 2 * b.chunk_bytes);
    w[0] = c1.x; w[1] = c1.y; w[2] = c2.x; w[3] = c2.y; w[4] = c2.z; w[5] = c2.w;
  }
}

// ---- LDS staging of x/y neighbours (16-bit formats) ------------------------------
// A workgroup of the slab mapping owns 256 consecutive slab positions, i.e.
// whole or partial rows of Lxh sites with y fastest.  Its x-neighbours lie in
// its own rows and its y-neighbours one row before or after (unless y wraps at
// a sub-slab edge), so the workgroup first copies the rows [first-1, last+1]
// of the input field, for each of its RHS slots, into LDS with coalesced
// loads; x- and in-plane y-gathers then read LDS, z- and t-gathers (and the
// wrapped y ones) read global memory.  This cuts the L2 requests of the
// gathers, which bound the multi-RHS kernel.
struct LdsCtx {
  const uint4* chunks;  // [slot][3][cap]
  const float* norms;   // [slot][cap]
  int cap;
  int base;             // first staged slab row
  int row;              // this thread's slab row
  int yl;               // this thread's y within its sub-slab
};

// Row table of the staged window: checkerboard index of each staged row's
// first site (-1: outside the slab, never read); returns the first staged row.
__device__ __forceinline__ int lds_rows(const DslashGeom& g, int xcd, int site_block, int* rowbase) {
  const int first = (int)fdiv((uint32_t)(site_block * blockDim.x), g.div_lxh);
  const int base = first - 1;
  const int nrows = g.lds_cap / g.Lxh;
  // checkerboard index of each staged row's first site (-1: outside the slab, never read)
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
    const int rs = base + r;
    int cb0 = -1;
    if (rs >= 0 && rs < g.slab_rows) {
      const int q1 = (int)fdiv((uint32_t)rs, g.div_suby);
      const int yl = rs - q1 * g.suby;
      const int q2 = (int)fdiv((uint32_t)q1, g.div_zl);
      const int zl = q1 - q2 * (g.L[2] >> 3);
      const int sub = (int)fdiv((uint32_t)q2, g.div_lt);
      const int t = q2 - sub * g.L[3];
      const int y = sub * g.suby + yl;
      const int z = xcd * (g.L[2] >> 3) + zl;
      cb0 = g.Lxh * (y + g.L[1] * (z + g.L[2] * t));
    }
    rowbase[r] = cb0;
  }
  return base;
}

// Copies the staged rows of every active RHS slot into LDS (the row table
// must be visible to every thread).
template <class S, int NR>
__device__ __forceinline__ void lds_copy(const DslashGeom& g, const SpinorBuf<S> (&in)[NR], const bool (&on)[NR],
                                         uint4* chunks, float* norms, const int* rowbase) {
  const int n = g.lds_cap;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (!on[k]) continue;  // uniform across the block
    for (int sl = threadIdx.x; sl < n; sl += blockDim.x) {
      const int rr = (int)fdiv((uint32_t)sl, g.div_lxh);
      const int cb0 = rowbase[rr];
      if (cb0 < 0) continue;
      const uint32_t cbi = (uint32_t)(cb0 + sl - rr * g.Lxh);
#pragma unroll
      for (int part = 0; part < 3; ++part)
        chunks[(k * 3 + part) * n + sl] = bload16(in[k].chunks, cbi * 16u, part * in[k].chunk_bytes);
      norms[k * n + sl] =
          __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(in[k].norms, cbi * 4u, 0, 0));
    }
  }
}

// Issues the copy of one RHS's staged rows straight into LDS (buffer loads
// that write LDS, no registers: a wave's 64 lanes fill 64 consecutive 16-byte
// or 4-byte slots from the wave-uniform base).  Returns at once; the data is
// there after the issuing wave's vmcnt reaches 0, and for the other waves
// after a barrier that follows that wait.  Rows outside the slab are skipped.
__device__ __forceinline__ void lds_issue16(const DslashGeom& g, const SpinorBuf<SF16>& in, uint4* chunks,
                                            float* norms, const int* rowbase) {
  using lds_ptr = __attribute__((address_space(3))) void*;
  const int n = g.lds_cap;
  for (int i = 0; i * (int)blockDim.x < n; ++i) {
    // first slot of this wave's 64 (uniform), and this lane's slot
    const int base = __builtin_amdgcn_readfirstlane(i * (int)blockDim.x + ((int)threadIdx.x & ~63));
    const int sl = i * (int)blockDim.x + (int)threadIdx.x;
    if (sl >= n) continue;
    const int rr = (int)fdiv((uint32_t)sl, g.div_lxh);
    const int cb0 = rowbase[rr];
    if (cb0 < 0) continue;
    const uint32_t cbi = (uint32_t)(cb0 + sl - rr * g.Lxh);
#pragma unroll
    for (int part = 0; part < 3; ++part)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(in.chunks, (lds_ptr)(chunks + part * n + base), 16, cbi * 16u,
                                               part * in.chunk_bytes, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(in.norms, (lds_ptr)(norms + base), 4, cbi * 4u, 0, 0, 0);
  }
}

template <class S, int NR>
__device__ __forceinline__ void lds_stage(const DslashGeom& g, int xcd, int site_block, const SpinorBuf<S> (&in)[NR],
                                          const bool (&on)[NR], uint4* chunks, float* norms, int* rowbase,
                                          int* base_out) {
  *base_out = lds_rows(g, xcd, site_block, rowbase);
  __syncthreads();
  lds_copy<S, NR>(g, in, on, chunks, norms, rowbase);
}

template <class S>
__device__ __forceinline__ void lds_gather16(const LdsCtx& c, int k, int sl, Raw16& s, float& scale) {
  const float nm = c.norms[k * c.cap + sl];
  scale = (S::prec == WD_HALF_I16) ? nm * (1.0f / 32767.0f) : nm;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint4 v = c.chunks[(k * 3 + q) * c.cap + sl];
    s.w[4 * q] = v.x;
    s.w[4 * q + 1] = v.y;
    s.w[4 * q + 2] = v.z;
    s.w[4 * q + 3] = v.w;
  }
}

// Splits the hops into one scheduling region per direction: every
// accumulator is pinned (empty asm, value in a register, memory clobber), so a
// direction's arithmetic completes before the next direction's loads are
// issued.  Without it the compiler either drains the loads of each RHS slot
// before issuing the next (few loads in flight per wave) or, in straight-line
// code, hoists every load of all eight hops and runs out of registers.
template <typename R, int NR>
__device__ __forceinline__ void hop_fence(Spinor<R> (&acc)[NR]) {
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        asm volatile("" : "+v"(acc[k].v[s][c].re) : : "memory");
        asm volatile("" : "+v"(acc[k].v[s][c].im) : : "memory");
      }
}

// Link of (par, mu) at site i for binary16 fields, in the dot-product form:
// 12 reals as stored (Appendix A.1), 8 reals rebuilt in binary32 (Appendix
// A.2), or the unit matrix (temporal gauge).
template <class S, int RECON, int AUX>
__device__ __forceinline__ void link_of16(const DslashGeom& g, const char* links, int par, int mu, int i, bool unit,
                                          Link16& L) {
  if constexpr (RECON == 8) {
    Link<float> U;
    if (unit) unit_link(U);
    else gather_link<S, RECON, AUX>(g, links, par, mu, i, U);
    link16_from(U, L);
  } else {
    if (unit) {
      Link<float> U;
      unit_link(U);
      link16_from(U, L);
    } else {
      gather_link16<AUX>(links, g.stride, par, mu, i, L);
    }
  }
}

// Both hops of direction MU for the NR right-hand sides of this thread.
template <class S, int MU, bool DAGGER, int NR, int RECON, bool LDS, int BASIS>
__device__ __forceinline__ void hop_pair(Spinor<typename S::real> (&acc)[NR], const DslashGeom& g,
                                         const char* __restrict__ links, const SpinorBuf<S> (&in)[NR],
                                         const bool (&on)[NR], int p, int cb, int xh, int row,
                                         const int (&X)[4], float one, const LdsCtx& lc) {
  using R = typename S::real;
  // neighbour checkerboard indices; row = y + Ly (z + Lz t)
  int nf, nb;
  bool flip_f = false, flip_b = false;
  if constexpr (MU == 0) {
    const int xf = (X[0] + 1 == g.L[0]) ? 0 : X[0] + 1;
    const int xb = (X[0] == 0) ? g.L[0] - 1 : X[0] - 1;
    nf = (xf >> 1) + g.Lxh * row;
    nb = (xb >> 1) + g.Lxh * row;
  } else {
    int step = 1;
    if constexpr (MU >= 2) step *= g.L[1];
    if constexpr (MU == 3) step *= g.L[2];
    const int rf = (X[MU] + 1 == g.L[MU]) ? row - (g.L[MU] - 1) * step : row + step;
    const int rb = (X[MU] == 0) ? row + (g.L[MU] - 1) * step : row - step;
    nf = xh + g.Lxh * rf;
    nb = xh + g.Lxh * rb;
    if constexpr (MU == 3) {
      flip_f = g.tap && (X[3] == g.L[3] - 1);
      flip_b = g.tap && (X[3] == 0);
    }
  }
  // staged neighbours: x always, y unless it wraps at a sub-slab edge
  int lf = -1, lb = -1;
  if constexpr (LDS && MU == 0) {
    const int r0 = (lc.row - lc.base) * g.Lxh;
    lf = r0 + (nf - g.Lxh * row);
    lb = r0 + (nb - g.Lxh * row);
  } else if constexpr (LDS && MU == 1) {
    if (lc.yl + 1 < g.suby) lf = (lc.row + 1 - lc.base) * g.Lxh + xh;
    if (lc.yl > 0) lb = (lc.row - 1 - lc.base) * g.Lxh + xh;
  }
  // temporal gauge: U_t is the unit matrix off the last time slice, so the
  // forward t-hop reads a link only from t = Lt - 1, the backward one only
  // into t = 0 (elsewhere the unit matrix is applied without a load)
  bool unit_f = false, unit_b = false;
  if constexpr (MU == 3) {
    unit_f = g.tgauge && X[3] != g.L[3] - 1;
    unit_b = g.tgauge && X[3] != 0;
  }
  // forward: (1 - gamma_mu) U_x^mu psi(x + mu); adjoint: (1 + gamma_mu)
  if constexpr (S::prec == WD_HALF_F16) {
    Link16 U;
    link_of16<S, RECON, (NR == 1 ? kStream : 0)>(g, links, p, MU, cb, unit_f, U);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if constexpr (MU == 3 && BASIS == kBasisUK) {
        constexpr int BASE = DAGGER ? 0 : 2;
        uint32_t w[6];
        float s16;
        gather_half16w<BASE>(in[k], nf, w, s16);
        mul_acc_half16<false, BASE>(acc[k], w, U, flip_f ? -2.0f * s16 : 2.0f * s16);
      } else {
        Raw16 psi;
        float sc;
        if (LDS && lf >= 0) lds_gather16<S>(lc, k, lf, psi, sc);
        else gather_spinor16<S>(in[k], nf, psi, sc);
        if (flip_f) sc = -sc;
        hop16d<MU, DAGGER ? +1 : -1, false, BASIS>(acc[k], psi, U, sc);
      }
    }
  } else {
    Link<R> U;
    if (unit_f) unit_link(U);
    else gather_link<S, RECON, (NR == 1 ? kStream : 0)>(g, links, p, MU, cb, U);
#pragma unroll
    for (int k = 0; k < NR; ++k) {  // an empty slot reads zeros (see spinor_buf)
      if constexpr (MU == 3 && BASIS == kBasisUK) {
        // 1 - gamma_t keeps the lower spins, its adjoint 1 + gamma_t the upper ones
        constexpr int BASE = DAGGER ? 0 : 2;
        cx<R> h[2][3];
        R sc = R(2);
        if constexpr (kHalf<S>) {
          float s16;
          gather_half16<S, BASE>(in[k], nf, h, s16);
          sc = 2.0f * s16;
        } else {
          gather_half<S, BASE>(in[k], nf, h);
        }
        mul_acc_half<false, BASE>(acc[k], h, U, flip_f ? -sc : sc);
      } else if constexpr (kHalf<S>) {
        Raw16 psi;
        float sc;
        if (LDS && lf >= 0) lds_gather16<S>(lc, k, lf, psi, sc);
        else gather_spinor16<S>(in[k], nf, psi, sc);
        if (flip_f) sc = -sc;
        hop16<MU, DAGGER ? +1 : -1, false, S, BASIS>(acc[k], psi, U, sc, one);
      } else {
        Spinor<R> psi;
        gather_spinor<S>(in[k], nf, psi);
        hop<MU, DAGGER ? +1 : -1, false, BASIS>(acc[k], psi, U, flip_f ? R(-1) : R(1));
      }
    }
  }
  // FP64 spinors are large enough that one hop's loads fill the registers
  if constexpr (S::prec == WD_FP64) hop_fence<R, NR>(acc);
  // backward: (1 + gamma_mu) U_{x-mu}^mu^dagger psi(x - mu); adjoint: (1 - gamma_mu)
  if constexpr (S::prec == WD_HALF_F16) {
    Link16 U;
    link_of16<S, RECON, (NR == 1 ? kStream : 0)>(g, links, 1 - p, MU, nb, unit_b, U);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if constexpr (MU == 3 && BASIS == kBasisUK) {
        constexpr int BASE = DAGGER ? 2 : 0;
        uint32_t w[6];
        float s16;
        gather_half16w<BASE>(in[k], nb, w, s16);
        mul_acc_half16<true, BASE>(acc[k], w, U, flip_b ? -2.0f * s16 : 2.0f * s16);
      } else {
        Raw16 psi;
        float sc;
        if (LDS && lb >= 0) lds_gather16<S>(lc, k, lb, psi, sc);
        else gather_spinor16<S>(in[k], nb, psi, sc);
        if (flip_b) sc = -sc;
        hop16d<MU, DAGGER ? -1 : +1, true, BASIS>(acc[k], psi, U, sc);
      }
    }
  } else {
    Link<R> U;
    if (unit_b) unit_link(U);
    else gather_link<S, RECON, (NR == 1 ? kStream : 0)>(g, links, 1 - p, MU, nb, U);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if constexpr (MU == 3 && BASIS == kBasisUK) {
        // 1 + gamma_t keeps the upper spins, its adjoint 1 - gamma_t the lower ones
        constexpr int BASE = DAGGER ? 2 : 0;
        cx<R> h[2][3];
        R sc = R(2);
        if constexpr (kHalf<S>) {
          float s16;
          gather_half16<S, BASE>(in[k], nb, h, s16);
          sc = 2.0f * s16;
        } else {
          gather_half<S, BASE>(in[k], nb, h);
        }
        mul_acc_half<true, BASE>(acc[k], h, U, flip_b ? -sc : sc);
      } else if constexpr (kHalf<S>) {
        Raw16 psi;
        float sc;
        if (LDS && lb >= 0) lds_gather16<S>(lc, k, lb, psi, sc);
        else gather_spinor16<S>(in[k], nb, psi, sc);
        if (flip_b) sc = -sc;
        hop16<MU, DAGGER ? -1 : +1, true, S, BASIS>(acc[k], psi, U, sc, one);
      } else {
        Spinor<R> psi;
        gather_spinor<S>(in[k], nb, psi);
        hop<MU, DAGGER ? -1 : +1, true, BASIS>(acc[k], psi, U, flip_b ? R(-1) : R(1));
      }
    }
  }
}

// out = D in, or out = x + a * D in (XPAY), optionally followed by per-block
// FP64 partial dot products of the result (DOT):
//   DOT_YO: <y, out>                 (complex; BiCGstab <r~, v>)
//   DOT_OX: <out, x>, |out|^2        (BiCGstab <t, s>, <t, t> with x = s)
//   DOT_OO: |out|^2                  (CG |M p|^2)
//   DOT_RES: out = y - (x + a * D in), |out|^2 (FP64 residual b_hat - M_hat x)
//   DOT_RES_ENC: r = y - (x + a * D in) re-encoded in format S2 into enc.rh
//     (out is not written), enc.xh = 0, with enc.set_rt also enc.rt = enc(r);
//     |r|^2, |enc(r)|^2, <enc.rt, enc(r)>
//   DOT_ENC: x + a * D^dag in encoded in format S2 into enc.rh (out is not
//     written), enc.xh = 0; |enc.rh|^2
// Right-hand sides whose active flag in `sel` is 0 are skipped; with g.mapped,
// `sel` instead lists the g.nrhs right-hand sides to process, packed into the
// RHS slots of as few groups as they fill.  BASIS: spin basis of in, out, x
// and y (kBasisDR or kBasisUK); the links do not depend on it.
struct EncView {
  FieldView rh, xh, rt;
  int set_rt;
};

// The epilogue fuses its products explicitly.  Left to the compiler, x + a*acc
// (x itself a product once decoded from 16 bits) and the two terms of a
// complex product can each be fused either way, and kernels that inline the
// same code have been compiled to different choices, so results depended on
// the launch shape.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
// re + i im += conj(u) v, one term at a time
template <class R>
__device__ __forceinline__ void acc_cdotc(R& re, R& im, const cx<R>& u, const cx<R>& v) {
  re = fmad(u.re, v.re, re);
  re = fmad(u.im, v.im, re);
  im = fmad(u.re, v.im, im);
  im = fmad(-u.im, v.re, im);
}
// nn += |u|^2
template <class R, class T>
__device__ __forceinline__ void acc_norm(T& nn, const cx<R>& u) {
  nn = fmad(T(u.re), T(u.re), nn);
  nn = fmad(T(u.im), T(u.im), nn);
}

// Per right-hand side after the hops: xpay, residual, store (or re-encode)
// and the fused FP64 partial dot products of one workgroup.  Every thread of
// the block calls it for the same r (the reductions synchronise the block).
template <class S, bool XPAY, int DOT, class S2>
__device__ __forceinline__ void finish_rhs(const DslashGeom& g, Spinor<typename S::real>& acc, int r, int cb,
                                           bool valid, int pid, FieldView out, FieldView xs, FieldView ys,
                                           typename S::real a, double* __restrict__ partials, const EncView& enc) {
  using R = typename S::real;
  Spinor<R> x;
  if (valid) {
    if constexpr (XPAY) {
      load_spinor<S>(xs, r, cb, x);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          acc.v[s][c] = {fmad(a, acc.v[s][c].re, x.v[s][c].re), fmad(a, acc.v[s][c].im, x.v[s][c].im)};
    }
    if constexpr (DOT == DOT_RES || DOT == DOT_RES_ENC) {
      Spinor<R> b;
      load_spinor<S>(ys, r, cb, b);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.v[s][c] = b.v[s][c] - acc.v[s][c];
    }
    if constexpr (DOT != DOT_RES_ENC && DOT != DOT_ENC) {
      if (g.out_nt) store_spinor<S, true>(out, r, cb, acc);
      else store_spinor<S>(out, r, cb, acc);
    }
  }
  if constexpr (DOT == DOT_ENC) {
    using R2 = typename S2::real;
    double d[1] = {0.0};
    if (valid) {
      Spinor<R2> e, z;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          e.v[s][c] = {static_cast<R2>(acc.v[s][c].re), static_cast<R2>(acc.v[s][c].im)};
          z.v[s][c] = {R2(0), R2(0)};
        }
      store_spinor<S2>(enc.rh, r, cb, e);
      store_spinor<S2>(enc.xh, r, cb, z);
      load_spinor<S2>(enc.rh, r, cb, e);  // the norm of the stored (re-encoded) value
      R2 n2 = 0;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc_norm(n2, e.v[s][c]);
      d[0] = n2;
    }
    const int nb = (g.slab ? 8 : 1) * g.site_blocks;
    block_sum_store<1>(d, partials + ((int64_t)r * nb + pid) * kMaxDot);
  }
  if constexpr (DOT == DOT_RES_ENC) {
    using R2 = typename S2::real;
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      Spinor<R2> e, z, t;
      double nn = 0.0;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc_norm(nn, acc.v[s][c]);
          e.v[s][c] = {static_cast<R2>(acc.v[s][c].re), static_cast<R2>(acc.v[s][c].im)};
          z.v[s][c] = {R2(0), R2(0)};
        }
      store_spinor<S2>(enc.rh, r, cb, e);
      store_spinor<S2>(enc.xh, r, cb, z);
      if (enc.set_rt) store_spinor<S2>(enc.rt, r, cb, e);
      // the dots see the stored (re-encoded) residual
      load_spinor<S2>(enc.rh, r, cb, e);
      load_spinor<S2>(enc.rt, r, cb, t);
      R2 n2 = 0, re = 0, im = 0;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc_norm(n2, e.v[s][c]);
          acc_cdotc(re, im, t.v[s][c], e.v[s][c]);
        }
      d[0] = nn;
      d[1] = n2;
      d[2] = re;
      d[3] = im;
    }
    const int nb = (g.slab ? 8 : 1) * g.site_blocks;
    block_sum_store<4>(d, partials + ((int64_t)r * nb + pid) * kMaxDot);
  }
  if constexpr (DOT != DOT_NONE && DOT != DOT_RES_ENC && DOT != DOT_ENC) {
    const int nb = (g.slab ? 8 : 1) * g.site_blocks;
    double* part = partials + ((int64_t)r * nb + pid) * kMaxDot;
    if constexpr (DOT == DOT_YO) {
      double d[2] = {0.0, 0.0};
      if (valid) {
        Spinor<R> y;
        load_spinor<S>(ys, r, cb, y);
        R re = 0, im = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc_cdotc(re, im, y.v[s][c], acc.v[s][c]);
        d[0] = re;
        d[1] = im;
      }
      block_sum_store<2>(d, part);
    } else if constexpr (DOT == DOT_OX) {
      double d[3] = {0.0, 0.0, 0.0};
      if (valid) {
        R re = 0, im = 0, nn = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc_cdotc(re, im, acc.v[s][c], x.v[s][c]);
            acc_norm(nn, acc.v[s][c]);
          }
        d[0] = re;
        d[1] = im;
        d[2] = nn;
      }
      block_sum_store<3>(d, part);
    } else {
      double d[1] = {0.0};
      if (valid) {
        R nn = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc_norm(nn, acc.v[s][c]);
        d[0] = nn;
      }
      block_sum_store<1>(d, part);
    }
  }
}

template <class S, bool DAGGER, bool XPAY, int DOT, int NR, int RECON, bool LDS, int BASIS, class S2 = S>
__global__ void __launch_bounds__(kBlock) dslash_kernel(DslashGeom g, const char* __restrict__ links,
                                                       FieldView out, FieldView in, FieldView xs,
                                                       FieldView ys, typename S::real a, int p,
                                                       const int* __restrict__ sel,
                                                       double* __restrict__ partials, EncView enc) {
  using R = typename S::real;
  // ---- which sites and RHS this workgroup owns ----
  const int xcd = blockIdx.x & 7;
  const int j = blockIdx.x >> 3;
  int site_block, group, pid, cb;
  int xh = 0, X1 = 0, X2 = 0, X3 = 0;  // site coordinates (x / 2, y, z, t)
  bool valid;
  if (g.slab) {
    if (g.gslow) {
      group = j / g.site_blocks;
      site_block = j - group * g.site_blocks;
    } else {
      site_block = j / g.ngroups;
      group = j - site_block * g.ngroups;
    }
    if (site_block >= g.site_blocks || group >= g.ngroups) return;
    pid = xcd * g.site_blocks + site_block;
    // position in this XCD's slab: sub-slab (slowest), t, z, y, x/2 (fastest);
    // a thread past the end works on the last site and stores nothing
    const int s_raw = site_block * blockDim.x + threadIdx.x;
    valid = s_raw < (g.Vh >> 3);
    const int s_local = valid ? s_raw : (g.Vh >> 3) - 1;
    const int sub = (int)fdiv((uint32_t)s_local, g.div_sub);
    const int r1 = s_local - sub * g.sub_sites;
    X3 = (int)fdiv((uint32_t)r1, g.div_sub_t);
    const int r2 = r1 - X3 * g.sub_t_sites;
    const int zl = (int)fdiv((uint32_t)r2, g.div_sub_plane);
    const int r3 = r2 - zl * g.sub_plane;
    const int yl = (int)fdiv((uint32_t)r3, g.div_lxh);
    xh = r3 - yl * g.Lxh;
    X1 = sub * (g.L[1] / g.nsub) + yl;
    X2 = xcd * (g.L[2] >> 3) + zl;
    cb = xh + g.Lxh * (X1 + g.L[1] * (X2 + g.L[2] * X3));
  } else {
    const int per = (g.site_blocks * g.ngroups + 7) >> 3;
    const int L = xcd * per + j;
    if (j >= per || L >= g.site_blocks * g.ngroups) return;
    site_block = L / g.ngroups;
    group = L - site_block * g.ngroups;
    pid = site_block;
    cb = site_block * blockDim.x + threadIdx.x;
    valid = cb < g.Vh;
    if (!valid) cb = g.Vh - 1;  // works on the last site and stores nothing
    const int row = (int)fdiv((uint32_t)cb, g.div_lxh);
    xh = cb - row * g.Lxh;
    const int zt = (int)fdiv((uint32_t)row, g.div_ly);
    X1 = row - zt * g.L[1];
    X3 = (int)fdiv((uint32_t)zt, g.div_lz);
    X2 = zt - X3 * g.L[2];
  }
  int rhs[NR];
  bool on[NR];
  bool any = false;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int slot = group * NR + k;
    if (g.mapped) {
      on[k] = slot < g.nrhs;
      rhs[k] = on[k] ? sel[slot] : 0;
    } else {
      rhs[k] = slot;
      on[k] = slot < g.nrhs && (!sel || sel[slot]);
    }
    any |= on[k];
  }
  if (!any) return;

  // LDS staging (uniform per workgroup: every thread takes part before the barrier)
  LdsCtx lc{nullptr, nullptr, 0, 0, 0, 0};
  if constexpr (LDS) {
    extern __shared__ uint4 lds_raw[];
    SpinorBuf<S> sb[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) sb[k] = spinor_buf<S>(in, on[k] ? rhs[k] : 0);
    uint4* chunks = lds_raw;
    float* norms = reinterpret_cast<float*>(lds_raw + NR * 3 * g.lds_cap);
    int* rowbase = reinterpret_cast<int*>(norms + NR * g.lds_cap);
    int base;
    lds_stage<S, NR>(g, xcd, site_block, sb, on, chunks, norms, rowbase, &base);
    __syncthreads();
    const int s_lds = valid ? site_block * (int)blockDim.x + (int)threadIdx.x : (g.Vh >> 3) - 1;
    lc = LdsCtx{chunks, norms, g.lds_cap, base, (int)fdiv((uint32_t)s_lds, g.div_lxh), X1 - (X1 / g.suby) * g.suby};
  }

  Spinor<R> acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[k].v[s][c] = {R(0), R(0)};
  {
    // coordinates of the output site (cb, parity p)
    const int row = X1 + g.L[1] * (X2 + g.L[2] * X3);
    const int X[4] = {2 * xh + ((p + X1 + X2 + X3) & 1), X1, X2, X3};
    const float one = pin_f32(1.0f);  // see proj16
    SpinorBuf<S> ib[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) ib[k] = spinor_buf<S>(in, on[k] ? rhs[k] : 0, on[k]);
    hop_pair<S, 0, DAGGER, NR, RECON, LDS, BASIS>(acc, g, links, ib, on, p, cb, xh, row, X, one, lc);
    hop_fence<R, NR>(acc);
    hop_pair<S, 1, DAGGER, NR, RECON, LDS, BASIS>(acc, g, links, ib, on, p, cb, xh, row, X, one, lc);
    hop_fence<R, NR>(acc);
    hop_pair<S, 2, DAGGER, NR, RECON, LDS, BASIS>(acc, g, links, ib, on, p, cb, xh, row, X, one, lc);
    hop_fence<R, NR>(acc);
    hop_pair<S, 3, DAGGER, NR, RECON, LDS, BASIS>(acc, g, links, ib, on, p, cb, xh, row, X, one, lc);
    hop_fence<R, NR>(acc);
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (!on[k]) continue;  // uniform across the block
    finish_rhs<S, XPAY, DOT, S2>(g, acc[k], rhs[k], cb, valid, pid, out, xs, ys, a, partials, enc);
  }
}

// ---- binary16, one thread per site for every right-hand side -----------------
// Neighbour indices, boundary signs and unit-link flags of direction MU for
// the output site (as computed inside hop_pair).
struct HopIdx {
  int nf, nb;
  bool flip_f, flip_b, unit_f, unit_b;
};
template <int MU>
__device__ __forceinline__ HopIdx hop_index(const DslashGeom& g, int xh, int row, const int (&X)[4]) {
  HopIdx h;
  h.flip_f = h.flip_b = h.unit_f = h.unit_b = false;
  if constexpr (MU == 0) {
    const int xf = (X[0] + 1 == g.L[0]) ? 0 : X[0] + 1;
    const int xb = (X[0] == 0) ? g.L[0] - 1 : X[0] - 1;
    h.nf = (xf >> 1) + g.Lxh * row;
    h.nb = (xb >> 1) + g.Lxh * row;
  } else {
    int step = 1;
    if constexpr (MU >= 2) step *= g.L[1];
    if constexpr (MU == 3) step *= g.L[2];
    const int rf = (X[MU] + 1 == g.L[MU]) ? row - (g.L[MU] - 1) * step : row + step;
    const int rb = (X[MU] == 0) ? row + (g.L[MU] - 1) * step : row - step;
    h.nf = xh + g.Lxh * rf;
    h.nb = xh + g.Lxh * rb;
    if constexpr (MU == 3) {
      h.flip_f = g.tap && (X[3] == g.L[3] - 1);
      h.flip_b = g.tap && (X[3] == 0);
      h.unit_f = g.tgauge && X[3] != g.L[3] - 1;
      h.unit_b = g.tgauge && X[3] != 0;
    }
  }
  return h;
}

// Both hops of direction MU for one right-hand side, links given.
// With LDS, lf / lb >= 0 name the staged slots of the forward / backward
// neighbour (x and in-plane y hops).
template <int MU, bool DAGGER, int BASIS, bool LDS>
__device__ __forceinline__ void hop_pair16(Spinor<float>& acc, const SpinorBuf<SF16>& ib, const HopIdx& h,
                                           const Link16& Uf, const Link16& Ub, const LdsCtx& lc, int lf, int lb) {
  if constexpr (MU == 3 && BASIS == kBasisUK) {
    constexpr int BF = DAGGER ? 0 : 2, BB = DAGGER ? 2 : 0;
    uint32_t w[6];
    float s16;
    gather_half16w<BF>(ib, h.nf, w, s16);
    mul_acc_half16<false, BF>(acc, w, Uf, h.flip_f ? -2.0f * s16 : 2.0f * s16);
    gather_half16w<BB>(ib, h.nb, w, s16);
    mul_acc_half16<true, BB>(acc, w, Ub, h.flip_b ? -2.0f * s16 : 2.0f * s16);
  } else {
    Raw16 psi;
    float sc;
    if (LDS && lf >= 0) lds_gather16<SF16>(lc, 0, lf, psi, sc);
    else gather_spinor16<SF16>(ib, h.nf, psi, sc);
    hop16d<MU, DAGGER ? +1 : -1, false, BASIS>(acc, psi, Uf, h.flip_f ? -sc : sc);
    if (LDS && lb >= 0) lds_gather16<SF16>(lc, 0, lb, psi, sc);
    else gather_spinor16<SF16>(ib, h.nb, psi, sc);
    hop16d<MU, DAGGER ? -1 : +1, true, BASIS>(acc, psi, Ub, h.flip_b ? -sc : sc);
  }
}

template <int MU>
__device__ __forceinline__ void link_pair16(const DslashGeom& g, const char* links, int p, int cb, const HopIdx& h,
                                            Link16& Uf, Link16& Ub) {
  link_of16<SF16, 12, 0>(g, links, p, MU, cb, h.unit_f, Uf);
  link_of16<SF16, 12, 0>(g, links, 1 - p, MU, h.nb, h.unit_b, Ub);
}

// One thread computes one output site for every right-hand side of the
// launch, one after another: the site's eight links (12 reals, binary16) are
// gathered once and held in registers for all of them, and only one
// right-hand side's neighbours are in flight at a time.  The workgroups
// running together on an XCD then share a working set of one right-hand side
// per site instead of all of them, so the t- and z-neighbours fetched by one
// workgroup are still in L2 when the next needs them, and each link is read
// once per launch.  Sites map to workgroups as in dslash_kernel with a single
// RHS group; the arithmetic per right-hand side is that of dslash_kernel, so
// results are bitwise the same.  With LDS (slab mapping only) the workgroup
// stages the x/y neighbour rows of each RHS in LDS (the rows of lds_stage),
// double-buffered: the rows of the next RHS are loaded straight into the
// other buffer while the current RHS computes, and one wait plus barrier per
// RHS hands the buffers over.
template <bool DAGGER, bool XPAY, int DOT, int BASIS, bool LDS, class S2 = SF16>
__global__ void __launch_bounds__(512) dslash16_rloop_kernel(DslashGeom g, const char* __restrict__ links,
                                                               FieldView out, FieldView in, FieldView xs,
                                                               FieldView ys, float a, int p,
                                                               const int* __restrict__ sel,
                                                               double* __restrict__ partials, EncView enc) {
  const int xcd = blockIdx.x & 7;
  const int j = blockIdx.x >> 3;
  int site_block, pid, cb;
  int xh = 0, X1 = 0, X2 = 0, X3 = 0;
  bool valid;
  if (g.slab) {
    site_block = j;
    if (site_block >= g.site_blocks) return;
    pid = xcd * g.site_blocks + site_block;
    const int s_raw = site_block * blockDim.x + threadIdx.x;
    valid = s_raw < (g.Vh >> 3);
    const int s_local = valid ? s_raw : (g.Vh >> 3) - 1;
    const int sub = (int)fdiv((uint32_t)s_local, g.div_sub);
    const int r1 = s_local - sub * g.sub_sites;
    X3 = (int)fdiv((uint32_t)r1, g.div_sub_t);
    const int r2 = r1 - X3 * g.sub_t_sites;
    const int zl = (int)fdiv((uint32_t)r2, g.div_sub_plane);
    const int r3 = r2 - zl * g.sub_plane;
    const int yl = (int)fdiv((uint32_t)r3, g.div_lxh);
    xh = r3 - yl * g.Lxh;
    X1 = sub * (g.L[1] / g.nsub) + yl;
    X2 = xcd * (g.L[2] >> 3) + zl;
    cb = xh + g.Lxh * (X1 + g.L[1] * (X2 + g.L[2] * X3));
  } else {
    const int per = (g.site_blocks + 7) >> 3;
    const int L = xcd * per + j;
    if (j >= per || L >= g.site_blocks) return;
    site_block = L;
    pid = site_block;
    cb = site_block * blockDim.x + threadIdx.x;
    valid = cb < g.Vh;
    if (!valid) cb = g.Vh - 1;
    const int row = (int)fdiv((uint32_t)cb, g.div_lxh);
    xh = cb - row * g.Lxh;
    const int zt = (int)fdiv((uint32_t)row, g.div_ly);
    X1 = row - zt * g.L[1];
    X3 = (int)fdiv((uint32_t)zt, g.div_lz);
    X2 = zt - X3 * g.L[2];
  }
  const int row = X1 + g.L[1] * (X2 + g.L[2] * X3);
  const int X[4] = {2 * xh + ((p + X1 + X2 + X3) & 1), X1, X2, X3};
  const HopIdx h0 = hop_index<0>(g, xh, row, X), h1 = hop_index<1>(g, xh, row, X);
  const HopIdx h2 = hop_index<2>(g, xh, row, X), h3 = hop_index<3>(g, xh, row, X);
  Link16 Uf[4], Ub[4];
  link_pair16<0>(g, links, p, cb, h0, Uf[0], Ub[0]);
  link_pair16<1>(g, links, p, cb, h1, Uf[1], Ub[1]);
  link_pair16<2>(g, links, p, cb, h2, Uf[2], Ub[2]);
  link_pair16<3>(g, links, p, cb, h3, Uf[3], Ub[3]);
  LdsCtx lc{nullptr, nullptr, 0, 0, 0, 0};
  [[maybe_unused]] uint4* lchunks = nullptr;  // [buffer][3][cap]
  [[maybe_unused]] float* lnorms = nullptr;   // [buffer][cap]
  [[maybe_unused]] int* rowbase = nullptr;
  int lf0 = -1, lb0 = -1, lf1 = -1, lb1 = -1;
  if constexpr (LDS) {
    extern __shared__ uint4 lds_raw[];
    lchunks = lds_raw;
    lnorms = reinterpret_cast<float*>(lds_raw + 6 * g.lds_cap);
    rowbase = reinterpret_cast<int*>(lnorms + 2 * g.lds_cap);
    const int base = lds_rows(g, xcd, site_block, rowbase);
    const int s_lds = valid ? site_block * (int)blockDim.x + (int)threadIdx.x : (g.Vh >> 3) - 1;
    lc = LdsCtx{lchunks, lnorms, g.lds_cap, base, (int)fdiv((uint32_t)s_lds, g.div_lxh), X1 - (X1 / g.suby) * g.suby};
    const int r0 = (lc.row - lc.base) * g.Lxh;
    lf0 = r0 + (h0.nf - g.Lxh * row);
    lb0 = r0 + (h0.nb - g.Lxh * row);
    if (lc.yl + 1 < g.suby) lf1 = (lc.row + 1 - lc.base) * g.Lxh + xh;
    if (lc.yl > 0) lb1 = (lc.row - 1 - lc.base) * g.Lxh + xh;
  }
  // RHS of batch slot k (with a map: the listed one) and the next slot from k
  // on that is active; all uniform across the block
  auto rhs_of = [&](int k) { return g.mapped ? sel[k] : k; };
  auto next_active = [&](int k) {
    if (!g.mapped && sel)
      while (k < g.nrhs && !sel[k]) ++k;
    return k;
  };
  int slot = next_active(0);
  int buf = 0;
  if constexpr (LDS) {
    __syncthreads();  // the row table is written
    if (slot < g.nrhs) lds_issue16(g, spinor_buf<SF16>(in, rhs_of(slot)), lchunks, lnorms, rowbase);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  while (slot < g.nrhs) {
    const int r = rhs_of(slot);
    const int nxt = next_active(slot + 1);
    const SpinorBuf<SF16> ib = spinor_buf<SF16>(in, r);
    if constexpr (LDS) {
      // the next RHS's rows go into the other buffer while this one computes
      if (nxt < g.nrhs)
        lds_issue16(g, spinor_buf<SF16>(in, rhs_of(nxt)), lchunks + 3 * g.lds_cap * (buf ^ 1),
                    lnorms + g.lds_cap * (buf ^ 1), rowbase);
      lc.chunks = lchunks + 3 * g.lds_cap * buf;
      lc.norms = lnorms + g.lds_cap * buf;
    }
    Spinor<float> acc[1];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[0].v[s][c] = {0.0f, 0.0f};
    hop_pair16<0, DAGGER, BASIS, LDS>(acc[0], ib, h0, Uf[0], Ub[0], lc, lf0, lb0);
    hop_fence<float, 1>(acc);
    hop_pair16<1, DAGGER, BASIS, LDS>(acc[0], ib, h1, Uf[1], Ub[1], lc, lf1, lb1);
    hop_fence<float, 1>(acc);
    hop_pair16<2, DAGGER, BASIS, LDS>(acc[0], ib, h2, Uf[2], Ub[2], lc, -1, -1);
    hop_fence<float, 1>(acc);
    hop_pair16<3, DAGGER, BASIS, LDS>(acc[0], ib, h3, Uf[3], Ub[3], lc, -1, -1);
    hop_fence<float, 1>(acc);
    finish_rhs<SF16, XPAY, DOT, S2>(g, acc[0], r, cb, valid, pid, out, xs, ys, a, partials, enc);
    if constexpr (LDS) {
      // this wave's copies of the next RHS have landed and its reads of this
      // buffer are done; after the barrier every wave's are
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    slot = nxt;
    buf ^= 1;
  }
}

// ---- launch configuration ---------------------------------------------------------
static DslashGeom make_dgeom(const Geom& geo, int nrhs, const LaunchCfg& c) {
  DslashGeom g;
  for (int m = 0; m < 4; ++m) g.L[m] = geo.L[m];
  g.Lxh = geo.Lxh;
  g.Vh = geo.Vh;
  g.tap = geo.tap;
  g.stride = geo.stride;
  g.div_lxh = make_fastdiv(geo.Lxh);
  g.div_ly = make_fastdiv(geo.L[1]);
  g.div_lz = make_fastdiv(geo.L[2]);
  g.nrhs = nrhs;
  g.mapped = 0;
  g.ngroups = (nrhs + c.nr - 1) / c.nr;
  g.gslow = c.gslow;
  g.link_nt = c.link_nt;
  g.out_nt = c.out_nt;
  g.tgauge = 0;
  g.slab = (geo.L[2] % 8 == 0) ? 1 : 0;
  g.nsub = (c.nsub >= 1 && geo.L[1] % c.nsub == 0) ? c.nsub : 1;
  g.sub_plane = geo.Lxh * (geo.L[1] / g.nsub);
  g.sub_t_sites = g.sub_plane * (geo.L[2] / 8);
  g.sub_sites = g.sub_t_sites * geo.L[3];
  g.div_sub = make_fastdiv(g.sub_sites > 0 ? g.sub_sites : 1);
  g.div_sub_t = make_fastdiv(g.sub_t_sites > 0 ? g.sub_t_sites : 1);
  g.div_sub_plane = make_fastdiv(g.sub_plane > 0 ? g.sub_plane : 1);
  if (g.slab) g.site_blocks = ((geo.Vh >> 3) + c.block - 1) / c.block;
  else g.site_blocks = (geo.Vh + c.block - 1) / c.block;
  g.suby = geo.L[1] / g.nsub;
  g.div_suby = make_fastdiv(g.suby);
  g.div_zl = make_fastdiv(geo.L[2] >= 8 ? geo.L[2] / 8 : 1);
  g.div_lt = make_fastdiv(geo.L[3]);
  g.slab_rows = g.slab ? (geo.Vh >> 3) / geo.Lxh : 0;
  g.lds_cap = ((c.block + geo.Lxh - 1) / geo.Lxh + 3) * geo.Lxh;
  return g;
}

static unsigned grid_blocks(const DslashGeom& g) {
  if (g.slab) return 8u * (unsigned)(g.site_blocks * g.ngroups);
  const unsigned per = (unsigned)((g.site_blocks * g.ngroups + 7) / 8);
  return 8u * per;
}

static FieldView fview(const Field& f) { return FieldView{f.ptr, f.stride, f.nrhs}; }
static FieldView fview(const Field* f) { return f ? fview(*f) : FieldView{nullptr, 0, 0}; }

// LDS reserved per workgroup (unused by the kernel) so that at most `wgs`
// workgroups fit on a CU (160 KiB of LDS); 0 leaves occupancy to registers.
static size_t lds_for(int wgs) {
  if (wgs < 2) return 0;
  const size_t per = (size_t(160) * 1024 / wgs) / 512 * 512;
  return per > 63488 ? 63488 : per;  // below the 64 KiB per-workgroup limit with the static LDS
}

// LDS bytes of the x/y staging: per RHS slot 3 chunks + 1 norm per staged
// site, and one row-start index per staged row.
static size_t lds_stage_bytes(const DslashGeom& g, int nr) {
  return ((size_t)nr * g.lds_cap * 52 + (size_t)(g.lds_cap / g.Lxh) * 4 + 15) / 16 * 16;
}

// The fused dot products serve the solvers, which work in the UKQCD basis;
// DeGrand-Rossi launches are built without them.
template <class S, bool DAGGER, bool XPAY, int NR, int RECON, bool LDS, int BASIS>
static void launch_dot(int dot, unsigned grid, int block, size_t lds, hipStream_t s, const DslashGeom& g,
                       const char* links, FieldView fo, FieldView fi, FieldView fx, FieldView fy,
                       typename S::real a, int p, const int* sel, double* partials, EncView enc,
                       wd_prec enc_prec) {
  if constexpr (BASIS == kBasisDR) {
    dslash_kernel<S, DAGGER, XPAY, DOT_NONE, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
  } else {
    switch (dot) {
      case DOT_YO:
        dslash_kernel<S, DAGGER, XPAY, DOT_YO, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_OX:
        dslash_kernel<S, DAGGER, XPAY, DOT_OX, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_OO:
        dslash_kernel<S, DAGGER, XPAY, DOT_OO, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_RES:
        if constexpr (S::prec == WD_FP64 && XPAY && !DAGGER && !LDS)
          dslash_kernel<S, DAGGER, XPAY, DOT_RES, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_RES_ENC:
        if constexpr (S::prec == WD_FP64 && XPAY && !DAGGER && !LDS) {
          switch (enc_prec) {
            case WD_FP32:
              dslash_kernel<S, DAGGER, XPAY, DOT_RES_ENC, NR, RECON, LDS, BASIS, SF32><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
              break;
            case WD_HALF_I16:
              dslash_kernel<S, DAGGER, XPAY, DOT_RES_ENC, NR, RECON, LDS, BASIS, SI16><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
              break;
            default:
              dslash_kernel<S, DAGGER, XPAY, DOT_RES_ENC, NR, RECON, LDS, BASIS, SF16><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
          }
        }
        break;
      case DOT_ENC:
        if constexpr (S::prec == WD_FP64 && XPAY && DAGGER && !LDS) {
          switch (enc_prec) {
            case WD_FP32:
              dslash_kernel<S, DAGGER, XPAY, DOT_ENC, NR, RECON, LDS, BASIS, SF32><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
              break;
            case WD_HALF_I16:
              dslash_kernel<S, DAGGER, XPAY, DOT_ENC, NR, RECON, LDS, BASIS, SI16><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
              break;
            default:
              dslash_kernel<S, DAGGER, XPAY, DOT_ENC, NR, RECON, LDS, BASIS, SF16><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
          }
        }
        break;
      default:
        dslash_kernel<S, DAGGER, XPAY, DOT_NONE, NR, RECON, LDS, BASIS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
    }
  }
}

template <class S, int NR, int RECON, bool LDS, int BASIS>
static void launch_nr(const wd_gauge* gg, const DslashArgs& d, const LaunchCfg& cfg, hipStream_t s) {
  LaunchCfg c = cfg;
  c.nr = NR;  // the RHS slots of the kernel actually launched
  if (c.block != 128) c.block = 256;  // the slot kernels are built for at most 256 threads
  DslashGeom g = make_dgeom(gg->geom, d.rhs_map ? d.n_map : d.out.nrhs, c);
  g.mapped = d.rhs_map ? 1 : 0;
  g.tgauge = gg->tgauge;
  const char* links = static_cast<const char*>(gg->link[S::prec]);
  const unsigned grid = grid_blocks(g);
  FieldView fo = fview(d.out), fi = fview(d.in), fx = fview(d.xpay), fy = fview(d.y);
  using R = typename S::real;
  const R ar = static_cast<R>(d.a);
  const int dot = d.xpay ? d.dot : DOT_NONE;
  const EncView ev{fview(d.enc_rh), fview(d.enc_xh), fview(d.enc_rt), d.enc_set_rt};
  size_t lds = lds_for(c.wgs);
  if constexpr (LDS) lds = std::max(lds, lds_stage_bytes(g, NR));
  if (d.dagger) {
    if (d.xpay) launch_dot<S, true, true, NR, RECON, LDS, BASIS>(dot, grid, c.block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.rhs_map ? d.rhs_map : d.active, d.partials, ev, d.enc_prec);
    else launch_dot<S, true, false, NR, RECON, LDS, BASIS>(DOT_NONE, grid, c.block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.rhs_map ? d.rhs_map : d.active, d.partials, ev, d.enc_prec);
  } else {
    if (d.xpay) launch_dot<S, false, true, NR, RECON, LDS, BASIS>(dot, grid, c.block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.rhs_map ? d.rhs_map : d.active, d.partials, ev, d.enc_prec);
    else launch_dot<S, false, false, NR, RECON, LDS, BASIS>(DOT_NONE, grid, c.block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.rhs_map ? d.rhs_map : d.active, d.partials, ev, d.enc_prec);
  }
}

template <bool DAGGER, bool XPAY, int BASIS, bool LDS>
static void launch_rloop_dot(int dot, unsigned grid, int block, size_t lds, hipStream_t s, const DslashGeom& g,
                             const char* links, FieldView fo, FieldView fi, FieldView fx, FieldView fy, float a, int p,
                             const int* sel, double* partials, EncView enc) {
  if constexpr (BASIS == kBasisDR || !XPAY) {
    dslash16_rloop_kernel<DAGGER, XPAY, DOT_NONE, BASIS, LDS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
  } else {
    switch (dot) {
      case DOT_YO:
        dslash16_rloop_kernel<DAGGER, XPAY, DOT_YO, BASIS, LDS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_OX:
        dslash16_rloop_kernel<DAGGER, XPAY, DOT_OX, BASIS, LDS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      case DOT_OO:
        dslash16_rloop_kernel<DAGGER, XPAY, DOT_OO, BASIS, LDS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
        break;
      default:
        dslash16_rloop_kernel<DAGGER, XPAY, DOT_NONE, BASIS, LDS><<<grid, block, lds, s>>>(g, links, fo, fi, fx, fy, a, p, sel, partials, enc);
    }
  }
}

template <int BASIS, bool LDS>
static void launch_rloop_dag(const DslashArgs& d, unsigned grid, int block, size_t lds, hipStream_t s,
                             const DslashGeom& g, const char* links) {
  FieldView fo = fview(d.out), fi = fview(d.in), fx = fview(d.xpay), fy = fview(d.y);
  const float ar = static_cast<float>(d.a);
  const int dot = d.xpay ? d.dot : DOT_NONE;
  const EncView ev{fview(d.enc_rh), fview(d.enc_xh), fview(d.enc_rt), d.enc_set_rt};
  const int* sel = d.rhs_map ? d.rhs_map : d.active;
  if (d.dagger) {
    if (d.xpay) launch_rloop_dot<true, true, BASIS, LDS>(dot, grid, block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, sel, d.partials, ev);
    else launch_rloop_dot<true, false, BASIS, LDS>(DOT_NONE, grid, block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, sel, d.partials, ev);
  } else {
    if (d.xpay) launch_rloop_dot<false, true, BASIS, LDS>(dot, grid, block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, sel, d.partials, ev);
    else launch_rloop_dot<false, false, BASIS, LDS>(DOT_NONE, grid, block, lds, s, g, links, fo, fi, fx, fy, ar, d.out_parity, sel, d.partials, ev);
  }
}

// The RHS-loop launch (binary16, 12-real links): one RHS group covering the
// whole batch, so the grid is one workgroup per site block.  LDS staging when
// asked for, on the slab mapping, if its rows fit 62 KiB.  Workgroups of
// 128, 256 or 512 threads; a fused dot needs 256 (its block reduction sums
// four waves).
template <int BASIS>
static void launch_rloop(const wd_gauge* gg, const DslashArgs& d, const LaunchCfg& cfg, hipStream_t s) {
  const int n = d.rhs_map ? d.n_map : d.out.nrhs;
  LaunchCfg c = cfg;
  c.nr = n;  // a single RHS group
  if (c.block != 128 && c.block != 512) c.block = 256;
  if (d.xpay && d.dot != DOT_NONE) c.block = 256;
  DslashGeom g = make_dgeom(gg->geom, n, c);
  g.mapped = d.rhs_map ? 1 : 0;
  g.tgauge = gg->tgauge;
  const char* links = static_cast<const char*>(gg->link[WD_HALF_F16]);
  const unsigned grid = grid_blocks(g);
  const size_t stage = lds_stage_bytes(g, 2);  // two buffers of one RHS each
  const size_t cap = lds_for(c.wgs);
  if (cfg.lds && g.slab && stage <= 63488)
    launch_rloop_dag<BASIS, true>(d, grid, c.block, std::max(stage, cap), s, g, links);
  else
    launch_rloop_dag<BASIS, false>(d, grid, c.block, cap, s, g, links);
}

// Threads carry 1 to 4 RHS slots (a slot past the last RHS reads zeros and
// its arithmetic is wasted, so one RHS runs in a one-slot thread).  8-real
// links are built for one and two slots only (their rebuild is long; wider
// shapes gain little when links are a small part of the bytes).
// The LDS-staged variant exists for the 16-bit formats with 12-real links and
// 2 or 3 slots, on the slab mapping, when its staging fits 62 KiB.
static bool lds_usable(const wd_gauge* gg, wd_prec prec, const LaunchCfg& c) {
  if (!c.lds || !is_half(prec) || gg->recon != 12 || gg->geom.L[2] % 8 != 0) return false;
  const int nr = c.nr <= 2 ? 2 : c.nr;
  if (nr > 3) return false;
  LaunchCfg cn = c;
  cn.nr = nr;
  const DslashGeom g = make_dgeom(gg->geom, 1, cn);
  return lds_stage_bytes(g, nr) <= 63488;
}

template <class S, int BASIS>
static void launch_cfg(const wd_gauge* gg, const DslashArgs& d, const LaunchCfg& c, hipStream_t s) {
  if constexpr (S::prec == WD_HALF_F16) {
    if (c.rloop && gg->recon == 12) {
      launch_rloop<BASIS>(gg, d, c, s);
      return;
    }
  }
  if (gg->recon == 8) {
    if (c.nr == 1) launch_nr<S, 1, 8, false, BASIS>(gg, d, c, s);
    else launch_nr<S, 2, 8, false, BASIS>(gg, d, c, s);
    return;
  }
  if constexpr (kHalf<S>) {
    if (lds_usable(gg, S::prec, c)) {
      if (c.nr == 3) launch_nr<S, 3, 12, true, BASIS>(gg, d, c, s);
      else launch_nr<S, 2, 12, true, BASIS>(gg, d, c, s);
      return;
    }
  }
  switch (c.nr) {
    case 1: launch_nr<S, 1, 12, false, BASIS>(gg, d, c, s); break;
    case 3: launch_nr<S, 3, 12, false, BASIS>(gg, d, c, s); break;
    case 4: launch_nr<S, 4, 12, false, BASIS>(gg, d, c, s); break;
    default: launch_nr<S, 2, 12, false, BASIS>(gg, d, c, s); break;
  }
}

}  // namespace wd
