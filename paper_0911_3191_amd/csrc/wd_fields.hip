// Conversions between the caller's canonical FP64 layouts and the device
// field formats: gauge links to 12-real rows (Appendix A.1) in each storage
// precision, spinors to site-coalesced chunk arrays with, for the 16-bit
// formats, a per-site norm (Section 4.6).
#include "wd_device.h"

namespace wd {

struct SiteMap {
  int L[4];
  int Lxh;
  int Vh;
};

// lex index of checkerboard site cb of parity p.
__device__ __forceinline__ int64_t lex_of(const SiteMap& m, int cb, int p) {
  int rest = cb / m.Lxh;
  const int xh = cb - rest * m.Lxh;
  const int y = rest % m.L[1];
  rest /= m.L[1];
  const int z = rest % m.L[2];
  const int t = rest / m.L[2];
  const int x = 2 * xh + ((p + y + z + t) & 1);
  return x + (int64_t)m.L[0] * (y + (int64_t)m.L[1] * (z + (int64_t)m.L[2] * t));
}

static SiteMap site_map(const Geom& g) {
  SiteMap m;
  for (int k = 0; k < 4; ++k) m.L[k] = g.L[k];
  m.Lxh = g.Lxh;
  m.Vh = g.Vh;
  return m;
}

// ---- gauge ------------------------------------------------------------------------
// One thread per (site cb, parity, mu): rows a, b of U[lex][mu] into every
// precision of the mask.  16-bit: int16 q = rint(u * 32767) or binary16 u.
__global__ void gauge_encode_kernel(SiteMap m, const double* __restrict__ U, int64_t stride,
                                    char* f64, char* f32, char* i16, char* h16) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const int par = blockIdx.y >> 2, mu = blockIdx.y & 3;
  if (cb >= m.Vh) return;
  const int64_t lex = lex_of(m, cb, par);
  const double* u = U + (lex * 4 + mu) * 18;  // rows a, b are the first 12 reals
  double v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = u[k];
  if (f64) {
#pragma unroll
    for (int k = 0; k < 6; ++k)
      reinterpret_cast<double2*>(const_cast<char*>(link_chunk<SF64>(f64, stride, par, mu, k)))[cb] =
          make_double2(v[2 * k], v[2 * k + 1]);
  }
  if (f32) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      reinterpret_cast<float4*>(const_cast<char*>(link_chunk<SF32>(f32, stride, par, mu, k)))[cb] =
          make_float4((float)v[4 * k], (float)v[4 * k + 1], (float)v[4 * k + 2], (float)v[4 * k + 3]);
  }
  if (i16) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float a = fminf(fmaxf(rintf((float)v[4 * k + 2 * j] * 32767.0f), -32767.0f), 32767.0f);
        float b = fminf(fmaxf(rintf((float)v[4 * k + 2 * j + 1] * 32767.0f), -32767.0f), 32767.0f);
        w[j] = (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
      }
      reinterpret_cast<uint2*>(const_cast<char*>(link_chunk<SI16>(i16, stride, par, mu, k)))[cb] =
          make_uint2(w[0], w[1]);
    }
  }
  if (h16) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[2];
#pragma unroll
      for (int j = 0; j < 2; ++j)
        w[j] = (uint32_t)f_to_h16(pin_f32((float)v[4 * k + 2 * j])) |
               ((uint32_t)f_to_h16(pin_f32((float)v[4 * k + 2 * j + 1])) << 16);
      reinterpret_cast<uint2*>(const_cast<char*>(link_chunk<SF16>(h16, stride, par, mu, k)))[cb] =
          make_uint2(w[0], w[1]);
    }
  }
}

hipError_t launch_gauge_encode(const wd_gauge* g, const double* U, hipStream_t s) {
  SiteMap m = site_map(g->geom);
  const int block = 256;
  dim3 grid((m.Vh + block - 1) / block, 8);
  gauge_encode_kernel<<<grid, block, 0, s>>>(
      m, U, g->geom.stride, static_cast<char*>(g->link[WD_FP64]), static_cast<char*>(g->link[WD_FP32]),
      static_cast<char*>(g->link[WD_HALF_I16]), static_cast<char*>(g->link[WD_HALF_F16]));
  return hipGetLastError();
}

// ---- spinors ----------------------------------------------------------------------
// Change of spin basis in FP64 (Appendix B), v = [spin][colour][re, im]:
// to_uk: v <- S v with S = [[0, 1, 0, 1], [-1, 0, -1, 0], [0, 1, 0, -1],
// [-1, 0, 1, 0]] / sqrt(2) (DeGrand-Rossi to UKQCD); otherwise v <- S^T v.
__device__ __forceinline__ void change_basis(double (&v)[24], bool to_uk) {
  constexpr double r = 0.70710678118654752440;  // 1 / sqrt(2)
#pragma unroll
  for (int k = 0; k < 6; ++k) {  // colour and re / im
    const double a0 = v[k], a1 = v[6 + k], a2 = v[12 + k], a3 = v[18 + k];
    if (to_uk) {
      v[k] = r * (a1 + a3);
      v[6 + k] = -r * (a0 + a2);
      v[12 + k] = r * (a1 - a3);
      v[18 + k] = r * (a2 - a0);
    } else {
      v[k] = -r * (a1 + a3);
      v[6 + k] = r * (a0 + a2);
      v[12 + k] = r * (a3 - a1);
      v[18 + k] = r * (a0 - a2);
    }
  }
}

// Per-RHS factor of the solver's unit-source scaling: 1 / |b| (scale = 1) or
// |b| (scale = 2) from the solver scalars sc; 1 without scaling or when |b|
// is zero or not finite.
__device__ __forceinline__ double bnorm_factor(const double* __restrict__ sc, int scale, int r) {
  if (!scale) return 1.0;
  const double bn = sc[r * SC_COUNT + SC_BNORM];
  if (!(bn > 0.0) || !isfinite(bn)) return 1.0;
  return scale == 1 ? 1.0 / bn : bn;
}

// One site: 24 canonical reals (DeGrand-Rossi basis) into the field in
// `basis`, times bnorm_factor after the change of basis when scale is set.
template <class S>
__device__ __forceinline__ void encode_site(FieldView f, int r, int cb, const double* __restrict__ src, int basis,
                                            const double* __restrict__ sc, int scale) {
  using R = typename S::real;
  double v[24];
#pragma unroll
  for (int n = 0; n < 24; ++n) v[n] = src[n];
  if (basis == kBasisUK) change_basis(v, true);
  if (scale) {
    const double k = bnorm_factor(sc, scale, r);
#pragma unroll
    for (int n = 0; n < 24; ++n) v[n] = k * v[n];
  }
  Spinor<R> s;
#pragma unroll
  for (int n = 0; n < 12; ++n) s.v[n / 3][n % 3] = {static_cast<R>(v[2 * n]), static_cast<R>(v[2 * n + 1])};
  store_spinor<S>(f, r, cb, s);
}

// One site back: the field's values, times bnorm_factor before the change of
// basis when scale is set, into 24 canonical reals.
template <class S>
__device__ __forceinline__ void decode_site(FieldView f, int r, int cb, double* __restrict__ dst, int basis,
                                            const double* __restrict__ sc, int scale) {
  using R = typename S::real;
  Spinor<R> s;
  load_spinor<S>(f, r, cb, s);
  double v[24];
#pragma unroll
  for (int n = 0; n < 12; ++n) {
    v[2 * n] = static_cast<double>(s.v[n / 3][n % 3].re);
    v[2 * n + 1] = static_cast<double>(s.v[n / 3][n % 3].im);
  }
  if (scale) {
    const double k = bnorm_factor(sc, scale, r);
#pragma unroll
    for (int n = 0; n < 24; ++n) v[n] = k * v[n];
  }
  if (basis == kBasisUK) change_basis(v, false);
#pragma unroll
  for (int n = 0; n < 24; ++n) dst[n] = v[n];
}

// full_parity < 0: canonical array is a parity array [nrhs][Vh][24];
// full_parity = p: canonical array is a full lattice [nrhs][V][24] and the
// field holds its parity-p sites.  The canonical array is in the
// DeGrand-Rossi basis, the field in `basis`.
template <class S>
__global__ void spinor_encode_kernel(SiteMap m, FieldView f, const double* __restrict__ canon,
                                     int full_parity, int basis, const double* __restrict__ sc, int scale) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (cb >= m.Vh) return;
  const int64_t V = 2 * (int64_t)m.Vh;
  const double* src = (full_parity < 0) ? canon + ((int64_t)r * m.Vh + cb) * 24
                                        : canon + ((int64_t)r * V + lex_of(m, cb, full_parity)) * 24;
  encode_site<S>(f, r, cb, src, basis, sc, scale);
}

template <class S>
__global__ void spinor_decode_kernel(SiteMap m, FieldView f, double* __restrict__ canon,
                                     int full_parity, int basis, const double* __restrict__ sc, int scale) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (cb >= m.Vh) return;
  const int64_t V = 2 * (int64_t)m.Vh;
  double* dst = (full_parity < 0) ? canon + ((int64_t)r * m.Vh + cb) * 24
                                  : canon + ((int64_t)r * V + lex_of(m, cb, full_parity)) * 24;
  decode_site<S>(f, r, cb, dst, basis, sc, scale);
}

// Parity of lexicographic site L; its checkerboard index is L / 2 (Lx is even).
__device__ __forceinline__ int parity_of(const SiteMap& m, int64_t L) {
  const int64_t row = L / m.L[0];
  const int x = (int)(L - row * m.L[0]);
  const int y = (int)(row % m.L[1]);
  const int64_t zt = row / m.L[1];
  const int z = (int)(zt % m.L[2]);
  const int t = (int)(zt / m.L[2]);
  return (x + y + z + t) & 1;
}

// Both parities of a canonical full lattice [nrhs][V][24] (FP64 fields) in one
// pass: a workgroup takes kBothSites consecutive lexicographic sites, whose
// canonical records form one contiguous block that is read (or written)
// with 16-byte accesses in address order and passed through LDS; thread k
// works on site L0 + k, whose even / odd sites come from (go to) fe / fo.
constexpr int kBothSites = 256;

__global__ void __launch_bounds__(kBothSites) spinor_encode_both_kernel(SiteMap m, FieldView fe, FieldView fo,
                                                                         const double* __restrict__ canon,
                                                                         int basis, const double* __restrict__ sc,
                                                                         int scale) {
  __shared__ double2 tile[kBothSites * 12];
  const int64_t V = 2 * (int64_t)m.Vh;
  const int64_t L0 = (int64_t)blockIdx.x * kBothSites;
  const int r = blockIdx.y;
  const int n = (int)min((int64_t)kBothSites, V - L0);  // sites in this block
  const double2* src = reinterpret_cast<const double2*>(canon + ((int64_t)r * V + L0) * 24);
  for (int j = threadIdx.x; j < n * 12; j += kBothSites) tile[j] = src[j];
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= n) return;
  const int64_t L = L0 + k;
  encode_site<SF64>(parity_of(m, L) ? fo : fe, r, (int)(L >> 1), reinterpret_cast<const double*>(tile + 12 * k),
                    basis, sc, scale);
}

__global__ void __launch_bounds__(kBothSites) spinor_decode_both_kernel(SiteMap m, FieldView fe, FieldView fo,
                                                                         double* __restrict__ canon, int basis,
                                                                         const double* __restrict__ sc, int scale) {
  __shared__ double2 tile[kBothSites * 12];
  const int64_t V = 2 * (int64_t)m.Vh;
  const int64_t L0 = (int64_t)blockIdx.x * kBothSites;
  const int r = blockIdx.y;
  const int n = (int)min((int64_t)kBothSites, V - L0);
  const int k = threadIdx.x;
  if (k < n) {
    const int64_t L = L0 + k;
    decode_site<SF64>(parity_of(m, L) ? fo : fe, r, (int)(L >> 1), reinterpret_cast<double*>(tile + 12 * k), basis,
                      sc, scale);
  }
  __syncthreads();
  double2* dst = reinterpret_cast<double2*>(canon + ((int64_t)r * V + L0) * 24);
  for (int j = threadIdx.x; j < n * 12; j += kBothSites) dst[j] = tile[j];
}

template <class S>
static hipError_t enc_typed(const Geom& g, Field f, const double* canon, int full_parity, int basis,
                            const double* sc, int scale, hipStream_t s) {
  const int block = 256;
  dim3 grid((g.Vh + block - 1) / block, f.nrhs);
  spinor_encode_kernel<S><<<grid, block, 0, s>>>(site_map(g), FieldView{f.ptr, f.stride, f.nrhs},
                                                 canon, full_parity, basis, sc, scale);
  return hipGetLastError();
}

template <class S>
static hipError_t dec_typed(const Geom& g, double* canon, Field f, int full_parity, int basis,
                            const double* sc, int scale, hipStream_t s) {
  const int block = 256;
  dim3 grid((g.Vh + block - 1) / block, f.nrhs);
  spinor_decode_kernel<S><<<grid, block, 0, s>>>(site_map(g), FieldView{f.ptr, f.stride, f.nrhs},
                                                 canon, full_parity, basis, sc, scale);
  return hipGetLastError();
}

hipError_t launch_spinor_encode_map(const Geom& g, wd_prec p, Field f, const double* canon,
                                    int full_parity, hipStream_t s, int basis, const double* sc,
                                    int scale) {
  if (basis != kBasisDR && basis != kBasisUK) return hipErrorInvalidValue;
  if (scale < 0 || scale > 2 || (scale && !sc)) return hipErrorInvalidValue;
  switch (p) {
    case WD_FP64: return enc_typed<SF64>(g, f, canon, full_parity, basis, sc, scale, s);
    case WD_FP32: return enc_typed<SF32>(g, f, canon, full_parity, basis, sc, scale, s);
    case WD_HALF_I16: return enc_typed<SI16>(g, f, canon, full_parity, basis, sc, scale, s);
    case WD_HALF_F16: return enc_typed<SF16>(g, f, canon, full_parity, basis, sc, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spinor_decode_map(const Geom& g, wd_prec p, double* canon, Field f,
                                    int full_parity, hipStream_t s, int basis, const double* sc,
                                    int scale) {
  if (basis != kBasisDR && basis != kBasisUK) return hipErrorInvalidValue;
  if (scale < 0 || scale > 2 || (scale && !sc)) return hipErrorInvalidValue;
  switch (p) {
    case WD_FP64: return dec_typed<SF64>(g, canon, f, full_parity, basis, sc, scale, s);
    case WD_FP32: return dec_typed<SF32>(g, canon, f, full_parity, basis, sc, scale, s);
    case WD_HALF_I16: return dec_typed<SI16>(g, canon, f, full_parity, basis, sc, scale, s);
    case WD_HALF_F16: return dec_typed<SF16>(g, canon, f, full_parity, basis, sc, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spinor_encode_both(const Geom& g, Field fe, Field fo, const double* canon, hipStream_t s,
                                     int basis, const double* sc, int scale) {
  if (basis != kBasisDR && basis != kBasisUK) return hipErrorInvalidValue;
  if (scale < 0 || scale > 2 || (scale && !sc) || fe.nrhs != fo.nrhs) return hipErrorInvalidValue;
  dim3 grid((unsigned)((2 * (int64_t)g.Vh + kBothSites - 1) / kBothSites), fe.nrhs);
  spinor_encode_both_kernel<<<grid, kBothSites, 0, s>>>(site_map(g), FieldView{fe.ptr, fe.stride, fe.nrhs},
                                                        FieldView{fo.ptr, fo.stride, fo.nrhs}, canon, basis, sc,
                                                        scale);
  return hipGetLastError();
}

hipError_t launch_spinor_decode_both(const Geom& g, double* canon, Field fe, Field fo, hipStream_t s,
                                     int basis, const double* sc, int scale) {
  if (basis != kBasisDR && basis != kBasisUK) return hipErrorInvalidValue;
  if (scale < 0 || scale > 2 || (scale && !sc) || fe.nrhs != fo.nrhs) return hipErrorInvalidValue;
  dim3 grid((unsigned)((2 * (int64_t)g.Vh + kBothSites - 1) / kBothSites), fe.nrhs);
  spinor_decode_both_kernel<<<grid, kBothSites, 0, s>>>(site_map(g), FieldView{fe.ptr, fe.stride, fe.nrhs},
                                                        FieldView{fo.ptr, fo.stride, fo.nrhs}, canon, basis, sc,
                                                        scale);
  return hipGetLastError();
}

hipError_t launch_spinor_encode(const Geom& g, wd_prec p, Field f, const double* canon,
                                hipStream_t s, int basis) {
  return launch_spinor_encode_map(g, p, f, canon, -1, s, basis);
}

hipError_t launch_spinor_decode(const Geom& g, wd_prec p, double* canon, Field f, hipStream_t s,
                                int basis) {
  return launch_spinor_decode_map(g, p, canon, f, -1, s, basis);
}

}  // namespace wd
