// Gauge-field preprocessing on the device, all in FP64:
//  - the 8-real link format (Appendix A.2): a2, a3, b1 and the phases of a1
//    and c1, written in every storage precision of the handle;
//  - the temporal gauge of Section 4.3: g(x,0) = 1, g(x,t+1) = g(x,t) U_t(x,t)
//    along each time line, U'_mu(x) = g(x) U_mu(x) g(x+mu)^dagger, so that
//    every temporal link but those of the last time slice is the unit
//    matrix; spinors rotate as psi'(x) = g(x) psi(x);
//  - the check that a field handed in as temporal-gauge really is one.
#include "wd_device.h"

namespace wd {

namespace {

struct Lat {
  int L[4];
  int Lxh, Vh;
  int64_t V;
};

Lat lat_of(const Geom& g) {
  Lat l;
  for (int k = 0; k < 4; ++k) l.L[k] = g.L[k];
  l.Lxh = g.Lxh;
  l.Vh = g.Vh;
  l.V = 2 * (int64_t)g.Vh;
  return l;
}

__device__ __forceinline__ int64_t lex_cb(const Lat& m, int cb, int p, int* t_out) {
  int rest = cb / m.Lxh;
  const int xh = cb - rest * m.Lxh;
  const int y = rest % m.L[1];
  rest /= m.L[1];
  const int z = rest % m.L[2];
  const int t = rest / m.L[2];
  *t_out = t;
  const int x = 2 * xh + ((p + y + z + t) & 1);
  return x + (int64_t)m.L[0] * (y + (int64_t)m.L[1] * (z + (int64_t)m.L[2] * t));
}

// 3x3 complex products on canonical [3][3][re,im] arrays.
__device__ __forceinline__ void mm(const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double ar = A[6 * i + 2 * k], ai = A[6 * i + 2 * k + 1];
        const double br = B[6 * k + 2 * j], bi = B[6 * k + 2 * j + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      C[6 * i + 2 * j] = re;
      C[6 * i + 2 * j + 1] = im;
    }
}
__device__ __forceinline__ void mmd(const double* A, const double* B, double* C) {  // C = A B^dagger
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double ar = A[6 * i + 2 * k], ai = A[6 * i + 2 * k + 1];
        const double br = B[6 * j + 2 * k], bi = -B[6 * j + 2 * k + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      C[6 * i + 2 * j] = re;
      C[6 * i + 2 * j + 1] = im;
    }
}

// One thread per (cb, parity, mu): the 8 reals of U[lex][mu] in every precision
// of the handle.  16-bit: the phases are stored divided by pi, so all 8 values
// lie in [-1, 1] and use the link encoding of the 12-real format.
__global__ void gauge_encode8_kernel(Lat m, const double* __restrict__ U, int64_t stride, char* f64, char* f32,
                                     char* i16, char* h16) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const int par = blockIdx.y >> 2, mu = blockIdx.y & 3;
  if (cb >= m.Vh) return;
  int t;
  const int64_t lex = lex_cb(m, cb, par, &t);
  const double* u = U + (lex * 4 + mu) * 18;
  double v[8] = {u[2], u[3], u[4], u[5], u[6], u[7], atan2(u[1], u[0]), atan2(u[13], u[12])};
  const int64_t chunk = (int64_t)(par * 4 + mu);
  if (f64) {
    for (int k = 0; k < 4; ++k)
      reinterpret_cast<double2*>(f64 + ((chunk * 4 + k) * stride) * 16)[cb] = make_double2(v[2 * k], v[2 * k + 1]);
  }
  if (f32) {
    for (int k = 0; k < 2; ++k)
      reinterpret_cast<float4*>(f32 + ((chunk * 2 + k) * stride) * 16)[cb] =
          make_float4((float)v[4 * k], (float)v[4 * k + 1], (float)v[4 * k + 2], (float)v[4 * k + 3]);
  }
  double w[8];
  for (int k = 0; k < 8; ++k) w[k] = (k < 6) ? v[k] : v[k] * (1.0 / M_PI);
  if (i16) {
    uint32_t q[4];
    for (int j = 0; j < 4; ++j) {
      const float a = fminf(fmaxf(rintf((float)w[2 * j] * 32767.0f), -32767.0f), 32767.0f);
      const float b = fminf(fmaxf(rintf((float)w[2 * j + 1] * 32767.0f), -32767.0f), 32767.0f);
      q[j] = (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
    }
    reinterpret_cast<uint4*>(i16 + (chunk * stride) * 16)[cb] = make_uint4(q[0], q[1], q[2], q[3]);
  }
  if (h16) {
    uint32_t q[4];
    for (int j = 0; j < 4; ++j)
      q[j] = (uint32_t)f_to_h16(pin_f32((float)w[2 * j])) | ((uint32_t)f_to_h16(pin_f32((float)w[2 * j + 1])) << 16);
    reinterpret_cast<uint4*>(h16 + (chunk * stride) * 16)[cb] = make_uint4(q[0], q[1], q[2], q[3]);
  }
}

// Largest |U_t(x) - 1| (max norm) over the temporal links of t < Lt - 1, as the
// bits of a non-negative double (their order is that of the values).
__global__ void temporal_check_kernel(Lat m, const double* __restrict__ U, unsigned long long* dev) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m.V) return;
  const int64_t V3 = (int64_t)m.L[0] * m.L[1] * m.L[2];
  if (i / V3 == m.L[3] - 1) return;
  const double* u = U + (i * 4 + 3) * 18;
  double d = 0.0;
  for (int k = 0; k < 18; ++k) {
    const double id = (k == 0 || k == 8 || k == 16) ? 1.0 : 0.0;
    d = fmax(d, fabs(u[k] - id));
  }
  if (!(d <= 1e300)) d = 1e300;  // NaN or Inf counts as far from 1
  atomicMax(dev, (unsigned long long)__double_as_longlong(d));
}

// g along each time line: one thread per spatial site.
__global__ void temporal_g_kernel(Lat m, const double* __restrict__ U, double* __restrict__ g) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t V3 = (int64_t)m.L[0] * m.L[1] * m.L[2];
  if (s >= V3) return;
  double cur[18], nxt[18];
  for (int k = 0; k < 18; ++k) cur[k] = (k == 0 || k == 8 || k == 16) ? 1.0 : 0.0;
  for (int t = 0; t < m.L[3]; ++t) {
    const int64_t lex = s + V3 * t;
    for (int k = 0; k < 18; ++k) g[lex * 18 + k] = cur[k];
    if (t + 1 < m.L[3]) {
      mm(cur, U + (lex * 4 + 3) * 18, nxt);
      for (int k = 0; k < 18; ++k) cur[k] = nxt[k];
    }
  }
}

// U'_mu(x) = g(x) U_mu(x) g(x + mu)^dagger: one thread per (site, mu).
__global__ void temporal_links_kernel(Lat m, const double* __restrict__ U, const double* __restrict__ g,
                                      double* __restrict__ Uo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m.V * 4) return;
  const int64_t lex = i >> 2;
  const int mu = (int)(i & 3);
  int64_t rest = lex;
  int x[4];
  for (int k = 0; k < 4; ++k) {
    x[k] = (int)(rest % m.L[k]);
    rest /= m.L[k];
  }
  x[mu] = (x[mu] + 1 == m.L[mu]) ? 0 : x[mu] + 1;
  const int64_t nb = x[0] + (int64_t)m.L[0] * (x[1] + (int64_t)m.L[1] * (x[2] + (int64_t)m.L[2] * x[3]));
  double tmp[18];
  mm(g + lex * 18, U + i * 18, tmp);
  mmd(tmp, g + nb * 18, Uo + i * 18);
}

// psi'(x) = g(x) psi(x) or g(x)^dagger psi(x): one thread per (rhs, site).
__global__ void rotate_kernel(Lat m, const double* __restrict__ g, const double* __restrict__ in,
                              double* __restrict__ out, int nrhs, int adjoint) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m.V * nrhs) return;
  const int64_t lex = i % m.V;
  const double* G = g + lex * 18;
  const double* src = in + i * 24;
  double res[24];
  for (int s = 0; s < 4; ++s)
    for (int a = 0; a < 3; ++a) {
      double re = 0.0, im = 0.0;
      for (int b = 0; b < 3; ++b) {
        const double gr = adjoint ? G[6 * b + 2 * a] : G[6 * a + 2 * b];
        const double gi = adjoint ? -G[6 * b + 2 * a + 1] : G[6 * a + 2 * b + 1];
        const double pr = src[6 * s + 2 * b], pi = src[6 * s + 2 * b + 1];
        re += gr * pr - gi * pi;
        im += gr * pi + gi * pr;
      }
      res[6 * s + 2 * a] = re;
      res[6 * s + 2 * a + 1] = im;
    }
  for (int k = 0; k < 24; ++k) out[i * 24 + k] = res[k];
}

unsigned grid1(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_gauge_encode8(const wd_gauge* g, const double* U, hipStream_t s) {
  const Lat m = lat_of(g->geom);
  dim3 grid(grid1(m.Vh, 256), 8);
  gauge_encode8_kernel<<<grid, 256, 0, s>>>(m, U, g->geom.stride, static_cast<char*>(g->link[WD_FP64]),
                                            static_cast<char*>(g->link[WD_FP32]),
                                            static_cast<char*>(g->link[WD_HALF_I16]),
                                            static_cast<char*>(g->link[WD_HALF_F16]));
  return hipGetLastError();
}

hipError_t launch_temporal_check(const Geom& geo, const double* U, unsigned long long* dev, hipStream_t s) {
  const Lat m = lat_of(geo);
  temporal_check_kernel<<<grid1(m.V, 256), 256, 0, s>>>(m, U, dev);
  return hipGetLastError();
}

hipError_t launch_gauge_fix_temporal(const Geom& geo, const double* U, double* Uo, double* g, hipStream_t s) {
  const Lat m = lat_of(geo);
  const int64_t V3 = (int64_t)m.L[0] * m.L[1] * m.L[2];
  temporal_g_kernel<<<grid1(V3, 128), 128, 0, s>>>(m, U, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  temporal_links_kernel<<<grid1(m.V * 4, 128), 128, 0, s>>>(m, U, g, Uo);
  return hipGetLastError();
}

hipError_t launch_gauge_rotate(const Geom& geo, const double* g, const double* in, double* out, int nrhs,
                               int adjoint, hipStream_t s) {
  const Lat m = lat_of(geo);
  rotate_kernel<<<grid1(m.V * nrhs, 128), 128, 0, s>>>(m, g, in, out, nrhs, adjoint);
  return hipGetLastError();
}

}  // namespace wd
