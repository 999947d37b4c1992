// Wilson-Dirac hopping term on one parity (Section 3, Eq. 1), for the
// storage formats FP64, FP32, int16 + norm and binary16 + norm.
//
// One thread computes one output site of parity p for one right-hand side:
// for each direction mu it gathers the two neighbours of the opposite parity,
// projects each onto its rank-2 spin subspace (6 complex numbers), multiplies
// by the 12-real link rebuilt to 3x3 (U forward, U^dagger backward), expands
// the result back to 4 spins and accumulates.  The t boundary sign is applied
// to the hop, never folded into the stored link.
//
// Spin projection in the DeGrand-Rossi basis (Appendix B): every gamma_mu is
// off-diagonal in 2x2 blocks, gamma_mu = [[0, A_mu], [A_mu^dag, 0]], so
//   (1 + s gamma_mu) psi = [ h ; s A_mu^dag h ],  h = psi_up + s A_mu psi_down,
// with s = -1 on the forward hop and s = +1 on the backward hop of D (the
// adjoint swaps them).  Each A_mu has one entry per row, a power of i:
//   A_x = [[0, i], [i, 0]],  A_y = [[0, -1], [1, 0]],
//   A_z = [[i, 0], [0, -i]], A_t = [[1, 0], [0, 1]].
#include "wd_device.h"
#include "wd_reduce.h"

namespace wd {

// Row k of A_mu has its entry in column PERM_k with value i^PH_k.
template <int MU>
struct Gamma;
template <> struct Gamma<0> { static constexpr int P0 = 1, P1 = 0, PH0 = 1, PH1 = 1; };
template <> struct Gamma<1> { static constexpr int P0 = 1, P1 = 0, PH0 = 2, PH1 = 0; };
template <> struct Gamma<2> { static constexpr int P0 = 0, P1 = 1, PH0 = 1, PH1 = 3; };
template <> struct Gamma<3> { static constexpr int P0 = 0, P1 = 1, PH0 = 0, PH1 = 0; };

struct GeomView {
  int L[4];
  int Lxh;
  int Vh;
  int tap;
  int64_t stride;  // chunk stride of every field and of the links
};

__device__ __forceinline__ int cb_index(const GeomView& g, int x, int y, int z, int t) {
  return (x >> 1) + g.Lxh * (y + g.L[1] * (z + g.L[2] * t));
}

// Accumulate one hop: acc += eta * (1 + s gamma_mu) (W psi), W = U or U^dagger.
template <int MU, int S, bool DAG_LINK, typename R>
__device__ __forceinline__ void hop(Spinor<R>& acc, const Spinor<R>& psi, const Link<R>& U, bool flip) {
  using G = Gamma<MU>;
  constexpr int sh = (S < 0) ? 2 : 0;  // multiplying by s = -1 is a factor i^2
  cx<R> h[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = psi.v[0][c] + iph<G::PH0 + sh>(psi.v[2 + G::P0][c]);
    h[1][c] = psi.v[1][c] + iph<G::PH1 + sh>(psi.v[2 + G::P1][c]);
  }
  cx<R> w[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> s;
      if constexpr (!DAG_LINK) {
        s = U.u[a][0] * h[k][0];
        s = s + U.u[a][1] * h[k][1];
        s = s + U.u[a][2] * h[k][2];
      } else {
        s = cmulc(U.u[0][a], h[k][0]);
        s = s + cmulc(U.u[1][a], h[k][1]);
        s = s + cmulc(U.u[2][a], h[k][2]);
      }
      w[k][a] = flip ? cx<R>{-s.re, -s.im} : s;
    }
  }
  // lower spin P_k of the result = s * conj(A[k][P_k]) * w_k = i^(sh - PH_k) w_k
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc.v[0][a] = acc.v[0][a] + w[0][a];
    acc.v[1][a] = acc.v[1][a] + w[1][a];
    acc.v[2 + G::P0][a] = acc.v[2 + G::P0][a] + iph<sh - G::PH0 + 4>(w[0][a]);
    acc.v[2 + G::P1][a] = acc.v[2 + G::P1][a] + iph<sh - G::PH1 + 4>(w[1][a]);
  }
}

template <class S, int MU, bool DAGGER>
__device__ __forceinline__ void hop_pair(Spinor<typename S::real>& acc, const GeomView& g,
                                         const char* links, int64_t stride, const FieldView& in,
                                         int r, int p, int cb, const int (&X)[4]) {
  using R = typename S::real;
  // forward: (1 - gamma_mu) U_x^mu psi(x + mu); adjoint: (1 + gamma_mu)
  {
    int Y[4] = {X[0], X[1], X[2], X[3]};
    Y[MU] = (X[MU] + 1 == g.L[MU]) ? 0 : X[MU] + 1;
    const bool flip = (MU == 3) && g.tap && (X[3] == g.L[3] - 1);
    const int nb = cb_index(g, Y[0], Y[1], Y[2], Y[3]);
    Spinor<R> psi;
    load_spinor<S>(in, r, nb, psi);
    Link<R> U;
    load_link<S>(links, stride, p, MU, cb, U);
    hop<MU, DAGGER ? +1 : -1, false>(acc, psi, U, flip);
  }
  // backward: (1 + gamma_mu) U_{x-mu}^mu^dagger psi(x - mu); adjoint: (1 - gamma_mu)
  {
    int Y[4] = {X[0], X[1], X[2], X[3]};
    Y[MU] = (X[MU] == 0) ? g.L[MU] - 1 : X[MU] - 1;
    const bool flip = (MU == 3) && g.tap && (X[3] == 0);
    const int nb = cb_index(g, Y[0], Y[1], Y[2], Y[3]);
    Spinor<R> psi;
    load_spinor<S>(in, r, nb, psi);
    Link<R> U;
    load_link<S>(links, stride, 1 - p, MU, nb, U);
    hop<MU, DAGGER ? -1 : +1, true>(acc, psi, U, flip);
  }
}

// out = D in, or out = x + a * D in (XPAY), optionally followed by per-block
// FP64 partial dot products of the result (DOT):
//   DOT_YO: <y, out>                 (complex; BiCGstab <r~, v>)
//   DOT_OX: <out, x>, |out|^2        (BiCGstab <t, s>, <t, t> with x = s)
//   DOT_OO: |out|^2                  (CG |M p|^2)
// Right-hand sides whose active flag is 0 are skipped (the block returns).
template <class S, bool DAGGER, bool XPAY, int DOT>
__global__ void __launch_bounds__(kBlock) dslash_kernel(GeomView g, const char* __restrict__ links,
                                                       FieldView out, FieldView in, FieldView xs,
                                                       FieldView ys, typename S::real a, int p,
                                                       const int* __restrict__ active,
                                                       double* __restrict__ partials) {
  using R = typename S::real;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = cb < g.Vh;
  Spinor<R> acc;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.v[s][c] = {R(0), R(0)};
  Spinor<R> x;
  if (valid) {
    // coordinates of the output site (cb, parity p)
    int rest = cb / g.Lxh;
    const int xh = cb - rest * g.Lxh;
    int X[4];
    X[1] = rest % g.L[1];
    rest /= g.L[1];
    X[2] = rest % g.L[2];
    X[3] = rest / g.L[2];
    X[0] = 2 * xh + ((p + X[1] + X[2] + X[3]) & 1);

    hop_pair<S, 0, DAGGER>(acc, g, links, g.stride, in, r, p, cb, X);
    hop_pair<S, 1, DAGGER>(acc, g, links, g.stride, in, r, p, cb, X);
    hop_pair<S, 2, DAGGER>(acc, g, links, g.stride, in, r, p, cb, X);
    hop_pair<S, 3, DAGGER>(acc, g, links, g.stride, in, r, p, cb, X);

    if constexpr (XPAY) {
      load_spinor<S>(xs, r, cb, x);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.v[s][c] = x.v[s][c] + a * acc.v[s][c];
    }
    store_spinor<S>(out, r, cb, acc);
  }
  if constexpr (DOT != DOT_NONE) {
    const int nb = gridDim.x;
    double* part = partials + ((int64_t)r * nb + blockIdx.x) * kMaxDot;
    if constexpr (DOT == DOT_YO) {
      double d[2] = {0.0, 0.0};
      if (valid) {
        Spinor<R> y;
        load_spinor<S>(ys, r, cb, y);
        R re = 0, im = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            cx<R> t = cmulc(y.v[s][c], acc.v[s][c]);
            re += t.re;
            im += t.im;
          }
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
            cx<R> t = cmulc(acc.v[s][c], x.v[s][c]);
            re += t.re;
            im += t.im;
            nn += acc.v[s][c].re * acc.v[s][c].re + acc.v[s][c].im * acc.v[s][c].im;
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
          for (int c = 0; c < 3; ++c)
            nn += acc.v[s][c].re * acc.v[s][c].re + acc.v[s][c].im * acc.v[s][c].im;
        d[0] = nn;
      }
      block_sum_store<1>(d, part);
    }
  }
}

static GeomView view(const Geom& g) {
  GeomView v;
  for (int m = 0; m < 4; ++m) v.L[m] = g.L[m];
  v.Lxh = g.Lxh;
  v.Vh = g.Vh;
  v.tap = g.tap;
  v.stride = g.stride;
  return v;
}

static FieldView fview(const Field& f) { return FieldView{f.ptr, f.stride, f.nrhs}; }
static FieldView fview(const Field* f) { return f ? fview(*f) : FieldView{nullptr, 0, 0}; }

template <class S, bool DAGGER, bool XPAY>
static void launch_dot(int dot, dim3 grid, hipStream_t s, const GeomView& g, const char* links,
                       FieldView fo, FieldView fi, FieldView fx, FieldView fy, typename S::real a,
                       int p, const int* active, double* partials) {
  switch (dot) {
    case DOT_YO:
      dslash_kernel<S, DAGGER, XPAY, DOT_YO><<<grid, kBlock, 0, s>>>(g, links, fo, fi, fx, fy, a, p, active, partials);
      break;
    case DOT_OX:
      dslash_kernel<S, DAGGER, XPAY, DOT_OX><<<grid, kBlock, 0, s>>>(g, links, fo, fi, fx, fy, a, p, active, partials);
      break;
    case DOT_OO:
      dslash_kernel<S, DAGGER, XPAY, DOT_OO><<<grid, kBlock, 0, s>>>(g, links, fo, fi, fx, fy, a, p, active, partials);
      break;
    default:
      dslash_kernel<S, DAGGER, XPAY, DOT_NONE><<<grid, kBlock, 0, s>>>(g, links, fo, fi, fx, fy, a, p, active, partials);
  }
}

template <class S>
static hipError_t launch_typed(const wd_gauge* gg, const DslashArgs& d, hipStream_t s) {
  const GeomView g = view(gg->geom);
  const char* links = static_cast<const char*>(gg->link[S::prec]);
  dim3 grid((g.Vh + kBlock - 1) / kBlock, d.out.nrhs);
  FieldView fo = fview(d.out), fi = fview(d.in), fx = fview(d.xpay), fy = fview(d.y);
  using R = typename S::real;
  const R ar = static_cast<R>(d.a);
  const int dot = d.xpay ? d.dot : DOT_NONE;
  if (d.dagger) {
    if (d.xpay) launch_dot<S, true, true>(dot, grid, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.active, d.partials);
    else launch_dot<S, true, false>(DOT_NONE, grid, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.active, d.partials);
  } else {
    if (d.xpay) launch_dot<S, false, true>(dot, grid, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.active, d.partials);
    else launch_dot<S, false, false>(DOT_NONE, grid, s, g, links, fo, fi, fx, fy, ar, d.out_parity, d.active, d.partials);
  }
  return hipGetLastError();
}

hipError_t launch_dslash_ex(const wd_gauge* g, wd_prec prec, const DslashArgs& d, hipStream_t s) {
  switch (prec) {
    case WD_FP64: return launch_typed<SF64>(g, d, s);
    case WD_FP32: return launch_typed<SF32>(g, d, s);
    case WD_HALF_I16: return launch_typed<SI16>(g, d, s);
    case WD_HALF_F16: return launch_typed<SF16>(g, d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dslash(const wd_gauge* g, wd_prec prec, Field out, Field in, int out_parity,
                         int dagger, const Field* xpay_src, double a, hipStream_t s) {
  DslashArgs d;
  d.out = out;
  d.in = in;
  d.out_parity = out_parity;
  d.dagger = dagger;
  d.xpay = xpay_src;
  d.a = a;
  return launch_dslash_ex(g, prec, d, s);
}

int dslash_blocks(const Geom& g) { return (g.Vh + kBlock - 1) / kBlock; }

}  // namespace wd
