// C ABI of libwdslash.so: argument validation, gauge handles, field
// encode/decode and the operator entry points.  Every check runs before any
// launch; no exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "wd_internal.h"

namespace wd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

wd_status fail(wd_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Chunk arrays are padded to a multiple of 64 sites (one wavefront) so that
// every chunk array starts 1 KiB-aligned relative to the field base.
int64_t field_stride(int64_t Vh) { return (Vh + 63) / 64 * 64; }

Geom make_geom(const wd_lattice& lat) {
  Geom g;
  int64_t V = 1;
  for (int m = 0; m < 4; ++m) {
    g.L[m] = lat.dims[m];
    V *= lat.dims[m];
  }
  g.Lxh = lat.dims[0] / 2;
  g.Vh = static_cast<int>(V / 2);
  g.tap = lat.t_antiperiodic ? 1 : 0;
  g.stride = field_stride(g.Vh);
  return g;
}

size_t spinor_field_bytes(const Geom& g, wd_prec p, int nrhs) {
  size_t b = static_cast<size_t>(nrhs) * spinor_chunks(p) * g.stride * 16;
  if (is_half(p)) b += static_cast<size_t>(nrhs) * g.stride * 4;
  return b;
}

// Largest Vh whose FP64 parity field (stride * 192 bytes, stride a multiple of
// 64 sites) fits a 32-bit buffer descriptor.
static constexpr int64_t kMaxVh = ((int64_t)UINT32_MAX / 192) / 64 * 64;

static bool prec_ok(wd_prec p) { return p >= WD_FP64 && p <= WD_HALF_F16; }

// Lattice check: dims even, >= 2, volume within int32 checkerboard indexing.
static wd_status check_lattice(const wd_lattice* lat) {
  if (!lat) return fail(WD_EINVAL, "lattice is NULL");
  int64_t V = 1;
  for (int m = 0; m < 4; ++m) {
    const int L = lat->dims[m];
    if (L < 2 || (L & 1))
      return fail(WD_EINVAL, "lattice dims must be even and >= 2 (dim " + std::to_string(m) +
                                 " = " + std::to_string(L) + ")");
    V *= L;
  }
  // The kernels address one right-hand side of a field, and one (parity, mu)
  // block of links, through a buffer descriptor whose size is 32-bit: the
  // largest such range, an FP64 spinor (12 chunks of 16 bytes per site), must
  // stay below 4 GiB.  A larger lattice would make loads read zeros.
  if (field_stride(V / 2) * 192 > (int64_t)UINT32_MAX)
    return fail(WD_EINVAL, "lattice too large: Vh = " + std::to_string(V / 2) + " > " +
                               std::to_string(kMaxVh) + " (one FP64 parity field must stay below 4 GiB)");
  if (lat->t_antiperiodic != 0 && lat->t_antiperiodic != 1)
    return fail(WD_EINVAL, "t_antiperiodic must be 0 or 1");
  return WD_OK;
}

static wd_status check_ptr(const void* p, const char* what) {
  if (!p) return fail(WD_EINVAL, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) % 256)
    return fail(WD_EINVAL, std::string(what) + " is not 256-byte aligned");
  return WD_OK;
}

static wd_status check_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 65535) return fail(WD_EINVAL, "nrhs must be in [1, 65535]");
  return WD_OK;
}

static wd_status check_gauge(const wd_gauge* g, wd_prec prec) {
  if (!g) return fail(WD_EINVAL, "gauge handle is NULL");
  if (!prec_ok(prec)) return fail(WD_EINVAL, "unknown precision");
  if (!(g->mask & WD_PREC_MASK(prec)) || !g->link[prec])
    return fail(WD_EINVAL, "gauge handle does not hold the requested precision");
  return WD_OK;
}

static wd_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return WD_OK;
  return fail(WD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

static Field field_of(const Geom& g, void* p, int nrhs) {
  return Field{static_cast<char*>(p), g.stride, nrhs};
}

}  // namespace wd

using namespace wd;

extern "C" {

const char* wd_last_error(void) { return g_last_error.c_str(); }

const char* wd_version(void) { return "wdslash 0.1 (gfx950)"; }

size_t wd_gauge_bytes_ex(const wd_lattice* lat, uint32_t prec_mask, int32_t recon, uint32_t flags) {
  if (check_lattice(lat) != WD_OK) return 0;
  if (prec_mask == 0 || (prec_mask & ~0xfu)) return 0;
  if ((recon != 12 && recon != 8) || (flags & ~WD_GAUGE_TEMPORAL)) return 0;
  const Geom g = make_geom(*lat);
  size_t b = 0;
  for (int p = 0; p < 4; ++p)
    if (prec_mask & WD_PREC_MASK(p)) b += static_cast<size_t>(8) * g.stride * link_bytes(p, recon);
  if (flags & WD_GAUGE_TEMPORAL) b += 256;  // the temporal-gauge check's result
  return b;
}

size_t wd_gauge_bytes(const wd_lattice* lat, uint32_t prec_mask) {
  return wd_gauge_bytes_ex(lat, prec_mask, 12, 0);
}

wd_status wd_gauge_create_ex(const wd_lattice* lat, const double* U_dev, uint32_t prec_mask, int32_t recon,
                             uint32_t flags, void* dev_buf, size_t bytes, void* stream, wd_gauge** out) {
  g_last_error.clear();
  if (!out) return fail(WD_EINVAL, "out is NULL");
  *out = nullptr;
  wd_status st = check_lattice(lat);
  if (st) return st;
  if (prec_mask == 0 || (prec_mask & ~0xfu)) return fail(WD_EINVAL, "invalid precision mask");
  if (recon != 12 && recon != 8) return fail(WD_EINVAL, "recon must be 12 or 8");
  if (flags & ~WD_GAUGE_TEMPORAL) return fail(WD_EINVAL, "unknown gauge flags");
  if ((st = check_ptr(U_dev, "U_dev"))) return st;
  if ((st = check_ptr(dev_buf, "dev_buf"))) return st;
  const size_t need = wd_gauge_bytes_ex(lat, prec_mask, recon, flags);
  if (bytes < need)
    return fail(WD_EINVAL, "dev_buf too small: " + std::to_string(bytes) + " < " + std::to_string(need));
  wd_gauge* g = new (std::nothrow) wd_gauge;
  if (!g) return fail(WD_ENOMEM, "host allocation of the gauge handle failed");
  g->lat = *lat;
  g->geom = make_geom(*lat);
  g->mask = prec_mask;
  g->recon = recon;
  g->tgauge = (flags & WD_GAUGE_TEMPORAL) ? 1 : 0;
  char* p = static_cast<char*>(dev_buf);
  for (int q = 0; q < 4; ++q) {
    g->link[q] = nullptr;
    if (prec_mask & WD_PREC_MASK(q)) {
      g->link[q] = p;
      p += static_cast<size_t>(8) * g->geom.stride * link_bytes(q, recon);
    }
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (g->tgauge) {
    // the largest distance of a checked temporal link from 1, as double bits
    auto* dev = reinterpret_cast<unsigned long long*>(p);
    unsigned long long host = 0;
    hipError_t e = hipMemsetAsync(dev, 0, sizeof(host), s);
    if (e == hipSuccess) e = launch_temporal_check(g->geom, U_dev, dev, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&host, dev, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      delete g;
      return hip_status(e, "temporal-gauge check");
    }
    double dev_max;
    std::memcpy(&dev_max, &host, sizeof(dev_max));
    if (!(dev_max <= 1e-10)) {
      delete g;
      return fail(WD_EINVAL, "links are not in temporal gauge (max |U_t - 1| = " + std::to_string(dev_max) +
                                 " off the last time slice)");
    }
  }
  st = hip_status(recon == 8 ? launch_gauge_encode8(g, U_dev, s) : launch_gauge_encode(g, U_dev, s),
                  "gauge encode");
  if (st) {
    delete g;
    return st;
  }
  *out = g;
  return WD_OK;
}

wd_status wd_gauge_create(const wd_lattice* lat, const double* U_dev, uint32_t prec_mask, void* dev_buf,
                          size_t bytes, void* stream, wd_gauge** out) {
  return wd_gauge_create_ex(lat, U_dev, prec_mask, 12, 0, dev_buf, bytes, stream, out);
}

wd_status wd_gauge_fix_temporal(const wd_lattice* lat, const double* U_in, double* U_out, double* g_out,
                                void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if ((st = check_ptr(U_in, "U_in")) || (st = check_ptr(U_out, "U_out")) || (st = check_ptr(g_out, "g_out")))
    return st;
  return hip_status(launch_gauge_fix_temporal(make_geom(*lat), U_in, U_out, g_out, static_cast<hipStream_t>(stream)),
                    "temporal gauge fixing");
}

wd_status wd_gauge_rotate_spinor(const wd_lattice* lat, const double* g, double* out, const double* in,
                                 int32_t nrhs, int32_t adjoint, void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(g, "g")) || (st = check_ptr(out, "out")) ||
      (st = check_ptr(in, "in")))
    return st;
  return hip_status(launch_gauge_rotate(make_geom(*lat), g, in, out, nrhs, adjoint ? 1 : 0,
                                        static_cast<hipStream_t>(stream)),
                    "spinor rotation");
}

void wd_gauge_destroy(wd_gauge* g) { delete g; }

size_t wd_spinor_bytes(const wd_lattice* lat, wd_prec prec, int32_t nrhs) {
  if (check_lattice(lat) != WD_OK || !prec_ok(prec) || check_nrhs(nrhs) != WD_OK) return 0;
  return spinor_field_bytes(make_geom(*lat), prec, nrhs);
}

wd_status wd_spinor_encode_basis(const wd_lattice* lat, wd_prec prec, int32_t nrhs, int32_t basis,
                                 void* field, const double* canon, void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if (!prec_ok(prec)) return fail(WD_EINVAL, "unknown precision");
  if (basis != WD_BASIS_DEGRAND_ROSSI && basis != WD_BASIS_UKQCD) return fail(WD_EINVAL, "unknown spin basis");
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(field, "field")) || (st = check_ptr(canon, "canon")))
    return st;
  const Geom g = make_geom(*lat);
  return hip_status(launch_spinor_encode(g, prec, field_of(g, field, nrhs), canon,
                                         static_cast<hipStream_t>(stream), basis),
                    "spinor encode");
}

wd_status wd_spinor_decode_basis(const wd_lattice* lat, wd_prec prec, int32_t nrhs, int32_t basis,
                                 double* canon, const void* field, void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if (!prec_ok(prec)) return fail(WD_EINVAL, "unknown precision");
  if (basis != WD_BASIS_DEGRAND_ROSSI && basis != WD_BASIS_UKQCD) return fail(WD_EINVAL, "unknown spin basis");
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(field, "field")) || (st = check_ptr(canon, "canon")))
    return st;
  const Geom g = make_geom(*lat);
  return hip_status(launch_spinor_decode(g, prec, canon, field_of(g, const_cast<void*>(field), nrhs),
                                         static_cast<hipStream_t>(stream), basis),
                    "spinor decode");
}

wd_status wd_spinor_encode(const wd_lattice* lat, wd_prec prec, int32_t nrhs, void* field,
                           const double* canon, void* stream) {
  return wd_spinor_encode_basis(lat, prec, nrhs, WD_BASIS_DEGRAND_ROSSI, field, canon, stream);
}

wd_status wd_spinor_decode(const wd_lattice* lat, wd_prec prec, int32_t nrhs, double* canon,
                           const void* field, void* stream) {
  return wd_spinor_decode_basis(lat, prec, nrhs, WD_BASIS_DEGRAND_ROSSI, canon, field, stream);
}

wd_status wd_spinor_encode_full(const wd_lattice* lat, wd_prec prec, int32_t nrhs, int32_t parity,
                                void* field, const double* canon_full, void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if (!prec_ok(prec)) return fail(WD_EINVAL, "unknown precision");
  if (parity != 0 && parity != 1) return fail(WD_EINVAL, "parity must be 0 or 1");
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(field, "field")) ||
      (st = check_ptr(canon_full, "canon_full")))
    return st;
  const Geom g = make_geom(*lat);
  return hip_status(launch_spinor_encode_map(g, prec, field_of(g, field, nrhs), canon_full, parity,
                                             static_cast<hipStream_t>(stream)),
                    "spinor encode (full lattice)");
}

wd_status wd_spinor_decode_full(const wd_lattice* lat, wd_prec prec, int32_t nrhs, int32_t parity,
                                double* canon_full, const void* field, void* stream) {
  g_last_error.clear();
  wd_status st = check_lattice(lat);
  if (st) return st;
  if (!prec_ok(prec)) return fail(WD_EINVAL, "unknown precision");
  if (parity != 0 && parity != 1) return fail(WD_EINVAL, "parity must be 0 or 1");
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(field, "field")) ||
      (st = check_ptr(canon_full, "canon_full")))
    return st;
  const Geom g = make_geom(*lat);
  return hip_status(launch_spinor_decode_map(g, prec, canon_full,
                                             field_of(g, const_cast<void*>(field), nrhs), parity,
                                             static_cast<hipStream_t>(stream)),
                    "spinor decode (full lattice)");
}

wd_status wd_dslash_field_basis(const wd_gauge* g, void* out, const void* in, int32_t out_parity,
                                int32_t dagger, wd_prec prec, int32_t nrhs, int32_t basis, void* stream) {
  g_last_error.clear();
  wd_status st = check_gauge(g, prec);
  if (st) return st;
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(out, "out")) || (st = check_ptr(in, "in"))) return st;
  if (out_parity != 0 && out_parity != 1) return fail(WD_EINVAL, "out_parity must be 0 or 1");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  if (basis != WD_BASIS_DEGRAND_ROSSI && basis != WD_BASIS_UKQCD) return fail(WD_EINVAL, "unknown spin basis");
  if (out == in) return fail(WD_EINVAL, "out and in must not alias");
  const Geom& geo = g->geom;
  return hip_status(launch_dslash(g, prec, field_of(geo, out, nrhs), field_of(geo, const_cast<void*>(in), nrhs),
                                  out_parity, dagger, nullptr, 0.0, static_cast<hipStream_t>(stream), basis),
                    "wd_dslash_field");
}

wd_status wd_dslash_field(const wd_gauge* g, void* out, const void* in, int32_t out_parity, int32_t dagger,
                          wd_prec prec, int32_t nrhs, void* stream) {
  return wd_dslash_field_basis(g, out, in, out_parity, dagger, prec, nrhs, WD_BASIS_DEGRAND_ROSSI, stream);
}

wd_status wd_mat_pc_field(const wd_gauge* g, double kappa, void* out, const void* in, void* tmp_odd,
                          int32_t dagger, wd_prec prec, int32_t nrhs, void* stream) {
  g_last_error.clear();
  wd_status st = check_gauge(g, prec);
  if (st) return st;
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(out, "out")) || (st = check_ptr(in, "in")) ||
      (st = check_ptr(tmp_odd, "tmp_odd")))
    return st;
  if (!std::isfinite(kappa) || kappa <= 0) return fail(WD_EINVAL, "kappa must be finite and > 0");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  if (out == in || tmp_odd == in || tmp_odd == out) return fail(WD_EINVAL, "fields must not alias");
  const Geom& geo = g->geom;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Field fo = field_of(geo, out, nrhs), fi = field_of(geo, const_cast<void*>(in), nrhs);
  Field ft = field_of(geo, tmp_odd, nrhs);
  hipError_t e = launch_dslash(g, prec, ft, fi, 1, dagger, nullptr, 0.0, s);
  if (e == hipSuccess) e = launch_dslash(g, prec, fo, ft, 0, dagger, &fi, -kappa * kappa, s);
  return hip_status(e, "wd_mat_pc_field");
}

wd_status wd_mdagm_field(const wd_gauge* g, double kappa, void* out, const void* in, void* tmp_odd,
                         void* tmp_even, wd_prec prec, int32_t nrhs, void* stream) {
  g_last_error.clear();
  wd_status st = check_gauge(g, prec);
  if (st) return st;
  if ((st = check_ptr(tmp_even, "tmp_even"))) return st;
  if (tmp_even == in || tmp_even == out || tmp_even == tmp_odd)
    return fail(WD_EINVAL, "fields must not alias");
  st = wd_mat_pc_field(g, kappa, tmp_even, in, tmp_odd, 0, prec, nrhs, stream);
  if (st) return st;
  return wd_mat_pc_field(g, kappa, out, tmp_even, tmp_odd, 1, prec, nrhs, stream);
}

// ---- operators on canonical FP64 parity spinors -------------------------------------
// The workspace holds four encoded parity fields of (prec, nrhs), each
// starting on a 256-byte boundary: the encoded input, the result and one odd
// and one even temporary.

size_t wd_operator_workspace_bytes(const wd_lattice* lat, wd_prec prec, int32_t nrhs) {
  if (check_lattice(lat) != WD_OK || !prec_ok(prec) || check_nrhs(nrhs) != WD_OK) return 0;
  return 4 * operator_field_slot(make_geom(*lat), prec, nrhs);
}

}  // extern "C"

namespace wd {

size_t operator_field_slot(const Geom& g, wd_prec prec, int nrhs) {
  return (spinor_field_bytes(g, prec, nrhs) + 255) / 256 * 256;
}

// Argument checks shared by the canonical operator entry points.
static wd_status check_canon_op(const wd_gauge* g, void* out, const void* in, wd_prec prec, int nrhs,
                                const void* ws, size_t ws_bytes, size_t* slot) {
  wd_status st = check_gauge(g, prec);
  if (st) return st;
  if ((st = check_nrhs(nrhs)) || (st = check_ptr(out, "out")) || (st = check_ptr(in, "in")) ||
      (st = check_ptr(ws, "workspace")))
    return st;
  *slot = operator_field_slot(g->geom, prec, nrhs);
  if (ws_bytes < 4 * *slot)
    return fail(WD_EINVAL, "workspace too small: " + std::to_string(ws_bytes) + " < " +
                               std::to_string(4 * *slot) + " (wd_operator_workspace_bytes)");
  return WD_OK;
}

// The canonical operators: encode `in`, apply the operator on encoded
// fields, decode into `out` (all on `s`).  op: 0 dslash, 1 M_hat (dagger
// selects the adjoint), 2 M_hat^dagger M_hat.  out may alias in: the input
// is encoded before anything is written to out.
hipError_t canon_operator(const wd_gauge* g, int op, double kappa, double* out, const double* in,
                          int out_parity, int dagger, wd_prec prec, int nrhs, char* ws, size_t slot,
                          hipStream_t s, bool no_tune) {
  const Geom& geo = g->geom;
  Field fin = field_of(geo, ws, nrhs), fout = field_of(geo, ws + slot, nrhs);
  Field fodd = field_of(geo, ws + 2 * slot, nrhs), feven = field_of(geo, ws + 3 * slot, nrhs);
  auto dslash = [&](Field o, Field i, int par, int dag, const Field* xpay, double a) {
    DslashArgs d;
    d.out = o;
    d.in = i;
    d.out_parity = par;
    d.dagger = dag;
    d.xpay = xpay;
    d.a = a;
    d.no_tune = no_tune ? 1 : 0;
    return launch_dslash_ex(g, prec, d, s);
  };
  hipError_t e = launch_spinor_encode(geo, prec, fin, in, s);
  if (e != hipSuccess) return e;
  if (op == 0) {
    e = dslash(fout, fin, out_parity, dagger, nullptr, 0.0);
  } else {
    const double a = -kappa * kappa;
    const int dag1 = op == 1 ? dagger : 0;
    e = dslash(fodd, fin, 1, dag1, nullptr, 0.0);
    if (e == hipSuccess) e = dslash(op == 1 ? fout : feven, fodd, 0, dag1, &fin, a);
    if (op == 2) {
      if (e == hipSuccess) e = dslash(fodd, feven, 1, 1, nullptr, 0.0);
      if (e == hipSuccess) e = dslash(fout, fodd, 0, 1, &feven, a);
    }
  }
  if (e != hipSuccess) return e;
  return launch_spinor_decode(geo, prec, out, fout, s);
}

}  // namespace wd

extern "C" {

wd_status wilson_dslash(const wd_gauge* g, double* out, const double* in, int32_t out_parity, int32_t dagger,
                        wd_prec prec, int32_t nrhs, void* workspace, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  size_t slot = 0;
  wd_status st = check_canon_op(g, out, in, prec, nrhs, workspace, ws_bytes, &slot);
  if (st) return st;
  if (out_parity != 0 && out_parity != 1) return fail(WD_EINVAL, "out_parity must be 0 or 1");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  return hip_status(canon_operator(g, 0, 0.0, out, in, out_parity, dagger, prec, nrhs,
                                   static_cast<char*>(workspace), slot, static_cast<hipStream_t>(stream)),
                    "wilson_dslash");
}

wd_status wilson_mat_pc(const wd_gauge* g, double kappa, double* out, const double* in, int32_t dagger,
                        wd_prec prec, int32_t nrhs, void* workspace, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  size_t slot = 0;
  wd_status st = check_canon_op(g, out, in, prec, nrhs, workspace, ws_bytes, &slot);
  if (st) return st;
  if (!std::isfinite(kappa) || kappa <= 0) return fail(WD_EINVAL, "kappa must be finite and > 0");
  if (dagger != 0 && dagger != 1) return fail(WD_EINVAL, "dagger must be 0 or 1");
  return hip_status(canon_operator(g, 1, kappa, out, in, 0, dagger, prec, nrhs, static_cast<char*>(workspace),
                                   slot, static_cast<hipStream_t>(stream)),
                    "wilson_mat_pc");
}

wd_status mdagm(const wd_gauge* g, double kappa, double* out, const double* in, wd_prec prec, int32_t nrhs,
                void* workspace, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  size_t slot = 0;
  wd_status st = check_canon_op(g, out, in, prec, nrhs, workspace, ws_bytes, &slot);
  if (st) return st;
  if (!std::isfinite(kappa) || kappa <= 0) return fail(WD_EINVAL, "kappa must be finite and > 0");
  return hip_status(canon_operator(g, 2, kappa, out, in, 0, 0, prec, nrhs, static_cast<char*>(workspace), slot,
                                   static_cast<hipStream_t>(stream)),
                    "mdagm");
}

}  // extern "C"
