/*
 * wd.h -- C ABI of the MI355X Wilson-Dirac library (libwdslash.so).
 *
 * The library applies the even-odd preconditioned Wilson-Dirac operator and
 * solves with it, following Clark, Babich, Barros, Brower and Rebbi, "Solving
 * Lattice QCD systems of equations using mixed precision solvers on GPUs"
 * (arXiv:0911.3191):
 *   - hopping term D of the Wilson-Dirac matrix (Section 3, Eq. 1), gamma
 *     matrices in the DeGrand-Rossi basis (Appendix B);
 *   - Schur complement on the even sites M_hat = 1 - kappa^2 D_eo D_oe with
 *     kappa = 1/(2(4+m)) (Section 3, Eq. 2);
 *   - 12-real SU(3) link storage, c = (a x b)^* (Appendix A.1);
 *   - FP64, FP32 and 16-bit storage with a per-site norm (Section 4.6);
 *   - BiCGstab on M_hat and CG on the normal equations (Section 5.1), with
 *     the reliable-update mixed-precision scheme (Section 5.3, Algorithm 2)
 *     and the defect-correction scheme (Section 5.2, Algorithm 1).
 *
 * Conventions
 *   Lattice dims (Lx, Ly, Lz, Lt), all even, each >= 2, with Vh = V/2 at most
 *   22,369,600 (one FP64 parity field of one right-hand side below 4 GiB, the
 *   range of the kernels' buffer descriptors).  Direction mu = 0..3
 *   is x, y, z, t (the paper's mu = 1..4).  Site index
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2 (0 = even);
 *   checkerboard index cb = lex / 2 within a parity.  Periodic in x, y, z;
 *   in t periodic or antiperiodic (t_antiperiodic = 1: every hop across the t
 *   boundary is multiplied by -1; the stored links are never changed).
 *   The library solves (1 - kappa D) x = b, i.e. the paper's M x = b with b
 *   divided by (4 + m).
 *
 * Canonical (caller-visible) layouts, FP64 on the device, complex = (re, im):
 *   gauge        double U[V][4][3][3][2]: U[lex][mu] is the link lex -> lex+mu,
 *                acting as (U psi)_a = sum_b U[a][b] psi_b.
 *   full spinor  double psi[nrhs][V][4][3][2] (spin, colour), DeGrand-Rossi.
 *   parity spinor double psi[nrhs][Vh][4][3][2], sites of one parity in cb order.
 *
 * Device field formats (opaque to the caller; sizes from wd_spinor_bytes):
 *   encoded spinor fields of one parity for nrhs right-hand sides, in one of
 *   the wd_prec storage formats.  Only the library reads or writes them.
 *
 * Memory and streams
 *   The caller allocates every device buffer (for example as PyTorch tensors)
 *   and passes raw device pointers; the library never frees caller memory and
 *   never allocates device memory in the operator or solver paths.  `stream`
 *   is a hipStream_t (NULL = default stream).  Device pointers must be
 *   256-byte aligned.
 *
 * Errors
 *   Every entry point validates its arguments before launching anything and
 *   returns a wd_status; no exception crosses the ABI.  wd_last_error() gives a
 *   thread-local message for the last failing call on the calling thread.
 *
 * Launch shapes (environment, read at run time)
 *   The first eager dslash launch of each (lattice, precision, RHS count, link
 *   format, spin basis, form) times candidate launch shapes on the caller's
 *   stream and keeps the fastest; launches under graph capture use a default
 *   shape.  Every shape gives the same bits.
 *   WD_TUNE=0             no tuning (default shapes)
 *   WD_TUNE_CACHE=<file>  keep the choices across processes (appended, one
 *                         line per key)
 *   WD_TUNE_VERBOSE=1     print every timed candidate to stderr
 *   WD_DSLASH_SHAPE=...   force one shape:
 *                         "nr,gslow,nsub[,link_nt[,out_nt[,wgs[,lds[,rloop[,block]]]]]]"
 *                         (RHS slots per thread, RHS-group order, y-sub-slabs,
 *                         cache hints, workgroups per CU cap, LDS staging,
 *                         binary16 RHS loop, workgroup size)
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wd_status;
#define WD_OK 0
#define WD_NOT_CONVERGED 1
#define WD_EINVAL (-1)
#define WD_ENOMEM (-2)
#define WD_EDEVICE (-3)
#define WD_EBREAKDOWN (-4)
#define WD_EUNSUPPORTED (-5)

/* Storage precision of fields (arithmetic is FP64 for WD_FP64, FP32 for the
 * others).  The 16-bit formats keep one binary32 norm per site (the largest
 * |real| among the site's 24 reals) and store each real relative to it:
 * WD_HALF_I16 as int16 fixed point q = rint(v * 32767/norm) (the paper's
 * format, Section 4.6), WD_HALF_F16 as IEEE binary16 v/norm.  16-bit links
 * carry no norm (their reals lie in [-1, 1]). */
typedef int32_t wd_prec;
#define WD_FP64 0
#define WD_FP32 1
#define WD_HALF_I16 2
#define WD_HALF_F16 3
#define WD_PREC_MASK(p) (1u << (p))

typedef struct {
  int32_t dims[4];        /* Lx, Ly, Lz, Lt */
  int32_t t_antiperiodic; /* 1: antiperiodic in t, 0: periodic */
} wd_lattice;

typedef struct wd_gauge wd_gauge;   /* resident gauge field (read-only once built) */
typedef struct wd_solver wd_solver; /* an in-flight solve (step API) */

/* Thread-local message for the last failing call ("" if none). */
const char *wd_last_error(void);

/* Library version string. */
const char *wd_version(void);

/* ---- gauge field ----------------------------------------------------------- */

/* Device bytes needed to hold the gauge field in every precision of
 * prec_mask (a bitwise OR of WD_PREC_MASK(p)), each stored as 12 reals per
 * link (rows a and b of Appendix A.1).  0 on invalid arguments. */
size_t wd_gauge_bytes(const wd_lattice *lat, uint32_t prec_mask);

/* Build a resident gauge field from the canonical FP64 links U_dev (device,
 * [V][4][3][3][2]).  The encoded copies are written into dev_buf (caller-owned,
 * >= wd_gauge_bytes bytes, kept alive until wd_gauge_destroy).  The handle
 * itself is host metadata.  Asynchronous on stream; U_dev may be released once
 * the stream has passed this point.  Links must be SU(3) to rounding (the third
 * row is rebuilt as (a x b)^*). */
wd_status wd_gauge_create(const wd_lattice *lat, const double *U_dev, uint32_t prec_mask,
                          void *dev_buf, size_t bytes, void *stream, wd_gauge **out);
void wd_gauge_destroy(wd_gauge *g);

/* Link compression and temporal gauge (Section 4.3, Appendix A). */
#define WD_RECON_12 12      /* rows a, b; c = (a x b)^* (Appendix A.1) */
#define WD_RECON_8 8        /* Re/Im a2, a3, b1 and the phases of a1, c1 (Appendix A.2); the
                               16-bit formats store the phases divided by pi.  Singular where
                               |a1| = 1; less accurate than WD_RECON_12 */
#define WD_GAUGE_TEMPORAL 1u /* the field is in temporal gauge: U_t(x) = 1 for t < Lt - 1;
                               those links are not read (wd_gauge_fix_temporal makes such a
                               field) */

/* Bytes of dev_buf for wd_gauge_create_ex (recon 12 or 8; flags as below). */
size_t wd_gauge_bytes_ex(const wd_lattice *lat, uint32_t prec_mask, int32_t recon, uint32_t flags);

/* wd_gauge_create with a link format and flags.  With WD_GAUGE_TEMPORAL the
 * temporal links of t < Lt - 1 are checked (max-norm distance to 1 at most
 * 1e-10, else WD_EINVAL); the check synchronises the stream.  Every
 * operator and solver on the handle then uses the unit matrix there. */
wd_status wd_gauge_create_ex(const wd_lattice *lat, const double *U_dev, uint32_t prec_mask,
                             int32_t recon, uint32_t flags, void *dev_buf, size_t bytes, void *stream,
                             wd_gauge **out);

/* Temporal gauge fixing in FP64 (Section 4.3): g(x, 0) = 1, g(x, t+1) =
 * g(x, t) U_t(x, t), U_out_mu(x) = g(x) U_mu(x) g(x + mu)^dagger.  U_in,
 * U_out: device [V][4][3][3][2] (may alias); g_out: device [V][3][3][2].
 * D[U_out] = G D[U_in] G^dagger, so solve with G b and rotate the solution
 * back with G^dagger (wd_gauge_rotate_spinor).  Asynchronous on stream. */
wd_status wd_gauge_fix_temporal(const wd_lattice *lat, const double *U_in, double *U_out, double *g_out,
                                void *stream);

/* out(x) = g(x) in(x) (adjoint: g(x)^dagger in(x)) for nrhs canonical
 * full-lattice spinors (device, [nrhs][V][4][3][2]; out may alias in). */
wd_status wd_gauge_rotate_spinor(const wd_lattice *lat, const double *g, double *out, const double *in,
                                 int32_t nrhs, int32_t adjoint, void *stream);

/* ---- spinor fields ------------------------------------------------------------ */

/* Device bytes of one encoded parity field with nrhs right-hand sides. */
size_t wd_spinor_bytes(const wd_lattice *lat, wd_prec prec, int32_t nrhs);

/* Encode canonical FP64 parity spinors (device, [nrhs][Vh][4][3][2]) into the
 * device field `field` of precision prec.  16-bit formats: per-site norm and
 * quantisation computed in binary32 from the binary32-rounded input,
 * round-to-nearest-even (Section 4.6). */
wd_status wd_spinor_encode(const wd_lattice *lat, wd_prec prec, int32_t nrhs, void *field,
                           const double *canon, void *stream);

/* Decode a device field into canonical FP64 parity spinors. */
wd_status wd_spinor_decode(const wd_lattice *lat, wd_prec prec, int32_t nrhs, double *canon,
                           const void *field, void *stream);

/* Encode the parity-`parity` sites of canonical FP64 full-lattice spinors
 * (device, [nrhs][V][4][3][2]) into a parity field (the even-odd split of
 * Section 3). */
wd_status wd_spinor_encode_full(const wd_lattice *lat, wd_prec prec, int32_t nrhs, int32_t parity,
                                void *field, const double *canon_full, void *stream);

/* Decode a parity field into the parity-`parity` sites of canonical FP64
 * full-lattice spinors; the other sites of canon_full are left untouched. */
wd_status wd_spinor_decode_full(const wd_lattice *lat, wd_prec prec, int32_t nrhs, int32_t parity,
                                double *canon_full, const void *field, void *stream);

/* Spin bases of encoded fields (Appendix B).  Canonical arrays are always in
 * the DeGrand-Rossi basis; every encode, decode and operator entry point
 * works on DeGrand-Rossi fields unless it takes a basis argument.  The UKQCD ("non-relativistic") basis is the
 * rotation psi_UK = S psi_DR with S = [[0, 1, 0, 1], [-1, 0, -1, 0],
 * [0, 1, 0, -1], [-1, 0, 1, 0]] / sqrt(2), in which gamma_t is
 * diag(1, 1, -1, -1): a temporal hop then reads half a spinor.  The solvers
 * rotate their fields into it internally. */
#define WD_BASIS_DEGRAND_ROSSI 0
#define WD_BASIS_UKQCD 1

/* As wd_spinor_encode / wd_spinor_decode, with the field in spin basis
 * `basis` (the rotation is applied in FP64 before storage / after loading).
 * WD_EINVAL for an unknown basis. */
wd_status wd_spinor_encode_basis(const wd_lattice *lat, wd_prec prec, int32_t nrhs, int32_t basis,
                                 void *field, const double *canon, void *stream);
wd_status wd_spinor_decode_basis(const wd_lattice *lat, wd_prec prec, int32_t nrhs, int32_t basis,
                                 double *canon, const void *field, void *stream);

/* ---- operators ------------------------------------------------------------------ */

/* Operators on canonical FP64 parity spinors (device, [nrhs][Vh][4][3][2],
 * DeGrand-Rossi basis, sites in cb order).  `prec` selects the storage and
 * arithmetic of the application: the input is encoded into `prec` inside
 * (16-bit formats: per-site norm, Section 4.6), the operator runs on the
 * encoded fields and the result is decoded back to FP64, so for prec !=
 * WD_FP64 the result carries that format's rounding.  The gauge handle must
 * hold `prec`.  Scratch fields live in the caller's device workspace
 * (>= wd_operator_workspace_bytes bytes, 256-byte aligned); out may alias in.
 * Asynchronous on stream; WD_EINVAL before any launch on a bad argument. */

/* Workspace bytes of wilson_dslash, wilson_mat_pc and mdagm for (lattice,
 * prec, nrhs): four encoded parity fields.  0 on invalid arguments. */
size_t wd_operator_workspace_bytes(const wd_lattice *lat, wd_prec prec, int32_t nrhs);

/* Hopping term restricted to parities (Section 3, Eq. 1):
 * out_p = D_{p,1-p} in_{1-p}, p = out_parity; with dagger = 1 its adjoint
 * (projectors 1 -+ gamma_mu swapped, links daggered).  No factor kappa. */
wd_status wilson_dslash(const wd_gauge *g, double *out, const double *in, int32_t out_parity,
                        int32_t dagger, wd_prec prec, int32_t nrhs, void *workspace, size_t ws_bytes,
                        void *stream);

/* Even-odd preconditioned operator (Section 3, Eq. 2) on even spinors:
 * out_e = in_e - kappa^2 D_eo D_oe in_e; dagger = 1 gives M_hat^dagger. */
wd_status wilson_mat_pc(const wd_gauge *g, double kappa, double *out, const double *in, int32_t dagger,
                        wd_prec prec, int32_t nrhs, void *workspace, size_t ws_bytes, void *stream);

/* Normal operator of the CG solver (Section 5.1): out_e = M_hat^dagger M_hat in_e. */
wd_status mdagm(const wd_gauge *g, double kappa, double *out, const double *in, wd_prec prec,
                int32_t nrhs, void *workspace, size_t ws_bytes, void *stream);

/* Fast path: the same operators on encoded device fields (wd_spinor_encode*),
 * with no conversion.  out and in are fields of precision prec with nrhs
 * right-hand sides; they must not alias.  Asynchronous on stream.
 *   wd_dslash_field:       out_p = D_{p,1-p} in (Eq. 1), or its adjoint.
 *   wd_dslash_field_basis: the same on fields in spin basis `basis`
 *                          (WD_BASIS_*): S D S^T applied to in (Appendix B).
 *   wd_mat_pc_field:       out_e = in_e - kappa^2 D_eo D_oe in_e (Eq. 2) or its
 *                          adjoint; tmp_odd is an odd field of (prec, nrhs).
 *   wd_mdagm_field:        out_e = M_hat^dagger M_hat in_e (Section 5.1);
 *                          tmp_odd, tmp_even are fields of (prec, nrhs). */
wd_status wd_dslash_field(const wd_gauge *g, void *out, const void *in, int32_t out_parity,
                          int32_t dagger, wd_prec prec, int32_t nrhs, void *stream);
wd_status wd_dslash_field_basis(const wd_gauge *g, void *out, const void *in, int32_t out_parity,
                                int32_t dagger, wd_prec prec, int32_t nrhs, int32_t basis, void *stream);
wd_status wd_mat_pc_field(const wd_gauge *g, double kappa, void *out, const void *in, void *tmp_odd,
                          int32_t dagger, wd_prec prec, int32_t nrhs, void *stream);
wd_status wd_mdagm_field(const wd_gauge *g, double kappa, void *out, const void *in, void *tmp_odd,
                         void *tmp_even, wd_prec prec, int32_t nrhs, void *stream);

/* mdagm for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out_e = M_hat^dagger M_hat in_e on canonical FP64 parity spinors, with no
 * workspace argument.  Its four encoded scratch fields live in a static
 * device array of 64 MiB that every GPU the library runs on holds until the
 * process ends; (lattice, prec, nrhs) needing more than that
 * (wd_operator_workspace_bytes > 64 MiB: for one RHS FP64 above Vh = 87,360,
 * FP32 above Vh = 174,720, 16-bit above Vh = 322,624) are refused with
 * WD_EINVAL.  The launch shape is the tuned one if already known, else the
 * default (no tuning runs).  Allocates nothing.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU race, so the caller serialises them.
 * Asynchronous on stream. */
wd_status mdagm_noalloc(const wd_gauge *g, double kappa, double *out, const double *in, wd_prec prec,
                        int32_t nrhs, void *stream);

/* ---- solvers ------------------------------------------------------------------- */

#define WD_SOLVER_BICGSTAB 0 /* BiCGstab on M_hat (Section 5.1) */
#define WD_SOLVER_CG 1       /* CG on M_hat^dag M_hat x_e = M_hat^dag b_hat_e (Section 5.1) */

typedef struct {
  double tol;          /* target ||b - (1 - kappa D) x|| / ||b||, FP64 true residual, > 0 */
  int32_t maxiter;     /* cap on k + l (iterations plus reliable updates), >= 1 */
  wd_prec inner;       /* storage precision of the Krylov vectors and of the M_hat applied to
                          them; WD_FP64 gives the plain double-precision solver */
  double delta;        /* reliable-update trigger of Algorithm 2: update when |r^| < delta *
                          max|r^| since the last update; 0 <= delta < 1 (0: update only to
                          confirm convergence) */
  int32_t nrhs;        /* right-hand sides solved together, 1..64 (one multi-RHS dslash per hop) */
  int32_t use_graph;   /* 1: the iteration body is captured once as a hipGraph and replayed
                          (needs a non-NULL stream) */
  int32_t check_every; /* inner iterations launched (and, with use_graph, captured in one
                          graph) between two reads of the per-RHS flags by the host, 0..64
                          (0 and 1: every iteration).  An RHS that triggers a reliable
                          update, converges or breaks down waits on the device for the
                          rest of the batch, so results do not depend on it; maxiter is
                          checked once per batch */
  int32_t x0_given;    /* reserved, must be 0 */
  int32_t restart;     /* 0: reliable updates (Algorithm 2), the Krylov space is kept across
                          updates.  1: defect correction (Algorithm 1): each update ends an
                          inner solve, whose tolerance relative to the residual it started
                          from is delta (> 0), and the next inner solve restarts the Krylov
                          recurrence from the new FP64 residual */
} wd_solve_params;

typedef struct {
  int32_t iters;            /* k + l: iterations plus reliable updates (Table 5 convention) */
  int32_t reliable_updates; /* l */
  int32_t converged;        /* 1 if the FP64 true residual reached tol */
  int32_t status;           /* WD_OK, WD_NOT_CONVERGED or WD_EBREAKDOWN for this RHS */
  double true_rel_resid;    /* ||b_hat - M_hat x_e|| / ||b|| in FP64 at exit; equals the
                               full-system relative residual (the odd-site residual vanishes) */
  double seconds;           /* wall time of the whole solve (host clock) */
  double gflops;            /* nominal rate: 1320 flops per site per dslash plus BLAS-1 flops */
} wd_solve_info;

/* Device workspace bytes for a solve (all fields, partial sums, scalars). */
size_t wd_solve_workspace_bytes(const wd_lattice *lat, const wd_solve_params *params,
                                int32_t solver);

/* Solve (1 - kappa D) x = b for params->nrhs right-hand sides: prepare
 * b_hat_e = b_e + kappa D_eo b_o, solve M_hat x_e = b_hat_e with reliable
 * updates in FP64 (Algorithm 2), reconstruct x_o = b_o + kappa D_oe x_e.
 * x, b: device, canonical full-lattice FP64 [nrhs][V][4][3][2].  The gauge
 * handle must hold WD_FP64 and params->inner.  Blocks until done.  info is an
 * array of nrhs records (may be NULL).  Returns WD_OK if every RHS converged,
 * WD_NOT_CONVERGED if one hit maxiter (x holds the best FP64 iterate),
 * WD_EBREAKDOWN if the Krylov recurrence broke down for one. */
wd_status bicgstab_solve(const wd_gauge *g, double kappa, double *x, const double *b,
                         const wd_solve_params *params, wd_solve_info *info, void *workspace,
                         size_t ws_bytes, void *stream);

/* Same contract with CG on the normal equations M_hat^dag M_hat. */
wd_status cg_solve(const wd_gauge *g, double kappa, double *x, const double *b,
                   const wd_solve_params *params, wd_solve_info *info, void *workspace,
                   size_t ws_bytes, void *stream);

/* Step API for interleaving several solves (one stream each).  begin
 * validates, prepares the source and the first residual; step runs up to
 * n_iters batches of check_every iterations (each batch followed by the
 * reliable updates it triggered) and
 * sets *done when every RHS has converged, broken down or reached maxiter;
 * end reconstructs x, fills info[nrhs] and releases the handle. */
wd_status wd_solver_begin(int32_t solver, const wd_gauge *g, double kappa, double *x,
                          const double *b, const wd_solve_params *params, void *workspace,
                          size_t ws_bytes, void *stream, wd_solver **out);
wd_status wd_solver_step(wd_solver *h, int32_t n_iters, int32_t *done);
wd_status wd_solver_end(wd_solver *h, wd_solve_info *info);

/* Diagnostics of an in-flight solve: copies, per RHS, the iterated squared
 * residual |r^|^2, the FP64 true squared residual at the last reliable update
 * and |b|^2 into out[nrhs][3] (host memory).  Synchronises the solver's stream. */
wd_status wd_solver_residuals(wd_solver *h, double *out);

/* ---- serving: continuous batching of independent solves ------------------------- */

typedef struct wd_server wd_server;

typedef struct {
  int32_t max_slots;      /* solves in flight at once (one HIP stream each), 1..64 */
  int32_t iters_per_pump; /* iterations each in-flight solve advances per wd_server_pump, >= 1 */
} wd_serve_params;

/* A scheduler over a caller-owned device arena (>= 256-byte aligned).  Each
 * admitted request gets its solver workspace (wd_solve_workspace_bytes) from
 * the arena and its own stream; requests wait in FIFO order until a slot and
 * enough arena memory are free (admission by HBM footprint).  Gauge handles
 * are shared read-only by the requests that use them. */
wd_status wd_server_create(void *arena, size_t arena_bytes, const wd_serve_params *params,
                           wd_server **out);

/* Queue a solve (solver = WD_SOLVER_BICGSTAB or WD_SOLVER_CG) of
 * (1 - kappa D) x = b with the given parameters (with use_graph, each solve
 * replays its own captured iteration on its slot's stream).  x and
 * b (device, full-lattice FP64, params->nrhs RHS) must stay valid until the
 * request is reported done; b must already hold its values (the slot streams
 * are non-blocking and do not wait on the caller's streams).  Returns
 * WD_ENOMEM if the request's workspace can never fit the arena.  Never
 * blocks. */
wd_status wd_server_submit(wd_server *s, int32_t solver, const wd_gauge *g, double kappa, double *x,
                           const double *b, const wd_solve_params *params, int64_t *request_id);

/* One scheduling round (iters_per_pump times over): admit queued requests
 * that fit, launch the next check_every iterations of every in-flight solve
 * that has none outstanding (each on its own stream, so they overlap on the
 * device), then wait until at least one in-flight solve's iterations have
 * landed and complete every solve whose iterations have (its reliable
 * updates run then); a solve is never held back by the others.  Finished
 * solves release their slot and memory and queued requests move in.
 * Reports the in-flight and queued counts. */
wd_status wd_server_pump(wd_server *s, int32_t *n_active, int32_t *n_queued);

/* Result of a request: *done = 1 once finished (info[0..nrhs) filled, status
 * = the solve's wd_status, e.g. WD_EINVAL for a NaN source), 0 while queued
 * or in flight.  Calls on one server must not overlap (one host thread). */
wd_status wd_server_poll(wd_server *s, int64_t request_id, int32_t *done, int32_t *status,
                         wd_solve_info *info);

/* Destroys the scheduler (requests still in flight are finished first). */
wd_status wd_server_destroy(wd_server *s);

#ifdef __cplusplus
}
#endif

#endif /* WD_H */
