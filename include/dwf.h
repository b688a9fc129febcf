/*
 * dwf.h -- C ABI of the MI355X (gfx950) domain-wall / Moebius hot path.
 *
 * Method: H. Yin and R. D. Mawhinney, "Improving DWF Simulations: the Force
 * Gradient Integrator and the Moebius Accelerated DWF Solver", Lattice 2011.
 *   Sec. 4  the Dirac equation D_DW(m) x = b, the Moebius operator D'_DW and
 *           the Moebius-accelerated solver (MADWF);
 *   Sec. 5  defect correction; Table 1 ("Op. count" = 4D Wilson applications);
 *   Sec. 2  the force e_i(S), e_i(U) = T_i U, and the force-gradient step
 *           U' = exp(-tau^2/24 F^j T_j) U with the first solve reused.
 *
 * Operator conventions (the paper defers the definitions to its
 * domain-wall/overlap transformation reference; these are the readings used):
 *   D_W psi(x) = (4 - M5) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                             + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *   chiral basis, g_5 = diag(1, 1, -1, -1), P+- = (1 +- g_5)/2;
 *   (D(m) psi)_s = (b D_W + 1) psi_s + (c D_W - 1)(P- psi_{s+1} + P+ psi_{s-1}),
 *   psi_{Ls} = -m psi_0, psi_{-1} = -m psi_{Ls-1}; Shamir DWF is b = 1, c = 0.
 *   Even-odd split on the 4D checkerboard, parity (x+y+z+t) mod 2:
 *   D = [[A, B_eo], [B_oe, A]], A = (b d + 1) + (c d - 1) S~, d = 4 - M5,
 *   B = -1/2 H (b + c S~), M_prec = 1 - A^-1 B_oe A^-1 B_eo (odd sites).
 *
 * Data layouts.  Every pointer argument named U, in, out, b, x, phi is a
 * DEVICE pointer (hipMalloc / torch CUDA tensor) owned by the caller.
 *   natural gauge   complex128 [4][T][Z][Y][X][3][3]   (mu = 0..3 <-> x,y,z,t)
 *   natural 5D      complex128 [Ls][T][Z][Y][X][4][3]
 *   natural force   complex128 [4][T][Z][Y][X][3][3]
 *   packed half     one parity: [x_cb][12][Ls] pairs (re, im) of the storage
 *                   type (fp64, fp32, fp16, bf16), x_cb = lexicographic index/2,
 *                   component 12 = spin*3 + colour; fp16 adds a trailing
 *                   float norm array [x_cb][Ls] (value = stored * norm).
 *   packed full     [even half][odd half].
 *   packed gauge    per output parity p: [x_cb][8][3][3] pairs: directions
 *                   0..3 = U_mu(x), 4..7 = U_mu(x-mu)^+, antiperiodic phase
 *                   folded in; parity 0 block then parity 1 block.
 * dwf_field_bytes() gives the size of every packed layout.
 *
 * Ownership and streams: the library owns only what a dwf_ctx allocates
 * (workspace, geometry tables, packed low-precision copies); it is freed by
 * dwf_ctx_destroy.  All work is ordered on the ctx stream.  Solver calls
 * return after the FP64 true residual has been read back to the host.
 *
 * Errors: every call returns DWF_OK (0), a negative error code, or
 * DWF_NOT_CONVERGED (> 0, the info struct is still filled and x holds the
 * best iterate).  dwf_last_error() returns a thread-local message for the
 * last failing call.  No C++ exception crosses this interface.  A call
 * whose arguments fail validation performs no device work.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DWF_OK 0
#define DWF_NOT_CONVERGED 1
#define DWF_ERR_ARG (-1)   /* invalid extents, Ls, precision, op or NULL pointer */
#define DWF_ERR_HIP (-2)   /* a HIP runtime error (message in dwf_last_error) */
#define DWF_ERR_NOMEM (-3) /* device allocation failed */
#define DWF_ERR_NAN (-4)   /* a NaN/Inf appeared in a source or a residual */

enum dwf_precision { DWF_FP64 = 0, DWF_FP32 = 1, DWF_FP16 = 2, DWF_BF16 = 3 };
enum dwf_kind { DWF_KIND_GAUGE = 0, DWF_KIND_FULL = 1, DWF_KIND_EVEN = 2, DWF_KIND_ODD = 3 };
enum dwf_op {
  DWF_OP_HOP = 0,   /* Wilson hop H (dwf_dslash) or H (b + c S~) (mobius_dslash), parity -> parity */
  DWF_OP_MPREC = 1, /* M_prec on odd halves */
  DWF_OP_FULL = 2,  /* D(m) on packed full fields */
  DWF_OP_A = 3,     /* site-local A on a half field */
  DWF_OP_AINV = 4   /* site-local A^-1 on a half field */
};
enum dwf_op5 {
  DWF_OP5_HOP = 0,  /* K = (5 - M5) - D(m), both 5D parities (dwf_dslash_5d) */
  DWF_OP5_SCHUR = 1 /* S = d0 - K_eo K_oe / d0 on the even 5D parity (dwf_dslash_5d) */
};

typedef struct {
  int dims[4];    /* X, Y, Z, T: each even and >= 2 */
  int Ls;         /* fifth-dimension extent, 2..128 */
  int tbc;        /* 0 periodic, 1 antiperiodic in T */
  double M5;      /* domain-wall height (D_W at mass -M5) */
  double mass;    /* quark mass m (1.0 = Pauli-Villars) */
  double b, c;    /* Moebius coefficients (Shamir: 1, 0) */
  int prec;       /* storage precision of packed operands of dslash calls */
  int prec_inner; /* inner-iteration precision of solvers (FP64 = plain FP64 CG) */
  /* optional s-dependent Moebius coefficients b_s, c_s (Sec. 4 admits any Moebius
   * operator): host arrays of Ls entries each, read during the call; NULL = the
   * constants b, c.  (D psi)_s = (b_s D_W + 1) psi_s + (c_s D_W - 1)(P- psi_{s+1} + P+ psi_{s-1}).
   * Not accepted by the batched solvers (cg_ne_batched, quotient_force). */
  const double* b_s;
  const double* c_s;
} dwf_params;

typedef struct {
  /* in */
  double tol;      /* target full-system true residual ||b - D x|| / ||b|| */
  double delta;    /* reliable-update trigger: iterated residual fell by this factor (0 -> 0.1) */
  int maxit;       /* iteration cap over all restarts (0 -> 100000) */
  /* out */
  int iters;                /* CG iterations (each one M_prec^+ M_prec application) */
  int reliable_updates;     /* FP64 residual recomputations */
  int restarts;             /* tightenings of the normal-equation tolerance */
  double true_rel_resid;    /* FP64 ||b - D x|| / ||b|| on return */
  double seconds;           /* wall time of the call */
  long long wilson_apps;    /* Table 1 "Op. count": iterations x Ls */
  int iters_first;          /* fermion_force with tau_fg > 0: iterations of the solve at U */
} dwf_solve_info;

typedef struct {
  /* in */
  int n_dc;           /* defect-correction steps (Sec. 5; the paper uses 3) */
  double tol_pv;      /* relative tolerance of the Pauli-Villars solves */
  double tol_mobius;  /* relative tolerance of the Moebius solve */
  double tol;         /* final full-system true residual */
  double delta;       /* reliable-update trigger (0 -> 0.1) */
  int maxit;          /* cap per solve (0 -> 100000) */
  int prec_pv;        /* inner precision of the PV solves */
  int prec_final;     /* inner precision of the final DWF solve */
  /* out */
  int pv_iters, mobius_iters, final_iters, n_pv, n_mobius;
  double resid_after_dc[8];
  double true_rel_resid;
  double seconds, seconds_pv, seconds_mobius, seconds_final;
  long long wilson_apps; /* pv_iters*L + mobius_iters*L' + final_iters*L */
} dwf_madwf_info;

typedef struct dwf_ctx dwf_ctx;

/* Create a context bound to a HIP stream (hipStream_t as void*; NULL = the
 * default stream) on the current device. */
int dwf_ctx_create(dwf_ctx** ctx, void* stream);
int dwf_ctx_destroy(dwf_ctx* ctx);
int dwf_ctx_set_stream(dwf_ctx* ctx, void* stream);
/* Free the context's solver workspace (after the work queued on its stream); the geometry
 * tables, fifth-dimension tables and tuned shapes stay.  The next call allocates what it
 * needs again.  For callers that switch between solvers whose workspaces do not fit in
 * device memory together. */
int dwf_ctx_release(dwf_ctx* ctx);
const char* dwf_last_error(void);

/* Bytes of a packed field of the given kind and precision (0 on bad arguments). */
size_t dwf_field_bytes(const dwf_params* p, int kind, int prec);

/* natural (complex128, device) <-> packed (device).  EVEN/ODD pack reads the
 * sites of that parity from a natural 5D field; unpack writes only them.
 * Gauge pack folds the boundary phase and the backward daggers in. */
int dwf_pack(dwf_ctx* ctx, const dwf_params* p, int kind, int prec, const void* natural, void* packed);
int dwf_unpack(dwf_ctx* ctx, const dwf_params* p, int kind, int prec, const void* packed, void* natural);
/* packed -> packed precision conversion (round to nearest even). */
int dwf_convert(dwf_ctx* ctx, const dwf_params* p, int kind, int prec_in, const void* in, int prec_out,
                void* out);

/* One application of the Shamir DWF operator family (b, c ignored: 1, 0) on packed
 * operands of precision p->prec (Sec. 4, D_DW(m); the hop is the paper's unit of
 * cost, Table 1).  op HOP: out (parity `parity`) = H in (other parity); MPREC:
 * odd -> odd; FULL: D(m) on full fields; A / AINV: site-local blocks.
 * dagger = 1 applies the adjoint.  in and out must not alias. */
int dwf_dslash(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int parity,
               int dagger);

/* The same for the Moebius operator D'_DW(m) with p->b, p->c (Sec. 4); op HOP
 * applies H (b + c S~). */
int mobius_dslash(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op,
                  int parity, int dagger);

/* dwf_dslash for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same operator, arguments, layouts
 * and errors as dwf_dslash, but the call performs no device allocation: the neighbour tables
 * and the intermediate half fields of M_prec live in one device array of 256 MiB per device,
 * set up by dwf_ctx_create on the context's device (which must be current).  The call returns
 * DWF_ERR_ARG, before any device work, when the op needs more than that (2 * V/2 * 8 index
 * words, plus one intermediate half field for M_prec and two for M_prec^+), or when it needs a
 * fifth-dimension block and Ls is not 8, 16 or 32 (the blocks run in recurrence form only).
 * Every call rebuilds what it reads from the array, so no state carries over between calls;
 * calls that overlap on one device (several streams or threads) share the array and race. */
int dwf_dslash_noalloc(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op,
                       int parity, int dagger);

/* Solve D(m) x = b (Sec. 4, the Dirac equation) for packed FP64 full fields by
 * CG on the even-odd normal equations.  U: packed FP64 gauge.  x holds the
 * initial guess on entry.  p->prec_inner < FP64 runs the iterations in that
 * storage precision (FP32 arithmetic) with FP64 reliable updates, FP64 CG
 * scalars and an FP64 solution accumulator.  Workspace (held by ctx from the
 * first call until dwf_ctx_destroy): eight search directions, the residual and
 * two temporaries as odd half fields of the iteration precision (one more for
 * Moebius operators, and one more, M_prec p, for FP64 iterations, s-dependent
 * coefficients, Ls other than 8, 16, 32, and launch shapes with several slices per
 * thread or LDS-staged neighbours: elsewhere the last hop of M_prec^+ q rebuilds q
 * from A^-+ q), an FP32 solution increment and eleven FP64 half fields
 * (one FP64 half field at 24^3x64, Ls = 32: 2.7 GB; the whole set in FP16
 * iterations about 40 GB). */
int cg_ne(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* b, void* x, dwf_solve_info* info);

/* Shamir DWF checkerboarded in five dimensions (an alternative to the 4D even-odd
 * split above; Sec. 4 admits any solver of D_DW(m) inside MADWF).  With the 5D parity
 * (x + y + z + t + s) mod 2 and d0 = 5 - M5, D(m) = d0 - K, where
 *   K psi = 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *           + P- psi_{s+1} + P+ psi_{s-1}       (psi_{Ls} = -m psi_0, psi_{-1} = -m psi_{Ls-1})
 * connects opposite 5D parities only, and the even-site Schur complement is
 * S = d0 - K_eo K_oe / d0.  Shamir only (b = 1, c = 0, no b_s / c_s; the c D_W term of a
 * Moebius operator hops x and s together) and Ls in {2, 4, 8, 16, 32, 64, 128}; otherwise
 * DWF_ERR_ARG.
 *
 * cg_ne_5d: solve D(m) x = b by CG on S^+ S x_e = S^+ (b_e + K_eo b_o / d0), then
 * x_o = (b_o + K_oe x_e) / d0, to the full-system true residual info->tol (computed with the
 * 4D even-odd D(m) of cg_ne).  Arguments, precisions, reliable updates, info and errors as
 * cg_ne; x holds the initial guess.  Workspace (held by ctx): the fields of cg_ne's iteration,
 * each one 5D-parity field (the size of one packed half), plus eight FP64 5D-parity fields and
 * one FP64 full field (the true residual).
 *
 * dwf_dslash_5d: one application of op on packed full fields of precision p->prec (U packed
 * in p->prec): DWF_OP5_HOP out = K in (dagger: K^+ in); DWF_OP5_SCHUR: the even-5D-parity part
 * of out = S in_even (dagger: S^+), its odd part zero (in's odd part is not read).  in and out
 * must not alias. */
int cg_ne_5d(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* b, void* x, dwf_solve_info* info);
int dwf_dslash_5d(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int dagger);

/* Several right-hand sides solved together (the Hasenbusch mass ladder of Sec. 3):
 * every hop stage of M_prec and M_prec^+ is ONE launch over all unconverged
 * right-hand sides, each workgroup loading the links of its sites once for all
 * right-hand sides on that lattice.  Shamir right-hand sides of one lattice with
 * Ls 8, 16 or 32 run interleaved along the fifth dimension (up to 256 / Ls of them
 * per launch: slice s of right-hand side r is slice r Ls + s of one field; tuning
 * kernel 2); the others run as separate fields in one launch (tuning kernel 1).
 * One device-to-host copy per iteration returns every residual.  per_rhs[k] may
 * differ in mass, and -- a ragged batch
 * -- in extents and Ls, with U[k] the packed FP64 links of that lattice (equal
 * pointers share link loads).  All entries share M5, b, c, tbc and prec_inner.
 * b[k], x[k]: packed FP64 full fields (x[k] = initial guess on entry).
 * per_rhs_info[k].tol is that right-hand side's target true residual; delta and
 * maxit are taken from per_rhs_info[0]. */
int cg_ne_batched(dwf_ctx* ctx, int nrhs, const dwf_params* per_rhs, const void* const* U, const void* const* b,
                  void* const* x, dwf_solve_info* per_rhs_info);

/* Moebius-accelerated DWF solve (Sec. 4 algorithm, Sec. 5 defect correction):
 * target = Shamir DWF (Ls = L), inner = Moebius (Ls = L', b', c', same dims,
 * M5, mass).  info->n_dc steps of: residual, PV solve, Moebius solve, PV
 * reconstruction; then a warm-started DWF solve to info->tol.  x is
 * overwritten (packed FP64 full, target Ls). */
int mobius_accel_solve(dwf_ctx* ctx, const dwf_params* target, const dwf_params* inner, const void* U,
                       const void* b, void* x, dwf_madwf_info* info);

/* Fermion force of S = phi^+ (M_prec^+ M_prec)^-1 phi (Sec. 2: e_i(S) with
 * e_i(U) = T_i U, T_a = i lambda_a / 2).  phi: packed FP64 odd half.  x_io:
 * optional packed FP64 odd half: initial guess in, X = (M^+M)^-1 phi out.
 * F (device, natural force layout, complex128) receives
 *   out_kind 0: F_mu(x) = sum_a e_a(S) T_a                (traceless anti-Hermitian)
 *   out_kind 1: G_mu(x) = dS/dU in the convention dS = Re sum conj(G) dU.
 * tau_fg > 0: force-gradient step -- F1 at U, U' = exp(-tau^2/24 F1) U, then the
 * force at U' with its solve started from X(U); U is left unchanged.
 * *S receives the action at the configuration whose force is returned.
 * Each solve runs until the FP64 true residual ||phi - M^+M X|| / ||phi|| of the normal
 * equations, recomputed after it, is at most info->tol (default 1e-12), within info->maxit
 * iterations over all solves of the call; info->true_rel_resid receives the largest such
 * residual.  Returns DWF_NOT_CONVERGED (F, S and x_io still written) if a solve stopped at
 * maxit above the tolerance. */
int fermion_force(dwf_ctx* ctx, const dwf_params* p, const void* U_natural, const void* phi, void* F, double* S,
                  double tau_fg, int out_kind, void* x_io, dwf_solve_info* info);

/* One molecular-dynamics trajectory of the force-gradient integrator (Sec. 2):
 * per step of size tau the PQPQP sequence
 *   P -= tau/6 F(U); U = exp(tau/2 P) U;
 *   P -= 2 tau/3 F(U') with U' = exp(-tau^2/24 F(U)) U (its solve started from X(U));
 *   U = exp(tau/2 P) U; P -= tau/6 F(U),
 * for H = sum_a p_a^2 / 2 + S_g + phi^+ (M_prec^+ M_prec)^-1 phi, S_g = the Wilson
 * plaquette action with coupling beta (periodic links), F = sum_a e_a(S) T_a.
 * U (natural link layout) and P (momenta P = sum_a p_a T_a, same layout, traceless
 * anti-Hermitian), both device complex128, are updated in place; phi: packed FP64
 * odd half (held fixed).  The force solves run in p->prec_inner to the normal-
 * equation tolerance info->tol (FP64 true residual, as for fermion_force), each within
 * info->maxit iterations.  Fills H_start, H_end and the counters; returns DWF_NOT_CONVERGED
 * (the trajectory still completed) if a force solve stopped at maxit above the tolerance. */
typedef struct {
  double beta;             /* plaquette coupling */
  double tau;              /* step size */
  int n_steps;
  double tol, delta;       /* force solves: normal-equation tolerance, reliable-update delta */
  int maxit;
  double H_start, H_end;   /* out */
  int force_evals;         /* out: force evaluations (3 per step + 1) */
  long long cg_iters;      /* out: all CG iterations */
  long long fg_iters_first, fg_iters_forecast; /* out: iterations of the solves at U and at U' */
  double seconds;          /* out */
} dwf_hmc_info;
int hmc_fgi_trajectory(dwf_ctx* ctx, const dwf_params* p, void* U_natural, void* P_natural, const void* phi,
                       dwf_hmc_info* info);

/* Hasenbusch mass ladder (Sec. 3): the quotient actions
 *   S_i = phi_i^+ M(m_i) (M(m_{i-1})^+ M(m_{i-1}))^-1 M(m_i)^+ phi_i,   i = 1..nq,
 * M = M_prec of p with its mass replaced by masses[] (nq + 1 entries,
 * masses[0] < masses[1] < ... < masses[nq]; the paper's m + mu_i, ending at the
 * Pauli-Villars mass 1).  The nq normal-equation solves (tolerance info->tol,
 * default 1e-10: Sec. 3 notes they need less than the usual accuracy) run as
 * one batched CG in p->prec_inner; then F (device, natural force layout,
 * complex128, out_kind as for fermion_force) receives the sum over i of the
 * forces e_a(S_i), and S[i] (host, nq entries, may be NULL) the actions.
 * phi[i]: packed FP64 odd halves.  x_io (may be NULL; entries may be NULL):
 * X_i = (M(m_{i-1})^+ M(m_{i-1}))^-1 M(m_i)^+ phi_i, initial guess in, solution
 * out.  Returns DWF_NOT_CONVERGED (F and S still filled) if a solve stopped at
 * maxit; DWF_ERR_ARG for nq < 1, masses not increasing, NULL pointers. */
int quotient_force(dwf_ctx* ctx, const dwf_params* p, int nq, const double* masses, const void* U_natural,
                   const void* const* phi, void* F, double* S, int out_kind, void* const* x_io,
                   dwf_solve_info* info);

/* Set / query the launch configuration of the hop kernels for one (precision,
 * Ls): 4D sites per workgroup, s-slices per thread, whether workgroups are
 * remapped so that each XCD walks a contiguous range of the lattice, and the
 * LDS mode link_lds: 0 nothing staged, 1 the workgroup's links staged in LDS,
 * 2 the neighbour spinors of every direction staged in LDS (FP16, Ls 8/16/32,
 * one slice per thread, 256 / Ls sites per workgroup).  Used by the autotuner;
 * kernel_id 0 = hop, 1 = the batched hop of cg_ne_batched / quotient_force on separate
 * fields (one slice per thread, link_lds 0 or 1; xcd_remap also keeps the right-hand
 * sides of one site block on one XCD), 2 = the batched hop on right-hand sides
 * interleaved along the fifth dimension (Shamir, Ls 8/16/32: the batched solvers use it
 * unless it is switched off; sites_per_block 1 = on, -1 = off, s_per_thread 1, link_lds
 * 0 or 1; the workgroup holds the whole site, 256 / (nrhs Ls) sites).
 * sites_per_block = s_per_thread = 0 restores the default.
 * Rejects shapes the kernel cannot run (more than 256 threads, Ls not divisible
 * by s_per_thread, LDS above 64 KiB, mode 2 outside its shape) with DWF_ERR_ARG. */
int dwf_tune_set(dwf_ctx* ctx, int kernel_id, int prec, int Ls, int sites_per_block, int s_per_thread,
                 int xcd_remap, int link_lds);
int dwf_tune_get(dwf_ctx* ctx, int kernel_id, int prec, int Ls, int* sites_per_block, int* s_per_thread,
                 int* xcd_remap, int* link_lds);

/* Set / query the traversal tile of the hop kernels on one lattice (dims[4], tbc as in
 * dwf_params): workgroups visit the output sites in 3D tiles of tile[0] x tile[1] x tile[2]
 * spatial sites, each tile walked along t before the next, so that the eight users of an
 * input spinor run close together in time and its re-reads hit the L2.  Only the order of
 * the visits changes; every result is bit-identical.  Each extent must divide the lattice
 * extent (DWF_ERR_ARG otherwise); 0, 0, 0 restores the default: among the tiles of at most
 * 600 sites per t-slice, the one with the smallest halo ratio (tx+2)(ty+2)(tz+2)/(tx ty tz).
 * dwf_tune_tile waits for the context stream before it replaces the order; tile is an int[3]
 * host array. */
int dwf_tune_tile(dwf_ctx* ctx, const int* dims, int tbc, const int* tile);
int dwf_tune_tile_get(dwf_ctx* ctx, const int* dims, int tbc, int* tile);

/* Measurement.  dwf_timing_enable(ctx, 1) starts recording a HIP event pair on the
 * context stream around every Wilson-hop, fifth-dimension and fermion-force kernel
 * launch the context makes (the events add a few microseconds between launches);
 * dwf_timing_enable(ctx, 0) stops recording and discards the records.
 * dwf_timing_report synchronizes the context stream and writes one line per
 * kernel variant launched since the last report,
 *   "<kernel name>\t<launches>\t<total ms>\t<total algorithmic bytes>\n",
 * into buf (NUL-terminated; the kernel name is the template instance as
 * profilers print it; algorithmic bytes count each input and output field and
 * the links once per launch), then clears the records.  Returns DWF_ERR_ARG if
 * buf is NULL or len is too small (the records are then lost). */
int dwf_timing_enable(dwf_ctx* ctx, int enable);
int dwf_timing_report(dwf_ctx* ctx, char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* DWF_H */
