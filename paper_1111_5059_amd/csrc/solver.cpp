// Solvers on the even-odd DWF/Moebius system:
//   * CG on the normal equations of M_prec (CGNR), optionally with iterations
//     in FP32 / FP16 / BF16 storage and FP64 reliable updates (Sleijpen and van
//     der Vorst 1996; as used for lattice QCD on GPUs by Clark et al. 2010) --
//     FP64 CG scalars, FP64 solution accumulator, FP64 true residual;
//   * the Moebius-accelerated DWF solve (Sec. 4 algorithm, Sec. 5 defect
//     correction, Table 1 operation counting);
//   * the fermion force and the force-gradient step (Sec. 2).
#include <chrono>
#include "runtime.hpp"
#include "solver.hpp"
#include "batch.hpp"

namespace dwf {

using Clock = std::chrono::steady_clock;

template <typename P>
static CHalf<P> chalf_at(const void* base, size_t off, const Geometry* g, int Ls) {
  return chview<P>(reinterpret_cast<const char*>(base) + off, g, Ls);
}
template <typename P>
static Half<P> half_at(void* base, size_t off, const Geometry* g, int Ls) {
  return hview<P>(reinterpret_cast<char*>(base) + off, g, Ls);
}

static std::string pname(int prec) {
  static const char* n[4] = {"f64", "f32", "f16", "bf16"};
  return n[prec & 3];
}

// packed links of precision prec converted from the packed FP64 links
static const void* links_in(dwf_ctx* ctx, const Geometry* g, const void* U64, int prec, const std::string& tag) {
  if (prec == DWF_FP64) return U64;
  const long n = 2 * g->nsites * 72;
  void* dst;
  switch (prec) {
    case DWF_FP32:
      dst = ws_get(ctx, tag + ".U32", n * sizeof(P32::S));
      DWF_CHECK_LAUNCH((launch_convert_links<P64, P32>(reinterpret_cast<const double2*>(U64),
                                                        reinterpret_cast<P32::S*>(dst), n, ctx->stream)));
      return dst;
    case DWF_FP16:
      dst = ws_get(ctx, tag + ".U16", n * sizeof(P16::S));
      DWF_CHECK_LAUNCH((launch_convert_links<P64, P16>(reinterpret_cast<const double2*>(U64),
                                                        reinterpret_cast<P16::S*>(dst), n, ctx->stream)));
      return dst;
    default:
      dst = ws_get(ctx, tag + ".Ub16", n * sizeof(PB16::S));
      DWF_CHECK_LAUNCH((launch_convert_links<P64, PB16>(reinterpret_cast<const double2*>(U64),
                                                         reinterpret_cast<PB16::S*>(dst), n, ctx->stream)));
      return dst;
  }
}

// ------------------------------------------------------------------ CG on M^dag M
// Solves M^dag M x = rhs (odd sites) until ||rhs - M^dag M x|| <= tol_n ||rhs||.
// x (FP64) holds the initial guess.  Iterations in storage precision Pi; for
// Pi != FP64 the iterate increment accumulates in FP32 and is folded into the
// FP64 x at every reliable update, where the residual is recomputed in FP64.
template <typename Pi>
static int cg_normal(dwf_ctx* ctx, const Op<P64>& op64, const Op<Pi>& opi, CHalf<P64> rhs, Half<P64> x,
                     double tol_n, int maxit, double delta, const std::string& tag, SolveStats* st) {
  const Geometry* g = op64.g;
  const int Ls = op64.Ls;
  const long n5 = g->nsites * Ls;
  const size_t hb64 = half_size<P64>(g, Ls), hbi = half_size<Pi>(g, Ls);
  double* part = partials_buf(ctx);
  double* sc = scalars_buf(ctx);
  hipStream_t s = ctx->stream;
  constexpr bool MIXED = !std::is_same<Pi, P64>::value;
  // solution increment between reliable updates (FP32, or FP64 for FP64 iterations)
  using PX = typename IncrementPrec<Pi>::type;
  constexpr bool RESTART = std::is_same<Pi, PB16>::value;

  // FP64 residual r_hi = rhs - M^dag M x
  Half<P64> rhi = hview<P64>(ws_get(ctx, tag + ".rhi", hb64), g, Ls);
  Half<P64> t64a = hview<P64>(ws_get(ctx, tag + ".t64a", hb64), g, Ls);
  Half<P64> t64b = hview<P64>(ws_get(ctx, tag + ".t64b", hb64), g, Ls);
  Half<P64> t64c = hview<P64>(ws_get(ctx, tag + ".t64c", hb64), g, Ls);
  auto true_residual = [&]() -> double {
    op64.mprec(cv(x), t64a, t64b);
    op64.mprec_dag(cv(t64a), rhi, t64b, t64c);
    DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, rhs, -1.0, rhi, n5, Ls, s));
    return norm2_sync<P64>(ctx, cv(rhi), g, Ls);
  };
  const double rhs2 = norm2_sync<P64>(ctx, rhs, g, Ls);
  if (rhs2 == 0.0) {
    DWF_CHECK_LAUNCH(launch_zero(x.data, hb64, s));
    return 0;
  }
  const double target = tol_n * tol_n * rhs2;
  // a zero initial guess (the inner solves of MADWF) needs no operator application: r = rhs
  double rr;
  if (norm2_sync<P64>(ctx, cv(x), g, Ls) == 0.0) {
    DWF_CHECK_HIP(hipMemcpyAsync(rhi.data, rhs.data, hb64, hipMemcpyDeviceToDevice, s));
    rr = rhs2;
  } else {
    rr = true_residual();
  }
  if (!std::isfinite(rr)) throw Error{DWF_ERR_NAN, "non-finite residual at CG start"};
  if (rr <= target) return 0;

  // inner vectors
  Half<Pi> r = hview<Pi>(MIXED ? ws_get(ctx, tag + ".r." + pname(Pi::ID), hbi) : (void*)rhi.data, g, Ls);
  if (!MIXED) r = hview<Pi>((void*)rhi.data, g, Ls);
  Half<Pi> q = hview<Pi>(ws_get(ctx, tag + ".q." + pname(Pi::ID), hbi), g, Ls);
  Half<Pi> te = hview<Pi>(ws_get(ctx, tag + ".te." + pname(Pi::ID), hbi), g, Ls);
  Half<Pi> to = hview<Pi>(ws_get(ctx, tag + ".to." + pname(Pi::ID), hbi), g, Ls);
  Half<PX> xl = hview<PX>(MIXED ? ws_get(ctx, tag + ".xlo", half_size<PX>(g, Ls)) : (void*)x.data, g, Ls);
  if (MIXED) {
    DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(cv(rhi), r, n5, Ls, s)));
    DWF_CHECK_LAUNCH(launch_zero(xl.data, half_size<PX>(g, Ls), s));
  }
  // The search directions rotate through a ring of KX buffers and the solution increment
  // xl += alpha_k p_k is applied KX iterations at a time (one pass that reads the KX
  // directions and xl once, instead of xl read and written in every iteration), and before
  // every reliable update and at the end.  The alphas wait in the scalar history slots.
  constexpr int KX = 8;
  static_assert(KX >= 2 && KX <= XFLUSH_MAX, "direction ring");
  Half<Pi> pr[KX];
  for (int j = 0; j < KX; ++j) pr[j] = hview<Pi>(ws_get(ctx, tag + ".p" + std::to_string(j) + "." + pname(Pi::ID), hbi), g, Ls);
  int cur = 0;  // ring index of the current direction
  XFlush<Pi> pend;
  auto flush = [&]() {
    DWF_CHECK_LAUNCH((launch_xflush<Pi, PX>(xl, pend, sc, n5, Ls, s)));
    pend.n = 0;
  };
  // Moebius operators: the p update also forms F p, and M p runs without the input factor in
  // its hops
  const bool PRE = opi.moebius;
  Half<Pi> fp = PRE ? hview<Pi>(ws_get(ctx, tag + ".fp." + pname(Pi::ID), hbi), g, Ls) : Half<Pi>{nullptr, nullptr};
  // the new direction goes to the next ring slot: never a pending one, since at most KX - 1
  // are pending here, the last of them the current one
  auto p_update = [&](double beta, double rr_new) {
    const int nxt = (cur + 1) % KX;
    if (PRE) {
      DWF_CHECK_LAUNCH(launch_cg_pupdate_f<Pi>(cv(r), cv(pr[cur]), pr[nxt], fp, beta, sc, rr_new, n5, Ls, opi.b, opi.c,
                                               opi.m, s, opi.sdep ? opi.coef_b : nullptr,
                                               opi.sdep ? opi.coef_c : nullptr));
    } else {
      DWF_CHECK_LAUNCH(launch_cg_pupdate<Pi>(cv(r), cv(pr[cur]), pr[nxt], beta, sc, rr_new, n5, Ls, s));
    }
    cur = nxt;
  };
  // p = r
  p_update(0.0, rr);
  double rr_max = rr, rr_true = rr;
  const bool OUT2 = opi.second_output_ok();
  const long nb_hop = (g->nsites + opi.cfg.spb - 1) / opi.cfg.spb;
  int it = 0;
  while (it < maxit) {
    const Half<Pi> p = pr[cur];
    // q = M p, |q|^2 -> alpha = rr / |q|^2 (also kept in the history slot of this direction)
    // (with A^-dag q, the first step of M^dag q, as a second output of the last hop)
    const Half<Pi> q2 = OUT2 ? to : Half<Pi>{nullptr, nullptr};
    if (PRE) opi.mprec_pre(cv(fp), cv(p), q, te, part, q2);
    else opi.mprec(cv(p), q, te, part, q2);
    DWF_CHECK_LAUNCH(launch_reduce(part, int(nb_hop), 1, sc, S_QQ, 1, s, pend.n));
    pend.p[pend.n] = cv(p);
    pend.slot[pend.n] = pend.n;
    ++pend.n;
    // r -= alpha M^dag q and |r|^2, fused into the last hop of M^dag q
    opi.mprec_dag_cg(cv(q), to, te, r, sc, part, OUT2);
    DWF_CHECK_LAUNCH(launch_reduce(part, int(nb_hop), 1, sc, S_RRNEW, 0, s));
    if (pend.n == KX) flush();
    double rr_new = read_scalar(ctx, sc, S_RRNEW);
    ++it;
    if (!std::isfinite(rr_new)) throw Error{DWF_ERR_NAN, "non-finite residual in CG iteration"};
    // reliable update when the iterated residual has dropped by delta since the last one,
    // when it claims convergence, or when it has grown 100x above the last true residual
    // (a diverging low-precision recurrence)
    const bool diverging = rr_new > 1e4 * rr_true;
    if (MIXED && (rr_new < delta * delta * rr_max || rr_new <= target || diverging)) {
      // reliable update: fold the FP32 increment into the FP64 solution, recompute r in FP64
      flush();
      DWF_CHECK_LAUNCH(launch_accumulate<PX>(x, xl, n5, Ls, s));
      rr_new = true_residual();
      DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(cv(rhi), r, n5, Ls, s)));
      rr_max = rr_new;
      rr_true = rr_new;
      st->reliable_updates++;
      if (rr_new > target && (RESTART || diverging)) {
        // BF16 (8-bit mantissa): the retained direction loses conjugacy and CG stagnates;
        // restart the Krylov space from the recomputed residual.
        p_update(0.0, rr_new);
        rr = rr_new;
        continue;
      }
    }
    if (rr_new <= target) {
      rr = rr_new;
      break;
    }
    const double beta = rr_new / rr;
    p_update(beta, rr_new);
    rr = rr_new;
    if (rr > rr_max) rr_max = rr;
  }
  flush();
  if (MIXED) DWF_CHECK_LAUNCH(launch_accumulate<PX>(x, xl, n5, Ls, s));
  st->iters += it;
  st->last_rel = std::sqrt(rr / rhs2);
  return rr <= target ? 0 : 1;
}

template <typename Pi>
static int cg_normal_dispatch(dwf_ctx* ctx, const Op<P64>& op64, const dwf_params& p, const void* U64,
                              CHalf<P64> rhs, Half<P64> x, double tol_n, int maxit, double delta,
                              const std::string& tag, SolveStats* st) {
  const void* Ui = links_in(ctx, op64.g, U64, Pi::ID, tag);
  Op<Pi> opi(ctx, op64.g, p, Ui);
  return cg_normal<Pi>(ctx, op64, opi, rhs, x, tol_n, maxit, delta, tag, st);
}

int normal_solve(dwf_ctx* ctx, const dwf_params& p, const void* U64, CHalf<P64> rhs, Half<P64> x, double tol_n,
                 int maxit, double delta, const std::string& tag, SolveStats* st) {
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  Op<P64> op64(ctx, g, p, U64);
  switch (p.prec_inner) {
    case DWF_FP64: return cg_normal_dispatch<P64>(ctx, op64, p, U64, rhs, x, tol_n, maxit, delta, tag, st);
    case DWF_FP32: return cg_normal_dispatch<P32>(ctx, op64, p, U64, rhs, x, tol_n, maxit, delta, tag, st);
    case DWF_FP16: return cg_normal_dispatch<P16>(ctx, op64, p, U64, rhs, x, tol_n, maxit, delta, tag, st);
    default: return cg_normal_dispatch<PB16>(ctx, op64, p, U64, rhs, x, tol_n, maxit, delta, tag, st);
  }
}

// ------------------------------------------------------------------ full-system solve
// D(m) x = b through the Schur complement on odd sites:
//   b'_o = A^-1 (b_o - B_oe A^-1 b_e),  M x_o = b'_o  (CGNR),  x_e = A^-1 (b_e - B_eo x_o),
// tightening the normal-equation tolerance until ||b - D x|| / ||b|| <= tol.
int solve_full(dwf_ctx* ctx, const dwf_params& p, const void* U64, const void* b, void* x, double tol, int maxit,
               double delta, const std::string& tag, dwf_solve_info* info) {
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const long n5 = g->nsites * Ls;
  const size_t hb = half_size<P64>(g, Ls);
  hipStream_t s = ctx->stream;
  Op<P64> op(ctx, g, p, U64);
  CHalf<P64> be = chalf_at<P64>(b, 0, g, Ls), bo = chalf_at<P64>(b, hb, g, Ls);
  Half<P64> xe = half_at<P64>(x, 0, g, Ls), xo = half_at<P64>(x, hb, g, Ls);
  Half<P64> te = hview<P64>(ws_get(ctx, tag + ".se", hb), g, Ls);
  Half<P64> to = hview<P64>(ws_get(ctx, tag + ".so", hb), g, Ls);
  Half<P64> bp = hview<P64>(ws_get(ctx, tag + ".bp", hb), g, Ls);
  Half<P64> rhs = hview<P64>(ws_get(ctx, tag + ".rhs", hb), g, Ls);
  Half<P64> t2 = hview<P64>(ws_get(ctx, tag + ".t2", hb), g, Ls);
  void* rfull = ws_get(ctx, tag + ".rfull", 2 * hb);
  Half<P64> re = half_at<P64>(rfull, 0, g, Ls), ro = half_at<P64>(rfull, hb, g, Ls);

  const double b2 = norm2_sync<P64>(ctx, be, g, Ls) + norm2_sync<P64>(ctx, bo, g, Ls);
  if (!std::isfinite(b2)) throw Error{DWF_ERR_NAN, "non-finite source"};
  SolveStats st;
  int status = 0;
  double rel = 0.0;
  if (b2 == 0.0) {
    DWF_CHECK_LAUNCH(launch_zero(x, 2 * hb, s));
  } else {
    // source preparation
    op.fifth(be, te, E_AINV);                                  // A^-1 b_e
    op.hop(1, cv(te), to, false, true, 0.5, nullptr, bo, 1.0);  // b_o - B_oe A^-1 b_e
    op.fifth(cv(to), bp, E_AINV);                              // b'_o
    op.mprec_dag(cv(bp), rhs, te, t2);                         // M^dag b'
    double tol_n = tol;
    status = 1;
    for (int attempt = 0; attempt < 12; ++attempt) {
      const int left = maxit - st.iters;
      if (left <= 0) break;
      normal_solve(ctx, p, U64, cv(rhs), xo, tol_n, left, delta, tag + ".cg", &st);
      // x_e = A^-1 (b_e - B_eo x_o)
      op.hop(0, cv(xo), te, false, true, 0.5, nullptr, be, 1.0);
      op.fifth(cv(te), xe, E_AINV);
      // true residual of the full system
      op.full(cv(xe), cv(xo), re, ro, false);
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, be, -1.0, re, n5, Ls, s));
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, bo, -1.0, ro, n5, Ls, s));
      const double r2 = norm2_sync<P64>(ctx, cv(re), g, Ls) + norm2_sync<P64>(ctx, cv(ro), g, Ls);
      rel = std::sqrt(r2 / b2);
      if (!std::isfinite(rel)) throw Error{DWF_ERR_NAN, "non-finite true residual"};
      if (rel <= tol) {
        status = 0;
        break;
      }
      tol_n *= std::max(0.02, std::min(0.5, 0.5 * tol / rel));
      st.restarts++;
    }
  }
  DWF_CHECK_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = st.iters;
    info->reliable_updates = st.reliable_updates;
    info->restarts = st.restarts;
    info->true_rel_resid = rel;
    info->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    info->wilson_apps = (long long)st.iters * Ls;
  }
  return status;
}

// ------------------------------------------------------------------ batched CG
// Several right-hand sides (the Hasenbusch mass ladder of Sec. 3; possibly on different
// lattices) iterate together: every hop stage of M_prec and M_prec^dag is one launch over all
// unconverged right-hand sides (links staged once per workgroup for all right-hand sides of a
// lattice), and one device-to-host copy per iteration returns every residual norm.  The
// per-RHS logic (FP64 scalars, reliable updates, convergence) is that of cg_normal.
struct BatchSys {
  dwf_params p;
  const Geometry* g;
  const void* U64;
  const void* Ui;
  std::unique_ptr<Op<P64>> op64;
  CHalf<P64> rhs;
  Half<P64> x;
  double rhs2 = 0, target = 0, rr = 0, rr_max = 0, rr_true = 0, tol_n = 0;
  int cap = 0;  // iterations this system may still run
  bool active = false;
  SolveStats st;
  // inner vectors (storage precision of the solve)
  void *r = nullptr, *pv = nullptr, *q = nullptr, *Ap = nullptr, *te = nullptr, *xl = nullptr;
  const void* E = nullptr;  // fifth-dimension matrices of this mass
  int group = -1;
};

template <typename Pi>
static void cg_batched(dwf_ctx* ctx, std::vector<BatchSys>& S, int maxit, double delta) {
  constexpr bool MIXED = !std::is_same<Pi, P64>::value;
  using PX = typename std::conditional<MIXED, P32, P64>::type;
  using R = typename Pi::R;
  constexpr bool RESTART = std::is_same<Pi, PB16>::value;
  hipStream_t s = ctx->stream;
  const int K = int(S.size());
  // partial sums and scalars: one stride per right-hand side
  long pstride = 1024;
  for (auto& b : S) pstride = std::max(pstride, b.g->nsites);
  double* part = reinterpret_cast<double*>(ws_get(ctx, "batch.partials", size_t(K) * pstride * sizeof(double)));
  double* sc = reinterpret_cast<double*>(ws_get(ctx, "batch.scalars", size_t(K) * S_COUNT * sizeof(double)));
  std::vector<double> hsc(size_t(K) * S_COUNT);
  // FP64 temporaries shared by the reliable updates (largest system)
  size_t hb64max = 0;
  for (auto& b : S) hb64max = std::max(hb64max, half_size<P64>(b.g, b.p.Ls));
  void* rhi_raw = ws_get(ctx, "batch.rhi", hb64max);
  void* t64a_raw = ws_get(ctx, "batch.t64a", hb64max);
  void* t64b_raw = ws_get(ctx, "batch.t64b", hb64max);
  void* t64c_raw = ws_get(ctx, "batch.t64c", hb64max);
  auto true_residual = [&](BatchSys& b) -> double {
    const int Ls = b.p.Ls;
    Half<P64> rhi = hview<P64>(rhi_raw, b.g, Ls), ta = hview<P64>(t64a_raw, b.g, Ls), tb = hview<P64>(t64b_raw, b.g, Ls),
              tc = hview<P64>(t64c_raw, b.g, Ls);
    b.op64->mprec(cv(b.x), ta, tb);
    b.op64->mprec_dag(cv(ta), rhi, tb, tc);
    DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, b.rhs, -1.0, rhi, b.g->nsites * Ls, Ls, s));
    return norm2_sync<P64>(ctx, cv(rhi), b.g, Ls);
  };
  // inner vectors and start
  for (int k = 0; k < K; ++k) {
    BatchSys& b = S[k];
    const int Ls = b.p.Ls;
    const long n5 = b.g->nsites * Ls;
    const size_t hbi = half_size<Pi>(b.g, Ls);
    const std::string t = "batch." + std::to_string(k) + ".";
    b.r = ws_get(ctx, t + "r", hbi);
    b.pv = ws_get(ctx, t + "p", hbi);
    b.q = ws_get(ctx, t + "q", hbi);
    b.Ap = ws_get(ctx, t + "Ap", hbi);
    b.te = ws_get(ctx, t + "te", hbi);
    b.xl = MIXED ? ws_get(ctx, t + "xlo", half_size<PX>(b.g, Ls)) : (void*)b.x.data;
    b.E = fifth_matrices(ctx, Ls, b.p.M5, b.p.mass, b.p.b, b.p.c, Pi::ID);
    b.rhs2 = norm2_sync<P64>(ctx, b.rhs, b.g, Ls);
    b.target = b.tol_n * b.tol_n * b.rhs2;
    b.active = b.rhs2 > 0.0;
    if (!b.active) {
      DWF_CHECK_LAUNCH(launch_zero(b.x.data, half_size<P64>(b.g, Ls), s));
      continue;
    }
    b.rr = true_residual(b);
    if (!std::isfinite(b.rr)) throw Error{DWF_ERR_NAN, "non-finite residual at batched CG start"};
    b.rr_max = b.rr_true = b.rr;
    if (b.rr <= b.target || b.cap <= 0) { b.active = false; continue; }
    Half<P64> rhi = hview<P64>(rhi_raw, b.g, Ls);
    Half<Pi> r = hview<Pi>(b.r, b.g, Ls);
    DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(cv(rhi), r, n5, Ls, s)));
    if (MIXED) DWF_CHECK_LAUNCH(launch_zero(b.xl, half_size<PX>(b.g, Ls), s));
    DWF_CHECK_LAUNCH(launch_axpby<Pi>(1.0, cv(r), 0.0, hview<Pi>(b.pv, b.g, Ls), n5, Ls, s));
    DWF_CHECK_LAUNCH(launch_set_scalar(sc + k * S_COUNT, S_RR, b.rr, s));
  }
  // descriptor tables of the four hop stages, rebuilt when the active set changes
  std::vector<MultiGroup<Pi>> hg[4];
  std::vector<MultiRhs<Pi>> hr[4];
  MultiGroup<Pi>* dg[4];
  MultiRhs<Pi>* dr[4];
  for (int st = 0; st < 4; ++st) {
    dg[st] = reinterpret_cast<MultiGroup<Pi>*>(ws_get(ctx, "batch.dg" + std::to_string(st), sizeof(MultiGroup<Pi>) * K));
    dr[st] = reinterpret_cast<MultiRhs<Pi>*>(ws_get(ctx, "batch.dr" + std::to_string(st), sizeof(MultiRhs<Pi>) * K));
  }
  const bool moebius = !(S[0].p.b == 1.0 && S[0].p.c == 0.0);
  std::vector<int> hop_blocks(K, 0);
  bool scan_st[4] = {false, false, false, false};  // every right-hand side of the stage has its scan form
  // the epilogue of slot `slot` of system b in recurrence form
  auto scan_of = [&](const BatchSys& b, int slot, FifthScan<R>& out) -> bool {
    FifthScan<double> e;
    if (!fifth_scan(b.p.Ls, b.p.M5, b.p.mass, b.p.b, b.p.c, slot, &e)) return false;
    out.m = R(e.m);
    for (int ch = 0; ch < 2; ++ch) {
      const FifthChir<double>& q = e.ch[ch];
      out.ch[ch] = FifthChir<R>{R(q.a1), R(q.b1), R(q.inv_alpha), R(q.a), R(q.corr), q.d1, q.d2, q.has_inv};
    }
    return true;
  };
  auto build_tables = [&]() {
    // group active systems by (lattice, links): consecutive entries of one group share links
    std::vector<int> order_k;
    std::vector<std::pair<const Geometry*, const void*>> keys;
    std::vector<std::vector<int>> members;
    for (int k = 0; k < K; ++k) {
      if (!S[k].active) continue;
      int gi = -1;
      for (size_t j = 0; j < keys.size(); ++j)
        if (keys[j].first == S[k].g && keys[j].second == S[k].Ui && S[members[j][0]].p.Ls == S[k].p.Ls) gi = int(j);
      if (gi < 0) { keys.push_back({S[k].g, S[k].Ui}); members.push_back({}); gi = int(keys.size()) - 1; }
      members[gi].push_back(k);
    }
    for (int st = 0; st < 4; ++st) {
      hg[st].clear();
      hr[st].clear();
      scan_st[st] = true;
      const int out_par = (st == 0 || st == 2) ? 0 : 1;
      long blocks = 0;
      for (size_t j = 0; j < keys.size(); ++j) {
        const BatchSys& b0 = S[members[j][0]];
        const int Ls = b0.p.Ls;
        MultiGroup<Pi> G;
        G.links = reinterpret_cast<const typename Pi::S*>(b0.Ui) + (out_par ? size_t(b0.g->nsites) * 72 : 0);
        G.nbr = b0.g->d_nbr[out_par];
        G.order = b0.g->d_order[out_par];
        G.nsites = b0.g->nsites;
        G.Ls = Ls;
        int spb = std::max(1, 256 / Ls);
        while (spb > 1 && multi_lds_bytes<Pi>(spb, Ls, true) > 65536) --spb;
        G.spb = spb;
        G.block_begin = blocks;
        G.rhs_begin = int(hr[st].size());
        G.nrhs = int(members[j].size());
        blocks += (G.nsites + spb - 1) / spb;
        hg[st].push_back(G);
        for (int k : members[j]) {
          BatchSys& b = S[k];
          hop_blocks[k] = int((G.nsites + spb - 1) / spb);
          const R* E = reinterpret_cast<const R*>(b.E);
          const size_t ls2 = size_t(Ls) * Ls;
          MultiRhs<Pi> Q;
          Q.pb = R(b.p.b);
          Q.pc = R(b.p.c);
          Q.pm = R(b.p.mass);
          Q.ax = R(0);
          Q.x = {nullptr, nullptr};
          Q.norm_partials = nullptr;
          if (st == 0) {  // te = A^-1 H_eo F p
            Q.in = chview<Pi>(b.pv, b.g, Ls); Q.out = hview<Pi>(b.te, b.g, Ls);
            Q.E = E + size_t(E_AINV) * 2 * ls2; Q.scale = R(1);
          } else if (st == 1) {  // q = p - 1/4 A^-1 H_oe F te, |q|^2
            Q.in = chview<Pi>(b.te, b.g, Ls); Q.out = hview<Pi>(b.q, b.g, Ls);
            Q.E = E + size_t(E_AINV) * 2 * ls2; Q.scale = R(-0.25);
            Q.x = chview<Pi>(b.pv, b.g, Ls); Q.ax = R(1);
            Q.norm_partials = part + size_t(k) * pstride;
          } else if (st == 2) {  // te = A^-dag F^dag H^dag_eo (A^-dag q)   [A^-dag q is in Ap]
            Q.in = chview<Pi>(b.Ap, b.g, Ls); Q.out = hview<Pi>(b.te, b.g, Ls);
            Q.E = E + size_t(E_AINVDAG_FDAG) * 2 * ls2; Q.scale = R(1);
          } else {  // r -= alpha (q - 1/4 F^dag H^dag_oe te), |r|^2   (M^dag q not stored)
            Q.in = chview<Pi>(b.te, b.g, Ls); Q.out = hview<Pi>(b.Ap, b.g, Ls);
            Q.E = moebius ? E + size_t(E_FDAG) * 2 * ls2 : nullptr; Q.scale = R(-0.25);
            Q.x = chview<Pi>(b.q, b.g, Ls); Q.ax = R(1);
            Q.cg_r = hview<Pi>(b.r, b.g, Ls);
            Q.cg_sc = sc + size_t(k) * S_COUNT;
            Q.norm_partials = part + size_t(k) * pstride;
          }
          if (Q.E) {
            const int slot = int((Q.E - E) / (2 * ls2));
            Q.scan = scan_of(b, slot, Q.es) ? 1 : 0;
            if (!Q.scan) scan_st[st] = false;
          }
          hr[st].push_back(Q);
        }
      }
      if (!hg[st].empty()) {
        DWF_CHECK_HIP(hipMemcpy(dg[st], hg[st].data(), sizeof(MultiGroup<Pi>) * hg[st].size(), hipMemcpyHostToDevice));
        DWF_CHECK_HIP(hipMemcpy(dr[st], hr[st].data(), sizeof(MultiRhs<Pi>) * hr[st].size(), hipMemcpyHostToDevice));
      }
    }
  };
  int nactive = 0;
  for (auto& b : S) nactive += b.active ? 1 : 0;
  if (nactive) build_tables();
  int it = 0;
  while (nactive > 0 && it < maxit) {
    // q = M p (one launch per stage for all right-hand sides), alpha = rr / |q|^2
    DWF_CHECK_LAUNCH(launch_hop_multi<Pi>(dg[0], hg[0], dr[0], false, moebius, true, s, scan_st[0]));
    DWF_CHECK_LAUNCH(launch_hop_multi<Pi>(dg[1], hg[1], dr[1], false, moebius, true, s, scan_st[1]));
    for (int k = 0; k < K; ++k) {
      if (!S[k].active) continue;
      BatchSys& b = S[k];
      DWF_CHECK_LAUNCH(launch_reduce(part + size_t(k) * pstride, hop_blocks[k], 1, sc + k * S_COUNT, S_QQ, 1, s, 0));
      // A^-dag q into Ap (consumed by the next stage before Ap is overwritten)
      DWF_CHECK_LAUNCH(launch_fifth<Pi>(chview<Pi>(b.q, b.g, b.p.Ls), hview<Pi>(b.Ap, b.g, b.p.Ls),
                                        reinterpret_cast<const R*>(b.E) + size_t(E_AINVDAG) * 2 * b.p.Ls * b.p.Ls,
                                        nullptr, CHalf<Pi>{nullptr, nullptr}, R(0), b.g->nsites, b.p.Ls, nullptr, s));
    }
    DWF_CHECK_LAUNCH(launch_hop_multi<Pi>(dg[2], hg[2], dr[2], true, false, true, s, scan_st[2]));
    DWF_CHECK_LAUNCH(launch_hop_multi<Pi>(dg[3], hg[3], dr[3], true, false, moebius, s, scan_st[3]));
    for (int k = 0; k < K; ++k) {
      if (!S[k].active) continue;
      BatchSys& b = S[k];
      const int Ls = b.p.Ls;
      const long n5 = b.g->nsites * Ls;
      // |r|^2 from the partials of the last stage; xl += alpha p (alpha kept in history slot 0)
      DWF_CHECK_LAUNCH(launch_reduce(part + size_t(k) * pstride, hop_blocks[k], 1, sc + k * S_COUNT, S_RRNEW, 0, s));
      XFlush<Pi> f;
      f.p[0] = chview<Pi>(b.pv, b.g, Ls);
      f.slot[0] = 0;
      f.n = 1;
      DWF_CHECK_LAUNCH((launch_xflush<Pi, PX>(hview<PX>(b.xl, b.g, Ls), f, sc + k * S_COUNT, n5, Ls, s)));
    }
    DWF_CHECK_HIP(hipMemcpyAsync(hsc.data(), sc, sizeof(double) * hsc.size(), hipMemcpyDeviceToHost, s));
    DWF_CHECK_HIP(hipStreamSynchronize(s));
    ++it;
    bool changed = false;
    for (int k = 0; k < K; ++k) {
      BatchSys& b = S[k];
      if (!b.active) continue;
      const int Ls = b.p.Ls;
      const long n5 = b.g->nsites * Ls;
      b.st.iters++;
      double rr_new = hsc[size_t(k) * S_COUNT + S_RRNEW];
      if (!std::isfinite(rr_new)) throw Error{DWF_ERR_NAN, "non-finite residual in batched CG"};
      const bool diverging = rr_new > 1e4 * b.rr_true;
      bool restart = false;
      if (MIXED && (rr_new < delta * delta * b.rr_max || rr_new <= b.target || diverging)) {
        DWF_CHECK_LAUNCH(launch_accumulate<PX>(b.x, hview<PX>(b.xl, b.g, Ls), n5, Ls, s));
        rr_new = true_residual(b);
        DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(chview<P64>(rhi_raw, b.g, Ls), hview<Pi>(b.r, b.g, Ls), n5, Ls, s)));
        b.rr_max = b.rr_true = rr_new;
        b.st.reliable_updates++;
        restart = rr_new > b.target && (RESTART || diverging);
      }
      if (rr_new <= b.target) {
        b.rr = rr_new;
        b.active = false;
        changed = true;
        continue;
      }
      if (b.st.iters >= b.cap) {  // out of iterations: stop with the current iterate
        b.rr = rr_new;
        b.active = false;
        changed = true;
        continue;
      }
      const double beta = restart ? 0.0 : rr_new / b.rr;
      DWF_CHECK_LAUNCH(launch_cg_pupdate<Pi>(chview<Pi>(b.r, b.g, Ls), chview<Pi>(b.pv, b.g, Ls),
                                             hview<Pi>(b.pv, b.g, Ls), beta, sc + k * S_COUNT, rr_new, n5, Ls, s));
      b.rr = rr_new;
      if (b.rr > b.rr_max) b.rr_max = b.rr;
    }
    nactive = 0;
    for (auto& b : S) nactive += b.active ? 1 : 0;
    if (changed && nactive) build_tables();
  }
  for (auto& b : S) {
    if (MIXED && b.rhs2 > 0.0)
      DWF_CHECK_LAUNCH(launch_accumulate<PX>(b.x, hview<PX>(b.xl, b.g, b.p.Ls), b.g->nsites * b.p.Ls, b.p.Ls, s));
    b.st.last_rel = b.rhs2 > 0 ? std::sqrt(b.rr / b.rhs2) : 0.0;
  }
}

// Full-system batched solve: per-RHS even-odd source preparation, the batched CG on the
// normal equations, per-RHS reconstruction and true residual, tightening the normal-equation
// tolerance of the right-hand sides that have not reached tol.
int solve_batched(dwf_ctx* ctx, int nrhs, const dwf_params* P, const void* const* U64, const void* const* b,
                  void* const* x, dwf_solve_info* info) {
  const auto t0 = Clock::now();
  hipStream_t s = ctx->stream;
  std::vector<BatchSys> S(nrhs);
  std::vector<double> b2(nrhs, 0.0), rel(nrhs, 1.0);
  std::vector<int> done(nrhs, 0);
  for (int k = 0; k < nrhs; ++k) {
    BatchSys& B = S[k];
    B.p = P[k];
    B.g = geometry(ctx, P[k].dims, P[k].tbc);
    B.U64 = U64[k];
    B.op64 = std::make_unique<Op<P64>>(ctx, B.g, P[k], U64[k]);
    const int Ls = P[k].Ls;
    const size_t hb = half_size<P64>(B.g, Ls);
    const long n5 = B.g->nsites * Ls;
    const std::string t = "batchfull." + std::to_string(k) + ".";
    CHalf<P64> be = chview<P64>(b[k], B.g, Ls), bo = chview<P64>(reinterpret_cast<const char*>(b[k]) + hb, B.g, Ls);
    Half<P64> te = hview<P64>(ws_get(ctx, "batchfull.se", hb), B.g, Ls);
    Half<P64> to = hview<P64>(ws_get(ctx, "batchfull.so", hb), B.g, Ls);
    Half<P64> bp = hview<P64>(ws_get(ctx, "batchfull.bp", hb), B.g, Ls);
    Half<P64> t2 = hview<P64>(ws_get(ctx, "batchfull.t2", hb), B.g, Ls);
    Half<P64> rhs = hview<P64>(ws_get(ctx, t + "rhs", hb), B.g, Ls);
    b2[k] = norm2_sync<P64>(ctx, be, B.g, Ls) + norm2_sync<P64>(ctx, bo, B.g, Ls);
    if (!std::isfinite(b2[k])) throw Error{DWF_ERR_NAN, "non-finite source"};
    B.op64->fifth(be, te, E_AINV);
    B.op64->hop(1, cv(te), to, false, true, 0.5, nullptr, bo, 1.0);
    B.op64->fifth(cv(to), bp, E_AINV);
    B.op64->mprec_dag(cv(bp), rhs, te, t2);
    (void)n5;
    B.rhs = cv(rhs);
    B.x = hview<P64>(reinterpret_cast<char*>(x[k]) + hb, B.g, Ls);
    B.tol_n = info[k].tol;
    if (b2[k] == 0.0) { DWF_CHECK_LAUNCH(launch_zero(x[k], 2 * hb, s)); done[k] = 1; rel[k] = 0.0; }
  }
  // links in the inner precision, converted once per distinct link field
  const int prec = P[0].prec_inner;
  std::map<const void*, const void*> conv;
  for (int k = 0; k < nrhs; ++k) {
    if (!conv.count(U64[k])) conv[U64[k]] = links_in(ctx, S[k].g, U64[k], prec, "batchU." + std::to_string(conv.size()));
    S[k].Ui = conv[U64[k]];
  }
  const double delta = info[0].delta > 0 ? info[0].delta : 0.1;
  int maxit = info[0].maxit > 0 ? info[0].maxit : 100000;
  int status = 0;
  for (int attempt = 0; attempt < 12; ++attempt) {
    std::vector<int> idx;
    for (int k = 0; k < nrhs; ++k) {
      if (!done[k] && S[k].st.iters >= maxit) done[k] = 2;  // the cap counts every attempt's iterations
      if (!done[k]) idx.push_back(k);
    }
    if (idx.empty()) break;
    std::vector<BatchSys> run;
    run.reserve(idx.size());
    for (int k : idx) {
      BatchSys c;
      c.p = S[k].p; c.g = S[k].g; c.U64 = S[k].U64; c.Ui = S[k].Ui;
      c.op64 = std::make_unique<Op<P64>>(ctx, S[k].g, S[k].p, S[k].U64);
      c.rhs = S[k].rhs; c.x = S[k].x; c.tol_n = S[k].tol_n;
      c.cap = maxit - S[k].st.iters;
      run.push_back(std::move(c));
    }
    switch (prec) {
      case DWF_FP64: cg_batched<P64>(ctx, run, maxit, delta); break;
      case DWF_FP32: cg_batched<P32>(ctx, run, maxit, delta); break;
      case DWF_FP16: cg_batched<P16>(ctx, run, maxit, delta); break;
      default: cg_batched<PB16>(ctx, run, maxit, delta); break;
    }
    int left = 0;
    for (size_t j = 0; j < idx.size(); ++j) {
      const int k = idx[j];
      BatchSys& B = S[k];
      B.st.iters += run[j].st.iters;
      B.st.reliable_updates += run[j].st.reliable_updates;
      const int Ls = B.p.Ls;
      const size_t hb = half_size<P64>(B.g, Ls);
      const long n5 = B.g->nsites * Ls;
      CHalf<P64> be = chview<P64>(b[k], B.g, Ls), bo = chview<P64>(reinterpret_cast<const char*>(b[k]) + hb, B.g, Ls);
      Half<P64> xe = hview<P64>(x[k], B.g, Ls);
      Half<P64> te = hview<P64>(ws_get(ctx, "batchfull.se", hb), B.g, Ls);
      void* rf = ws_get(ctx, "batchfull.rfull", 2 * hb);
      Half<P64> re = hview<P64>(rf, B.g, Ls), ro = hview<P64>(reinterpret_cast<char*>(rf) + hb, B.g, Ls);
      B.op64->hop(0, cv(B.x), te, false, true, 0.5, nullptr, be, 1.0);
      B.op64->fifth(cv(te), xe, E_AINV);
      B.op64->full(cv(xe), cv(B.x), re, ro, false);
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, be, -1.0, re, n5, Ls, s));
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, bo, -1.0, ro, n5, Ls, s));
      const double r2 = norm2_sync<P64>(ctx, cv(re), B.g, Ls) + norm2_sync<P64>(ctx, cv(ro), B.g, Ls);
      rel[k] = std::sqrt(r2 / b2[k]);
      if (!std::isfinite(rel[k])) throw Error{DWF_ERR_NAN, "non-finite true residual"};
      if (rel[k] <= info[k].tol) {
        done[k] = 1;
      } else {
        B.tol_n *= std::max(0.02, std::min(0.5, 0.5 * info[k].tol / rel[k]));
        B.st.restarts++;
        ++left;
      }
      if (B.st.iters >= maxit && !done[k]) done[k] = 2;
    }
    if (left == 0) break;
  }
  DWF_CHECK_HIP(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(Clock::now() - t0).count();
  for (int k = 0; k < nrhs; ++k) {
    info[k].iters = S[k].st.iters;
    info[k].reliable_updates = S[k].st.reliable_updates;
    info[k].restarts = S[k].st.restarts;
    info[k].true_rel_resid = rel[k];
    info[k].seconds = secs;
    info[k].wilson_apps = (long long)S[k].st.iters * S[k].p.Ls;
    if (done[k] != 1) status = 1;
  }
  return status;
}

// ------------------------------------------------------------------ MADWF
// Sec. 4 algorithm with Sec. 5 defect correction.  target: Shamir DWF D(m), Ls = L;
// inner: Moebius D'(m), Ls = L'.  Per step k:
//   r = b - D(m) x;  c = P^-1 D(1)^-1 r;  z = D'(m)^-1 D'(1) P' (c_1, 0, .., 0);
//   y'_1 = (P'^-1 z)_1;  w = P^-1 D(1)^-1 D(m) P (-y'_1, c_2, .., c_L);  w_1 = y'_1;  x += P w.
// then a warm-started DWF solve to the final tolerance.
int madwf(dwf_ctx* ctx, const dwf_params& pt, const dwf_params& pi, const void* U64, const void* b, void* x,
          dwf_madwf_info* info) {
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, pt.dims, pt.tbc);
  const int L = pt.Ls, Lp = pi.Ls;
  const size_t hb = half_size<P64>(g, L), hbp = half_size<P64>(g, Lp);
  const long ns = g->nsites;
  hipStream_t s = ctx->stream;
  const double delta = info->delta > 0 ? info->delta : 0.1;
  const int maxit = info->maxit > 0 ? info->maxit : 100000;
  dwf_params ppv = pt;
  ppv.mass = 1.0;
  ppv.prec_inner = info->prec_pv;
  dwf_params pipv = pi;
  pipv.mass = 1.0;
  Op<P64> opt(ctx, g, pt, U64);
  Op<P64> opi1(ctx, g, pipv, U64);
  void* r = ws_get(ctx, "madwf.r", 2 * hb);
  void* c = ws_get(ctx, "madwf.c", 2 * hb);
  void* t = ws_get(ctx, "madwf.t", 2 * hb);
  void* w = ws_get(ctx, "madwf.w", 2 * hb);
  void* cp = ws_get(ctx, "madwf.cp", 2 * hbp);
  void* zp = ws_get(ctx, "madwf.zp", 2 * hbp);
  void* yp = ws_get(ctx, "madwf.yp", 2 * hbp);
  void* rp = ws_get(ctx, "madwf.rp", 2 * hbp);
  auto H = [&](void* base, int par, int Lx, size_t hbx) { return half_at<P64>(base, par ? hbx : 0, g, Lx); };
  auto CH = [&](const void* base, int par, int Lx, size_t hbx) { return chalf_at<P64>(base, par ? hbx : 0, g, Lx); };
  auto pshift = [&](const void* in, void* out, int inverse, int Lx, size_t hbx) {
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_pshift(CH(in, par, Lx, hbx), H(out, par, Lx, hbx), inverse, ns, Lx, s));
  };
  auto residual = [&](void* out) -> double {  // out = b - D(m) x, returns |out|^2
    opt.full(CH(x, 0, L, hb), CH(x, 1, L, hb), H(out, 0, L, hb), H(out, 1, L, hb), false);
    double r2 = 0.0;
    for (int par = 0; par < 2; ++par) {
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, CH(b, par, L, hb), -1.0, H(out, par, L, hb), ns * L, L, s));
      r2 += norm2_sync<P64>(ctx, CH(out, par, L, hb), g, L);
    }
    return r2;
  };
  double b2 = 0.0;
  for (int par = 0; par < 2; ++par) b2 += norm2_sync<P64>(ctx, CH(b, par, L, hb), g, L);
  if (!std::isfinite(b2)) throw Error{DWF_ERR_NAN, "non-finite source"};
  DWF_CHECK_LAUNCH(launch_zero(x, 2 * hb, s));
  info->pv_iters = info->mobius_iters = info->final_iters = info->n_pv = info->n_mobius = 0;
  info->seconds_pv = info->seconds_mobius = info->seconds_final = 0.0;
  dwf_solve_info si;
  const int ndc = std::min(info->n_dc, 8);
  for (int k = 0; k < ndc; ++k) {
    residual(r);
    // c = P^-1 D(1)^-1 r
    DWF_CHECK_LAUNCH(launch_zero(t, 2 * hb, s));
    std::memset(&si, 0, sizeof(si));
    solve_full(ctx, ppv, U64, r, t, info->tol_pv, maxit, delta, "pv", &si);
    info->pv_iters += si.iters; info->n_pv++; info->seconds_pv += si.seconds;
    pshift(t, c, 1, L, hb);
    // rhs' = D'(1) P' (c_1, 0, ..., 0)
    DWF_CHECK_LAUNCH(launch_zero(cp, 2 * hbp, s));
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_slice_copy(CH(c, par, L, hb), L, 0, H(cp, par, Lp, hbp), Lp, 0, 1.0, ns, s));
    pshift(cp, zp, 0, Lp, hbp);
    opi1.full(CH(zp, 0, Lp, hbp), CH(zp, 1, Lp, hbp), H(rp, 0, Lp, hbp), H(rp, 1, Lp, hbp), false);
    // D'(m) z = rhs'
    DWF_CHECK_LAUNCH(launch_zero(zp, 2 * hbp, s));
    std::memset(&si, 0, sizeof(si));
    solve_full(ctx, pi, U64, rp, zp, info->tol_mobius, maxit, delta, "mob", &si);
    info->mobius_iters += si.iters; info->n_mobius++; info->seconds_mobius += si.seconds;
    pshift(zp, yp, 1, Lp, hbp);  // y' = P'^-1 z ; y'_1 = slice 0
    // v = (-y'_1, c_2, ..., c_L) in c ; t = D(m) P v
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_slice_copy(CH(yp, par, Lp, hbp), Lp, 0, H(c, par, L, hb), L, 0, -1.0, ns, s));
    pshift(c, w, 0, L, hb);
    opt.full(CH(w, 0, L, hb), CH(w, 1, L, hb), H(t, 0, L, hb), H(t, 1, L, hb), false);
    // w = P^-1 D(1)^-1 t, started from P (0, c_2, .., c_L): for any y with y_1 = 0,
    // P^-1 D(1)^-1 D(m) P y = y (Sec. 4: the PV-transformed operator is the identity off the
    // first slice), so that guess is exact except for the part D(m) P (-y'_1, 0, .., 0) of t
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_slice_copy(CH(yp, par, Lp, hbp), Lp, 0, H(c, par, L, hb), L, 0, 0.0, ns, s));
    pshift(c, w, 0, L, hb);
    std::memset(&si, 0, sizeof(si));
    solve_full(ctx, ppv, U64, t, w, info->tol_pv, maxit, delta, "pv", &si);
    info->pv_iters += si.iters; info->n_pv++; info->seconds_pv += si.seconds;
    pshift(w, c, 1, L, hb);
    // replace the first slice by y'_1, back to the domain-wall basis, add to x
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_slice_copy(CH(yp, par, Lp, hbp), Lp, 0, H(c, par, L, hb), L, 0, 1.0, ns, s));
    pshift(c, t, 0, L, hb);
    for (int par = 0; par < 2; ++par)
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, CH(t, par, L, hb), 1.0, H(x, par, L, hb), ns * L, L, s));
    info->resid_after_dc[k] = std::sqrt(residual(r) / b2);
  }
  dwf_params pf = pt;
  pf.prec_inner = info->prec_final;
  std::memset(&si, 0, sizeof(si));
  const int st = solve_full(ctx, pf, U64, b, x, info->tol, maxit, delta, "final", &si);
  info->final_iters = si.iters;
  info->seconds_final = si.seconds;
  info->true_rel_resid = si.true_rel_resid;
  info->wilson_apps = (long long)info->pv_iters * L + (long long)info->mobius_iters * Lp + (long long)info->final_iters * L;
  info->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
  return st;
}

// ------------------------------------------------------------------ force
// S = phi^dag (M^dag M)^-1 phi.  X = (M^dag M)^-1 phi (warm start from x_io), Y = M X,
// X_e = A^-1 B_eo X, Y_o' = A^-dag Y, Y_e' = A^-dag B_oe^dag Y_o', W = F (X, X_e),
// Z = (Y_e', Y_o'); one thread per link contracts them into F_mu(x) or G_mu(x).
// The derivative of -2 Re <Y, M X> (X, Y odd half fields, M = M_prec of op) along every link
// and generator, written as F = sum_a e_a T_a (kind 0) or as the ambient gradient (kind 1):
// Fout = coef * that (+ Fout with accumulate).
//   dM = -A^-1 dB_oe A^-1 B_eo - A^-1 B_oe A^-1 dB_eo
static void force_terms(dwf_ctx* ctx, const Op<P64>& op, const void* Unat, CHalf<P64> X, CHalf<P64> Y, void* Fout,
                        int kind, double coef, int accumulate) {
  const Geometry* g = op.g;
  const int Ls = op.Ls;
  const size_t hb = half_size<P64>(g, Ls);
  Half<P64> Xe = hview<P64>(ws_get(ctx, "force.Xe", hb), g, Ls);
  Half<P64> Zo = hview<P64>(ws_get(ctx, "force.Zo", hb), g, Ls);
  Half<P64> Ze = hview<P64>(ws_get(ctx, "force.Ze", hb), g, Ls);
  Half<P64> We = hview<P64>(ws_get(ctx, "force.We", hb), g, Ls);
  Half<P64> Wo = hview<P64>(ws_get(ctx, "force.Wo", hb), g, Ls);
  op.hop(0, X, Xe, false, true, -0.5, op.em(E_AINV));                   // X_e = A^-1 B_eo X
  op.fifth(Y, Zo, E_AINVDAG);                                           // Y_o' = A^-dag Y
  op.hop(0, cv(Zo), Ze, true, false, -0.5, op.em(E_AINVDAG_FDAG));      // Y_e' = A^-dag B_oe^dag Y_o'
  op.fifth(X, Wo, E_F);                                                 // W_o = F X
  op.fifth(cv(Xe), We, E_F);                                            // W_e = F X_e
  const long mark = ctx->timer.on ? timer_begin(ctx, "force_kernel") : -1;
  DWF_CHECK_LAUNCH(launch_force(g->tables(), Ls, cv(We), cv(Wo), cv(Ze), cv(Zo),
                                reinterpret_cast<const double2*>(Unat), g->tbc, g->dims, kind,
                                reinterpret_cast<double2*>(Fout), ctx->stream, coef, accumulate));
  // algorithmic bytes: the four FP64 half fields W_e, W_o, Z_e, Z_o and the links read once, the
  // force written once (and read once when accumulating)
  if (mark >= 0)
    timer_end(ctx, mark, 4.0 * double(hb) + double(4 * g->V) * 9 * sizeof(double2) * (accumulate ? 3 : 2));
}

// S and the force at the links Unat.  X solves M^dag M X = phi to the normal-equation tolerance
// tol_n, judged by the FP64 true residual ||phi - M^dag M X|| / ||phi|| recomputed after the
// solve (the stop test of an FP64 recurrence uses its iterated residual); while it is above tol_n
// the solve continues from X with a tightened stop, within maxit iterations in all.  *converged
// turns false if it does not get there; *true_rel receives the largest true residual seen.
static double force_at(dwf_ctx* ctx, const dwf_params& p, const void* Unat, const void* phi, void* X, void* Fout,
                       int kind, double tol_n, int maxit, double delta, SolveStats* st, bool* converged,
                       double* true_rel) {
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const long n5 = g->nsites * Ls;
  const size_t hb = half_size<P64>(g, Ls);
  hipStream_t s = ctx->stream;
  void* U64 = ws_get(ctx, "force.U64", 2 * g->nsites * 72 * sizeof(double2));
  DWF_CHECK_LAUNCH(launch_pack_gauge<P64>(g->tables(), reinterpret_cast<const double2*>(Unat),
                                          reinterpret_cast<double2*>(U64), s));
  Op<P64> op(ctx, g, p, U64);
  CHalf<P64> ph = chview<P64>(phi, g, Ls);
  Half<P64> Xo = hview<P64>(X, g, Ls);
  Half<P64> Y = hview<P64>(ws_get(ctx, "force.Y", hb), g, Ls);
  Half<P64> tmp = hview<P64>(ws_get(ctx, "force.tmp", hb), g, Ls);
  Half<P64> r = hview<P64>(ws_get(ctx, "force.r", hb), g, Ls);
  Half<P64> tmp2 = hview<P64>(ws_get(ctx, "force.tmp2", hb), g, Ls);
  const double p2 = norm2_sync<P64>(ctx, ph, g, Ls);
  const int iters0 = st->iters;
  double tol_try = tol_n, rel = 0.0;
  for (int attempt = 0; attempt < 8; ++attempt) {
    const int left = maxit - (st->iters - iters0);
    if (attempt > 0 && left <= 0) break;
    normal_solve(ctx, p, U64, ph, Xo, tol_try, std::max(0, left), delta, "force.cg", st);
    op.mprec(cv(Xo), Y, tmp);  // Y = M X
    // FP64 true residual of the normal equations, phi - M^dag Y
    op.mprec_dag(cv(Y), r, tmp, tmp2);
    DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, ph, -1.0, r, n5, Ls, s));
    const double r2 = norm2_sync<P64>(ctx, cv(r), g, Ls);
    rel = p2 > 0.0 ? std::sqrt(r2 / p2) : 0.0;
    if (!std::isfinite(rel)) throw Error{DWF_ERR_NAN, "non-finite residual of the force solve"};
    if (rel <= tol_n) break;
    tol_try *= std::max(0.02, std::min(0.5, 0.5 * tol_n / rel));
    st->restarts++;
  }
  *true_rel = std::max(*true_rel, rel);
  if (rel > tol_n) *converged = false;
  // S = Re <phi, X>
  double* part = partials_buf(ctx);
  double* sc = scalars_buf(ctx);
  DWF_CHECK_LAUNCH(launch_dot<P64>(ph, cv(Xo), n5, Ls, part, s));
  DWF_CHECK_LAUNCH(launch_reduce(part, reduction_blocks(n5), 2, sc, S_TMP1, 0, s));
  const double S = read_scalar(ctx, sc, S_TMP1);
  force_terms(ctx, op, Unat, cv(Xo), cv(Y), Fout, kind, 1.0, 0);
  return S;
}

int fermion_force(dwf_ctx* ctx, const dwf_params& p, const void* Unat, const void* phi, void* F, double* S,
                  double tau_fg, int out_kind, void* x_io, dwf_solve_info* info) {
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const size_t hb = half_size<P64>(g, Ls);
  hipStream_t s = ctx->stream;
  const double tol = info && info->tol > 0 ? info->tol : 1e-12;
  const double delta = info && info->delta > 0 ? info->delta : 0.1;
  const int maxit = info && info->maxit > 0 ? info->maxit : 100000;
  void* X = ws_get(ctx, "force.X", hb);
  if (x_io) DWF_CHECK_HIP(hipMemcpyAsync(X, x_io, hb, hipMemcpyDeviceToDevice, s));
  else DWF_CHECK_LAUNCH(launch_zero(X, hb, s));
  SolveStats st;
  double Sv;
  bool conv = true;
  double rel = 0.0;
  if (tau_fg > 0.0) {
    // force-gradient step: F1 at U; U' = exp(-tau^2/24 F1) U; force at U' from X(U)
    const long nlinks = 4 * g->V;
    void* F1 = ws_get(ctx, "force.F1", nlinks * 9 * sizeof(double2));
    void* Up = ws_get(ctx, "force.Uprime", nlinks * 9 * sizeof(double2));
    force_at(ctx, p, Unat, phi, X, F1, 0, tol, maxit, delta, &st, &conv, &rel);
    const int it1 = st.iters;
    DWF_CHECK_LAUNCH(launch_fg_update(reinterpret_cast<const double2*>(F1), reinterpret_cast<const double2*>(Unat),
                                      tau_fg * tau_fg / 24.0, reinterpret_cast<double2*>(Up), nlinks, s));
    Sv = force_at(ctx, p, Up, phi, X, F, out_kind, tol, std::max(0, maxit - it1), delta, &st, &conv, &rel);
    if (info) info->iters_first = it1;
  } else {
    Sv = force_at(ctx, p, Unat, phi, X, F, out_kind, tol, maxit, delta, &st, &conv, &rel);
  }
  if (x_io) DWF_CHECK_HIP(hipMemcpyAsync(x_io, X, hb, hipMemcpyDeviceToDevice, s));
  DWF_CHECK_HIP(hipStreamSynchronize(s));
  if (S) *S = Sv;
  if (info) {
    info->iters = st.iters;
    info->reliable_updates = st.reliable_updates;
    info->restarts = st.restarts;
    info->true_rel_resid = rel;
    info->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    info->wilson_apps = (long long)st.iters * Ls;
  }
  return conv ? DWF_OK : DWF_NOT_CONVERGED;
}

// ------------------------------------------------------------------ Hasenbusch quotients
// S_i = phi_i^dag M(m_i) (M(m_{i-1})^dag M(m_{i-1}))^-1 M(m_i)^dag phi_i  (Sec. 3 mass ladder),
// i = 1..nq: the nq normal-equation solves run as one batched CG (every hop stage one launch
// for all of them); then F = sum_i [e(-2 Re <Y_i, M(m_{i-1}) X_i>) - e(-2 Re <phi_i, M(m_i) X_i>)],
// Y_i = M(m_{i-1}) X_i, accumulated into one force field.
int quotient_force(dwf_ctx* ctx, const dwf_params& p, int nq, const double* masses, const void* Unat,
                   const void* const* phi, void* F, double* S, int out_kind, void* const* x_io,
                   dwf_solve_info* info) {
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const size_t hb = half_size<P64>(g, Ls);
  hipStream_t s = ctx->stream;
  const double tol = info && info->tol > 0 ? info->tol : 1e-10;
  const double delta = info && info->delta > 0 ? info->delta : 0.1;
  const int maxit = info && info->maxit > 0 ? info->maxit : 100000;
  void* U64 = ws_get(ctx, "quot.U64", 2 * g->nsites * 72 * sizeof(double2));
  DWF_CHECK_LAUNCH(launch_pack_gauge<P64>(g->tables(), reinterpret_cast<const double2*>(Unat),
                                          reinterpret_cast<double2*>(U64), s));
  const void* Ui = links_in(ctx, g, U64, p.prec_inner, "quot");
  Half<P64> to = hview<P64>(ws_get(ctx, "quot.to", hb), g, Ls);
  Half<P64> te = hview<P64>(ws_get(ctx, "quot.te", hb), g, Ls);
  std::vector<BatchSys> B(nq);
  std::vector<void*> X(nq), chi(nq);
  for (int i = 0; i < nq; ++i) {
    dwf_params pn = p, pd = p;
    pn.mass = masses[i + 1];
    pd.mass = masses[i];
    Op<P64> opn(ctx, g, pn, U64);
    chi[i] = ws_get(ctx, "quot.chi." + std::to_string(i), hb);
    X[i] = ws_get(ctx, "quot.X." + std::to_string(i), hb);
    opn.mprec_dag(chview<P64>(phi[i], g, Ls), hview<P64>(chi[i], g, Ls), to, te);  // chi = M(m_i)^dag phi
    if (x_io && x_io[i]) DWF_CHECK_HIP(hipMemcpyAsync(X[i], x_io[i], hb, hipMemcpyDeviceToDevice, s));
    else DWF_CHECK_LAUNCH(launch_zero(X[i], hb, s));
    BatchSys& b = B[i];
    b.p = pd;
    b.g = g;
    b.U64 = U64;
    b.Ui = Ui;
    b.op64 = std::make_unique<Op<P64>>(ctx, g, pd, U64);
    b.rhs = chview<P64>(chi[i], g, Ls);
    b.x = hview<P64>(X[i], g, Ls);
    b.tol_n = tol;
    b.cap = maxit;
  }
  switch (p.prec_inner) {
    case DWF_FP64: cg_batched<P64>(ctx, B, maxit, delta); break;
    case DWF_FP32: cg_batched<P32>(ctx, B, maxit, delta); break;
    case DWF_FP16: cg_batched<P16>(ctx, B, maxit, delta); break;
    default: cg_batched<PB16>(ctx, B, maxit, delta); break;
  }
  double* part = partials_buf(ctx);
  double* sc = scalars_buf(ctx);
  Half<P64> Y = hview<P64>(ws_get(ctx, "quot.Y", hb), g, Ls);
  long long iters = 0;
  int status = 0;
  for (int i = 0; i < nq; ++i) {
    dwf_params pn = p, pd = p;
    pn.mass = masses[i + 1];
    pd.mass = masses[i];
    Op<P64> opn(ctx, g, pn, U64), opd(ctx, g, pd, U64);
    CHalf<P64> Xi = chview<P64>(X[i], g, Ls);
    DWF_CHECK_LAUNCH(launch_dot<P64>(chview<P64>(chi[i], g, Ls), Xi, g->nsites * Ls, Ls, part, s));
    DWF_CHECK_LAUNCH(launch_reduce(part, reduction_blocks(g->nsites * Ls), 2, sc, S_TMP1, 0, s));
    if (S) S[i] = read_scalar(ctx, sc, S_TMP1);
    opd.mprec(Xi, Y, te);  // Y = M(m_{i-1}) X
    force_terms(ctx, opd, Unat, Xi, cv(Y), F, out_kind, 1.0, i > 0);
    force_terms(ctx, opn, Unat, Xi, chview<P64>(phi[i], g, Ls), F, out_kind, -1.0, 1);
    if (x_io && x_io[i]) DWF_CHECK_HIP(hipMemcpyAsync(x_io[i], X[i], hb, hipMemcpyDeviceToDevice, s));
    iters += B[i].st.iters;
    if (B[i].rr > B[i].target) status = DWF_NOT_CONVERGED;
  }
  DWF_CHECK_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = int(iters);
    info->reliable_updates = 0;
    for (auto& b : B) info->reliable_updates += b.st.reliable_updates;
    double worst = 0.0;
    for (auto& b : B) worst = std::max(worst, b.rhs2 > 0 ? std::sqrt(b.rr / b.rhs2) : 0.0);
    info->true_rel_resid = worst;
    info->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
    info->wilson_apps = iters * Ls;
  }
  return status;
}


// ------------------------------------------------------------------ force-gradient integrator
// One molecular-dynamics trajectory (Sec. 2) of
//   exp(tau/6 z_S) exp(tau/2 z_T) exp(2 tau/3 z_S - tau^3/72 z_{S,{S,T}}) exp(tau/2 z_T) exp(tau/6 z_S)
// per step for H = sum p_a^2 / 2 + S_g + phi^+ (M^+ M)^-1 phi, z_T: U <- exp(eps P) U,
// z_S: P <- P - eps F.  The middle momentum update uses the force at
// U' = exp(-tau^2/24 F(U)) U with its solve started from X(U) (force-gradient forecasting);
// the other solves start from zero; the force at the end of a step opens the next one.
static double total_force(dwf_ctx* ctx, const dwf_params& p, double beta, const void* U, const void* phi, void* X,
                          void* F, double tol_n, int maxit, double delta, SolveStats* st, bool* conv, double* rel) {
  const double Sf = force_at(ctx, p, U, phi, X, F, 0, tol_n, maxit, delta, st, conv, rel);
  DWF_CHECK_LAUNCH(launch_gauge_force(reinterpret_cast<const double2*>(U), p.dims, beta, 1.0, 1,
                                      reinterpret_cast<double2*>(F), ctx->stream));
  return Sf;
}

static double partial_sum(dwf_ctx* ctx, int nblocks) {
  double* sc = scalars_buf(ctx);
  DWF_CHECK_LAUNCH(launch_reduce(partials_buf(ctx), nblocks, 1, sc, S_TMP2, 0, ctx->stream));
  return read_scalar(ctx, sc, S_TMP2);
}

static double hamiltonian(dwf_ctx* ctx, const dwf_params& p, double beta, const void* U, const void* P, double Sf,
                          long nlinks) {
  int nb = 0;
  DWF_CHECK_LAUNCH(launch_kinetic(reinterpret_cast<const double2*>(P), nlinks, partials_buf(ctx), &nb, ctx->stream));
  const double K = partial_sum(ctx, nb);
  DWF_CHECK_LAUNCH(launch_plaquette(reinterpret_cast<const double2*>(U), p.dims, partials_buf(ctx), &nb, ctx->stream));
  const double Sg = beta * partial_sum(ctx, nb);
  return K + Sg + Sf;
}

int fgi_trajectory(dwf_ctx* ctx, const dwf_params& p, void* U, void* P, const void* phi, dwf_hmc_info* info) {
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const size_t hb = half_size<P64>(g, p.Ls);
  const long nl = 4 * g->V;
  hipStream_t s = ctx->stream;
  const double beta = info->beta, tau = info->tau;
  const double tol = info->tol > 0 ? info->tol : 1e-10;
  const double delta = info->delta > 0 ? info->delta : 0.1;
  const int maxit = info->maxit > 0 ? info->maxit : 100000;
  void* F = ws_get(ctx, "hmc.F", nl * 9 * sizeof(double2));
  void* F1 = ws_get(ctx, "hmc.F1", nl * 9 * sizeof(double2));
  void* Up = ws_get(ctx, "hmc.Uprime", nl * 9 * sizeof(double2));
  void* X = ws_get(ctx, "hmc.X", hb);
  void* X1 = ws_get(ctx, "hmc.X1", hb);
  double2* Pd = reinterpret_cast<double2*>(P);
  double2* Ud = reinterpret_cast<double2*>(U);
  SolveStats st;
  bool conv = true;
  double rel = 0.0;
  int evals = 0, fg_first = 0, fg_second = 0;
  DWF_CHECK_LAUNCH(launch_zero(X, hb, s));
  double Sf = total_force(ctx, p, beta, U, phi, X, F, tol, maxit, delta, &st, &conv, &rel);
  ++evals;
  info->H_start = hamiltonian(ctx, p, beta, U, P, Sf, nl);
  for (int step = 0; step < info->n_steps; ++step) {
    DWF_CHECK_LAUNCH(launch_mom_update(Pd, reinterpret_cast<const double2*>(F), tau / 6.0, nl, s));
    DWF_CHECK_LAUNCH(launch_fg_update(Pd, Ud, -tau / 2.0, Ud, nl, s));  // U <- exp(tau/2 P) U
    DWF_CHECK_LAUNCH(launch_zero(X1, hb, s));
    int before = st.iters;
    total_force(ctx, p, beta, U, phi, X1, F1, tol, maxit, delta, &st, &conv, &rel);
    fg_first += st.iters - before;
    // force-gradient step: U' = exp(-tau^2/24 F1) U, force at U' from X(U)
    DWF_CHECK_LAUNCH(launch_fg_update(reinterpret_cast<const double2*>(F1), Ud, tau * tau / 24.0,
                                      reinterpret_cast<double2*>(Up), nl, s));
    before = st.iters;
    total_force(ctx, p, beta, Up, phi, X1, F1, tol, maxit, delta, &st, &conv, &rel);
    fg_second += st.iters - before;
    DWF_CHECK_LAUNCH(launch_mom_update(Pd, reinterpret_cast<const double2*>(F1), 2.0 * tau / 3.0, nl, s));
    DWF_CHECK_LAUNCH(launch_fg_update(Pd, Ud, -tau / 2.0, Ud, nl, s));
    DWF_CHECK_LAUNCH(launch_zero(X, hb, s));
    Sf = total_force(ctx, p, beta, U, phi, X, F, tol, maxit, delta, &st, &conv, &rel);
    DWF_CHECK_LAUNCH(launch_mom_update(Pd, reinterpret_cast<const double2*>(F), tau / 6.0, nl, s));
    evals += 3;
  }
  info->H_end = hamiltonian(ctx, p, beta, U, P, Sf, nl);
  DWF_CHECK_HIP(hipStreamSynchronize(s));
  info->force_evals = evals;
  info->cg_iters = st.iters;
  info->fg_iters_first = fg_first;
  info->fg_iters_forecast = fg_second;
  info->seconds = std::chrono::duration<double>(Clock::now() - t0).count();
  return conv ? DWF_OK : DWF_NOT_CONVERGED;
}

}  // namespace dwf
