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
// OpT: Op (4D even-odd, M_prec) or Op5 (5D even-odd Shamir, its Schur complement S).
template <typename Pi, template <typename> class OpT = Op>
static int cg_normal(dwf_ctx* ctx, const OpT<P64>& op64, const OpT<Pi>& opi, CHalf<P64> rhs, Half<P64> x,
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
  // q = M p is stored only where the last hop of M^dag q cannot rebuild it from A^-dag q
  const bool OUT2 = opi.second_output_ok(), QREB = OUT2 && opi.rebuild_q_ok();
  Half<Pi> q = QREB ? Half<Pi>{nullptr, nullptr} : hview<Pi>(ws_get(ctx, tag + ".q." + pname(Pi::ID), hbi), g, Ls);
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
  const long nb_hop = opi.hop_blocks();
  int it = 0;
  while (it < maxit) {
    const Half<Pi> p = pr[cur];
    // q = M p, |q|^2 -> alpha = rr / |q|^2 (also kept in the history slot of this direction)
    // (with A^-dag q, the first step of M^dag q, as a second output of the last hop, and then,
    // where the last hop of M^dag q rebuilds q from it, q itself is not stored)
    const Half<Pi> q2 = OUT2 ? to : Half<Pi>{nullptr, nullptr};
    if (PRE) opi.mprec_pre(cv(fp), cv(p), q, te, part, q2);
    else opi.mprec(cv(p), q, te, part, q2);
    DWF_CHECK_LAUNCH(launch_reduce(part, int(nb_hop), 1, sc, S_QQ, 1, s, pend.n));
    pend.p[pend.n] = cv(p);
    pend.slot[pend.n] = pend.n;
    ++pend.n;
    // r -= alpha M^dag q and |r|^2, fused into the last hop of M^dag q
    opi.mprec_dag_cg(cv(q), to, te, r, sc, part, OUT2, QREB);
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

// ------------------------------------------------------------------ 5D even-odd (Shamir)
// the operator family the 5D checkerboard applies to: Shamir, Ls / 2 a divisor of 64 (a site's
// slices of one 5D parity form one wave segment)
static void eo5_check(const dwf_params& p) {
  if (!(p.b == 1.0 && p.c == 0.0) || p.b_s || p.c_s)
    throw Error{DWF_ERR_ARG, "the 5D even-odd operator is Shamir DWF only (b = 1, c = 0, constant)"};
  if (p.Ls < 2 || p.Ls % 2 || 64 % (p.Ls / 2) != 0)
    throw Error{DWF_ERR_ARG, "the 5D even-odd operator needs Ls in {2, 4, 8, 16, 32, 64, 128}"};
}

template <typename Pi>
static int cg5_dispatch(dwf_ctx* ctx, const Op5<P64>& op64, const dwf_params& p, const void* U64, CHalf<P64> rhs,
                        Half<P64> x, double tol_n, int maxit, double delta, const std::string& tag, SolveStats* st) {
  const void* Ui = links_in(ctx, op64.g4, U64, Pi::ID, tag);
  Op5<Pi> opi(ctx, op64.g4, p, Ui);
  return cg_normal<Pi, Op5>(ctx, op64, opi, rhs, x, tol_n, maxit, delta, tag, st);
}

// D(m) x = b through the 5D even-odd Schur complement:
//   b'_e = b_e + K_eo b_o / d0,  S^dag S x_e = S^dag b'_e  (CGNR),  x_o = (b_o + K_oe x_e) / d0,
// tightening the normal-equation tolerance until ||b - D x|| / ||b|| <= tol (the residual through
// the 4D even-odd operator's D).
int solve_full_5d(dwf_ctx* ctx, const dwf_params& p, const void* U64, const void* b, void* x, double tol, int maxit,
                  double delta, const std::string& tag, dwf_solve_info* info) {
  eo5_check(p);
  const auto t0 = Clock::now();
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const long n5 = g->nsites * Ls;
  const size_t hb = half_size<P64>(g, Ls);
  hipStream_t s = ctx->stream;
  Op<P64> op(ctx, g, p, U64);
  Op5<P64> op5(ctx, g, p, U64);
  const Geometry* gv = op5.g;
  const int LH = op5.Ls;
  const double d0 = op5.d0;
  const size_t fb = half_size<P64>(gv, LH);
  auto field = [&](const char* name) { return hview<P64>(ws_get(ctx, tag + name, fb), gv, LH); };
  Half<P64> be = field(".be"), bo = field(".bo"), xe = field(".xe"), xo = field(".xo"), bp = field(".bp"),
            rhs = field(".rhs"), t1 = field(".t1"), t2 = field(".t2");
  CHalf<P64> b4e = chalf_at<P64>(b, 0, g, Ls), b4o = chalf_at<P64>(b, hb, g, Ls);
  Half<P64> x4e = half_at<P64>(x, 0, g, Ls), x4o = half_at<P64>(x, hb, g, Ls);
  void* rfull = ws_get(ctx, tag + ".rfull", 2 * hb);
  Half<P64> re = half_at<P64>(rfull, 0, g, Ls), ro = half_at<P64>(rfull, hb, g, Ls);

  const double b2 = norm2_sync<P64>(ctx, b4e, g, Ls) + norm2_sync<P64>(ctx, b4o, g, Ls);
  if (!std::isfinite(b2)) throw Error{DWF_ERR_NAN, "non-finite source"};
  SolveStats st;
  int status = 0;
  double rel = 0.0;
  if (b2 == 0.0) {
    DWF_CHECK_LAUNCH(launch_zero(x, 2 * hb, s));
  } else {
    DWF_CHECK_LAUNCH(launch_eo5_split<P64>(Half<P64>{const_cast<double2*>(b4e.data), nullptr},
                                           Half<P64>{const_cast<double2*>(b4o.data), nullptr}, be, bo, g->nsites, Ls,
                                           0, s));
    // the initial guess: x split the same way (a zero x gives zero fields)
    DWF_CHECK_LAUNCH(launch_eo5_split<P64>(x4e, x4o, xe, xo, g->nsites, Ls, 0, s));
    op5.K(0, cv(bo), bp, false, 0.5 / d0, 1.0 / d0, cv(be), 1.0);  // b'_e
    op5.mprec_dag(cv(bp), rhs, t1, t2);                            // S^dag b'_e
    double tol_n = tol;
    status = 1;
    for (int attempt = 0; attempt < 12; ++attempt) {
      const int left = maxit - st.iters;
      if (left <= 0) break;
      switch (p.prec_inner) {
        case DWF_FP64: cg5_dispatch<P64>(ctx, op5, p, U64, cv(rhs), xe, tol_n, left, delta, tag + ".cg", &st); break;
        case DWF_FP32: cg5_dispatch<P32>(ctx, op5, p, U64, cv(rhs), xe, tol_n, left, delta, tag + ".cg", &st); break;
        case DWF_FP16: cg5_dispatch<P16>(ctx, op5, p, U64, cv(rhs), xe, tol_n, left, delta, tag + ".cg", &st); break;
        default: cg5_dispatch<PB16>(ctx, op5, p, U64, cv(rhs), xe, tol_n, left, delta, tag + ".cg", &st); break;
      }
      op5.K(1, cv(xe), xo, false, 0.5 / d0, 1.0 / d0, cv(bo), 1.0 / d0);  // x_o
      DWF_CHECK_LAUNCH(launch_eo5_split<P64>(x4e, x4o, xe, xo, g->nsites, Ls, 1, s));
      // true residual of the full system (4D even-odd D)
      op.full(cv(x4e), cv(x4o), re, ro, false);
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, b4e, -1.0, re, n5, Ls, s));
      DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, b4o, -1.0, ro, n5, Ls, s));
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

// one application of K (op 0: both 5D parities) or S (op 1: the even 5D parity; the odd part of
// out is zero) in precision P on packed fields of that precision
template <typename P>
static void dslash_5d_t(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op,
                        bool dag) {
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  const int Ls = p.Ls;
  const size_t hb = half_size<P>(g, Ls);
  hipStream_t s = ctx->stream;
  Op5<P> op5(ctx, g, p, U);
  const Geometry* gv = op5.g;
  const int LH = op5.Ls;
  const size_t fb = half_size<P>(gv, LH);
  auto field = [&](const char* name) { return hview<P>(ws_get(ctx, std::string("d5") + name, fb), gv, LH); };
  Half<P> ie = field(".ie"), io = field(".io"), oe = field(".oe"), oo = field(".oo"), t = field(".t");
  Half<P> i4e = hview<P>(const_cast<void*>(in), g, Ls), i4o = hview<P>(reinterpret_cast<char*>(const_cast<void*>(in)) + hb, g, Ls);
  Half<P> o4e = hview<P>(out, g, Ls), o4o = hview<P>(reinterpret_cast<char*>(out) + hb, g, Ls);
  DWF_CHECK_LAUNCH(launch_eo5_split<P>(i4e, i4o, ie, io, g->nsites, Ls, 0, s));
  if (op == 0) {
    op5.K(0, cv(io), oe, dag, 0.5, 1.0);
    op5.K(1, cv(ie), oo, dag, 0.5, 1.0);
  } else {
    if (dag) op5.mprec_dag(cv(ie), oe, t, oo);
    else op5.mprec(cv(ie), oe, t);
    DWF_CHECK_LAUNCH(launch_zero(oo.data, fb, s));  // (the FP16 norms follow the data in the buffer)
  }
  DWF_CHECK_LAUNCH(launch_eo5_split<P>(o4e, o4o, oe, oo, g->nsites, Ls, 1, s));
}

int dslash_5d(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op, int dagger) {
  eo5_check(p);
  if (op != 0 && op != 1) throw Error{DWF_ERR_ARG, "op must be 0 (K) or 1 (S)"};
  switch (p.prec) {
    case DWF_FP64: dslash_5d_t<P64>(ctx, p, U, in, out, op, dagger != 0); break;
    case DWF_FP32: dslash_5d_t<P32>(ctx, p, U, in, out, op, dagger != 0); break;
    case DWF_FP16: dslash_5d_t<P16>(ctx, p, U, in, out, op, dagger != 0); break;
    default: dslash_5d_t<PB16>(ctx, p, U, in, out, op, dagger != 0); break;
  }
  return 0;
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
// lattices) iterate in lock step, each with the iteration of cg_normal (the same fused hops,
// direction ring and deferred increment, FP64 scalars and reliable updates).  Each of the four
// hop stages of an iteration is one launch over the unconverged right-hand sides of a lattice
// (hop_batch_kernel: the right-hand sides of one site block run together, so its links are
// read from memory once and then hit in L2); one device-to-host copy per iteration returns
// every residual.
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
};

// The right-hand sides of one lattice with Ls = RS in {8, 16, 32}, Shamir operator, interleaved
// along the fifth dimension: every vector of the iteration is one field of extent K RS (slice s of
// right-hand side r at r RS + s), so that each hop stage is one launch whose workgroups take all K
// right-hand sides of a site (the site's neighbour indices and links serve K RS lanes, each
// neighbour's K RS slices are one contiguous gather).  The fifth-dimension blocks, CG scalars and
// norm partials are per right-hand side.  When a right-hand side converges it leaves the field
// (the others are moved together); the FP64 solutions, residuals and reliable updates stay
// separate per right-hand side.
template <typename Pi>
static void cg_batched_ilv(dwf_ctx* ctx, std::vector<BatchSys*> sys, double delta) {
  constexpr bool MIXED = !std::is_same<Pi, P64>::value;
  using PX = typename IncrementPrec<Pi>::type;
  using R = typename Pi::R;
  using SS = typename Pi::S;
  constexpr bool RESTART = std::is_same<Pi, PB16>::value;
  constexpr int KX = 8;
  hipStream_t s = ctx->stream;
  const int K0 = int(sys.size());
  const Geometry* g = sys[0]->g;
  const int RS = sys[0]->p.Ls;
  const long ns = g->nsites;
  const int LT0 = K0 * RS;
  // launch shape: the whole site (LT lanes) in a workgroup; LDS link staging and XCD order from
  // the interleaved hop's tuning entry
  const LaunchCfg tuned = ilv_config(ctx, Pi::ID, RS);
  auto cfg_for = [&](int LT) {
    LaunchCfg c;
    c.ns = 1;
    c.spb = std::max(1, 256 / LT);
    c.xcd = tuned.xcd;
    c.ll = tuned.ll;
    c.stage = 0;
    return c;
  };
  const long pstride = (ns + cfg_for(LT0).spb - 1) / cfg_for(LT0).spb;
  double* part = reinterpret_cast<double*>(ws_get(ctx, "ilv.partials", size_t(K0) * pstride * sizeof(double)));
  double* sc = reinterpret_cast<double*>(ws_get(ctx, "ilv.scalars", size_t(K0) * S_COUNT * sizeof(double)));
  double* dcoef = reinterpret_cast<double*>(ws_get(ctx, "ilv.coef", size_t(2) * K0 * sizeof(double)));
  // the fifth-dimension tables per right-hand side: A^-1, A^-dag, A^-dag (F^dag), A^dag
  const size_t nscan = size_t(4) * K0;
  FifthScan<R>* dscan = reinterpret_cast<FifthScan<R>*>(ws_get(ctx, "ilv.scan", nscan * sizeof(FifthScan<R>)));
  // pinned host mirrors: scalars, p-update coefficients, fifth-dimension tables (freed on every
  // exit, also when a later allocation throws)
  struct HostFree {
    void* p[3] = {nullptr, nullptr, nullptr};
    ~HostFree() {
      for (void* q : p)
        if (q) (void)hipHostFree(q);
    }
  } host_free;
  DWF_CHECK_HIP(hipHostMalloc(&host_free.p[0], size_t(K0) * S_COUNT * sizeof(double)));
  DWF_CHECK_HIP(hipHostMalloc(&host_free.p[1], size_t(2) * K0 * sizeof(double)));
  DWF_CHECK_HIP(hipHostMalloc(&host_free.p[2], nscan * sizeof(FifthScan<R>)));
  double* hsc = static_cast<double*>(host_free.p[0]);
  double* hcoef = static_cast<double*>(host_free.p[1]);
  FifthScan<R>* hscan = static_cast<FifthScan<R>*>(host_free.p[2]);
  // interleaved inner vectors (sized for all K0 right-hand sides)
  const size_t hbi = half_bytes<Pi>(ns, LT0);
  void* rb = ws_get(ctx, "ilv.r", hbi);
  // q = M p is rebuilt by the last hop from A^-dag q (as in cg_normal), except in FP64
  constexpr bool QREB = MIXED;
  void* qb = QREB ? nullptr : ws_get(ctx, "ilv.q", hbi);
  void* teb = ws_get(ctx, "ilv.te", hbi);
  void* tob = ws_get(ctx, "ilv.to", hbi);
  void* pb[KX];
  for (int j = 0; j < KX; ++j) pb[j] = ws_get(ctx, "ilv.p" + std::to_string(j), hbi);
  void* xlb = MIXED ? ws_get(ctx, "ilv.xlo", half_bytes<PX>(ns, LT0)) : nullptr;
  // FP64 per-right-hand-side solution increment for FP64 iterations (PX = P64): kept interleaved too
  if (!MIXED) xlb = ws_get(ctx, "ilv.x64", half_bytes<PX>(ns, LT0));
  const size_t hb64 = half_size<P64>(g, RS);
  void* rhi_raw = ws_get(ctx, "ilv.rhi", hb64);
  void* t64a_raw = ws_get(ctx, "ilv.t64a", hb64);
  void* t64b_raw = ws_get(ctx, "ilv.t64b", hb64);
  void* t64c_raw = ws_get(ctx, "ilv.t64c", hb64);
  auto true_residual = [&](BatchSys& b) -> double {
    Half<P64> rhi = hview<P64>(rhi_raw, g, RS), ta = hview<P64>(t64a_raw, g, RS), tb = hview<P64>(t64b_raw, g, RS),
              tc = hview<P64>(t64c_raw, g, RS);
    b.op64->mprec(cv(b.x), ta, tb);
    b.op64->mprec_dag(cv(ta), rhi, tb, tc);
    DWF_CHECK_LAUNCH(launch_axpby<P64>(1.0, b.rhs, -1.0, rhi, ns * RS, RS, s));
    return norm2_sync<P64>(ctx, cv(rhi), g, RS);
  };
  auto H = [&](void* base, int LT) { return half_view<Pi>(base, ns, LT); };
  auto HX = [&](void* base, int LT) { return half_view<PX>(base, ns, LT); };
  // the operators in the iteration precision (fifth-dimension coefficients per mass)
  std::vector<std::unique_ptr<Op<Pi>>> ops(K0);
  for (int k = 0; k < K0; ++k) ops[k] = std::make_unique<Op<Pi>>(ctx, g, sys[k]->p, sys[k]->Ui);
  const SS* links = reinterpret_cast<const SS*>(sys[0]->Ui);
  // start: the residual of every system into its segment
  std::vector<int> seg;  // segment -> system
  int LT = LT0;
  DWF_CHECK_LAUNCH(launch_zero(xlb, half_bytes<PX>(ns, LT0), s));
  for (int k = 0; k < K0; ++k) {
    BatchSys& b = *sys[k];
    b.rhs2 = norm2_sync<P64>(ctx, b.rhs, g, RS);
    b.target = b.tol_n * b.tol_n * b.rhs2;
    b.active = false;
    if (b.rhs2 == 0.0) {
      DWF_CHECK_LAUNCH(launch_zero(b.x.data, hb64, s));
      continue;
    }
    CHalf<P64> r0 = b.rhs;
    if (norm2_sync<P64>(ctx, cv(b.x), g, RS) == 0.0) {
      b.rr = b.rhs2;
    } else {
      b.rr = true_residual(b);
      r0 = chview<P64>(rhi_raw, g, RS);
    }
    if (!std::isfinite(b.rr)) throw Error{DWF_ERR_NAN, "non-finite residual at batched CG start"};
    b.rr_max = b.rr_true = b.rr;
    if (b.rr <= b.target || b.cap <= 0) continue;
    b.active = true;
    DWF_CHECK_LAUNCH((launch_ilv_move<P64, Pi>(r0, RS, 0, H(rb, LT0), LT0, int(seg.size()), ns, RS, s)));
    seg.push_back(k);
  }
  int K = int(seg.size());
  LT = K * RS;
  auto upload_tables = [&]() {
    for (int r = 0; r < K; ++r) {
      const Op<Pi>& o = *ops[seg[r]];
      hscan[0 * K0 + r] = o.es[E_AINV];
      hscan[1 * K0 + r] = o.es[E_AINVDAG];
      hscan[2 * K0 + r] = o.es[E_AINVDAG_FDAG];
      hscan[3 * K0 + r] = o.es[E_ADAG];
    }
    DWF_CHECK_HIP(hipMemcpyAsync(dscan, hscan, nscan * sizeof(FifthScan<R>), hipMemcpyHostToDevice, s));
  };
  int cur = 0;
  XFlush<Pi> pend;
  auto upload_coef = [&](const std::vector<double>& beta) {
    for (int r = 0; r < K; ++r) {
      hcoef[r] = beta[r];
      hcoef[K + r] = sys[seg[r]]->rr;
    }
    DWF_CHECK_HIP(hipMemcpyAsync(dcoef, hcoef, size_t(2) * K * sizeof(double), hipMemcpyHostToDevice, s));
  };
  auto p_update = [&](const std::vector<double>& beta) {
    upload_coef(beta);
    const int nxt = (cur + 1) % KX;
    DWF_CHECK_LAUNCH(launch_ilv_pupdate<Pi>(cv(H(rb, LT)), cv(H(pb[cur], LT)), H(pb[nxt], LT), dcoef, sc, ns, LT, RS, s));
    cur = nxt;
  };
  auto flush = [&]() {
    DWF_CHECK_LAUNCH((launch_ilv_xflush<Pi, PX>(HX(xlb, LT), pend, sc, ns, LT, RS, s)));
    pend.n = 0;
  };
  if (K > 0) {
    upload_tables();
    p_update(std::vector<double>(K, 0.0));
  }
  auto launch = [&](const HopArgs<Pi>& a, bool dag) {
    long mark = -1;
    if (ctx->timer.on) {
      const int epi = a.epi_scan ? (a.out2.data ? 3 : 2) : 0;
      const LaunchCfg c = cfg_for(LT);
      mark = timer_begin(ctx, std::string("hop_ilv_kernel<") + prec_tag(Pi::ID) + ", " + (dag ? "true" : "false") +
                                  ", " + std::to_string(epi) + ", " + (c.ll ? "true" : "false") + ", " +
                                  (a.cg_r.data ? "true" : "false") + ", " + std::to_string(RS) + ">");
    }
    DWF_CHECK_LAUNCH(launch_hop_ilv<Pi>(a, dag, RS, cfg_for(LT), s));
    if (mark >= 0) {
      const double fb = spinor_site_bytes<Pi>();
      const bool xin = a.x.data != nullptr;
      const double nb = a.cg_r.data ? 3 + (xin ? 1 : 0) : 1 + (a.out.data ? 1 : 0) + (xin ? 1 : 0) + (a.out2.data ? 1 : 0);
      timer_end(ctx, mark, double(ns) * LT * fb * nb + double(ns) * 72 * sizeof(SS));
    }
  };
  while (K > 0) {
    const LaunchCfg cfg = cfg_for(LT);
    const int nb = int((ns + cfg.spb - 1) / cfg.spb);
    HopArgs<Pi> a = HopArgs<Pi>();  // value-initialized: every optional operand absent
    a.x = CHalf<Pi>{nullptr, nullptr};
    a.ax = R(0);
    a.norm_partials = nullptr;
    a.es = FifthScan<R>();
    a.es2 = FifthScan<R>();
    a.nsites = ns;
    a.Ls = LT;
    a.pb = R(1);
    a.pc = R(0);
    a.pm = R(0);
    a.E = nullptr;
    a.part_stride = pstride;
    auto base = [&](HopArgs<Pi>& h, int out_par) {
      h = a;
      h.links = links + (out_par ? size_t(ns) * 72 : 0);
      h.nbr = g->d_nbr[out_par];
      h.order = g->d_order[out_par];
    };
    const Half<Pi> p = H(pb[cur], LT), r = H(rb, LT), te = H(teb, LT), to = H(tob, LT);
    const Half<Pi> q = QREB ? Half<Pi>{nullptr, nullptr} : H(qb, LT);
    HopArgs<Pi> h0, h1, h2, h3;
    base(h0, 0);  // te = A^-1 H_eo p
    h0.in = cv(p);
    h0.out = te;
    h0.scale = R(1);
    h0.epi_scan = 1;
    h0.es_tab = dscan;
    base(h1, 1);  // q = p - 1/4 A^-1 H_oe te (stored in FP64 only), |q|^2, and to = A^-dag q
    h1.in = cv(te);
    h1.out = q;
    h1.scale = R(-0.25);
    h1.epi_scan = 1;
    h1.es_tab = dscan;
    h1.x = cv(p);
    h1.ax = R(1);
    h1.norm_partials = part;
    h1.out2 = to;
    h1.es2_tab = dscan + K0;
    base(h2, 0);  // te = A^-dag H^dag_eo to
    h2.in = cv(to);
    h2.out = te;
    h2.scale = R(1);
    h2.epi_scan = 1;
    h2.es_tab = dscan + 2 * K0;
    base(h3, 1);  // r -= alpha (q - 1/4 H^dag_oe te), |r|^2 (q = A^dag to unless stored)
    h3.in = cv(te);
    h3.out = Half<Pi>{nullptr, nullptr};
    h3.scale = R(-0.25);
    h3.x = QREB ? cv(to) : cv(q);
    if (QREB) {
      h3.x_es2 = 1;
      h3.es2_tab = dscan + 3 * K0;
    }
    h3.ax = R(1);
    h3.norm_partials = part;
    h3.cg_r = r;
    h3.cg_scalars = sc;
    // every operand of the four stages is one of the iteration's own buffers (or absent)
    for (const HopArgs<Pi>* h : {&h0, &h1, &h2, &h3}) {
      const void* bufs[] = {p.data, te.data, to.data, q.data, r.data};
      auto known = [&](const void* v, bool may_be_null) {
        if (!v) return may_be_null;
        for (const void* b : bufs)
          if (v == b) return true;
        return false;
      };
      if (!known(h->in.data, false) || !known(h->out.data, true) || !known(h->x.data, true) ||
          !known(h->out2.data, true) || !known(h->cg_r.data, true) || (h->norm_partials && h->norm_partials != part))
        throw Error{DWF_ERR_ARG, "internal: an interleaved hop operand is not one of the iteration's buffers"};
    }
    launch(h0, false);
    launch(h1, false);
    for (int k = 0; k < K; ++k)
      DWF_CHECK_LAUNCH(launch_reduce(part + size_t(k) * pstride, nb, 1, sc + size_t(k) * S_COUNT, S_QQ, 1, s, pend.n));
    pend.p[pend.n] = cv(p);
    pend.slot[pend.n] = pend.n;
    ++pend.n;
    launch(h2, true);
    launch(h3, true);
    for (int k = 0; k < K; ++k)
      DWF_CHECK_LAUNCH(launch_reduce(part + size_t(k) * pstride, nb, 1, sc + size_t(k) * S_COUNT, S_RRNEW, 0, s));
    if (pend.n == KX) flush();
    DWF_CHECK_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * size_t(K) * S_COUNT, hipMemcpyDeviceToHost, s));
    DWF_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<double> rr_new(K), beta(K, 0.0);
    std::vector<int> ru, restart(K, 0), keep(K, 1);
    for (int r2 = 0; r2 < K; ++r2) {
      BatchSys& b = *sys[seg[r2]];
      b.st.iters++;
      rr_new[r2] = hsc[size_t(r2) * S_COUNT + S_RRNEW];
      if (!std::isfinite(rr_new[r2])) throw Error{DWF_ERR_NAN, "non-finite residual in batched CG"};
      if (MIXED && (rr_new[r2] < delta * delta * b.rr_max || rr_new[r2] <= b.target || rr_new[r2] > 1e4 * b.rr_true))
        ru.push_back(r2);
    }
    if (!ru.empty()) {
      // reliable updates: fold the increments into the FP64 solutions, recompute the residuals
      flush();
      for (int r2 : ru) {
        BatchSys& b = *sys[seg[r2]];
        const bool diverging = rr_new[r2] > 1e4 * b.rr_true;
        DWF_CHECK_LAUNCH(launch_ilv_accumulate<PX>(b.x, HX(xlb, LT), LT, r2, ns, RS, s));
        rr_new[r2] = true_residual(b);
        DWF_CHECK_LAUNCH((launch_ilv_move<P64, Pi>(chview<P64>(rhi_raw, g, RS), RS, 0, r, LT, r2, ns, RS, s)));
        b.rr_max = b.rr_true = rr_new[r2];
        b.st.reliable_updates++;
        restart[r2] = rr_new[r2] > b.target && (RESTART || diverging);
      }
    }
    int leaving = 0;
    for (int r2 = 0; r2 < K; ++r2) {
      BatchSys& b = *sys[seg[r2]];
      if (rr_new[r2] <= b.target || b.st.iters >= b.cap) {  // converged, or out of iterations
        b.rr = rr_new[r2];
        b.active = false;
        keep[r2] = 0;
        ++leaving;
        continue;
      }
      beta[r2] = restart[r2] ? 0.0 : rr_new[r2] / b.rr;
      b.rr = rr_new[r2];
      if (b.rr > b.rr_max) b.rr_max = b.rr;
    }
    if (leaving) {
      // every increment into its FP64 solution, then the staying right-hand sides moved together
      flush();
      for (int r2 = 0; r2 < K; ++r2)
        DWF_CHECK_LAUNCH(launch_ilv_accumulate<PX>(sys[seg[r2]]->x, HX(xlb, LT), LT, r2, ns, RS, s));
      std::vector<int> nseg;
      std::vector<double> nbeta;
      for (int r2 = 0; r2 < K; ++r2)
        if (keep[r2]) {
          nseg.push_back(seg[r2]);
          nbeta.push_back(beta[r2]);
        }
      const int K2 = int(nseg.size()), LT2 = K2 * RS;
      for (int j = 0, r2 = 0; r2 < K; ++r2) {
        if (!keep[r2]) continue;
        DWF_CHECK_LAUNCH((launch_ilv_move<Pi, Pi>(cv(H(rb, LT)), LT, r2, H(teb, LT2), LT2, j, ns, RS, s)));
        DWF_CHECK_LAUNCH((launch_ilv_move<Pi, Pi>(cv(H(pb[cur], LT)), LT, r2, H(tob, LT2), LT2, j, ns, RS, s)));
        ++j;
      }
      std::swap(rb, teb);
      std::swap(pb[cur], tob);
      seg = nseg;
      beta = nbeta;
      K = K2;
      LT = LT2;
      if (K == 0) break;
      DWF_CHECK_LAUNCH(launch_zero(xlb, half_bytes<PX>(ns, LT), s));
      upload_tables();
    }
    p_update(beta);
  }
  if (K > 0) {
    flush();
    for (int r2 = 0; r2 < K; ++r2)
      DWF_CHECK_LAUNCH(launch_ilv_accumulate<PX>(sys[seg[r2]]->x, HX(xlb, LT), LT, r2, ns, RS, s));
  }
  for (BatchSys* b : sys)
    if (b->rhs2 > 0.0) b->st.last_rel = std::sqrt(b->rr / b->rhs2);
  DWF_CHECK_HIP(hipStreamSynchronize(s));  // (the pinned mirrors are freed on return)
}

// Right-hand sides on separate fields: the single-field fused hops, one launch per lattice and
// stage over all of them (hop_batch_kernel).
template <typename Pi>
static void cg_batched_fields(dwf_ctx* ctx, std::vector<BatchSys>& S, int maxit, double delta) {
  constexpr bool MIXED = !std::is_same<Pi, P64>::value;
  using PX = typename IncrementPrec<Pi>::type;
  constexpr bool RESTART = std::is_same<Pi, PB16>::value;
  constexpr int KX = 8;
  hipStream_t s = ctx->stream;
  const int K = int(S.size());
  (void)maxit;
  // per-system iteration state
  struct Inner {
    std::unique_ptr<Op<Pi>> op;
    LaunchCfg cfg;
    Half<Pi> r, q, te, to, fp;
    Half<PX> xl;
    Half<Pi> pr[KX];
    int cur = 0;
    XFlush<Pi> pend;
    double* sc = nullptr;
    double* part = nullptr;
    int nb = 0;          // workgroups of one field in a batched hop (= partials per stage)
    bool out2 = false;   // A^-dag q as the second output of the second hop
    int group = 0;
  };
  std::vector<Inner> I(K);
  long pstride = 1024;
  size_t hb64max = 0;
  for (auto& b : S) {
    pstride = std::max(pstride, long(reduction_blocks(b.g->nsites * b.p.Ls)));
    pstride = std::max(pstride, b.g->nsites);  // (at least one site per workgroup)
    hb64max = std::max(hb64max, half_size<P64>(b.g, b.p.Ls));
  }
  double* part = reinterpret_cast<double*>(ws_get(ctx, "batch.partials", size_t(K) * pstride * sizeof(double)));
  double* sc = reinterpret_cast<double*>(ws_get(ctx, "batch.scalars", size_t(K) * S_COUNT * sizeof(double)));
  // pinned host scalars and the host table of the four stages' launch arguments (freed on every
  // exit, also when a later allocation throws)
  struct HostFree {
    void* p[2] = {nullptr, nullptr};
    ~HostFree() {
      for (void* q : p)
        if (q) (void)hipHostFree(q);
    }
  } host_free;
  DWF_CHECK_HIP(hipHostMalloc(&host_free.p[0], size_t(K) * S_COUNT * sizeof(double)));
  DWF_CHECK_HIP(hipHostMalloc(&host_free.p[1], size_t(4) * K * sizeof(HopArgs<Pi>)));
  double* hsc = static_cast<double*>(host_free.p[0]);
  HopArgs<Pi>* htab = static_cast<HopArgs<Pi>*>(host_free.p[1]);
  HopArgs<Pi>* dtab = reinterpret_cast<HopArgs<Pi>*>(ws_get(ctx, "batch.table", size_t(4) * K * sizeof(HopArgs<Pi>)));
  // FP64 temporaries shared by the reliable updates (largest system)
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
  const bool moebius = !(S[0].p.b == 1.0 && S[0].p.c == 0.0);
  auto p_update = [&](int k, double beta, double rr_new) {
    Inner& in = I[k];
    BatchSys& b = S[k];
    const long n5 = b.g->nsites * b.p.Ls;
    const int nxt = (in.cur + 1) % KX;
    const Op<Pi>& o = *in.op;
    if (moebius) {
      DWF_CHECK_LAUNCH(launch_cg_pupdate_f<Pi>(cv(in.r), cv(in.pr[in.cur]), in.pr[nxt], in.fp, beta, in.sc, rr_new, n5,
                                               b.p.Ls, o.b, o.c, o.m, s));
    } else {
      DWF_CHECK_LAUNCH(launch_cg_pupdate<Pi>(cv(in.r), cv(in.pr[in.cur]), in.pr[nxt], beta, in.sc, rr_new, n5, b.p.Ls, s));
    }
    in.cur = nxt;
  };
  auto flush = [&](int k) {
    Inner& in = I[k];
    const long n5 = S[k].g->nsites * S[k].p.Ls;
    DWF_CHECK_LAUNCH((launch_xflush<Pi, PX>(in.xl, in.pend, in.sc, n5, S[k].p.Ls, s)));
    in.pend.n = 0;
  };
  // set up and start every system
  for (int k = 0; k < K; ++k) {
    BatchSys& b = S[k];
    Inner& in = I[k];
    const int Ls = b.p.Ls;
    const long n5 = b.g->nsites * Ls;
    const size_t hbi = half_size<Pi>(b.g, Ls);
    const std::string t = "batch." + std::to_string(k) + ".";
    in.op = std::make_unique<Op<Pi>>(ctx, b.g, b.p, b.Ui);
    in.cfg = batch_config(ctx, Pi::ID, Ls);
    in.sc = sc + size_t(k) * S_COUNT;
    in.part = part + size_t(k) * pstride;
    in.nb = int((b.g->nsites + in.cfg.spb - 1) / in.cfg.spb);
    in.out2 = in.op->scan_ok && (Ls == 8 || Ls == 16 || Ls == 32);
    in.r = hview<Pi>(ws_get(ctx, t + "r", hbi), b.g, Ls);
    in.q = hview<Pi>(ws_get(ctx, t + "q", hbi), b.g, Ls);
    in.te = hview<Pi>(ws_get(ctx, t + "te", hbi), b.g, Ls);
    in.to = hview<Pi>(ws_get(ctx, t + "to", hbi), b.g, Ls);
    in.fp = moebius ? hview<Pi>(ws_get(ctx, t + "fp", hbi), b.g, Ls) : Half<Pi>{nullptr, nullptr};
    in.xl = hview<PX>(MIXED ? ws_get(ctx, t + "xlo", half_size<PX>(b.g, Ls)) : (void*)b.x.data, b.g, Ls);
    for (int j = 0; j < KX; ++j) in.pr[j] = hview<Pi>(ws_get(ctx, t + "p" + std::to_string(j), hbi), b.g, Ls);
    b.rhs2 = norm2_sync<P64>(ctx, b.rhs, b.g, Ls);
    b.target = b.tol_n * b.tol_n * b.rhs2;
    b.active = b.rhs2 > 0.0;
    if (!b.active) {
      DWF_CHECK_LAUNCH(launch_zero(b.x.data, half_size<P64>(b.g, Ls), s));
      continue;
    }
    Half<P64> rhi = hview<P64>(rhi_raw, b.g, Ls);
    if (norm2_sync<P64>(ctx, cv(b.x), b.g, Ls) == 0.0) {
      DWF_CHECK_HIP(hipMemcpyAsync(rhi.data, b.rhs.data, half_size<P64>(b.g, Ls), hipMemcpyDeviceToDevice, s));
      b.rr = b.rhs2;
    } else {
      b.rr = true_residual(b);
    }
    if (!std::isfinite(b.rr)) throw Error{DWF_ERR_NAN, "non-finite residual at batched CG start"};
    b.rr_max = b.rr_true = b.rr;
    if (b.rr <= b.target || b.cap <= 0) { b.active = false; continue; }
    if (MIXED) {
      DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(cv(rhi), in.r, n5, Ls, s)));
      DWF_CHECK_LAUNCH(launch_zero(in.xl.data, half_size<PX>(b.g, Ls), s));
    } else {
      DWF_CHECK_HIP(hipMemcpyAsync(in.r.data, rhi.data, half_size<P64>(b.g, Ls), hipMemcpyDeviceToDevice, s));
    }
    p_update(k, 0.0, b.rr);
  }
  // lattices: systems on one geometry with one link field, Ls and epilogue form (the same kernel
  // variant) share the batched launches
  std::vector<int> group_first;
  for (int k = 0; k < K; ++k) {
    int gi = -1;
    for (size_t j = 0; j < group_first.size(); ++j) {
      const int f = group_first[j];
      if (S[f].g == S[k].g && S[f].Ui == S[k].Ui && S[f].p.Ls == S[k].p.Ls && I[f].op->scan_ok == I[k].op->scan_ok)
        gi = int(j);
    }
    if (gi < 0) {
      group_first.push_back(k);
      gi = int(group_first.size()) - 1;
    }
    I[k].group = gi;
  }
  // one launch per lattice and stage over the systems in act (their tables at htab + stage * K)
  std::vector<int> act;
  auto launch_stage = [&](int stage, bool dag, bool pro) {
    for (size_t gi = 0; gi < group_first.size(); ++gi) {
      int first = -1, n = 0;
      for (size_t j = 0; j < act.size(); ++j)
        if (I[act[j]].group == int(gi)) {
          if (first < 0) first = int(j);
          ++n;
        }
      if (n == 0) continue;
      const int k0 = act[first];
      const HopArgs<Pi>& a0 = htab[size_t(stage) * K + first];
      long mark = -1;
      if (ctx->timer.on) mark = timer_begin(ctx, I[k0].op->hop_name(a0, dag, pro, I[k0].cfg, true));
      DWF_CHECK_LAUNCH(launch_hop<Pi>(a0, dag, pro, I[k0].cfg, s, dtab + size_t(stage) * K + first, n));
      if (mark >= 0) timer_end(ctx, mark, double(n) * I[k0].op->hop_bytes(a0));
    }
  };
  int nactive = 0;
  for (auto& b : S) nactive += b.active ? 1 : 0;
  int it = 0;
  while (nactive > 0) {
    // the active systems, grouped by lattice (consecutive table entries of one group)
    act.clear();
    for (size_t gi = 0; gi < group_first.size(); ++gi)
      for (int k = 0; k < K; ++k)
        if (S[k].active && I[k].group == int(gi)) act.push_back(k);
    const int na = int(act.size());
    for (int j = 0; j < na; ++j) {
      const int k = act[j];
      Inner& in = I[k];
      const Op<Pi>& o = *in.op;
      const Half<Pi> p = in.pr[in.cur];
      typename Op<Pi>::CgStep cg;
      cg.r = in.r;
      cg.scalars = in.sc;
      const Half<Pi> q2 = in.out2 ? in.to : Half<Pi>{nullptr, nullptr};
      // q = M p (Moebius: from F p), |q|^2, and A^-dag q
      htab[0 * K + j] = o.hop_args(0, cv(moebius ? in.fp : p), in.te, o.em(moebius ? E_F_AINV : E_AINV), 1.0);
      htab[1 * K + j] = o.hop_args(1, cv(in.te), in.q, o.em(E_AINV), -0.25, cv(p), 1.0, in.part, typename Op<Pi>::CgStep(),
                                   q2, E_AINVDAG);
      // r -= alpha M^dag q, |r|^2
      htab[2 * K + j] = o.hop_args(0, cv(in.to), in.te, o.em(E_AINVDAG_FDAG), 1.0);
      htab[3 * K + j] = o.hop_args(1, cv(in.te), Half<Pi>{nullptr, nullptr}, moebius ? o.em(E_FDAG) : nullptr, -0.25,
                                   cv(in.q), 1.0, in.part, cg);
    }
    for (int stage = 0; stage < 4; ++stage)
      DWF_CHECK_HIP(hipMemcpyAsync(dtab + size_t(stage) * K, htab + size_t(stage) * K, na * sizeof(HopArgs<Pi>),
                                   hipMemcpyHostToDevice, s));
    launch_stage(0, false, false);
    launch_stage(1, false, false);
    for (int k : act) {
      Inner& in = I[k];
      if (!in.out2)
        in.op->fifth(cv(in.q), in.to, E_AINVDAG);  // A^-dag q (dense-epilogue extents)
      DWF_CHECK_LAUNCH(launch_reduce(in.part, in.nb, 1, in.sc, S_QQ, 1, s, in.pend.n));
      in.pend.p[in.pend.n] = cv(in.pr[in.cur]);
      in.pend.slot[in.pend.n] = in.pend.n;
      ++in.pend.n;
    }
    launch_stage(2, true, false);
    launch_stage(3, true, false);
    for (int k : act) {
      Inner& in = I[k];
      DWF_CHECK_LAUNCH(launch_reduce(in.part, in.nb, 1, in.sc, S_RRNEW, 0, s));
      if (in.pend.n == KX) flush(k);
    }
    DWF_CHECK_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * size_t(K) * S_COUNT, hipMemcpyDeviceToHost, s));
    DWF_CHECK_HIP(hipStreamSynchronize(s));
    ++it;
    bool changed = false;
    for (int k : act) {
      BatchSys& b = S[k];
      Inner& in = I[k];
      const int Ls = b.p.Ls;
      const long n5 = b.g->nsites * Ls;
      b.st.iters++;
      double rr_new = hsc[size_t(k) * S_COUNT + S_RRNEW];
      if (!std::isfinite(rr_new)) throw Error{DWF_ERR_NAN, "non-finite residual in batched CG"};
      const bool diverging = rr_new > 1e4 * b.rr_true;
      bool restart = false;
      if (MIXED && (rr_new < delta * delta * b.rr_max || rr_new <= b.target || diverging)) {
        // reliable update: fold the increment into the FP64 solution, recompute r in FP64
        flush(k);
        DWF_CHECK_LAUNCH(launch_accumulate<PX>(b.x, in.xl, n5, Ls, s));
        rr_new = true_residual(b);
        DWF_CHECK_LAUNCH((launch_convert<P64, Pi>(chview<P64>(rhi_raw, b.g, Ls), in.r, n5, Ls, s)));
        b.rr_max = b.rr_true = rr_new;
        b.st.reliable_updates++;
        restart = rr_new > b.target && (RESTART || diverging);
      }
      if (rr_new <= b.target || b.st.iters >= b.cap) {  // converged, or out of iterations
        b.rr = rr_new;
        b.active = false;
        changed = true;
        continue;
      }
      const double beta = restart ? 0.0 : rr_new / b.rr;
      p_update(k, beta, rr_new);
      b.rr = rr_new;
      if (b.rr > b.rr_max) b.rr_max = b.rr;
    }
    if (changed) {
      nactive = 0;
      for (auto& b : S) nactive += b.active ? 1 : 0;
    }
  }
  for (int k = 0; k < K; ++k) {
    BatchSys& b = S[k];
    if (b.rhs2 <= 0.0) continue;
    if (I[k].pend.n) flush(k);
    if (MIXED) DWF_CHECK_LAUNCH(launch_accumulate<PX>(b.x, I[k].xl, b.g->nsites * b.p.Ls, b.p.Ls, s));
    b.st.last_rel = std::sqrt(b.rr / b.rhs2);
  }
  DWF_CHECK_HIP(hipStreamSynchronize(s));  // (the pinned tables are freed on return)
}

// The batched CG: the right-hand sides that can be interleaved (Shamir operator, Ls 8, 16 or 32,
// recurrence-form blocks; per lattice, at most 256 / Ls at a time) run interleaved, the others on
// separate fields.
template <typename Pi>
static void cg_batched(dwf_ctx* ctx, std::vector<BatchSys>& S, int maxit, double delta) {
  std::vector<char> done(S.size(), 0);
  for (size_t k = 0; k < S.size(); ++k) {
    const dwf_params& p = S[k].p;
    const bool ok = p.b == 1.0 && p.c == 0.0 && !p.b_s && !p.c_s && (p.Ls == 8 || p.Ls == 16 || p.Ls == 32) &&
                    !ilv_config(ctx, Pi::ID, p.Ls).off;
    if (!ok || done[k]) continue;
    FifthScan<double> e;
    bool scan = true;
    for (int slot = 0; scan && slot < E_COUNT; ++slot) scan = fifth_scan(p.Ls, p.M5, p.mass, p.b, p.c, slot, &e);
    if (!scan) continue;
    std::vector<BatchSys*> chunk;
    for (size_t j = k; j < S.size() && int(chunk.size()) < 256 / p.Ls; ++j) {
      const dwf_params& q = S[j].p;
      if (done[j] || S[j].g != S[k].g || S[j].Ui != S[k].Ui || q.Ls != p.Ls || !(q.b == 1.0 && q.c == 0.0) || q.b_s ||
          q.c_s)
        continue;
      bool sj = true;
      for (int slot = 0; sj && slot < E_COUNT; ++slot) sj = fifth_scan(q.Ls, q.M5, q.mass, q.b, q.c, slot, &e);
      if (!sj) continue;
      chunk.push_back(&S[j]);
      done[j] = 1;
    }
    cg_batched_ilv<Pi>(ctx, chunk, delta);
  }
  std::vector<BatchSys> rest;
  std::vector<size_t> idx;
  for (size_t k = 0; k < S.size(); ++k)
    if (!done[k]) idx.push_back(k);
  if (idx.empty()) return;
  if (idx.size() == S.size()) {
    cg_batched_fields<Pi>(ctx, S, maxit, delta);
    return;
  }
  rest.reserve(idx.size());
  for (size_t k : idx) rest.push_back(std::move(S[k]));
  cg_batched_fields<Pi>(ctx, rest, maxit, delta);
  for (size_t j = 0; j < idx.size(); ++j) S[idx[j]] = std::move(rest[j]);
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
// tol_n, checked by the FP64 true residual ||phi - M^dag M X|| / ||phi|| recomputed after the
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
