// extern "C" boundary: argument validation, dispatch on storage precision,
// error mapping.  No C++ exception crosses this file.
#include "runtime.hpp"
#include "solver.hpp"

namespace dwf {
const char* last_error();
}

using namespace dwf;

namespace {

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return DWF_ERR_HIP;
  } catch (...) {
    set_error("unknown error");
    return DWF_ERR_HIP;
  }
}

int check_params(const dwf_params* p, bool need_solver = false) {
  if (!p) return fail(DWF_ERR_ARG, "params is NULL");
  for (int k = 0; k < 4; ++k)
    if (p->dims[k] < 2 || (p->dims[k] & 1))
      return fail(DWF_ERR_ARG, "every lattice extent must be even and >= 2");
  if (p->Ls < 2 || p->Ls > 128) return fail(DWF_ERR_ARG, "Ls must be in [2, 128]");
  if (p->tbc != 0 && p->tbc != 1) return fail(DWF_ERR_ARG, "tbc must be 0 or 1");
  if (p->prec < 0 || p->prec > 3) return fail(DWF_ERR_ARG, "unknown storage precision");
  if (need_solver && (p->prec_inner < 0 || p->prec_inner > 3))
    return fail(DWF_ERR_ARG, "unknown inner precision");
  if (!std::isfinite(p->M5) || !std::isfinite(p->mass) || !std::isfinite(p->b) || !std::isfinite(p->c))
    return fail(DWF_ERR_ARG, "non-finite operator parameter");
  for (int s = 0; s < p->Ls; ++s) {
    if ((p->b_s && !std::isfinite(p->b_s[s])) || (p->c_s && !std::isfinite(p->c_s[s])))
      return fail(DWF_ERR_ARG, "non-finite s-dependent Moebius coefficient");
    const double bb = p->b_s ? p->b_s[s] : p->b;
    if (std::fabs(bb * (4.0 - p->M5) + 1.0) < 1e-12) return fail(DWF_ERR_ARG, "b_s (4 - M5) + 1 = 0: singular A");
  }
  const double V = double(p->dims[0]) * p->dims[1] * p->dims[2] * p->dims[3];
  if (8.0 * V >= 2147483648.0) return fail(DWF_ERR_ARG, "lattice volume too large");
  return DWF_OK;
}

size_t elem_size(int prec) {
  switch (prec) {
    case DWF_FP64: return sizeof(double2);
    case DWF_FP32: return sizeof(float2);
    default: return 4;
  }
}

size_t half_bytes_p(long nsites, int Ls, int prec) {
  switch (prec) {
    case DWF_FP64: return half_bytes<P64>(nsites, Ls);
    case DWF_FP32: return half_bytes<P32>(nsites, Ls);
    case DWF_FP16: return half_bytes<P16>(nsites, Ls);
    default: return half_bytes<PB16>(nsites, Ls);
  }
}

template <typename P>
int pack_t(dwf_ctx* ctx, const dwf_params* p, int kind, const void* natural, void* packed) {
  const Geometry* g = geometry(ctx, p->dims, p->tbc);
  const GeomTables t = g->tables();
  const double2* nat = reinterpret_cast<const double2*>(natural);
  if (kind == DWF_KIND_GAUGE) {
    DWF_CHECK_LAUNCH(launch_pack_gauge<P>(t, nat, reinterpret_cast<typename P::S*>(packed), ctx->stream));
  } else {
    const size_t hb = half_bytes<P>(g->nsites, p->Ls);
    for (int par = 0; par < 2; ++par) {
      if (kind == DWF_KIND_EVEN && par == 1) continue;
      if (kind == DWF_KIND_ODD && par == 0) continue;
      char* base = reinterpret_cast<char*>(packed) + (kind == DWF_KIND_FULL && par == 1 ? hb : 0);
      DWF_CHECK_LAUNCH(launch_pack_half<P>(t, par, p->Ls, nat, half_view<P>(base, g->nsites, p->Ls), ctx->stream));
    }
  }
  return DWF_OK;
}

template <typename P>
int unpack_t(dwf_ctx* ctx, const dwf_params* p, int kind, const void* packed, void* natural) {
  const Geometry* g = geometry(ctx, p->dims, p->tbc);
  const GeomTables t = g->tables();
  double2* nat = reinterpret_cast<double2*>(natural);
  const size_t hb = half_bytes<P>(g->nsites, p->Ls);
  for (int par = 0; par < 2; ++par) {
    if (kind == DWF_KIND_EVEN && par == 1) continue;
    if (kind == DWF_KIND_ODD && par == 0) continue;
    const char* base = reinterpret_cast<const char*>(packed) + (kind == DWF_KIND_FULL && par == 1 ? hb : 0);
    DWF_CHECK_LAUNCH(launch_unpack_half<P>(t, par, p->Ls, chalf_view<P>(base, g->nsites, p->Ls), nat, ctx->stream));
  }
  return DWF_OK;
}

template <typename P>
int dslash_t(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op, int parity,
             int dagger) {
  const Geometry* g = geometry(ctx, p.dims, p.tbc);
  Op<P> o(ctx, g, p, U);
  const int Ls = p.Ls;
  const size_t hb = half_bytes<P>(g->nsites, Ls);
  switch (op) {
    case DWF_OP_HOP: {
      // H F in (or (H F)^dag = F^dag H^dag in)
      if (!dagger) o.hop(parity, chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), false, true, 1.0, nullptr);
      else
        o.hop(parity, chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), true, false, 1.0,
              o.moebius ? o.em(E_FDAG) : nullptr);
      return DWF_OK;
    }
    case DWF_OP_MPREC: {
      void* t1 = ws_get(ctx, "dslash.t1", hb);
      void* t2 = ws_get(ctx, "dslash.t2", hb);
      if (!dagger) o.mprec(chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), half_view<P>(t1, g->nsites, Ls));
      else
        o.mprec_dag(chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), half_view<P>(t1, g->nsites, Ls),
                    half_view<P>(t2, g->nsites, Ls));
      return DWF_OK;
    }
    case DWF_OP_FULL: {
      const char* ib = reinterpret_cast<const char*>(in);
      char* ob = reinterpret_cast<char*>(out);
      o.full(chalf_view<P>(ib, g->nsites, Ls), chalf_view<P>(ib + hb, g->nsites, Ls), half_view<P>(ob, g->nsites, Ls),
             half_view<P>(ob + hb, g->nsites, Ls), dagger != 0);
      return DWF_OK;
    }
    case DWF_OP_A:
      o.fifth(chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), dagger ? E_ADAG : E_A);
      return DWF_OK;
    case DWF_OP_AINV:
      o.fifth(chalf_view<P>(in, g->nsites, Ls), half_view<P>(out, g->nsites, Ls), dagger ? E_AINVDAG : E_AINV);
      return DWF_OK;
    default:
      return fail(DWF_ERR_ARG, "unknown op");
  }
}

int dslash_any(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int parity,
               int dagger, bool moebius) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!U || !in || !out) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (in == out) return fail(DWF_ERR_ARG, "in and out must not alias");
  if (parity != 0 && parity != 1) return fail(DWF_ERR_ARG, "parity must be 0 or 1");
  if (op < DWF_OP_HOP || op > DWF_OP_AINV) return fail(DWF_ERR_ARG, "unknown op");
  dwf_params q = *p;
  if (!moebius) {
    q.b = 1.0;
    q.c = 0.0;
    q.b_s = nullptr;
    q.c_s = nullptr;
  }
  return guarded([&]() {
    switch (q.prec) {
      case DWF_FP64: return dslash_t<P64>(ctx, q, U, in, out, op, parity, dagger);
      case DWF_FP32: return dslash_t<P32>(ctx, q, U, in, out, op, parity, dagger);
      case DWF_FP16: return dslash_t<P16>(ctx, q, U, in, out, op, parity, dagger);
      default: return dslash_t<PB16>(ctx, q, U, in, out, op, parity, dagger);
    }
  });
}

}  // namespace

extern "C" {

const char* dwf_last_error(void) { return dwf::last_error(); }

int dwf_ctx_create(dwf_ctx** out, void* stream) {
  if (!out) return fail(DWF_ERR_ARG, "ctx out-pointer is NULL");
  return guarded([&]() {
    std::unique_ptr<dwf_ctx> c(new dwf_ctx());  // (freed if a step below fails)
    c->stream = reinterpret_cast<hipStream_t>(stream);
    DWF_CHECK_HIP(hipGetDevice(&c->device));
    scratch_init();  // device address of the no-allocation entry point's array on this device
    DWF_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_scalars), S_COUNT * sizeof(double)));
    *out = c.release();
    return DWF_OK;
  });
}

int dwf_ctx_destroy(dwf_ctx* ctx) {
  if (!ctx) return DWF_OK;
  return guarded([&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->ws) (void)hipFree(kv.second.first);
    for (auto& kv : ctx->emats) (void)hipFree(kv.second.first);
    ctx->geoms.clear();
    timer_release(ctx);
    if (ctx->h_scalars) (void)hipHostFree(ctx->h_scalars);
    delete ctx;
    return DWF_OK;
  });
}

int dwf_ctx_release(dwf_ctx* ctx) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  return guarded([&]() {
    DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& kv : ctx->ws) DWF_CHECK_HIP(hipFree(kv.second.first));
    ctx->ws.clear();
    return DWF_OK;
  });
}

int dwf_ctx_set_stream(dwf_ctx* ctx, void* stream) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return DWF_OK;
}

size_t dwf_field_bytes(const dwf_params* p, int kind, int prec) {
  if (check_params(p) != DWF_OK || prec < 0 || prec > 3) return 0;
  const long V = long(p->dims[0]) * p->dims[1] * p->dims[2] * p->dims[3];
  const long ns = V / 2;
  switch (kind) {
    case DWF_KIND_GAUGE: return size_t(2) * ns * 72 * elem_size(prec);
    case DWF_KIND_FULL: return 2 * half_bytes_p(ns, p->Ls, prec);
    case DWF_KIND_EVEN:
    case DWF_KIND_ODD: return half_bytes_p(ns, p->Ls, prec);
    default: return 0;
  }
}

int dwf_pack(dwf_ctx* ctx, const dwf_params* p, int kind, int prec, const void* natural, void* packed) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!natural || !packed) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (kind < 0 || kind > 3 || prec < 0 || prec > 3) return fail(DWF_ERR_ARG, "bad kind or precision");
  return guarded([&]() {
    switch (prec) {
      case DWF_FP64: return pack_t<P64>(ctx, p, kind, natural, packed);
      case DWF_FP32: return pack_t<P32>(ctx, p, kind, natural, packed);
      case DWF_FP16: return pack_t<P16>(ctx, p, kind, natural, packed);
      default: return pack_t<PB16>(ctx, p, kind, natural, packed);
    }
  });
}

int dwf_unpack(dwf_ctx* ctx, const dwf_params* p, int kind, int prec, const void* packed, void* natural) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!natural || !packed) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (kind < 1 || kind > 3 || prec < 0 || prec > 3) return fail(DWF_ERR_ARG, "bad kind or precision (gauge unpack unsupported)");
  return guarded([&]() {
    switch (prec) {
      case DWF_FP64: return unpack_t<P64>(ctx, p, kind, packed, natural);
      case DWF_FP32: return unpack_t<P32>(ctx, p, kind, packed, natural);
      case DWF_FP16: return unpack_t<P16>(ctx, p, kind, packed, natural);
      default: return unpack_t<PB16>(ctx, p, kind, packed, natural);
    }
  });
}

int dwf_convert(dwf_ctx* ctx, const dwf_params* p, int kind, int prec_in, const void* in, int prec_out, void* out) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!in || !out) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (kind < 0 || kind > 3 || prec_in < 0 || prec_in > 3 || prec_out < 0 || prec_out > 3)
    return fail(DWF_ERR_ARG, "bad kind or precision");
  if (prec_in != DWF_FP64 && prec_out != DWF_FP64) return fail(DWF_ERR_ARG, "one side of a conversion must be FP64");
  return guarded([&]() {
    const Geometry* g = geometry(ctx, p->dims, p->tbc);
    const int Ls = p->Ls;
    const long ns = g->nsites;
    if (kind == DWF_KIND_GAUGE) {
      if (prec_in != DWF_FP64) throw Error{DWF_ERR_ARG, "gauge conversion is FP64 -> lower only"};
      const long n = 2 * ns * 72;
      const double2* src = reinterpret_cast<const double2*>(in);
      switch (prec_out) {
        case DWF_FP64: DWF_CHECK_HIP(hipMemcpyAsync(out, in, n * sizeof(double2), hipMemcpyDeviceToDevice, ctx->stream)); break;
        case DWF_FP32: DWF_CHECK_LAUNCH((launch_convert_links<P64, P32>(src, reinterpret_cast<P32::S*>(out), n, ctx->stream))); break;
        case DWF_FP16: DWF_CHECK_LAUNCH((launch_convert_links<P64, P16>(src, reinterpret_cast<P16::S*>(out), n, ctx->stream))); break;
        default: DWF_CHECK_LAUNCH((launch_convert_links<P64, PB16>(src, reinterpret_cast<PB16::S*>(out), n, ctx->stream))); break;
      }
      return DWF_OK;
    }
    const int halves = kind == DWF_KIND_FULL ? 2 : 1;
    const size_t hbi = half_bytes_p(ns, Ls, prec_in), hbo = half_bytes_p(ns, Ls, prec_out);
    for (int h = 0; h < halves; ++h) {
      const void* a = reinterpret_cast<const char*>(in) + h * hbi;
      void* b = reinterpret_cast<char*>(out) + h * hbo;
      const long n5 = ns * Ls;
      if (prec_in == DWF_FP64) {
        switch (prec_out) {
          case DWF_FP64: DWF_CHECK_HIP(hipMemcpyAsync(b, a, hbi, hipMemcpyDeviceToDevice, ctx->stream)); break;
          case DWF_FP32: DWF_CHECK_LAUNCH((launch_convert<P64, P32>(chalf_view<P64>(a, ns, Ls), half_view<P32>(b, ns, Ls), n5, Ls, ctx->stream))); break;
          case DWF_FP16: DWF_CHECK_LAUNCH((launch_convert<P64, P16>(chalf_view<P64>(a, ns, Ls), half_view<P16>(b, ns, Ls), n5, Ls, ctx->stream))); break;
          default: DWF_CHECK_LAUNCH((launch_convert<P64, PB16>(chalf_view<P64>(a, ns, Ls), half_view<PB16>(b, ns, Ls), n5, Ls, ctx->stream))); break;
        }
      } else {
        switch (prec_in) {
          case DWF_FP32: DWF_CHECK_LAUNCH((launch_convert<P32, P64>(chalf_view<P32>(a, ns, Ls), half_view<P64>(b, ns, Ls), n5, Ls, ctx->stream))); break;
          case DWF_FP16: DWF_CHECK_LAUNCH((launch_convert<P16, P64>(chalf_view<P16>(a, ns, Ls), half_view<P64>(b, ns, Ls), n5, Ls, ctx->stream))); break;
          default: DWF_CHECK_LAUNCH((launch_convert<PB16, P64>(chalf_view<PB16>(a, ns, Ls), half_view<P64>(b, ns, Ls), n5, Ls, ctx->stream))); break;
        }
      }
    }
    return DWF_OK;
  });
}

int dwf_dslash(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int parity,
               int dagger) {
  return dslash_any(ctx, p, U, in, out, op, parity, dagger, false);
}

int mobius_dslash(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int parity,
                  int dagger) {
  return dslash_any(ctx, p, U, in, out, op, parity, dagger, true);
}

int dwf_dslash_noalloc(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op,
                       int parity, int dagger) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!U || !in || !out) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (in == out) return fail(DWF_ERR_ARG, "in and out must not alias");
  if (parity != 0 && parity != 1) return fail(DWF_ERR_ARG, "parity must be 0 or 1");
  if (op < DWF_OP_HOP || op > DWF_OP_AINV) return fail(DWF_ERR_ARG, "unknown op");
  dwf_params q = *p;  // the Shamir operator, as dwf_dslash
  q.b = 1.0;
  q.c = 0.0;
  q.b_s = nullptr;
  q.c_s = nullptr;
  return guarded([&]() { return dslash_noalloc(ctx, q, U, in, out, op, parity, dagger); });
}

int cg_ne(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* b, void* x, dwf_solve_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p, true);
  if (rc) return rc;
  if (!U || !b || !x || !info) return fail(DWF_ERR_ARG, "NULL pointer");
  if (b == x) return fail(DWF_ERR_ARG, "b and x must not alias");
  if (!(info->tol > 0.0)) return fail(DWF_ERR_ARG, "tol must be positive");
  return guarded([&]() {
    const double delta = info->delta > 0 ? info->delta : 0.1;
    const int maxit = info->maxit > 0 ? info->maxit : 100000;
    const int st = solve_full(ctx, *p, U, b, x, info->tol, maxit, delta, "cg", info);
    if (st != 0) set_error("cg_ne: iteration cap reached before the true residual met tol");
    return st == 0 ? DWF_OK : DWF_NOT_CONVERGED;
  });
}

int cg_ne_5d(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* b, void* x, dwf_solve_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p, true);
  if (rc) return rc;
  if (!U || !b || !x || !info) return fail(DWF_ERR_ARG, "NULL pointer");
  if (b == x) return fail(DWF_ERR_ARG, "b and x must not alias");
  if (!(info->tol > 0.0)) return fail(DWF_ERR_ARG, "tol must be positive");
  return guarded([&]() {
    const double delta = info->delta > 0 ? info->delta : 0.1;
    const int maxit = info->maxit > 0 ? info->maxit : 100000;
    const int st = solve_full_5d(ctx, *p, U, b, x, info->tol, maxit, delta, "cg5", info);
    if (st != 0) set_error("cg_ne_5d: iteration cap reached before the true residual met tol");
    return st == 0 ? DWF_OK : DWF_NOT_CONVERGED;
  });
}

int dwf_dslash_5d(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* in, void* out, int op, int dagger) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p);
  if (rc) return rc;
  if (!U || !in || !out) return fail(DWF_ERR_ARG, "NULL field pointer");
  if (in == out) return fail(DWF_ERR_ARG, "in and out must not alias");
  if (op != DWF_OP5_HOP && op != DWF_OP5_SCHUR) return fail(DWF_ERR_ARG, "unknown op");
  return guarded([&]() { return dslash_5d(ctx, *p, U, in, out, op, dagger); });
}

int cg_ne_batched(dwf_ctx* ctx, int nrhs, const dwf_params* per_rhs, const void* const* U, const void* const* b,
                  void* const* x, dwf_solve_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  if (nrhs < 1 || nrhs > 64 || !per_rhs || !U || !b || !x || !info) return fail(DWF_ERR_ARG, "bad batched arguments");
  for (int k = 0; k < nrhs; ++k) {
    int rc = check_params(&per_rhs[k], true);
    if (rc) return rc;
    if (!U[k] || !b[k] || !x[k]) return fail(DWF_ERR_ARG, "NULL pointer in the batch");
    if (b[k] == x[k]) return fail(DWF_ERR_ARG, "b and x must not alias");
    if (!(info[k].tol > 0.0)) return fail(DWF_ERR_ARG, "tol must be positive");
    if (per_rhs[k].b_s || per_rhs[k].c_s)
      return fail(DWF_ERR_ARG, "s-dependent Moebius coefficients are not supported by the batched solver");
    if (per_rhs[k].M5 != per_rhs[0].M5 || per_rhs[k].b != per_rhs[0].b || per_rhs[k].c != per_rhs[0].c ||
        per_rhs[k].tbc != per_rhs[0].tbc || per_rhs[k].prec_inner != per_rhs[0].prec_inner)
      return fail(DWF_ERR_ARG, "batched right-hand sides must share M5, b, c, tbc and prec_inner");
    for (int j = 0; j < k; ++j)
      if (x[j] == x[k]) return fail(DWF_ERR_ARG, "solution fields must be distinct");
  }
  return guarded([&]() {
    const int st = solve_batched(ctx, nrhs, per_rhs, U, b, x, info);
    if (st != 0) set_error("cg_ne_batched: iteration cap reached before every true residual met tol");
    return st == 0 ? DWF_OK : DWF_NOT_CONVERGED;
  });
}

int mobius_accel_solve(dwf_ctx* ctx, const dwf_params* target, const dwf_params* inner, const void* U, const void* b,
                       void* x, dwf_madwf_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(target, true);
  if (rc) return rc;
  rc = check_params(inner, true);
  if (rc) return rc;
  if (!U || !b || !x || !info) return fail(DWF_ERR_ARG, "NULL pointer");
  for (int d = 0; d < 4; ++d)
    if (target->dims[d] != inner->dims[d]) return fail(DWF_ERR_ARG, "target and inner must share the 4D lattice");
  if (target->M5 != inner->M5 || target->mass != inner->mass || target->tbc != inner->tbc)
    return fail(DWF_ERR_ARG, "target and inner must share M5, mass and boundary conditions");
  if (info->n_dc < 0 || info->n_dc > 8) return fail(DWF_ERR_ARG, "n_dc must be in [0, 8]");
  if (!(info->tol > 0) || !(info->tol_pv > 0) || !(info->tol_mobius > 0)) return fail(DWF_ERR_ARG, "tolerances must be positive");
  if (info->prec_pv < 0 || info->prec_pv > 3 || info->prec_final < 0 || info->prec_final > 3)
    return fail(DWF_ERR_ARG, "unknown precision");
  return guarded([&]() {
    dwf_params t = *target;
    t.b = 1.0;
    t.c = 0.0;
    t.b_s = nullptr;
    t.c_s = nullptr;
    const int st = madwf(ctx, t, *inner, U, b, x, info);
    return st == 0 ? DWF_OK : DWF_NOT_CONVERGED;
  });
}

int fermion_force(dwf_ctx* ctx, const dwf_params* p, const void* U, const void* phi, void* F, double* S,
                  double tau_fg, int out_kind, void* x_io, dwf_solve_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p, true);
  if (rc) return rc;
  if (!U || !phi || !F) return fail(DWF_ERR_ARG, "NULL pointer");
  if (out_kind != 0 && out_kind != 1) return fail(DWF_ERR_ARG, "out_kind must be 0 or 1");
  if (!(tau_fg >= 0.0) || !std::isfinite(tau_fg)) return fail(DWF_ERR_ARG, "tau_fg must be >= 0");
  return guarded([&]() { return dwf::fermion_force(ctx, *p, U, phi, F, S, tau_fg, out_kind, x_io, info); });
}

int hmc_fgi_trajectory(dwf_ctx* ctx, const dwf_params* p, void* U, void* P, const void* phi, dwf_hmc_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p, true);
  if (rc) return rc;
  if (!U || !P || !phi || !info) return fail(DWF_ERR_ARG, "NULL pointer");
  if (info->n_steps < 0 || !(info->tau > 0.0) || !std::isfinite(info->tau) || !std::isfinite(info->beta))
    return fail(DWF_ERR_ARG, "need tau > 0, n_steps >= 0, finite beta");
  return guarded([&]() { return dwf::fgi_trajectory(ctx, *p, U, P, phi, info); });
}

int quotient_force(dwf_ctx* ctx, const dwf_params* p, int nq, const double* masses, const void* U,
                   const void* const* phi, void* F, double* S, int out_kind, void* const* x_io,
                   dwf_solve_info* info) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  int rc = check_params(p, true);
  if (rc) return rc;
  if (nq < 1 || nq > 64) return fail(DWF_ERR_ARG, "nq must be in 1..64");
  if (p->b_s || p->c_s)
    return fail(DWF_ERR_ARG, "s-dependent Moebius coefficients are not supported by the batched solver");
  if (!masses || !U || !phi || !F) return fail(DWF_ERR_ARG, "NULL pointer");
  for (int i = 0; i < nq; ++i)
    if (!phi[i]) return fail(DWF_ERR_ARG, "NULL pseudofermion");
  for (int i = 0; i <= nq; ++i)
    if (!std::isfinite(masses[i]) || masses[i] < 0.0) return fail(DWF_ERR_ARG, "masses must be finite and >= 0");
  for (int i = 0; i < nq; ++i)
    if (!(masses[i] < masses[i + 1])) return fail(DWF_ERR_ARG, "masses must increase along the ladder");
  if (out_kind != 0 && out_kind != 1) return fail(DWF_ERR_ARG, "out_kind must be 0 or 1");
  return guarded([&]() { return dwf::quotient_force(ctx, *p, nq, masses, U, phi, F, S, out_kind, x_io, info); });
}

int dwf_tune_set(dwf_ctx* ctx, int kernel_id, int prec, int Ls, int spb, int ns, int xcd, int ll) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  if (kernel_id < 0 || kernel_id > 2 || prec < 0 || prec > 3 || Ls < 2 || Ls > 128)
    return fail(DWF_ERR_ARG, "bad tune key");
  const long long key = tune_key(kernel_id, prec, Ls);
  if (spb == 0 && ns == 0) {
    ctx->tune.erase(key);
    return DWF_OK;
  }
  if (kernel_id == 2) {
    // the interleaved batched hop: spb 1 = on (workgroup shape fixed by the number of
    // right-hand sides), -1 = off
    if ((spb != 1 && spb != -1) || ns != 1 || (ll != 0 && ll != 1))
      return fail(DWF_ERR_ARG, "interleaved hop: sites_per_block 1 (on) or -1 (off), s_per_thread 1, link_lds 0 or 1");
    LaunchCfg c;
    c.spb = 1;
    c.ns = 1;
    c.xcd = xcd ? 1 : 0;
    c.ll = ll;
    c.stage = 0;
    c.off = spb < 0 ? 1 : 0;
    ctx->tune[key] = c;
    return DWF_OK;
  }
  if (ns != 1 && ns != 2 && ns != 4) return fail(DWF_ERR_ARG, "s_per_thread must be 1, 2 or 4");
  if (kernel_id == 1 && (ns != 1 || ll == 2))
    return fail(DWF_ERR_ARG, "the batched hop runs one slice per thread without staged neighbours");
  if (Ls % ns != 0) return fail(DWF_ERR_ARG, "Ls must be divisible by s_per_thread");
  if (spb < 1 || spb * (Ls / ns) > 256) return fail(DWF_ERR_ARG, "sites_per_block * Ls / s_per_thread must be <= 256");
  const size_t elem = prec == DWF_FP64 ? 16 : 8;
  const size_t lelem = prec == DWF_FP64 ? 16 : prec == DWF_FP32 ? 8 : 4;
  if (ll < 0 || ll > 2) return fail(DWF_ERR_ARG, "lds mode must be 0, 1 or 2");
  if (ll == 2 && (prec != DWF_FP16 || ns != 1 || spb * Ls != 256 || (Ls != 8 && Ls != 16 && Ls != 32)))
    return fail(DWF_ERR_ARG, "staged neighbour spinors need FP16, Ls 8/16/32, one slice per thread and 256 threads");
  const size_t lsite = prec == DWF_FP16 ? 160 : 72;  // FP16 links are staged in two forms
  if (size_t(spb) * 12 * Ls * elem + (ll == 1 ? size_t(spb) * lsite * lelem : 0) > 65536)
    return fail(DWF_ERR_ARG, "workgroup LDS (epilogue + staged links) exceeds 64 KiB");
  LaunchCfg c;
  c.spb = spb;
  c.ns = ns;
  c.xcd = xcd ? 1 : 0;
  c.ll = ll == 1 ? 1 : 0;
  c.stage = ll == 2 ? 1 : 0;
  ctx->tune[key] = c;
  return DWF_OK;
}

int dwf_tune_get(dwf_ctx* ctx, int kernel_id, int prec, int Ls, int* spb, int* ns, int* xcd, int* ll) {
  if (!ctx || !spb || !ns || !xcd || !ll) return fail(DWF_ERR_ARG, "NULL pointer");
  if (kernel_id < 0 || kernel_id > 2 || prec < 0 || prec > 3 || Ls < 2) return fail(DWF_ERR_ARG, "bad tune key");
  if (kernel_id == 2) {
    const LaunchCfg c = ilv_config(ctx, prec, Ls);
    *spb = c.off ? -1 : 1;
    *ns = 1;
    *xcd = c.xcd;
    *ll = c.ll;
    return DWF_OK;
  }
  LaunchCfg c = kernel_id == 1 ? batch_config(ctx, prec, Ls) : hop_config(ctx, prec, Ls);
  *spb = c.spb;
  *ns = c.ns;
  *xcd = c.xcd;
  *ll = stage_shape(c, Ls) ? 2 : c.ll;
  return DWF_OK;
}

int dwf_tune_tile(dwf_ctx* ctx, const int* dims, int tbc, const int* tile) {
  if (!ctx || !dims || !tile) return fail(DWF_ERR_ARG, "NULL pointer");
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || dims[k] % 2) return fail(DWF_ERR_ARG, "lattice extents must be even and >= 2");
  return guarded([&]() {
    set_tile(ctx, dims, tbc, tile);
    return DWF_OK;
  });
}

int dwf_tune_tile_get(dwf_ctx* ctx, const int* dims, int tbc, int* tile) {
  if (!ctx || !dims || !tile) return fail(DWF_ERR_ARG, "NULL pointer");
  for (int k = 0; k < 4; ++k)
    if (dims[k] < 2 || dims[k] % 2) return fail(DWF_ERR_ARG, "lattice extents must be even and >= 2");
  return guarded([&]() {
    const Geometry* g = geometry(ctx, dims, tbc);
    for (int k = 0; k < 3; ++k) tile[k] = g->tile[k];
    return DWF_OK;
  });
}

int dwf_timing_enable(dwf_ctx* ctx, int enable) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  return guarded([&]() {
    if (!enable) {
      DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));
      ctx->timer.marks.clear();
      ctx->timer.used = 0;
    }
    ctx->timer.on = enable != 0;
    return DWF_OK;
  });
}

int dwf_timing_report(dwf_ctx* ctx, char* buf, size_t len) {
  if (!ctx) return fail(DWF_ERR_ARG, "ctx is NULL");
  if (!buf || len == 0) return fail(DWF_ERR_ARG, "NULL report buffer");
  return guarded([&]() {
    const std::string r = timer_report(ctx);
    if (r.size() + 1 > len) {
      buf[0] = 0;
      return fail(DWF_ERR_ARG, "report buffer too small: need " + std::to_string(r.size() + 1) + " bytes");
    }
    std::memcpy(buf, r.c_str(), r.size() + 1);
    return DWF_OK;
  });
}

}  // extern "C"
