// Host runtime: context, geometry tables, workspace arena and the even-odd
// operator composition on top of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <map>
#include <memory>
#include <string>
#include <vector>
#include <cmath>
#include <cstring>
#include "kernels.hpp"
#include "../../include/dwf.h"

namespace dwf {

// error carried to the C boundary
struct Error {
  int code;
  std::string msg;
};
void set_error(const std::string& msg);

#define DWF_CHECK_HIP(expr)                                                                 \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) throw ::dwf::Error{DWF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)}; \
  } while (0)
#define DWF_CHECK_LAUNCH(expr)                                                              \
  do {                                                                                      \
    int rc_ = (expr);                                                                       \
    if (rc_ == -1) throw ::dwf::Error{DWF_ERR_ARG, std::string("launch shape rejected: ") + #expr}; \
    if (rc_ != 0) throw ::dwf::Error{DWF_ERR_HIP, std::string("kernel launch failed: ") + #expr + ": " + \
                                     hipGetErrorString(hipGetLastError())};                 \
  } while (0)

// ------------------------------------------------------------------ geometry
struct Geometry {
  int dims[4];
  int tbc;
  long V, nsites;
  int* d_site[2] = {nullptr, nullptr};
  int* d_nbr[2] = {nullptr, nullptr};
  int* d_linksrc[2] = {nullptr, nullptr};
  int* d_order[2] = {nullptr, nullptr};
  int tile[3] = {0, 0, 0};
  GeomTables tables() const {
    GeomTables t;
    for (int p = 0; p < 2; ++p) {
      t.site[p] = d_site[p];
      t.nbr[p] = d_nbr[p];
      t.linksrc[p] = d_linksrc[p];
      t.order[p] = d_order[p];
    }
    t.V = V;
    t.nsites = nsites;
    return t;
  }
  ~Geometry() {
    for (int p = 0; p < 2; ++p) {
      if (d_site[p]) (void)hipFree(d_site[p]);
      if (d_nbr[p]) (void)hipFree(d_nbr[p]);
      if (d_linksrc[p]) (void)hipFree(d_linksrc[p]);
      if (d_order[p]) (void)hipFree(d_order[p]);
    }
  }
};

// Optional per-launch timing of the hop and fifth-dimension kernels: a HIP event
// pair on the context stream around each launch, aggregated per kernel variant
// (named as the compiler names the template instance) with its algorithmic bytes.
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;  // reused across reports
  size_t used = 0;
  struct Mark {
    int cls;
    size_t e0, e1;
    double bytes;
  };
  std::vector<Mark> marks;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
};

}  // namespace dwf

struct dwf_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::map<std::string, std::pair<void*, size_t>> ws;
  std::vector<std::unique_ptr<dwf::Geometry>> geoms;
  std::map<std::string, std::pair<void*, size_t>> emats;  // fifth-dimension matrices by key
  std::map<long long, dwf::LaunchCfg> tune;              // (prec, Ls) -> hop launch configuration
  double* h_scalars = nullptr;                           // pinned host mirror of the CG scalars
  dwf::KernelTimer timer;
};

namespace dwf {

void* ws_get(dwf_ctx* ctx, const std::string& name, size_t bytes);

// The no-allocation operator (dwf_dslash_noalloc): a device array of this size per device holds
// its neighbour tables and intermediates.  scratch_init takes the array's device address on the
// current device (once per device; called when a context is created).
#define NOALLOC_SCRATCH_BYTES (size_t(256) << 20)
void* scratch_init();
int dslash_noalloc(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op, int parity,
                   int dagger);
const Geometry* geometry(dwf_ctx* ctx, const int dims[4], int tbc);
// traversal tile of the hop kernels on one lattice (0, 0, 0: the default)
void set_tile(dwf_ctx* ctx, const int dims[4], int tbc, const int tile[3]);
// launch configuration of the hop (kernel 0) and of the batched hop (kernel 1) for (prec, Ls):
// the tuned entry, else the default shape (one slice per thread)
inline long long tune_key(int kernel, int prec, int Ls) { return (long long)kernel * 1000000 + prec * 100000 + Ls; }
LaunchCfg hop_config(dwf_ctx* ctx, int prec, int Ls);
LaunchCfg batch_config(dwf_ctx* ctx, int prec, int Ls);
// the interleaved batched hop (kernel 2): XCD order, link staging, or off (separate fields)
LaunchCfg ilv_config(dwf_ctx* ctx, int prec, int Ls);
// device buffer of the fifth-dimension matrices for one parameter set
// (bs, cs: optional s-dependent Moebius coefficients, Ls entries each)
const void* fifth_matrices(dwf_ctx* ctx, int Ls, double M5, double m, double b, double c, int prec,
                           const double* bs = nullptr, const double* cs = nullptr);
double read_scalar(dwf_ctx* ctx, const double* dscalars, int slot);
// timer marks around one launch (no-ops while timing is off); begin returns the mark index or -1
long timer_begin(dwf_ctx* ctx, const std::string& kernel);
void timer_end(dwf_ctx* ctx, long mark, double bytes);
std::string timer_report(dwf_ctx* ctx);  // synchronizes; one line per kernel variant; clears the marks
void timer_release(dwf_ctx* ctx);

// bytes of one 5D site of a spinor field in storage precision P (with the FP16 norm)
template <typename P>
constexpr double spinor_site_bytes() { return 12.0 * sizeof(typename P::S) + (P::NORM ? 4.0 : 0.0); }
inline const char* prec_tag(int id) {
  static const char* n[4] = {"dwf::P64", "dwf::P32", "dwf::P16", "dwf::PB16"};
  return n[id & 3];
}

// slots of the per-parameter fifth-dimension matrix table ([slot][2][Ls][Ls])
// (E_F_AINV = F A^-1; with constant coefficients F and A^-1 commute, per chirality both
// being functions of one shift, which the recurrence form uses)
enum EMat { E_A = 0, E_ADAG, E_AINV, E_AINVDAG, E_F, E_FDAG, E_AINVDAG_FDAG, E_F_AINV, E_COUNT };
bool fifth_scan(int Ls, double M5, double m, double b, double c, int slot, FifthScan<double>* out);

template <typename P>
size_t half_size(const Geometry* g, int Ls) { return half_bytes<P>(g->nsites, Ls); }

template <typename P>
Half<P> hview(void* base, const Geometry* g, int Ls) { return half_view<P>(base, g->nsites, Ls); }
template <typename P>
CHalf<P> chview(const void* base, const Geometry* g, int Ls) { return chalf_view<P>(base, g->nsites, Ls); }
template <typename P>
CHalf<P> cv(Half<P> h) { return {h.data, h.norm}; }
template <typename P>
CHalf<P> none() { return {nullptr, nullptr}; }

// ------------------------------------------------------------------ operator
// Even-odd operator pieces in storage precision P for one parameter set:
//   B = -1/2 H F,  F = b + c S~,  M_prec = 1 - A^-1 B_oe A^-1 B_eo  (odd sites)
template <typename P>
struct Op {
  using R = typename P::R;
  using S = typename P::S;
  dwf_ctx* ctx;
  const Geometry* g;
  int Ls;
  double M5, m, b, c;
  bool moebius;  // F != 1
  bool sdep;     // s-dependent Moebius coefficients
  const S* U[2];
  const R* E;
  const R* coef_b;  // device b_s, c_s (Ls each), in the table after the matrices
  const R* coef_c;
  FifthScan<R> es[E_COUNT];  // the slots in recurrence form
  bool scan_ok;
  LaunchCfg cfg;

  Op(dwf_ctx* ctx_, const Geometry* g_, const dwf_params& p, const void* packed_links)
      : ctx(ctx_), g(g_), Ls(p.Ls), M5(p.M5), m(p.mass), b(p.b), c(p.c) {
    sdep = p.b_s || p.c_s;
    moebius = sdep || !(b == 1.0 && c == 0.0);
    const S* base = reinterpret_cast<const S*>(packed_links);
    U[0] = base;
    U[1] = base + size_t(g->nsites) * 72;
    E = reinterpret_cast<const R*>(fifth_matrices(ctx, Ls, M5, m, b, c, P::ID, p.b_s, p.c_s));
    coef_b = E + size_t(E_COUNT) * 2 * Ls * Ls;
    coef_c = coef_b + Ls;
    cfg = hop_config(ctx, P::ID, Ls);
    // the recurrence (scan) form assumes constant coefficients: dense epilogues otherwise
    scan_ok = !sdep;
    for (int slot = 0; scan_ok && slot < E_COUNT; ++slot) {
      FifthScan<double> e;
      if (!fifth_scan(Ls, M5, m, b, c, slot, &e)) { scan_ok = false; break; }
      es[slot].m = R(e.m);
      for (int ch = 0; ch < 2; ++ch) {
        const FifthChir<double>& q = e.ch[ch];
        es[slot].ch[ch] = FifthChir<R>{R(q.a1), R(q.b1), R(q.inv_alpha), R(q.a), R(q.corr), q.d1, q.d2, q.has_inv};
      }
    }
  }
  const R* em(int slot) const { return E + size_t(slot) * 2 * Ls * Ls; }
  size_t hb() const { return half_size<P>(g, Ls); }
  long n5() const { return g->nsites * Ls; }

  // out(out_par) = ax x + Epi . (scale H [F] in)   (H^dag F^dag ... when dag: no prologue)
  // CG step fused into a dagger hop (r.data == nullptr: none)
  struct CgStep {
    Half<P> r = {nullptr, nullptr};
    const double* scalars = nullptr;
    int x_slot = -1;  // >= 0: the axpy operand is es[x_slot] . x (applied in the launch)
  };

  // the launch arguments of one hop (see hop)
  HopArgs<P> hop_args(int out_par, CHalf<P> in, Half<P> out, const R* epi, double scale,
                      CHalf<P> x = {nullptr, nullptr}, double ax = 0.0, double* partials = nullptr,
                      const CgStep& cg = CgStep(), Half<P> out2 = {nullptr, nullptr}, int slot2 = 0) const {
    HopArgs<P> a;
    a.out2 = out2;
    if (out2.data) a.es2 = es[slot2];
    a.cg_r = cg.r;
    a.cg_scalars = cg.scalars;
    a.in = in;
    a.out = out;
    a.links = U[out_par];
    a.nbr = g->d_nbr[out_par];
    a.order = g->d_order[out_par];
    a.nsites = g->nsites;
    a.Ls = Ls;
    a.scale = R(scale);
    a.pb = R(b);
    a.pc = R(c);
    a.pm = R(m);
    if (sdep) {
      a.pbs = coef_b;
      a.pcs = coef_c;
    }
    a.E = epi;
    a.epi_scan = 0;
    if (epi && scan_ok) {
      a.es = es[(epi - E) / (2 * Ls * Ls)];
      a.epi_scan = 1;
    }
    a.x = x;
    a.ax = R(ax);
    if (cg.x_slot >= 0) {
      a.es2 = es[cg.x_slot];
      a.x_es2 = 1;
    }
    a.norm_partials = partials;
    return a;
  }
  // algorithmic bytes of one hop launch: fields read and written once (in, out -- or with the CG
  // step r read and written --, the axpy operand, the second output) and the links once
  double hop_bytes(const HopArgs<P>& a) const {
    const double fb = spinor_site_bytes<P>();
    const bool xin = a.x.data != nullptr;
    const double bytes = a.cg_r.data ? fb * (3 + (xin ? 1 : 0))
                                     : fb * (1 + (a.out.data ? 1 : 0) + (xin ? 1 : 0) + (a.out2.data ? 1 : 0));
    return double(n5()) * bytes + double(g->nsites) * 72 * sizeof(S);
  }
  // out2 (optional): slot2 applied to the final result, a second output of the same launch
  void hop(int out_par, CHalf<P> in, Half<P> out, bool dag, bool pro, double scale, const R* epi,
           CHalf<P> x = {nullptr, nullptr}, double ax = 0.0, double* partials = nullptr,
           const CgStep& cg = CgStep(), Half<P> out2 = {nullptr, nullptr}, int slot2 = 0) const {
    const HopArgs<P> a = hop_args(out_par, in, out, epi, scale, x, ax, partials, cg, out2, slot2);
    long mark = -1;
    if (ctx->timer.on) mark = timer_begin(ctx, hop_name(a, dag, pro && moebius, cfg));
    DWF_CHECK_LAUNCH(launch_hop<P>(a, dag, pro && moebius, cfg, ctx->stream));
    if (mark >= 0) timer_end(ctx, mark, hop_bytes(a));
  }
  // the template instance launch_hop selects for these arguments and launch shape (kernel name as
  // demangled; batch: the batched kernel)
  std::string hop_name(const HopArgs<P>& a, bool dag, bool pro, const LaunchCfg& cfg, bool batch = false) const {
    const int ls = (Ls == 8 || Ls == 12 || Ls == 16 || Ls == 32) ? Ls : 0;
    int epi = 0;
    if (a.E) epi = (a.epi_scan && cfg.ns == 1 && (ls == 8 || ls == 16 || ls == 32)) ? (a.out2.data ? 3 : 2) : 1;
    const bool st = !batch && P::ID == DWF_FP16 && cfg.ns == 1 && !pro && epi != 1 &&
                    (ls == 8 || ls == 16 || ls == 32) && stage_shape(cfg, Ls);
    return std::string(batch ? "hop_batch_kernel<" : "hop_kernel<") + prec_tag(P::ID) + ", " + std::to_string(ls) +
           ", " + std::to_string(cfg.ns) +
           ", " + (dag ? "true" : "false") + ", " + (pro ? "true" : "false") + ", " + std::to_string(epi) + ", " +
           (cfg.ll || st ? "true" : "false") + ", " + (a.cg_r.data ? "true" : "false") + ", " +
           (st ? "true" : "false") + ">";
  }
  void fifth(CHalf<P> in, Half<P> out, int slot, CHalf<P> x = {nullptr, nullptr}, double ax = 0.0,
             double* partials = nullptr) const {
    long mark = -1;
    if (ctx->timer.on) {
      const int seg = (scan_ok && (Ls == 8 || Ls == 16 || Ls == 32)) ? Ls : 0;
      mark = timer_begin(ctx, std::string("fifth_kernel<") + prec_tag(P::ID) + ", " + std::to_string(seg) + ">");
    }
    DWF_CHECK_LAUNCH(launch_fifth<P>(in, out, em(slot), scan_ok ? &es[slot] : nullptr, x, R(ax), g->nsites, Ls,
                                     partials, ctx->stream));
    if (mark >= 0) timer_end(ctx, mark, double(n5()) * spinor_site_bytes<P>() * (x.data ? 3 : 2));
  }
  // the scan epilogue can carry a second output (one s-slice per lane, Ls a wave segment)
  bool second_output_ok() const { return scan_ok && cfg.ns == 1 && (Ls == 8 || Ls == 16 || Ls == 32); }
  // ... and the last hop of M^dag q can rebuild q from that second output (q need not be stored)
  bool rebuild_q_ok() const { return second_output_ok() && x_es2_shape<P>(cfg, Ls); }
  // workgroups of one hop launch (the norm partials it writes)
  long hop_blocks() const { return (g->nsites + cfg.spb - 1) / cfg.spb; }
  // M_prec psi = psi - 1/4 A^-1 H_oe F A^-1 H_eo F psi      (odd -> odd);
  // ainvdag_out (optional, see second_output_ok): also A^-dag (M_prec psi); with it, out may be
  // empty (the norm partials and A^-dag (M_prec psi) only)
  void mprec(CHalf<P> in, Half<P> out, Half<P> tmp_e, double* partials = nullptr,
             Half<P> ainvdag_out = {nullptr, nullptr}) const {
    hop(0, in, tmp_e, false, true, 1.0, em(E_AINV));
    hop(1, cv(tmp_e), out, false, true, -0.25, em(E_AINV), in, 1.0, partials, CgStep(), ainvdag_out, E_AINVDAG);
  }
  // M_prec psi from fpsi = F psi prepared by the caller (the CG p update): both hops without
  // the input factor, the first with the epilogue F A^-1 (Moebius operators)
  void mprec_pre(CHalf<P> fin, CHalf<P> in, Half<P> out, Half<P> tmp_e, double* partials = nullptr,
                 Half<P> ainvdag_out = {nullptr, nullptr}) const {
    hop(0, fin, tmp_e, false, false, 1.0, em(E_F_AINV));
    hop(1, cv(tmp_e), out, false, false, -0.25, em(E_AINV), in, 1.0, partials, CgStep(), ainvdag_out, E_AINVDAG);
  }
  // M_prec^dag psi = psi - 1/4 F^dag H^dag_oe (A^-dag F^dag) H^dag_eo A^-dag psi
  void mprec_dag(CHalf<P> in, Half<P> out, Half<P> tmp_o, Half<P> tmp_e, double* partials = nullptr) const {
    fifth(in, tmp_o, E_AINVDAG);
    hop(0, cv(tmp_o), tmp_e, true, false, 1.0, em(E_AINVDAG_FDAG));
    hop(1, cv(tmp_e), out, true, false, -0.25, moebius ? em(E_FDAG) : nullptr, in, 1.0, partials);
  }
  // M_prec^dag q with the CG step fused into its last hop: r -= alpha M_prec^dag q and the
  // per-workgroup partials of |r|^2 (alpha read from scalars on the device)
  // (ainvdag_ready: tmp_o already holds A^-dag q, the second output of mprec; q_rebuilt (needs
  // rebuild_q_ok): in is not read, the last hop forms q = A^dag (A^-dag q) at its own sites)
  void mprec_dag_cg(CHalf<P> in, Half<P> tmp_o, Half<P> tmp_e, Half<P> r, const double* scalars, double* partials,
                    bool ainvdag_ready = false, bool q_rebuilt = false) const {
    if (!ainvdag_ready) fifth(in, tmp_o, E_AINVDAG);
    hop(0, cv(tmp_o), tmp_e, true, false, 1.0, em(E_AINVDAG_FDAG));
    CgStep cg;
    cg.r = r;
    cg.scalars = scalars;
    const bool reb = ainvdag_ready && q_rebuilt;
    if (reb) cg.x_slot = E_ADAG;
    hop(1, cv(tmp_e), Half<P>{nullptr, nullptr}, true, false, -0.25, moebius ? em(E_FDAG) : nullptr,
        reb ? cv(tmp_o) : in, 1.0, partials, cg);
  }
  // full D (or D^dag):  (D psi)_p = A psi_p - 1/2 H F psi_{1-p};  (D^dag psi)_p = A^dag psi_p - 1/2 F^dag H^dag psi_{1-p}
  void full(CHalf<P> in_e, CHalf<P> in_o, Half<P> out_e, Half<P> out_o, bool dag) const {
    fifth(in_e, out_e, dag ? E_ADAG : E_A);
    fifth(in_o, out_o, dag ? E_ADAG : E_A);
    if (!dag) {
      hop(0, in_o, out_e, false, true, -0.5, nullptr, cv(out_e), 1.0);
      hop(1, in_e, out_o, false, true, -0.5, nullptr, cv(out_o), 1.0);
    } else {
      hop(0, in_o, out_e, true, false, -0.5, moebius ? em(E_FDAG) : nullptr, cv(out_e), 1.0);
      hop(1, in_e, out_o, true, false, -0.5, moebius ? em(E_FDAG) : nullptr, cv(out_o), 1.0);
    }
  }
};

// ------------------------------------------------------------------ 5D even-odd (Shamir)
// Shamir DWF checkerboarded in five dimensions, parity (x + y + z + t + s) mod 2:
//   D = d0 - K,  d0 = 5 - M5,  K = 1/2 H4 + H5,  H5 psi_s = P- psi_{s+1} + P+ psi_{s-1}
// (psi_{Ls} = -m psi_0, psi_{-1} = -m psi_{Ls-1}).  K connects opposite 5D parities only, so on
// the even sites the Schur complement is  S = d0 - K_eo K_oe / d0.
// A field of 5D parity p holds, for each 4D parity q, the slices s = 2 j + (p ^ q), j < Ls/2, of
// every site x_cb of that parity: [q][x_cb][12][Ls/2].  Vector operations see it as one half
// field of 2 nsites sites and Ls/2 slices (the geometry gv, which has no tables).
template <typename P>
struct Op5 {
  using R = typename P::R;
  using S = typename P::S;
  dwf_ctx* ctx;
  const Geometry* g4;
  Geometry gv;
  const Geometry* g = &gv;
  int Ls;  // slices of one field per site: Ls / 2
  double M5, m, d0;
  const S* U[2];
  LaunchCfg cfg;
  // read by the CG driver: no Moebius input factor here
  bool moebius = false, sdep = false;
  double b = 1.0, c = 0.0;
  const R* coef_b = nullptr;
  const R* coef_c = nullptr;

  Op5(const Op5&) = delete;
  Op5& operator=(const Op5&) = delete;
  Op5(dwf_ctx* ctx_, const Geometry* g4_, const dwf_params& p, const void* packed_links)
      : ctx(ctx_), g4(g4_), Ls(p.Ls / 2), M5(p.M5), m(p.mass), d0(5.0 - p.M5) {
    for (int k = 0; k < 4; ++k) gv.dims[k] = g4->dims[k];
    gv.tbc = g4->tbc;
    gv.V = g4->V;
    gv.nsites = 2 * g4->nsites;
    const S* base = reinterpret_cast<const S*>(packed_links);
    U[0] = base;
    U[1] = base + size_t(g4->nsites) * 72;
    cfg = hop_config(ctx, P::ID, Ls);
    cfg.ns = 1;
    cfg.stage = 0;
    cfg.off = 0;
    if (cfg.spb < 1 || cfg.spb * Ls > 256) cfg.spb = 256 / Ls;
  }
  // the 4D-parity half q of a field
  Half<P> half(Half<P> f, int q) const {
    const size_t n = size_t(q) * g4->nsites * Ls;
    return {f.data ? f.data + n * 12 : nullptr, f.norm ? f.norm + n : nullptr};
  }
  CHalf<P> half(CHalf<P> f, int q) const {
    const size_t n = size_t(q) * g4->nsites * Ls;
    return {f.data ? f.data + n * 12 : nullptr, f.norm ? f.norm + n : nullptr};
  }
  long hop_blocks() const { return 2 * ((g4->nsites + cfg.spb - 1) / cfg.spb); }
  bool second_output_ok() const { return false; }
  bool rebuild_q_ok() const { return false; }
  long n5() const { return gv.nsites * Ls; }

  // out (5D parity p) = ax x + scale4 H4 in + r5 H5 in, in of parity 1 - p (dag: the adjoint
  // hops); with cg_r: not stored, cg_r -= alpha (...) instead (dag only)
  void K(int p, CHalf<P> in, Half<P> out, bool dag, double scale4, double r5, CHalf<P> x = {nullptr, nullptr},
         double ax = 0.0, double* partials = nullptr, Half<P> cg_r = {nullptr, nullptr},
         const double* scalars = nullptr) const {
    HopArgs<P> a[2];
    for (int q = 0; q < 2; ++q) {
      HopArgs<P> h = HopArgs<P>();
      h.in = half(in, 1 - q);
      h.loc = half(in, q);
      h.out = cg_r.data ? Half<P>{nullptr, nullptr} : half(out, q);
      h.links = U[q];
      h.nbr = g4->d_nbr[q];
      h.order = g4->d_order[q];
      h.nsites = g4->nsites;
      h.Ls = Ls;
      h.scale = R(scale4);
      h.r5 = R(r5);
      h.pb = R(1);
      h.pc = R(0);
      h.pm = R(m);
      h.E = nullptr;
      h.x = x.data ? half(x, q) : CHalf<P>{nullptr, nullptr};
      h.ax = R(ax);
      h.norm_partials = partials;
      h.sigma = p ^ q;
      if (cg_r.data) {
        h.cg_r = half(cg_r, q);
        h.cg_scalars = scalars;
      }
      a[q] = h;
    }
    long mark = -1;
    if (ctx->timer.on) {
      const int ls = (Ls == 8 || Ls == 16 || Ls == 32) ? Ls : 0;
      mark = timer_begin(ctx, std::string("hop_eo5_kernel<") + prec_tag(P::ID) + ", " + std::to_string(ls) + ", " +
                                  (dag ? "true" : "false") + ", " + (cfg.ll ? "true" : "false") + ", " +
                                  (cg_r.data ? "true" : "false") + ">");
    }
    DWF_CHECK_LAUNCH(launch_hop_eo5<P>(a[0], a[1], dag, cfg, ctx->stream));
    if (mark >= 0) {
      const double fb = spinor_site_bytes<P>();
      const double fields = cg_r.data ? 3 + (x.data ? 1 : 0) : 2 + (x.data ? 1 : 0);
      timer_end(ctx, mark, double(n5()) * fb * fields + 2.0 * double(g4->nsites) * 72 * sizeof(S));
    }
  }
  // S psi = d0 psi - K_eo K_oe psi / d0  (even -> even; tmp: an odd field)
  void mprec(CHalf<P> in, Half<P> out, Half<P> tmp, double* partials = nullptr,
             Half<P> unused = {nullptr, nullptr}) const {
    (void)unused;
    K(1, in, tmp, false, 0.5, 1.0);
    K(0, cv(tmp), out, false, -0.5 / d0, -1.0 / d0, in, d0, partials);
  }
  void mprec_pre(CHalf<P> fin, CHalf<P> in, Half<P> out, Half<P> tmp, double* partials = nullptr,
                 Half<P> unused = {nullptr, nullptr}) const {
    (void)fin;
    mprec(in, out, tmp, partials, unused);
  }
  // S^dag psi = d0 psi - K^dag_eo K^dag_oe psi / d0
  void mprec_dag(CHalf<P> in, Half<P> out, Half<P> tmp_o, Half<P> tmp_e, double* partials = nullptr) const {
    (void)tmp_e;
    K(1, in, tmp_o, true, 0.5, 1.0);
    K(0, cv(tmp_o), out, true, -0.5 / d0, -1.0 / d0, in, d0, partials);
  }
  // S^dag q with the CG step fused into its last hop (see Op::mprec_dag_cg)
  void mprec_dag_cg(CHalf<P> in, Half<P> tmp_o, Half<P> tmp_e, Half<P> r, const double* scalars, double* partials,
                    bool ready = false, bool q_rebuilt = false) const {
    (void)tmp_e;
    (void)q_rebuilt;
    (void)ready;
    K(1, in, tmp_o, true, 0.5, 1.0);
    K(0, cv(tmp_o), Half<P>{nullptr, nullptr}, true, -0.5 / d0, -1.0 / d0, in, d0, partials, r, scalars);
  }
};

// reduction helpers: n partials -> scalar slot
// per-workgroup FP64 partial sums (room for 4M workgroups)
inline double* partials_buf(dwf_ctx* ctx) { return reinterpret_cast<double*>(ws_get(ctx, "partials", (size_t(1) << 22) * sizeof(double))); }
inline double* scalars_buf(dwf_ctx* ctx) { return reinterpret_cast<double*>(ws_get(ctx, "scalars", S_COUNT * sizeof(double))); }

template <typename P>
double norm2_sync(dwf_ctx* ctx, CHalf<P> a, const Geometry* g, int Ls, int slot = S_TMP0) {
  double* part = partials_buf(ctx);
  double* sc = scalars_buf(ctx);
  const long n5 = g->nsites * Ls;
  DWF_CHECK_LAUNCH(launch_norm2<P>(a, n5, Ls, part, ctx->stream));
  DWF_CHECK_LAUNCH(launch_reduce(part, reduction_blocks(n5), 1, sc, slot, 0, ctx->stream));
  return read_scalar(ctx, sc, slot);
}

}  // namespace dwf
