// Host-side launch interface of the gfx950 kernels (no torch types).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "device.hpp"

namespace dwf {

// Storage precision of the CG solution increment accumulated between reliable updates for
// iterations in storage precision P: FP32 (an FP16 increment would carry errors of relative
// size 2^-11 in every eigen-direction of M^dag M, which the condition number amplifies in
// the residual), FP64 for FP64 iterations.
template <typename P>
struct IncrementPrec {
  using type = P32;
};
template <>
struct IncrementPrec<P64> {
  using type = P64;
};

// Arguments of one Wilson-hop launch over a half field (output parity fixed by
// the link block and neighbour table handed in).
//   out = ax * x + E . (scale * H F in)       (H^dag when dagger)
// F = pb + pc S~ (prologue, optional), E = per-chirality Ls x Ls matrices
// (epilogue, optional), x (axpy, optional).  norm_partials (optional) receives
// one FP64 partial sum of |out|^2 per block.
template <typename P>
struct HopArgs {
  CHalf<P> in;
  Half<P> out;
  const typename P::S* links;  // [nsites][8][9] for the output parity
  const int* nbr;              // [nsites][8] neighbour x_cb in the input half
  const int* order;            // [nsites] traversal order of the output sites (nullptr: x_cb order)
  long nsites;
  int Ls;
  typename P::R scale;
  typename P::R pb, pc, pm;    // prologue F = pb + pc S~, boundary factor -pm
  const typename P::R* pbs = nullptr;  // s-dependent prologue coefficients b_s, c_s (device, Ls
  const typename P::R* pcs = nullptr;  // each; nullptr: the constants pb, pc)
  const typename P::R* E;      // epilogue [2][Ls][Ls] or nullptr
  FifthScan<typename P::R> es; // the same epilogue in recurrence form
  int epi_scan = 0;            // es is valid (used when the site's lanes form a wave segment)
  CHalf<P> x;                  // axpy operand (data == nullptr: none)
  typename P::R ax;
  // x_es2 != 0 (fused CG step, scan epilogue shapes only): the axpy operand is es2 . x, the
  // site-local operator applied to x in registers (the CG hop then reads A^-dag q, which it
  // turns back into q = A^dag (A^-dag q), and q itself need not be stored); interleaved right-
  // hand sides take the operator of each from es2_tab
  int x_es2 = 0;
  double* norm_partials;       // per-block sum |out|^2 (|cg_r|^2 with the fused CG step) or nullptr
  // second output (scan epilogue only): out2 = es2 . out, a site-local operator applied to
  // the final result (out2.data == nullptr: none)
  Half<P> out2 = {nullptr, nullptr};
  FifthScan<typename P::R> es2;
  // CG step fused into the last hop of M^dag M p (cg_r.data == nullptr: none).  With it the
  // result v is not stored; instead r -= alpha v, alpha = cg_scalars[S_ALPHA], and the
  // partials are those of the new |r|^2 (the solution increment is summed separately, a few
  // iterations at a time).
  Half<P> cg_r = {nullptr, nullptr};
  const double* cg_scalars = nullptr;
  // right-hand sides interleaved along s (launch_hop_ilv): per right-hand side epilogue
  // coefficients (device tables) and the stride of the norm partials between right-hand sides
  const FifthScan<typename P::R>* es_tab = nullptr;
  const FifthScan<typename P::R>* es2_tab = nullptr;
  long part_stride = 0;
  // 5D even-odd Shamir hop (launch_hop_eo5): loc = the input field's slices at the output sites
  // (its half of the same 4D parity), sigma = the offset of the output slices (slot j holds
  // s = 2 j + sigma; loc's slot j holds s = 2 j + 1 - sigma), r5 = the coefficient of the
  // fifth-dimension hop (the 4D hop's is scale)
  CHalf<P> loc = {nullptr, nullptr};
  int sigma = 0;
  typename P::R r5 = 0;
};

struct LaunchCfg {
  int spb;        // 4D sites per block
  int ns;         // s-values per thread
  int xcd;        // XCD-aware block order
  int ll;         // links staged in LDS
  int stage = 0;  // neighbour spinors (and links) staged through LDS (FP16, Ls 8/16/32, spb = 256/Ls, ns 1)
  int off = 0;    // (the interleaved batched hop's entry) interleaving switched off
};
// the launch shape the LDS-staged hop runs with
inline bool stage_shape(const LaunchCfg& cfg, int Ls) {
  return cfg.stage && cfg.ns == 1 && cfg.spb * Ls == 256 && (Ls == 8 || Ls == 16 || Ls == 32);
}

// the launches that apply a site-local operator to the fused CG step's axpy operand
// (HopArgs::x_es2): one slice per lane, the site's Ls lanes a wave segment, not the LDS-staged
// shape, and not FP64 storage (where the extra live operand costs a wave per SIMD)
template <typename P>
inline bool x_es2_shape(const LaunchCfg& cfg, int Ls) {
  return !std::is_same<P, P64>::value && cfg.ns == 1 && (Ls == 8 || Ls == 16 || Ls == 32) && !stage_shape(cfg, Ls);
}

// batch: optional device table of nrhs fields' arguments for one launch over all of them (a is
// then the host copy of the first)
template <typename P>
int launch_hop(const HopArgs<P>& a, bool dagger, bool prologue, const LaunchCfg& cfg, hipStream_t st,
               const HopArgs<P>* batch = nullptr, int nrhs = 1);

// the hop on right-hand sides interleaved along s in segments of rs slices (see hop_impl.hpp)
template <typename P>
int launch_hop_ilv(const HopArgs<P>& a, bool dagger, int rs, const LaunchCfg& cfg, hipStream_t st);
// The Shamir hop K = (5 - M5) - D(m) on 5D-checkerboarded fields: one launch over both 4D-parity
// halves of the output field (a0: half 0, a1: half 1; workgroup pairs take the two halves of one
// traversal tile).  Each half: out = ax x + scale H4(in) + r5 H5(loc), where in is the input
// field's half of the other 4D parity (the hop's usual operand) and H5 the fifth-dimension hop
// from loc.  a.Ls = Ls / 2 must divide 64; one slice per thread; no prologue or epilogue
// matrices; the fused CG step only with the dagger.
template <typename P>
int launch_hop_eo5(const HopArgs<P>& a0, const HopArgs<P>& a1, bool dagger, const LaunchCfg& cfg, hipStream_t st);
// The two 4D-parity halves h0, h1 of a field ([x_cb][12][Ls] each) <-> its two 5D-parity fields
// ([4D parity q][x_cb][12][Ls/2] each: slice s of 4D parity q lies in field (s + q) mod 2, slot
// s / 2); merge = 0 splits, 1 merges
template <typename P>
int launch_eo5_split(Half<P> h0, Half<P> h1, Half<P> f5_even, Half<P> f5_odd, long nsites, int Ls, int merge,
                     hipStream_t st);

// out = ax * x + E . in  (site-local fifth-dimension matrices), optional |out|^2 partials
template <typename P>
int launch_fifth(CHalf<P> in, Half<P> out, const typename P::R* E, const FifthScan<typename P::R>* es, CHalf<P> x,
                 typename P::R ax, long nsites, int Ls, double* norm_partials, hipStream_t st);

// ---------------------------------------------------------------- BLAS-1 / reductions
// Every reduction writes per-block FP64 partials; reduce_partials sums them in
// a fixed order (deterministic) into dst.
int reduction_blocks(long n5);  // number of partial sums the BLAS reductions produce for n5 5D sites
template <typename P>
int launch_norm2(CHalf<P> a, long n5, int Ls, double* partials, hipStream_t st);
template <typename P>
int launch_dot(CHalf<P> a, CHalf<P> b, long n5, int Ls, double* partials /* 2 per block */, hipStream_t st);
// y = a*x + b*y   (a, b real, host scalars)
template <typename P>
int launch_axpby(double a, CHalf<P> x, double b, Half<P> y, long n5, int Ls, hipStream_t st);
// precision conversion of a half field
template <typename Pi, typename Po>
int launch_convert(CHalf<Pi> in, Half<Po> out, long n5, int Ls, hipStream_t st);
// scalar slots on the device (CG scalars)
// S_AHIST .. S_AHIST + XFLUSH_MAX - 1: alpha of the iterations whose increments are pending
enum ScalarSlot { S_RR = 0, S_RRNEW, S_QQ, S_ALPHA, S_BETA, S_TMP0, S_TMP1, S_TMP2, S_AHIST = 8, S_COUNT = 16 };
constexpr int XFLUSH_MAX = S_COUNT - S_AHIST;
// dst[slot] = sum(partials[0..n)) and the CG scalar update selected by mode:
//   0: just store;  1: alpha = rr/qq (slot = S_QQ), also stored at S_AHIST + hist when hist >= 0;
//   2: beta = rrnew/rr, rr = rrnew (slot = S_RRNEW)
int launch_reduce(const double* partials, int n, int ncomp, double* scalars, int slot, int mode, hipStream_t st,
                  int hist = -1);
// pending CG directions: x += sum_j scalars[S_AHIST + slot[j]] p[j], j < n
template <typename P>
struct XFlush {
  CHalf<P> p[XFLUSH_MAX];
  int slot[XFLUSH_MAX];
  int n = 0;
};
template <typename P, typename Px>
int launch_xflush(Half<Px> x, const XFlush<P>& f, const double* scalars, long n5, int Ls, hipStream_t st);
// p_out = r + beta p_in (p_in unused when beta = 0; it may be p_out) and scalars[S_RR] = rr_new
template <typename P>
int launch_cg_pupdate(CHalf<P> r, CHalf<P> pin, Half<P> pout, double beta, double* scalars, double rr_new, long n5,
                      int Ls, hipStream_t st);
// p_out = r + beta p_in (p_in unused when beta = 0) and fp = (b + c S~) p_out, rr_new -> S_RR
template <typename P>
int launch_cg_pupdate_f(CHalf<P> r, CHalf<P> pin, Half<P> pout, Half<P> fp, double beta, double* scalars,
                        double rr_new, long n5, int Ls, double b, double c, double m, hipStream_t st,
                        const typename P::R* bs = nullptr, const typename P::R* cs = nullptr);
// P / P^-1 of the domain-wall <-> overlap transformation on an FP64 half field
int launch_pshift(CHalf<P64> in, Half<P64> out, int inverse, long nsites, int Ls, hipStream_t st);
// out(s_out) = scale * in(s_in) on FP64 half fields of extents Ls_in, Ls_out
int launch_slice_copy(CHalf<P64> in, int Ls_in, int s_in, Half<P64> out, int Ls_out, int s_out, double scale,
                      long nsites, hipStream_t st);
// x_hi += x_lo (then x_lo = 0)
template <typename Px>
int launch_accumulate(Half<P64> hi, Half<Px> lo, long n5, int Ls, hipStream_t st);
int launch_zero(void* p, size_t bytes, hipStream_t st);
// Fields of several right-hand sides interleaved along s: slice s of right-hand side r is slice
// r RS + s of a field of extent LT (a separate field: r = 0, LT = RS).
// p_out = r + coef[k] p_in per right-hand side k (device table; 0: p_in unread), and
// scalars[k S_COUNT + S_RR] = coef[K + k] (K = LT / RS)
template <typename P>
int launch_ilv_pupdate(CHalf<P> r, CHalf<P> pin, Half<P> pout, const double* coef, double* scalars, long nsites, int LT,
                       int RS, hipStream_t st);
// x += sum_j alpha_{k,j} p_j with alpha_{k,j} = scalars[k S_COUNT + S_AHIST + slot_j]
template <typename P, typename Px>
int launch_ilv_xflush(Half<Px> x, const XFlush<P>& f, const double* scalars, long nsites, int LT, int RS,
                      hipStream_t st);
// segment r_out of out = segment r_in of in (precision conversion), out-of-place
template <typename Pi, typename Po>
int launch_ilv_move(CHalf<Pi> in, int LT_in, int r_in, Half<Po> out, int LT_out, int r_out, long nsites, int RS,
                    hipStream_t st);
// hi (separate FP64 field, extent RS) += segment r of lo (extent LT); the segment is zeroed
template <typename Px>
int launch_ilv_accumulate(Half<P64> hi, Half<Px> lo, int LT, int r, long nsites, int RS, hipStream_t st);
int launch_set_scalar(double* scalars, int slot, double v, hipStream_t st);

// ---------------------------------------------------------------- packing
struct GeomTables {
  const int* site[2];    // [nsites] lexicographic index of x_cb, per parity
  const int* order[2];   // [nsites] tiled traversal order of the x_cb of each parity
  const int* nbr[2];     // [nsites][8] neighbour x_cb (other parity) for output parity p
  const int* linksrc[2]; // [nsites][8] (mu*V + i) of the link used, sign bit = boundary phase -1
  long V, nsites;
};
template <typename P>
int launch_pack_gauge(const GeomTables& g, const double2* natural, typename P::S* packed, hipStream_t st);
template <typename P>
int launch_pack_half(const GeomTables& g, int parity, int Ls, const double2* natural, Half<P> out,
                     hipStream_t st);
template <typename P>
int launch_unpack_half(const GeomTables& g, int parity, int Ls, CHalf<P> in, double2* natural, hipStream_t st);
template <typename Pi, typename Po>
int launch_convert_links(const typename Pi::S* in, typename Po::S* out, long n, hipStream_t st);

// ---------------------------------------------------------------- force
// Per link (x, mu) of parity p sites x:  Q = sum_{s,spin} outer products (see force.hip)
// writes either F = -1/2 TA(M) (kind 0) or the ambient gradient G (kind 1) to the
// natural force layout.
// F = coef * value, or F += coef * value with accumulate (one link per thread: no race)
int launch_force(const GeomTables& g, int Ls, CHalf<P64> W_e, CHalf<P64> W_o, CHalf<P64> Z_e, CHalf<P64> Z_o,
                 const double2* U_natural, int tbc, const int dims[4], int kind, double2* F, hipStream_t st,
                 double coef = 1.0, int accumulate = 0);
// gauge-field kernels (natural layouts, periodic links): plaquette action partial sums
// (sum (1 - Re tr U_P / 3) per workgroup), the plaquette force F = coef (beta/6) TA(U A)
// (+ F with accumulate), P <- P - eps F, kinetic-energy partial sums (-tr P P per link)
int launch_plaquette(const double2* U, const int dims[4], double* partials, int* nblocks, hipStream_t st);
int launch_gauge_force(const double2* U, const int dims[4], double beta, double coef, int accumulate, double2* F,
                       hipStream_t st);
int launch_mom_update(double2* P, const double2* F, double eps, long nlinks, hipStream_t st);
int launch_kinetic(const double2* P, long nlinks, double* partials, int* nblocks, hipStream_t st);
// U' = exp(-eps F) U per link (Cayley-Hamilton exponential), natural layouts
int launch_fg_update(const double2* F, const double2* U, double eps, double2* Uout, long nlinks, hipStream_t st);

}  // namespace dwf
