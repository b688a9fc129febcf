// Fermion force (Sec. 2: e_a(S) with e_a(U) = T_a U) as the adjoint of the hop:
// for S = phi^+ (M^+ M)^-1 phi, X = (M^+M)^-1 phi, the derivative along a link
// reduces to   dS = -Re <Z, dH W>   with W = F (X + X_e), Z = Y_o' + Y_e'
// (X_e = A^-1 B_eo X, Y_o' = A^-dag M X, Y_e' = A^-dag B_oe^dag Y_o', F = b + c S~).
// For the link U_mu(x) only two hop terms contribute:
//   <Z, dH W> = tr(dU Q1) + tr(dU^+ Q2),
//   Q1 = sum_{s,spin} [(1 - g_mu) W(x+mu)] Z(x)^+,  Q2 = sum_{s,spin} [(1 + g_mu) W(x)] Z(x+mu)^+ .
// The lanes of one link accumulate Q1, Q2 over their slices s (FP64) and sum them; one writes either
//   F = sum_a e_a T_a = -1/2 TA(Q2 U^+ - U Q1)     (T_a = i lambda_a / 2)
// or the ambient gradient G = -(Q1^+ + Q2) (dS = Re sum conj(G) dU).
// The force-gradient update U' = exp(-eps F) U uses the Cayley-Hamilton form of
// the SU(3) exponential of Morningstar and Peardon (Phys. Rev. D 69, 054501, 2004).
#include "kernels.hpp"

namespace dwf {

using C = cx<double>;

__device__ __forceinline__ C cconj(C a) { return {a.re, -a.im}; }

// The spin trace of the projected outer product: with P = 1 + sg g_mu (hermitian, and P^2 = 2P),
//   sum_spin [P w] z^+ = h0(w) h0(z)^+ + h1(w) h1(z)^+,
// h0, h1 the two independent rows of the projection (device.hpp); so each slice contributes
// two 3x3 colour outer products of projected half spinors.
template <int MU, int SG>
__device__ __forceinline__ void load_project(CHalf<P64> f, long x, int s, int Ls, C h[6]) {
  const double2* p = f.data + size_t(x) * 12 * Ls + s;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    project_colour<MU, SG, double>(P64::ld(p[c * Ls]), P64::ld(p[(3 + c) * Ls]), P64::ld(p[(6 + c) * Ls]),
                                   P64::ld(p[(9 + c) * Ls]), h[c], h[3 + c]);
}

template <int MU, int SG>
__device__ __forceinline__ void proj_outer_acc(CHalf<P64> W, long xw, CHalf<P64> Z, long xz, int s, int Ls, C Q[9]) {
  C hw[6], hz[6];
  load_project<MU, SG>(W, xw, s, Ls, hw);
  load_project<MU, SG>(Z, xz, s, Ls, hz);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Q[i * 3 + j] = cfma(hw[r * 3 + i], cconj(hz[r * 3 + j]), Q[i * 3 + j]);
}

struct ForceArgs {
  CHalf<P64> W[2], Z[2];
  const int* nbr[2];
  const int* linksrc[2];
  const double2* U;
  long nsites;
  int Ls;
  int kind;
  double coef;     // F = coef * value (+ F when accumulate)
  int accumulate;
  double2* F;
};

// Lane layout: the SEG lanes (SEG >= 16) of one aligned wave segment share one link and take the
// slices s = lane, lane + SEG, ... of the fifth dimension, so that their loads of the s-fastest
// [x_cb][12][Ls] fields are contiguous.  The lanes' partial sums of Q1 (then Q2) go to LDS, and lane
// e < 9 of the segment adds element e (row e / 3, column e % 3) over the segment's lanes in lane
// order; it then computes element e of the link's result, taking the other elements it needs
// from the lanes that hold them.  One 3x3 accumulator is live at a time.
__device__ __forceinline__ C shfl_c(C v, int src) { return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)}; }

// the segment sum of one slice loop's outer products, element e (< 9) of it in lane e
template <int MU, int SG, int SEG>
__device__ __forceinline__ C link_term(CHalf<P64> W, long xw, CHalf<P64> Z, long xz, int Ls, int lane, bool active,
                                       C* part) {
  C Q[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Q[k] = {0.0, 0.0};
  if (active) {
#pragma unroll 1
    for (int s = lane; s < Ls; s += SEG) proj_outer_acc<MU, SG>(W, xw, Z, xz, s, Ls, Q);
  }
  C* mine = part + threadIdx.x * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) mine[k] = Q[k];
  __syncthreads();
  C sum = {0.0, 0.0};
  if (lane < 9) {
    const C* seg = part + (threadIdx.x - lane) * 9 + lane;
    for (int i = 0; i < SEG; ++i) sum = sum + seg[i * 9];
  }
  __syncthreads();  // (the buffer is reused by the next term)
  return sum;
}

template <int MU, int SEG>
__device__ void force_link(const ForceArgs& a, int p, long x, int lane, bool active, C* part) {
  static_assert(SEG >= 16 && SEG <= 64, "a segment holds the nine elements of a link");
  // (the parity's operands selected, not indexed: a runtime index into the argument arrays would
  // copy them to private memory)
  const int* nbr = p ? a.nbr[1] : a.nbr[0];
  const int* lsrc = p ? a.linksrc[1] : a.linksrc[0];
  const CHalf<P64> Wp = p ? a.W[1] : a.W[0], Wq = p ? a.W[0] : a.W[1];
  const CHalf<P64> Zp = p ? a.Z[1] : a.Z[0], Zq = p ? a.Z[0] : a.Z[1];
  const long xf = active ? nbr[x * 8 + MU] : 0;
  const int base = int(threadIdx.x & 63) - lane;  // first lane of the segment in the wave
  const int e = lane < 9 ? lane : 8;              // (lanes >= 9 repeat element 8 and store nothing)
  const int r = e / 3, c = e - 3 * r;
  const C q1 = link_term<MU, -1, SEG>(Wq, xf, Zp, x, a.Ls, lane, active, part);
  const C q2 = link_term<MU, +1, SEG>(Wp, x, Zq, xf, a.Ls, lane, active, part);
  int code = 0;
  if (active) code = lsrc[x * 8 + MU];
  const long l = code >> 1;
  const double ph = (code & 1) ? -1.0 : 1.0;
  C out;
  if (a.kind == 0) {
    // M = Q2 U^+ - U Q1 ; F = -1/2 [ (M - M^+)/2 - tr(M - M^+)/6 ]:  M[r][c] and M[c][r] here
    C mrc = {0.0, 0.0}, mcr = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const C q2rk = shfl_c(q2, base + r * 3 + k), q2ck = shfl_c(q2, base + c * 3 + k);
      const C q1kc = shfl_c(q1, base + k * 3 + c), q1kr = shfl_c(q1, base + k * 3 + r);
      C urk = {0.0, 0.0}, uck = {0.0, 0.0};
      if (active) {
        urk = {ph * a.U[l * 9 + r * 3 + k].x, ph * a.U[l * 9 + r * 3 + k].y};
        uck = {ph * a.U[l * 9 + c * 3 + k].x, ph * a.U[l * 9 + c * 3 + k].y};
      }
      mrc = cfma(q2rk, cconj(uck), mrc) - cmul(urk, q1kc);
      mcr = cfma(q2ck, cconj(urk), mcr) - cmul(uck, q1kr);
    }
    // tr(M - M^+) = 2 i Im tr M: the diagonal elements are held by lanes 0, 4, 8
    const double trim = __shfl(mrc.im, base + 0, 64) + __shfl(mrc.im, base + 4, 64) + __shfl(mrc.im, base + 8, 64);
    C ta = {0.5 * (mrc.re - mcr.re), 0.5 * (mrc.im + mcr.im)};
    if (r == c) ta.im -= trim / 3.0;
    out = {-0.5 * ta.re, -0.5 * ta.im};
  } else {
    // G = -ph (Q1^+ + Q2)
    const C q1t = shfl_c(q1, base + c * 3 + r);
    out = {-ph * (q1t.re + q2.re), -ph * (-q1t.im + q2.im)};
  }
  if (!active || lane >= 9) return;
  double2 v = make_double2(a.coef * out.re, a.coef * out.im);
  if (a.accumulate) {
    const double2 o = a.F[l * 9 + e];
    v.x += o.x;
    v.y += o.y;
  }
  a.F[l * 9 + e] = v;
}

// SEG lanes per link (SEG a power of two, at least Ls when Ls <= 64).  One wave takes 64 / SEG
// sites in one direction mu (so that the branch on mu is uniform over the wave); four consecutive
// waves take the same sites in the four directions.
template <int SEG>
__global__ void __launch_bounds__(256) force_kernel(ForceArgs a) {
  constexpr int SPW = 64 / SEG;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long wave = t >> 6;
  const int mu = int(wave & 3);
  const long j = (wave >> 2) * SPW + ((t & 63) / SEG);  // site index over both parities
  const int lane = int(t & (SEG - 1));
  const bool active = j < 2 * a.nsites;
  const int p = j >= a.nsites ? 1 : 0;
  const long x = active ? j - p * a.nsites : 0;
  __shared__ C part[256 * 9];  // the lanes' partial sums of one term
  switch (mu) {
    case 0: force_link<0, SEG>(a, p, x, lane, active, part); break;
    case 1: force_link<1, SEG>(a, p, x, lane, active, part); break;
    case 2: force_link<2, SEG>(a, p, x, lane, active, part); break;
    default: force_link<3, SEG>(a, p, x, lane, active, part); break;
  }
}

int launch_force(const GeomTables& g, int Ls, CHalf<P64> W_e, CHalf<P64> W_o, CHalf<P64> Z_e, CHalf<P64> Z_o,
                 const double2* U_natural, int tbc, const int dims[4], int kind, double2* F, hipStream_t st,
                 double coef, int accumulate) {
  (void)tbc;
  (void)dims;
  ForceArgs a;
  a.W[0] = W_e; a.W[1] = W_o;
  a.Z[0] = Z_e; a.Z[1] = Z_o;
  a.nbr[0] = g.nbr[0]; a.nbr[1] = g.nbr[1];
  a.linksrc[0] = g.linksrc[0]; a.linksrc[1] = g.linksrc[1];
  a.U = U_natural;
  a.nsites = g.nsites;
  a.Ls = Ls;
  a.kind = kind;
  a.coef = coef;
  a.accumulate = accumulate;
  a.F = F;
  // lanes per link: the smallest power of two covering Ls, at least 16 (the nine elements of the
  // result are spread over the segment) and at most 64; 4 waves per 64 / seg sites
  int seg = 16;
  while (seg < Ls && seg < 64) seg <<= 1;
  const long spw = 64 / seg;
  const long waves = 4 * ((2 * g.nsites + spw - 1) / spw);
  const unsigned blocks = (unsigned)((waves * 64 + 255) / 256);
  switch (seg) {
    case 16: hipLaunchKernelGGL(force_kernel<16>, dim3(blocks), dim3(256), 0, st, a); break;
    case 32: hipLaunchKernelGGL(force_kernel<32>, dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL(force_kernel<64>, dim3(blocks), dim3(256), 0, st, a); break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------------ SU(3) exponential
__device__ void mat3_mul(const C* A, const C* B, C* R) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(A[r * 3 + k], B[k * 3 + c], s);
      R[r * 3 + c] = s;
    }
}

// exp(i Q) for Hermitian traceless Q:  f0 + f1 Q + f2 Q^2  (Morningstar-Peardon)
__device__ void expi_hermitian(const C Q[9], C E[9]) {
  C Q2[9];
  mat3_mul(Q, Q, Q2);
  const double c1 = 0.5 * (Q2[0].re + Q2[4].re + Q2[8].re);
  C f0, f1, f2;
  if (c1 < 1e-12) {
    // |Q| < 1e-6: series through Q^2 is exact to rounding for these terms; keep to third order
    // exp(iQ) = 1 + iQ - Q^2/2 - i Q^3/6 ; with Q^3 = c1 Q + c0 (Cayley-Hamilton for traceless Q)
    C Q3[9];
    mat3_mul(Q2, Q, Q3);
    const double c0 = (Q3[0].re + Q3[4].re + Q3[8].re) / 3.0;
    f0 = {1.0, -c0 / 6.0};
    f1 = {0.0, 1.0 - c1 / 6.0};
    f2 = {-0.5, 0.0};
  } else {
    C Q3[9];
    mat3_mul(Q2, Q, Q3);
    double c0 = (Q3[0].re + Q3[4].re + Q3[8].re) / 3.0;  // det Q
    const bool neg = c0 < 0.0;
    if (neg) c0 = -c0;
    const double c0max = 2.0 * pow(c1 / 3.0, 1.5);
    double r = c0 / c0max;
    if (r > 1.0) r = 1.0;
    const double theta = acos(r);
    const double u = sqrt(c1 / 3.0) * cos(theta / 3.0);
    const double w = sqrt(c1) * sin(theta / 3.0);
    const double u2 = u * u, w2 = w * w;
    const double xi0 = fabs(w) < 0.05 ? 1.0 - w2 / 6.0 * (1.0 - w2 / 20.0 * (1.0 - w2 / 42.0)) : sin(w) / w;
    const double cw = cos(w);
    const C e2iu = {cos(2.0 * u), sin(2.0 * u)};
    const C emiu = {cos(u), -sin(u)};
    const C h0 = cmul(C{u2 - w2, 0.0}, e2iu) + cmul(emiu, C{8.0 * u2 * cw, 2.0 * u * (3.0 * u2 + w2) * xi0});
    const C h1 = cmul(C{2.0 * u, 0.0}, e2iu) - cmul(emiu, C{2.0 * u * cw, -(3.0 * u2 - w2) * xi0});
    const C h2 = e2iu - cmul(emiu, C{cw, 3.0 * u * xi0});
    const double inv = 1.0 / (9.0 * u2 - w2);
    f0 = inv * h0;
    f1 = inv * h1;
    f2 = inv * h2;
    if (neg) {
      f0 = cconj(f0);
      f1 = {-f1.re, f1.im};
      f2 = cconj(f2);
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    C v = cmul(f1, Q[k]) + cmul(f2, Q2[k]);
    if (k % 4 == 0) v = v + f0;
    E[k] = v;
  }
}

// U' = exp(-eps F) U, F anti-Hermitian traceless: -eps F = i Q with Q = i eps F Hermitian
__global__ void __launch_bounds__(256) fg_update_kernel(const double2* F, const double2* U, double eps, double2* Uout,
                                                         long nlinks) {
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlinks) return;
  C Q[9], E[9], Ul[9], R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 f = F[l * 9 + k];
    Q[k] = {-eps * f.y, eps * f.x};  // i eps F
    Ul[k] = {U[l * 9 + k].x, U[l * 9 + k].y};
  }
  // enforce exact hermiticity / tracelessness of Q against rounding in F
  C Qh[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C a = Q[r * 3 + c], b = cconj(Q[c * 3 + r]);
      Qh[r * 3 + c] = {0.5 * (a.re + b.re), 0.5 * (a.im + b.im)};
    }
  const double tr = (Qh[0].re + Qh[4].re + Qh[8].re) / 3.0;
  Qh[0].re -= tr; Qh[4].re -= tr; Qh[8].re -= tr;
  expi_hermitian(Qh, E);
  mat3_mul(E, Ul, R);
#pragma unroll
  for (int k = 0; k < 9; ++k) Uout[l * 9 + k] = make_double2(R[k].re, R[k].im);
}

int launch_fg_update(const double2* F, const double2* U, double eps, double2* Uout, long nlinks, hipStream_t st) {
  if (nlinks <= 0) return 0;
  hipLaunchKernelGGL(fg_update_kernel, dim3((unsigned)((nlinks + 255) / 256)), dim3(256), 0, st, F, U, eps, Uout,
                     nlinks);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace dwf
