// Packing, precision conversion, BLAS-1 and deterministic FP64 reductions on
// 5D half fields (layout [x_cb][12][Ls], one thread per 5D site).
#include "hop_impl.hpp"

namespace dwf {

static constexpr int RED_THREADS = 256;
static constexpr int RED_MAX_BLOCKS = 1024;

int reduction_blocks(long n5) {
  long b = (n5 + RED_THREADS - 1) / RED_THREADS;
  if (b > RED_MAX_BLOCKS) b = RED_MAX_BLOCKS;
  if (b < 1) b = 1;
  return int(b);
}

template <typename P>
__device__ __forceinline__ double site_norm2(const cx<typename P::R> v[12]) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 12; ++k) s += double(v[k].re) * double(v[k].re) + double(v[k].im) * double(v[k].im);
  return s;
}

// --------------------------------------------------------------------------- reductions
template <typename P>
__global__ void __launch_bounds__(RED_THREADS) norm2_kernel(CHalf<P> a, long n5, int Ls, double* partials) {
  __shared__ double red[16];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n5; i += (long)gridDim.x * blockDim.x) {
    const long x = i / Ls;
    const int s = int(i - x * Ls);
    cx<typename P::R> v[12];
    load_spinor<P>(a, x, s, Ls, v);
    acc += site_norm2<P>(v);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename P>
__global__ void __launch_bounds__(RED_THREADS) dot_kernel(CHalf<P> a, CHalf<P> b, long n5, int Ls, double* partials) {
  __shared__ double red[16];
  double re = 0.0, im = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n5; i += (long)gridDim.x * blockDim.x) {
    const long x = i / Ls;
    const int s = int(i - x * Ls);
    cx<typename P::R> u[12], v[12];
    load_spinor<P>(a, x, s, Ls, u);
    load_spinor<P>(b, x, s, Ls, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      re += double(u[k].re) * double(v[k].re) + double(u[k].im) * double(v[k].im);
      im += double(u[k].re) * double(v[k].im) - double(u[k].im) * double(v[k].re);
    }
  }
  const double tr = block_sum(re, red);
  __syncthreads();
  const double ti = block_sum(im, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = tr;
    partials[2 * blockIdx.x + 1] = ti;
  }
}

// One workgroup of 1024 threads; each thread keeps four independent partial sums (loads in
// flight) over a fixed set of indices, combined in a fixed order: deterministic.
__global__ void __launch_bounds__(1024) reduce_kernel(const double* partials, int n, int ncomp, double* scalars,
                                                       int slot, int mode, int hist) {
  __shared__ double red[16];
  for (int c = 0; c < ncomp; ++c) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int stride = blockDim.x;
    int i = threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
      a0 += partials[i * ncomp + c];
      a1 += partials[(i + stride) * ncomp + c];
      a2 += partials[(i + 2 * stride) * ncomp + c];
      a3 += partials[(i + 3 * stride) * ncomp + c];
    }
    for (; i < n; i += stride) a0 += partials[i * ncomp + c];
    const double t = block_sum((a0 + a1) + (a2 + a3), red);
    __syncthreads();
    if (threadIdx.x == 0) {
      scalars[slot + c] = t;
      if (mode == 1) {
        // alpha = rr / qq
        scalars[S_ALPHA] = scalars[S_RR] / t;
        if (hist >= 0) scalars[S_AHIST + hist] = scalars[S_ALPHA];
      } else if (mode == 2) {
        // beta = rr_new / rr ; rr = rr_new
        scalars[S_BETA] = t / scalars[S_RR];
        scalars[S_RR] = t;
      }
    }
  }
}

int launch_reduce(const double* partials, int n, int ncomp, double* scalars, int slot, int mode, hipStream_t st,
                  int hist) {
  if (hist >= XFLUSH_MAX) return -1;
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, partials, n, ncomp, scalars, slot, mode, hist);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ void set_scalar_kernel(double* scalars, int slot, double v) {
  if (threadIdx.x == 0) scalars[slot] = v;
}
int launch_set_scalar(double* scalars, int slot, double v, hipStream_t st) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, st, scalars, slot, v);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P>
int launch_norm2(CHalf<P> a, long n5, int Ls, double* partials, hipStream_t st) {
  const int nb = reduction_blocks(n5);
  hipLaunchKernelGGL((norm2_kernel<P>), dim3(nb), dim3(RED_THREADS), 0, st, a, n5, Ls, partials);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P>
int launch_dot(CHalf<P> a, CHalf<P> b, long n5, int Ls, double* partials, hipStream_t st) {
  const int nb = reduction_blocks(n5);
  hipLaunchKernelGGL((dot_kernel<P>), dim3(nb), dim3(RED_THREADS), 0, st, a, b, n5, Ls, partials);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// --------------------------------------------------------------------------- elementwise
template <typename P>
__global__ void __launch_bounds__(256) axpby_kernel(double a, CHalf<P> x, double b, Half<P> y, long n5, int Ls) {
  using R = typename P::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  cx<R> u[12], v[12];
  load_spinor<P>(x, xs, s, Ls, u);
  if (b != 0.0) {
    load_spinor<P>(CHalf<P>{y.data, y.norm}, xs, s, Ls, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = R(a) * u[k] + R(b) * v[k];
  } else {
    // y is not read: its previous contents may be uninitialised (0 * NaN = NaN)
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = R(a) * u[k];
  }
  store_spinor<P>(y, xs, s, Ls, v);
}

template <typename P>
int launch_axpby(double a, CHalf<P> x, double b, Half<P> y, long n5, int Ls, hipStream_t st) {
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((axpby_kernel<P>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, a, x, b, y, n5, Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename Pi, typename Po>
__global__ void __launch_bounds__(256) convert_kernel(CHalf<Pi> in, Half<Po> out, long n5, int Ls) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  cx<typename Pi::R> u[12];
  cx<typename Po::R> v[12];
  load_spinor<Pi>(in, xs, s, Ls, u);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = {typename Po::R(u[k].re), typename Po::R(u[k].im)};
  store_spinor<Po>(out, xs, s, Ls, v);
}

template <typename Pi, typename Po>
int launch_convert(CHalf<Pi> in, Half<Po> out, long n5, int Ls, hipStream_t st) {
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((convert_kernel<Pi, Po>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, in, out, n5, Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// p_out = r + beta p_in ; the first thread also records rr_new as the current |r|^2 (S_RR)
template <typename P>
__global__ void __launch_bounds__(256) cg_pupdate_kernel(CHalf<P> r, CHalf<P> pin, Half<P> pout, double beta,
                                                          double* scalars, double rr_new, long n5, int Ls) {
  using R = typename P::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) scalars[S_RR] = rr_new;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  cx<R> rv[12], pv[12];
  load_spinor<P>(r, xs, s, Ls, rv);
  if (beta != 0.0) {
    load_spinor<P>(pin, xs, s, Ls, pv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      pv[k].re = R(double(rv[k].re) + beta * double(pv[k].re));
      pv[k].im = R(double(rv[k].im) + beta * double(pv[k].im));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) pv[k] = rv[k];
  }
  store_spinor<P>(pout, xs, s, Ls, pv);
}

template <typename P>
int launch_cg_pupdate(CHalf<P> r, CHalf<P> pin, Half<P> pout, double beta, double* scalars, double rr_new, long n5,
                      int Ls, hipStream_t st) {
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((cg_pupdate_kernel<P>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, r, pin, pout,
                     beta, scalars, rr_new, n5, Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// x += sum_j alpha_j p_j over the pending CG directions (alpha_j = scalars[S_AHIST + slot_j]):
// the solution increment of several iterations in one pass, the sum formed in FP64
template <typename P, typename Px>
__global__ void __launch_bounds__(256) xflush_kernel(Half<Px> x, XFlush<P> f, const double* scalars, long n5,
                                                      int Ls) {
  using RX = typename Px::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  double sr[12], si[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) sr[k] = si[k] = 0.0;
  for (int j = 0; j < f.n; ++j) {
    const double a = scalars[S_AHIST + f.slot[j]];
    cx<typename P::R> pv[12];
    load_spinor<P>(f.p[j], xs, s, Ls, pv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      sr[k] += a * double(pv[k].re);
      si[k] += a * double(pv[k].im);
    }
  }
  cx<RX> xv[12];
  load_spinor<Px>(CHalf<Px>{x.data, x.norm}, xs, s, Ls, xv);
#pragma unroll
  for (int k = 0; k < 12; ++k) xv[k] = {RX(double(xv[k].re) + sr[k]), RX(double(xv[k].im) + si[k])};
  store_spinor<Px>(x, xs, s, Ls, xv);
}

template <typename P, typename Px>
int launch_xflush(Half<Px> x, const XFlush<P>& f, const double* scalars, long n5, int Ls, hipStream_t st) {
  if (f.n < 0 || f.n > XFLUSH_MAX) return -1;
  for (int j = 0; j < f.n; ++j)
    if (f.slot[j] < 0 || f.slot[j] >= XFLUSH_MAX || !f.p[j].data) return -1;
  if (n5 <= 0 || f.n == 0) return 0;
  hipLaunchKernelGGL((xflush_kernel<P, Px>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, x, f, scalars, n5,
                     Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// p_out = r + beta p_in and fp = (fb + fc S~) p_out: the p update of CG with the Moebius input
// factor F = b + c S~ applied to the new direction, so that the hops of M p need no prologue.
// Each thread forms the new p on its slice and on the two neighbouring slices F reads (upper
// spins of s-1, lower spins of s+1; -m at the ends); p_in and p_out are different buffers.
template <typename P>
__global__ void __launch_bounds__(256) cg_pupdate_f_kernel(CHalf<P> r, CHalf<P> pin, Half<P> pout, Half<P> fp,
                                                            double beta, double* scalars, double rr_new, long n5,
                                                            int Ls, double fb0, double fc0, double fm,
                                                            const typename P::R* bs, const typename P::R* cs) {
  using R = typename P::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) scalars[S_RR] = rr_new;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  const double fb = bs ? double(bs[s]) : fb0, fc = cs ? double(cs[s]) : fc0;  // coefficients of slice s
  int su = s - 1, sl = s + 1;
  R fu = R(fc), fl = R(fc);
  if (su < 0) { su = Ls - 1; fu = R(-fc * fm); }
  if (sl >= Ls) { sl = 0; fl = R(-fc * fm); }
  cx<R> v[12], up[6], lo[6];
  load_spinor<P>(r, xs, s, Ls, v);
  load_half_spinor<P>(r, xs, su, Ls, 0, up);
  load_half_spinor<P>(r, xs, sl, Ls, 6, lo);
  if (beta != 0.0) {
    cx<R> pv[12], pu[6], pl[6];
    load_spinor<P>(pin, xs, s, Ls, pv);
    load_half_spinor<P>(pin, xs, su, Ls, 0, pu);
    load_half_spinor<P>(pin, xs, sl, Ls, 6, pl);
    const R b = R(beta);
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = v[k] + b * pv[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      up[k] = up[k] + b * pu[k];
      lo[k] = lo[k] + b * pl[k];
    }
  }
  store_spinor<P>(pout, xs, s, Ls, v);
  cx<R> f[12];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    f[k] = R(fb) * v[k] + fu * up[k];
    f[6 + k] = R(fb) * v[6 + k] + fl * lo[k];
  }
  store_spinor<P>(fp, xs, s, Ls, f);
}

template <typename P>
int launch_cg_pupdate_f(CHalf<P> r, CHalf<P> pin, Half<P> pout, Half<P> fp, double beta, double* scalars,
                        double rr_new, long n5, int Ls, double b, double c, double m, hipStream_t st,
                        const typename P::R* bs, const typename P::R* cs) {
  if (n5 <= 0) return 0;
  if (pin.data == pout.data || (beta != 0.0 && !pin.data)) return -1;
  hipLaunchKernelGGL((cg_pupdate_f_kernel<P>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, r, pin, pout,
                     fp, beta, scalars, rr_new, n5, Ls, b, c, m, bs, cs);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Domain-wall <-> overlap basis change on a half field (site-local):
//   (P^-1 x)_s = P- x_s + P+ x_{s-1 mod Ls},   (P y)_s = P- y_s + P+ y_{s+1 mod Ls}
// P+ = spins 0,1 (components 0..5), P- = spins 2,3 (components 6..11).
__global__ void __launch_bounds__(256) pshift_kernel(CHalf<P64> in, Half<P64> out, int inverse, long n5, int Ls) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  const int so = inverse ? (s + Ls - 1) % Ls : (s + 1) % Ls;
  cx<double> v[12], up[6];
  load_spinor<P64>(in, xs, s, Ls, v);
  load_half_spinor<P64>(in, xs, so, Ls, 0, up);
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = up[k];
  store_spinor<P64>(out, xs, s, Ls, v);
}

int launch_pshift(CHalf<P64> in, Half<P64> out, int inverse, long nsites, int Ls, hipStream_t st) {
  const long n5 = nsites * Ls;
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL(pshift_kernel, dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, in, out, inverse, n5, Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// out(slice s_out) = scale * in(slice s_in) for every 4D site (fields of different Ls)
__global__ void __launch_bounds__(256) slice_copy_kernel(CHalf<P64> in, int Ls_in, int s_in, Half<P64> out, int Ls_out,
                                                          int s_out, double scale, long nsites) {
  const long xs = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (xs >= nsites) return;
  cx<double> v[12];
  load_spinor<P64>(in, xs, s_in, Ls_in, v);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = scale * v[k];
  store_spinor<P64>(out, xs, s_out, Ls_out, v);
}

int launch_slice_copy(CHalf<P64> in, int Ls_in, int s_in, Half<P64> out, int Ls_out, int s_out, double scale,
                      long nsites, hipStream_t st) {
  if (nsites <= 0) return 0;
  hipLaunchKernelGGL(slice_copy_kernel, dim3((unsigned)((nsites + 255) / 256)), dim3(256), 0, st, in, Ls_in, s_in, out,
                     Ls_out, s_out, scale, nsites);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// 4D even-odd field halves <-> 5D-parity fields.  Slice s of 4D parity q belongs to the 5D
// parity (s + q) mod 2, where it is slot s / 2 of half q: element ((q nsites + x) 12 + k) Ls/2 + s/2
// (FP16 norm: (q nsites + x) Ls/2 + s/2).  Thread per element of the 4D fields (grid-stride).
template <typename P>
__global__ void __launch_bounds__(256) eo5_split_kernel(Half<P> h0, Half<P> h1, Half<P> f5e, Half<P> f5o, long nsites,
                                                        int Ls, int merge) {
  const long per = nsites * 12 * Ls;
  const int LH = Ls / 2;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * per; i += (long)gridDim.x * blockDim.x) {
    const int q = i >= per ? 1 : 0;
    const long r = i - q * per;
    const long xk = r / Ls;  // x_cb * 12 + k
    const int s = int(r - xk * Ls);
    const Half<P> h = q ? h1 : h0;
    const Half<P> f5 = ((s + q) & 1) ? f5o : f5e;
    const long j5 = (q * nsites * 12 + xk) * LH + (s >> 1);
    if (merge) h.data[r] = f5.data[j5];
    else f5.data[j5] = h.data[r];
    if constexpr (P::NORM) {
      const long x = xk / 12;
      if (xk - x * 12 == 0) {
        const long n4 = x * Ls + s, n5 = (q * nsites + x) * LH + (s >> 1);
        if (merge) h.norm[n4] = f5.norm[n5];
        else f5.norm[n5] = h.norm[n4];
      }
    }
  }
}

template <typename P>
int launch_eo5_split(Half<P> h0, Half<P> h1, Half<P> f5_even, Half<P> f5_odd, long nsites, int Ls, int merge,
                     hipStream_t st) {
  if (Ls < 2 || Ls % 2 || nsites <= 0) return -1;
  const long n = 2 * nsites * 12 * Ls;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((eo5_split_kernel<P>), dim3((unsigned)blocks), dim3(256), 0, st, h0, h1, f5_even, f5_odd, nsites,
                     Ls, merge);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
template int launch_eo5_split<P64>(Half<P64>, Half<P64>, Half<P64>, Half<P64>, long, int, int, hipStream_t);
template int launch_eo5_split<P32>(Half<P32>, Half<P32>, Half<P32>, Half<P32>, long, int, int, hipStream_t);
template int launch_eo5_split<P16>(Half<P16>, Half<P16>, Half<P16>, Half<P16>, long, int, int, hipStream_t);
template int launch_eo5_split<PB16>(Half<PB16>, Half<PB16>, Half<PB16>, Half<PB16>, long, int, int, hipStream_t);

// hi += lo ; lo = 0
template <typename Px>
__global__ void __launch_bounds__(256) accumulate_kernel(Half<P64> hi, Half<Px> lo, long n5, int Ls) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / Ls;
  const int s = int(i - xs * Ls);
  cx<double> h[12];
  cx<typename Px::R> l[12];
  load_spinor<P64>(CHalf<P64>{hi.data, nullptr}, xs, s, Ls, h);
  load_spinor<Px>(CHalf<Px>{lo.data, lo.norm}, xs, s, Ls, l);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    h[k].re += double(l[k].re);
    h[k].im += double(l[k].im);
    l[k] = {typename Px::R(0), typename Px::R(0)};
  }
  store_spinor<P64>(hi, xs, s, Ls, h);
  store_spinor<Px>(lo, xs, s, Ls, l);
}

template <typename Px>
int launch_accumulate(Half<P64> hi, Half<Px> lo, long n5, int Ls, hipStream_t st) {
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((accumulate_kernel<Px>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, hi, lo, n5, Ls);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------- interleaved right-hand sides
// Fields holding nrhs right-hand sides interleaved along s: slice s of right-hand side r is slice
// r * RS + s of a field of extent LT = nrhs * RS (one thread per 5D site of the whole field).

// p_out = r + beta_k p_in with beta_k = coef[k] of the slice's right-hand side k (0: p_in unread);
// the first threads also record |r_k|^2 = coef[K + k] at scalars[k S_COUNT + S_RR]
template <typename P>
__global__ void __launch_bounds__(256) ilv_pupdate_kernel(CHalf<P> r, CHalf<P> pin, Half<P> pout, const double* coef,
                                                           double* scalars, long n5, int LT, int RS) {
  using R = typename P::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int K = LT / RS;
  if (i < K) scalars[i * S_COUNT + S_RR] = coef[K + i];
  if (i >= n5) return;
  const double* betas = coef;
  const long xs = i / LT;
  const int s = int(i - xs * LT);
  const double beta = betas[s / RS];
  cx<R> rv[12], pv[12];
  load_spinor<P>(r, xs, s, LT, rv);
  if (beta != 0.0) {
    load_spinor<P>(pin, xs, s, LT, pv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      pv[k].re = R(double(rv[k].re) + beta * double(pv[k].re));
      pv[k].im = R(double(rv[k].im) + beta * double(pv[k].im));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) pv[k] = rv[k];
  }
  store_spinor<P>(pout, xs, s, LT, pv);
}

template <typename P>
int launch_ilv_pupdate(CHalf<P> r, CHalf<P> pin, Half<P> pout, const double* coef, double* scalars, long nsites, int LT,
                       int RS, hipStream_t st) {
  if (RS < 1 || LT % RS != 0 || pin.data == pout.data) return -1;
  const long n5 = nsites * LT;
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((ilv_pupdate_kernel<P>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, r, pin, pout, coef,
                     scalars, n5, LT, RS);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// x += sum_j alpha_{k,j} p_j, alpha_{k,j} = scalars[k S_COUNT + S_AHIST + slot_j] of the slice's
// right-hand side k (the sum in FP64)
template <typename P, typename Px>
__global__ void __launch_bounds__(256) ilv_xflush_kernel(Half<Px> x, XFlush<P> f, const double* scalars, long n5,
                                                          int LT, int RS) {
  using RX = typename Px::R;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / LT;
  const int s = int(i - xs * LT);
  const double* sc = scalars + size_t(s / RS) * S_COUNT;
  double sr[12], si[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) sr[k] = si[k] = 0.0;
  for (int j = 0; j < f.n; ++j) {
    const double a = sc[S_AHIST + f.slot[j]];
    cx<typename P::R> pv[12];
    load_spinor<P>(f.p[j], xs, s, LT, pv);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      sr[k] += a * double(pv[k].re);
      si[k] += a * double(pv[k].im);
    }
  }
  cx<RX> xv[12];
  load_spinor<Px>(CHalf<Px>{x.data, x.norm}, xs, s, LT, xv);
#pragma unroll
  for (int k = 0; k < 12; ++k) xv[k] = {RX(double(xv[k].re) + sr[k]), RX(double(xv[k].im) + si[k])};
  store_spinor<Px>(x, xs, s, LT, xv);
}

template <typename P, typename Px>
int launch_ilv_xflush(Half<Px> x, const XFlush<P>& f, const double* scalars, long nsites, int LT, int RS,
                      hipStream_t st) {
  if (f.n < 0 || f.n > XFLUSH_MAX || RS < 1 || LT % RS != 0) return -1;
  for (int j = 0; j < f.n; ++j)
    if (f.slot[j] < 0 || f.slot[j] >= XFLUSH_MAX || !f.p[j].data) return -1;
  const long n5 = nsites * LT;
  if (n5 <= 0 || f.n == 0) return 0;
  hipLaunchKernelGGL((ilv_xflush_kernel<P, Px>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, x, f, scalars,
                     n5, LT, RS);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// segment r_out of out (extent LT_out) = segment r_in of in (extent LT_in), each of RS slices, with
// conversion between storage precisions (a separate field is a single segment: r = 0, LT = RS)
template <typename Pi, typename Po>
__global__ void __launch_bounds__(256) ilv_move_kernel(CHalf<Pi> in, int LT_in, int r_in, Half<Po> out, int LT_out,
                                                        int r_out, long n5, int RS) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / RS;
  const int s = int(i - xs * RS);
  cx<typename Pi::R> u[12];
  cx<typename Po::R> v[12];
  load_spinor<Pi>(in, xs, r_in * RS + s, LT_in, u);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = {typename Po::R(u[k].re), typename Po::R(u[k].im)};
  store_spinor<Po>(out, xs, r_out * RS + s, LT_out, v);
}

template <typename Pi, typename Po>
int launch_ilv_move(CHalf<Pi> in, int LT_in, int r_in, Half<Po> out, int LT_out, int r_out, long nsites, int RS,
                    hipStream_t st) {
  if (RS < 1 || r_in < 0 || r_out < 0 || (r_in + 1) * RS > LT_in || (r_out + 1) * RS > LT_out) return -1;
  if (static_cast<const void*>(in.data) == static_cast<const void*>(out.data)) return -1;
  const long n5 = nsites * RS;
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((ilv_move_kernel<Pi, Po>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, in, LT_in, r_in,
                     out, LT_out, r_out, n5, RS);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// hi (a separate FP64 field of extent RS) += segment r of lo (extent LT); that segment = 0
template <typename Px>
__global__ void __launch_bounds__(256) ilv_accumulate_kernel(Half<P64> hi, Half<Px> lo, int LT, int r, long n5,
                                                              int RS) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const long xs = i / RS;
  const int s = int(i - xs * RS);
  cx<double> h[12];
  cx<typename Px::R> l[12];
  load_spinor<P64>(CHalf<P64>{hi.data, nullptr}, xs, s, RS, h);
  load_spinor<Px>(CHalf<Px>{lo.data, lo.norm}, xs, r * RS + s, LT, l);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    h[k].re += double(l[k].re);
    h[k].im += double(l[k].im);
    l[k] = {typename Px::R(0), typename Px::R(0)};
  }
  store_spinor<P64>(hi, xs, s, RS, h);
  store_spinor<Px>(lo, xs, r * RS + s, LT, l);
}

template <typename Px>
int launch_ilv_accumulate(Half<P64> hi, Half<Px> lo, int LT, int r, long nsites, int RS, hipStream_t st) {
  if (RS < 1 || r < 0 || (r + 1) * RS > LT) return -1;
  const long n5 = nsites * RS;
  if (n5 <= 0) return 0;
  hipLaunchKernelGGL((ilv_accumulate_kernel<Px>), dim3((unsigned)((n5 + 255) / 256)), dim3(256), 0, st, hi, lo, LT, r,
                     n5, RS);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// zero fill with a kernel (also safe inside captured graphs)
__global__ void __launch_bounds__(256) zero_kernel(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
int launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return 0;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<uint32_t*>(p), n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// --------------------------------------------------------------------------- packing
// gauge: thread per (parity, x_cb, direction); backward links stored daggered,
// boundary phase folded in (linksrc code = 2*(mu*V + i) + phase bit)
template <typename P>
__global__ void __launch_bounds__(256) pack_gauge_kernel(const int* linksrc0, const int* linksrc1, long nsites,
                                                          const double2* nat, typename P::S* packed) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = nsites * 8;
  if (i >= 2 * per) return;
  const int par = i >= per ? 1 : 0;
  const long j = i - par * per;  // x_cb*8 + d
  const int d = int(j & 7);
  const int code = (par ? linksrc1 : linksrc0)[j];
  const long l = code >> 1;
  const double ph = (code & 1) ? -1.0 : 1.0;
  const double2* U = nat + l * 9;
  typename P::S* o = packed + (size_t)par * per * 9 + j * 9;
  using R = typename P::R;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double2 u = d < 4 ? U[r * 3 + c] : U[c * 3 + r];
      if (d >= 4) u.y = -u.y;
      o[r * 3 + c] = P::st({R(ph * u.x), R(ph * u.y)});
    }
}

template <typename P>
int launch_pack_gauge(const GeomTables& g, const double2* natural, typename P::S* packed, hipStream_t st) {
  const long n = 2 * g.nsites * 8;
  hipLaunchKernelGGL((pack_gauge_kernel<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.linksrc[0],
                     g.linksrc[1], g.nsites, natural, packed);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P>
__global__ void __launch_bounds__(256) pack_half_kernel(const int* site, long nsites, long V, int Ls,
                                                         const double2* nat, Half<P> out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsites * Ls) return;
  const long x = i / Ls;
  const int s = int(i - x * Ls);
  const double2* src = nat + ((size_t)s * V + site[x]) * 12;
  cx<typename P::R> v[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = {typename P::R(src[k].x), typename P::R(src[k].y)};
  store_spinor<P>(out, x, s, Ls, v);
}

template <typename P>
int launch_pack_half(const GeomTables& g, int parity, int Ls, const double2* natural, Half<P> out, hipStream_t st) {
  const long n = g.nsites * Ls;
  hipLaunchKernelGGL((pack_half_kernel<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.site[parity],
                     g.nsites, g.V, Ls, natural, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P>
__global__ void __launch_bounds__(256) unpack_half_kernel(const int* site, long nsites, long V, int Ls, CHalf<P> in,
                                                           double2* nat) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsites * Ls) return;
  const long x = i / Ls;
  const int s = int(i - x * Ls);
  double2* dst = nat + ((size_t)s * V + site[x]) * 12;
  cx<typename P::R> v[12];
  load_spinor<P>(in, x, s, Ls, v);
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = make_double2(double(v[k].re), double(v[k].im));
}

template <typename P>
int launch_unpack_half(const GeomTables& g, int parity, int Ls, CHalf<P> in, double2* natural, hipStream_t st) {
  const long n = g.nsites * Ls;
  hipLaunchKernelGGL((unpack_half_kernel<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.site[parity],
                     g.nsites, g.V, Ls, in, natural);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename Pi, typename Po>
__global__ void __launch_bounds__(256) convert_links_kernel(const typename Pi::S* in, typename Po::S* out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const cx<typename Pi::R> v = Pi::ld(in[i]);
  out[i] = Po::st({typename Po::R(v.re), typename Po::R(v.im)});
}

template <typename Pi, typename Po>
int launch_convert_links(const typename Pi::S* in, typename Po::S* out, long n, hipStream_t st) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL((convert_links_kernel<Pi, Po>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// --------------------------------------------------------------------------- instantiations
#define DWF_INST_FIELD(P)                                                                                        \
  template int launch_norm2<P>(CHalf<P>, long, int, double*, hipStream_t);                                       \
  template int launch_dot<P>(CHalf<P>, CHalf<P>, long, int, double*, hipStream_t);                               \
  template int launch_axpby<P>(double, CHalf<P>, double, Half<P>, long, int, hipStream_t);                        \
  template int launch_cg_pupdate<P>(CHalf<P>, CHalf<P>, Half<P>, double, double*, double, long, int, hipStream_t); \
  template int launch_cg_pupdate_f<P>(CHalf<P>, CHalf<P>, Half<P>, Half<P>, double, double*, double, long, int,   \
                                      double, double, double, hipStream_t, const P::R*, const P::R*);           \
  template int launch_pack_gauge<P>(const GeomTables&, const double2*, P::S*, hipStream_t);                      \
  template int launch_pack_half<P>(const GeomTables&, int, int, const double2*, Half<P>, hipStream_t);           \
  template int launch_unpack_half<P>(const GeomTables&, int, int, CHalf<P>, double2*, hipStream_t);              \
  template int launch_convert_links<P64, P>(const P64::S*, P::S*, long, hipStream_t);

DWF_INST_FIELD(P64)
DWF_INST_FIELD(P32)
DWF_INST_FIELD(P16)
DWF_INST_FIELD(PB16)

template int launch_convert<P64, P64>(CHalf<P64>, Half<P64>, long, int, hipStream_t);
template int launch_convert<P64, P32>(CHalf<P64>, Half<P32>, long, int, hipStream_t);
template int launch_convert<P64, P16>(CHalf<P64>, Half<P16>, long, int, hipStream_t);
template int launch_convert<P64, PB16>(CHalf<P64>, Half<PB16>, long, int, hipStream_t);
template int launch_convert<P32, P64>(CHalf<P32>, Half<P64>, long, int, hipStream_t);
template int launch_convert<P16, P64>(CHalf<P16>, Half<P64>, long, int, hipStream_t);
template int launch_convert<PB16, P64>(CHalf<PB16>, Half<P64>, long, int, hipStream_t);
template int launch_convert<P32, P16>(CHalf<P32>, Half<P16>, long, int, hipStream_t);
template int launch_convert<P16, P32>(CHalf<P16>, Half<P32>, long, int, hipStream_t);
template int launch_convert<P32, PB16>(CHalf<P32>, Half<PB16>, long, int, hipStream_t);
template int launch_convert<PB16, P32>(CHalf<PB16>, Half<P32>, long, int, hipStream_t);

template int launch_xflush<P64, P64>(Half<P64>, const XFlush<P64>&, const double*, long, int, hipStream_t);
template int launch_xflush<P32, P32>(Half<P32>, const XFlush<P32>&, const double*, long, int, hipStream_t);
template int launch_xflush<P16, P32>(Half<P32>, const XFlush<P16>&, const double*, long, int, hipStream_t);
template int launch_xflush<PB16, P32>(Half<P32>, const XFlush<PB16>&, const double*, long, int, hipStream_t);

template int launch_accumulate<P32>(Half<P64>, Half<P32>, long, int, hipStream_t);
template int launch_accumulate<P16>(Half<P64>, Half<P16>, long, int, hipStream_t);
template int launch_accumulate<P64>(Half<P64>, Half<P64>, long, int, hipStream_t);

#define DWF_INST_ILV(P, PX)                                                                                      \
  template int launch_ilv_pupdate<P>(CHalf<P>, CHalf<P>, Half<P>, const double*, double*, long, int, int,       \
                                     hipStream_t);                                                               \
  template int launch_ilv_xflush<P, PX>(Half<PX>, const XFlush<P>&, const double*, long, int, int, hipStream_t); \
  template int launch_ilv_move<P, P>(CHalf<P>, int, int, Half<P>, int, int, long, int, hipStream_t);
DWF_INST_ILV(P64, P64)
DWF_INST_ILV(P32, P32)
DWF_INST_ILV(P16, P32)
DWF_INST_ILV(PB16, P32)
template int launch_ilv_move<P64, P32>(CHalf<P64>, int, int, Half<P32>, int, int, long, int, hipStream_t);
template int launch_ilv_move<P64, P16>(CHalf<P64>, int, int, Half<P16>, int, int, long, int, hipStream_t);
template int launch_ilv_move<P64, PB16>(CHalf<P64>, int, int, Half<PB16>, int, int, long, int, hipStream_t);
template int launch_ilv_accumulate<P64>(Half<P64>, Half<P64>, int, int, long, int, hipStream_t);
template int launch_ilv_accumulate<P32>(Half<P64>, Half<P32>, int, int, long, int, hipStream_t);

}  // namespace dwf
