// Device-side building blocks for gfx950: storage precisions, complex
// arithmetic, and the chiral-basis spin projectors (1 -+ gamma_mu).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace dwf {

// ----------------------------------------------------------------- complex
template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmake(R a, R b) { return {a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <typename R>
__device__ __forceinline__ cx<R> ci(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> acc) {  // acc + a*b
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}

// ----------------------------------------------------------------- bf16 (round to nearest even)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ----------------------------------------------------------------- storage precisions
// Each precision stores one complex number as a pair (re, im) of its storage
// type; arithmetic is FP64 for FP64 and FP32 for everything else.  FP16 spinors
// carry a per-(site, s) FP32 norm (max |component| of the 5D site).
struct P64 {
  using S = double2;
  using R = double;
  static constexpr bool NORM = false;
  static constexpr int ID = 0;
  __device__ __forceinline__ static cx<R> ld(const S& v) { return {v.x, v.y}; }
  __device__ __forceinline__ static S st(cx<R> a) { return make_double2(a.re, a.im); }
};
struct P32 {
  using S = float2;
  using R = float;
  static constexpr bool NORM = false;
  static constexpr int ID = 1;
  __device__ __forceinline__ static cx<R> ld(const S& v) { return {v.x, v.y}; }
  __device__ __forceinline__ static S st(cx<R> a) { return make_float2(a.re, a.im); }
};
struct P16 {
  using S = __half2;
  using R = float;
  static constexpr bool NORM = true;
  static constexpr int ID = 2;
  __device__ __forceinline__ static cx<R> ld(const S& v) {
    float2 f = __half22float2(v);
    return {f.x, f.y};
  }
  __device__ __forceinline__ static S st(cx<R> a) { return __floats2half2_rn(a.re, a.im); }
};
struct PB16 {
  using S = uint32_t;
  using R = float;
  static constexpr bool NORM = false;
  static constexpr int ID = 3;
  __device__ __forceinline__ static cx<R> ld(const S& v) {
    return {bf16_to_f32(uint16_t(v & 0xffffu)), bf16_to_f32(uint16_t(v >> 16))};
  }
  __device__ __forceinline__ static S st(cx<R> a) {
    return uint32_t(f32_to_bf16(a.re)) | (uint32_t(f32_to_bf16(a.im)) << 16);
  }
};

// A half field of one parity: data[(x_cb*12 + k)*Ls + s], norm[x_cb*Ls + s] (FP16 only)
template <typename P>
struct Half {
  typename P::S* data;
  float* norm;
};
template <typename P>
struct CHalf {
  const typename P::S* data;
  const float* norm;
};

// bytes of one half field (nsites 4D checkerboard sites, Ls slices)
template <typename P>
__host__ __device__ inline size_t half_bytes(long nsites, int Ls) {
  size_t b = size_t(nsites) * 12 * Ls * sizeof(typename P::S);
  if (P::NORM) b += size_t(nsites) * Ls * sizeof(float);
  b = (b + 255) & ~size_t(255);
  return b;
}

template <typename P>
__host__ __device__ inline Half<P> half_view(void* base, long nsites, int Ls) {
  Half<P> h;
  h.data = reinterpret_cast<typename P::S*>(base);
  h.norm = P::NORM ? reinterpret_cast<float*>(reinterpret_cast<char*>(base) +
                                              size_t(nsites) * 12 * Ls * sizeof(typename P::S))
                   : nullptr;
  return h;
}
template <typename P>
__host__ __device__ inline CHalf<P> chalf_view(const void* base, long nsites, int Ls) {
  Half<P> h = half_view<P>(const_cast<void*>(base), nsites, Ls);
  return {h.data, h.norm};
}

// Load the 12 complex components of 5D site (x, s)
template <typename P>
__device__ __forceinline__ void load_spinor(CHalf<P> f, long x, int s, int Ls, cx<typename P::R> v[12]) {
  using R = typename P::R;
  const typename P::S* p = f.data + size_t(x) * 12 * Ls + s;
#pragma unroll
  for (int k = 0; k < 12; ++k) v[k] = P::ld(p[k * Ls]);
  if constexpr (P::NORM) {
    const R n = f.norm[size_t(x) * Ls + s];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = n * v[k];
  }
}

// Load spin components [k0, k0+6) of 5D site (x, s)
template <typename P>
__device__ __forceinline__ void load_half_spinor(CHalf<P> f, long x, int s, int Ls, int k0, cx<typename P::R> v[6]) {
  using R = typename P::R;
  const typename P::S* p = f.data + (size_t(x) * 12 + k0) * Ls + s;
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = P::ld(p[k * Ls]);
  if constexpr (P::NORM) {
    const R n = f.norm[size_t(x) * Ls + s];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = n * v[k];
  }
}

template <typename P>
__device__ __forceinline__ void store_spinor(Half<P> f, long x, int s, int Ls, const cx<typename P::R> v[12]) {
  using R = typename P::R;
  typename P::S* p = f.data + size_t(x) * 12 * Ls + s;
  if constexpr (P::NORM) {
    R m = R(0);
#pragma unroll
    for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
    const R n = m > R(0) ? m : R(1);
    const R inv = R(1) / n;
    f.norm[size_t(x) * Ls + s] = n;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k * Ls] = P::st(inv * v[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k * Ls] = P::st(v[k]);
  }
}

// ----------------------------------------------------------------- spin projection
// Chiral basis: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]].
// For the projector (1 + sg g_mu), sg = +-1, the two independent rows are
//   h0 = psi0 + a0 psi_j0,  h1 = psi1 + a1 psi_j1
// and rows 2, 3 are multiples of h0/h1.  (Derived from the matrices above.)
//   mu=x: h0 = psi0 - sg i psi3, h1 = psi1 - sg i psi2; r2 = sg i h1, r3 = sg i h0
//   mu=y: h0 = psi0 - sg psi3,   h1 = psi1 + sg psi2;   r2 = sg h1,   r3 = -sg h0
//   mu=z: h0 = psi0 - sg i psi2, h1 = psi1 + sg i psi3; r2 = sg i h0, r3 = -sg i h1
//   mu=t: h0 = psi0 + sg psi2,   h1 = psi1 + sg psi3;   r2 = sg h0,   r3 = sg h1
// the two rows for one colour, from the four spin components p0..p3 of that colour
template <int MU, int SG, typename R>
__device__ __forceinline__ void project_colour(cx<R> p0, cx<R> p1, cx<R> p2, cx<R> p3, cx<R>& h0, cx<R>& h1) {
  const R sg = R(SG);
  if constexpr (MU == 0) {
    h0 = p0 - sg * ci(p3);
    h1 = p1 - sg * ci(p2);
  } else if constexpr (MU == 1) {
    h0 = p0 - sg * p3;
    h1 = p1 + sg * p2;
  } else if constexpr (MU == 2) {
    h0 = p0 - sg * ci(p2);
    h1 = p1 + sg * ci(p3);
  } else {
    h0 = p0 + sg * p2;
    h1 = p1 + sg * p3;
  }
}
template <int MU, int SG, typename R>
__device__ __forceinline__ void project(const cx<R> psi[12], cx<R> h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) project_colour<MU, SG, R>(psi[c], psi[3 + c], psi[6 + c], psi[9 + c], h[c], h[3 + c]);
}

// acc += (1 + sg g_mu)-reconstruction of the projected, link-multiplied half spinor u
template <int MU, int SG, typename R>
__device__ __forceinline__ void reconstruct_acc(const cx<R> u[6], cx<R> acc[12]) {
  const R sg = R(SG);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R> u0 = u[c], u1 = u[3 + c];
    acc[0 * 3 + c] = acc[0 * 3 + c] + u0;
    acc[1 * 3 + c] = acc[1 * 3 + c] + u1;
    if constexpr (MU == 0) {
      acc[2 * 3 + c] = acc[2 * 3 + c] + sg * ci(u1);
      acc[3 * 3 + c] = acc[3 * 3 + c] + sg * ci(u0);
    } else if constexpr (MU == 1) {
      acc[2 * 3 + c] = acc[2 * 3 + c] + sg * u1;
      acc[3 * 3 + c] = acc[3 * 3 + c] - sg * u0;
    } else if constexpr (MU == 2) {
      acc[2 * 3 + c] = acc[2 * 3 + c] + sg * ci(u0);
      acc[3 * 3 + c] = acc[3 * 3 + c] - sg * ci(u1);
    } else {
      acc[2 * 3 + c] = acc[2 * 3 + c] + sg * u0;
      acc[3 * 3 + c] = acc[3 * 3 + c] + sg * u1;
    }
  }
}

// u = M h for both half-spinor rows (M: 3x3 complex, row-major)
template <typename R>
__device__ __forceinline__ void su3_mul_half(const cx<R> M[9], const cx<R> h[6], cx<R> u[6]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> s = cmul(M[a * 3 + 0], h[r * 3 + 0]);
      s = cfma(M[a * 3 + 1], h[r * 3 + 1], s);
      s = cfma(M[a * 3 + 2], h[r * 3 + 2], s);
      u[r * 3 + a] = s;
    }
}

// ----------------------------------------------------------------- fifth-dimension operators along s
// Each site-local operator of the even-odd DWF/Moebius system is, per chirality, a
// bidiagonal factor (a1 + b1 S_d1) followed optionally by the inverse of another
// bidiagonal (alpha + beta S_d2), where S_{-1} x_s = x_{s-1} (x_{-1} = -m x_{Ls-1}) and
// S_{+1} x_s = x_{s+1} (x_{Ls} = -m x_0).  Chirality 0 = spins 0,1 (P+), 1 = spins 2,3 (P-).
template <typename R>
struct FifthChir {
  R a1, b1;           // bidiagonal factor; b1 == 0: scalar
  R inv_alpha, a;     // inverse of (alpha + beta S_d2): 1/alpha and a = -beta/alpha
  R corr;             // m / (1 + m a^Ls)
  int d1, d2;         // shift directions (-1 or +1)
  int has_inv;
};
template <typename R>
struct FifthScan {
  FifthChir<R> ch[2];
  R m;
};

// Apply the operator to the 12 components v[] held by this lane (slice s) when the Ls
// lanes of a site are the consecutive lanes [seg*Ls, seg*Ls + Ls) of one wave.  The
// inverse of (alpha + beta S_d) is the first-order recurrence y_s = u_s + a y_{s-+1},
// u = w/alpha: a Hillis-Steele scan over the segment (log2 Ls shuffle steps) with zero
// start, then the cyclic boundary y_{-1} = -m y_{Ls-1} (resp. y_{Ls} = -m y_0) is
// restored in closed form:  y_s = P_s - m a^{s+1} P_{Ls-1} / (1 + m a^Ls)  (forward)
// or y_s = Q_s - m a^{Ls-s} Q_0 / (1 + m a^Ls)  (backward).
template <int LSEG, typename R>
__device__ __forceinline__ R seg_shfl(R v, int src) {
  return __shfl(v, src, LSEG);
}

template <int LSEG, typename R>
__device__ __forceinline__ void fifth_scan_apply(cx<R> v[12], int s, const FifthScan<R>& e) {
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const FifthChir<R> c = e.ch[ch];
    // bidiagonal factor
    if (c.b1 != R(0)) {
      const int src = (s + c.d1) & (LSEG - 1);
      const bool wrap = (c.d1 < 0) ? (s == 0) : (s == LSEG - 1);
      const R f = wrap ? -e.m * c.b1 : c.b1;
#pragma unroll
      for (int k = ch * 6; k < ch * 6 + 6; ++k) {
        const R nr = seg_shfl<LSEG>(v[k].re, src), ni = seg_shfl<LSEG>(v[k].im, src);
        v[k] = {c.a1 * v[k].re + f * nr, c.a1 * v[k].im + f * ni};
      }
    } else if (c.a1 != R(1)) {
#pragma unroll
      for (int k = ch * 6; k < ch * 6 + 6; ++k) v[k] = c.a1 * v[k];
    }
    if (!c.has_inv) continue;
    // inverse of the bidiagonal (alpha + beta S_d2)
#pragma unroll
    for (int k = ch * 6; k < ch * 6 + 6; ++k) v[k] = c.inv_alpha * v[k];
    R apow = c.a;
    if (c.d2 < 0) {
#pragma unroll
      for (int off = 1; off < LSEG; off <<= 1) {
#pragma unroll
        for (int k = ch * 6; k < ch * 6 + 6; ++k) {
          const R tr = __shfl_up(v[k].re, off, LSEG), ti = __shfl_up(v[k].im, off, LSEG);
          if (s >= off) v[k] = {v[k].re + apow * tr, v[k].im + apow * ti};
        }
        apow *= apow;
      }
      // a^{s+1}
      R as = R(1), base = c.a;
      for (int e2 = s + 1; e2; e2 >>= 1) {
        if (e2 & 1) as *= base;
        base *= base;
      }
      const R w = -c.corr * as;
#pragma unroll
      for (int k = ch * 6; k < ch * 6 + 6; ++k) {
        const R lr = seg_shfl<LSEG>(v[k].re, LSEG - 1), li = seg_shfl<LSEG>(v[k].im, LSEG - 1);
        v[k] = {v[k].re + w * lr, v[k].im + w * li};
      }
    } else {
#pragma unroll
      for (int off = 1; off < LSEG; off <<= 1) {
#pragma unroll
        for (int k = ch * 6; k < ch * 6 + 6; ++k) {
          const R tr = __shfl_down(v[k].re, off, LSEG), ti = __shfl_down(v[k].im, off, LSEG);
          if (s + off < LSEG) v[k] = {v[k].re + apow * tr, v[k].im + apow * ti};
        }
        apow *= apow;
      }
      // a^{Ls-s}
      R as = R(1), base = c.a;
      for (int e2 = LSEG - s; e2; e2 >>= 1) {
        if (e2 & 1) as *= base;
        base *= base;
      }
      const R w = -c.corr * as;
#pragma unroll
      for (int k = ch * 6; k < ch * 6 + 6; ++k) {
        const R fr = seg_shfl<LSEG>(v[k].re, 0), fi = seg_shfl<LSEG>(v[k].im, 0);
        v[k] = {v[k].re + w * fr, v[k].im + w * fi};
      }
    }
  }
}

// XCD-aware block order: the hardware deals workgroups round-robin over the 8
// XCDs; remap so that each XCD walks one contiguous range of the lattice and
// neighbouring sites share its L2.
__device__ __forceinline__ long xcd_block(long bid, long nblocks) {
  const long q = nblocks >> 3, r = nblocks & 7;
  const long xcd = bid & 7, idx = bid >> 3;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

}  // namespace dwf
