// Wilson hop (the 4D operator the paper counts as its unit of cost, Table 1)
// over a 5D half field, and the site-local fifth-dimension kernel, for gfx950.
//
// Mapping: one thread owns one 4D checkerboard site and NS of its Ls slices
// (s = s0, s0 + Ls/NS, ...); the Ls/NS threads of a site are consecutive, so
// a wave reads contiguous runs of the s-fastest layout [x_cb][12][Ls] for
// every neighbour, and all threads of a site read the same link addresses
// (one request per wave).  Each of the 8 links is loaded once per thread and
// reused for its NS slices.  Spinors are spin-projected to half spinors before
// the SU(3) multiply (two 3x3 mat-vecs instead of four).
//
// Optional fused stages (Sec. 4 operators, even-odd form):
//   prologue  F = b + c S~ applied to each neighbour spinor as it is read
//             (Moebius input factor: needs the upper spins of s-1 and the lower
//             spins of s+1 of the same neighbour, same cache lines);
//   epilogue  per-chirality Ls x Ls matrix along s (A^-1, A^-dag F^dag, ...),
//             through LDS: a workgroup holds all Ls slices of its sites;
//   axpy      out = ax * x + result;  |out|^2 partials per workgroup.
#pragma once
#include "kernels.hpp"

namespace dwf {

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;
}

// LDS elements per site of the staged links: FP16 links are staged as (Uc, Us) pairs
template <typename P>
constexpr int staged_link_elems() { return std::is_same<P, P16>::value ? 160 : 72; }

// dynamic LDS of one hop workgroup: dense-epilogue staging + staged links
template <typename P>
inline size_t hop_lds_bytes(const LaunchCfg& cfg, int Ls, bool epi) {
  size_t b = epi ? size_t(cfg.spb) * 12 * Ls * sizeof(cx<typename P::R>) : 0;
  if (cfg.ll) b += size_t(cfg.spb) * staged_link_elems<P>() * sizeof(typename P::S);
  return b;
}

// Moebius prologue of one slice s: the hop's input becomes b_s psi_s + u P+ psi_{s-1} +
// l P- psi_{s+1} (F = b + c S~ with the -m wrap at the ends of the fifth dimension).  The
// coefficients depend on s only; they are formed once per thread, before the direction loop,
// so that the eight directions form one straight-line block the scheduler can interleave
// (selected per direction, they split it into small blocks and the loads of all directions
// were issued before any arithmetic, which spilled).
template <typename R>
struct ProCoef {
  R b, u, l;
  int su, sl;
};

template <typename P, bool PRO>
__device__ __forceinline__ ProCoef<typename P::R> pro_coef(const HopArgs<P>& a, int s) {
  using R = typename P::R;
  ProCoef<R> c{R(0), R(0), R(0), 0, 0};
  if constexpr (PRO) {
    const int Ls = a.Ls;
    const R pb = a.pbs ? a.pbs[s] : a.pb, pc = a.pcs ? a.pcs[s] : a.pc;  // coefficients of slice s
    c.b = pb;
    c.su = s == 0 ? Ls - 1 : s - 1;
    c.sl = s == Ls - 1 ? 0 : s + 1;
    c.u = s == 0 ? -pc * a.pm : pc;
    c.l = s == Ls - 1 ? -pc * a.pm : pc;
  }
  return c;
}

template <typename P, bool PRO>
__device__ __forceinline__ void load_input(const HopArgs<P>& a, long y, int s, const ProCoef<typename P::R>& pc,
                                           cx<typename P::R> psi[12]) {
  using R = typename P::R;
  load_spinor<P>(a.in, y, s, a.Ls, psi);
  if constexpr (PRO) {
    cx<R> up[6], lo[6];
    load_half_spinor<P>(a.in, y, pc.su, a.Ls, 0, up);  // P+ (spins 0,1) picks psi_{s-1}
    load_half_spinor<P>(a.in, y, pc.sl, a.Ls, 6, lo);  // P- (spins 2,3) picks psi_{s+1}
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      psi[k] = pc.b * psi[k] + pc.u * up[k];
      psi[6 + k] = pc.b * psi[6 + k] + pc.l * lo[k];
    }
  }
}

// FP16 storage: the half spinor is formed in packed FP16 on the norm-scaled values (one
// v_pk_add_f16 per colour and row, the factor i folded into the operand selectors), the
// SU(3) product uses v_dot2_f32_f16 (two FP16 products accumulated in FP32 per
// instruction) on link elements the workgroup stages in the two forms the real and the
// imaginary part need, and the neighbour's norm is applied in the FP32 accumulation.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f16x2 as_f16x2(const __half2& v) {
  f16x2 r;
  __builtin_memcpy(&r, &v, 4);
  return r;
}
__device__ __forceinline__ __half2 from_f16x2(f16x2 v) {
  __half2 r;
  __builtin_memcpy(&r, &v, 4);
  return r;
}
__device__ __forceinline__ f16x2 i_f16x2(f16x2 x) { return f16x2{-x.y, x.x}; }

// One row of the SU(3) product: three v_dot2_f32_f16 chained through the FP32 accumulator,
// on link elements staged as uc = (Ur, -Ui) for the real part, Ur hr - Ui hi, and
// us = (Ui, Ur) for the imaginary part, Ui hr + Ur hi (builtins, so that the compiler sees
// the DOT instructions and inserts the wait states their results need).
__device__ __forceinline__ float row_dot(f16x2 u0, f16x2 u1, f16x2 u2, f16x2 h0, f16x2 h1, f16x2 h2) {
  float r = __builtin_amdgcn_fdot2(u0, h0, 0.0f, false);
  r = __builtin_amdgcn_fdot2(u1, h1, r, false);
  return __builtin_amdgcn_fdot2(u2, h2, r, false);
}

template <int MU, int SG>
__device__ __forceinline__ void project_f16(const f16x2 p[12], f16x2 h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const f16x2 p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if constexpr (MU == 0) {
      h[c] = SG > 0 ? p0 - i_f16x2(p3) : p0 + i_f16x2(p3);
      h[3 + c] = SG > 0 ? p1 - i_f16x2(p2) : p1 + i_f16x2(p2);
    } else if constexpr (MU == 1) {
      h[c] = SG > 0 ? p0 - p3 : p0 + p3;
      h[3 + c] = SG > 0 ? p1 + p2 : p1 - p2;
    } else if constexpr (MU == 2) {
      h[c] = SG > 0 ? p0 - i_f16x2(p2) : p0 + i_f16x2(p2);
      h[3 + c] = SG > 0 ? p1 + i_f16x2(p3) : p1 - i_f16x2(p3);
    } else {
      h[c] = SG > 0 ? p0 + p2 : p0 - p2;
      h[3 + c] = SG > 0 ? p1 + p3 : p1 - p3;
    }
  }
}

// acc += n * reconstruction of u = (re, im): reconstruct_acc with the neighbour norm folded
// into fused multiply-adds
template <int MU, int SG>
__device__ __forceinline__ void reconstruct_fma(const float re[6], const float im[6], float n, cx<float> acc[12]) {
  const float sn = SG * n;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float r0 = re[c], i0 = im[c], r1 = re[3 + c], i1 = im[3 + c];
    acc[c] = {fmaf(n, r0, acc[c].re), fmaf(n, i0, acc[c].im)};
    acc[3 + c] = {fmaf(n, r1, acc[3 + c].re), fmaf(n, i1, acc[3 + c].im)};
    if constexpr (MU == 0) {  // + sg i u1, + sg i u0
      acc[6 + c] = {fmaf(-sn, i1, acc[6 + c].re), fmaf(sn, r1, acc[6 + c].im)};
      acc[9 + c] = {fmaf(-sn, i0, acc[9 + c].re), fmaf(sn, r0, acc[9 + c].im)};
    } else if constexpr (MU == 1) {  // + sg u1, - sg u0
      acc[6 + c] = {fmaf(sn, r1, acc[6 + c].re), fmaf(sn, i1, acc[6 + c].im)};
      acc[9 + c] = {fmaf(-sn, r0, acc[9 + c].re), fmaf(-sn, i0, acc[9 + c].im)};
    } else if constexpr (MU == 2) {  // + sg i u0, - sg i u1
      acc[6 + c] = {fmaf(-sn, i0, acc[6 + c].re), fmaf(sn, r0, acc[6 + c].im)};
      acc[9 + c] = {fmaf(sn, i1, acc[9 + c].re), fmaf(-sn, r1, acc[9 + c].im)};
    } else {  // + sg u0, + sg u1
      acc[6 + c] = {fmaf(sn, r0, acc[6 + c].re), fmaf(sn, i0, acc[6 + c].im)};
      acc[9 + c] = {fmaf(sn, r1, acc[9 + c].re), fmaf(sn, i1, acc[9 + c].im)};
    }
  }
}

// the link elements of one direction as (Uc, Us) = ((Ur, -Ui), (Ui, Ur)): staged in LDS in
// pairs (stride 20 per direction) or formed from the packed field (stride 9)
template <bool PAIRED>
__device__ __forceinline__ void links_f16(const __half2* L, int D, f16x2 Uc[9], f16x2 Us[9]) {
  if constexpr (PAIRED) {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      Uc[e] = as_f16x2(L[D * 20 + 2 * e]);
      Us[e] = as_f16x2(L[D * 20 + 2 * e + 1]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      const f16x2 u = as_f16x2(L[D * 9 + e]);
      Uc[e] = u * f16x2{(_Float16)1, (_Float16)-1};
      Us[e] = u.yx;
    }
  }
}

// Moebius input factor F = b + c S~ on one FP16 neighbour spinor, in packed FP16: the three
// terms (psi_s, the upper spins of psi_{s-1}, the lower spins of psi_{s+1}, each with its own
// norm) are weighted relative to the largest weight, so every packed value stays within the
// FP16 range (|value| <= 2); the largest weight is returned as the norm of the result.
__device__ __forceinline__ float load_input_f16_pro(const HopArgs<P16>& a, long y, int s, const ProCoef<float>& pc,
                                                  f16x2 psi[12]) {
  const int Ls = a.Ls, su = pc.su, sl = pc.sl;
  const __half2* p = a.in.data + size_t(y) * 12 * Ls;
  const float* nb = a.in.norm + size_t(y) * Ls;
  const float ws = pc.b * nb[s], wu = pc.u * nb[su], wl = pc.l * nb[sl];
  const float m = fmaxf(fabsf(ws), fmaxf(fabsf(wu), fabsf(wl)));
  const float inv = m > 1e-37f ? __builtin_amdgcn_rcpf(m) : 0.0f;  // (ratios only need FP16 accuracy)
  const _Float16 hs = (_Float16)(ws * inv), hu = (_Float16)(wu * inv), hl = (_Float16)(wl * inv);
  const f16x2 cs = {hs, hs}, cu = {hu, hu}, cl = {hl, hl};
#pragma unroll
  for (int k = 0; k < 6; ++k) psi[k] = cs * as_f16x2(p[k * Ls + s]) + cu * as_f16x2(p[k * Ls + su]);
#pragma unroll
  for (int k = 6; k < 12; ++k) psi[k] = cs * as_f16x2(p[k * Ls + s]) + cl * as_f16x2(p[k * Ls + sl]);
  return m;
}

// The FP16 direction step in two stages: the neighbour's spinors (with the prologue, if any)
// and norms are loaded first, the projection, SU(3) product and reconstruction follow.  The
// kernel issues the loads of the next direction before the arithmetic of the current one, so
// that two directions' gathers are always in flight (left to itself the compiler kept fewer
// loads outstanding in some variants: dagger hops waited at vmcnt 3 on average, the others at 8).
template <int NS>
struct F16In {
  f16x2 psi[NS][12];
  float n[NS];
};

template <int NS, bool PRO>
__device__ __forceinline__ void load_dir_f16(const HopArgs<P16>& a, long y, int s0, int tps,
                                             const ProCoef<float> (&pro)[NS], F16In<NS>& in) {
  const int Ls = a.Ls;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int s = s0 + j * tps;
    if constexpr (PRO) {
      in.n[j] = load_input_f16_pro(a, y, s, pro[j], in.psi[j]);
    } else {
      const __half2* p = a.in.data + size_t(y) * 12 * Ls + s;
#pragma unroll
      for (int k = 0; k < 12; ++k) in.psi[j][k] = as_f16x2(p[k * Ls]);
      in.n[j] = a.in.norm[size_t(y) * Ls + s];
    }
  }
}

template <int MU, int SG, int NS, bool PAIRED>
__device__ __forceinline__ void apply_dir_f16(const HopArgs<P16>& a, const __half2* L, int D, const F16In<NS>& in,
                                              cx<float> (&acc)[NS][12]) {
  f16x2 Uc[9], Us[9];
  links_f16<PAIRED>(L, D, Uc, Us);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    f16x2 h[6];
    const float n = in.n[j] * a.scale;  // the hop's overall scale folded in
    project_f16<MU, SG>(in.psi[j], h);
    float re[6], im[6];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int row = 0; row < 3; ++row) {
        re[r * 3 + row] = row_dot(Uc[row * 3], Uc[row * 3 + 1], Uc[row * 3 + 2], h[r * 3], h[r * 3 + 1], h[r * 3 + 2]);
        im[r * 3 + row] = row_dot(Us[row * 3], Us[row * 3 + 1], Us[row * 3 + 2], h[r * 3], h[r * 3 + 1], h[r * 3 + 2]);
      }
    reconstruct_fma<MU, SG>(re, im, n, acc[j]);
  }
}

template <int MU, int SG, int NS, bool PRO, bool PAIRED>
__device__ __forceinline__ void hop_dir_f16(const HopArgs<P16>& a, long y, const __half2* L, int D, int s0, int tps,
                                            const ProCoef<float> (&pro)[NS], cx<float> (&acc)[NS][12]) {
  F16In<NS> in;
  load_dir_f16<NS, PRO>(a, y, s0, tps, pro, in);
  apply_dir_f16<MU, SG, NS, PAIRED>(a, L, D, in, acc);
}

// the eight FP16 directions with the loads of direction D + 1 issued before the arithmetic of D
template <int D, bool DAG, bool PRO, int NS, bool PAIRED>
__device__ __forceinline__ void hop_dirs_f16(const HopArgs<P16>& a, const int* nb, const __half2* L, int s0, int tps,
                                             const ProCoef<float> (&pro)[NS], F16In<NS>& cur, F16In<NS>& nxt,
                                             cx<float> (&acc)[NS][12]) {
  constexpr int MU = D & 3;
  constexpr bool FWD = D < 4;
  constexpr int SG = (FWD != DAG) ? -1 : +1;
  if constexpr (D + 1 < 8) load_dir_f16<NS, PRO>(a, nb[D + 1], s0, tps, pro, nxt);
  apply_dir_f16<MU, SG, NS, PAIRED>(a, L, D, cur, acc);
  if constexpr (D + 1 < 8) hop_dirs_f16<D + 1, DAG, PRO, NS, PAIRED>(a, nb, L, s0, tps, pro, nxt, cur, acc);
}

// ------------------------------------------------------------------ LDS-staged neighbour spinors
// FP16 with a compile-time Ls and one slice per lane: for each direction the workgroup copies
// the spinors of its sites' neighbours (one contiguous [12][Ls] block of half2 and Ls norms per
// site) into LDS with global_load_lds_dwordx4 (16 bytes per lane, no registers held while the
// copy is in flight), and the lanes then read their operands from LDS.  The per-lane gathers of
// the plain hop are bound by their latency; the bulk copies keep many more bytes in flight.
template <int LS>
struct Stage {
  static constexpr int SPINOR_CHUNKS = 12 * LS * 4 / 16;      // 16-byte chunks of one site's spinor
  static constexpr int CHUNKS = SPINOR_CHUNKS + LS * 4 / 16;  // ... and its norms
  static constexpr int SITE_BYTES = CHUNKS * 16;
  static constexpr int SPB = 256 / LS;
  static constexpr int WG_CHUNKS = SPB * CHUNKS;
  static constexpr int ROUNDS = (WG_CHUNKS + 255) / 256;
  static constexpr int BUF = ROUNDS * 256 * 16;               // bytes per direction buffer
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// issue the copies of the nact sites' neighbours in one direction (ys[j] = neighbour x_cb);
// chunk c lands at buf + 16 c: the lanes of one wave write consecutive 16-byte slots
template <int LS>
__device__ __forceinline__ void stage_dir(const HopArgs<P16>& a, const int* ys, int nact, unsigned char* buf) {
  using G = Stage<LS>;
  const int wave_base = threadIdx.x & ~63;
#pragma unroll
  for (int r = 0; r < G::ROUNDS; ++r) {
    const int c = r * 256 + int(threadIdx.x);
    if (c < nact * G::CHUNKS) {
      const int j = c / G::CHUNKS;
      const int part = c - j * G::CHUNKS;
      const size_t y = size_t(ys[j]);
      const char* src = part < G::SPINOR_CHUNKS
                            ? reinterpret_cast<const char*>(a.in.data + y * 12 * LS) + part * 16
                            : reinterpret_cast<const char*>(a.in.norm + y * LS) + (part - G::SPINOR_CHUNKS) * 16;
      __builtin_amdgcn_global_load_lds(src, (lds_void_ptr)(buf + (r * 256 + wave_base) * 16), 16, 0, 0);
    }
  }
}

// one direction of the FP16 hop with the neighbour's spinor read from its staged copy sb
template <int MU, int SG, int LS>
__device__ __forceinline__ void hop_dir_f16_staged(const unsigned char* sb, int s, float scale, const __half2* L,
                                                   int D, cx<float> (&acc)[1][12]) {
  f16x2 Uc[9], Us[9];
  links_f16<true>(L, D, Uc, Us);  // the workgroup's links, staged in LDS
  const __half2* p = reinterpret_cast<const __half2*>(sb) + s;
  f16x2 psi[12], h[6];
#pragma unroll
  for (int k = 0; k < 12; ++k) psi[k] = as_f16x2(p[k * LS]);
  const float n = reinterpret_cast<const float*>(sb + 48 * LS)[s] * scale;
  project_f16<MU, SG>(psi, h);
  float re[6], im[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int row = 0; row < 3; ++row) {
      re[r * 3 + row] = row_dot(Uc[row * 3], Uc[row * 3 + 1], Uc[row * 3 + 2], h[r * 3], h[r * 3 + 1], h[r * 3 + 2]);
      im[r * 3 + row] = row_dot(Us[row * 3], Us[row * 3 + 1], Us[row * 3 + 2], h[r * 3], h[r * 3 + 1], h[r * 3 + 2]);
    }
  reconstruct_fma<MU, SG>(re, im, n, acc[0]);
}

// direction D: copy the neighbours' spinors into the buffer, wait for every wave's copies,
// compute, and release the buffer.  One buffer per workgroup (about 22 KB of LDS with the
// staged links): several workgroups per CU are at different phases, so that copies of some
// overlap the arithmetic of others.
template <int D, bool DAG, int LS>
__device__ __forceinline__ void staged_step(const HopArgs<P16>& a, const int* ys, int spb, int nact, bool active,
                                            int lsite, int s, const __half2* L, unsigned char* buf,
                                            cx<float> (&acc)[1][12]) {
  constexpr int MU = D & 3;
  constexpr bool FWD = D < 4;
  constexpr int SG = (FWD != DAG) ? -1 : +1;
  using G = Stage<LS>;
  stage_dir<LS>(a, ys + D * spb, nact, buf);
  __syncthreads();  // (waits for this wave's copies, then for every wave)
  if (active) hop_dir_f16_staged<MU, SG, LS>(buf + lsite * G::SITE_BYTES, s, a.scale, L, D, acc);
  __syncthreads();  // the buffer is free for the next direction
}

// One of the 8 hop directions: D = 0..3 forward (x+mu), 4..7 backward (x-mu).
// H uses (1 - g_mu) forward and (1 + g_mu) backward; H^dag the opposite.
// PAIRED: FP16 links staged as (U, Us) pairs, 20 elements per direction.
template <int D, bool DAG, bool PRO, int NS, bool PAIRED, typename P>
__device__ __forceinline__ void hop_dir(const HopArgs<P>& a, const int* nb, const typename P::S* L, int s0, int tps,
                                        const ProCoef<typename P::R> (&pro)[NS], cx<typename P::R> (&acc)[NS][12]) {
  using R = typename P::R;
  constexpr int MU = D & 3;
  constexpr bool FWD = D < 4;
  constexpr int SG = (FWD != DAG) ? -1 : +1;
  const long y = nb[D];
  if constexpr (std::is_same<P, P16>::value) {
    hop_dir_f16<MU, SG, NS, PRO, PAIRED>(a, y, L, D, s0, tps, pro, acc);
    return;
  }
  constexpr int LSTR = PAIRED ? 20 : 9, LEL = PAIRED ? 2 : 1;
  cx<R> U[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) U[e] = P::ld(L[D * LSTR + e * LEL]);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    cx<R> psi[12], h[6], u[6];
    load_input<P, PRO>(a, y, s0 + j * tps, pro[j], psi);
    project<MU, SG>(psi, h);
    su3_mul_half(U, h, u);
    reconstruct_acc<MU, SG>(u, acc[j]);
  }
}

// FP16 with one slice per thread: at least 5 waves per SIMD (at most 102 VGPRs), since the
// kernel is bound by the latency of its gathers; 4 for the fused CG step without an epilogue
// matrix, which would spill at 5.  Several slices per thread keep the default.
template <typename P, int NS, int EPI, bool CG>
constexpr int hop_min_waves() { return std::is_same<P, P16>::value && NS == 1 ? (CG && EPI == 0 ? 4 : 5) : 1; }

// ST: neighbour spinors staged through LDS (FP16, compile-time Ls, one slice per lane, no
// prologue, spb = 256 / Ls); its links are staged too (LL), so that the direction loop issues
// no other vector-memory loads than the copies
// The body of the hop on workgroup bid of the field a (pidx: the slot of its norm partial).
// RS > 0: the field holds Ls / RS right-hand sides of fifth-dimension extent RS interleaved along
// s (slice s of right-hand side r is slice r RS + s), each with its own epilogue coefficients,
// CG scalars and norm partials (see HopArgs).
// The fifth-dimension hop of the Shamir operator on 5D-checkerboarded fields, added to acc:
//   r5 (P- psi_{s+1} + P+ psi_{s-1})   (dagger: r5 (P- psi_{s-1} + P+ psi_{s+1})),
// psi_{Ls} = -m psi_0, psi_{-1} = -m psi_{Ls-1}, psi = a.loc at this 4D site.  The lane's output
// slice is s = 2 j + sigma and loc's slot j' holds s' = 2 j' + 1 - sigma, so one chirality comes
// from the lane's own slot and the other from the next lane of the site's segment (j - 1 for
// sigma = 0, j + 1 for sigma = 1, wrapping round the segment with the factor -m).  All lanes of
// the wave take part in the shuffle; a site's lanes are active or inactive together.
template <typename P, bool DAG>
__device__ __forceinline__ void eo5_fifth_hop(const HopArgs<P>& a, typename P::R r5, long x, int j, int LH,
                                              bool active, cx<typename P::R> acc[12]) {
  using R = typename P::R;
  cx<R> v[12];
  if (active) {
    load_spinor<P>(a.loc, x, j, LH, v);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {R(0), R(0)};
  }
  const int sigma = a.sigma;
  // the neighbouring lane supplies P- (spins 2, 3) or P+ (spins 0, 1)
  const bool nbr_minus = (sigma != 0) != DAG;
  const bool wrap = sigma ? (j == LH - 1) : (j == 0);
  const int jn = sigma ? (wrap ? 0 : j + 1) : (wrap ? LH - 1 : j - 1);
  const int src = int(threadIdx.x & 63) - j + jn;
  const R fn = wrap ? -a.pm * r5 : r5;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const cx<R> t = nbr_minus ? v[6 + k] : v[k];
    cx<R> w;
    w.re = __shfl(t.re, src, 64);
    w.im = __shfl(t.im, src, 64);
    if (nbr_minus) {
      acc[6 + k] = acc[6 + k] + fn * w;
      acc[k] = acc[k] + r5 * v[k];
    } else {
      acc[k] = acc[k] + fn * w;
      acc[6 + k] = acc[6 + k] + r5 * v[6 + k];
    }
  }
}

// FP16: the same with the operand kept packed until it is used; the neighbouring lane's six
// components and its norm travel as 32-bit words (one shuffle per complex number)
template <bool DAG>
__device__ __forceinline__ void eo5_fifth_hop_f16(const HopArgs<P16>& a, float r5, long x, int j, int LH, bool active,
                                                  cx<float> acc[12]) {
  int w[12];
  float n = 0.0f;
  if (active) {
    const int* p = reinterpret_cast<const int*>(a.loc.data) + size_t(x) * 12 * LH + j;
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = p[k * LH];
    n = a.loc.norm[size_t(x) * LH + j];
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) w[k] = 0;
  }
  const int sigma = a.sigma;
  const bool nbr_minus = (sigma != 0) != DAG;
  const bool wrap = sigma ? (j == LH - 1) : (j == 0);
  const int jn = sigma ? (wrap ? 0 : j + 1) : (wrap ? LH - 1 : j - 1);
  const int src = int(threadIdx.x & 63) - j + jn;
  const float cn = (wrap ? -a.pm * r5 : r5) * __shfl(n, src, 64);  // the neighbour's norm
  const float co = r5 * n;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const f16x2 hn = __builtin_bit_cast(f16x2, __shfl(nbr_minus ? w[6 + k] : w[k], src, 64));
    const f16x2 ho = __builtin_bit_cast(f16x2, nbr_minus ? w[k] : w[6 + k]);
    const cx<float> vn = {cn * float(hn.x), cn * float(hn.y)}, vo = {co * float(ho.x), co * float(ho.y)};
    if (nbr_minus) {
      acc[6 + k] = acc[6 + k] + vn;
      acc[k] = acc[k] + vo;
    } else {
      acc[k] = acc[k] + vn;
      acc[6 + k] = acc[6 + k] + vo;
    }
  }
}

template <typename P, int LS, int NS, bool DAG, bool PRO, int EPI, bool LL, bool CG, bool ST, int RS = 0,
          bool EO5 = false>
__device__ __forceinline__ void hop_body(const HopArgs<P>& a, long bid, long pidx, int spb) {
  using R = typename P::R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  // LS > 0: the fifth-dimension extent is a compile-time constant (immediate load offsets)
  const int Ls = LS > 0 ? LS : a.Ls, tps = Ls / NS;
  HopArgs<P> ak = a;
  ak.Ls = Ls;
  // interleaved right-hand sides: their epilogue coefficients staged in LDS (read per lane there,
  // instead of per-lane vector loads beside the gathers)
  constexpr int NSEG = RS > 0 ? 256 / RS : 1;
  __shared__ FifthScan<R> es_lds[(RS > 0 && EPI >= 2) ? (EPI == 3 ? 2 : 1) : 1][NSEG];
  if constexpr (RS > 0 && EPI >= 2) {
    const int K = Ls / RS;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
      es_lds[0][i] = a.es_tab[i];
      if constexpr (EPI == 3) es_lds[1][i] = a.es2_tab[i];
    }
    __syncthreads();
  } else if constexpr (RS > 0 && CG) {
    // (the fused CG step's operator on the axpy operand, per right-hand side: see x_es2)
    if (a.x_es2) {
      const int K = Ls / RS;
      for (int i = threadIdx.x; i < K; i += blockDim.x) es_lds[0][i] = a.es2_tab[i];
      __syncthreads();
    }
  }
  const int lsite = threadIdx.x / tps;
  const int s0 = threadIdx.x - lsite * tps;
  const long slot = bid * spb + lsite;
  const bool active = (lsite < spb) && (slot < a.nsites);
  const long x = active ? (a.order ? long(a.order[slot]) : slot) : 0;
  cx<R> acc[NS][12];
#pragma unroll
  for (int j = 0; j < NS; ++j)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[j][k] = {R(0), R(0)};
  using S = typename P::S;
  constexpr bool PAIRED = LL && std::is_same<P, P16>::value;
  const S* L;
  if constexpr (LL) {
    // Stage the 8 links of each of the workgroup's sites in LDS with coalesced loads
    // (one read per element instead of one per s-slice lane); lanes then read them
    // through the LDS pipe, which leaves the texture-data path to the spinors.
    constexpr int NE = staged_link_elems<P>();
    S* llds = reinterpret_cast<S*>(smem_raw + (EPI == 1 ? size_t(spb) * 12 * Ls * sizeof(cx<R>) : 0));
    const long base = bid * spb;
    for (int i = threadIdx.x; i < spb * 72; i += blockDim.x) {
      const int ls = i / 72;
      const long sl = base + ls;
      if (sl < a.nsites) {
        const long xs = a.order ? long(a.order[sl]) : sl;
        const int j = i - ls * 72;
        const S u = a.links[xs * 72 + j];
        if constexpr (PAIRED) {
          const int d = j / 9, e = j - d * 9;
          const f16x2 v = as_f16x2(u);
          llds[ls * NE + d * 20 + 2 * e] = from_f16x2(v * f16x2{(_Float16)1, (_Float16)-1});
          llds[ls * NE + d * 20 + 2 * e + 1] = from_f16x2(v.yx);
        } else {
          llds[i] = u;
        }
      }
    }
    __syncthreads();
    L = llds + lsite * NE;
  } else {
    L = a.links + x * 72;
  }
  if constexpr (ST) {
    static_assert(std::is_same<P, P16>::value && NS == 1 && !PRO && LL && LS > 0 && EPI != 1, "staged hop");
    __shared__ int ys[8 * 32];  // [direction][site]: neighbour x_cb of the workgroup's sites
    const long base = bid * spb;
    const int nact = int(a.nsites - base < spb ? a.nsites - base : spb);
    for (int i = threadIdx.x; i < 8 * spb; i += blockDim.x) {
      const int j = i / 8, d = i - j * 8;
      if (j < nact) {
        const long xs = a.order ? long(a.order[base + j]) : base + j;
        ys[d * spb + j] = a.nbr[xs * 8 + d];
      }
    }
    __shared__ __align__(16) unsigned char sbuf[Stage<LS>::BUF];
    __syncthreads();
    staged_step<0, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<1, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<2, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<3, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<4, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<5, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<6, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
    staged_step<7, DAG, LS>(ak, ys, spb, nact, active, lsite, s0, L, sbuf, acc);
  } else if (active) {
    const int* nb = a.nbr + x * 8;
    ProCoef<R> pro[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) pro[j] = pro_coef<P, PRO>(ak, s0 + j * tps);
    if constexpr (std::is_same<P, P16>::value) {
      F16In<NS> b0, b1;
      load_dir_f16<NS, PRO>(ak, nb[0], s0, tps, pro, b0);
      hop_dirs_f16<0, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, b0, b1, acc);
    } else {
      // (FP64 / FP32: the same pipelining was measured slower for the prologue and epilogue
      // variants, which already run at low occupancy)
      hop_dir<0, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<1, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<2, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<3, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<4, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<5, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<6, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
      hop_dir<7, DAG, PRO, NS, PAIRED>(ak, nb, L, s0, tps, pro, acc);
    }
  }
  if constexpr (!std::is_same<P, P16>::value) {  // (the FP16 path folds the scale into the norm)
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int k = 0; k < 12; ++k) acc[j][k] = a.scale * acc[j][k];
  }
  if constexpr (EO5) {
    // (placed after the gathers: before them it raises the register count further)
    static_assert(NS == 1 && !PRO && EPI == 0 && RS == 0 && !ST, "5D even-odd hop: one slice per lane, no matrices");
    if constexpr (std::is_same<P, P16>::value) eo5_fifth_hop_f16<DAG>(a, a.r5, x, s0, Ls, active, acc[0]);
    else eo5_fifth_hop<P, DAG>(a, a.r5, x, s0, Ls, active, acc[0]);
  }
  // the lane's right-hand side and slice within it (interleaved fields)
  const int rhs = RS > 0 ? s0 / (RS > 0 ? RS : 1) : 0;
  const int sr = RS > 0 ? s0 - rhs * RS : s0;
  if constexpr (EPI >= 2) {
    // recurrence form along s: the site's Ls lanes (a right-hand side's RS lanes) are one
    // segment of the wave
    constexpr int SEG = RS > 0 ? RS : LS;
    static_assert(NS == 1 && SEG > 0 && (64 % SEG) == 0, "scan epilogue needs one slice per lane");
    if constexpr (RS > 0) fifth_scan_apply<SEG>(acc[0], sr, es_lds[0][rhs]);
    else fifth_scan_apply<SEG>(acc[0], s0, a.es);
  }
  if constexpr (EPI == 1) {
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    if (active) {
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int k = 0; k < 12; ++k) lds[(lsite * 12 + k) * Ls + s0 + j * tps] = acc[j][k];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int s = s0 + j * tps;
        const R* E0 = a.E + s * Ls;
        const R* E1 = a.E + Ls * Ls + s * Ls;
        cx<R> o[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
        const cx<R>* row = lds + lsite * 12 * Ls;
        for (int sp = 0; sp < Ls; ++sp) {
          const R e0 = E0[sp], e1 = E1[sp];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const cx<R> v = row[k * Ls + sp];
            o[k].re = fma(e0, v.re, o[k].re);
            o[k].im = fma(e0, v.im, o[k].im);
          }
#pragma unroll
          for (int k = 6; k < 12; ++k) {
            const cx<R> v = row[k * Ls + sp];
            o[k].re = fma(e1, v.re, o[k].re);
            o[k].im = fma(e1, v.im, o[k].im);
          }
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[j][k] = o[k];
      }
    }
  }
  // the axpy operand given through a site-local operator (x_es2): es2 applied along the site's
  // segment right after the read (every lane of a site is active or inactive together, so the
  // segment's shuffles read active lanes only)
  constexpr bool XS = CG && NS == 1 && RS == 0 && !ST && !std::is_same<P, P64>::value && (LS == 8 || LS == 16 || LS == 32);
  constexpr bool XSI = CG && RS > 0 && EPI < 2 && !std::is_same<P, P64>::value;  // per right-hand side
  double nrm = 0.0;
  if (active) {
    const R alpha = CG ? R(a.cg_scalars[rhs * S_COUNT + S_ALPHA]) : R(0);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int s = s0 + j * tps;
      if (a.x.data) {
        cx<R> xv[12];
        load_spinor<P>(a.x, x, s, Ls, xv);
        if constexpr (XS) {
          if (a.x_es2) fifth_scan_apply<(LS > 0 ? LS : 1)>(xv, s, a.es2);
        } else if constexpr (XSI) {
          if (a.x_es2) fifth_scan_apply<(RS > 0 ? RS : 1)>(xv, sr, es_lds[0][rhs]);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[j][k] = acc[j][k] + a.ax * xv[k];
      }
      if constexpr (CG) {
        // r -= alpha v: the CG residual update on the site this thread holds
        cx<R> rv[12];
        load_spinor<P>(CHalf<P>{a.cg_r.data, a.cg_r.norm}, x, s, Ls, rv);
#pragma unroll
        for (int k = 0; k < 12; ++k) rv[k] = {rv[k].re - alpha * acc[j][k].re, rv[k].im - alpha * acc[j][k].im};
        store_spinor<P>(a.cg_r, x, s, Ls, rv);
        if (a.norm_partials) {
#pragma unroll
          for (int k = 0; k < 12; ++k)
            nrm += double(rv[k].re) * double(rv[k].re) + double(rv[k].im) * double(rv[k].im);
        }
      } else {
        if (a.norm_partials) {
#pragma unroll
          for (int k = 0; k < 12; ++k)
            nrm += double(acc[j][k].re) * double(acc[j][k].re) + double(acc[j][k].im) * double(acc[j][k].im);
        }
        // (no out with a second output: only the norm and out2 are wanted)
        if (a.out.data) store_spinor<P>(a.out, x, s, Ls, acc[j]);
      }
    }
  }
  if constexpr (EPI == 3 && !CG) {
    // second output: the site-local operator es2 on the final result (all lanes of a site
    // are active or inactive together, so the segment shuffles stay within active lanes)
    constexpr int SEG = RS > 0 ? RS : LS;
    if constexpr (RS > 0) fifth_scan_apply<SEG>(acc[0], sr, es_lds[EPI == 3 ? 1 : 0][rhs]);
    else fifth_scan_apply<SEG>(acc[0], s0, a.es2);
    if (active) store_spinor<P>(a.out2, x, s0, Ls, acc[0]);
  }
  if (a.norm_partials) {
    if constexpr (RS > 0) {
      // per right-hand side: the sum over its segment (butterfly within the RS lanes), then over
      // the workgroup's sites; partial of right-hand side r at norm_partials[r part_stride + pidx]
      static_assert(NS == 1 && (64 % (RS > 0 ? RS : 1)) == 0, "interleaved right-hand sides: one slice per lane");
      __shared__ double redr[256 / (RS > 0 ? RS : 1)];
      double v = nrm;
#pragma unroll
      for (int off = 1; off < RS; off <<= 1) v += __shfl_xor(v, off, 64);
      if (sr == 0) redr[threadIdx.x / RS] = v;
      __syncthreads();
      const int K = Ls / RS;
      if (int(threadIdx.x) < K) {
        double t = 0.0;
        for (int j = 0; j < spb; ++j) t += redr[j * K + threadIdx.x];
        a.norm_partials[threadIdx.x * a.part_stride + pidx] = t;
      }
    } else {
      const double t = block_sum(nrm, red);
      if (threadIdx.x == 0) a.norm_partials[pidx] = t;
    }
  }
}

template <typename P, int LS, int NS, bool DAG, bool PRO, int EPI, bool LL, bool CG, bool ST>
__global__ void __launch_bounds__(256, (hop_min_waves<P, NS, EPI, CG>())) hop_kernel(HopArgs<P> a, int spb, int xcd) {
  const long bid = xcd ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x;
  hop_body<P, LS, NS, DAG, PRO, EPI, LL, CG, ST>(a, bid, blockIdx.x, spb);
}

// Several fields (right-hand sides) of one lattice in one launch: workgroup b takes field
// b % nrhs and site block b / nrhs, so that the nrhs workgroups of one site block are dispatched
// together (and, with the XCD-aware order, on one XCD): the links of those sites are read once
// from memory and then hit in that XCD's L2 for the other fields.  args: device table of the
// fields' arguments (the same kernel variant for all of them); each field's norm partials are
// indexed by its site block.
template <typename P, int LS, int NS, bool DAG, bool PRO, int EPI, bool LL, bool CG, bool ST>
__global__ void __launch_bounds__(256, (hop_min_waves<P, NS, EPI, CG>()))
    hop_batch_kernel(const HopArgs<P>* __restrict__ args, int nrhs, int spb, int xcd) {
  const long b = xcd ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x;
  const long bid = b / nrhs;
  hop_body<P, LS, NS, DAG, PRO, EPI, LL, CG, ST>(args[b - bid * nrhs], bid, bid, spb);
}

// Right-hand sides interleaved along the fifth dimension (segments of RS slices, a.Ls = their
// number times RS; no Moebius prologue): one slice per lane, the site's a.Ls lanes contiguous.
template <typename P, bool DAG, int EPI, bool LL, bool CG, int RS>
__global__ void __launch_bounds__(256, (hop_min_waves<P, 1, EPI, CG>())) hop_ilv_kernel(HopArgs<P> a, int spb, int xcd) {
  const long bid = xcd ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x;
  hop_body<P, 0, 1, DAG, false, EPI, LL, CG, false, RS>(a, bid, blockIdx.x, spb);
}

template <typename P, bool DAG, int EPI, bool CG, int RS>
static int launch_ilv_t(const HopArgs<P>& a, const LaunchCfg& cfg, hipStream_t st) {
  const int threads = cfg.spb * a.Ls;
  const long blocks = (a.nsites + cfg.spb - 1) / cfg.spb;
  const size_t lds = hop_lds_bytes<P>(cfg, a.Ls, false);
  if (cfg.ll)
    hipLaunchKernelGGL((hop_ilv_kernel<P, DAG, EPI, true, CG, RS>), dim3((unsigned)blocks), dim3(threads), lds, st, a,
                       cfg.spb, cfg.xcd);
  else
    hipLaunchKernelGGL((hop_ilv_kernel<P, DAG, EPI, false, CG, RS>), dim3((unsigned)blocks), dim3(threads), lds, st, a,
                       cfg.spb, cfg.xcd);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P, int RS>
static int launch_ilv_rs(const HopArgs<P>& a, bool dag, const LaunchCfg& cfg, hipStream_t st) {
  const bool epi = a.epi_scan != 0;
  if (dag) {
    if (a.cg_r.data) return epi ? -1 : launch_ilv_t<P, true, 0, true, RS>(a, cfg, st);
    return epi ? launch_ilv_t<P, true, 2, false, RS>(a, cfg, st) : launch_ilv_t<P, true, 0, false, RS>(a, cfg, st);
  }
  if (!epi) return a.out2.data ? -1 : launch_ilv_t<P, false, 0, false, RS>(a, cfg, st);
  return a.out2.data ? launch_ilv_t<P, false, 3, false, RS>(a, cfg, st) : launch_ilv_t<P, false, 2, false, RS>(a, cfg, st);
}

// The hop on a field of right-hand sides interleaved along s in segments of rs slices (8, 16
// or 32): a.Ls = nrhs rs, the epilogue (a.epi_scan) from a.es_tab / a.es2_tab (one entry per
// right-hand side), the fused CG step's alpha of right-hand side r at a.cg_scalars[r S_COUNT +
// S_ALPHA], norm partials at a.norm_partials[r a.part_stride + block].  Validates the shape:
// one slice per thread, a.Ls * sites per workgroup <= 256, no dense epilogue, no prologue.
template <typename P>
int launch_hop_ilv(const HopArgs<P>& a, bool dagger, int rs, const LaunchCfg& cfg, hipStream_t st) {
  if (rs != 8 && rs != 16 && rs != 32) return -1;
  if (a.Ls < rs || a.Ls % rs != 0 || cfg.ns != 1 || cfg.spb < 1 || cfg.spb * a.Ls > 256) return -1;
  if (a.E || (a.epi_scan && !a.es_tab) || (a.out2.data && (!a.epi_scan || !a.es2_tab || dagger))) return -1;
  if (a.cg_r.data && (!dagger || !a.cg_scalars)) return -1;
  if (!a.cg_r.data && !a.out.data && !a.out2.data) return -1;
  // the operator on the fused CG step's axpy operand: per right-hand side from es2_tab
  if (a.x_es2 && (!a.cg_r.data || !a.x.data || !a.es2_tab || a.epi_scan || std::is_same<P, P64>::value)) return -1;
  if (a.norm_partials && a.part_stride < (a.nsites + cfg.spb - 1) / cfg.spb) return -1;
  if (hop_lds_bytes<P>(cfg, a.Ls, false) > 65536) return -1;
  if (a.nsites <= 0) return 0;
  switch (rs) {
    case 8: return launch_ilv_rs<P, 8>(a, dagger, cfg, st);
    case 16: return launch_ilv_rs<P, 16>(a, dagger, cfg, st);
    default: return launch_ilv_rs<P, 32>(a, dagger, cfg, st);
  }
}

// 5D even-odd hop: workgroup pairs (2t, 2t + 1) take block t of output halves 0 and 1, the two
// 4D parities of one traversal tile, dispatched together (and with the XCD-aware order on one
// XCD), so that each input half read as neighbours by one is read as loc by the other while it
// is in that XCD's L2.
// (occupancy floor of 4 waves per SIMD only for FP32 with links in LDS: the other bodies spill
// there with the fifth-dimension hop's operand)
template <typename P, int LS, bool DAG, bool LL, bool CG>
__global__ void __launch_bounds__(256, ((std::is_same<P, P32>::value && LL) ? 4 : 1))
    hop_eo5_kernel(HopArgs<P> a0, HopArgs<P> a1, int spb, int xcd) {
  const long b = xcd ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x;
  // (one body per half: the arguments stay in the kernel-argument segment, no private copy)
  if (b & 1) hop_body<P, LS, 1, DAG, false, 0, LL, CG, false, 0, true>(a1, b >> 1, blockIdx.x, spb);
  else hop_body<P, LS, 1, DAG, false, 0, LL, CG, false, 0, true>(a0, b >> 1, blockIdx.x, spb);
}

template <typename P, int LS, bool DAG, bool CG>
static int launch_eo5_t(const HopArgs<P>& a0, const HopArgs<P>& a1, const LaunchCfg& cfg, hipStream_t st) {
  const int threads = cfg.spb * a0.Ls;
  const long blocks = 2 * ((a0.nsites + cfg.spb - 1) / cfg.spb);
  const size_t lds = hop_lds_bytes<P>(cfg, a0.Ls, false);
  if (cfg.ll)
    hipLaunchKernelGGL((hop_eo5_kernel<P, LS, DAG, true, CG>), dim3((unsigned)blocks), dim3(threads), lds, st, a0, a1,
                       cfg.spb, cfg.xcd);
  else
    hipLaunchKernelGGL((hop_eo5_kernel<P, LS, DAG, false, CG>), dim3((unsigned)blocks), dim3(threads), lds, st, a0,
                       a1, cfg.spb, cfg.xcd);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename P, int LS>
int launch_hop_eo5_ls(const HopArgs<P>& a0, const HopArgs<P>& a1, bool dag, const LaunchCfg& cfg, hipStream_t st) {
  if (dag) {
    if (a0.cg_r.data) return launch_eo5_t<P, LS, true, true>(a0, a1, cfg, st);
    return launch_eo5_t<P, LS, true, false>(a0, a1, cfg, st);
  }
  return launch_eo5_t<P, LS, false, false>(a0, a1, cfg, st);
}

// the staged variant applies to this instantiation and launch shape
template <typename P, int LS, int NS, bool PRO, int EPI>
constexpr bool stage_capable() {
  return std::is_same<P, P16>::value && NS == 1 && !PRO && EPI != 1 && (LS == 8 || LS == 16 || LS == 32);
}

// batch (device table of nrhs fields' arguments, a = the host copy of the first): one launch over
// all of them (one slice per thread, no LDS-staged neighbours)
template <typename P, int LS, int NS, bool DAG, bool PRO, int EPI, bool CG>
static int launch_hop_t(const HopArgs<P>& a, const LaunchCfg& cfg, hipStream_t st, const HopArgs<P>* batch,
                        int nrhs) {
  const int tps = a.Ls / NS;
  const int threads = cfg.spb * tps;
  const long blocks = (a.nsites + cfg.spb - 1) / cfg.spb;
  if (batch) {
    if constexpr (NS == 1) {
      const size_t lds = hop_lds_bytes<P>(cfg, a.Ls, EPI == 1);
      if (cfg.ll)
        hipLaunchKernelGGL((hop_batch_kernel<P, LS, NS, DAG, PRO, EPI, true, CG, false>),
                           dim3((unsigned)(blocks * nrhs)), dim3(threads), lds, st, batch, nrhs, cfg.spb, cfg.xcd);
      else
        hipLaunchKernelGGL((hop_batch_kernel<P, LS, NS, DAG, PRO, EPI, false, CG, false>),
                           dim3((unsigned)(blocks * nrhs)), dim3(threads), lds, st, batch, nrhs, cfg.spb, cfg.xcd);
      return hipGetLastError() == hipSuccess ? 0 : -2;
    } else {
      return -1;
    }
  }
  if constexpr (stage_capable<P, LS, NS, PRO, EPI>()) {
    if (stage_shape(cfg, a.Ls)) {
      LaunchCfg c2 = cfg;
      c2.ll = 1;
      hipLaunchKernelGGL((hop_kernel<P, LS, NS, DAG, PRO, EPI, true, CG, true>), dim3((unsigned)blocks),
                         dim3(threads), hop_lds_bytes<P>(c2, a.Ls, false), st, a, cfg.spb, cfg.xcd);
      return hipGetLastError() == hipSuccess ? 0 : -2;
    }
  }
  const size_t lds = hop_lds_bytes<P>(cfg, a.Ls, EPI == 1);
  if (cfg.ll)
    hipLaunchKernelGGL((hop_kernel<P, LS, NS, DAG, PRO, EPI, true, CG, false>), dim3((unsigned)blocks), dim3(threads),
                       lds, st, a, cfg.spb, cfg.xcd);
  else
    hipLaunchKernelGGL((hop_kernel<P, LS, NS, DAG, PRO, EPI, false, CG, false>), dim3((unsigned)blocks),
                       dim3(threads), lds, st, a, cfg.spb, cfg.xcd);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// epilogue: 0 none, 1 dense matrices in LDS, 2 recurrence (scan) form, 3 scan form and a
// second, scanned output (only where the site's Ls slices form one wave segment).  An epilogue
// is given by its matrices E, by its recurrence form (epi_scan) or both; the dense form needs E.
template <typename P, int LS, int NS, bool DAG, bool PRO, bool CG>
static int launch_hop_epi(const HopArgs<P>& a, const LaunchCfg& cfg, hipStream_t st, const HopArgs<P>* batch,
                          int nrhs) {
  if (!a.E && !a.epi_scan) return a.out2.data ? -1 : launch_hop_t<P, LS, NS, DAG, PRO, 0, CG>(a, cfg, st, batch, nrhs);
  if constexpr (NS == 1 && (LS == 8 || LS == 16 || LS == 32)) {
    if (a.epi_scan) {
      if constexpr (!DAG && !CG) {
        if (a.out2.data) return launch_hop_t<P, LS, NS, DAG, PRO, 3, CG>(a, cfg, st, batch, nrhs);
      }
      return a.out2.data ? -1 : launch_hop_t<P, LS, NS, DAG, PRO, 2, CG>(a, cfg, st, batch, nrhs);
    }
  }
  if (!a.E) return -1;  // the recurrence form does not apply to this launch shape
  return a.out2.data ? -1 : launch_hop_t<P, LS, NS, DAG, PRO, 1, CG>(a, cfg, st, batch, nrhs);
}

// the fused CG step exists for the dagger hop only (the last hop of M^dag M)
template <typename P, int LS, int NS>
static int launch_hop_ns(const HopArgs<P>& a, bool dag, bool pro, const LaunchCfg& cfg, hipStream_t st,
                         const HopArgs<P>* batch, int nrhs) {
  if (dag) {
    if (a.cg_r.data) return launch_hop_epi<P, LS, NS, true, false, true>(a, cfg, st, batch, nrhs);
    return launch_hop_epi<P, LS, NS, true, false, false>(a, cfg, st, batch, nrhs);
  }
  if (pro) return launch_hop_epi<P, LS, NS, false, true, false>(a, cfg, st, batch, nrhs);
  return launch_hop_epi<P, LS, NS, false, false, false>(a, cfg, st, batch, nrhs);
}

// One compile-time fifth-dimension extent (0: runtime extent).  Each (precision, LS)
// pair is instantiated in its own translation unit (see the build script).
template <typename P, int LS>
int launch_hop_ls(const HopArgs<P>& a, bool dag, bool pro, const LaunchCfg& cfg, hipStream_t st,
                  const HopArgs<P>* batch, int nrhs) {
  switch (cfg.ns) {
    case 1: return launch_hop_ns<P, LS, 1>(a, dag, pro, cfg, st, batch, nrhs);
    case 2: return launch_hop_ns<P, LS, 2>(a, dag, pro, cfg, st, batch, nrhs);
    default: return launch_hop_ns<P, LS, 4>(a, dag, pro, cfg, st, batch, nrhs);
  }
}

// Validates the launch shape against the kernel's assumptions before launching:
// Ls divisible by NS, at most 256 threads per workgroup, LDS within 64 KiB.
// batch != nullptr: one launch over nrhs fields (device table; a = the host copy of the first,
// which fixes the kernel variant: every field must have the same Ls, nsites and optional stages);
// one slice per thread only, no LDS-staged neighbours.
template <typename P>
int launch_hop(const HopArgs<P>& a, bool dagger, bool prologue, const LaunchCfg& cfg, hipStream_t st,
               const HopArgs<P>* batch, int nrhs) {
  using R = typename P::R;
  if (cfg.ns != 1 && cfg.ns != 2 && cfg.ns != 4) return -1;
  if (a.Ls % cfg.ns != 0 || cfg.spb < 1) return -1;
  if (dagger && prologue) return -1;
  if (a.cg_r.data && (!dagger || !a.cg_scalars)) return -1;
  // the operator on the axpy operand and a missing out need the scan shapes (one slice per
  // lane, the site's Ls lanes a wave segment)
  const bool seg_shape = cfg.ns == 1 && (a.Ls == 8 || a.Ls == 16 || a.Ls == 32);
  if (a.x_es2 && (!a.cg_r.data || !a.x.data || !x_es2_shape<P>(cfg, a.Ls) || batch)) return -1;
  if (!a.cg_r.data && !a.out.data && !(a.out2.data && a.E && a.epi_scan && seg_shape)) return -1;
  const int threads = cfg.spb * (a.Ls / cfg.ns);
  if (threads > 256) return -1;
  if (hop_lds_bytes<P>(cfg, a.Ls, a.E != nullptr) > 65536) return -1;
  if (a.epi_scan && !a.E && !(cfg.ns == 1 && (a.Ls == 8 || a.Ls == 16 || a.Ls == 32))) return -1;
  if (batch && (nrhs < 1 || cfg.ns != 1 || stage_shape(cfg, a.Ls))) return -1;
  if (a.nsites <= 0) return 0;
  // common extents get a compile-time Ls; the others run the generic kernel
  switch (a.Ls) {
    case 8: return launch_hop_ls<P, 8>(a, dagger, prologue, cfg, st, batch, nrhs);
    case 12: return launch_hop_ls<P, 12>(a, dagger, prologue, cfg, st, batch, nrhs);
    case 16: return launch_hop_ls<P, 16>(a, dagger, prologue, cfg, st, batch, nrhs);
    case 32: return launch_hop_ls<P, 32>(a, dagger, prologue, cfg, st, batch, nrhs);
    default: return launch_hop_ls<P, 0>(a, dagger, prologue, cfg, st, batch, nrhs);
  }
}

template <typename P>
int launch_hop_eo5(const HopArgs<P>& a0, const HopArgs<P>& a1, bool dagger, const LaunchCfg& cfg, hipStream_t st) {
  const int LH = a0.Ls;
  if (LH < 1 || 64 % LH != 0 || a1.Ls != LH || a1.nsites != a0.nsites) return -1;
  if (cfg.ns != 1 || cfg.spb < 1 || cfg.spb * LH > 256) return -1;
  for (const HopArgs<P>* a : {&a0, &a1}) {
    if (a->E || a->epi_scan || a->out2.data || !a->loc.data || (a->sigma != 0 && a->sigma != 1)) return -1;
    if (a->cg_r.data ? (!dagger || !a->cg_scalars) : !a->out.data) return -1;
  }
  if ((a0.cg_r.data == nullptr) != (a1.cg_r.data == nullptr)) return -1;
  if (hop_lds_bytes<P>(cfg, LH, false) > 65536) return -1;
  if (a0.nsites <= 0) return 0;
  switch (LH) {
    case 8: return launch_hop_eo5_ls<P, 8>(a0, a1, dagger, cfg, st);
    case 16: return launch_hop_eo5_ls<P, 16>(a0, a1, dagger, cfg, st);
    case 32: return launch_hop_eo5_ls<P, 32>(a0, a1, dagger, cfg, st);
    default: return launch_hop_eo5_ls<P, 0>(a0, a1, dagger, cfg, st);
  }
}

// ------------------------------------------------------------------ site-local fifth-dimension matrices
template <typename P, int LSEG>
__global__ void __launch_bounds__(256) fifth_kernel(CHalf<P> in, Half<P> out, const typename P::R* E,
                                                     FifthScan<typename P::R> es, CHalf<P> xin, typename P::R ax,
                                                     long nsites, int Ls_rt, int spb, double* norm_partials) {
  using R = typename P::R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int Ls = LSEG > 0 ? LSEG : Ls_rt;
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
  const int lsite = threadIdx.x / Ls;
  const int s = threadIdx.x - lsite * Ls;
  const long x = (long)blockIdx.x * spb + lsite;
  const bool active = (lsite < spb) && (x < nsites);
  if constexpr (LSEG > 0) {
    // recurrence form: the site's Ls lanes are one segment of the wave
    cx<R> o[12];
    if (active) load_spinor<P>(in, x, s, Ls, o);
    else
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
    fifth_scan_apply<LSEG>(o, s, es);
    double nrm = 0.0;
    if (active) {
      if (xin.data) {
        cx<R> xv[12];
        load_spinor<P>(xin, x, s, Ls, xv);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = o[k] + ax * xv[k];
      }
      if (norm_partials) {
#pragma unroll
        for (int k = 0; k < 12; ++k) nrm += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
      }
      store_spinor<P>(out, x, s, Ls, o);
    }
    if (norm_partials) {
      const double t = block_sum(nrm, red);
      if (threadIdx.x == 0) norm_partials[blockIdx.x] = t;
    }
    return;
  }
  if (active) {
    cx<R> v[12];
    load_spinor<P>(in, x, s, Ls, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) lds[(lsite * 12 + k) * Ls + s] = v[k];
  }
  __syncthreads();
  double nrm = 0.0;
  if (active) {
    cx<R> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
    const R* E0 = E + s * Ls;
    const R* E1 = E + Ls * Ls + s * Ls;
    const cx<R>* row = lds + lsite * 12 * Ls;
    for (int sp = 0; sp < Ls; ++sp) {
      const R e0 = E0[sp], e1 = E1[sp];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        o[k].re = fma(e0, row[k * Ls + sp].re, o[k].re);
        o[k].im = fma(e0, row[k * Ls + sp].im, o[k].im);
      }
#pragma unroll
      for (int k = 6; k < 12; ++k) {
        o[k].re = fma(e1, row[k * Ls + sp].re, o[k].re);
        o[k].im = fma(e1, row[k * Ls + sp].im, o[k].im);
      }
    }
    if (xin.data) {
      cx<R> xv[12];
      load_spinor<P>(xin, x, s, Ls, xv);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = o[k] + ax * xv[k];
    }
    if (norm_partials) {
#pragma unroll
      for (int k = 0; k < 12; ++k) nrm += double(o[k].re) * double(o[k].re) + double(o[k].im) * double(o[k].im);
    }
    store_spinor<P>(out, x, s, Ls, o);
  }
  if (norm_partials) {
    const double t = block_sum(nrm, red);
    if (threadIdx.x == 0) norm_partials[blockIdx.x] = t;
  }
}

template <typename P>
int launch_fifth(CHalf<P> in, Half<P> out, const typename P::R* E, const FifthScan<typename P::R>* es, CHalf<P> x,
                 typename P::R ax, long nsites, int Ls, double* norm_partials, hipStream_t st) {
  using R = typename P::R;
  if (Ls < 1 || Ls > 256) return -1;
  if (nsites <= 0) return 0;
  if (es && (Ls == 8 || Ls == 16 || Ls == 32)) {
    // one slice per lane, sites aligned to wave segments (256 / Ls sites per workgroup)
    const int spb = 256 / Ls;
    const long blocks = (nsites + spb - 1) / spb;
    FifthScan<R> e = *es;
    if (Ls == 8)
      hipLaunchKernelGGL((fifth_kernel<P, 8>), dim3((unsigned)blocks), dim3(256), 0, st, in, out, E, e, x, ax, nsites, Ls,
                         spb, norm_partials);
    else if (Ls == 16)
      hipLaunchKernelGGL((fifth_kernel<P, 16>), dim3((unsigned)blocks), dim3(256), 0, st, in, out, E, e, x, ax, nsites,
                         Ls, spb, norm_partials);
    else
      hipLaunchKernelGGL((fifth_kernel<P, 32>), dim3((unsigned)blocks), dim3(256), 0, st, in, out, E, e, x, ax, nsites,
                         Ls, spb, norm_partials);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
  int spb = 256 / Ls;
  if (spb < 1) spb = 1;
  while (spb > 1 && size_t(spb) * 12 * Ls * sizeof(cx<R>) > 65536) --spb;
  const long blocks = (nsites + spb - 1) / spb;
  const size_t lds = size_t(spb) * 12 * Ls * sizeof(cx<R>);
  FifthScan<R> e{};
  hipLaunchKernelGGL((fifth_kernel<P, 0>), dim3((unsigned)blocks), dim3(spb * Ls), lds, st, in, out, E, e, x, ax, nsites,
                     Ls, spb, norm_partials);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// number of workgroups launch_fifth / launch_hop use (partials array sizing)
inline long fifth_blocks(long nsites, int Ls, size_t elem) {
  int spb = 256 / Ls;
  if (spb < 1) spb = 1;
  while (spb > 1 && size_t(spb) * 12 * Ls * elem > 65536) --spb;
  return (nsites + spb - 1) / spb;
}

}  // namespace dwf

#define DWF_HOP_LS_ONE(P, L)                                                                           \
  template int dwf::launch_hop_ls<P, L>(const HopArgs<P>&, bool, bool, const LaunchCfg&, hipStream_t, \
                                        const HopArgs<P>*, int);                                       \
  template int dwf::launch_hop_eo5_ls<P, L>(const HopArgs<P>&, const HopArgs<P>&, bool, const LaunchCfg&, hipStream_t);
#define DWF_HOP_LS_EXTERN(P, L)                                                                               \
  extern template int dwf::launch_hop_ls<P, L>(const HopArgs<P>&, bool, bool, const LaunchCfg&, hipStream_t, \
                                               const HopArgs<P>*, int);                                       \
  extern template int dwf::launch_hop_eo5_ls<P, L>(const HopArgs<P>&, const HopArgs<P>&, bool, const LaunchCfg&, \
                                                   hipStream_t);
#define DWF_INSTANTIATE_HOP(P)                                                                                   \
  DWF_HOP_LS_EXTERN(P, 0) DWF_HOP_LS_EXTERN(P, 8) DWF_HOP_LS_EXTERN(P, 12) DWF_HOP_LS_EXTERN(P, 16)               \
  DWF_HOP_LS_EXTERN(P, 32)                                                                                      \
  template int dwf::launch_hop<P>(const HopArgs<P>&, bool, bool, const LaunchCfg&, hipStream_t,                \
                                  const HopArgs<P>*, int);                                                      \
  template int dwf::launch_hop_ilv<P>(const HopArgs<P>&, bool, int, const LaunchCfg&, hipStream_t);             \
  template int dwf::launch_hop_eo5<P>(const HopArgs<P>&, const HopArgs<P>&, bool, const LaunchCfg&, hipStream_t); \
  template int dwf::launch_fifth<P>(CHalf<P>, Half<P>, const P::R*, const FifthScan<P::R>*, CHalf<P>, P::R,   \
                                    long, int, double*, hipStream_t);
