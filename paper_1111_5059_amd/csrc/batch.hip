// Batched Wilson hop: one launch applies the hop (with the same fused stages as
// the single-field kernel) to every right-hand side of one or more lattices.
//
// A *group* is one lattice (links, neighbour table, traversal order, Ls) with a
// list of right-hand sides on it -- e.g. the Hasenbusch mass ladder of Sec. 3,
// where every RHS has its own mass and therefore its own A^-1 epilogue.  Groups
// may differ in extents and Ls (a ragged batch); workgroups are dealt to groups
// by a prefix table.  Each workgroup stages the links of its 4D sites in LDS once
// and then loops over the group's right-hand sides, so a link is fetched from
// memory once for all of them.
#include "hop_impl.hpp"
#include "batch.hpp"

namespace dwf {

// LS > 0: every group has Ls = LS and the epilogue runs in recurrence form (one slice per
// lane, the site's LS lanes one wave segment); LS = 0: the dense Ls x Ls epilogue through LDS
template <typename P, bool DAG, bool PRO, bool EPI, int LS>
__global__ void __launch_bounds__(256) hop_multi_kernel(const MultiGroup<P>* groups, int ngroups,
                                                        const MultiRhs<P>* rhs) {
  using R = typename P::R;
  using S = typename P::S;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  int gi = 0;
  while (gi + 1 < ngroups && (long)blockIdx.x >= groups[gi + 1].block_begin) ++gi;
  const MultiGroup<P> g = groups[gi];
  const int Ls = LS > 0 ? LS : g.Ls;
  constexpr bool DENSE = EPI && LS == 0;
  const long bid = (long)blockIdx.x - g.block_begin;
  const int lsite = threadIdx.x / Ls;
  const int s0 = threadIdx.x - lsite * Ls;
  const long slot = bid * g.spb + lsite;
  const bool active = (lsite < g.spb) && (slot < g.nsites);
  const long x = active ? (g.order ? long(g.order[slot]) : slot) : 0;
  // links of the workgroup's sites, staged once for all right-hand sides
  S* llds = reinterpret_cast<S*>(smem_raw + (DENSE ? size_t(g.spb) * 12 * Ls * sizeof(cx<R>) : 0));
  for (int i = threadIdx.x; i < g.spb * 72; i += blockDim.x) {
    const int ls = i / 72;
    const long sl = bid * g.spb + ls;
    if (sl < g.nsites) {
      const long xs = g.order ? long(g.order[sl]) : sl;
      llds[i] = g.links[xs * 72 + (i - ls * 72)];
    }
  }
  __syncthreads();
  const S* L = llds + (lsite < g.spb ? lsite : 0) * 72;
  const int* nb = g.nbr + x * 8;
  for (int r = 0; r < g.nrhs; ++r) {
    const MultiRhs<P> q = rhs[g.rhs_begin + r];
    HopArgs<P> a;
    a.in = q.in;
    a.Ls = Ls;
    a.pb = q.pb;
    a.pc = q.pc;
    a.pm = q.pm;
    a.scale = R(1);  // (q.scale is applied below)
    cx<R> acc[1][12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[0][k] = {R(0), R(0)};
    if (active) {
      const ProCoef<R> pro[1] = {pro_coef<P, PRO>(a, s0)};
      hop_dir<0, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<1, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<2, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<3, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<4, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<5, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<6, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
      hop_dir<7, DAG, PRO, 1, false>(a, nb, L, s0, Ls, pro, acc);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[0][k] = q.scale * acc[0][k];
    if constexpr (EPI && LS > 0) {
      fifth_scan_apply<LS>(acc[0], s0, q.es);  // (all lanes: inactive ones hold zeros)
    }
    if constexpr (DENSE) {
      cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
      __syncthreads();  // the previous right-hand side's epilogue reads are complete
      if (active) {
#pragma unroll
        for (int k = 0; k < 12; ++k) lds[(lsite * 12 + k) * Ls + s0] = acc[0][k];
      }
      __syncthreads();
      if (active) {
        const R* E0 = q.E + s0 * Ls;
        const R* E1 = q.E + Ls * Ls + s0 * Ls;
        cx<R> o[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = {R(0), R(0)};
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
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0][k] = o[k];
      }
    }
    double nrm = 0.0;
    if (active) {
      if (q.x.data) {
        cx<R> xv[12];
        load_spinor<P>(q.x, x, s0, Ls, xv);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[0][k] = acc[0][k] + q.ax * xv[k];
      }
      if (q.cg_r.data) {
        // r -= alpha v: the CG residual update of this right-hand side on the site
        const R alpha = R(q.cg_sc[S_ALPHA]);
        cx<R> rv[12];
        load_spinor<P>(CHalf<P>{q.cg_r.data, q.cg_r.norm}, x, s0, Ls, rv);
#pragma unroll
        for (int k = 0; k < 12; ++k) rv[k] = {rv[k].re - alpha * acc[0][k].re, rv[k].im - alpha * acc[0][k].im};
        store_spinor<P>(q.cg_r, x, s0, Ls, rv);
        if (q.norm_partials) {
#pragma unroll
          for (int k = 0; k < 12; ++k) nrm += double(rv[k].re) * double(rv[k].re) + double(rv[k].im) * double(rv[k].im);
        }
      } else {
        if (q.norm_partials) {
#pragma unroll
          for (int k = 0; k < 12; ++k)
            nrm += double(acc[0][k].re) * double(acc[0][k].re) + double(acc[0][k].im) * double(acc[0][k].im);
        }
        store_spinor<P>(q.out, x, s0, Ls, acc[0]);
      }
    }
    if (q.norm_partials) {
      const double t = block_sum(nrm, red);
      if (threadIdx.x == 0) q.norm_partials[bid] = t;
      __syncthreads();
    }
  }
}

template <typename P>
size_t multi_lds_bytes(int spb, int Ls, bool epi) {
  return (epi ? size_t(spb) * 12 * Ls * sizeof(cx<typename P::R>) : 0) + size_t(spb) * 72 * sizeof(typename P::S);
}

// Validates every group's shape against the kernel's assumptions before launching:
// spb * Ls <= 256 threads, LDS within 64 KiB, consistent block prefix.
template <typename P, bool DAG, bool PRO, bool EPI>
static void launch_multi_ls(int ls, long blocks, int threads, size_t lds, hipStream_t st, const MultiGroup<P>* d_groups,
                            int ng, const MultiRhs<P>* d_rhs) {
  switch (ls) {
    case 8: hipLaunchKernelGGL((hop_multi_kernel<P, DAG, PRO, EPI, 8>), dim3((unsigned)blocks), dim3(threads), lds, st, d_groups, ng, d_rhs); break;
    case 16: hipLaunchKernelGGL((hop_multi_kernel<P, DAG, PRO, EPI, 16>), dim3((unsigned)blocks), dim3(threads), lds, st, d_groups, ng, d_rhs); break;
    case 32: hipLaunchKernelGGL((hop_multi_kernel<P, DAG, PRO, EPI, 32>), dim3((unsigned)blocks), dim3(threads), lds, st, d_groups, ng, d_rhs); break;
    default: hipLaunchKernelGGL((hop_multi_kernel<P, DAG, PRO, EPI, 0>), dim3((unsigned)blocks), dim3(threads), lds, st, d_groups, ng, d_rhs); break;
  }
}

template <typename P>
int launch_hop_multi(const MultiGroup<P>* d_groups, const std::vector<MultiGroup<P>>& h_groups, const MultiRhs<P>* d_rhs,
                     bool dagger, bool prologue, bool epi, hipStream_t st, bool scan) {
  if (h_groups.empty()) return 0;
  if (dagger && prologue) return -1;
  // the recurrence form needs one Ls of 8, 16 or 32 for the whole launch (a compile-time segment)
  int ls = 0;
  if (epi && scan) {
    ls = h_groups[0].Ls;
    for (const auto& g : h_groups)
      if (g.Ls != ls) ls = 0;
    if (ls != 8 && ls != 16 && ls != 32) ls = 0;
  }
  long blocks = 0;
  size_t lds = 0;
  int threads = 0;
  for (const auto& g : h_groups) {
    if (g.Ls < 1 || g.spb < 1 || g.spb * g.Ls > 256 || g.nrhs < 1) return -1;
    if (g.block_begin != blocks) return -1;
    blocks += (g.nsites + g.spb - 1) / g.spb;
    lds = std::max(lds, multi_lds_bytes<P>(g.spb, g.Ls, epi && ls == 0));
    threads = std::max(threads, g.spb * g.Ls);
  }
  if (lds > 65536) return -1;
  if (blocks <= 0) return 0;
  const int ng = int(h_groups.size());
  if (dagger) {
    if (epi) launch_multi_ls<P, true, false, true>(ls, blocks, threads, lds, st, d_groups, ng, d_rhs);
    else launch_multi_ls<P, true, false, false>(0, blocks, threads, lds, st, d_groups, ng, d_rhs);
  } else if (prologue) {
    if (epi) launch_multi_ls<P, false, true, true>(ls, blocks, threads, lds, st, d_groups, ng, d_rhs);
    else launch_multi_ls<P, false, true, false>(0, blocks, threads, lds, st, d_groups, ng, d_rhs);
  } else {
    if (epi) launch_multi_ls<P, false, false, true>(ls, blocks, threads, lds, st, d_groups, ng, d_rhs);
    else launch_multi_ls<P, false, false, false>(0, blocks, threads, lds, st, d_groups, ng, d_rhs);
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define DWF_INST_MULTI(P)                                                                                        \
  template int launch_hop_multi<P>(const MultiGroup<P>*, const std::vector<MultiGroup<P>>&, const MultiRhs<P>*, \
                                   bool, bool, bool, hipStream_t, bool);                                        \
  template size_t multi_lds_bytes<P>(int, int, bool);

DWF_INST_MULTI(P64)
DWF_INST_MULTI(P32)
DWF_INST_MULTI(P16)
DWF_INST_MULTI(PB16)

}  // namespace dwf
