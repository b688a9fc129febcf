// Batched hop launch: descriptor tables of lattice groups and their right-hand sides.
#pragma once
#include <vector>
#include "kernels.hpp"

namespace dwf {

// One lattice: its links for the output parity, neighbour table and traversal order.
template <typename P>
struct MultiGroup {
  const typename P::S* links;
  const int* nbr;
  const int* order;
  long nsites;
  int Ls;
  int spb;           // 4D sites per workgroup (spb * Ls <= 256)
  long block_begin;  // first workgroup of this group in the launch
  int rhs_begin;     // first entry of this group in the right-hand-side table
  int nrhs;
};

// One right-hand side: out = ax x + E . (scale H F in), with its own E (mass).
template <typename P>
struct MultiRhs {
  CHalf<P> in;
  Half<P> out;
  const typename P::R* E;
  CHalf<P> x;
  typename P::R ax, scale, pb, pc, pm;
  double* norm_partials;  // one FP64 partial per workgroup of the group, or nullptr
  FifthScan<typename P::R> es;  // E in recurrence form (used when every right-hand side of the
  int scan = 0;                 // launch has it and the groups share Ls = 8, 16 or 32)
  // CG step fused into the last hop of M^dag M p (cg_r.data == nullptr: none): the result v is
  // not stored; r -= alpha v with alpha = cg_sc[S_ALPHA], norm_partials of the new |r|^2
  Half<P> cg_r = {nullptr, nullptr};
  const double* cg_sc = nullptr;
};

template <typename P>
size_t multi_lds_bytes(int spb, int Ls, bool epi);

// scan: every right-hand side carries its epilogue in recurrence form (MultiRhs::scan); the
// launch then applies it with wave-segment scans when all groups share Ls = 8, 16 or 32
template <typename P>
int launch_hop_multi(const MultiGroup<P>* d_groups, const std::vector<MultiGroup<P>>& h_groups, const MultiRhs<P>* d_rhs,
                     bool dagger, bool prologue, bool epi, hipStream_t st, bool scan = false);

}  // namespace dwf
