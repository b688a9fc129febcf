// Solver entry points used by the C ABI.
#pragma once
#include <string>
#include "runtime.hpp"

namespace dwf {

struct SolveStats {
  int iters = 0;
  int reliable_updates = 0;
  int restarts = 0;
  double last_rel = 0.0;
};

int normal_solve(dwf_ctx* ctx, const dwf_params& p, const void* U64, CHalf<P64> rhs, Half<P64> x, double tol_n,
                 int maxit, double delta, const std::string& tag, SolveStats* st);
int solve_full(dwf_ctx* ctx, const dwf_params& p, const void* U64, const void* b, void* x, double tol, int maxit,
               double delta, const std::string& tag, dwf_solve_info* info);
int solve_full_5d(dwf_ctx* ctx, const dwf_params& p, const void* U64, const void* b, void* x, double tol, int maxit,
                  double delta, const std::string& tag, dwf_solve_info* info);
int dslash_5d(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op, int dagger);
int solve_batched(dwf_ctx* ctx, int nrhs, const dwf_params* P, const void* const* U64, const void* const* b,
                  void* const* x, dwf_solve_info* info);
int madwf(dwf_ctx* ctx, const dwf_params& pt, const dwf_params& pi, const void* U64, const void* b, void* x,
          dwf_madwf_info* info);
int fermion_force(dwf_ctx* ctx, const dwf_params& p, const void* Unat, const void* phi, void* F, double* S,
                  double tau_fg, int out_kind, void* x_io, dwf_solve_info* info);
int fgi_trajectory(dwf_ctx* ctx, const dwf_params& p, void* U, void* P, const void* phi, dwf_hmc_info* info);
int quotient_force(dwf_ctx* ctx, const dwf_params& p, int nq, const double* masses, const void* Unat,
                   const void* const* phi, void* F, double* S, int out_kind, void* const* x_io,
                   dwf_solve_info* info);

}  // namespace dwf
