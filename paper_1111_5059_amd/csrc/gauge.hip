// Gauge-field kernels of the molecular-dynamics step (Sec. 2), natural layouts
// U[mu][i][3][3], P[mu][i][3][3] (complex128), i = x + X (y + Y (z + Z t)), periodic links:
//   * the Wilson plaquette action beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3);
//   * its force F_mu(x) = sum_a e_a(S_g) T_a = (beta/6) TA(U_mu(x) A_mu(x)), A = the six
//     staples, TA(M) = (M - M^+)/2 - tr(M - M^+)/6  (T_a = i lambda_a / 2);
//   * the momentum update P <- P - eps F and the kinetic energy -sum tr(P P) = sum p_a^2 / 2.
// One thread per site (action) or per link (force); FP64 partial sums per workgroup.
#include "kernels.hpp"
#include "hop_impl.hpp"

namespace dwf {

using C = cx<double>;

struct NatGeom {
  int L[4];
  long V;
};

__device__ __forceinline__ long nat_step(const NatGeom& g, long i, int mu, int dir) {
  long c[4];
  long r = i;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = r % g.L[k];
    r /= g.L[k];
  }
  c[mu] = (c[mu] + dir + g.L[mu]) % g.L[mu];
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

__device__ __forceinline__ void ld3(const double2* U, long l, C M[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = {U[l * 9 + k].x, U[l * 9 + k].y};
}
__device__ __forceinline__ void mul3(const C* A, const C* B, C* R) {
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
// A B^+
__device__ __forceinline__ void mul3_nd(const C* A, const C* B, C* R) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(A[r * 3 + k], C{B[c * 3 + k].re, -B[c * 3 + k].im}, s);
      R[r * 3 + c] = s;
    }
}
// A^+ B
__device__ __forceinline__ void mul3_dn(const C* A, const C* B, C* R) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      C s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(C{A[k * 3 + r].re, -A[k * 3 + r].im}, B[k * 3 + c], s);
      R[r * 3 + c] = s;
    }
}

__global__ void __launch_bounds__(256) plaquette_kernel(const double2* U, NatGeom g, double* partials) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < g.V) {
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        C a[9], b[9], c[9], d[9], t1[9], t2[9];
        ld3(U, long(mu) * g.V + i, a);
        ld3(U, long(nu) * g.V + nat_step(g, i, mu, +1), b);
        ld3(U, long(mu) * g.V + nat_step(g, i, nu, +1), c);
        ld3(U, long(nu) * g.V + i, d);
        mul3(a, b, t1);       // U_mu(x) U_nu(x+mu)
        mul3_nd(t1, c, t2);   // .. U_mu(x+nu)^+
        mul3_nd(t2, d, t1);   // .. U_nu(x)^+
        acc += 1.0 - (t1[0].re + t1[4].re + t1[8].re) / 3.0;
      }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

int launch_plaquette(const double2* U, const int dims[4], double* partials, int* nblocks, hipStream_t st) {
  NatGeom g;
  g.V = 1;
  for (int k = 0; k < 4; ++k) { g.L[k] = dims[k]; g.V *= dims[k]; }
  const long nb = (g.V + 255) / 256;
  *nblocks = int(nb);
  hipLaunchKernelGGL(plaquette_kernel, dim3((unsigned)nb), dim3(256), 0, st, U, g, partials);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ void __launch_bounds__(256) gauge_force_kernel(const double2* U, NatGeom g, double beta, double coef,
                                                          int accumulate, double2* F) {
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= 4 * g.V) return;
  const int mu = int(l / g.V);
  const long i = l - long(mu) * g.V;
  C A[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) A[k] = {0.0, 0.0};
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    C a[9], b[9], c[9], t1[9], t2[9];
    // U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    ld3(U, long(nu) * g.V + nat_step(g, i, mu, +1), a);
    ld3(U, long(mu) * g.V + nat_step(g, i, nu, +1), b);
    ld3(U, long(nu) * g.V + i, c);
    mul3_nd(a, b, t1);
    mul3_nd(t1, c, t2);
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = A[k] + t2[k];
    // U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
    const long xm = nat_step(g, i, nu, -1);
    ld3(U, long(nu) * g.V + nat_step(g, xm, mu, +1), a);
    ld3(U, long(mu) * g.V + xm, b);
    ld3(U, long(nu) * g.V + xm, c);
    mul3(b, a, t1);        // U_mu(x-nu) U_nu(x+mu-nu)
    mul3_dn(t1, c, t2);    // (U_mu(x-nu) U_nu(x+mu-nu))^+ U_nu(x-nu)
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = A[k] + t2[k];
  }
  C u[9], M[9];
  ld3(U, l, u);
  mul3(u, A, M);
  const double trim = (M[0].im + M[4].im + M[8].im) / 3.0;  // tr(M - M^+) / 6 = i Im tr M / 3
  const double s = coef * beta / 6.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const C a1 = M[r * 3 + c], a2 = {M[c * 3 + r].re, -M[c * 3 + r].im};
      C ta = {0.5 * (a1.re - a2.re), 0.5 * (a1.im - a2.im)};
      if (r == c) ta.im -= trim;
      double2 v = make_double2(s * ta.re, s * ta.im);
      if (accumulate) {
        v.x += F[l * 9 + r * 3 + c].x;
        v.y += F[l * 9 + r * 3 + c].y;
      }
      F[l * 9 + r * 3 + c] = v;
    }
}

int launch_gauge_force(const double2* U, const int dims[4], double beta, double coef, int accumulate, double2* F,
                       hipStream_t st) {
  NatGeom g;
  g.V = 1;
  for (int k = 0; k < 4; ++k) { g.L[k] = dims[k]; g.V *= dims[k]; }
  const long n = 4 * g.V;
  hipLaunchKernelGGL(gauge_force_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U, g, beta, coef,
                     accumulate, F);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// P <- P - eps F (complex arrays of n entries)
__global__ void __launch_bounds__(256) mom_update_kernel(double2* P, const double2* F, double eps, long n) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double2 f = F[k];
  double2 p = P[k];
  p.x -= eps * f.x;
  p.y -= eps * f.y;
  P[k] = p;
}

int launch_mom_update(double2* P, const double2* F, double eps, long nlinks, hipStream_t st) {
  const long n = nlinks * 9;
  if (n <= 0) return 0;
  hipLaunchKernelGGL(mom_update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, P, F, eps, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// -tr(P P) per link, FP64 partial sums per workgroup
__global__ void __launch_bounds__(256) kinetic_kernel(const double2* P, long nlinks, double* partials) {
  __shared__ double red[16];
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (l < nlinks) {
    C m[9];
    ld3(P, l, m);
    C t = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) t = cfma(m[r * 3 + c], m[c * 3 + r], t);
    acc = -t.re;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int launch_kinetic(const double2* P, long nlinks, double* partials, int* nblocks, hipStream_t st) {
  const long nb = (nlinks + 255) / 256;
  *nblocks = int(nb);
  hipLaunchKernelGGL(kinetic_kernel, dim3((unsigned)nb), dim3(256), 0, st, P, nlinks, partials);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace dwf
