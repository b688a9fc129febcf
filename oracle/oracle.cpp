// FP64 reference ("oracle") for the domain-wall / Moebius hot path of
// Yin & Mawhinney, "Improving DWF Simulations: the Force Gradient Integrator
// and the Moebius Accelerated DWF Solver" (Lattice 2011).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark may load or call this library.  It shares
// no code, header, table or helper with the HIP library: it is a plain, slow,
// obviously-correct restatement of the definitions, written for reading, not
// for speed (OpenMP over 4D sites is the only concession).
//
// Natural layouts (all complex<double>, row-major):
//   4D site index     i = x + X*(y + Y*(z + Z*t))
//   gauge field       U[mu][i][a][b]        mu = 0..3 <-> x,y,z,t
//   4D spinor         psi[i][spin][colour]
//   5D spinor         psi[s][i][spin][colour]  s = 0..Ls-1 (the paper's s=1..L)
//
// Readings of the paper (it defers the operator definitions to its
// domain-wall/overlap transformation reference):
//   * gamma matrices: chiral basis, gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
//     gamma_4 = [[0,1],[1,0]], gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
//     = diag(1,1,-1,-1); P+- = (1 +- gamma_5)/2.
//   * Wilson operator  D_W psi(x) = (4-M5) psi(x)
//        - 1/2 sum_mu [(1-gamma_mu) U_mu(x) psi(x+mu) + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
//     periodic, or antiperiodic in T when tbc = 1.
//   * 5D operator (Moebius; Shamir at b=1, c=0):
//        (D psi)_s = (b D_W + 1) psi_s + (c D_W - 1)(P- psi_{s+1} + P+ psi_{s-1})
//     with psi_{Ls} = -m psi_0 and psi_{-1} = -m psi_{Ls-1}.
//   * P: (P^-1 x)_s = P- x_s + P+ x_{s-1 mod Ls},  (P y)_s = P- y_s + P+ y_{s+1 mod Ls}.
//   * Even-odd (not in the paper): 4D checkerboard, parity (x+y+z+t) mod 2,
//     D = [[A, B_eo],[B_oe, A]], A = (b d + 1) + (c d - 1) S~, d = 4 - M5,
//     B = -1/2 H (b + c S~), M_prec = 1 - A^-1 B_oe A^-1 B_eo on odd sites.
//   * Generators T_a = i lambda_a / 2 (Gell-Mann), e_a(U) = T_a U (Sec. 2).
#include <complex>
#include <vector>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <omp.h>

typedef std::complex<double> cplx;

extern "C" {
typedef struct {
  int dims[4];
  int Ls;
  int tbc;
  double M5, mass, b, c;
  const double* bs;  // optional s-dependent Moebius coefficients b_s, c_s (Ls entries each;
  const double* cs;  // NULL: the constants b, c)
} ora_params;

// Moebius coefficients of slice s (Sec. 4 admits any Moebius operator: s-dependent b_s, c_s)
static inline double bco(const ora_params* p, int s) { return p->bs ? p->bs[s] : p->b; }
static inline double cco(const ora_params* p, int s) { return p->cs ? p->cs[s] : p->c; }

typedef struct {
  int iters;             // CG iterations (normal-equation operator applications)
  int restarts;          // number of tightening restarts to reach the true residual
  double true_rel_resid; // ||b - D x|| / ||b|| (full 5D system)
  double seconds;
} ora_solve_info;

typedef struct {
  int pv_iters;          // total CG iterations in the Pauli-Villars solves
  int mob_iters;         // total CG iterations in the Moebius solves
  int final_iters;       // iterations of the final warm-started DWF solve
  int n_pv, n_mob;       // number of solves of each kind
  double resid_after_dc[16]; // true residual after each defect-correction step
  double true_rel_resid;
  double seconds;
} ora_madwf_info;
}

namespace {

// ---------------------------------------------------------------- geometry
struct Geom {
  int L[4];
  long V;
  int tbc;
};

Geom geom_of(const ora_params* p) {
  Geom g;
  g.V = 1;
  for (int m = 0; m < 4; ++m) { g.L[m] = p->dims[m]; g.V *= p->dims[m]; }
  g.tbc = p->tbc;
  return g;
}

void coords_of(const Geom& g, long i, int c[4]) {
  for (int m = 0; m < 4; ++m) { c[m] = int(i % g.L[m]); i /= g.L[m]; }
}

long index_of(const Geom& g, const int c[4]) {
  long i = 0;
  for (int m = 3; m >= 0; --m) i = i * g.L[m] + c[m];
  return i;
}

int parity_of(const Geom& g, long i) {
  int c[4];
  coords_of(g, i, c);
  return (c[0] + c[1] + c[2] + c[3]) & 1;
}

// neighbour x +- mu with the boundary phase picked up by the hop (antiperiodic in T)
long step(const Geom& g, long i, int mu, int dir, double* phase) {
  int c[4];
  coords_of(g, i, c);
  *phase = 1.0;
  c[mu] += dir;
  if (c[mu] >= g.L[mu]) { c[mu] -= g.L[mu]; if (mu == 3 && g.tbc) *phase = -1.0; }
  if (c[mu] < 0)        { c[mu] += g.L[mu]; if (mu == 3 && g.tbc) *phase = -1.0; }
  return index_of(g, c);
}

// ---------------------------------------------------------------- Dirac algebra
struct Gammas {
  cplx g[5][4][4];  // g[0..3] = gamma_1..gamma_4, g[4] = gamma_5
  cplx pplus[4][4], pminus[4][4];
  Gammas() {
    const cplx I(0, 1);
    cplx sigma[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    std::memset((void*)g, 0, sizeof(g));
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          g[k][a][2 + b] = -I * sigma[k][a][b];
          g[k][2 + a][b] = I * sigma[k][a][b];
        }
    for (int a = 0; a < 2; ++a) { g[3][a][2 + a] = 1; g[3][2 + a][a] = 1; }
    // gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4
    cplx t1[4][4], t2[4][4];
    matmul4(g[0], g[1], t1);
    matmul4(t1, g[2], t2);
    matmul4(t2, g[3], g[4]);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        cplx id = (a == b) ? 1.0 : 0.0;
        pplus[a][b] = 0.5 * (id + g[4][a][b]);
        pminus[a][b] = 0.5 * (id - g[4][a][b]);
      }
  }
  static void matmul4(const cplx A[4][4], const cplx B[4][4], cplx C[4][4]) {
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        cplx s = 0;
        for (int k = 0; k < 4; ++k) s += A[a][k] * B[k][b];
        C[a][b] = s;
      }
  }
};

const Gammas& gam() {
  static Gammas G;
  return G;
}

// out[spin][col] += coef * M[spin][spin'] v[spin'][col]
void spin_mul_acc(const cplx M[4][4], const cplx* v, cplx coef, cplx* out) {
  for (int a = 0; a < 4; ++a)
    for (int col = 0; col < 3; ++col) {
      cplx s = 0;
      for (int b = 0; b < 4; ++b) s += M[a][b] * v[b * 3 + col];
      out[a * 3 + col] += coef * s;
    }
}

const cplx* link(const Geom& g, const cplx* U, int mu, long i) { return U + ((long)mu * g.V + i) * 9; }

// ---------------------------------------------------------------- 4D Wilson hop
// (H psi)(x) = sum_mu [(1 - sg gamma_mu) U_mu(x) psi(x+mu) + (1 + sg gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
// sg = +1 for H, -1 for H^dag.  Both neighbour terms are accumulated even when
// x+mu == x-mu (extent-2 directions).
void hop_site(const Geom& g, const cplx* U, const cplx* in, long i, int dagger, cplx* out) {
  const Gammas& G = gam();
  const double sg = dagger ? -1.0 : 1.0;
  for (int k = 0; k < 12; ++k) out[k] = 0;
  for (int mu = 0; mu < 4; ++mu) {
    double ph;
    // forward neighbour
    long f = step(g, i, mu, +1, &ph);
    const cplx* Uf = link(g, U, mu, i);
    cplx v[12];
    for (int s = 0; s < 4; ++s)
      for (int a = 0; a < 3; ++a) {
        cplx acc = 0;
        for (int b = 0; b < 3; ++b) acc += Uf[a * 3 + b] * in[f * 12 + s * 3 + b];
        v[s * 3 + a] = ph * acc;
      }
    for (int k = 0; k < 12; ++k) out[k] += v[k];
    spin_mul_acc(G.g[mu], v, -sg, out);
    // backward neighbour
    long bk = step(g, i, mu, -1, &ph);
    const cplx* Ub = link(g, U, mu, bk);
    for (int s = 0; s < 4; ++s)
      for (int a = 0; a < 3; ++a) {
        cplx acc = 0;
        for (int b = 0; b < 3; ++b) acc += std::conj(Ub[b * 3 + a]) * in[bk * 12 + s * 3 + b];
        v[s * 3 + a] = ph * acc;
      }
    for (int k = 0; k < 12; ++k) out[k] += v[k];
    spin_mul_acc(G.g[mu], v, +sg, out);
  }
}

void hop4(const Geom& g, const cplx* U, const cplx* in, cplx* out, int dagger) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i) hop_site(g, U, in, i, dagger, out + i * 12);
}

// D_W = (4 - M5) - 1/2 H ;  D_W^dag = (4 - M5) - 1/2 H^dag
void dw4(const Geom& g, double M5, const cplx* U, const cplx* in, cplx* out, int dagger) {
  hop4(g, U, in, out, dagger);
  const long n = g.V * 12;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) out[k] = (4.0 - M5) * in[k] - 0.5 * out[k];
}

// ---------------------------------------------------------------- fifth dimension
// (S~ psi)_s = P- psi_{s+1} + P+ psi_{s-1},  psi_{Ls} = -m psi_0, psi_{-1} = -m psi_{Ls-1}
// (S~^dag psi)_s = P- psi_{s-1} + P+ psi_{s+1} (same boundary factors)
void stilde(const Geom& g, int Ls, double m, const cplx* in, cplx* out, int dagger) {
  const Gammas& G = gam();
  const long V12 = g.V * 12;
  for (int s = 0; s < Ls; ++s) {
    int sp = s + 1, sm = s - 1;
    double fp = 1.0, fm = 1.0;
    if (sp == Ls) { sp = 0; fp = -m; }
    if (sm < 0) { sm = Ls - 1; fm = -m; }
    const int s_minus_src = dagger ? sm : sp;  // slice that P- picks up
    const double f_minus = dagger ? fm : fp;
    const int s_plus_src = dagger ? sp : sm;   // slice that P+ picks up
    const double f_plus = dagger ? fp : fm;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g.V; ++i) {
      cplx* o = out + s * V12 + i * 12;
      for (int k = 0; k < 12; ++k) o[k] = 0;
      spin_mul_acc(G.pminus, in + s_minus_src * V12 + i * 12, f_minus, o);
      spin_mul_acc(G.pplus, in + s_plus_src * V12 + i * 12, f_plus, o);
    }
  }
}

// 5D operator D(m) (Moebius; Shamir at b=1,c=0) and its explicitly written adjoint
//   D   = (b D_W + 1) + (c D_W - 1) S~
//   D^+ = (b D_W^+ + 1) + S~^+ (c D_W^+ - 1)
// (b = diag(b_s), c = diag(c_s) with s-dependent coefficients)
void dwf5(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger) {
  Geom g = geom_of(p);
  const int Ls = p->Ls;
  const long V12 = g.V * 12, n = V12 * Ls;
  std::vector<cplx> w(n), t(n);
  if (!dagger) {
    stilde(g, Ls, p->mass, in, t.data(), 0);  // t = S~ psi
    for (int s = 0; s < Ls; ++s) {
      dw4(g, p->M5, U, in + s * V12, out + s * V12, 0);        // D_W psi_s
      dw4(g, p->M5, U, t.data() + s * V12, w.data() + s * V12, 0); // D_W (S~psi)_s
    }
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) {
      const int s = int(k / V12);
      out[k] = bco(p, s) * out[k] + in[k] + cco(p, s) * w[k] - t[k];
    }
  } else {
    for (int s = 0; s < Ls; ++s) dw4(g, p->M5, U, in + s * V12, w.data() + s * V12, 1);
    // t = c D_W^+ psi - psi
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) t[k] = cco(p, int(k / V12)) * w[k] - in[k];
    stilde(g, Ls, p->mass, t.data(), out, 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) out[k] += bco(p, int(k / V12)) * w[k] + in[k];
  }
}

// ---------------------------------------------------------------- even-odd pieces
// Site-local A = (b d + 1) + (c d - 1) S~ as a dense (Ls*4) x (Ls*4) matrix over
// (s, spin) (colour-diagonal), and its inverse by Gauss-Jordan elimination.
struct FifthMatrix {
  int n;
  std::vector<cplx> a;  // row-major n x n
};

FifthMatrix build_A(const ora_params* p) {
  const Gammas& G = gam();
  const int Ls = p->Ls, n = 4 * Ls;
  const double d = 4.0 - p->M5;
  FifthMatrix A;
  A.n = n;
  A.a.assign((size_t)n * n, 0.0);
  for (int s = 0; s < Ls; ++s) {
    for (int al = 0; al < 4; ++al) A.a[(s * 4 + al) * n + s * 4 + al] += bco(p, s) * d + 1.0;
    int sp = s + 1, sm = s - 1;
    double fp = 1.0, fm = 1.0;
    if (sp == Ls) { sp = 0; fp = -p->mass; }
    if (sm < 0) { sm = Ls - 1; fm = -p->mass; }
    for (int al = 0; al < 4; ++al)
      for (int be = 0; be < 4; ++be) {
        A.a[(s * 4 + al) * n + sp * 4 + be] += (cco(p, s) * d - 1.0) * fp * G.pminus[al][be];
        A.a[(s * 4 + al) * n + sm * 4 + be] += (cco(p, s) * d - 1.0) * fm * G.pplus[al][be];
      }
  }
  return A;
}

FifthMatrix invert(const FifthMatrix& M) {
  const int n = M.n;
  std::vector<cplx> a = M.a, inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(a[(size_t)r * n + col]) > std::abs(a[(size_t)piv * n + col])) piv = r;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
        std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
      }
    const cplx d = a[(size_t)col * n + col];
    for (int k = 0; k < n; ++k) { a[(size_t)col * n + k] /= d; inv[(size_t)col * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const cplx f = a[(size_t)r * n + col];
      if (f == cplx(0.0)) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)col * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
      }
    }
  }
  FifthMatrix R;
  R.n = n;
  R.a = inv;
  return R;
}

FifthMatrix adjoint(const FifthMatrix& M) {
  FifthMatrix R;
  R.n = M.n;
  R.a.assign(M.a.size(), 0.0);
  for (int i = 0; i < M.n; ++i)
    for (int j = 0; j < M.n; ++j) R.a[(size_t)j * M.n + i] = std::conj(M.a[(size_t)i * M.n + j]);
  return R;
}

// out(s,spin,col) at every 4D site = sum_{s',spin'} M[(s,spin),(s',spin')] in(s',spin',col)
void apply_fifth(const Geom& g, int Ls, const FifthMatrix& M, const cplx* in, cplx* out) {
  const long V12 = g.V * 12;
  const int n = M.n;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i) {
    for (int s = 0; s < Ls; ++s)
      for (int al = 0; al < 4; ++al)
        for (int col = 0; col < 3; ++col) {
          cplx acc = 0;
          for (int s2 = 0; s2 < Ls; ++s2)
            for (int be = 0; be < 4; ++be)
              acc += M.a[(size_t)(s * 4 + al) * n + s2 * 4 + be] * in[s2 * V12 + i * 12 + be * 3 + col];
          out[s * V12 + i * 12 + al * 3 + col] = acc;
        }
  }
}

// zero the sites of 4D parity != keep
void mask_parity(const Geom& g, int Ls, cplx* f, int keep) {
  const long V12 = g.V * 12;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i)
    if (parity_of(g, i) != keep)
      for (int s = 0; s < Ls; ++s)
        for (int k = 0; k < 12; ++k) f[s * V12 + i * 12 + k] = 0;
}

// F = b + c S~ (and F^dag = b + S~^dag c), site-local, b = diag(b_s), c = diag(c_s)
void apply_F(const ora_params* p, const Geom& g, const cplx* in, cplx* out, int dagger) {
  const long V12 = g.V * 12, n = V12 * p->Ls;
  if (!dagger) {
    stilde(g, p->Ls, p->mass, in, out, 0);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) out[k] = bco(p, int(k / V12)) * in[k] + cco(p, int(k / V12)) * out[k];
  } else {
    std::vector<cplx> t(n);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) t[k] = cco(p, int(k / V12)) * in[k];
    stilde(g, p->Ls, p->mass, t.data(), out, 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) out[k] += bco(p, int(k / V12)) * in[k];
  }
}

// hop on every s-slice: H (or H^dag) applied slice by slice
void hop5(const ora_params* p, const Geom& g, const cplx* U, const cplx* in, cplx* out, int dagger) {
  const long V12 = g.V * 12;
  for (int s = 0; s < p->Ls; ++s) hop4(g, U, in + s * V12, out + s * V12, dagger);
}

// B = -1/2 H F ;  B^dag = -1/2 F^dag H^dag ;  output restricted to parity out_par (-1: none)
void apply_B(const ora_params* p, const Geom& g, const cplx* U, const cplx* in, cplx* out, int dagger,
             int out_par) {
  const long n = g.V * 12 * p->Ls;
  std::vector<cplx> t(n);
  if (!dagger) {
    apply_F(p, g, in, t.data(), 0);
    hop5(p, g, U, t.data(), out, 0);
  } else {
    hop5(p, g, U, in, t.data(), 1);
    apply_F(p, g, t.data(), out, 1);
  }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) out[k] *= -0.5;
  if (out_par >= 0) mask_parity(g, p->Ls, out, out_par);
}

struct EOContext {
  FifthMatrix A, Ainv, Adag, Ainvdag;
  explicit EOContext(const ora_params* p) {
    A = build_A(p);
    Ainv = invert(A);
    Adag = adjoint(A);
    Ainvdag = adjoint(Ainv);
  }
};

// M_prec = 1 - A^-1 B_oe A^-1 B_eo   (odd -> odd);  in must vanish on even sites
// M_prec^dag = 1 - B_eo^dag A^-dag B_oe^dag A^-dag = 1 - (B^dag)_oe A^-dag (B^dag)_eo A^-dag
void mprec(const ora_params* p, const EOContext& E, const cplx* U, const cplx* in, cplx* out, int dagger) {
  Geom g = geom_of(p);
  const long n = g.V * 12 * p->Ls;
  std::vector<cplx> t(n), u(n);
  std::vector<cplx> src(in, in + n);
  mask_parity(g, p->Ls, src.data(), 1);
  if (!dagger) {
    apply_B(p, g, U, src.data(), t.data(), 0, 0);   // B_eo psi_o
    apply_fifth(g, p->Ls, E.Ainv, t.data(), u.data());
    apply_B(p, g, U, u.data(), t.data(), 0, 1);     // B_oe A^-1 B_eo psi_o
    apply_fifth(g, p->Ls, E.Ainv, t.data(), u.data());
  } else {
    apply_fifth(g, p->Ls, E.Ainvdag, src.data(), u.data());
    apply_B(p, g, U, u.data(), t.data(), 1, 0);
    apply_fifth(g, p->Ls, E.Ainvdag, t.data(), u.data());
    apply_B(p, g, U, u.data(), t.data(), 1, 1);
    u.swap(t);
  }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) out[k] = src[k] - u[k];
  mask_parity(g, p->Ls, out, 1);
}

// ---------------------------------------------------------------- vector algebra
double norm2(const cplx* a, long n) {
  double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (long k = 0; k < n; ++k) s += std::norm(a[k]);
  return s;
}

cplx dot(const cplx* a, const cplx* b, long n) {  // <a, b> = sum conj(a) b
  double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
  for (long k = 0; k < n; ++k) {
    cplx z = std::conj(a[k]) * b[k];
    re += z.real();
    im += z.imag();
  }
  return cplx(re, im);
}

// CG on the normal equations M^dag M x = rhs (M = M_prec, odd sites).  Stops
// when ||rhs - M^dag M x|| <= tol ||rhs||.  Returns iterations (or -1).
int cg_normal(const ora_params* p, const EOContext& E, const cplx* U, const cplx* rhs, cplx* x, double tol,
              int maxit, int* iters_out) {
  Geom g = geom_of(p);
  const long n = g.V * 12 * p->Ls;
  std::vector<cplx> r(n), pv(n), q(n), Ap(n);
  mprec(p, E, U, x, q.data(), 0);
  mprec(p, E, U, q.data(), Ap.data(), 1);
  for (long k = 0; k < n; ++k) { r[k] = rhs[k] - Ap[k]; pv[k] = r[k]; }
  double rr = norm2(r.data(), n);
  const double target = tol * tol * norm2(rhs, n);
  int it = 0;
  while (rr > target && it < maxit) {
    mprec(p, E, U, pv.data(), q.data(), 0);
    const double qq = norm2(q.data(), n);
    const double alpha = rr / qq;
    mprec(p, E, U, q.data(), Ap.data(), 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) { x[k] += alpha * pv[k]; r[k] -= alpha * Ap[k]; }
    const double rr_new = norm2(r.data(), n);
    const double beta = rr_new / rr;
    rr = rr_new;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; ++k) pv[k] = r[k] + beta * pv[k];
    ++it;
  }
  *iters_out = it;
  return rr <= target ? 0 : 1;
}

// Solve D(m) x = b for the full 5D system through the even-odd Schur complement
//   b'_o = A^-1 (b_o - B_oe A^-1 b_e),  M_prec x_o = b'_o,  x_e = A^-1 (b_e - B_eo x_o)
// with CGNR on M_prec, tightening the normal-equation tolerance until the
// full-system true residual ||b - D x|| / ||b|| <= tol.  x holds the guess on entry.
int solve_full(const ora_params* p, const cplx* U, const cplx* b, cplx* x, double tol, int maxit,
               ora_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  Geom g = geom_of(p);
  const int Ls = p->Ls;
  const long n = g.V * 12 * Ls;
  EOContext E(p);
  std::vector<cplx> be(b, b + n), bo(b, b + n), t(n), u(n), bprime(n), rhs(n), xo(x, x + n), r(n);
  mask_parity(g, Ls, be.data(), 0);
  mask_parity(g, Ls, bo.data(), 1);
  mask_parity(g, Ls, xo.data(), 1);
  apply_fifth(g, Ls, E.Ainv, be.data(), t.data());       // A^-1 b_e
  apply_B(p, g, U, t.data(), u.data(), 0, 1);             // B_oe A^-1 b_e
  for (long k = 0; k < n; ++k) t[k] = bo[k] - u[k];
  apply_fifth(g, Ls, E.Ainv, t.data(), bprime.data());   // b'_o
  mprec(p, E, U, bprime.data(), rhs.data(), 1);           // M^dag b'
  const double bnorm = std::sqrt(norm2(b, n));
  double tol_in = tol;
  int total = 0, restarts = 0, status = 1;
  double rel = 1.0;
  for (int attempt = 0; attempt < 8; ++attempt) {
    int it = 0;
    cg_normal(p, E, U, rhs.data(), xo.data(), tol_in, maxit - total, &it);
    total += it;
    // x_e = A^-1 (b_e - B_eo x_o)
    apply_B(p, g, U, xo.data(), u.data(), 0, 0);
    for (long k = 0; k < n; ++k) t[k] = be[k] - u[k];
    apply_fifth(g, Ls, E.Ainv, t.data(), u.data());
    mask_parity(g, Ls, u.data(), 0);
    for (long k = 0; k < n; ++k) x[k] = u[k] + xo[k];
    dwf5(p, U, x, r.data(), 0);
    for (long k = 0; k < n; ++k) r[k] = b[k] - r[k];
    rel = std::sqrt(norm2(r.data(), n)) / bnorm;
    if (rel <= tol) { status = 0; break; }
    if (total >= maxit) break;
    tol_in *= 0.5 * tol / rel;
    ++restarts;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iters = total;
    info->restarts = restarts;
    info->true_rel_resid = rel;
    info->seconds = std::chrono::duration<double>(t1 - t0).count();
  }
  return status;
}

// P and P^-1 (the domain-wall <-> overlap basis change, Sec. 4 footnote)
//   (P^-1 x)_s = P- x_s + P+ x_{s-1 mod Ls},   (P y)_s = P- y_s + P+ y_{s+1 mod Ls}
void apply_P(const Geom& g, int Ls, const cplx* in, cplx* out, int inverse) {
  const Gammas& G = gam();
  const long V12 = g.V * 12;
  for (int s = 0; s < Ls; ++s) {
    const int other = inverse ? (s + Ls - 1) % Ls : (s + 1) % Ls;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < g.V; ++i) {
      cplx* o = out + s * V12 + i * 12;
      for (int k = 0; k < 12; ++k) o[k] = 0;
      spin_mul_acc(G.pminus, in + s * V12 + i * 12, 1.0, o);
      spin_mul_acc(G.pplus, in + other * V12 + i * 12, 1.0, o);
    }
  }
}

// ---------------------------------------------------------------- SU(3) algebra
struct GellMann {
  cplx T[8][9];  // T_a = i lambda_a / 2
  GellMann() {
    const cplx I(0, 1);
    cplx lam[8][9];
    std::memset((void*)lam, 0, sizeof(lam));
    lam[0][1] = 1; lam[0][3] = 1;
    lam[1][1] = -I; lam[1][3] = I;
    lam[2][0] = 1; lam[2][4] = -1;
    lam[3][2] = 1; lam[3][6] = 1;
    lam[4][2] = -I; lam[4][6] = I;
    lam[5][5] = 1; lam[5][7] = 1;
    lam[6][5] = -I; lam[6][7] = I;
    const double r3 = 1.0 / std::sqrt(3.0);
    lam[7][0] = r3; lam[7][4] = r3; lam[7][8] = -2.0 * r3;
    for (int a = 0; a < 8; ++a)
      for (int k = 0; k < 9; ++k) T[a][k] = 0.5 * I * lam[a][k];
  }
};

const GellMann& gm() {
  static GellMann G;
  return G;
}

void mat3_mul(const cplx* A, const cplx* B, cplx* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}

// exp(A) by its power series, summed until the terms no longer change the sum
void mat3_exp(const cplx* A, cplx* out) {
  cplx term[9], tmp[9];
  for (int k = 0; k < 9; ++k) { out[k] = (k % 4 == 0) ? 1.0 : 0.0; term[k] = out[k]; }
  for (int n = 1; n < 200; ++n) {
    mat3_mul(term, A, tmp);
    double tn = 0, sn = 0;
    for (int k = 0; k < 9; ++k) {
      term[k] = tmp[k] / double(n);
      out[k] += term[k];
      tn += std::norm(term[k]);
      sn += std::norm(out[k]);
    }
    if (tn <= 1e-36 * sn) break;
  }
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void ora_gamma(cplx* out /* [5][4][4] */) {
  const Gammas& G = gam();
  std::memcpy((void*)out, (const void*)G.g, sizeof(G.g));
}

void ora_generators(cplx* out /* [8][3][3] */) {
  const GellMann& G = gm();
  std::memcpy((void*)out, (const void*)G.T, sizeof(G.T));
}

int ora_num_threads(void) { return omp_get_max_threads(); }

// 4D Wilson hopping term H (dagger=0) or H^dag (dagger=1) on one 4D field
void ora_hop4(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger) {
  Geom g = geom_of(p);
  hop4(g, U, in, out, dagger);
}

// 4D Wilson operator D_W(-M5) or its adjoint
void ora_dw4(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger) {
  Geom g = geom_of(p);
  dw4(g, p->M5, U, in, out, dagger);
}

// Wilson hop on every s-slice of a 5D field, output restricted to parity out_par (-1: all)
void ora_hop5(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger, int out_par) {
  Geom g = geom_of(p);
  hop5(p, g, U, in, out, dagger);
  if (out_par >= 0) mask_parity(g, p->Ls, out, out_par);
}

// Wilson hop evaluated only at n sampled 5D sites (4D lexicographic index, s) of a
// natural 5D field; out[n][12].  The same per-site definition as ora_hop5.
void ora_hop5_sample(const ora_params* p, const cplx* U, const cplx* in, long n, const long* sites, const int* svals,
                     int dagger, cplx* out) {
  Geom g = geom_of(p);
  const long V12 = g.V * 12;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) hop_site(g, U, in + (long)svals[k] * V12, sites[k], dagger, out + k * 12);
}

// 5D DWF / Moebius operator D(m) or D(m)^dag
void ora_dwf(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger) {
  dwf5(p, U, in, out, dagger);
}

void ora_stilde(const ora_params* p, const cplx* in, cplx* out, int dagger) {
  Geom g = geom_of(p);
  stilde(g, p->Ls, p->mass, in, out, dagger);
}

// site-local fifth-dimension operators: which = 0 A, 1 A^dag, 2 A^-1, 3 A^-dag, 4 F, 5 F^dag
void ora_fifth(const ora_params* p, const cplx* in, cplx* out, int which) {
  Geom g = geom_of(p);
  if (which >= 4) { apply_F(p, g, in, out, which - 4); return; }
  EOContext E(p);
  const FifthMatrix* M = which == 0 ? &E.A : which == 1 ? &E.Adag : which == 2 ? &E.Ainv : &E.Ainvdag;
  apply_fifth(g, p->Ls, *M, in, out);
}

// the dense (4 Ls) x (4 Ls) matrix of A over (s, spin) (colour-diagonal)
void ora_fifth_matrix(const ora_params* p, cplx* out, int which) {
  EOContext E(p);
  const FifthMatrix* M = which == 0 ? &E.A : which == 1 ? &E.Adag : which == 2 ? &E.Ainv : &E.Ainvdag;
  std::memcpy((void*)out, (const void*)M->a.data(), M->a.size() * sizeof(cplx));
}

// B = -1/2 H F (dagger: -1/2 F^dag H^dag), output restricted to parity out_par (-1: all)
void ora_bhop(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger, int out_par) {
  Geom g = geom_of(p);
  apply_B(p, g, U, in, out, dagger, out_par);
}

void ora_mprec(const ora_params* p, const cplx* U, const cplx* in, cplx* out, int dagger) {
  EOContext E(p);
  mprec(p, E, U, in, out, dagger);
}

void ora_P(const ora_params* p, const cplx* in, cplx* out, int inverse) {
  Geom g = geom_of(p);
  apply_P(g, p->Ls, in, out, inverse);
}

void ora_parity_mask(const ora_params* p, cplx* f, int keep) {
  Geom g = geom_of(p);
  mask_parity(g, p->Ls, f, keep);
}

// CGNR on M_prec: M^dag M x = M^dag b (b, x odd-only full-size arrays)
int ora_cgne(const ora_params* p, const cplx* U, const cplx* b, cplx* x, double tol, int maxit, int* iters) {
  Geom g = geom_of(p);
  const long n = g.V * 12 * p->Ls;
  EOContext E(p);
  std::vector<cplx> rhs(n);
  mprec(p, E, U, b, rhs.data(), 1);
  return cg_normal(p, E, U, rhs.data(), x, tol, maxit, iters);
}

// full 5D solve D(m) x = b to a true residual tol (x = initial guess on entry)
int ora_solve(const ora_params* p, const cplx* U, const cplx* b, cplx* x, double tol, int maxit,
              ora_solve_info* info) {
  return solve_full(p, U, b, x, tol, maxit, info);
}

// Moebius-accelerated DWF solve (Sec. 4 algorithm, Sec. 5 defect correction).
// target: the DWF operator (Ls = L); inner: the Moebius operator (Ls = L', b', c'),
// same M5 and m.  n_dc defect-correction steps build the guess, then a
// warm-started DWF solve reaches the true residual tol.  x is overwritten.
int ora_madwf(const ora_params* pt, const ora_params* pi, const cplx* U, const cplx* b, cplx* x, int n_dc,
              double tol_pv, double tol_mob, double tol, int maxit, ora_madwf_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  Geom g = geom_of(pt);
  const int L = pt->Ls, Lp = pi->Ls;
  const long V12 = g.V * 12, n = V12 * L, np = V12 * Lp;
  ora_params pv_t = *pt;  pv_t.mass = 1.0;   // Pauli-Villars D_DW(1)
  ora_params pv_i = *pi;  pv_i.mass = 1.0;   // D'_DW(1)
  std::vector<cplx> r(n), c(n), t(n), v(n), w(n), cp(np), rhs_p(np), z(np), yp(np);
  std::memset((void*)x, 0, n * sizeof(cplx));
  ora_madwf_info loc;
  std::memset(&loc, 0, sizeof(loc));
  ora_solve_info si;
  for (int k = 0; k < n_dc; ++k) {
    // residue of the current guess (Sec. 5)
    dwf5(pt, U, x, t.data(), 0);
    for (long q = 0; q < n; ++q) r[q] = b[q] - t[q];
    // step 1: c = P^-1 D(1)^-1 r
    std::fill(t.begin(), t.end(), cplx(0));
    solve_full(&pv_t, U, r.data(), t.data(), tol_pv, maxit, &si);
    loc.pv_iters += si.iters; loc.n_pv++;
    apply_P(g, L, t.data(), c.data(), 1);
    // steps 2-3: solve D'(m) P y' = D'(1) P c',  c' = (c_1, 0, ..., 0)
    std::fill(cp.begin(), cp.end(), cplx(0));
    std::memcpy((void*)cp.data(), (const void*)c.data(), V12 * sizeof(cplx));
    apply_P(g, Lp, cp.data(), z.data(), 0);
    dwf5(&pv_i, U, z.data(), rhs_p.data(), 0);
    std::fill(z.begin(), z.end(), cplx(0));
    solve_full(pi, U, rhs_p.data(), z.data(), tol_mob, maxit, &si);
    loc.mob_iters += si.iters; loc.n_mob++;
    apply_P(g, Lp, z.data(), yp.data(), 1);   // y' = P'^-1 z ; y'_1 = slice 0
    // step 4: (-D_OV y'_1, y'_2..y'_L) = P^-1 D(1)^-1 D(m) P (-y'_1, c_2, ..., c_L)
    std::memcpy((void*)v.data(), (const void*)c.data(), n * sizeof(cplx));
    for (long q = 0; q < V12; ++q) v[q] = -yp[q];
    apply_P(g, L, v.data(), t.data(), 0);
    dwf5(pt, U, t.data(), w.data(), 0);
    std::fill(t.begin(), t.end(), cplx(0));
    solve_full(&pv_t, U, w.data(), t.data(), tol_pv, maxit, &si);
    loc.pv_iters += si.iters; loc.n_pv++;
    apply_P(g, L, t.data(), w.data(), 1);
    for (long q = 0; q < V12; ++q) w[q] = yp[q];   // replace the first slice by y'_1
    apply_P(g, L, w.data(), t.data(), 0);          // the 5D guess for this residue
    for (long q = 0; q < n; ++q) x[q] += t[q];
    dwf5(pt, U, x, t.data(), 0);
    for (long q = 0; q < n; ++q) r[q] = b[q] - t[q];
    if (k < 16) loc.resid_after_dc[k] = std::sqrt(norm2(r.data(), n) / norm2(b, n));
  }
  int st = solve_full(pt, U, b, x, tol, maxit, &si);
  loc.final_iters = si.iters;
  loc.true_rel_resid = si.true_rel_resid;
  auto t1 = std::chrono::steady_clock::now();
  loc.seconds = std::chrono::duration<double>(t1 - t0).count();
  if (info) *info = loc;
  return st;
}

// S = phi^dag (M^dag M)^-1 phi with phi on odd sites; X = (M^dag M)^-1 phi
// (X holds the initial guess on entry).  Returns S; *iters gets the CG count.
double ora_action(const ora_params* p, const cplx* U, const cplx* phi, cplx* X, double tol, int maxit,
                  int* iters) {
  Geom g = geom_of(p);
  const long n = g.V * 12 * p->Ls;
  EOContext E(p);
  cg_normal(p, E, U, phi, X, tol, maxit, iters);
  return dot(phi, X, n).real();
}

static void link_force(const Geom& g, int Ls, const cplx* U, const cplx* W, const cplx* Z, long i, int mu, cplx* Fm,
                       double* e);
static void force_fields(const ora_params* p, const cplx* U, const cplx* X, const cplx* Yin, std::vector<cplx>& W,
                         std::vector<cplx>& Z);

// The derivative of the bilinear form -2 Re <Y, M X> (X, Y on odd sites, M = M_prec of p)
// along every link and generator: e_a = d/dw [-2 Re <Y, M[exp(w T_a) U_mu(x)] X>] at w = 0
// (Sec. 2: e_a acts on the link as left multiplication by T_a).  With Y = M X this is
// e_a(S) of S = phi^dag (M^dag M)^-1 phi, X = (M^dag M)^-1 phi, since dS = -2 Re <Y, dM X>.
// Writes F_mu(x) = sum_a e_a T_a into F[mu][i][3][3]; e (optional) gets e[mu][i][a].
//   dM = -A^-1 dB_oe A^-1 B_eo - A^-1 B_oe A^-1 dB_eo
static void force_xy(const ora_params* p, const cplx* U, const cplx* X, const cplx* Yin, cplx* F, double* e_out) {
  Geom g = geom_of(p);
  const int Ls = p->Ls;
  std::vector<cplx> W, Z;
  force_fields(p, U, X, Yin, W, Z);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i)
    for (int mu = 0; mu < 4; ++mu)
      link_force(g, Ls, U, W.data(), Z.data(), i, mu, F + ((long)mu * g.V + i) * 9,
                 e_out ? e_out + ((long)mu * g.V + i) * 8 : nullptr);
}

// The fields the force contracts: W = F (X + X_e) and Z = Y_o' + Y_e' (both parities), with
// X_e = A^-1 B_eo X, Y_o' = A^-dag Y, Y_e' = A^-dag B_oe^dag Y_o'.
static void force_fields(const ora_params* p, const cplx* U, const cplx* X, const cplx* Yin, std::vector<cplx>& W,
                         std::vector<cplx>& Z) {
  Geom g = geom_of(p);
  const int Ls = p->Ls;
  const long V12 = g.V * 12, n = V12 * Ls;
  EOContext E(p);
  std::vector<cplx> Y(Yin, Yin + n), Xe(n), Yo(n), Ye(n), t(n), Xo(X, X + n);
  W.assign(n, cplx(0));
  Z.assign(n, cplx(0));
  mask_parity(g, Ls, Xo.data(), 1);
  mask_parity(g, Ls, Y.data(), 1);
  apply_B(p, g, U, Xo.data(), t.data(), 0, 0);
  apply_fifth(g, Ls, E.Ainv, t.data(), Xe.data());           // X_e = A^-1 B_eo X
  apply_fifth(g, Ls, E.Ainvdag, Y.data(), Yo.data());        // Y_o' = A^-dag Y
  apply_B(p, g, U, Yo.data(), t.data(), 1, 0);
  apply_fifth(g, Ls, E.Ainvdag, t.data(), Ye.data());        // Y_e' = A^-dag B_oe^dag Y_o'
  for (long k = 0; k < n; ++k) { t[k] = Xo[k] + Xe[k]; Z[k] = Yo[k] + Ye[k]; }
  apply_F(p, g, t.data(), W.data(), 0);                      // W = F (X + X_e)
}

// The force on one link (x = site i, direction mu) from the fields W = F (X + X_e) and
// Z = Y_o' + Y_e' of force_xy: Fm = sum_a e_a T_a, e (optional) = the eight e_a.
static void link_force(const Geom& g, int Ls, const cplx* U, const cplx* W, const cplx* Z, long i, int mu, cplx* Fm,
                       double* e) {
  const long V12 = g.V * 12;
  const Gammas& G = gam();
  const GellMann& T = gm();
  // e_a(S) = -Re sum_s [ Z(x)^dag (1-g_mu) dU W(x+mu) + Z(x+mu)^dag (1+g_mu) dU^dag W(x) ]
  // with dU = T_a U (times the boundary phase of the link), dU^dag = -U^dag T_a.
  {
    {
      double ph;
      const long f = step(g, i, mu, +1, &ph);
      const cplx* Ul = link(g, U, mu, i);
      for (int k = 0; k < 9; ++k) Fm[k] = 0;
      for (int a = 0; a < 8; ++a) {
        cplx dU[9], dUd[9];
        mat3_mul(T.T[a], Ul, dU);
        for (int k = 0; k < 9; ++k) dU[k] *= ph;
        // dU^dag = (T_a U)^dag = U^dag T_a^dag
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) dUd[r * 3 + cc] = std::conj(dU[cc * 3 + r]);
        cplx acc = 0;
        for (int s = 0; s < Ls; ++s) {
          // term 1: Z(x)^dag (1 - gamma_mu) dU W(x+mu)
          cplx v[12], pv[12];
          for (int sp = 0; sp < 4; ++sp)
            for (int r = 0; r < 3; ++r) {
              cplx q = 0;
              for (int cc = 0; cc < 3; ++cc) q += dU[r * 3 + cc] * W[s * V12 + f * 12 + sp * 3 + cc];
              v[sp * 3 + r] = q;
            }
          for (int k = 0; k < 12; ++k) pv[k] = v[k];
          spin_mul_acc(G.g[mu], v, -1.0, pv);
          for (int k = 0; k < 12; ++k) acc += std::conj(Z[s * V12 + i * 12 + k]) * pv[k];
          // term 2: Z(x+mu)^dag (1 + gamma_mu) dU^dag W(x)
          for (int sp = 0; sp < 4; ++sp)
            for (int r = 0; r < 3; ++r) {
              cplx q = 0;
              for (int cc = 0; cc < 3; ++cc) q += dUd[r * 3 + cc] * W[s * V12 + i * 12 + sp * 3 + cc];
              v[sp * 3 + r] = q;
            }
          for (int k = 0; k < 12; ++k) pv[k] = v[k];
          spin_mul_acc(G.g[mu], v, +1.0, pv);
          for (int k = 0; k < 12; ++k) acc += std::conj(Z[s * V12 + f * 12 + k]) * pv[k];
        }
        const double ea = -acc.real();
        if (e) e[a] = ea;
        for (int k = 0; k < 9; ++k) Fm[k] += ea * T.T[a][k];
      }
    }
  }
}

// Fermion force of S = phi^dag (M^dag M)^-1 phi given X = (M^dag M)^-1 phi (Y = M X).
void ora_force(const ora_params* p, const cplx* U, const cplx* X, cplx* F, double* e_out) {
  Geom g = geom_of(p);
  const long n = g.V * 12 * p->Ls;
  EOContext E(p);
  std::vector<cplx> Xo(X, X + n), Y(n);
  mask_parity(g, p->Ls, Xo.data(), 1);
  mprec(p, E, U, Xo.data(), Y.data(), 0);
  force_xy(p, U, Xo.data(), Y.data(), F, e_out);
}

// The force of ora_force evaluated only on n sampled links (lexicographic 4D site sites[k],
// direction mus[k]): F[n][3][3], e (optional) [n][8].  The same per-link definition.
void ora_force_sample(const ora_params* p, const cplx* U, const cplx* X, long n, const long* sites, const int* mus,
                      cplx* F, double* e_out) {
  Geom g = geom_of(p);
  const long nf = g.V * 12 * p->Ls;
  EOContext E(p);
  std::vector<cplx> Xo(X, X + nf), Y(nf), W, Z;
  mask_parity(g, p->Ls, Xo.data(), 1);
  mprec(p, E, U, Xo.data(), Y.data(), 0);
  force_fields(p, U, Xo.data(), Y.data(), W, Z);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k)
    link_force(g, p->Ls, U, W.data(), Z.data(), sites[k], mus[k], F + k * 9, e_out ? e_out + k * 8 : nullptr);
}

// Hasenbusch quotient action (Sec. 3): with a numerator mass pn->mass and a denominator mass
// pd->mass (same operator otherwise),
//   S = phi^dag M_n (M_d^dag M_d)^-1 M_n^dag phi,   X = (M_d^dag M_d)^-1 M_n^dag phi,
//   dS = 2 Re <phi, dM_n X> - 2 Re <Y, dM_d X>,     Y = M_d X,
// so e_a(S) = e_a[-2 Re <Y, M_d X>] - e_a[-2 Re <phi, M_n X>].  X holds the initial guess on
// entry and the solution on exit; F and e (optional) as for ora_force.  Returns S.
double ora_quotient_force(const ora_params* pn, const ora_params* pd, const cplx* U, const cplx* phi, cplx* X,
                          cplx* F, double* e_out, double tol, int maxit, int* iters) {
  Geom g = geom_of(pn);
  const int Ls = pn->Ls;
  const long n = g.V * 12 * Ls, nl = 4 * g.V;
  EOContext En(pn), Ed(pd);
  std::vector<cplx> ph(phi, phi + n), chi(n), Y(n), F2(nl * 9);
  mask_parity(g, Ls, ph.data(), 1);
  mprec(pn, En, U, ph.data(), chi.data(), 1);  // chi = M_n^dag phi
  cg_normal(pd, Ed, U, chi.data(), X, tol, maxit, iters);
  const double S = dot(chi.data(), X, n).real();
  mprec(pd, Ed, U, X, Y.data(), 0);  // Y = M_d X
  std::vector<double> e2(e_out ? nl * 8 : 0);
  force_xy(pd, U, X, Y.data(), F, e_out);
  force_xy(pn, U, X, ph.data(), F2.data(), e_out ? e2.data() : nullptr);
  for (long k = 0; k < nl * 9; ++k) F[k] -= F2[k];
  if (e_out)
    for (long k = 0; k < nl * 8; ++k) e_out[k] -= e2[k];
  return S;
}

// exp of n 3x3 complex matrices (power series)
void ora_mat3_exp(const cplx* A, cplx* out, long n) {
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) mat3_exp(A + k * 9, out + k * 9);
}

// Force-gradient step (Sec. 2, two-step list): F = e(S[U]); U' = exp(-tau^2/24 F^j T_j) U;
// then the force at U', its solve started from X(U) (force-gradient forecasting).
// Writes F' (force at U') into Fp, X' into X (X = initial guess for the first solve on
// entry), iteration counts into iters[0..1].  U is left unchanged.
void ora_fg_force(const ora_params* p, const cplx* U, const cplx* phi, double tau, cplx* X, cplx* Fp,
                  double* S_pair, double tol, int maxit, int* iters) {
  Geom g = geom_of(p);
  const long nl = 4 * g.V;
  std::vector<cplx> F(nl * 9), Up(nl * 9), Ex(nl * 9), A(nl * 9);
  S_pair[0] = ora_action(p, U, phi, X, tol, maxit, &iters[0]);
  ora_force(p, U, X, F.data(), nullptr);
  for (long k = 0; k < nl * 9; ++k) A[k] = -(tau * tau / 24.0) * F[k];
  ora_mat3_exp(A.data(), Ex.data(), nl);
  for (long l = 0; l < nl; ++l) mat3_mul(Ex.data() + l * 9, U + l * 9, Up.data() + l * 9);
  S_pair[1] = ora_action(p, Up.data(), phi, X, tol, maxit, &iters[1]);
  ora_force(p, Up.data(), X, Fp, nullptr);
}


// ---------------------------------------------------------------- gauge action, HMC (FGI)
// Wilson plaquette action S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3) with
// U_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag, periodic links (the
// antiperiodic time boundary is a fermion boundary condition only).
static void mat3_dag(const cplx* A, cplx* D) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) D[r * 3 + c] = std::conj(A[c * 3 + r]);
}

static long nb_periodic(const Geom& g, long i, int mu, int dir) {
  int c[4];
  coords_of(g, i, c);
  c[mu] = (c[mu] + dir + g.L[mu]) % g.L[mu];
  return index_of(g, c);
}

double ora_gauge_action(const ora_params* p, const cplx* U, double beta) {
  Geom g = geom_of(p);
  double sum = 0.0;
#pragma omp parallel for reduction(+ : sum) schedule(static)
  for (long i = 0; i < g.V; ++i)
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        cplx a[9], b[9], c[9], d[9], t1[9], t2[9];
        mat3_mul(link(g, U, mu, i), link(g, U, nu, nb_periodic(g, i, mu, +1)), t1);
        mat3_dag(link(g, U, mu, nb_periodic(g, i, nu, +1)), c);
        mat3_dag(link(g, U, nu, i), d);
        mat3_mul(t1, c, t2);
        mat3_mul(t2, d, a);
        (void)b;
        sum += 1.0 - (a[0] + a[4] + a[8]).real() / 3.0;
      }
  return beta * sum;
}

// Force of the plaquette action: e_a(S_g) = -(beta/3) Re tr(T_a U_mu(x) A_mu(x)) with A the
// sum of the six staples, so F_mu(x) = sum_a e_a T_a = (beta/6) TA(U_mu(x) A_mu(x)),
// TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6 (tr(T_a T_b) = -delta_ab / 2).
void ora_gauge_force(const ora_params* p, const cplx* U, double beta, cplx* F) {
  Geom g = geom_of(p);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < g.V; ++i)
    for (int mu = 0; mu < 4; ++mu) {
      cplx A[9];
      for (int k = 0; k < 9; ++k) A[k] = 0;
      for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        cplx t1[9], t2[9], x1[9], x2[9];
        // U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        mat3_dag(link(g, U, mu, nb_periodic(g, i, nu, +1)), x1);
        mat3_mul(link(g, U, nu, nb_periodic(g, i, mu, +1)), x1, t1);
        mat3_dag(link(g, U, nu, i), x2);
        mat3_mul(t1, x2, t2);
        for (int k = 0; k < 9; ++k) A[k] += t2[k];
        // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        const long xm = nb_periodic(g, i, nu, -1);
        mat3_dag(link(g, U, nu, nb_periodic(g, xm, mu, +1)), x1);
        mat3_dag(link(g, U, mu, xm), x2);
        mat3_mul(x1, x2, t1);
        mat3_mul(t1, link(g, U, nu, xm), t2);
        for (int k = 0; k < 9; ++k) A[k] += t2[k];
      }
      cplx M[9], Md[9];
      mat3_mul(link(g, U, mu, i), A, M);
      mat3_dag(M, Md);
      cplx T[9];
      for (int k = 0; k < 9; ++k) T[k] = 0.5 * (M[k] - Md[k]);
      const cplx tr = (T[0] + T[4] + T[8]) / 3.0;
      for (int d = 0; d < 3; ++d) T[d * 4] -= tr;
      cplx* Fo = F + ((long)mu * g.V + i) * 9;
      for (int k = 0; k < 9; ++k) Fo[k] = (beta / 6.0) * T[k];
    }
}

// kinetic energy of momenta P = sum_a p_a T_a: sum p_a^2 / 2 = -sum tr(P P)
static double kinetic(const Geom& g, const cplx* P) {
  double k = 0.0;
  for (long l = 0; l < 4 * g.V; ++l) {
    const cplx* m = P + l * 9;
    cplx t = 0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) t += m[r * 3 + c] * m[c * 3 + r];
    k -= t.real();
  }
  return k;
}

// U <- exp(eps A) U on every link
static void link_update(const Geom& g, const cplx* A, double eps, cplx* U) {
#pragma omp parallel for schedule(static)
  for (long l = 0; l < 4 * g.V; ++l) {
    cplx a[9], e[9], u[9];
    for (int k = 0; k < 9; ++k) a[k] = eps * A[l * 9 + k];
    mat3_exp(a, e);
    mat3_mul(e, U + l * 9, u);
    for (int k = 0; k < 9; ++k) U[l * 9 + k] = u[k];
  }
}

// force of S = S_g + phi^dag (M^dag M)^-1 phi at U; X: initial guess in, solution out.
// Returns S_f; F = F_g + F_f.
static double total_force(const ora_params* p, double beta, const cplx* U, const cplx* phi, cplx* X, cplx* F,
                          double tol, int maxit, int* iters) {
  Geom g = geom_of(p);
  const long nl = 4 * g.V;
  std::vector<cplx> Fg(nl * 9);
  int it = 0;
  const double Sf = ora_action(p, U, phi, X, tol, maxit, &it);
  *iters += it;
  ora_force(p, U, X, F, nullptr);
  ora_gauge_force(p, U, beta, Fg.data());
  for (long k = 0; k < nl * 9; ++k) F[k] += Fg[k];
  return Sf;
}

// One molecular-dynamics trajectory of the force-gradient integrator (Sec. 2), n_steps steps
// of size tau of
//   exp(tau/6 z_S) exp(tau/2 z_T) exp(2 tau/3 z_S - tau^3/72 z_{S,{S,T}}) exp(tau/2 z_T) exp(tau/6 z_S)
// for H = sum p_a^2 / 2 + S_g + phi^dag (M^dag M)^-1 phi, with z_T: U <- exp(eps P) U and
// z_S: P <- P - eps F.  The middle momentum update takes the force at
// U' = exp(-tau^2/24 F(U)) U (the two-step form of the force-gradient term), its solve
// started from X(U); every other solve starts from zero.  The force at the end of a step is
// the force at the start of the next.  U, P (natural layouts) are updated in place;
// H[0], H[1] get H at the start and at the end; *iters the CG iteration total.
void ora_fgi_trajectory(const ora_params* p, double beta, double tau, int n_steps, cplx* U, cplx* P,
                        const cplx* phi, double tol, int maxit, double* H, int* iters) {
  Geom g = geom_of(p);
  const long nl = 4 * g.V, n = g.V * 12 * p->Ls;
  std::vector<cplx> F(nl * 9), F1(nl * 9), Up(nl * 9), X(n), X1(n);
  *iters = 0;
  std::fill(X.begin(), X.end(), cplx(0));
  double Sf = total_force(p, beta, U, phi, X.data(), F.data(), tol, maxit, iters);
  H[0] = kinetic(g, P) + ora_gauge_action(p, U, beta) + Sf;
  for (int step = 0; step < n_steps; ++step) {
    for (long k = 0; k < nl * 9; ++k) P[k] -= (tau / 6.0) * F[k];
    link_update(g, P, tau / 2.0, U);
    std::fill(X1.begin(), X1.end(), cplx(0));
    total_force(p, beta, U, phi, X1.data(), F1.data(), tol, maxit, iters);
    std::copy(U, U + nl * 9, Up.begin());
    link_update(g, F1.data(), -tau * tau / 24.0, Up.data());
    total_force(p, beta, Up.data(), phi, X1.data(), F1.data(), tol, maxit, iters);
    for (long k = 0; k < nl * 9; ++k) P[k] -= (2.0 * tau / 3.0) * F1[k];
    link_update(g, P, tau / 2.0, U);
    std::fill(X.begin(), X.end(), cplx(0));
    Sf = total_force(p, beta, U, phi, X.data(), F.data(), tol, maxit, iters);
    for (long k = 0; k < nl * 9; ++k) P[k] -= (tau / 6.0) * F[k];
  }
  H[1] = kinetic(g, P) + ora_gauge_action(p, U, beta) + Sf;
}

}  // extern "C"
