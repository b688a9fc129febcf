// Context, geometry tables, workspace arena and fifth-dimension matrices.
#include "runtime.hpp"

namespace dwf {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

void* ws_get(dwf_ctx* ctx, const std::string& name, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  auto it = ctx->ws.find(name);
  if (it != ctx->ws.end() && it->second.second >= bytes) return it->second.first;
  if (it != ctx->ws.end()) {
    DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    DWF_CHECK_HIP(hipFree(it->second.first));
    ctx->ws.erase(it);
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{DWF_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed (" + name + ")"};
  }
  ctx->ws[name] = {p, bytes};
  return p;
}

double read_scalar(dwf_ctx* ctx, const double* dscalars, int slot) {
  DWF_CHECK_HIP(hipMemcpyAsync(ctx->h_scalars + slot, dscalars + slot, sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return ctx->h_scalars[slot];
}

long timer_begin(dwf_ctx* ctx, const std::string& kernel) {
  KernelTimer& t = ctx->timer;
  if (!t.on) return -1;
  auto it = t.ids.find(kernel);
  int cls;
  if (it == t.ids.end()) {
    cls = int(t.names.size());
    t.names.push_back(kernel);
    t.ids[kernel] = cls;
  } else {
    cls = it->second;
  }
  while (t.pool.size() < t.used + 2) {
    hipEvent_t e;
    DWF_CHECK_HIP(hipEventCreate(&e));
    t.pool.push_back(e);
  }
  const size_t e0 = t.used++;
  DWF_CHECK_HIP(hipEventRecord(t.pool[e0], ctx->stream));
  t.marks.push_back({cls, e0, 0, 0.0});
  return long(t.marks.size()) - 1;
}

void timer_end(dwf_ctx* ctx, long mark, double bytes) {
  KernelTimer& t = ctx->timer;
  if (mark < 0 || size_t(mark) >= t.marks.size()) return;
  const size_t e1 = t.used++;
  DWF_CHECK_HIP(hipEventRecord(t.pool[e1], ctx->stream));
  t.marks[mark].e1 = e1;
  t.marks[mark].bytes = bytes;
}

std::string timer_report(dwf_ctx* ctx) {
  KernelTimer& t = ctx->timer;
  DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<long long> n(t.names.size(), 0);
  std::vector<double> ms(t.names.size(), 0.0), bytes(t.names.size(), 0.0);
  for (const auto& m : t.marks) {
    float e = 0.f;
    DWF_CHECK_HIP(hipEventElapsedTime(&e, t.pool[m.e0], t.pool[m.e1]));
    n[m.cls] += 1;
    ms[m.cls] += e;
    bytes[m.cls] += m.bytes;
  }
  std::string out;
  char line[64];
  for (size_t c = 0; c < t.names.size(); ++c) {
    if (!n[c]) continue;
    snprintf(line, sizeof(line), "\t%lld\t%.6f\t%.6e\n", n[c], ms[c], bytes[c]);
    out += t.names[c] + line;
  }
  t.marks.clear();
  t.used = 0;
  return out;
}

void timer_release(dwf_ctx* ctx) {
  KernelTimer& t = ctx->timer;
  for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
  t.pool.clear();
  t.marks.clear();
  t.used = 0;
}

// Default traversal tile: among the tiles whose extents divide the spatial extents and whose
// t-slice holds at most 600 sites, the one with the smallest halo ratio
// (tx+2)(ty+2)(tz+2) / (tx ty tz) -- the input sites one tile column reads per site it
// writes -- ties going to the larger tz, then the larger tx.  A t-slice of a few hundred
// sites keeps the three slices that share an input spinor within one XCD's L2 at FP64 too.
void default_tile(const int dims[4], int tile[3]) {
  double best = 1e300;
  tile[0] = tile[1] = tile[2] = 1;
  for (int tz = 1; tz <= dims[2]; ++tz) {
    if (dims[2] % tz) continue;
    for (int ty = 1; ty <= dims[1]; ++ty) {
      if (dims[1] % ty) continue;
      for (int tx = 1; tx <= dims[0]; ++tx) {
        if (dims[0] % tx || long(tx) * ty * tz > 600) continue;
        const double r = double(tx + 2) * (ty + 2) * (tz + 2) / (double(tx) * ty * tz);
        const bool tie = r < best * (1 + 1e-12) && r > best * (1 - 1e-12);
        if (r < best * (1 - 1e-12) || (tie && (tz > tile[2] || (tz == tile[2] && tx > tile[0])))) {
          best = r;
          tile[0] = tx;
          tile[1] = ty;
          tile[2] = tz;
        }
      }
    }
  }
}

// Tiled traversal order of the output sites: 3D tiles of (tx, ty, tz) sites walked along t,
// tile after tile.  The 8 users of an input spinor are then processed within a few t-slices
// of one tile (its halo also by the neighbouring tiles), a window that one XCD's L2 can hold.
// Only the order in which workgroups visit sites changes; every result is the same.
void upload_order(Geometry* g) {
  const int X = g->dims[0], Y = g->dims[1], Z = g->dims[2], T = g->dims[3];
  const int tx = g->tile[0], ty = g->tile[1], tz = g->tile[2];
  const long ns = g->nsites;
  auto idx = [&](int x, int y, int z, int t) { return long(x) + X * (long(y) + Y * (long(z) + long(Z) * t)); };
  for (int p = 0; p < 2; ++p) {
    std::vector<int> order;
    order.reserve(ns);
    for (int z0 = 0; z0 < Z; z0 += tz)
      for (int y0 = 0; y0 < Y; y0 += ty)
        for (int x0 = 0; x0 < X; x0 += tx)
          for (int t = 0; t < T; ++t)
            for (int z = z0; z < z0 + tz; ++z)
              for (int y = y0; y < y0 + ty; ++y)
                for (int x = x0; x < x0 + tx; ++x)
                  if (((x + y + z + t) & 1) == p) order.push_back(int(idx(x, y, z, t) / 2));
    if ((long)order.size() != ns) throw Error{DWF_ERR_ARG, "internal: traversal order incomplete"};
    if (!g->d_order[p]) DWF_CHECK_HIP(hipMalloc(&g->d_order[p], ns * sizeof(int)));
    DWF_CHECK_HIP(hipMemcpy(g->d_order[p], order.data(), ns * sizeof(int), hipMemcpyHostToDevice));
  }
}

void set_tile(dwf_ctx* ctx, const int dims[4], int tbc, const int tile[3]) {
  Geometry* g = const_cast<Geometry*>(geometry(ctx, dims, tbc));
  int t[3];
  if (tile[0] == 0 && tile[1] == 0 && tile[2] == 0) {
    default_tile(dims, t);
  } else {
    for (int k = 0; k < 3; ++k) {
      if (tile[k] < 1 || dims[k] % tile[k] != 0) throw Error{DWF_ERR_ARG, "each tile extent must divide its lattice extent"};
      t[k] = tile[k];
    }
  }
  if (t[0] == g->tile[0] && t[1] == g->tile[1] && t[2] == g->tile[2]) return;
  DWF_CHECK_HIP(hipStreamSynchronize(ctx->stream));  // no kernel may read the old order
  for (int k = 0; k < 3; ++k) g->tile[k] = t[k];
  upload_order(g);
}

// 4D checkerboard tables.  Lexicographic index i = x + X(y + Y(z + Z t)), parity
// (x+y+z+t) mod 2, x_cb = i / 2 (X even).  For output parity p and site x_cb:
// nbr = x_cb of x +- mu (in the other parity), linksrc = code of the link the hop
// uses in that direction: 2 (mu V + i) + (1 if the hop crosses the antiperiodic T boundary).
const Geometry* geometry(dwf_ctx* ctx, const int dims[4], int tbc) {
  for (auto& g : ctx->geoms)
    if (g->dims[0] == dims[0] && g->dims[1] == dims[1] && g->dims[2] == dims[2] && g->dims[3] == dims[3] &&
        g->tbc == tbc)
      return g.get();
  auto g = std::make_unique<Geometry>();
  for (int k = 0; k < 4; ++k) g->dims[k] = dims[k];
  g->tbc = tbc;
  const int X = dims[0], Y = dims[1], Z = dims[2], T = dims[3];
  g->V = long(X) * Y * Z * T;
  g->nsites = g->V / 2;
  if (4 * g->V * 2 >= (1L << 31)) throw Error{DWF_ERR_ARG, "lattice too large for 32-bit link codes"};
  const long ns = g->nsites;
  default_tile(dims, g->tile);
  std::vector<int> site(ns), nbr(ns * 8), lsrc(ns * 8);
  auto idx = [&](int x, int y, int z, int t) { return long(x) + X * (long(y) + Y * (long(z) + long(Z) * t)); };
  for (int p = 0; p < 2; ++p) {
    for (long xc = 0; xc < ns; ++xc) {
      const long i0 = 2 * xc;
      const int xh = int(i0 % X);
      long rest = i0 / X;
      const int y = int(rest % Y);
      rest /= Y;
      const int z = int(rest % Z);
      const int t = int(rest / Z);
      const int x = xh + ((y + z + t + p) & 1);
      const long i = idx(x, y, z, t);
      site[xc] = int(i);
      const int c[4] = {x, y, z, t};
      for (int mu = 0; mu < 4; ++mu) {
        int f[4] = {c[0], c[1], c[2], c[3]}, bk[4] = {c[0], c[1], c[2], c[3]};
        f[mu] = (c[mu] + 1) % dims[mu];
        bk[mu] = (c[mu] - 1 + dims[mu]) % dims[mu];
        const long jf = idx(f[0], f[1], f[2], f[3]);
        const long jb = idx(bk[0], bk[1], bk[2], bk[3]);
        nbr[xc * 8 + mu] = int(jf / 2);
        nbr[xc * 8 + 4 + mu] = int(jb / 2);
        const int phf = (tbc && mu == 3 && c[3] == T - 1) ? 1 : 0;
        const int phb = (tbc && mu == 3 && c[3] == 0) ? 1 : 0;
        lsrc[xc * 8 + mu] = int(2 * (long(mu) * g->V + i) + phf);
        lsrc[xc * 8 + 4 + mu] = int(2 * (long(mu) * g->V + jb) + phb);
      }
    }
    DWF_CHECK_HIP(hipMalloc(&g->d_site[p], ns * sizeof(int)));
    DWF_CHECK_HIP(hipMalloc(&g->d_nbr[p], ns * 8 * sizeof(int)));
    DWF_CHECK_HIP(hipMalloc(&g->d_linksrc[p], ns * 8 * sizeof(int)));
    DWF_CHECK_HIP(hipMemcpy(g->d_site[p], site.data(), ns * sizeof(int), hipMemcpyHostToDevice));
    DWF_CHECK_HIP(hipMemcpy(g->d_nbr[p], nbr.data(), ns * 8 * sizeof(int), hipMemcpyHostToDevice));
    DWF_CHECK_HIP(hipMemcpy(g->d_linksrc[p], lsrc.data(), ns * 8 * sizeof(int), hipMemcpyHostToDevice));
  }
  upload_order(g.get());
  ctx->geoms.push_back(std::move(g));
  return ctx->geoms.back().get();
}

static LaunchCfg default_config(int prec, int Ls);

LaunchCfg hop_config(dwf_ctx* ctx, int prec, int Ls) {
  auto it = ctx->tune.find(tune_key(0, prec, Ls));
  if (it != ctx->tune.end()) return it->second;
  return default_config(prec, Ls);
}

// the batched hop (one launch over several fields): its own tuning entry, else the default shape
LaunchCfg batch_config(dwf_ctx* ctx, int prec, int Ls) {
  auto it = ctx->tune.find(tune_key(1, prec, Ls));
  if (it != ctx->tune.end()) return it->second;
  return default_config(prec, Ls);
}

LaunchCfg ilv_config(dwf_ctx* ctx, int prec, int Ls) {
  auto it = ctx->tune.find(tune_key(2, prec, Ls));
  if (it != ctx->tune.end()) return it->second;
  LaunchCfg c = default_config(prec, Ls);
  c.ns = 1;
  c.stage = 0;
  c.off = 0;
  return c;
}

static LaunchCfg default_config(int prec, int Ls) {
  LaunchCfg c;
  c.ns = 1;
  c.xcd = 1;
  // links staged in LDS, except FP16: its links are read by every lane of a site at one
  // address (a broadcast) and the two staged forms would double the LDS footprint
  c.ll = prec == DWF_FP16 ? 0 : 1;
  // neighbour spinors staged through LDS (LDS mode 2) only on request: at the 24^3 x 64 shapes
  // (Ls 16, 32) the staged FP16 hops measured 1.2-1.4x slower than the per-lane gathers
  c.stage = 0;
  int spb = 256 / Ls;
  if (spb < 1) spb = 1;
  while (spb > 1 && (spb * Ls) % 64 != 0) --spb;
  if ((spb * Ls) % 64 != 0) spb = 256 / Ls > 0 ? 256 / Ls : 1;
  // the workgroup's LDS (epilogue staging + staged links) must fit in 64 KiB
  // (FP16 links are staged in two forms: 160 elements per site)
  const size_t per_site = size_t(12) * Ls * (prec == 0 ? 16 : 8) + (prec == 2 ? 160 : 72) * (prec == 0 ? 16 : prec == 1 ? 8 : 4);
  while (spb > 1 && spb * per_site > 65536) spb /= 2;
  c.spb = spb;
  return c;
}

// Per-chirality Ls x Ls matrices of the site-local fifth-dimension operators.
// Chirality 0 (spins 0,1; P+) sees S~ as S- (psi_{s-1}, psi_{-1} = -m psi_{Ls-1});
// chirality 1 (spins 2,3; P-) sees S+ (psi_{s+1}, psi_{Ls} = -m psi_0).
// A = alpha + beta S with alpha = b d + 1, beta = c d - 1, d = 4 - M5; F = b + c S.
// A^-1 by the closed form (alpha + beta S)^-1 = sum_{k<Ls} (-z)^k S^k / (alpha (1 + m (-z)^Ls)),
// z = beta / alpha, which follows from S^Ls = -m.
static std::vector<double> shift_matrix(int Ls, double m, int ch) {
  std::vector<double> S(size_t(Ls) * Ls, 0.0);
  for (int s = 0; s < Ls; ++s) {
    if (ch == 0) {
      if (s >= 1) S[s * Ls + s - 1] = 1.0; else S[s * Ls + Ls - 1] = -m;
    } else {
      if (s + 1 < Ls) S[s * Ls + s + 1] = 1.0; else S[s * Ls + 0] = -m;
    }
  }
  return S;
}

static std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n) {
  std::vector<double> C(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double a = A[i * n + k];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
  return C;
}

static std::vector<double> transpose(const std::vector<double>& A, int n) {
  std::vector<double> T(size_t(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[j * n + i] = A[i * n + j];
  return T;
}

// The same operators in recurrence form (bidiagonal factor, then the inverse of a
// bidiagonal).  Valid when |a| = |beta/alpha| <= 1, so that the scan's powers of a stay
// bounded, and 1 + m a^Ls is not close to 0.
bool fifth_scan(int Ls, double M5, double m, double b, double c, int slot, FifthScan<double>* out) {
  const double d = 4.0 - M5, alpha = b * d + 1.0, beta = c * d - 1.0;
  if (std::fabs(alpha) < 1e-14) return false;
  const double a = -beta / alpha;
  const double den = 1.0 + m * std::pow(a, Ls);
  if (std::fabs(a) > 1.0 || std::fabs(den) < 1e-6) return false;
  FifthScan<double> e{};
  e.m = m;
  for (int ch = 0; ch < 2; ++ch) {
    FifthChir<double> q{};
    const int dS = ch == 0 ? -1 : +1;  // direction S~ takes in this chirality; the adjoint takes -dS
    q.a1 = 1.0; q.b1 = 0.0; q.d1 = dS; q.has_inv = 0; q.d2 = dS;
    q.inv_alpha = 1.0 / alpha; q.a = a; q.corr = m / den;
    switch (slot) {
      case E_A: q.a1 = alpha; q.b1 = beta; q.d1 = dS; break;
      case E_ADAG: q.a1 = alpha; q.b1 = beta; q.d1 = -dS; break;
      case E_AINV: q.has_inv = 1; q.d2 = dS; break;
      case E_AINVDAG: q.has_inv = 1; q.d2 = -dS; break;
      case E_F: q.a1 = b; q.b1 = c; q.d1 = dS; break;
      case E_FDAG: q.a1 = b; q.b1 = c; q.d1 = -dS; break;
      case E_AINVDAG_FDAG: q.a1 = b; q.b1 = c; q.d1 = -dS; q.has_inv = 1; q.d2 = -dS; break;
      case E_F_AINV: q.a1 = b; q.b1 = c; q.d1 = dS; q.has_inv = 1; q.d2 = dS; break;
      default: return false;
    }
    e.ch[ch] = q;
  }
  *out = e;
  return true;
}

// inverse of a dense n x n matrix by Gauss-Jordan elimination with partial pivoting
static std::vector<double> invert_dense(std::vector<double> M, int n) {
  std::vector<double> I(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (std::fabs(M[piv * n + c]) < 1e-300) throw Error{DWF_ERR_ARG, "singular fifth-dimension block A"};
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[c * n + k], M[piv * n + k]);
        std::swap(I[c * n + k], I[piv * n + k]);
      }
    const double inv = 1.0 / M[c * n + c];
    for (int k = 0; k < n; ++k) {
      M[c * n + k] *= inv;
      I[c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[r * n + k] -= f * M[c * n + k];
        I[r * n + k] -= f * I[c * n + k];
      }
    }
  }
  return I;
}

// Table layout: [slot][chirality][Ls][Ls] matrices, then the Moebius coefficients b_s, c_s
// (2 Ls values; the constants repeated when not s-dependent), in the storage's real type.
// With s-dependent coefficients A = diag(alpha_s) + diag(beta_s) S and F = diag(b_s) + diag(c_s) S
// (row s carries the coefficients of slice s), and A^-1 is computed numerically.
const void* fifth_matrices(dwf_ctx* ctx, int Ls, double M5, double m, double b, double c, int prec,
                           const double* bs, const double* cs) {
  std::string key;
  {
    char head[160];
    snprintf(head, sizeof(head), "%d|%.17g|%.17g|%.17g|%.17g|%d", Ls, M5, m, b, c, prec == 0 ? 0 : 1);
    key = head;
    char v[40];
    for (int s = 0; bs && s < Ls; ++s) { snprintf(v, sizeof(v), "|b%.17g", bs[s]); key += v; }
    for (int s = 0; cs && s < Ls; ++s) { snprintf(v, sizeof(v), "|c%.17g", cs[s]); key += v; }
  }
  auto it = ctx->emats.find(key);
  if (it != ctx->emats.end()) return it->second.first;
  const int n = Ls;
  const bool sdep = bs || cs;
  std::vector<double> bv(n), cv(n);
  for (int s = 0; s < n; ++s) {
    bv[s] = bs ? bs[s] : b;
    cv[s] = cs ? cs[s] : c;
  }
  const double d = 4.0 - M5, alpha = b * d + 1.0, beta = c * d - 1.0;
  if (!sdep && std::fabs(alpha) < 1e-14)
    throw Error{DWF_ERR_ARG, "b (4 - M5) + 1 = 0: A is not invertible by the closed form"};
  const double z = sdep ? 0.0 : beta / alpha;
  const double denom = sdep ? 1.0 : alpha * (1.0 + m * std::pow(-z, Ls));
  if (std::fabs(denom) < 1e-300) throw Error{DWF_ERR_ARG, "singular fifth-dimension block A"};
  std::vector<double> table(size_t(E_COUNT) * 2 * n * n + 2 * n, 0.0);
  for (int s = 0; s < n; ++s) {
    table[size_t(E_COUNT) * 2 * n * n + s] = bv[s];
    table[size_t(E_COUNT) * 2 * n * n + n + s] = cv[s];
  }
  for (int ch = 0; ch < 2; ++ch) {
    const std::vector<double> S = shift_matrix(Ls, m, ch);
    std::vector<double> I(size_t(n) * n, 0.0);
    for (int s = 0; s < n; ++s) I[s * n + s] = 1.0;
    std::vector<double> A(size_t(n) * n), F(size_t(n) * n), Ainv(size_t(n) * n, 0.0), Sk = I;
    for (int k = 0; k < n * n; ++k) {
      const int row = k / n;
      A[k] = (bv[row] * d + 1.0) * I[k] + (cv[row] * d - 1.0) * S[k];
      F[k] = bv[row] * I[k] + cv[row] * S[k];
    }
    if (sdep) {
      Ainv = invert_dense(A, n);
    } else {
      double coef = 1.0 / denom;
      for (int k = 0; k < Ls; ++k) {
        for (int q = 0; q < n * n; ++q) Ainv[q] += coef * Sk[q];
        Sk = matmul(Sk, S, n);
        coef *= -z;
      }
    }
    const std::vector<double> Adag = transpose(A, n), Ainvdag = transpose(Ainv, n), Fdag = transpose(F, n);
    const std::vector<double> AinvdagFdag = matmul(Ainvdag, Fdag, n), FAinv = matmul(F, Ainv, n);
    const std::vector<double>* mats[E_COUNT] = {&A, &Adag, &Ainv, &Ainvdag, &F, &Fdag, &AinvdagFdag, &FAinv};
    for (int e = 0; e < E_COUNT; ++e)
      std::memcpy(&table[(size_t(e) * 2 + ch) * n * n], mats[e]->data(), sizeof(double) * n * n);
  }
  void* dptr = nullptr;
  size_t bytes;
  if (prec == 0) {
    bytes = table.size() * sizeof(double);
    DWF_CHECK_HIP(hipMalloc(&dptr, bytes));
    DWF_CHECK_HIP(hipMemcpy(dptr, table.data(), bytes, hipMemcpyHostToDevice));
  } else {
    std::vector<float> tf(table.begin(), table.end());
    bytes = tf.size() * sizeof(float);
    DWF_CHECK_HIP(hipMalloc(&dptr, bytes));
    DWF_CHECK_HIP(hipMemcpy(dptr, tf.data(), bytes, hipMemcpyHostToDevice));
  }
  ctx->emats[key] = {dptr, bytes};
  return dptr;
}

}  // namespace dwf
