// dwf_dslash without device allocation, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid it).
//
// Everything the operator needs beyond the caller's inputs and outputs -- the neighbour tables
// of both checkerboard parities and, for M_prec, the even-parity (and for its adjoint the
// odd-parity) intermediate half fields -- lives in one file-scope device array, `scratch`, of
// NOALLOC_SCRATCH_BYTES.  Each device holds its own copy from the library's first use until the
// process ends; its address on a device is taken once, with that device current, when a context
// is created there (dwf_ctx_create), and host code uses only that address.  The fifth-dimension
// blocks run in their recurrence (scan) form, whose coefficients travel in the kernel arguments,
// so no matrix table is needed.  Every call rebuilds the neighbour tables and writes every
// intermediate before reading it: nothing has to start at zero.  Calls that overlap on one
// device (several streams, several threads) share the array and race.
#include <mutex>
#include "runtime.hpp"

namespace dwf {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (taken once per device).
void* scratch_init() {
  int dev = 0;
  DWF_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw Error{DWF_ERR_ARG, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw Error{DWF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

static void* scratch_of(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// Neighbour x_cb of every output site of both parities, the convention of the geometry tables:
// lexicographic index i = x + X (y + Y (z + Z t)), parity (x + y + z + t) mod 2, x_cb = i / 2;
// directions 0..3 forward (x + mu), 4..7 backward (x - mu).  nbr[p][x_cb][8].
__global__ void __launch_bounds__(256) noalloc_nbr_kernel(int* nbr, int X, int Y, int Z, int T, long nsites) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * nsites) return;
  const int p = int(k / nsites);
  const long xc = k - p * nsites;
  const long i0 = 2 * xc;
  const int xh = int(i0 % X);
  long rest = i0 / X;
  const int y = int(rest % Y);
  rest /= Y;
  const int z = int(rest % Z);
  const int t = int(rest / Z);
  const int x = xh + ((y + z + t + p) & 1);
  const int c[4] = {x, y, z, t}, d[4] = {X, Y, Z, T};
  int* out = nbr + k * 8;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int f[4] = {c[0], c[1], c[2], c[3]}, b[4] = {c[0], c[1], c[2], c[3]};
    f[mu] = c[mu] + 1 == d[mu] ? 0 : c[mu] + 1;
    b[mu] = c[mu] == 0 ? d[mu] - 1 : c[mu] - 1;
    const long jf = f[0] + long(X) * (f[1] + long(Y) * (f[2] + long(Z) * f[3]));
    const long jb = b[0] + long(X) * (b[1] + long(Y) * (b[2] + long(Z) * b[3]));
    out[mu] = int(jf / 2);
    out[4 + mu] = int(jb / 2);
  }
}

static size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename P>
static int noalloc_t(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op,
                     int parity, int dagger) {
  using R = typename P::R;
  using S = typename P::S;
  const int Ls = p.Ls;
  const long V = long(p.dims[0]) * p.dims[1] * p.dims[2] * p.dims[3], ns = V / 2;
  const size_t hb = half_bytes<P>(ns, Ls);
  const size_t nbr_bytes = round256(size_t(2) * ns * 8 * sizeof(int));
  const int ntmp = op == DWF_OP_MPREC ? (dagger ? 2 : 1) : 0;
  const size_t need = nbr_bytes + ntmp * round256(hb);
  if (need > size_t(NOALLOC_SCRATCH_BYTES))
    throw Error{DWF_ERR_ARG, "lattice needs " + std::to_string(need) + " bytes of scratch; the no-allocation "
                             "entry point holds " + std::to_string(size_t(NOALLOC_SCRATCH_BYTES))};
  const bool moebius = !(p.b == 1.0 && p.c == 0.0);
  // the fifth-dimension blocks this op applies, in recurrence form
  FifthScan<R> es[E_COUNT];
  const bool needs_fifth = op == DWF_OP_MPREC || op == DWF_OP_FULL || op == DWF_OP_A || op == DWF_OP_AINV ||
                           (op == DWF_OP_HOP && dagger && moebius);
  if (needs_fifth) {
    if (!(Ls == 8 || Ls == 16 || Ls == 32))
      throw Error{DWF_ERR_ARG, "the no-allocation entry point applies the fifth-dimension blocks in recurrence "
                               "form only: Ls must be 8, 16 or 32 for this op"};
    for (int slot = 0; slot < E_COUNT; ++slot) {
      FifthScan<double> e;
      if (!fifth_scan(Ls, p.M5, p.mass, p.b, p.c, slot, &e))
        throw Error{DWF_ERR_ARG, "these M5, b, c, m admit no recurrence form of the fifth-dimension blocks"};
      es[slot].m = R(e.m);
      for (int ch = 0; ch < 2; ++ch) {
        const FifthChir<double>& q = e.ch[ch];
        es[slot].ch[ch] = FifthChir<R>{R(q.a1), R(q.b1), R(q.inv_alpha), R(q.a), R(q.corr), q.d1, q.d2, q.has_inv};
      }
    }
  }
  void* base = scratch_of(ctx->device);
  int cur = -1;
  DWF_CHECK_HIP(hipGetDevice(&cur));
  if (!base || cur != ctx->device)
    throw Error{DWF_ERR_ARG, "the context's device must be current (its scratch address is taken there)"};
  hipStream_t st = ctx->stream;
  int* nbr = reinterpret_cast<int*>(base);
  unsigned char* tmp = reinterpret_cast<unsigned char*>(base) + nbr_bytes;
  {
    const long n = 2 * ns;
    hipLaunchKernelGGL(noalloc_nbr_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nbr, p.dims[0],
                       p.dims[1], p.dims[2], p.dims[3], ns);
    DWF_CHECK_HIP(hipGetLastError());
  }
  // the launch shape of the recurrence-form hops: one slice per lane
  LaunchCfg cfg = hop_config(ctx, P::ID, Ls);
  if (cfg.ns != 1 || cfg.spb * Ls > 256 || cfg.stage) {
    cfg.ns = 1;
    cfg.spb = Ls <= 256 ? 256 / Ls : 1;
    cfg.stage = 0;
  }
  const S* links = reinterpret_cast<const S*>(U);
  auto hop = [&](int out_par, CHalf<P> src, Half<P> dst, bool dag, bool pro, double scale, int slot,
                 CHalf<P> x = {nullptr, nullptr}, double ax = 0.0) {
    HopArgs<P> a;
    a.in = src;
    a.out = dst;
    a.links = links + (out_par ? size_t(ns) * 72 : 0);
    a.nbr = nbr + (out_par ? size_t(ns) * 8 : 0);
    a.order = nullptr;
    a.nsites = ns;
    a.Ls = Ls;
    a.scale = R(scale);
    a.pb = R(p.b);
    a.pc = R(p.c);
    a.pm = R(p.mass);
    a.E = nullptr;
    if (slot >= 0) {
      a.es = es[slot];
      a.epi_scan = 1;
    }
    a.x = x;
    a.ax = R(ax);
    a.norm_partials = nullptr;
    DWF_CHECK_LAUNCH(launch_hop<P>(a, dag, pro && moebius, cfg, st));
  };
  auto fifth = [&](CHalf<P> src, Half<P> dst, int slot) {
    DWF_CHECK_LAUNCH(launch_fifth<P>(src, dst, nullptr, &es[slot], CHalf<P>{nullptr, nullptr}, R(0), ns, Ls, nullptr,
                                     st));
  };
  const CHalf<P> cin = chalf_view<P>(in, ns, Ls);
  const Half<P> hout = half_view<P>(out, ns, Ls);
  switch (op) {
    case DWF_OP_HOP:
      if (!dagger) hop(parity, cin, hout, false, true, 1.0, -1);
      else hop(parity, cin, hout, true, false, 1.0, moebius ? E_FDAG : -1);
      return DWF_OK;
    case DWF_OP_MPREC: {
      const Half<P> t1 = half_view<P>(tmp, ns, Ls), t2 = half_view<P>(tmp + round256(hb), ns, Ls);
      if (!dagger) {
        // M_prec psi = psi - 1/4 A^-1 H_oe F A^-1 H_eo F psi
        hop(0, cin, t1, false, true, 1.0, E_AINV);
        hop(1, CHalf<P>{t1.data, t1.norm}, hout, false, true, -0.25, E_AINV, cin, 1.0);
      } else {
        // M_prec^dag psi = psi - 1/4 F^dag H^dag_oe (A^-dag F^dag) H^dag_eo A^-dag psi
        fifth(cin, t2, E_AINVDAG);
        hop(0, CHalf<P>{t2.data, t2.norm}, t1, true, false, 1.0, E_AINVDAG_FDAG);
        hop(1, CHalf<P>{t1.data, t1.norm}, hout, true, false, -0.25, moebius ? E_FDAG : -1, cin, 1.0);
      }
      return DWF_OK;
    }
    case DWF_OP_FULL: {
      const char* ib = reinterpret_cast<const char*>(in);
      char* ob = reinterpret_cast<char*>(out);
      const CHalf<P> ie = chalf_view<P>(ib, ns, Ls), io = chalf_view<P>(ib + hb, ns, Ls);
      const Half<P> oe = half_view<P>(ob, ns, Ls), oo = half_view<P>(ob + hb, ns, Ls);
      fifth(ie, oe, dagger ? E_ADAG : E_A);
      fifth(io, oo, dagger ? E_ADAG : E_A);
      if (!dagger) {
        hop(0, io, oe, false, true, -0.5, -1, CHalf<P>{oe.data, oe.norm}, 1.0);
        hop(1, ie, oo, false, true, -0.5, -1, CHalf<P>{oo.data, oo.norm}, 1.0);
      } else {
        hop(0, io, oe, true, false, -0.5, moebius ? E_FDAG : -1, CHalf<P>{oe.data, oe.norm}, 1.0);
        hop(1, ie, oo, true, false, -0.5, moebius ? E_FDAG : -1, CHalf<P>{oo.data, oo.norm}, 1.0);
      }
      return DWF_OK;
    }
    case DWF_OP_A:
      fifth(cin, hout, dagger ? E_ADAG : E_A);
      return DWF_OK;
    case DWF_OP_AINV:
      fifth(cin, hout, dagger ? E_AINVDAG : E_AINV);
      return DWF_OK;
    default:
      throw Error{DWF_ERR_ARG, "unknown op"};
  }
}

int dslash_noalloc(dwf_ctx* ctx, const dwf_params& p, const void* U, const void* in, void* out, int op, int parity,
                   int dagger) {
  switch (p.prec) {
    case DWF_FP64: return noalloc_t<P64>(ctx, p, U, in, out, op, parity, dagger);
    case DWF_FP32: return noalloc_t<P32>(ctx, p, U, in, out, op, parity, dagger);
    case DWF_FP16: return noalloc_t<P16>(ctx, p, U, in, out, op, parity, dagger);
    default: return noalloc_t<PB16>(ctx, p, U, in, out, op, parity, dagger);
  }
}

}  // namespace dwf
