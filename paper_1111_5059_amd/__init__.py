"""MI355X (gfx950) domain-wall / Moebius hot path: Python binding of libdwf.so.

A thin ctypes layer over the C ABI declared in ``include/dwf.h``; every step
of the computation runs in the HIP kernels of the library.  PyTorch supplies
device memory and the stream; tensors are passed by ``data_ptr()``.  If the
library is not built, importing works but every call raises.

Method: Yin & Mawhinney, "Improving DWF Simulations: the Force Gradient
Integrator and the Moebius Accelerated DWF Solver", Lattice 2011 (Secs. 2, 4, 5).
"""
import ctypes

import numpy as np
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdwf.so")

DWF_OK, DWF_NOT_CONVERGED = 0, 1
DWF_ERR_ARG, DWF_ERR_HIP, DWF_ERR_NOMEM, DWF_ERR_NAN = -1, -2, -3, -4
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
KIND_GAUGE, KIND_FULL, KIND_EVEN, KIND_ODD = 0, 1, 2, 3
OP_HOP, OP_MPREC, OP_FULL, OP_A, OP_AINV = 0, 1, 2, 3, 4
OP5_HOP, OP5_SCHUR = 0, 1  # dwf_dslash_5d: K, and the even-site Schur complement S
PREC_NAMES = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}


class DwfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dwf error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("Ls", ctypes.c_int), ("tbc", ctypes.c_int),
                ("M5", ctypes.c_double), ("mass", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("prec", ctypes.c_int), ("prec_inner", ctypes.c_int),
                ("b_s", ctypes.c_void_p), ("c_s", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("delta", ctypes.c_double), ("maxit", ctypes.c_int),
                ("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("restarts", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("wilson_apps", ctypes.c_longlong), ("iters_first", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MadwfInfo(ctypes.Structure):
    _fields_ = [("n_dc", ctypes.c_int), ("tol_pv", ctypes.c_double), ("tol_mobius", ctypes.c_double),
                ("tol", ctypes.c_double), ("delta", ctypes.c_double), ("maxit", ctypes.c_int),
                ("prec_pv", ctypes.c_int), ("prec_final", ctypes.c_int),
                ("pv_iters", ctypes.c_int), ("mobius_iters", ctypes.c_int), ("final_iters", ctypes.c_int),
                ("n_pv", ctypes.c_int), ("n_mobius", ctypes.c_int),
                ("resid_after_dc", ctypes.c_double * 8), ("true_rel_resid", ctypes.c_double),
                ("seconds", ctypes.c_double), ("seconds_pv", ctypes.c_double),
                ("seconds_mobius", ctypes.c_double), ("seconds_final", ctypes.c_double),
                ("wilson_apps", ctypes.c_longlong)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "resid_after_dc"}
        d["resid_after_dc"] = [self.resid_after_dc[i] for i in range(max(0, min(self.n_dc, 8)))]
        return d


class HmcInfo(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("tau", ctypes.c_double), ("n_steps", ctypes.c_int),
                ("tol", ctypes.c_double), ("delta", ctypes.c_double), ("maxit", ctypes.c_int),
                ("H_start", ctypes.c_double), ("H_end", ctypes.c_double), ("force_evals", ctypes.c_int),
                ("cg_iters", ctypes.c_longlong), ("fg_iters_first", ctypes.c_longlong),
                ("fg_iters_forecast", ctypes.c_longlong), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# exported symbols of include/dwf.h with their ctypes signatures
_vp, _ci, _cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_PP = ctypes.POINTER(Params)
SIGNATURES = {
    "dwf_ctx_create": ([ctypes.POINTER(_vp), _vp], _ci),
    "dwf_ctx_destroy": ([_vp], _ci),
    "dwf_ctx_set_stream": ([_vp, _vp], _ci),
    "dwf_ctx_release": ([_vp], _ci),
    "dwf_last_error": ([], ctypes.c_char_p),
    "dwf_field_bytes": ([_PP, _ci, _ci], ctypes.c_size_t),
    "dwf_pack": ([_vp, _PP, _ci, _ci, _vp, _vp], _ci),
    "dwf_unpack": ([_vp, _PP, _ci, _ci, _vp, _vp], _ci),
    "dwf_convert": ([_vp, _PP, _ci, _ci, _vp, _ci, _vp], _ci),
    "dwf_dslash": ([_vp, _PP, _vp, _vp, _vp, _ci, _ci, _ci], _ci),
    "mobius_dslash": ([_vp, _PP, _vp, _vp, _vp, _ci, _ci, _ci], _ci),
    "dwf_dslash_noalloc": ([_vp, _PP, _vp, _vp, _vp, _ci, _ci, _ci], _ci),
    "cg_ne": ([_vp, _PP, _vp, _vp, _vp, ctypes.POINTER(SolveInfo)], _ci),
    "cg_ne_5d": ([_vp, _PP, _vp, _vp, _vp, ctypes.POINTER(SolveInfo)], _ci),
    "dwf_dslash_5d": ([_vp, _PP, _vp, _vp, _vp, _ci, _ci], _ci),
    "cg_ne_batched": ([_vp, _ci, _PP, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                       ctypes.POINTER(SolveInfo)], _ci),
    "mobius_accel_solve": ([_vp, _PP, _PP, _vp, _vp, _vp, ctypes.POINTER(MadwfInfo)], _ci),
    "fermion_force": ([_vp, _PP, _vp, _vp, _vp, ctypes.POINTER(_cd), _cd, _ci, _vp, ctypes.POINTER(SolveInfo)], _ci),
    "dwf_tune_set": ([_vp, _ci, _ci, _ci, _ci, _ci, _ci, _ci], _ci),
    "dwf_tune_get": ([_vp, _ci, _ci, _ci] + [ctypes.POINTER(_ci)] * 4, _ci),
    "dwf_tune_tile": ([_vp, ctypes.POINTER(_ci), _ci, ctypes.POINTER(_ci)], _ci),
    "dwf_tune_tile_get": ([_vp, ctypes.POINTER(_ci), _ci, ctypes.POINTER(_ci)], _ci),
    "quotient_force": ([_vp, _PP, _ci, ctypes.POINTER(_cd), _vp, ctypes.POINTER(_vp), _vp, ctypes.POINTER(_cd), _ci,
                        ctypes.POINTER(_vp), ctypes.POINTER(SolveInfo)], _ci),
    "hmc_fgi_trajectory": ([_vp, _PP, _vp, _vp, _vp, ctypes.POINTER(HmcInfo)], _ci),
    "dwf_timing_enable": ([_vp, _ci], _ci),
    "dwf_timing_report": ([_vp, ctypes.c_char_p, ctypes.c_size_t], _ci),
}


def lib():
    """Load libdwf.so (built by paper_1111_5059_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DwfError(DWF_ERR_ARG, f"{LIB_PATH} is not built: run python -m paper_1111_5059_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc, allow_not_converged=False):
    if rc == DWF_OK or (allow_not_converged and rc == DWF_NOT_CONVERGED):
        return rc
    msg = lib().dwf_last_error()
    raise DwfError(rc, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def params(dims, Ls, M5=1.8, mass=0.01, b=1.0, c=0.0, tbc=0, prec=FP64, prec_inner=FP64, b_s=None, c_s=None):
    """Operator parameters; b_s, c_s (optional, Ls values each): s-dependent Moebius
    coefficients (host arrays kept alive with the parameter block)."""
    p = Params()
    for k in range(4):
        p.dims[k] = int(dims[k])
    p.Ls, p.tbc = int(Ls), int(tbc)
    p.M5, p.mass, p.b, p.c = float(M5), float(mass), float(b), float(c)
    p.prec, p.prec_inner = int(prec), int(prec_inner)
    keep = []
    for name, arr in (("b_s", b_s), ("c_s", c_s)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            if a.shape != (int(Ls),):
                raise ValueError(f"{name} must hold Ls values")
            keep.append(a)
            setattr(p, name, a.ctypes.data)
    p._keep = keep
    return p


class Context:
    """Owns a dwf_ctx bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.handle = _vp()
        _check(lib().dwf_ctx_create(ctypes.byref(self.handle), _vp(stream)))

    def release(self):
        """Free the solver workspace (dwf_ctx_release); geometry and tuned shapes stay."""
        _check(lib().dwf_ctx_release(self.handle))

    def close(self):
        if self.handle:
            lib().dwf_ctx_destroy(self.handle)
            self.handle = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dwf_ctx_create(stream=None):
    return Context(stream)


def dwf_field_bytes(p, kind, prec):
    return lib().dwf_field_bytes(ctypes.byref(p), int(kind), int(prec))


def dwf_pack(ctx, p, kind, prec, natural, packed):
    _check(lib().dwf_pack(ctx.handle, ctypes.byref(p), int(kind), int(prec), _vp(_ptr(natural)), _vp(_ptr(packed))))


def dwf_unpack(ctx, p, kind, prec, packed, natural):
    _check(lib().dwf_unpack(ctx.handle, ctypes.byref(p), int(kind), int(prec), _vp(_ptr(packed)), _vp(_ptr(natural))))


def dwf_convert(ctx, p, kind, prec_in, src, prec_out, dst):
    _check(lib().dwf_convert(ctx.handle, ctypes.byref(p), int(kind), int(prec_in), _vp(_ptr(src)),
                             int(prec_out), _vp(_ptr(dst))))


def dwf_dslash(ctx, p, U, src, dst, op, parity=0, dagger=False):
    _check(lib().dwf_dslash(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(src)), _vp(_ptr(dst)),
                            int(op), int(parity), int(bool(dagger))))


def mobius_dslash(ctx, p, U, src, dst, op, parity=0, dagger=False):
    _check(lib().mobius_dslash(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(src)), _vp(_ptr(dst)),
                               int(op), int(parity), int(bool(dagger))))


def dwf_dslash_noalloc(ctx, p, U, src, dst, op, parity=0, dagger=False):
    """dwf_dslash without device allocation (the library's fixed per-device scratch array)."""
    _check(lib().dwf_dslash_noalloc(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(src)), _vp(_ptr(dst)),
                                    int(op), int(parity), int(bool(dagger))))


def cg_ne(ctx, p, U, b, x, tol=1e-10, delta=0.1, maxit=100000):
    info = SolveInfo()
    info.tol, info.delta, info.maxit = float(tol), float(delta), int(maxit)
    rc = _check(lib().cg_ne(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(b)), _vp(_ptr(x)),
                            ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["converged"] = rc == DWF_OK
    return d


def cg_ne_5d(ctx, p, U, b, x, tol=1e-10, delta=0.1, maxit=100000):
    """cg_ne on the 5D even-odd Schur complement (Shamir DWF only)."""
    info = SolveInfo()
    info.tol, info.delta, info.maxit = float(tol), float(delta), int(maxit)
    rc = _check(lib().cg_ne_5d(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(b)), _vp(_ptr(x)),
                               ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["converged"] = rc == DWF_OK
    return d


def dwf_dslash_5d(ctx, p, U, src, dst, op, dagger=False):
    _check(lib().dwf_dslash_5d(ctx.handle, ctypes.byref(p), _vp(_ptr(U)), _vp(_ptr(src)), _vp(_ptr(dst)), int(op),
                               int(bool(dagger))))


def cg_ne_batched(ctx, per_rhs, U, bs, xs, tol=1e-10, delta=0.1, maxit=100000):
    """Batched solve; U is one packed link field for all right-hand sides or a list (one per
    right-hand side, for a ragged batch of lattices)."""
    n = len(per_rhs)
    Us = list(U) if isinstance(U, (list, tuple)) else [U] * n
    P = (Params * n)(*per_rhs)
    Uv = (_vp * n)(*[_ptr(u) for u in Us])
    B = (_vp * n)(*[_ptr(b) for b in bs])
    X = (_vp * n)(*[_ptr(x) for x in xs])
    tols = list(tol) if isinstance(tol, (list, tuple)) else [tol] * n
    infos = (SolveInfo * n)()
    for k in range(n):
        infos[k].tol, infos[k].delta, infos[k].maxit = float(tols[k]), float(delta), int(maxit)
    _check(lib().cg_ne_batched(ctx.handle, n, P, Uv, B, X, infos), allow_not_converged=True)
    out = [infos[k].as_dict() for k in range(n)]
    for k, d in enumerate(out):
        d["converged"] = d["true_rel_resid"] <= tols[k]
    return out


def mobius_accel_solve(ctx, target, inner, U, b, x, n_dc=3, tol_pv=1e-8, tol_mobius=1e-5, tol=1e-10,
                       delta=0.1, maxit=100000, prec_pv=FP32, prec_final=FP32):
    """Moebius-accelerated DWF solve (Sec. 4 algorithm, Sec. 5 defect correction) of D(m) x = b
    to the full-system true residual tol.  The defaults are the conservative reading of the
    paper (three defect-correction steps, tight PV solves in FP32).  On the 24^3 x 64, Ls = 32,
    m = 0.005 benchmark the fastest settings found were n_dc = 2, tol_pv = tol_mobius = 2e-4
    with FP16 PV and final solves (bench.py uses them): 6.0 s against 15.2 s with these defaults,
    whose three steps alone reach 4e-12."""
    info = MadwfInfo()
    info.n_dc, info.tol_pv, info.tol_mobius, info.tol = int(n_dc), float(tol_pv), float(tol_mobius), float(tol)
    info.delta, info.maxit, info.prec_pv, info.prec_final = float(delta), int(maxit), int(prec_pv), int(prec_final)
    rc = _check(lib().mobius_accel_solve(ctx.handle, ctypes.byref(target), ctypes.byref(inner), _vp(_ptr(U)),
                                         _vp(_ptr(b)), _vp(_ptr(x)), ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["converged"] = rc == DWF_OK
    return d


def fermion_force(ctx, p, U_natural, phi, F, tau_fg=0.0, out_kind=0, x_io=None, tol=1e-12, delta=0.1,
                  maxit=100000):
    info = SolveInfo()
    info.tol, info.delta, info.maxit = float(tol), float(delta), int(maxit)
    S = ctypes.c_double(0.0)
    rc = _check(lib().fermion_force(ctx.handle, ctypes.byref(p), _vp(_ptr(U_natural)), _vp(_ptr(phi)), _vp(_ptr(F)),
                                    ctypes.byref(S), float(tau_fg), int(out_kind), _vp(_ptr(x_io)),
                                    ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["S"] = S.value
    d["converged"] = rc == DWF_OK
    return d


def quotient_force(ctx, p, masses, U_natural, phis, F, out_kind=0, x_io=None, tol=1e-10, delta=0.1,
                   maxit=100000):
    """Hasenbusch quotient actions of the mass ladder ``masses`` (Sec. 3) and the sum of their
    forces into F; returns a dict with the per-quotient actions "S" and the solve statistics."""
    nq = len(phis)
    if len(masses) != nq + 1:
        raise ValueError("masses must hold one more entry than phis")
    m = (_cd * (nq + 1))(*[float(v) for v in masses])
    P = (_vp * nq)(*[_ptr(t) for t in phis])
    X = (_vp * nq)(*[_ptr(t) if t is not None else None for t in x_io]) if x_io is not None else None
    S = (_cd * nq)()
    info = SolveInfo()
    info.tol, info.delta, info.maxit = float(tol), float(delta), int(maxit)
    rc = _check(lib().quotient_force(ctx.handle, ctypes.byref(p), nq, m, _vp(_ptr(U_natural)), P, _vp(_ptr(F)), S,
                                     int(out_kind), X, ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["S"] = [S[i] for i in range(nq)]
    d["converged"] = rc == DWF_OK
    return d


def hmc_fgi_trajectory(ctx, p, U_natural, P_natural, phi, beta, tau, n_steps, tol=1e-10, delta=0.1, maxit=100000):
    """One force-gradient-integrator trajectory (Sec. 2); U and P are updated in place."""
    info = HmcInfo()
    info.beta, info.tau, info.n_steps = float(beta), float(tau), int(n_steps)
    info.tol, info.delta, info.maxit = float(tol), float(delta), int(maxit)
    rc = _check(lib().hmc_fgi_trajectory(ctx.handle, ctypes.byref(p), _vp(_ptr(U_natural)), _vp(_ptr(P_natural)),
                                         _vp(_ptr(phi)), ctypes.byref(info)), allow_not_converged=True)
    d = info.as_dict()
    d["converged"] = rc == DWF_OK
    return d


def dwf_tune_set(ctx, prec, Ls, sites_per_block, s_per_thread, xcd_remap=1, link_lds=1, kernel_id=0):
    _check(lib().dwf_tune_set(ctx.handle, int(kernel_id), int(prec), int(Ls), int(sites_per_block),
                              int(s_per_thread), int(xcd_remap), int(link_lds)))


def dwf_tune_get(ctx, prec, Ls, kernel_id=0):
    v = [_ci(0) for _ in range(4)]
    _check(lib().dwf_tune_get(ctx.handle, int(kernel_id), int(prec), int(Ls), *[ctypes.byref(t) for t in v]))
    return tuple(t.value for t in v)


def dwf_tune_tile(ctx, dims, tile=(0, 0, 0), tbc=0):
    """Traversal tile (tx, ty, tz) of the hop kernels on the lattice ``dims``; (0, 0, 0)
    restores the default.  Results do not depend on it."""
    d, t = (_ci * 4)(*[int(v) for v in dims]), (_ci * 3)(*[int(v) for v in tile])
    _check(lib().dwf_tune_tile(ctx.handle, d, int(tbc), t))


def dwf_tune_tile_get(ctx, dims, tbc=0):
    d, t = (_ci * 4)(*[int(v) for v in dims]), (_ci * 3)()
    _check(lib().dwf_tune_tile_get(ctx.handle, d, int(tbc), t))
    return tuple(t)


def dwf_timing_enable(ctx, enable=True):
    _check(lib().dwf_timing_enable(ctx.handle, int(bool(enable))))


def dwf_timing_report(ctx):
    """{kernel name: {"launches", "ms", "bytes"}} for the hop / fifth-dimension launches
    since the last report (HIP events on the context stream)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().dwf_timing_report(ctx.handle, buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms, nbytes = line.split("\t")
        out[name] = {"launches": int(n), "ms": float(ms), "bytes": float(nbytes)}
    return out


from .fields import Lattice  # noqa: E402,F401
from . import autograd, autotune  # noqa: E402,F401
