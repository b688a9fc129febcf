"""FP64 CPU oracle for the domain-wall / Moebius hot path (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.cpp`` (plain C++17 +
OpenMP, complex<double>) through ctypes and shares no code with the HIP
library.  Every function takes and returns numpy complex128 arrays in the
natural layouts documented in ``oracle.cpp``:

    gauge  U[mu][t][z][y][x][3][3]      5D spinor  psi[s][t][z][y][x][4][3]

Citations refer to Yin & Mawhinney, Lattice 2011 (sections and equations).
Functions whose result has no independent pin say so in their docstring.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile oracle.cpp into liboracle.so with g++ (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("Ls", ctypes.c_int), ("tbc", ctypes.c_int),
                ("M5", ctypes.c_double), ("mass", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("bs", ctypes.c_void_p), ("cs", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


class MadwfInfo(ctypes.Structure):
    _fields_ = [("pv_iters", ctypes.c_int), ("mob_iters", ctypes.c_int), ("final_iters", ctypes.c_int),
                ("n_pv", ctypes.c_int), ("n_mob", ctypes.c_int),
                ("resid_after_dc", ctypes.c_double * 16),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        ci, cd = ctypes.c_int, ctypes.c_double
        sig = {
            "ora_gamma": ([vp], None),
            "ora_generators": ([vp], None),
            "ora_num_threads": ([], ci),
            "ora_hop4": ([P, vp, vp, vp, ci], None),
            "ora_dw4": ([P, vp, vp, vp, ci], None),
            "ora_hop5": ([P, vp, vp, vp, ci, ci], None),
            "ora_dwf": ([P, vp, vp, vp, ci], None),
            "ora_hop5_sample": ([P, vp, vp, ctypes.c_long, vp, vp, ci, vp], None),
            "ora_stilde": ([P, vp, vp, ci], None),
            "ora_fifth": ([P, vp, vp, ci], None),
            "ora_fifth_matrix": ([P, vp, ci], None),
            "ora_bhop": ([P, vp, vp, vp, ci, ci], None),
            "ora_mprec": ([P, vp, vp, vp, ci], None),
            "ora_P": ([P, vp, vp, ci], None),
            "ora_parity_mask": ([P, vp, ci], None),
            "ora_cgne": ([P, vp, vp, vp, cd, ci, ctypes.POINTER(ci)], ci),
            "ora_solve": ([P, vp, vp, vp, cd, ci, ctypes.POINTER(SolveInfo)], ci),
            "ora_madwf": ([P, P, vp, vp, vp, ci, cd, cd, cd, ci, ctypes.POINTER(MadwfInfo)], ci),
            "ora_action": ([P, vp, vp, vp, cd, ci, ctypes.POINTER(ci)], cd),
            "ora_force": ([P, vp, vp, vp, vp], None),
            "ora_force_sample": ([P, vp, vp, ctypes.c_long, vp, vp, vp, vp], None),
            "ora_gauge_action": ([P, vp, cd], cd),
            "ora_gauge_force": ([P, vp, cd, vp], None),
            "ora_fgi_trajectory": ([P, cd, cd, ci, vp, vp, vp, cd, ci, ctypes.POINTER(cd), ctypes.POINTER(ci)], None),
            "ora_quotient_force": ([P, P, vp, vp, vp, vp, vp, cd, ci, ctypes.POINTER(ci)], cd),
            "ora_mat3_exp": ([vp, vp, ctypes.c_long], None),
            "ora_fg_force": ([P, vp, vp, cd, vp, vp, vp, cd, ci, vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def params(dims, Ls, M5=1.8, mass=0.01, b=1.0, c=0.0, tbc=0, bs=None, cs=None):
    """Operator parameters: extents (X,Y,Z,T), Ls, M5, m, Moebius b and c (Shamir: 1, 0);
    bs, cs (optional, Ls entries each): s-dependent Moebius coefficients b_s, c_s."""
    p = Params()
    for k in range(4):
        p.dims[k] = int(dims[k])
    p.Ls, p.tbc = int(Ls), int(tbc)
    p.M5, p.mass, p.b, p.c = float(M5), float(mass), float(b), float(c)
    keep = []
    for name, arr in (("bs", bs), ("cs", cs)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            if a.shape != (int(Ls),):
                raise ValueError(f"{name} must hold Ls entries")
            keep.append(a)
            setattr(p, name, a.ctypes.data)
    p._keep = keep  # the arrays live as long as the parameter block
    return p


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads():
    return lib().ora_num_threads()


def gammas():
    """gamma_1..gamma_4 and gamma_5 (chiral basis), shape (5, 4, 4)."""
    out = np.zeros((5, 4, 4), np.complex128)
    lib().ora_gamma(_ptr(out))
    return out


def generators():
    """T_a = i lambda_a / 2, shape (8, 3, 3)."""
    out = np.zeros((8, 3, 3), np.complex128)
    lib().ora_generators(_ptr(out))
    return out


def hop4(p, U, psi, dagger=False):
    """4D Wilson hopping term H (or H^dag) on a 4D spinor psi[t][z][y][x][4][3]."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_hop4(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def dw4(p, U, psi, dagger=False):
    """4D Wilson operator D_W(-M5) = (4 - M5) - H/2 (or its adjoint)."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_dw4(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def hop5(p, U, psi, dagger=False, out_parity=-1):
    """Wilson hop on each s-slice of a 5D field; output restricted to a 4D parity (-1: all)."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_hop5(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger), int(out_parity))
    return out


def hop5_sample(p, U, psi, sites, svals, dagger=False):
    """Wilson hop H (or H^dag) of a natural 5D field at sampled (4D index, s) pairs: [n][4][3]."""
    U, psi = _c(U), _c(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    svals = np.ascontiguousarray(svals, dtype=np.int32)
    out = np.zeros((len(sites), 4, 3), np.complex128)
    lib().ora_hop5_sample(ctypes.byref(p), _ptr(U), _ptr(psi), len(sites), sites.ctypes.data_as(ctypes.c_void_p),
                          svals.ctypes.data_as(ctypes.c_void_p), int(dagger), _ptr(out))
    return out


def dwf(p, U, psi, dagger=False):
    """5D operator D(m) of Sec. 4 (Moebius form; Shamir DWF at b=1, c=0) or D(m)^dag."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_dwf(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def stilde(p, psi, dagger=False):
    psi = _c(psi)
    out = np.empty_like(psi)
    lib().ora_stilde(ctypes.byref(p), _ptr(psi), _ptr(out), int(dagger))
    return out


FIFTH = {"A": 0, "Adag": 1, "Ainv": 2, "Ainvdag": 3, "F": 4, "Fdag": 5}


def fifth(p, psi, which):
    """Site-local fifth-dimension operator: A, A^dag, A^-1, A^-dag, F = b + c S~, F^dag."""
    psi = _c(psi)
    out = np.empty_like(psi)
    lib().ora_fifth(ctypes.byref(p), _ptr(psi), _ptr(out), FIFTH[which])
    return out


def fifth_matrix(p, which):
    """Dense (4 Ls x 4 Ls) matrix over (s, spin) of A, A^dag, A^-1 or A^-dag."""
    n = 4 * p.Ls
    out = np.zeros((n, n), np.complex128)
    lib().ora_fifth_matrix(ctypes.byref(p), _ptr(out), FIFTH[which])
    return out


def bhop(p, U, psi, dagger=False, out_parity=-1):
    """Even-odd hopping block B = -1/2 H (b + c S~) (or its adjoint), masked to out_parity."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_bhop(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger), int(out_parity))
    return out


def mprec(p, U, psi, dagger=False):
    """Schur operator M_prec = 1 - A^-1 B_oe A^-1 B_eo on odd sites (or its adjoint)."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().ora_mprec(ctypes.byref(p), _ptr(U), _ptr(psi), _ptr(out), int(dagger))
    return out


def P(p, psi, inverse=False):
    """Domain-wall <-> overlap basis change P (Sec. 4 footnote), or P^-1."""
    psi = _c(psi)
    out = np.empty_like(psi)
    lib().ora_P(ctypes.byref(p), _ptr(psi), _ptr(out), int(inverse))
    return out


def parity_mask(p, psi, keep):
    out = _c(psi).copy()
    lib().ora_parity_mask(ctypes.byref(p), _ptr(out), int(keep))
    return out


def cgne(p, U, b_odd, x0=None, tol=1e-12, maxit=100000):
    """CGNR on M_prec: returns (x, iterations, converged)."""
    U, b_odd = _c(U), _c(b_odd)
    x = np.zeros_like(b_odd) if x0 is None else _c(x0).copy()
    it = ctypes.c_int(0)
    st = lib().ora_cgne(ctypes.byref(p), _ptr(U), _ptr(b_odd), _ptr(x), float(tol), int(maxit), ctypes.byref(it))
    return x, it.value, st == 0


def solve(p, U, b, x0=None, tol=1e-10, maxit=100000):
    """Solve D(m) x = b (Sec. 4, eq. D_DW(m) x = b) to a full-system true residual tol."""
    U, b = _c(U), _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    info = SolveInfo()
    st = lib().ora_solve(ctypes.byref(p), _ptr(U), _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(info))
    return x, {"iters": info.iters, "restarts": info.restarts, "true_rel_resid": info.true_rel_resid,
               "seconds": info.seconds, "converged": st == 0}


def madwf(pt, pi, U, b, n_dc=3, tol_pv=1e-8, tol_mob=1e-5, tol=1e-10, maxit=100000):
    """Moebius-accelerated DWF solve (Sec. 4 four-step algorithm + Sec. 5 defect correction)."""
    U, b = _c(U), _c(b)
    x = np.zeros_like(b)
    info = MadwfInfo()
    st = lib().ora_madwf(ctypes.byref(pt), ctypes.byref(pi), _ptr(U), _ptr(b), _ptr(x), int(n_dc),
                         float(tol_pv), float(tol_mob), float(tol), int(maxit), ctypes.byref(info))
    d = {k: getattr(info, k) for k in ("pv_iters", "mob_iters", "final_iters", "n_pv", "n_mob",
                                        "true_rel_resid", "seconds")}
    d["resid_after_dc"] = [info.resid_after_dc[k] for k in range(min(n_dc, 16))]
    d["converged"] = st == 0
    return x, d


def action(p, U, phi, x0=None, tol=1e-13, maxit=100000):
    """S = phi^dag (M^dag M)^-1 phi (phi on odd sites): returns (S, X, iterations)."""
    U, phi = _c(U), _c(phi)
    X = np.zeros_like(phi) if x0 is None else _c(x0).copy()
    it = ctypes.c_int(0)
    S = lib().ora_action(ctypes.byref(p), _ptr(U), _ptr(phi), _ptr(X), float(tol), int(maxit), ctypes.byref(it))
    return S, X, it.value


def force(p, U, X):
    """Force F_mu(x) = sum_a e_a(S) T_a (Sec. 2) given X = (M^dag M)^-1 phi.

    Returns (F[4][t][z][y][x][3][3], e[4][t][z][y][x][8])."""
    U, X = _c(U), _c(X)
    V = int(np.prod(p.dims))
    F = np.zeros((4, V, 3, 3), np.complex128)
    e = np.zeros((4, V, 8), np.float64)
    lib().ora_force(ctypes.byref(p), _ptr(U), _ptr(X), _ptr(F), e.ctypes.data_as(ctypes.c_void_p))
    dims_r = tuple(int(p.dims[k]) for k in (3, 2, 1, 0))
    return F.reshape((4,) + dims_r + (3, 3)), e.reshape((4,) + dims_r + (8,))


def force_sample(p, U, X, sites, mus):
    """The force of force() on sampled links (lexicographic 4D index sites[k], direction mus[k]):
    returns (F[n][3][3], e[n][8])."""
    U, X = _c(U), _c(X)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    n = len(sites)
    F = np.zeros((n, 3, 3), np.complex128)
    e = np.zeros((n, 8), np.float64)
    lib().ora_force_sample(ctypes.byref(p), _ptr(U), _ptr(X), n, sites.ctypes.data_as(ctypes.c_void_p),
                           mus.ctypes.data_as(ctypes.c_void_p), _ptr(F), e.ctypes.data_as(ctypes.c_void_p))
    return F, e


def quotient_force(pn, pd, U, phi, x0=None, tol=1e-13, maxit=100000):
    """Hasenbusch quotient action S = phi^dag M_n (M_d^dag M_d)^-1 M_n^dag phi (Sec. 3) and its
    force; pn / pd carry the numerator / denominator mass.  Returns (S, F, e, X, iters) with
    F, e shaped as in force()."""
    U, phi = _c(U), _c(phi)
    X = np.zeros_like(phi) if x0 is None else _c(x0).copy()
    V = int(np.prod(pn.dims))
    F = np.zeros((4, V, 3, 3), np.complex128)
    e = np.zeros((4, V, 8), np.float64)
    it = ctypes.c_int(0)
    S = lib().ora_quotient_force(ctypes.byref(pn), ctypes.byref(pd), _ptr(U), _ptr(phi), _ptr(X), _ptr(F),
                                 e.ctypes.data_as(ctypes.c_void_p), float(tol), int(maxit), ctypes.byref(it))
    dims_r = tuple(int(pn.dims[k]) for k in (3, 2, 1, 0))
    return S, F.reshape((4,) + dims_r + (3, 3)), e.reshape((4,) + dims_r + (8,)), X, it.value


def gauge_action(p, U, beta):
    """Wilson plaquette action beta sum (1 - Re tr U_P / 3)."""
    return lib().ora_gauge_action(ctypes.byref(p), _ptr(_c(U)), float(beta))


def gauge_force(p, U, beta):
    """F_mu(x) = sum_a e_a(S_g) T_a of the plaquette action, shaped like force()'s F."""
    U = _c(U)
    V = int(np.prod(p.dims))
    F = np.zeros((4, V, 3, 3), np.complex128)
    lib().ora_gauge_force(ctypes.byref(p), _ptr(U), float(beta), _ptr(F))
    dims_r = tuple(int(p.dims[k]) for k in (3, 2, 1, 0))
    return F.reshape((4,) + dims_r + (3, 3))


def fgi_trajectory(p, beta, tau, n_steps, U, P, phi, tol=1e-13, maxit=100000):
    """Force-gradient-integrator trajectory (Sec. 2) for S_g + phi^dag (M^dag M)^-1 phi.
    Returns (U', P', (H_start, H_end), CG iterations); U, P are not modified."""
    U1, P1, phi = _c(U).copy(), _c(P).copy(), _c(phi)
    H = (ctypes.c_double * 2)()
    it = ctypes.c_int(0)
    lib().ora_fgi_trajectory(ctypes.byref(p), float(beta), float(tau), int(n_steps), _ptr(U1), _ptr(P1), _ptr(phi),
                             float(tol), int(maxit), H, ctypes.byref(it))
    return U1, P1, (H[0], H[1]), it.value


def mat3_exp(A):
    """exp of a stack of 3x3 complex matrices by the power series."""
    A = _c(A)
    out = np.empty_like(A)
    lib().ora_mat3_exp(_ptr(A), _ptr(out), int(A.size // 9))
    return out


def fg_force(p, U, phi, tau, tol=1e-13, maxit=100000, x0=None):
    """Force-gradient step (Sec. 2): force at U' = exp(-tau^2/24 F^j T_j) U, with the
    second solve started from the first one's solution.  Returns (F', X', (S, S'), iters)."""
    U, phi = _c(U), _c(phi)
    X = np.zeros_like(phi) if x0 is None else _c(x0).copy()
    Fp = np.zeros(U.shape, np.complex128)
    S = np.zeros(2)
    iters = np.zeros(2, np.int32)
    lib().ora_fg_force(ctypes.byref(p), _ptr(U), _ptr(phi), float(tau), _ptr(X), _ptr(Fp),
                       S.ctypes.data_as(ctypes.c_void_p), float(tol), int(maxit),
                       iters.ctypes.data_as(ctypes.c_void_p))
    return Fp, X, (S[0], S[1]), (int(iters[0]), int(iters[1]))
