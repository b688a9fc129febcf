"""The 5D even-odd (Shamir) operator and solver against the oracle.

With d0 = 5 - M5 the Shamir operator is D(m) = d0 - K, K connecting opposite 5D parities
(x + y + z + t + s) mod 2; the oracle side is that definition written with the oracle's D:
K psi = d0 psi - D psi, and the even-site Schur complement S psi_e = d0 psi_e - P_e K P_o K psi_e / d0.
Every application is compared in the four storage precisions at their tolerances; the solver
reaches the full-system true residual through the oracle's D.  Extents give a ragged last
workgroup; Ls 2, 4 and 8 run the runtime-extent kernel (one, two and four lanes per site), Ls 16, 32
and 64 the compile-time ones.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import PREC_TOL, gpu_ctx, rel_err

pytestmark = pytest.mark.gpu

CASES = [((6, 4, 6, 10), 8), ((4, 4, 2, 6), 16), ((2, 4, 2, 6), 32), ((2, 2, 2, 4), 64), ((4, 2, 2, 2), 4),
         ((2, 2, 4, 2), 2)]


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


def parity5(dims, Ls):
    """5D parity (x + y + z + t + s) mod 2, broadcastable against a natural 5D spinor"""
    p4 = synth.parity_array(dims)
    return ((np.arange(Ls)[:, None, None, None, None] + p4[None]) & 1)[..., None, None]


def K_oracle(ora, po, U, psi, d0, dagger=False):
    return d0 * psi - ora.dwf(po, U, psi, dagger=dagger)


@pytest.mark.parametrize("dims,Ls", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_hop_K(env, ora, dims, Ls, prec, dagger):
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    tbc = 1 if Ls == 16 else 0
    U = synth.random_links(dims, 0.5, 900 + Ls)
    psi = synth.gaussian_spinor(dims, Ls, 910 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.07, tbc=tbc)
    po = ora.params(dims, Ls, M5=1.8, mass=0.07, tbc=tbc)
    dst = lat.empty(dwf.KIND_FULL, P)
    dwf.dwf_dslash_5d(ctx, lat.params(P), lat.pack_gauge(U, P), lat.pack(psi, dwf.KIND_FULL, P), dst, dwf.OP5_HOP,
                      dagger)
    got = lat.unpack_np(dst, dwf.KIND_FULL, P)
    ref = K_oracle(ora, po, U, psi, 5 - 1.8, dagger)
    err = rel_err(got, ref)
    print(f"K {prec} dims={dims} Ls={Ls} dag={dagger}: rel err {err:.2e}")
    assert err < PREC_TOL[prec]


@pytest.mark.parametrize("dims,Ls", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_S(env, ora, dims, Ls, prec, dagger):
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    U = synth.random_links(dims, 0.5, 920 + Ls)
    psi = synth.gaussian_spinor(dims, Ls, 930 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.02)
    po = ora.params(dims, Ls, M5=1.8, mass=0.02)
    even = parity5(dims, Ls) == 0
    d0 = 5 - 1.8
    dst = lat.empty(dwf.KIND_FULL, P)
    dwf.dwf_dslash_5d(ctx, lat.params(P), lat.pack_gauge(U, P), lat.pack(psi, dwf.KIND_FULL, P), dst,
                      dwf.OP5_SCHUR, dagger)
    got = lat.unpack_np(dst, dwf.KIND_FULL, P)
    pe = psi * even
    t = K_oracle(ora, po, U, pe, d0, dagger) * ~even
    ref = d0 * pe - K_oracle(ora, po, U, t, d0, dagger) * even / d0
    assert np.max(np.abs(got[np.broadcast_to(~even, got.shape)])) == 0.0  # the odd part is zero
    err = rel_err(got, ref)
    print(f"S {prec} dims={dims} Ls={Ls} dag={dagger}: rel err {err:.2e}")
    assert err < PREC_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_cg_ne_5d_true_residual(env, ora, prec):
    """cg_ne_5d reaches 1e-10 through the oracle's D, in about as many iterations as cg_ne."""
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 8), 16
    U = synth.random_links(dims, 0.5, 940)
    b = synth.gaussian_spinor(dims, Ls, 941)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.01, tbc=1)
    Ug, bg = lat.pack_gauge(U), lat.pack(b)
    p = lat.params(prec_inner=dwf.PREC_NAMES[prec])
    x5 = lat.zeros(dwf.KIND_FULL)
    info5 = dwf.cg_ne_5d(ctx, p, Ug, bg, x5, tol=1e-10)
    x4 = lat.zeros(dwf.KIND_FULL)
    info4 = dwf.cg_ne(ctx, p, Ug, bg, x4, tol=1e-10)
    print(prec, "5D even-odd", info5, "4D even-odd", info4)
    assert info5["converged"] and info5["true_rel_resid"] <= 1e-10
    po = ora.params(dims, Ls, M5=1.8, mass=0.01, tbc=1)
    x = lat.unpack_np(x5)
    rel = np.linalg.norm(b - ora.dwf(po, U, x)) / np.linalg.norm(b)
    print("oracle true residual", rel)
    assert rel <= 1.05e-10
    assert rel_err(x, lat.unpack_np(x4)) < 1e-7
    assert 0.7 * info4["iters"] < info5["iters"] < 1.3 * info4["iters"]


def test_cg_ne_5d_warm_start_and_zero_source(env):
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 4), 8
    U = synth.random_links(dims, 0.4, 950)
    b = synth.gaussian_spinor(dims, Ls, 951)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.05)
    Ug, bg = lat.pack_gauge(U), lat.pack(b)
    x = lat.zeros(dwf.KIND_FULL)
    first = dwf.cg_ne_5d(ctx, lat.params(), Ug, bg, x, tol=1e-10)
    again = dwf.cg_ne_5d(ctx, lat.params(), Ug, bg, x, tol=1e-10)
    assert first["converged"] and again["converged"] and again["iters"] <= 2
    z = lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne_5d(ctx, lat.params(), Ug, lat.zeros(dwf.KIND_FULL), z, tol=1e-10)
    assert info["iters"] == 0 and int(z.max()) == 0


def test_eo5_rejects_what_it_does_not_cover(env):
    dwf, ctx = env
    dims = (4, 4, 2, 4)
    U = synth.random_links(dims, 0.4, 960)
    for Ls, b, c in [(8, 1.5, 0.5), (12, 1.0, 0.0)]:
        lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.05, b=b, c=c)
        src = lat.pack(synth.gaussian_spinor(dims, Ls, 961))
        with pytest.raises(dwf.DwfError):
            dwf.cg_ne_5d(ctx, lat.params(), lat.pack_gauge(U), src, lat.zeros(dwf.KIND_FULL), tol=1e-8)
        with pytest.raises(dwf.DwfError):
            dwf.dwf_dslash_5d(ctx, lat.params(), lat.pack_gauge(U), src, lat.empty(dwf.KIND_FULL), dwf.OP5_HOP)
