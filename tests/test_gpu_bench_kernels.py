"""Parity of the kernel instances the benchmark's solve runs, at the fifth-dimension extents
and launch shapes of the benchmark (Ls = 32 Shamir target, Ls' = 16 Moebius inner operator),
on lattices small enough for the oracle.

The benchmark step -- the Moebius-accelerated solve of the 24^3 x 64, Ls = 32 Shamir system with
an Ls' = 16, b = 1.5, c = 0.5 inner operator, FP16 inner, PV and final solves -- launches the
kernel instances listed in BENCH_STEP_KERNELS.  Each test here drives the library through its
C ABI with the default (benchmark) launch configuration, compares with the FP64 oracle, and
records, through the library's per-launch timer, which instances it launched; the last test
checks that the tests together launched every instance of the list.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import PREC_TOL, gpu_ctx, mask, rel_err

pytestmark = pytest.mark.gpu

# every kernel instance of one benchmark step (the template instance names the library's
# timer reports): FP16 Wilson hops of the two CG systems, FP64 hops of the reliable updates,
# source preparation, reconstruction and true residuals, and the standalone fifth-dimension
# kernel
BENCH_STEP_KERNELS = {
    "hop_kernel<dwf::P16, 32, 1, false, false, 3, false, false, false>",
    "hop_kernel<dwf::P16, 32, 1, true, false, 0, false, true, false>",
    "hop_kernel<dwf::P16, 32, 1, true, false, 2, false, false, false>",
    "hop_kernel<dwf::P16, 32, 1, false, false, 2, false, false, false>",
    "hop_kernel<dwf::P16, 16, 1, false, false, 3, false, false, false>",
    "hop_kernel<dwf::P16, 16, 1, true, false, 2, false, true, false>",
    "hop_kernel<dwf::P16, 16, 1, false, false, 2, false, false, false>",
    "hop_kernel<dwf::P16, 16, 1, true, false, 2, false, false, false>",
    "hop_kernel<dwf::P64, 32, 1, false, false, 2, true, false, false>",
    "hop_kernel<dwf::P64, 32, 1, false, false, 0, true, false, false>",
    "hop_kernel<dwf::P64, 32, 1, true, false, 0, true, false, false>",
    "fifth_kernel<dwf::P64, 32>",
    "hop_kernel<dwf::P64, 32, 1, true, false, 2, true, false, false>",
    "hop_kernel<dwf::P64, 16, 1, false, true, 2, true, false, false>",
    "hop_kernel<dwf::P64, 16, 1, true, false, 2, true, false, false>",
    "hop_kernel<dwf::P64, 16, 1, false, true, 0, true, false, false>",
    "fifth_kernel<dwf::P64, 16>",
}

LAUNCHED = {}  # kernel instance -> the tests that launched it against the oracle

DIMS = (4, 4, 4, 8)


@pytest.fixture(scope="module")
def env():
    dwf, ctx = gpu_ctx()
    dwf.dwf_timing_report(ctx)
    dwf.dwf_timing_enable(ctx, True)
    yield dwf, ctx
    dwf.dwf_timing_enable(ctx, False)


def record(dwf, ctx, name):
    for k in dwf.dwf_timing_report(ctx):
        LAUNCHED.setdefault(k, set()).add(name)


def system(dims, Ls, seed, eps=0.6):
    U = synth.random_links(dims, eps, synth.link_seed(seed))
    b = synth.gaussian_spinor(dims, Ls, synth.source_seed(seed))
    return U, b


# (Ls, b, c, mass): the target system, the inner operator, and a Shamir Ls = 16 system
SYSTEMS = [(32, 1.0, 0.0, 0.005), (16, 1.5, 0.5, 0.005), (16, 1.0, 0.0, 0.01)]


@pytest.mark.parametrize("Ls,b,c,m", SYSTEMS)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_cg_ne_at_bench_extents(env, ora, Ls, b, c, m, prec):
    """Even-odd CG-NE to a full-system true residual of 1e-10, checked with the oracle's D(m):
    the second-output hop (A^-dag q written beside q), the CG step fused into the last dagger hop
    and the deferred solution increment, at the benchmark's Ls."""
    dwf, ctx = env
    U, src = system(DIMS, Ls, 20 + Ls)
    lat = dwf.Lattice(ctx, DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(src), lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), Ug, bg, xg, tol=1e-10)
    record(dwf, ctx, f"cg Ls={Ls} b={b} {prec}")
    print(prec, Ls, b, c, info)
    assert info["converged"], info
    po = ora.params(DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    x = lat.unpack_np(xg)
    assert np.linalg.norm(src - ora.dwf(po, U, x)) <= 1.05e-10 * np.linalg.norm(src)
    if prec != "fp64":
        assert info["reliable_updates"] >= 1


@pytest.mark.parametrize("Ls,b,c,m", SYSTEMS)
@pytest.mark.parametrize("k", [3, 11])
def test_partial_cg_iterates_at_bench_extents(env, ora, Ls, b, c, m, k):
    """After exactly k FP64 iterations from zero, the iterate is the oracle's CGNR iterate after k
    iterations (to 1e-11): every step of the iteration, not only the converged answer."""
    dwf, ctx = env
    U, src = system(DIMS, Ls, 40 + Ls)
    po = ora.params(DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    xo, info_o = ora.solve(po, U, src, tol=1e-14, maxit=k)
    assert info_o["iters"] == k and not info_o["converged"]
    lat = dwf.Lattice(ctx, DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(src), lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(), Ug, bg, xg, tol=1e-14, maxit=k)
    record(dwf, ctx, f"partial cg Ls={Ls} b={b} k={k}")
    assert info["iters"] == k and not info["converged"], info
    err = rel_err(lat.unpack_np(xg), xo)
    print(Ls, b, k, err)
    assert err < 1e-11
    assert abs(info["true_rel_resid"] - info_o["true_rel_resid"]) < 1e-9 * info_o["true_rel_resid"]


# k iterations of CG with FP32/FP16/BF16 stored fields against the exact CGNR iterate: each stored
# field carries a relative rounding of the storage unit roundoff u (2^-24, 2^-11, 2^-8) per iteration,
# so the iterate stays within a modest multiple of k u of the exact one (bound 10 k u; about 1-3 u
# measured)
LOW_PREC_U = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("Ls,b,c,m", SYSTEMS)
@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_partial_cg_iterates_low_precision(env, ora, Ls, b, c, m, prec):
    """The mixed-precision CG after k = 3 iterations (where q = M_prec p is not stored: the last hop
    of M_prec^dag q rebuilds it from A^-dag q) follows the oracle's CGNR iterates to the storage
    precision; a wrong rebuild changes the direction and the iterate at O(1)."""
    dwf, ctx = env
    k = 3
    U, src = system(DIMS, Ls, 40 + Ls)
    po = ora.params(DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    xo, info_o = ora.solve(po, U, src, tol=1e-14, maxit=k)
    lat = dwf.Lattice(ctx, DIMS, Ls, M5=1.8, mass=m, b=b, c=c)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(src), lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), Ug, bg, xg, tol=1e-14, maxit=k)
    record(dwf, ctx, f"partial cg {prec} Ls={Ls} b={b}")
    assert info["iters"] == k and not info["converged"], info
    err = rel_err(lat.unpack_np(xg), xo)
    print(prec, Ls, b, err)
    assert err < 10 * k * LOW_PREC_U[prec]


@pytest.mark.parametrize("b,c,m", [(1.0, 0.0, 0.005), (1.5, 0.5, 0.005), (1.0, 0.0, 1.0)])
def test_fp64_operators_at_Ls32(env, ora, b, c, m):
    """D(m), A, A^-1, M_prec and their adjoints in FP64 at Ls = 32 (the operators of the
    benchmark's residuals, source preparation and reconstruction; m = 1 is the Pauli-Villars
    operator), 1e-12 against the oracle."""
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 6), 32
    U = synth.random_links(dims, 0.6, 61)
    psi = synth.gaussian_spinor(dims, Ls, 62)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=m, b=b, c=c)
    po = ora.params(dims, Ls, M5=1.8, mass=m, b=b, c=c)
    Ug, p = lat.pack_gauge(U), lat.params()
    full = lat.pack(psi)
    psio = mask(psi, dims, 1)
    odd = lat.pack(psio, dwf.KIND_ODD)
    for dag in (False, True):
        dst = lat.empty(dwf.KIND_FULL)
        dwf.mobius_dslash(ctx, p, Ug, full, dst, dwf.OP_FULL, 0, dag)
        assert rel_err(lat.unpack_np(dst), ora.dwf(po, U, psi, dagger=dag)) < 1e-12, ("D", dag)
        for op, which in ((dwf.OP_A, "A"), (dwf.OP_AINV, "Ainv")):
            dst = lat.empty(dwf.KIND_ODD)
            dwf.mobius_dslash(ctx, p, Ug, odd, dst, op, 1, dag)
            ref = mask(ora.fifth(po, psio, which + ("dag" if dag else "")), dims, 1)
            assert rel_err(lat.unpack_np(dst, dwf.KIND_ODD), ref) < 1e-12, (which, dag)
        dst = lat.empty(dwf.KIND_ODD)
        dwf.mobius_dslash(ctx, p, Ug, odd, dst, dwf.OP_MPREC, 1, dag)
        assert rel_err(lat.unpack_np(dst, dwf.KIND_ODD), ora.mprec(po, U, psio, dagger=dag)) < 1e-12, ("Mprec", dag)
    record(dwf, ctx, f"fp64 operators Ls=32 b={b} m={m}")


def test_madwf_at_bench_settings(env, ora):
    """The benchmark's MADWF settings -- Shamir L = 32 target, Moebius L' = 16 (b = 1.5, c = 0.5)
    inner operator, FP16 inner, PV and final solves, two defect-correction steps at tolerances
    2e-4, m = 0.005, eps = 0.6 links -- on a 4^4 lattice: the final true residual through the
    oracle's D(m), the solution against the oracle's direct solve, and the residual after each
    defect-correction step against the oracle's MADWF (FP64 inner solves) to within 1.5 decades."""
    dwf, ctx = env
    dims, L, Lp, m = (4, 4, 4, 4), 32, 16, 0.005
    U, src = system(dims, L, 3)
    lat = dwf.Lattice(ctx, dims, L, M5=1.8, mass=m)
    inner = lat.with_(Ls=Lp, b=1.5, c=0.5)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(src), lat.zeros(dwf.KIND_FULL)
    info = dwf.mobius_accel_solve(ctx, lat.params(), inner.params(prec_inner=dwf.FP16), Ug, bg, xg, n_dc=2,
                                  tol_pv=2e-4, tol_mobius=2e-4, tol=1e-10, prec_pv=dwf.FP16, prec_final=dwf.FP16)
    record(dwf, ctx, "madwf bench settings")
    print(info)
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    r = info["resid_after_dc"]
    assert len(r) == 2 and r[1] < r[0] < 1.0
    pt = ora.params(dims, L, M5=1.8, mass=m)
    x = lat.unpack_np(xg)
    assert np.linalg.norm(src - ora.dwf(pt, U, x)) <= 1.05e-10 * np.linalg.norm(src)
    xo, _ = ora.solve(pt, U, src, tol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-7 * np.linalg.norm(xo)
    pi = ora.params(dims, Lp, M5=1.8, mass=m, b=1.5, c=0.5)
    _, oinfo = ora.madwf(pt, pi, U, src, n_dc=2, tol_pv=2e-4, tol_mob=2e-4, tol=1e-10)
    print("oracle", oinfo)
    for g_r, o_r in zip(r, oinfo["resid_after_dc"]):
        assert abs(np.log10(g_r) - np.log10(o_r)) < 1.5


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_batched_ladder_at_Ls16(env, ora, prec):
    """A Hasenbusch mass ladder at Ls = 16 (the batched CG's stages in recurrence form at the
    benchmark's inner extent): every right-hand side reaches the full-system true residual of
    1e-10 against the oracle's operator."""
    dwf, ctx = env
    Ls, masses = 16, [0.005, 0.05, 0.4]
    U = synth.random_links(DIMS, 0.5, 71)
    lat = dwf.Lattice(ctx, DIMS, Ls, M5=1.8)
    Ug = lat.pack_gauge(U)
    P = dwf.PREC_NAMES[prec]
    pars, bs, xs, srcs = [], [], [], []
    for k, m in enumerate(masses):
        src = synth.gaussian_spinor(DIMS, Ls, 72 + k)
        srcs.append(src)
        pars.append(lat.params(mass=m, prec_inner=P))
        bs.append(lat.pack(src))
        xs.append(lat.zeros(dwf.KIND_FULL))
    infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-10)
    record(dwf, ctx, f"batched ladder Ls=16 {prec}")
    for k, (info, m) in enumerate(zip(infos, masses)):
        assert info["converged"], (k, info)
        po = ora.params(DIMS, Ls, M5=1.8, mass=m)
        r = srcs[k] - ora.dwf(po, U, lat.unpack_np(xs[k]))
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k]), (k, m)


def test_every_bench_kernel_was_checked():
    """Runs after the tests above (same module, file order): every kernel instance of the
    benchmark step was launched by at least one of them."""
    if not LAUNCHED:
        pytest.skip("needs the module's parity tests to run first")
    missing = sorted(BENCH_STEP_KERNELS - set(LAUNCHED))
    for k in sorted(BENCH_STEP_KERNELS):
        print(k, "<-", sorted(LAUNCHED.get(k, ())))
    assert not missing, missing
