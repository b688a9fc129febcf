"""Solver, MADWF and force parity of the HIP path against the FP64 oracle.

The solution of D(m) x = b is unique (m > 0), so the HIP and oracle solutions
are compared through the true residual each reaches and their difference,
bounded by the condition number times the tolerance.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_ctx, mask, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


def cfg1():
    dims, Ls = (4, 4, 4, 4), 8
    U = synth.random_links(dims, 0.3, synth.link_seed(1))
    b = synth.gaussian_spinor(dims, Ls, synth.source_seed(1))
    return dims, Ls, U, b


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_cg_ne_cfg1(env, ora, prec):
    """4^4, Ls=8, M5=1.8, m=0.01, links exp(0.3 i H): even-odd CGNR to a true residual 1e-10."""
    dwf, ctx = env
    dims, Ls, U, b = cfg1()
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.01)
    Ug = lat.pack_gauge(U)
    bg = lat.pack(b)
    xg = lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), Ug, bg, xg, tol=1e-10)
    print(prec, info)
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    x = lat.unpack_np(xg)
    po = ora.params(dims, Ls, M5=1.8, mass=0.01)
    r = b - ora.dwf(po, U, x)
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(b)
    xo, oinfo = ora.solve(po, U, b, tol=1e-12)
    assert np.linalg.norm(x - xo) <= 1e-7 * np.linalg.norm(xo)
    if prec != "fp64":
        assert info["reliable_updates"] >= 1


def test_cg_ne_moebius_warm_start(env, ora):
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 6), 6
    U = synth.random_links(dims, 0.5, 1101)
    b = synth.gaussian_spinor(dims, Ls, 1102)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    Ug = lat.pack_gauge(U)
    po = ora.params(dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    xo, _ = ora.solve(po, U, b, tol=1e-13)
    bg = lat.pack(b)
    xg = lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.FP32), Ug, bg, xg, tol=1e-11)
    assert info["converged"]
    assert rel_err(lat.unpack_np(xg), xo) < 1e-8
    # warm start from the solution: no iterations needed
    info2 = dwf.cg_ne(ctx, lat.params(), Ug, bg, xg, tol=1e-10)
    assert info2["iters"] == 0 and info2["converged"]


def test_cg_ne_not_converged_reports(env):
    dwf, ctx = env
    dims, Ls, U, b = cfg1()
    lat = dwf.Lattice(ctx, dims, Ls)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(b), lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(), Ug, bg, xg, tol=1e-10, maxit=5)
    assert not info["converged"] and info["iters"] <= 5 and info["true_rel_resid"] > 1e-10


@pytest.mark.parametrize("k", [3, 8, 11])
def test_partial_cg_iterate_matches_oracle(env, ora, k):
    """After exactly k iterations from zero (not converged), the FP64 CG iterate -- whose increment
    the library sums eight iterations at a time from a ring of directions -- is the oracle's CGNR
    iterate after k iterations; an FP32 run (FP64 reliable updates) stays close to it."""
    dwf, ctx = env
    dims, Ls, U, b = cfg1()
    xo, info_o = ora.solve(ora.params(dims, Ls), U, b, tol=1e-14, maxit=k)
    assert info_o["iters"] == k and not info_o["converged"]
    lat = dwf.Lattice(ctx, dims, Ls)
    Ug, bg = lat.pack_gauge(U), lat.pack(b)
    for prec, tol in ((dwf.FP64, 1e-11), (dwf.FP32, 1e-4)):
        xg = lat.zeros(dwf.KIND_FULL)
        info = dwf.cg_ne(ctx, lat.params(prec_inner=prec), Ug, bg, xg, tol=1e-14, maxit=k)
        assert info["iters"] == k and not info["converged"], (prec, info)
        assert rel_err(lat.unpack_np(xg), xo) < tol, (prec, k)
        assert abs(info["true_rel_resid"] - info_o["true_rel_resid"]) < 10 * tol * info_o["true_rel_resid"]


def test_cg_ne_zero_source(env):
    dwf, ctx = env
    dims, Ls = (2, 2, 2, 2), 4
    lat = dwf.Lattice(ctx, dims, Ls)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.3, 5))
    bg = lat.zeros(dwf.KIND_FULL)
    xg = lat.pack(synth.gaussian_spinor(dims, Ls, 6))
    info = dwf.cg_ne(ctx, lat.params(), Ug, bg, xg, tol=1e-10)
    assert info["converged"] and np.all(lat.unpack_np(xg) == 0)


def test_workspace_release_keeps_results(env):
    """dwf_ctx_release frees the workspace; the next solve allocates it again and gives the same
    (bit-identical) solution in the same number of iterations."""
    import torch
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 4), 8
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.4, 9))
    bg = lat.pack(synth.gaussian_spinor(dims, Ls, 10))
    runs = []
    for _ in range(2):
        x = lat.zeros(dwf.KIND_FULL)
        info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.FP32), Ug, bg, x, tol=1e-10)
        runs.append((info["iters"], x))
        ctx.release()
    assert runs[0][0] == runs[1][0]
    assert torch.equal(runs[0][1], runs[1][1])


def test_cg_ne_nan_source_is_an_error(env):
    dwf, ctx = env
    dims, Ls = (2, 2, 2, 2), 4
    lat = dwf.Lattice(ctx, dims, Ls)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.3, 7))
    b = synth.gaussian_spinor(dims, Ls, 8)
    b[0, 0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(dwf.DwfError) as e:
        dwf.cg_ne(ctx, lat.params(), Ug, lat.pack(b), lat.zeros(dwf.KIND_FULL), tol=1e-10)
    assert e.value.code == dwf.DWF_ERR_NAN


@pytest.mark.parametrize("prec_mob", ["fp64", "fp16", "bf16"])
def test_madwf_matches_oracle(env, ora, prec_mob):
    """Sec. 4/5: MADWF (target Shamir L=8, inner Moebius L'=4, b=1.5, c=0.5) reaches the
    same 1e-10 true residual; the defect-correction residuals decrease."""
    dwf, ctx = env
    dims, L, Lp = (4, 4, 4, 4), 8, 4
    U = synth.random_links(dims, 0.3, 1201)
    b = synth.gaussian_spinor(dims, L, 1202)
    lat = dwf.Lattice(ctx, dims, L, mass=0.02)
    inner = lat.with_(Ls=Lp, b=1.5, c=0.5)
    Ug = lat.pack_gauge(U)
    bg = lat.pack(b)
    xg = lat.zeros(dwf.KIND_FULL)
    info = dwf.mobius_accel_solve(ctx, lat.params(), inner.params(prec_inner=dwf.PREC_NAMES[prec_mob]), Ug, bg, xg,
                                  n_dc=3, tol_pv=1e-10, tol_mobius=1e-6, tol=1e-10)
    print(info)
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    r = info["resid_after_dc"]
    assert r[1] < r[0] and r[2] < r[1]
    pt = ora.params(dims, L, mass=0.02)
    x = lat.unpack_np(xg)
    assert np.linalg.norm(b - ora.dwf(pt, U, x)) <= 1.05e-10 * np.linalg.norm(b)
    # the same algorithm on the oracle: residual after each defect-correction step agrees
    pi = ora.params(dims, Lp, mass=0.02, b=1.5, c=0.5)
    _, oinfo = ora.madwf(pt, pi, U, b, n_dc=3, tol_pv=1e-10, tol_mob=1e-6, tol=1e-10)
    for g_r, o_r in zip(r, oinfo["resid_after_dc"]):
        assert abs(np.log10(g_r) - np.log10(o_r)) < 0.5


@pytest.mark.parametrize("Ls", [6, 20, 32, 40])
@pytest.mark.parametrize("bc,tbc", [((1.0, 0.0), 0), ((1.5, 0.5), 1)])
def test_force_kernel_parity(env, ora, bc, tbc, Ls):
    """Force at given X (the oracle's, solved to 1e-14): GPU outer-product kernel vs the
    oracle's per-generator definition, 1e-10; also the ambient gradient kind.  Ls 6 and 20 leave
    lanes of the link's 16- and 32-lane segments idle, 32 fills a segment, 40 takes two slices per
    lane of a 64-lane segment."""
    import torch
    dwf, ctx = env
    dims = (4, 4, 2, 4)
    U = synth.random_links(dims, 0.5, 1301)
    phi = synth.gaussian_spinor_parity(dims, Ls, 1302, 1)
    po = ora.params(dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=tbc)
    S, X, _ = ora.action(po, U, phi, tol=1e-14)
    Fo, eo = ora.force(po, U, X)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=tbc)
    Ud = lat.to_device(U)
    phig = lat.pack(phi, dwf.KIND_ODD)
    xg = lat.pack(X, dwf.KIND_ODD)
    F = torch.zeros_like(Ud)
    info = dwf.fermion_force(ctx, lat.params(), Ud, phig, F, x_io=xg, tol=1e-10)
    assert info["iters"] == 0
    assert abs(info["S"] - S) < 1e-12 * abs(S)
    assert rel_err(F.cpu().numpy(), Fo) < 1e-10
    # ambient gradient: e_a = Re tr(G^dag T_a U)
    G = torch.zeros_like(Ud)
    dwf.fermion_force(ctx, lat.params(), Ud, phig, G, out_kind=1, x_io=xg, tol=1e-10)
    T = ora.generators()
    Gn = G.cpu().numpy()
    e_from_G = np.einsum("mtzyxji,ajk,mtzyxki->mtzyxa", np.conj(Gn), T, U).real
    assert rel_err(e_from_G, eo) < 1e-10


def test_force_full_pipeline_and_fg_step(env, ora):
    """cfg4-style (reduced volume): force from the GPU's own FP64 solve, and the force-gradient
    step U' = exp(-tau^2/24 F) U with the second solve started from the first (Sec. 2)."""
    import torch
    dwf, ctx = env
    dims, Ls, tau = (4, 4, 4, 4), 8, 0.1
    U = synth.random_links(dims, 0.5, 1401)
    phi = synth.gaussian_spinor_parity(dims, Ls, 1402, 1)
    po = ora.params(dims, Ls, mass=0.01)
    S, X, _ = ora.action(po, U, phi, tol=1e-14)
    Fo, _ = ora.force(po, U, X)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.01)
    Ud = lat.to_device(U)
    phig = lat.pack(phi, dwf.KIND_ODD)
    F = torch.zeros_like(Ud)
    dwf.fermion_force(ctx, lat.params(), Ud, phig, F, tol=1e-13)
    assert rel_err(F.cpu().numpy(), Fo) < 1e-9
    Fpo, Xpo, (S0, S1), iters = ora.fg_force(po, U, phi, tau, tol=1e-14)
    xg = lat.zeros(dwf.KIND_ODD)
    info = dwf.fermion_force(ctx, lat.params(), Ud, phig, F, tau_fg=tau, x_io=xg, tol=1e-13)
    assert rel_err(F.cpu().numpy(), Fpo) < 1e-9
    assert abs(info["S"] - S1) < 1e-11 * abs(S1)
    # forecasting: the second solve, started from X(U), needs fewer iterations than the first
    assert info["iters"] - info["iters_first"] < info["iters_first"]
    # U unchanged
    assert rel_err(Ud.cpu().numpy(), U) == 0.0


@pytest.mark.parametrize("prec,bc", [("fp64", (1.5, 0.5)), ("fp32", (1.0, 0.0))])
def test_quotient_force_ladder_matches_oracle(env, ora, prec, bc):
    """Hasenbusch mass ladder (Sec. 3): two quotient actions solved as one batched CG; the sum of
    their forces and each action against the oracle's quotient force."""
    import torch
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 6), 8
    masses = [0.02, 0.15, 1.0]
    U = synth.random_links(dims, 0.5, 1501)
    phis = [synth.gaussian_spinor_parity(dims, Ls, 1502 + i, 1) for i in range(2)]
    Fo = 0.0
    So = []
    for i in range(2):
        pn = ora.params(dims, Ls, mass=masses[i + 1], b=bc[0], c=bc[1], tbc=1)
        pd = ora.params(dims, Ls, mass=masses[i], b=bc[0], c=bc[1], tbc=1)
        S, F, _, _, _ = ora.quotient_force(pn, pd, U, phis[i], tol=1e-14)
        Fo = Fo + F
        So.append(S)
    lat = dwf.Lattice(ctx, dims, Ls, mass=masses[0], b=bc[0], c=bc[1], tbc=1)
    Ud = lat.to_device(U)
    phig = [lat.pack(ph, dwf.KIND_ODD) for ph in phis]
    F = torch.zeros_like(Ud)
    xs = [lat.zeros(dwf.KIND_ODD) for _ in range(2)]
    tol = 1e-12 if prec == "fp64" else 1e-10
    info = dwf.quotient_force(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), masses, Ud, phig, F, x_io=xs,
                              tol=tol)
    print(prec, bc, info)
    assert info["converged"]
    err = rel_err(F.cpu().numpy(), Fo)
    print("force rel err", err)
    assert err < (1e-9 if prec == "fp64" else 1e-7)
    for i in range(2):
        assert abs(info["S"][i] - So[i]) < 1e-9 * abs(So[i])
    # warm start from the returned solutions: (almost) no iterations
    info2 = dwf.quotient_force(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), masses, Ud, phig, F, x_io=xs,
                               tol=tol)
    assert info2["iters"] <= 2 * 2
    assert rel_err(F.cpu().numpy(), Fo) < (1e-9 if prec == "fp64" else 1e-7)


def test_quotient_force_rejects_bad_ladders(env):
    import torch
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 4), 4
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.1)
    Ud = lat.to_device(synth.random_links(dims, 0.5, 1510))
    ph = lat.pack(synth.gaussian_spinor_parity(dims, Ls, 1511, 1), dwf.KIND_ODD)
    F = torch.zeros_like(Ud)
    for masses in ([0.2, 0.1], [0.1, 0.1], [0.1]):
        with pytest.raises((dwf.DwfError, ValueError)):
            dwf.quotient_force(ctx, lat.params(), masses, Ud, [ph], F)
