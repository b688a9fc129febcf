"""The benchmark configurations that are not the headline solve, at their own size.

Solver configuration: Shamir DWF 16^3 x 32, Ls = 16, M5 = 1.8, m = 0.01, eps = 0.5 links,
Gaussian source.  FP32 iterations with FP64 reliable updates, and plain FP64, each to a
full-system true residual of 1e-10, checked on the host with the oracle's D(m).

Force configuration (Sec. 2): the same lattice, S = phi^dag (M_prec^dag M_prec)^-1 phi with a
Gaussian phi on odd sites.  At 64 seeded links (site, direction, generator):
  * the GPU force against the oracle's per-link force evaluated at the GPU's X (1e-10);
  * central differences of the GPU's FP64 action at h = 1e-4 against the GPU force;
  * the force-gradient step at tau = 0.1 (with the heatbath pseudofermion phi = M^dag eta): the
    force at U' = exp(-tau^2/24 F) U against the oracle at the GPU's X', and the second solve,
    started from X(U), needing fewer iterations than from zero.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_ctx, rel_err

pytestmark = pytest.mark.gpu

DIMS, LS = (16, 16, 16, 32), 16


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_solver_config_to_true_residual(env, ora, prec):
    dwf, ctx = env
    U = synth.random_links(DIMS, 0.5, synth.link_seed(2))
    src = synth.gaussian_spinor(DIMS, LS, synth.source_seed(2))
    lat = dwf.Lattice(ctx, DIMS, LS, M5=1.8, mass=0.01)
    Ug, bg, xg = lat.pack_gauge(U), lat.pack(src), lat.zeros(dwf.KIND_FULL)
    info = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.PREC_NAMES[prec]), Ug, bg, xg, tol=1e-10)
    print(prec, info)
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    if prec == "fp32":
        assert info["reliable_updates"] >= 1
    x = lat.unpack_np(xg)
    del xg, bg
    po = ora.params(DIMS, LS, M5=1.8, mass=0.01)
    rel = np.linalg.norm(src - ora.dwf(po, U, x)) / np.linalg.norm(src)
    print(prec, "oracle true residual", rel)
    assert rel <= 1.05e-10


# 64 seeded links: (lexicographic 4D site, direction, generator)
N_LINKS = 64


def sampled_links():
    rng = np.random.default_rng(4040)
    V = int(np.prod(DIMS))
    return rng.integers(0, V, N_LINKS), rng.integers(0, 4, N_LINKS), rng.integers(0, 8, N_LINKS)


def coords(i):
    X, Y, Z, T = DIMS
    return i // (X * Y * Z), (i // (X * Y)) % Z, (i // X) % Y, i % X  # (t, z, y, x)


@pytest.fixture(scope="module")
def force_state(env, ora):
    """The GPU's FP64 force and solution X at U (normal-equation tolerance 1e-12)."""
    import torch
    dwf, ctx = env
    U = synth.random_links(DIMS, 0.5, synth.link_seed(4))
    phi = synth.gaussian_spinor_parity(DIMS, LS, synth.source_seed(4), 1)
    lat = dwf.Lattice(ctx, DIMS, LS, M5=1.8, mass=0.01)
    Ud = lat.to_device(U)
    phig = lat.pack(phi, dwf.KIND_ODD)
    xg = lat.zeros(dwf.KIND_ODD)
    F = torch.zeros_like(Ud)
    info = dwf.fermion_force(ctx, lat.params(), Ud, phig, F, x_io=xg, tol=1e-12)
    print("force solve", info)
    assert info["converged"] and info["true_rel_resid"] <= 1e-12
    return {"lat": lat, "U": U, "phi": phi, "Ud": Ud, "phig": phig, "X": xg, "F": F.cpu().numpy(), "info": info}


def test_force_matches_oracle_at_sampled_links(env, ora, force_state):
    dwf, ctx = env
    st = force_state
    lat = st["lat"]
    X = lat.unpack_np(st["X"], dwf.KIND_ODD)
    assert abs(st["info"]["S"] - np.vdot(st["phi"], X).real) < 1e-12 * abs(st["info"]["S"])
    sites, mus, _ = sampled_links()
    po = ora.params(DIMS, LS, M5=1.8, mass=0.01)
    Fo, _ = ora.force_sample(po, st["U"], X, sites, mus)
    V = int(np.prod(DIMS))
    Fg = st["F"].reshape(4, V, 3, 3)[mus, sites]
    err = rel_err(Fg, Fo)
    print("sampled force rel err", err)
    assert err < 1e-10


def test_force_with_fp32_iterations(env, force_state):
    """The force from FP32 solver iterations (FP64 reliable updates, FP64 solution) to the same
    normal-equation tolerance: converged, and within 1e-8 of the FP64-iteration force (both solutions
    meet 1e-12, so they differ by less than the operator's condition number times that)."""
    import torch
    dwf, ctx = env
    st = force_state
    lat = st["lat"]
    F = torch.zeros_like(st["Ud"])
    info = dwf.fermion_force(ctx, lat.params(prec_inner=dwf.FP32), st["Ud"], st["phig"], F, tol=1e-12)
    print("fp32-iteration force solve", info)
    assert info["converged"] and info["reliable_updates"] >= 1
    F = F.cpu().numpy()
    err = rel_err(F, st["F"])
    print("fp32 vs fp64 iterations, force rel diff", err)
    assert err < 1e-8


def action_variational(dwf, ctx, lat, Ud, phig, x):
    """S at the links Ud from a solve warm-started at x (updated in place): the estimate
    2 Re <phi, X> - |M X|^2, whose error is quadratic in the solve's error."""
    import torch
    F = torch.empty_like(Ud)
    info = dwf.fermion_force(ctx, lat.params(), Ud, phig, F, x_io=x, tol=1e-10)
    assert info["converged"], info
    Ug = lat.pack_gauge(Ud)
    MX = lat.empty(dwf.KIND_ODD)
    dwf.dwf_dslash(ctx, lat.params(), Ug, x, MX, dwf.OP_MPREC, 1, False)
    mx = MX.view(torch.complex128)
    return 2.0 * info["S"] - float(torch.vdot(mx, mx).real), info["iters"]


@pytest.mark.parametrize("chunk", range(4))
def test_force_central_differences(env, ora, force_state, chunk):
    """(S(exp(h T_a) U) - S(exp(-h T_a) U)) / 2h at h = 1e-4 on 16 of the 64 links per chunk,
    S from the GPU's FP64 solves, against e_a = -2 tr(T_a F) of the GPU force."""
    import torch
    dwf, ctx = env
    st = force_state
    lat, U, Ud = st["lat"], st["U"], st["Ud"]
    T = ora.generators()
    sites, mus, gens = sampled_links()
    h = 1e-4
    V = int(np.prod(DIMS))
    F = st["F"].reshape(4, V, 3, 3)
    worst = 0.0
    for k in range(chunk * 16, chunk * 16 + 16):
        i, mu, a = int(sites[k]), int(mus[k]), int(gens[k])
        t, z, y, x = coords(i)
        U0 = U[mu, t, z, y, x]
        S = []
        for sg in (+1, -1):
            Ud[mu, t, z, y, x] = torch.from_numpy(ora.mat3_exp(sg * h * T[a][None])[0] @ U0).to(Ud.device)
            xw = st["X"].clone()
            S.append(action_variational(dwf, ctx, lat, Ud, st["phig"], xw)[0])
        Ud[mu, t, z, y, x] = torch.from_numpy(U0).to(Ud.device)
        fd = (S[0] - S[1]) / (2 * h)
        ea = -2.0 * np.trace(T[a] @ F[mu, i]).real
        err = abs(fd - ea) / max(abs(ea), 1e-3 * np.max(np.abs(F)))
        worst = max(worst, err)
        print(f"link {k}: site {i} mu {mu} a {a}: e_a {ea:.8e} fd {fd:.8e} rel {err:.2e}")
    assert worst < 1e-4


def test_force_gradient_step(env, ora, force_state):
    """tau = 0.1 with the pseudofermion of the molecular-dynamics heatbath, phi = M^dag eta (eta
    Gaussian): F' at U' = exp(-tau^2/24 F) U from the GPU against the oracle's per-link force at the
    GPU's X' (U' formed on the host from the GPU force at U), and the forecast: the solve at U'
    started from X(U) takes fewer iterations than the same solve started from zero."""
    import torch
    dwf, ctx = env
    st = force_state
    lat, U, Ud = st["lat"], st["U"], st["Ud"]
    tau = 0.1
    eta = lat.pack(synth.gaussian_spinor_parity(DIMS, LS, synth.source_seed(4, 1), 1), dwf.KIND_ODD)
    phi = lat.empty(dwf.KIND_ODD)
    dwf.dwf_dslash(ctx, lat.params(), lat.pack_gauge(Ud), eta, phi, dwf.OP_MPREC, 1, True)
    F1 = torch.zeros_like(Ud)
    info1 = dwf.fermion_force(ctx, lat.params(), Ud, phi, F1, tol=1e-12)
    assert info1["converged"]
    xg = lat.zeros(dwf.KIND_ODD)
    Fp = torch.zeros_like(Ud)
    info = dwf.fermion_force(ctx, lat.params(), Ud, phi, Fp, tau_fg=tau, x_io=xg, tol=1e-12)
    print("force-gradient step", info)
    assert info["converged"] and info["iters_first"] == info1["iters"]
    forecast = info["iters"] - info["iters_first"]
    V = int(np.prod(DIMS))
    F1 = F1.cpu().numpy().reshape(4 * V, 3, 3)
    Up = (ora.mat3_exp(-(tau * tau / 24.0) * F1) @ U.reshape(4 * V, 3, 3)).reshape(U.shape)
    # the same solve at U' from zero
    F0 = torch.zeros_like(Ud)
    info0 = dwf.fermion_force(ctx, lat.params(), lat.to_device(Up), phi, F0, tol=1e-12)
    print(f"iterations: at U {info['iters_first']}, at U' from zero {info0['iters']}, from X(U) {forecast}")
    assert forecast < info0["iters"]
    assert abs(info0["S"] - info["S"]) < 1e-10 * abs(info["S"])
    Xp = lat.unpack_np(xg, dwf.KIND_ODD)
    sites, mus, _ = sampled_links()
    po = ora.params(DIMS, LS, M5=1.8, mass=0.01)
    Fo, _ = ora.force_sample(po, Up, Xp, sites, mus)
    err = rel_err(Fp.cpu().numpy().reshape(4, V, 3, 3)[mus, sites], Fo)
    print("force at U' rel err", err)
    assert err < 1e-10
