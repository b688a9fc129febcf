"""Force-gradient-integrator trajectory (Sec. 2) on the GPU against the oracle: same start
(U, P, phi), FP64 force solves; final links and momenta and the energies agree to the solver
tolerance.  Plus reversibility of the GPU trajectory itself."""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_ctx, rel_err

pytestmark = pytest.mark.gpu


def momenta(ora, dims, seed):
    T = ora.generators()
    V = int(np.prod(dims))
    c = synth.random_su3_algebra(4 * V, seed)
    return np.einsum("na,aij->nij", c, T).reshape((4,) + tuple(dims[::-1]) + (3, 3))


@pytest.mark.parametrize("bc,tbc", [((1.0, 0.0), 0), ((1.5, 0.5), 1)])
def test_fgi_trajectory_matches_oracle(ora, bc, tbc):
    dwf, ctx = gpu_ctx()
    dims, Ls, beta, tau, n = (4, 2, 2, 4), 4, 2.0, 0.125, 4
    po = ora.params(dims, Ls, M5=1.8, mass=0.1, b=bc[0], c=bc[1], tbc=tbc)
    U = synth.random_links(dims, 0.3, 1601)
    phi = ora.mprec(po, U, synth.gaussian_spinor_parity(dims, Ls, 1602, 1), dagger=True)
    P = momenta(ora, dims, 1603)
    Uo, Po, Ho, _ = ora.fgi_trajectory(po, beta, tau, n, U, P, phi, tol=1e-13)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.1, b=bc[0], c=bc[1], tbc=tbc)
    Ud, Pd = lat.to_device(U), lat.to_device(P)
    info = dwf.hmc_fgi_trajectory(ctx, lat.params(), Ud, Pd, lat.pack(phi, dwf.KIND_ODD), beta, tau, n, tol=1e-13)
    print(info, Ho)
    assert abs(info["H_start"] - Ho[0]) < 1e-10 * abs(Ho[0])
    assert abs(info["H_end"] - Ho[1]) < 1e-10 * abs(Ho[1])
    assert rel_err(Ud.cpu().numpy(), Uo) < 1e-10
    assert rel_err(Pd.cpu().numpy(), Po) < 1e-9
    assert info["force_evals"] == 3 * n + 1
    # force-gradient forecasting: the solves at U' start from X(U) and need fewer iterations
    assert info["fg_iters_forecast"] < info["fg_iters_first"]


def test_fgi_trajectory_reversible_on_gpu(ora):
    dwf, ctx = gpu_ctx()
    dims, Ls = (4, 4, 2, 4), 8
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05)
    po = ora.params(dims, Ls, M5=1.8, mass=0.05)
    U = synth.random_links(dims, 0.3, 1611)
    phi = ora.mprec(po, U, synth.gaussian_spinor_parity(dims, Ls, 1612, 1), dagger=True)
    P = momenta(ora, dims, 1613)
    Ud, Pd = lat.to_device(U), lat.to_device(P)
    phig = lat.pack(phi, dwf.KIND_ODD)
    i1 = dwf.hmc_fgi_trajectory(ctx, lat.params(), Ud, Pd, phig, 2.0, 0.1, 5, tol=1e-13)
    Pd.neg_()
    i2 = dwf.hmc_fgi_trajectory(ctx, lat.params(), Ud, Pd, phig, 2.0, 0.1, 5, tol=1e-13)
    assert rel_err(Ud.cpu().numpy(), U) < 1e-11
    assert rel_err(-Pd.cpu().numpy(), P) < 1e-10
    assert abs(i2["H_end"] - i1["H_start"]) < 1e-9 * abs(i1["H_start"])
