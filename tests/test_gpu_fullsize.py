"""Parity at the benchmark's full size and launch configuration.

The 24^3 x 64, Ls = 32 half lattice of the MADWF target (eps = 0.6 links), hopped in FP64,
FP32 and FP16 with the default (benchmark) launch shape; the oracle evaluates the hop at 512
sampled output sites one by one.  The adjoint identity <x, H y> = <H^dag x, y> is checked over
the whole lattice (a property that holds at any size).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import PREC_TOL, gpu_ctx

pytestmark = pytest.mark.gpu

DIMS, LS = (24, 24, 24, 64), 32


@pytest.fixture(scope="module")
def big():
    dwf, ctx = gpu_ctx()
    U = synth.random_links(DIMS, 0.6, synth.link_seed(3))
    psi = synth.gaussian_spinor(DIMS, LS, synth.source_seed(3, 5))
    lat = dwf.Lattice(ctx, DIMS, LS, M5=1.8, mass=0.005)
    U64 = lat.pack_gauge(U)
    return dwf, ctx, lat, U, psi, U64


def sample(dims, Ls, parity, n, seed):
    rng = np.random.default_rng(seed)
    par = synth.parity_array(dims).ravel()
    cand = np.where(par == parity)[0]
    sites = rng.choice(cand, n, replace=False)
    svals = rng.integers(0, Ls, n)
    return sites, svals


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_fullsize_hop_sampled(big, ora, prec):
    import torch
    dwf, ctx, lat, U, psi, U64 = big
    P = dwf.PREC_NAMES[prec]
    Ug = U64
    if P != dwf.FP64:
        Ug = lat.empty(dwf.KIND_GAUGE, P)
        dwf.dwf_convert(ctx, lat.params(P), dwf.KIND_GAUGE, dwf.FP64, U64, P, Ug)
    src = lat.pack(psi, dwf.KIND_ODD, P)
    dst = lat.empty(dwf.KIND_EVEN, P)
    dwf.dwf_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_HOP, 0, False)
    got = lat.unpack(dst, dwf.KIND_EVEN, P)
    torch.cuda.synchronize()
    sites, svals = sample(DIMS, LS, 0, 512, 77)
    po = ora.params(DIMS, LS, M5=1.8, mass=0.005)
    psi_odd = psi.copy()
    psi_odd[:, synth.parity_array(DIMS) != 1] = 0
    ref = ora.hop5_sample(po, U, psi_odd, sites, svals)
    g = got.reshape(LS, -1, 4, 3)[torch.as_tensor(svals, device=got.device), torch.as_tensor(sites, device=got.device)]
    g = g.cpu().numpy()
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"full-size hop {prec}: sampled rel err {err:.2e}")
    assert err < PREC_TOL[prec]


def test_fullsize_adjoint_identity(big):
    """<x, H y> = <H^dag x, y> over the whole 24^3 x 64 x 32 lattice in FP64."""
    import torch
    dwf, ctx, lat, U, psi, U64 = big
    p = lat.params()
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x_e = lat.zeros(dwf.KIND_EVEN)
    y_o = lat.zeros(dwf.KIND_ODD)
    x_e.view(torch.float64).normal_(generator=g)
    y_o.view(torch.float64).normal_(generator=g)
    Hy = lat.empty(dwf.KIND_EVEN)
    Hdx = lat.empty(dwf.KIND_ODD)
    dwf.dwf_dslash(ctx, p, U64, y_o, Hy, dwf.OP_HOP, 0, False)
    dwf.dwf_dslash(ctx, p, U64, x_e, Hdx, dwf.OP_HOP, 1, True)
    a = torch.vdot(x_e.view(torch.complex128), Hy.view(torch.complex128))
    b = torch.vdot(Hdx.view(torch.complex128), y_o.view(torch.complex128))
    assert abs(complex(a - b)) < 1e-12 * abs(complex(a))
