"""dwf_dslash_noalloc, the variant of dwf_dslash for callers that cannot allocate device memory:
through the C ABI, every op and dagger gives what dwf_dslash gives (the same kernels: bit for
bit), FP64 also within 1e-12 of the oracle, on two calls in a row, the second on a smaller
lattice (its scratch array keeps the first call's contents); a second call allocates no device
memory; a lattice beyond the array is refused before any device work."""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_ctx, mask, rel_err

pytestmark = pytest.mark.gpu

# (dims, Ls): the second is smaller; odd extents of checkerboard sites leave a ragged last workgroup
LATTICES = [((6, 4, 6, 10), 16), ((4, 4, 2, 6), 8)]


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


def fields(dwf, ctx, dims, Ls, prec, seed):
    U = synth.random_links(dims, 0.5, seed)
    psi = synth.gaussian_spinor(dims, Ls, seed + 1)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=0.03, tbc=1)
    return lat, U, psi, lat.pack_gauge(U, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_noalloc_matches_dslash(env, ora, prec):
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    for call, (dims, Ls) in enumerate(LATTICES):
        lat, U, psi, Ug = fields(dwf, ctx, dims, Ls, P, 900 + 10 * call)
        p = lat.params(P)
        po = ora.params(dims, Ls, M5=1.8, mass=0.03, tbc=1)
        psio, psie = mask(psi, dims, 1), mask(psi, dims, 0)
        cases = []
        for dag in (False, True):
            cases += [(dwf.OP_HOP, 0, dag, psio, dwf.KIND_ODD, dwf.KIND_EVEN),
                      (dwf.OP_HOP, 1, dag, psie, dwf.KIND_EVEN, dwf.KIND_ODD),
                      (dwf.OP_MPREC, 1, dag, psio, dwf.KIND_ODD, dwf.KIND_ODD),
                      (dwf.OP_FULL, 0, dag, psi, dwf.KIND_FULL, dwf.KIND_FULL),
                      (dwf.OP_A, 1, dag, psio, dwf.KIND_ODD, dwf.KIND_ODD),
                      (dwf.OP_AINV, 1, dag, psio, dwf.KIND_ODD, dwf.KIND_ODD)]
        for op, par, dag, src_nat, kin, kout in cases:
            src = lat.pack(src_nat, kin, P)
            a, b = lat.empty(kout, P), lat.empty(kout, P)
            a.fill_(0x5A)
            b.fill_(0xA5)
            dwf.dwf_dslash(ctx, p, Ug, src, a, op, par, dag)
            dwf.dwf_dslash_noalloc(ctx, p, Ug, src, b, op, par, dag)
            got = lat.unpack_np(b, kout, P)
            assert np.array_equal(lat.unpack_np(a, kout, P), got), (call, op, par, dag)
            if prec == "fp64":
                if op == dwf.OP_HOP:
                    ref = ora.hop5(po, U, src_nat, dagger=dag, out_parity=par)
                elif op == dwf.OP_MPREC:
                    ref = ora.mprec(po, U, src_nat, dagger=dag)
                elif op == dwf.OP_FULL:
                    ref = ora.dwf(po, U, src_nat, dagger=dag)
                else:
                    which = ("A" if op == dwf.OP_A else "Ainv") + ("dag" if dag else "")
                    ref = mask(ora.fifth(po, src_nat, which), dims, 1)
                assert rel_err(got, ref) < 1e-12, (call, op, par, dag)


def test_noalloc_second_call_allocates_nothing(env):
    import torch
    dwf, ctx = env
    for call, (dims, Ls) in enumerate(LATTICES):
        lat, U, psi, Ug = fields(dwf, ctx, dims, Ls, dwf.FP32, 950 + call)
        src = lat.pack(mask(psi, dims, 1), dwf.KIND_ODD, dwf.FP32)
        dst = lat.empty(dwf.KIND_ODD, dwf.FP32)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for dag in (False, True):
            dwf.dwf_dslash_noalloc(ctx, lat.params(dwf.FP32), Ug, src, dst, dwf.OP_MPREC, 1, dag)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        if call > 0:  # (the first call may load the code object of the kernels)
            assert free1 == free0, (free0, free1)


def test_noalloc_refuses_lattices_beyond_its_scratch(env):
    dwf, ctx = env
    lat = dwf.Lattice(ctx, (4, 4, 4, 4), 8)
    buf = lat.zeros(dwf.KIND_FULL)
    # 32^3 x 64, Ls = 16, FP64: the two intermediate half fields of M_prec^dag need 6.4 GB
    big = dwf.params((32, 32, 32, 64), 16, prec=dwf.FP64)
    with pytest.raises(dwf.DwfError) as e:
        dwf.dwf_dslash_noalloc(ctx, big, buf, buf, lat.zeros(dwf.KIND_FULL), dwf.OP_MPREC, 1, True)
    assert e.value.code == dwf.DWF_ERR_ARG and "scratch" in str(e.value)
    # a fifth-dimension block at an Ls without the recurrence form
    odd_ls = dwf.params((4, 4, 4, 4), 12)
    with pytest.raises(dwf.DwfError) as e:
        dwf.dwf_dslash_noalloc(ctx, odd_ls, buf, buf, lat.zeros(dwf.KIND_FULL), dwf.OP_MPREC, 1, False)
    assert e.value.code == dwf.DWF_ERR_ARG
