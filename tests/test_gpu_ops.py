"""Parity of every operator application of the HIP path against the FP64 oracle.

FP64 within 1e-12 relative (max-norm), FP32 within 1e-5 per application; FP16
(with per-site norm) and BF16 storage are gated at their format's precision
(4e-3 and 3e-2) and their error is printed.  Extents are chosen so that the
half-lattice spans several workgroups with a ragged last one.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import PREC_TOL, gpu_ctx, mask, rel_err

pytestmark = pytest.mark.gpu

# (dims, Ls): 720 and 72 checkerboard sites -> ragged last workgroup for Ls = 8, 12, 16
CASES = [((6, 4, 6, 10), 8), ((6, 2, 2, 6), 12), ((4, 4, 4, 4), 16), ((2, 2, 2, 2), 4)]


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


def make(dims, Ls, seed, eps=0.5):
    U = synth.random_links(dims, eps, seed)
    psi = synth.gaussian_spinor(dims, Ls, seed + 1)
    return U, psi


@pytest.mark.parametrize("dims,Ls", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_hop_parity(env, ora, dims, Ls, prec, dagger):
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    tbc = 1 if Ls == 12 else 0
    U, psi = make(dims, Ls, 300 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, tbc=tbc)
    Ug = lat.pack_gauge(U, P)
    p = lat.params(P)
    po = ora.params(dims, Ls, tbc=tbc)
    for out_par in (0, 1):
        kin = dwf.KIND_ODD if out_par == 0 else dwf.KIND_EVEN
        kout = dwf.KIND_EVEN if out_par == 0 else dwf.KIND_ODD
        src = lat.pack(psi, kin, P)
        dst = lat.empty(kout, P)
        dwf.dwf_dslash(ctx, p, Ug, src, dst, dwf.OP_HOP, out_par, dagger)
        got = lat.unpack_np(dst, kout, P)
        ref = ora.hop5(po, U, mask(psi, dims, 1 - out_par), dagger=dagger, out_parity=out_par)
        err = rel_err(got, ref)
        print(f"hop {prec} dims={dims} Ls={Ls} dag={dagger} par={out_par}: rel err {err:.2e}")
        assert err < PREC_TOL[prec]


@pytest.mark.parametrize("dims,Ls", CASES[:3])
@pytest.mark.parametrize("bc", [(1.0, 0.0), (1.5, 0.5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_mprec_parity(env, ora, dims, Ls, bc, prec):
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    U, psi = make(dims, Ls, 400 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=1)
    Ug = lat.pack_gauge(U, P)
    p = lat.params(P)
    po = ora.params(dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=1)
    psio = mask(psi, dims, 1)
    src = lat.pack(psio, dwf.KIND_ODD, P)
    for dagger in (False, True):
        dst = lat.empty(dwf.KIND_ODD, P)
        dwf.mobius_dslash(ctx, p, Ug, src, dst, dwf.OP_MPREC, 1, dagger)
        got = lat.unpack_np(dst, dwf.KIND_ODD, P)
        ref = ora.mprec(po, U, psio, dagger=dagger)
        err = rel_err(got, ref)
        print(f"mprec {prec} bc={bc} dims={dims} Ls={Ls} dag={dagger}: rel err {err:.2e}")
        assert err < PREC_TOL[prec]


@pytest.mark.parametrize("dims,Ls", CASES)
@pytest.mark.parametrize("bc", [(1.0, 0.0), (1.5, 0.5)])
def test_full_operator_parity(env, ora, dims, Ls, bc):
    dwf, ctx = env
    U, psi = make(dims, Ls, 500 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.02, b=bc[0], c=bc[1])
    Ug = lat.pack_gauge(U)
    p = lat.params()
    po = ora.params(dims, Ls, mass=0.02, b=bc[0], c=bc[1])
    src = lat.pack(psi)
    for dagger in (False, True):
        dst = lat.empty(dwf.KIND_FULL)
        dwf.mobius_dslash(ctx, p, Ug, src, dst, dwf.OP_FULL, 0, dagger)
        got = lat.unpack_np(dst)
        ref = ora.dwf(po, U, psi, dagger=dagger)
        err = rel_err(got, ref)
        print(f"D bc={bc} dims={dims} Ls={Ls} dag={dagger}: rel err {err:.2e}")
        assert err < 1e-12


@pytest.mark.parametrize("Ls,bc,m", [(8, (1.0, 0.0), 0.01), (16, (1.5, 0.5), 0.005), (12, (2.0, 1.0), 1.0)])
def test_fifth_blocks_parity(env, ora, Ls, bc, m):
    dwf, ctx = env
    dims = (4, 4, 2, 2)
    psi = synth.gaussian_spinor(dims, Ls, 600 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, mass=m, b=bc[0], c=bc[1])
    U = synth.random_links(dims, 0.5, 601)
    Ug = lat.pack_gauge(U)
    p = lat.params()
    po = ora.params(dims, Ls, mass=m, b=bc[0], c=bc[1])
    psie = mask(psi, dims, 0)
    src = lat.pack(psie, dwf.KIND_EVEN)
    for op, which in ((dwf.OP_A, "A"), (dwf.OP_AINV, "Ainv")):
        for dagger in (False, True):
            dst = lat.empty(dwf.KIND_EVEN)
            dwf.mobius_dslash(ctx, p, Ug, src, dst, op, 0, dagger)
            got = lat.unpack_np(dst, dwf.KIND_EVEN)
            ref = mask(ora.fifth(po, psie, which + ("dag" if dagger else "")), dims, 0)
            assert rel_err(got, ref) < 1e-13


def test_moebius_hop_includes_input_factor(env, ora):
    """mobius_dslash HOP applies H (b + c S~) (and its adjoint F^dag H^dag)."""
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 6), 8
    U, psi = make(dims, Ls, 700)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.1, b=1.5, c=0.5)
    Ug = lat.pack_gauge(U)
    p = lat.params()
    po = ora.params(dims, Ls, mass=0.1, b=1.5, c=0.5)
    psio = mask(psi, dims, 1)
    src = lat.pack(psio, dwf.KIND_ODD)
    dst = lat.empty(dwf.KIND_EVEN)
    dwf.mobius_dslash(ctx, p, Ug, src, dst, dwf.OP_HOP, 0, False)
    ref = ora.hop5(po, U, ora.fifth(po, psio, "F"), out_parity=0)
    assert rel_err(lat.unpack_np(dst, dwf.KIND_EVEN), ref) < 1e-12
    dwf.mobius_dslash(ctx, p, Ug, src, dst, dwf.OP_HOP, 0, True)
    ref = mask(ora.fifth(po, ora.hop5(po, U, psio, dagger=True), "Fdag"), dims, 0)
    assert rel_err(lat.unpack_np(dst, dwf.KIND_EVEN), ref) < 1e-12


def test_moebius_b1_c0_is_shamir(env):
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 4), 8
    U, psi = make(dims, Ls, 800)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.01)
    Ug = lat.pack_gauge(U)
    src = lat.pack(mask(psi, dims, 1), dwf.KIND_ODD)
    a, b = lat.empty(dwf.KIND_ODD), lat.empty(dwf.KIND_ODD)
    dwf.dwf_dslash(ctx, lat.params(), Ug, src, a, dwf.OP_MPREC, 1, False)
    dwf.mobius_dslash(ctx, lat.params(), Ug, src, b, dwf.OP_MPREC, 1, False)
    assert rel_err(lat.unpack_np(a, dwf.KIND_ODD), lat.unpack_np(b, dwf.KIND_ODD)) == 0.0


def test_pack_roundtrip_and_errors(env):
    dwf, ctx = env
    dims, Ls = (4, 2, 2, 2), 4
    psi = synth.gaussian_spinor(dims, Ls, 900)
    lat = dwf.Lattice(ctx, dims, Ls)
    assert rel_err(lat.unpack_np(lat.pack(psi)), psi) == 0.0
    bad = dwf.params((3, 4, 4, 4), 4)
    with pytest.raises(dwf.DwfError) as e:
        dwf.dwf_dslash(ctx, bad, 1, 2, 3, dwf.OP_HOP, 0, False)
    assert e.value.code == dwf.DWF_ERR_ARG
    src = lat.pack(psi)
    with pytest.raises(dwf.DwfError):
        dwf.dwf_dslash(ctx, lat.params(), src, src, src, dwf.OP_HOP, 0, False)


def test_kernel_timing_report(env):
    """Per-launch HIP-event timing: one record per hop / fifth-dimension launch, named as the
    template instance the dispatcher selects, with the algorithmic bytes of each launch."""
    dwf, ctx = env
    dims, Ls = (8, 8, 8, 8), 16
    U, psi = make(dims, Ls, 810)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.02)
    P = dwf.FP16
    Ug = lat.pack_gauge(U, P)
    src = lat.pack(mask(psi, dims, 1), dwf.KIND_ODD, P)
    dst = lat.empty(dwf.KIND_ODD, P)
    dwf.dwf_timing_report(ctx)  # discard earlier records
    dwf.dwf_timing_enable(ctx, True)
    try:
        dwf.dwf_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_MPREC, 1, False)
        dwf.dwf_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_MPREC, 1, True)
        rep = dwf.dwf_timing_report(ctx)
    finally:
        dwf.dwf_timing_enable(ctx, False)
    spb, ns, xcd, ll = dwf.dwf_tune_get(ctx, P, Ls)
    llb = "true" if ll in (1, 2) else "false"  # (the staged variant also stages its links)
    st = "true" if ll == 2 else "false"
    epi = 2 if ns == 1 else 1
    nsites = 8 ** 4 // 2
    site = 12 * 4 + 4  # FP16 spinor (12 half2) + FP32 norm per 5D site
    links = nsites * 72 * 4
    want = {
        # M_prec: two hops with the A^-1 epilogue, the second with the axpy operand
        f"hop_kernel<dwf::P16, 16, {ns}, false, false, {epi}, {llb}, false, {st}>": (2, nsites * Ls * site * 5 + 2 * links),
        # M_prec^dag: A^-dag, then a dagger hop with an epilogue and one without
        f"hop_kernel<dwf::P16, 16, {ns}, true, false, {epi}, {llb}, false, {st}>": (1, nsites * Ls * site * 2 + links),
        f"hop_kernel<dwf::P16, 16, {ns}, true, false, 0, {llb}, false, {st}>": (1, nsites * Ls * site * 3 + links),
        "fifth_kernel<dwf::P16, 16>": (1, nsites * Ls * site * 2),
    }
    assert set(rep) == set(want), rep
    for k, (n, nbytes) in want.items():
        assert rep[k]["launches"] == n, k
        assert rep[k]["bytes"] == pytest.approx(nbytes, rel=1e-12), k
        assert rep[k]["ms"] > 0.0
    assert dwf.dwf_timing_report(ctx) == {}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_every_launch_shape_gives_the_same_operator(env, ora, prec):
    """Every launch shape the autotuner may install (sites per workgroup, s-slices per thread,
    XCD-aware order, links staged in LDS) gives M_prec and M_prec^dag to the precision's
    tolerance against the oracle (Moebius operator, ragged last workgroup)."""
    from paper_1111_5059_amd import autotune
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    dims, Ls = (6, 4, 6, 10), 16
    U, psi = make(dims, Ls, 820)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    Ug = lat.pack_gauge(U, P)
    po = ora.params(dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    psio = mask(psi, dims, 1)
    src = lat.pack(psio, dwf.KIND_ODD, P)
    refs = {dag: ora.mprec(po, U, psio, dagger=dag) for dag in (False, True)}
    tried = 0
    try:
        for c in autotune.candidates(P, Ls):
            try:
                dwf.dwf_tune_set(ctx, P, Ls, c["spb"], c["ns"], c["xcd"], c["ll"])
            except dwf.DwfError:
                continue  # a shape the kernel cannot run is rejected before launch
            tried += 1
            for dag in (False, True):
                dst = lat.empty(dwf.KIND_ODD, P)
                dwf.mobius_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_MPREC, 1, dag)
                err = rel_err(lat.unpack_np(dst, dwf.KIND_ODD, P), refs[dag])
                assert err < PREC_TOL[prec], (c, dag, err)
    finally:
        dwf.dwf_tune_set(ctx, P, Ls, 0, 0)
    assert tried >= 8


def test_autotuner_installs_the_fastest_shape(env, tmp_path):
    from paper_1111_5059_amd import autotune
    dwf, ctx = env
    dims, Ls = (8, 8, 8, 8), 8
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05)
    U64 = lat.pack_gauge(synth.random_links(dims, 0.5, 830))
    cache = str(tmp_path / "tune.json")
    shapes = [{"spb": 8, "ns": 1, "xcd": 1, "ll": 1}, {"spb": 16, "ns": 2, "xcd": 0, "ll": 0}]
    try:
        best, ms, table = autotune.tune_hop(lat, U64, "fp32", reps=2, cache=cache, shapes=shapes)
        assert len(table) == 2 and ms == min(r["ms"] for r in table)
        assert autotune.current(lat, "fp32") == best
        dwf.dwf_tune_set(ctx, dwf.FP32, Ls, 0, 0)
        assert autotune.load(lat, "fp32", cache) == dict(best, ms=ms)
        assert autotune.current(lat, "fp32") == best
    finally:
        dwf.dwf_tune_set(ctx, dwf.FP32, Ls, 0, 0)


def test_traversal_tile_changes_nothing_but_the_order(env, ora):
    """Every traversal tile gives bit-identical M_prec and M_prec^dag (the tile only reorders
    the workgroups' sites) that agree with the oracle; tiles that do not divide the lattice
    are rejected; (0, 0, 0) restores the default; the tile search installs its fastest tile."""
    from paper_1111_5059_amd import autotune
    dwf, ctx = env
    P = dwf.FP32
    dims, Ls = (12, 4, 6, 8), 8
    U, psi = make(dims, Ls, 840)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    Ug = lat.pack_gauge(U, P)
    po = ora.params(dims, Ls, mass=0.05, b=1.5, c=0.5, tbc=1)
    psio = mask(psi, dims, 1)
    src = lat.pack(psio, dwf.KIND_ODD, P)
    default = dwf.dwf_tune_tile_get(ctx, dims, 1)
    assert all(dims[k] % default[k] == 0 for k in range(3))

    def apply(dag):
        dst = lat.empty(dwf.KIND_ODD, P)
        dwf.mobius_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_MPREC, 1, dag)
        return lat.unpack_np(dst, dwf.KIND_ODD, P)

    first = {dag: apply(dag) for dag in (False, True)}
    for dag in (False, True):
        assert rel_err(first[dag], ora.mprec(po, U, psio, dagger=dag)) < PREC_TOL["fp32"]
    try:
        for tile in [(2, 2, 2), (12, 4, 6), (4, 2, 3), (6, 4, 2), (3, 1, 1)]:
            dwf.dwf_tune_tile(ctx, dims, tile, 1)
            assert dwf.dwf_tune_tile_get(ctx, dims, 1) == tile
            for dag in (False, True):
                assert np.array_equal(apply(dag), first[dag]), (tile, dag)
        for bad in [(5, 4, 6), (12, 4, 0), (24, 4, 6), (-2, 4, 6)]:
            with pytest.raises(dwf.DwfError):
                dwf.dwf_tune_tile(ctx, dims, bad, 1)
        best, ms, table = autotune.tune_tile(lat, lat.pack_gauge(U), "fp32", tiles=[(2, 2, 2), (6, 4, 6)], reps=2)
        assert len(table) == 2 and ms == min(r["ms"] for r in table)
        assert dwf.dwf_tune_tile_get(ctx, dims, 1) == best
    finally:
        dwf.dwf_tune_tile(ctx, dims, (0, 0, 0), 1)
    assert dwf.dwf_tune_tile_get(ctx, dims, 1) == default
    for dag in (False, True):
        assert np.array_equal(apply(dag), first[dag])


@pytest.mark.parametrize("Ls", [8, 16, 32])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("bc", [(1.0, 0.0), (1.5, 0.5)])
def test_scan_epilogue_every_segment_length(env, ora, Ls, prec, bc):
    """The recurrence form of the fifth-dimension blocks in FP32 arithmetic (cross-lane moves
    within rows of 16 lanes, and across rows for Ls = 32), in the hop's epilogue (M_prec, M_prec^dag)
    and in the standalone kernel (A^-1, A^-dag), against the oracle at every segment length."""
    dwf, ctx = env
    P = dwf.PREC_NAMES[prec]
    dims = (4, 2, 2, 4)
    U, psi = make(dims, Ls, 850 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=1)
    po = ora.params(dims, Ls, mass=0.05, b=bc[0], c=bc[1], tbc=1)
    Ug = lat.pack_gauge(U, P)
    psio = mask(psi, dims, 1)
    src = lat.pack(psio, dwf.KIND_ODD, P)
    for dag in (False, True):
        dst = lat.empty(dwf.KIND_ODD, P)
        dwf.mobius_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_MPREC, 1, dag)
        err = rel_err(lat.unpack_np(dst, dwf.KIND_ODD, P), ora.mprec(po, U, psio, dagger=dag))
        assert err < PREC_TOL[prec], ("mprec", dag, err)
        dst = lat.empty(dwf.KIND_ODD, P)
        dwf.mobius_dslash(ctx, lat.params(P), Ug, src, dst, dwf.OP_AINV, 1, dag)
        ref = mask(ora.fifth(po, psio, "Ainv" + ("dag" if dag else "")), dims, 1)
        err = rel_err(lat.unpack_np(dst, dwf.KIND_ODD, P), ref)
        assert err < PREC_TOL[prec], ("Ainv", dag, err)
