"""Batched multi-right-hand-side solve: a Hasenbusch mass ladder (Sec. 3) on one lattice and
a ragged batch of two lattices with different Ls, each solved together; every solution is
checked against its own true residual and against the single-right-hand-side solve."""
import numpy as np
import pytest

import synth
from gpu_helpers import gpu_ctx, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return gpu_ctx()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mass_ladder_batch(env, ora, prec):
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 8), 8
    masses = [0.005, 0.02, 0.1, 0.4]
    U = synth.random_links(dims, 0.4, 1501)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    Ug = lat.pack_gauge(U)
    P = dwf.PREC_NAMES[prec]
    pars, bs, xs, srcs = [], [], [], []
    for k, m in enumerate(masses * 2):
        b = synth.gaussian_spinor(dims, Ls, 1510 + k)
        srcs.append(b)
        pars.append(lat.params(mass=m, prec_inner=P))
        bs.append(lat.pack(b))
        xs.append(lat.zeros(dwf.KIND_FULL))
    infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-10)
    for k, (info, m) in enumerate(zip(infos, masses * 2)):
        assert info["converged"], (k, info)
        x = lat.unpack_np(xs[k])
        po = ora.params(dims, Ls, M5=1.8, mass=m)
        r = srcs[k] - ora.dwf(po, U, x)
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k])
    # heavier masses converge in fewer iterations
    assert infos[3]["iters"] < infos[0]["iters"]
    # the same right-hand side solved alone gives the same solution
    x1 = lat.zeros(dwf.KIND_FULL)
    dwf.cg_ne(ctx, pars[1], Ug, bs[1], x1, tol=1e-12)
    assert rel_err(lat.unpack_np(xs[1]), lat.unpack_np(x1)) < 1e-7


@pytest.mark.parametrize("Ls", [8, 12])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_moebius_mass_ladder_batch(env, ora, Ls, prec):
    """A Moebius ladder (b = 1.5, c = 0.5): input factor and F^dag epilogue in the batched stages,
    the CG step fused into the last one; Ls = 8 takes the recurrence-form epilogue, Ls = 12 the
    dense one.  Every solve reaches the full-system true residual against the oracle's operator."""
    dwf, ctx = env
    dims = (4, 4, 2, 4)
    masses = [0.01, 0.1, 0.5]
    U = synth.random_links(dims, 0.4, 1520 + Ls)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, b=1.5, c=0.5)
    Ug = lat.pack_gauge(U)
    P = dwf.PREC_NAMES[prec]
    pars, bs, xs, srcs = [], [], [], []
    for k, m in enumerate(masses):
        b = synth.gaussian_spinor(dims, Ls, 1530 + k)
        srcs.append(b)
        pars.append(lat.params(mass=m, prec_inner=P))
        bs.append(lat.pack(b))
        xs.append(lat.zeros(dwf.KIND_FULL))
    infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-10)
    for k, (info, m) in enumerate(zip(infos, masses)):
        assert info["converged"], (k, info)
        po = ora.params(dims, Ls, M5=1.8, mass=m, b=1.5, c=0.5)
        r = srcs[k] - ora.dwf(po, U, lat.unpack_np(xs[k]))
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k]), (k, m)


def test_ragged_batch(env, ora):
    """8^4 Ls=8 and 12^2x4x6 Ls=12 (scaled-down versions of the ragged batch) in one solve."""
    dwf, ctx = env
    cases = [((8, 8, 8, 8), 8, 0.02, 1601), ((12, 12, 4, 6), 12, 0.05, 1602)]
    pars, Us, bs, xs, ref = [], [], [], [], []
    for dims, Ls, m, seed in cases:
        U = synth.random_links(dims, 0.4, seed)
        b = synth.gaussian_spinor(dims, Ls, seed + 50)
        lat = dwf.Lattice(ctx, dims, Ls, M5=1.8, mass=m)
        pars.append(lat.params(prec_inner=dwf.FP32))
        Us.append(lat.pack_gauge(U))
        bs.append(lat.pack(b))
        xs.append(lat.zeros(dwf.KIND_FULL))
        ref.append((lat, U, b, ora.params(dims, Ls, M5=1.8, mass=m)))
    infos = dwf.cg_ne_batched(ctx, pars, Us, bs, xs, tol=1e-10)
    for (lat, U, b, po), x, info in zip(ref, xs, infos):
        assert info["converged"], info
        r = b - ora.dwf(po, U, lat.unpack_np(x))
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(b)


def test_batch_validation(env):
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 4), 4
    lat = dwf.Lattice(ctx, dims, Ls)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.3, 3))
    b = lat.pack(synth.gaussian_spinor(dims, Ls, 4))
    x = lat.zeros(dwf.KIND_FULL)
    with pytest.raises(dwf.DwfError):  # different M5 in one batch
        dwf.cg_ne_batched(ctx, [lat.params(), lat.params(M5=1.5)], Ug, [b, b], [x, lat.zeros(dwf.KIND_FULL)])
    with pytest.raises(dwf.DwfError):  # the same solution field twice
        dwf.cg_ne_batched(ctx, [lat.params(), lat.params()], Ug, [b, b], [x, x])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_respects_maxit(env, prec):
    """The iteration cap holds per right-hand side over all restarts of the normal-equation
    tolerance: no right-hand side runs more than maxit iterations."""
    dwf, ctx = env
    dims, Ls = (4, 4, 4, 4), 8
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.4, 1621))
    masses = [0.01, 0.3]
    bs = [lat.pack(synth.gaussian_spinor(dims, Ls, 1622 + k)) for k in range(2)]
    xs = [lat.zeros(dwf.KIND_FULL) for _ in range(2)]
    pars = [lat.params(mass=m, prec_inner=dwf.PREC_NAMES[prec]) for m in masses]
    for maxit in (7, 40):
        infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-12, maxit=maxit)
        for info in infos:
            assert info["iters"] <= maxit, (maxit, info)
        assert not infos[0]["converged"]
        for x in xs:
            x.zero_()


def test_bf16_interleaved_ladder(env, ora):
    """BF16 storage in the interleaved batch: each right-hand side restarts its Krylov space at its
    reliable updates (as the single solve does) and still reaches 1e-10 through the oracle's D."""
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 4), 16
    masses = [0.02, 0.1, 0.4]
    U = synth.random_links(dims, 0.4, 1820)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    srcs = [synth.gaussian_spinor(dims, Ls, 1830 + k) for k in range(len(masses))]
    xs = [lat.zeros(dwf.KIND_FULL) for _ in masses]
    infos = dwf.cg_ne_batched(ctx, [lat.params(mass=m, prec_inner=dwf.BF16) for m in masses], lat.pack_gauge(U),
                              [lat.pack(b) for b in srcs], xs, tol=1e-10)
    for k, (m, info) in enumerate(zip(masses, infos)):
        assert info["converged"] and info["reliable_updates"] >= 1, (k, info)
        po = ora.params(dims, Ls, M5=1.8, mass=m)
        r = srcs[k] - ora.dwf(po, U, lat.unpack_np(xs[k]))
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k]), (k, m)


# storage unit roundoff of the iteration precisions (see test_partial_cg_iterates_low_precision)
LOW_PREC_U = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_interleaved_iterates_follow_cgnr(env, ora, prec):
    """A four-mass Shamir ladder at Ls = 16 runs interleaved, where the last stage rebuilds each
    right-hand side's q = M_prec p from A^-dag q with that right-hand side's A^dag; after k = 3
    iterations every iterate is the oracle's CGNR iterate for its mass to within 10 k u."""
    dwf, ctx = env
    dims, Ls, k = (4, 4, 4, 8), 16, 3
    masses = [0.005, 0.02, 0.1, 0.4]
    U = synth.random_links(dims, 0.6, 1561)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    Ug = lat.pack_gauge(U)
    P = dwf.PREC_NAMES[prec]
    pars, bs, xs, srcs = [], [], [], []
    for j, m in enumerate(masses):
        b = synth.gaussian_spinor(dims, Ls, 1570 + j)
        srcs.append(b)
        pars.append(lat.params(mass=m, prec_inner=P))
        bs.append(lat.pack(b))
        xs.append(lat.zeros(dwf.KIND_FULL))
    infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-14, maxit=k)
    for j, (info, m) in enumerate(zip(infos, masses)):
        assert info["iters"] == k and not info["converged"], (j, info)
        xo, info_o = ora.solve(ora.params(dims, Ls, M5=1.8, mass=m), U, srcs[j], tol=1e-14, maxit=k)
        err = rel_err(lat.unpack_np(xs[j]), xo)
        print(prec, m, err)
        assert err < 10 * k * LOW_PREC_U[prec], (j, m, err)


def test_batch_beyond_one_launch(env, ora):
    """Nine Shamir right-hand sides at Ls = 32: the interleaved hop takes at most 256 / Ls = 8 per
    launch, so they run as a chunk of 8 and a chunk of 1; a tenth at Ls = 12 (no interleaved form) in
    the same call runs on a separate field.  Every solve reaches 1e-10 through the oracle's D."""
    dwf, ctx = env
    dims = (4, 2, 2, 4)
    U = synth.random_links(dims, 0.4, 1801)
    lats = {Ls: dwf.Lattice(ctx, dims, Ls, M5=1.8) for Ls in (32, 12)}
    Ug = lats[32].pack_gauge(U)
    cases = [(32, 0.01 * (k + 1)) for k in range(9)] + [(12, 0.05)]
    srcs = [synth.gaussian_spinor(dims, Ls, 1810 + k) for k, (Ls, _) in enumerate(cases)]
    pars = [lats[Ls].params(mass=m, prec_inner=dwf.FP32) for Ls, m in cases]
    bs = [lats[Ls].pack(b) for (Ls, _), b in zip(cases, srcs)]
    xs = [lats[Ls].zeros(dwf.KIND_FULL) for Ls, _ in cases]
    infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-10)
    for k, ((Ls, m), info) in enumerate(zip(cases, infos)):
        assert info["converged"], (k, info)
        po = ora.params(dims, Ls, M5=1.8, mass=m)
        r = srcs[k] - ora.dwf(po, U, lats[Ls].unpack_np(xs[k]))
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k]), (k, Ls, m)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_every_batched_shape_solves(env, ora, prec):
    """Every shape the batched tuner may install (right-hand sides interleaved along s, or on
    separate fields with 1..32 sites per workgroup, XCD order, links in LDS) solves a Shamir mass
    ladder to the full-system true residual against the oracle."""
    from paper_1111_5059_amd import autotune
    dwf, ctx = env
    dims, Ls = (4, 4, 2, 6), 16
    masses = [0.01, 0.05, 0.2]
    U = synth.random_links(dims, 0.4, 1701)
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    Ug = lat.pack_gauge(U)
    P = dwf.PREC_NAMES[prec]
    srcs = [synth.gaussian_spinor(dims, Ls, 1710 + k) for k in range(len(masses))]
    pars = [lat.params(mass=m, prec_inner=P) for m in masses]
    bs = [lat.pack(b) for b in srcs]
    tried = set()
    try:
        for c in autotune.batch_candidates(P, Ls, len(masses)):
            try:
                autotune.install_batched(ctx, P, Ls, c)
            except dwf.DwfError:
                continue  # a shape the kernel cannot run is rejected before launch
            assert autotune.current_batched(ctx, P, Ls) == c
            tried.add(c["mode"])
            xs = [lat.zeros(dwf.KIND_FULL) for _ in masses]
            infos = dwf.cg_ne_batched(ctx, pars, Ug, bs, xs, tol=1e-10)
            for k, (info, m) in enumerate(zip(infos, masses)):
                assert info["converged"], (c, k, info)
                po = ora.params(dims, Ls, M5=1.8, mass=m)
                r = srcs[k] - ora.dwf(po, U, lat.unpack_np(xs[k]))
                assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(srcs[k]), (c, k)
    finally:
        autotune.install_batched(ctx, P, Ls, None)
    assert tried == {"interleaved", "separate"}


def test_batched_tuner_installs_the_fastest_shape(env, tmp_path):
    from paper_1111_5059_amd import autotune
    dwf, ctx = env
    dims, Ls = (8, 8, 8, 8), 16
    lat = dwf.Lattice(ctx, dims, Ls, M5=1.8)
    Ug = lat.pack_gauge(synth.random_links(dims, 0.5, 1720))
    cache = str(tmp_path / "tune.json")
    shapes = [{"mode": "interleaved", "spb": 1, "xcd": 1, "ll": 0},
              {"mode": "separate", "spb": 8, "xcd": 1, "ll": 1}]
    try:
        best, ms, table = autotune.tune_batched(lat, Ug, "fp32", [0.01, 0.02, 0.05, 0.1], iters=4,
                                                cache=cache, shapes=shapes)
        assert len(table) == 2 and ms == min(r["ms"] for r in table)
        assert autotune.current_batched(ctx, "fp32", Ls) == best
        with open(cache) as fh:
            import json
            assert json.load(fh)["batch|1|16|4|8x8x8x8"] == dict(best, ms=ms)
    finally:
        autotune.install_batched(ctx, dwf.FP32, Ls, None)
    assert autotune.current_batched(ctx, dwf.FP32, Ls)["mode"] == "interleaved"
