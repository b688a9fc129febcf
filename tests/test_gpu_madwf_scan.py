"""Moebius-tolerance scan of the MADWF guess (Sec. 5, Figure 1) on a small lattice.

With the inner operator equal to the target (L' = L, b = 1, c = 0) the one-step guess is the
exact solve, so its residual follows the Moebius tolerance down and the warm-started DWF solve
needs fewer iterations than the zero-start one.  With a shorter inner operator the guess
saturates at the operators' difference (the turning point of Figure 1): tightening the Moebius
tolerance past it buys Moebius iterations and no better guess."""
import pytest

import synth
from gpu_helpers import gpu_ctx

pytestmark = pytest.mark.gpu


def test_scan_turning_point():
    dwf, ctx = gpu_ctx()
    from paper_1111_5059_amd import madwf_scan
    dims, Ls = (4, 4, 4, 8), 8
    lat = dwf.Lattice(ctx, dims, Ls, mass=0.05)
    U64 = lat.pack_gauge(synth.random_links(dims, 0.3, 1500))
    b = lat.pack(synth.gaussian_spinor(dims, Ls, 1501))
    ref = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.FP32), U64, b, lat.zeros(dwf.KIND_FULL), tol=1e-10)
    tols = [1e-1, 1e-3, 1e-5]
    exact = madwf_scan.scan(lat, U64, b, [(Ls, 1.0, 0.0)], tols)
    short = madwf_scan.scan(lat, U64, b, [(4, 1.5, 0.5)], tols)
    for r in exact + short:
        print(r)
        assert r["converged"]
    for rows in (exact, short):
        assert [r["tol_mobius"] for r in rows] == tols
        mob = [r["mobius_iters"] for r in rows]
        assert mob == sorted(mob) and mob[-1] > mob[0]
    # exact inner: the guess follows the tolerance (PV solves at 1e-8 bound it from below)
    assert exact[-1]["guess_resid"] < 1e-4
    assert exact[-1]["guess_resid"] < 1e-2 * exact[0]["guess_resid"]
    assert exact[-1]["dwf_iters_after"] < ref["iters"]
    # short inner: saturated guess, 100x more Moebius accuracy gains less than 2x in the guess
    assert short[-1]["guess_resid"] > 1e-3
    assert short[-1]["guess_resid"] > 0.5 * short[1]["guess_resid"]


def test_scan_rows_match_the_oracle(ora):
    """Every row of the scan (one defect-correction step at a given Moebius tolerance, FP64
    solves) against the oracle's MADWF with n_dc = 1 at the same tolerances on the same lattice:
    the guess residual to within a factor 1.5 and the DWF iterations after the guess to within
    15 % (the two start the second PV solve from different guesses and tighten the final
    normal-equation tolerance by slightly different rules)."""
    dwf, ctx = gpu_ctx()
    from paper_1111_5059_amd import madwf_scan
    dims, Ls, m = (4, 4, 4, 8), 8, 0.05
    U = synth.random_links(dims, 0.3, 1500)
    src = synth.gaussian_spinor(dims, Ls, 1501)
    lat = dwf.Lattice(ctx, dims, Ls, mass=m)
    U64, b = lat.pack_gauge(U), lat.pack(src)
    tols = [1e-1, 1e-3, 1e-5]
    inners = [(4, 1.5, 0.5), (Ls, 1.0, 0.0)]
    rows = madwf_scan.scan(lat, U64, b, inners, tols, tol_pv=1e-8, prec_inner=dwf.FP64, prec_final=dwf.FP64)
    pt = ora.params(dims, Ls, M5=1.8, mass=m)
    for r in rows:
        pi = ora.params(dims, r["Lp"], M5=1.8, mass=m, b=r["b"], c=r["c"])
        _, o = ora.madwf(pt, pi, U, src, n_dc=1, tol_pv=1e-8, tol_mob=r["tol_mobius"], tol=1e-10)
        print(r, o["resid_after_dc"][0], o["final_iters"])
        assert r["converged"] and o["converged"]
        ratio = r["guess_resid"] / o["resid_after_dc"][0]
        assert 1 / 1.5 < ratio < 1.5, (r, o)
        assert abs(r["dwf_iters_after"] - o["final_iters"]) <= 0.15 * o["final_iters"] + 2, (r, o)
