"""Moebius-parameter scan for the Moebius-accelerated DWF solver.

Sec. 5 / Figure 1 of the paper: the quality of the Moebius guess saturates -- past a
"turning point" a more accurate Moebius solve no longer reduces the number of DWF CG
iterations needed afterwards.  This module reproduces the method on synthetic fields: for
each inner operator (L', b, c) and each Moebius tolerance it runs one MADWF step (n_dc = 1)
and records the Moebius CG count, the true residual of the guess, and the DWF CG count of
the warm-started final solve to 1e-10; the zero-start DWF CG count is the reference.

The library call only: the inputs (links, source) are the caller's packed device fields.
``python bench.py --madwf-scan`` runs the Figure-1 scan on synthetic fields (a 32^3 x 8 lattice
with L = 32 and the inner L' = 16, b = 1.5, c = 0.5, plus L' = 12 and a Shamir inner operator).
"""


def scan(lat, U64, b, inners, tols, tol_pv=1e-8, prec_inner=None, prec_final=None):
    """inners: list of (Lp, bm, cm); returns a list of records (one per inner and tolerance)."""
    import paper_1111_5059_amd as dwf
    prec_inner = dwf.FP32 if prec_inner is None else prec_inner
    prec_final = dwf.FP32 if prec_final is None else prec_final
    out = []
    for Lp, bm, cm in inners:
        inner = lat.with_(Ls=Lp, b=bm, c=cm)
        for tm in tols:
            x = lat.zeros(dwf.KIND_FULL)
            info = dwf.mobius_accel_solve(lat.ctx, lat.params(), inner.params(prec_inner=prec_inner), U64, b, x,
                                          n_dc=1, tol_pv=tol_pv, tol_mobius=tm, tol=1e-10, prec_pv=prec_final,
                                          prec_final=prec_final)
            out.append({"Lp": Lp, "b": bm, "c": cm, "tol_mobius": tm, "mobius_iters": info["mobius_iters"],
                        "guess_resid": info["resid_after_dc"][0], "dwf_iters_after": info["final_iters"],
                        "pv_iters": info["pv_iters"], "wilson_apps": info["wilson_apps"],
                        "converged": info["converged"]})
    return out
