"""Moebius-parameter scan for the Moebius-accelerated DWF solver.

Sec. 5 / Figure 1 of the paper: the quality of the Moebius guess saturates -- past a
"turning point" a more accurate Moebius solve no longer reduces the number of DWF CG
iterations needed afterwards.  This module reproduces the method on synthetic fields: for
each inner operator (L', b, c) and each Moebius tolerance it runs one MADWF step (n_dc = 1)
and records the Moebius CG count, the true residual of the guess, and the DWF CG count of
the warm-started final solve to 1e-10; the zero-start DWF CG count is the reference.

python -m paper_1111_5059_amd.madwf_scan [--dims 32 32 32 8] [--Ls 32] [--mass 0.005] [--eps 0.6]
    [--inner-prec fp32|fp16|bf16]

Defaults follow Figure 1: a 32^3 x 8 lattice with L = 32 and the inner L' = 16, b = 1.5,
c = 0.5; the scan adds L' = 12 (Table 1's inner extent) and a Shamir inner (b = 1, c = 0) for
comparison.  Output: one JSON object.
"""
import argparse
import json
import os
import sys


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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[32, 32, 32, 8])
    ap.add_argument("--Ls", type=int, default=32)
    ap.add_argument("--mass", type=float, default=0.005)
    ap.add_argument("--eps", type=float, default=0.6)
    ap.add_argument("--seed", type=int, default=6)
    ap.add_argument("--inner-prec", default="fp32", choices=["fp32", "fp16", "bf16"])
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import paper_1111_5059_amd as dwf
    import synth
    ctx = dwf.Context()
    dims = tuple(args.dims)
    lat = dwf.Lattice(ctx, dims, args.Ls, M5=1.8, mass=args.mass)
    U64 = lat.pack_gauge(synth.random_links(dims, args.eps, synth.link_seed(args.seed)))
    b = lat.pack(synth.gaussian_spinor(dims, args.Ls, synth.source_seed(args.seed)))
    x = lat.zeros(dwf.KIND_FULL)
    ref = dwf.cg_ne(ctx, lat.params(prec_inner=dwf.FP32), U64, b, x, tol=1e-10)
    print(f"zero-start DWF CG: {ref['iters']} iterations", file=sys.stderr, flush=True)
    L = args.Ls
    inners = [(L // 2, 1.5, 0.5), (3 * L // 8, 1.5, 0.5), (L // 2, 1.0, 0.0)]
    tols = [1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 1e-6]
    rows = []
    for inner in inners:
        rows += scan(lat, U64, b, [inner], tols, prec_inner=dwf.PREC_NAMES[args.inner_prec])
        for r in rows[-len(tols):]:
            print(f"L'={r['Lp']} b={r['b']} c={r['c']} tol={r['tol_mobius']:.0e}: Moebius CG {r['mobius_iters']}, "
                  f"guess resid {r['guess_resid']:.2e}, DWF CG after {r['dwf_iters_after']}", file=sys.stderr, flush=True)
    print(json.dumps({"dims": dims, "Ls": L, "mass": args.mass, "eps": args.eps, "inner_prec": args.inner_prec,
                      "zero_start_dwf_iters": ref["iters"], "rows": rows}))


if __name__ == "__main__":
    main()
