"""Autotuner for the hop-kernel launch shape.

For one (precision, Ls, lattice) it times the even-odd operator M_prec (the solver's inner
kernel mix: hops with the fused fifth-dimension epilogue, prologue and axpy) over every valid
launch shape -- 4D sites per workgroup, s-slices per thread, XCD-aware workgroup order, links
or neighbour spinors staged in LDS -- keeps the fastest, installs it with ``dwf_tune_set`` and caches it in a JSON
file keyed by (kernel, precision, Ls, lattice).  Shapes the kernel cannot run (more than 256
threads, LDS above 64 KiB) are never tried: the library rejects them before launching.
"""
import json
import os

from . import (FP64, KIND_GAUGE, KIND_ODD, OP_MPREC, PREC_NAMES, DwfError, dwf_convert, dwf_dslash,
               dwf_tune_get, dwf_tune_set)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dwf_mi355x_tune.json")


def _key(prec, Ls, dims):
    return f"hop|{prec}|{Ls}|{'x'.join(str(d) for d in dims)}"


def candidates(prec, Ls):
    elem_c = 16 if prec == FP64 else 8
    elem_s = {0: 16, 1: 8}.get(prec, 4)
    out = []
    for ns in (1, 2, 4):
        if Ls % ns:
            continue
        for spb in (1, 2, 4, 8, 16, 32, 64):
            threads = spb * Ls // ns
            if threads > 256 or threads < 32:
                continue
            for ll in (0, 1, 2):  # LDS mode: none, links, neighbour spinors (FP16)
                if ll == 2 and not (prec == 2 and ns == 1 and threads == 256 and Ls in (8, 16, 32)):
                    continue
                lds = spb * 12 * Ls * elem_c + (spb * 72 * elem_s if ll == 1 else 0)
                if lds > 65536:
                    continue
                for xcd in (0, 1):
                    out.append({"spb": spb, "ns": ns, "xcd": xcd, "ll": ll})
    return out


def _time_mprec(lattice, Ug, src, dst, p, reps):
    import torch
    for _ in range(2):
        dwf_dslash(lattice.ctx, p, Ug, src, dst, OP_MPREC, 1, False)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        dwf_dslash(lattice.ctx, p, Ug, src, dst, OP_MPREC, 1, False)
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_hop(lattice, U64, prec, reps=5, cache=DEFAULT_CACHE, shapes=None, verbose=False):
    """Search the launch shapes for ``prec`` on ``lattice``; returns (best shape, ms, table)."""
    import torch
    P = PREC_NAMES.get(prec, prec)
    p = lattice.params(P)
    Ug = U64
    if P != FP64:
        Ug = lattice.empty(KIND_GAUGE, P)
        dwf_convert(lattice.ctx, lattice.params(P), KIND_GAUGE, FP64, U64, P, Ug)
    tmp = lattice.zeros(KIND_ODD, FP64)
    g = torch.Generator(device=tmp.device)
    g.manual_seed(11)
    tmp.view(torch.float64).normal_(generator=g)
    src = lattice.empty(KIND_ODD, P)
    dwf_convert(lattice.ctx, p, KIND_ODD, FP64, tmp, P, src)
    dst = lattice.empty(KIND_ODD, P)
    table = []
    best = None
    for c in shapes or candidates(P, lattice.Ls):
        try:
            dwf_tune_set(lattice.ctx, P, lattice.Ls, c["spb"], c["ns"], c["xcd"], c["ll"])
        except DwfError:
            continue
        ms = _time_mprec(lattice, Ug, src, dst, p, reps)
        table.append(dict(c, ms=ms))
        if verbose:
            print(f"tune {prec} Ls={lattice.Ls} {c}: {ms:.3f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (c, ms)
    dwf_tune_set(lattice.ctx, P, lattice.Ls, best[0]["spb"], best[0]["ns"], best[0]["xcd"], best[0]["ll"])
    if cache:
        save(cache, _key(P, lattice.Ls, lattice.dims), dict(best[0], ms=best[1]))
    return best[0], best[1], table


def save(path, key, value):
    d = {}
    if os.path.exists(path):
        with open(path) as fh:
            d = json.load(fh)
    d[key] = value
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(lattice, prec, cache=DEFAULT_CACHE):
    """Install a cached shape for (prec, lattice); returns it or None."""
    P = PREC_NAMES.get(prec, prec)
    if not os.path.exists(cache):
        return None
    with open(cache) as fh:
        d = json.load(fh)
    c = d.get(_key(P, lattice.Ls, lattice.dims))
    if c is None:
        return None
    dwf_tune_set(lattice.ctx, P, lattice.Ls, c["spb"], c["ns"], c["xcd"], c["ll"])
    return c


def current(lattice, prec):
    P = PREC_NAMES.get(prec, prec)
    spb, ns, xcd, ll = dwf_tune_get(lattice.ctx, P, lattice.Ls)
    return {"spb": spb, "ns": ns, "xcd": xcd, "ll": ll}
