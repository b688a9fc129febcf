"""Autotuner for the hop-kernel launch shape.

For one (precision, Ls, lattice) it times the even-odd operator M_prec (the solver's inner
kernel mix: hops with the fused fifth-dimension epilogue, prologue and axpy) over every valid
launch shape -- 4D sites per workgroup, s-slices per thread, XCD-aware workgroup order, links
or neighbour spinors staged in LDS -- keeps the fastest, installs it with ``dwf_tune_set`` and caches it in a JSON
file keyed by (kernel, precision, Ls, lattice).  Shapes the kernel cannot run (more than 256
threads, LDS above 64 KiB) are never tried: the library rejects them before launching.

``tune_tile`` searches the traversal tile of a lattice the same way (``dwf_tune_tile``): the
3D tile of spatial sites the workgroups walk along t, which sets how much of each input
spinor's re-reads the L2 serves.

``tune_batched`` searches the batched solve (``cg_ne_batched``) over its hop's launch shapes:
right-hand sides interleaved along the fifth dimension (kernel 2: XCD order, links in LDS) or
on separate fields (kernel 1: sites per workgroup, XCD order, links in LDS), timing a fixed
number of iterations of the batched CG for (precision, Ls, number of right-hand sides, lattice).
"""
import json
import os

from . import (FP64, KIND_FULL, KIND_GAUGE, KIND_ODD, OP_MPREC, PREC_NAMES, DwfError, cg_ne_batched, dwf_convert,
               dwf_dslash, dwf_tune_get, dwf_tune_set, dwf_tune_tile, dwf_tune_tile_get)

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
    P = PREC_NAMES.get(prec, prec)
    p, Ug, src, dst = _operands(lattice, U64, P)
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


def tile_candidates(dims, lo=64, hi=2048):
    """3D traversal tiles whose extents divide the spatial extents, lo..hi sites per t-slice"""
    def divs(L):
        return [d for d in range(2, L + 1) if L % d == 0]
    out = []
    for tx in divs(dims[0]):
        for ty in divs(dims[1]):
            for tz in divs(dims[2]):
                if lo <= tx * ty * tz <= hi:
                    out.append((tx, ty, tz))
    return out


def _operands(lattice, U64, P):
    import torch
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
    return p, Ug, src, lattice.empty(KIND_ODD, P)


def tune_tile(lattice, U64, prec, tiles=None, reps=5, verbose=False):
    """Search the traversal tile of the hop kernels for ``prec`` on ``lattice`` (timing M_prec
    with the installed launch shape); installs the fastest and returns (tile, ms, table).  The
    tile is a property of the lattice, shared by every precision and Ls on it."""
    P = PREC_NAMES.get(prec, prec)
    p, Ug, src, dst = _operands(lattice, U64, P)
    default = dwf_tune_tile_get(lattice.ctx, lattice.dims, lattice.tbc)
    table, best = [], None
    for t in tiles or tile_candidates(lattice.dims):
        try:
            dwf_tune_tile(lattice.ctx, lattice.dims, t, lattice.tbc)
        except DwfError:
            continue
        ms = _time_mprec(lattice, Ug, src, dst, p, reps)
        table.append({"tile": list(t), "ms": ms, "default": tuple(t) == default})
        if verbose:
            print(f"tile {t}: {ms:.3f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (tuple(t), ms)
    dwf_tune_tile(lattice.ctx, lattice.dims, best[0], lattice.tbc)
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


# ------------------------------------------------------------------ batched solve
BATCH_SEPARATE, BATCH_INTERLEAVED = 1, 2  # kernel ids of the two batched hops


def batch_candidates(prec, Ls, nrhs):
    """Launch shapes of the batched solve: interleaved right-hand sides (Shamir, Ls 8/16/32, at
    most 256 / Ls of them per launch) and separate fields (one slice per thread)."""
    elem_c = 16 if prec == FP64 else 8
    elem_s = {0: 16, 1: 8}.get(prec, 4)
    lsite = 160 if prec == 2 else 72  # FP16 links are staged in two forms
    out = []
    if Ls in (8, 16, 32):
        for ll in (0, 1):
            for xcd in (0, 1):
                out.append({"mode": "interleaved", "spb": 1, "xcd": xcd, "ll": ll})
    for spb in (1, 2, 4, 8, 16, 32):
        if spb * Ls > 256 or spb * Ls < 32:
            continue
        for ll in (0, 1):
            if spb * 12 * Ls * elem_c + ll * spb * lsite * elem_s > 65536:
                continue
            for xcd in (0, 1):
                out.append({"mode": "separate", "spb": spb, "xcd": xcd, "ll": ll})
    return out


def install_batched(ctx, prec, Ls, c):
    """Install a batched-solve shape; c None restores the defaults."""
    P = PREC_NAMES.get(prec, prec)
    if c is None:
        dwf_tune_set(ctx, P, Ls, 0, 0, kernel_id=BATCH_INTERLEAVED)
        dwf_tune_set(ctx, P, Ls, 0, 0, kernel_id=BATCH_SEPARATE)
        return
    if c["mode"] == "interleaved":
        dwf_tune_set(ctx, P, Ls, 1, 1, c["xcd"], c["ll"], kernel_id=BATCH_INTERLEAVED)
    else:
        dwf_tune_set(ctx, P, Ls, -1, 1, 1, 0, kernel_id=BATCH_INTERLEAVED)  # interleaving off
        dwf_tune_set(ctx, P, Ls, c["spb"], 1, c["xcd"], c["ll"], kernel_id=BATCH_SEPARATE)


def _batch_key(prec, Ls, nrhs, dims):
    return f"batch|{prec}|{Ls}|{nrhs}|{'x'.join(str(d) for d in dims)}"


def tune_batched(lattice, U64, prec, masses, iters=10, cache=DEFAULT_CACHE, shapes=None, verbose=False,
                 sources=None, solutions=None):
    """Time ``iters`` iterations of the batched CG of len(masses) right-hand sides (zero guesses)
    for every shape; installs the fastest and returns (shape, ms per iteration, table).  sources /
    solutions: the caller's full-lattice FP64 fields (one per mass; the solutions are zeroed on
    return), so that a search at the largest sizes allocates nothing beside the solver's own
    workspace; by default one seeded Gaussian source and fresh solution fields."""
    import time
    import torch
    P = PREC_NAMES.get(prec, prec)
    ctx, Ls, n = lattice.ctx, lattice.Ls, len(masses)
    bs = sources
    if bs is None:
        g = torch.Generator(device="cuda")
        g.manual_seed(17)
        b = lattice.empty(KIND_FULL)
        b.view(torch.float64).normal_(generator=g)
        bs = [b] * n
    xs = solutions if solutions is not None else [lattice.zeros(KIND_FULL) for _ in range(n)]
    if len(bs) != n or len(xs) != n:
        raise ValueError("one source and one solution field per mass")
    pars = [lattice.params(mass=m, prec_inner=P) for m in masses]
    table, best, mode = [], None, None
    for c in shapes or batch_candidates(P, Ls, n):
        try:
            install_batched(ctx, P, Ls, c)
        except DwfError:
            continue
        if mode is not None and c["mode"] != mode:
            ctx.release()  # the two modes' workspaces need not fit together
        mode = c["mode"]
        for x in xs:
            x.zero_()
        cg_ne_batched(ctx, pars, U64, bs, xs, tol=1e-14, maxit=2)  # workspace
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        cg_ne_batched(ctx, pars, U64, bs, xs, tol=1e-14, maxit=iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / iters
        table.append(dict(c, ms=ms))
        if verbose:
            print(f"batch tune {prec} Ls={Ls} nrhs={n} {c}: {ms:.3f} ms per iteration", flush=True)
        if best is None or ms < best[1]:
            best = (c, ms)
    for x in xs:
        x.zero_()
    if best[0]["mode"] != mode:
        ctx.release()
    install_batched(ctx, P, Ls, best[0])
    if cache:
        save(cache, _batch_key(P, Ls, n, lattice.dims), dict(best[0], ms=best[1]))
    return best[0], best[1], table


def current_batched(ctx, prec, Ls):
    """The installed batched-solve shape."""
    P = PREC_NAMES.get(prec, prec)
    on, _, xcd, ll = dwf_tune_get(ctx, P, Ls, kernel_id=BATCH_INTERLEAVED)
    if on > 0 and Ls in (8, 16, 32):
        return {"mode": "interleaved", "spb": 1, "xcd": xcd, "ll": ll}
    spb, _, xcd, ll = dwf_tune_get(ctx, P, Ls, kernel_id=BATCH_SEPARATE)
    return {"mode": "separate", "spb": spb, "xcd": xcd, "ll": ll}
