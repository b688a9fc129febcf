"""Device buffers in the packed layouts of include/dwf.h, backed by torch tensors.

Natural layouts (complex128): gauge [4][T][Z][Y][X][3][3], 5D [Ls][T][Z][Y][X][4][3].
Packing and unpacking run in the library's kernels; this module only sizes
and allocates the byte buffers.
"""
import numpy as np

from . import (FP64, KIND_EVEN, KIND_FULL, KIND_GAUGE, KIND_ODD, dwf_field_bytes, dwf_pack, dwf_unpack,
               params)


def _torch():
    import torch
    return torch


class Lattice:
    """One 4D lattice and fifth-dimension extent with its operator parameters."""

    def __init__(self, ctx, dims, Ls, M5=1.8, mass=0.01, b=1.0, c=0.0, tbc=0, device="cuda", b_s=None, c_s=None):
        self.ctx, self.dims, self.Ls = ctx, tuple(int(d) for d in dims), int(Ls)
        self.M5, self.mass, self.b, self.c, self.tbc = float(M5), float(mass), float(b), float(c), int(tbc)
        self.b_s = None if b_s is None else np.asarray(b_s, dtype=np.float64)
        self.c_s = None if c_s is None else np.asarray(c_s, dtype=np.float64)
        self.device = device

    def params(self, prec=FP64, prec_inner=FP64, **kw):
        d = dict(dims=self.dims, Ls=self.Ls, M5=self.M5, mass=self.mass, b=self.b, c=self.c, tbc=self.tbc,
                 prec=prec, prec_inner=prec_inner, b_s=self.b_s, c_s=self.c_s)
        d.update(kw)
        return params(**d)

    def with_(self, **kw):
        d = dict(dims=self.dims, Ls=self.Ls, M5=self.M5, mass=self.mass, b=self.b, c=self.c, tbc=self.tbc,
                 b_s=self.b_s, c_s=self.c_s)
        if "Ls" in kw and "b_s" not in kw and "c_s" not in kw:
            d["b_s"] = d["c_s"] = None  # coefficient arrays belong to one fifth-dimension extent
        d.update(kw)
        return Lattice(self.ctx, device=self.device, **d)

    def bytes(self, kind, prec=FP64):
        return dwf_field_bytes(self.params(prec), kind, prec)

    def empty(self, kind, prec=FP64):
        torch = _torch()
        n = self.bytes(kind, prec)
        if n == 0:
            raise ValueError("invalid lattice parameters")
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def zeros(self, kind, prec=FP64):
        t = self.empty(kind, prec)
        t.zero_()
        return t

    def to_device(self, a):
        torch = _torch()
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
        return a.to(self.device, dtype=torch.complex128).contiguous()

    def pack_gauge(self, U, prec=FP64):
        Ud = self.to_device(U)
        out = self.empty(KIND_GAUGE, prec)
        dwf_pack(self.ctx, self.params(prec), KIND_GAUGE, prec, Ud, out)
        return out

    def pack(self, psi, kind=KIND_FULL, prec=FP64):
        pd = self.to_device(psi)
        out = self.empty(kind, prec)
        dwf_pack(self.ctx, self.params(prec), kind, prec, pd, out)
        return out

    def unpack(self, packed, kind=KIND_FULL, prec=FP64):
        torch = _torch()
        X, Y, Z, T = self.dims
        nat = torch.zeros((self.Ls, T, Z, Y, X, 4, 3), dtype=torch.complex128, device=self.device)
        dwf_unpack(self.ctx, self.params(prec), kind, prec, packed, nat)
        return nat

    def unpack_np(self, packed, kind=KIND_FULL, prec=FP64):
        _torch().cuda.synchronize()
        return self.unpack(packed, kind, prec).cpu().numpy()


__all__ = ["Lattice", "KIND_EVEN", "KIND_ODD", "KIND_FULL", "KIND_GAUGE"]
