"""Shared helpers of the GPU parity tests: the HIP path via its C ABI binding,
the oracle on the CPU, identical seeded inputs from ``synth``."""
import numpy as np

import synth


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def mask(psi, dims, parity):
    out = np.array(psi, copy=True)
    out[:, synth.parity_array(dims) != parity] = 0
    return out


def gpu_ctx():
    import torch
    import paper_1111_5059_amd as dwf
    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    dwf.lib()
    return dwf, dwf.Context()


PREC_TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 4e-3, "bf16": 3e-2}
