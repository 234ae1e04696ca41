"""Shared helpers of the GPU tests (import only from tests marked gpu)."""

import ctypes

import numpy as np
import torch

import paper_1901_07294_amd.wilson as w
from paper_1901_07294_amd.buffers import DeviceGauge

PRECS = {"fp64": w.WD_FP64, "fp32": w.WD_FP32, "fp16": w.WD_FP16}
# relative tolerance against the FP64 oracle on the original FP64 inputs
TOL = {w.WD_FP64: 1e-13, w.WD_FP32: 1e-6, w.WD_FP16: 2e-3}


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def gpu_dslash(U, psi, m, prec=w.WD_FP64, c12=False, flags=0, gauge=None):
    """D psi through the C ABI: import, apply, export."""
    g = gauge or DeviceGauge(U, prec, c12)
    src = g.pack(psi)
    dst = g.spinor()
    w.dslash_apply(g.handle, m, src, dst, g.prec, flags)
    return g.unpack(dst)


class HipMem:
    """Exact-size device allocation through the HIP runtime (for range checks)."""

    _hip = None

    def __init__(self, nbytes):
        if HipMem._hip is None:
            HipMem._hip = ctypes.CDLL("libamdhip64.so")
        self.ptr = ctypes.c_void_p()
        rc = HipMem._hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes))
        assert rc == 0, f"hipMalloc failed: {rc}"
        self.nbytes = nbytes

    @property
    def value(self):
        return self.ptr.value

    def free(self):
        if self.ptr.value:
            torch.cuda.synchronize()
            HipMem._hip.hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()
