"""Device-memory plumbing around the C ABI, with torch as the allocator.

No arithmetic happens here: these helpers allocate uint8 torch tensors of the
sizes the library reports, move canonical complex128 numpy arrays to and from
the device, and call the binding's import/export entry points.
"""

from __future__ import annotations

import numpy as np
import torch

from . import wilson as w


def dims_of(field: np.ndarray) -> tuple:
    """(X, Y, Z, T) of a canonical field whose leading site axes are (T, Z, Y, X)."""
    T, Z, Y, X = field.shape[:4]
    return (X, Y, Z, T)


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """A canonical complex128 array as a contiguous device tensor."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)


class DeviceGauge:
    """Packed gauge field on the device plus its library handle."""

    def __init__(self, U: np.ndarray | torch.Tensor, prec: int, compress12: bool = False,
                 device="cuda", stream=None, eo: bool = False):
        if isinstance(U, np.ndarray):
            self.dims = dims_of(U)
            Ud = to_device(U, device)
        else:
            T, Z, Y, X = U.shape[:4]
            self.dims = (X, Y, Z, T)
            Ud = U
        self.prec = prec
        self.compress12 = bool(compress12)
        self.eo = bool(eo)
        if self.eo:  # links split by site parity (even-odd preconditioned solves)
            self.buf = torch.empty(w.wd_gauge_eo_bytes(self.dims, prec, compress12), dtype=torch.uint8,
                                   device=device)
            self.handle = w.wd_gauge_import_eo(self.dims, Ud, prec, compress12, self.buf, stream=stream)
        else:
            self.buf = torch.empty(w.wd_gauge_bytes(self.dims, prec, compress12), dtype=torch.uint8,
                                   device=device)
            self.handle = w.wd_gauge_import(self.dims, Ud, prec, compress12, self.buf, stream=stream)
        torch.cuda.current_stream(self.buf.device).synchronize()
        del Ud

    @property
    def volume(self) -> int:
        X, Y, Z, T = self.dims
        return X * Y * Z * T

    def spinor(self, nrhs: int = 1) -> torch.Tensor:
        """An uninitialised packed spinor buffer for nrhs fields."""
        return torch.empty(max(1, w.wd_spinor_bytes(self.dims, self.prec, nrhs)),
                           dtype=torch.uint8, device=self.buf.device)

    def pack(self, psi: np.ndarray | torch.Tensor, nrhs: int | None = None, stream=None) -> torch.Tensor:
        """Packed copy of canonical spinor(s) psi ([nrhs] + [T,Z,Y,X,4,3])."""
        if nrhs is None:
            nrhs = 1 if psi.ndim == 6 else psi.shape[0]
        src = to_device(psi, self.buf.device) if isinstance(psi, np.ndarray) else psi
        dst = self.spinor(nrhs)
        w.wd_spinor_import(self.handle, src, self.prec, nrhs, dst, stream=stream)
        return dst

    def unpack(self, packed: torch.Tensor, nrhs: int = 1, stream=None) -> np.ndarray:
        """Canonical complex128 numpy copy of packed spinor(s)."""
        X, Y, Z, T = self.dims
        shape = (T, Z, Y, X, 4, 3) if nrhs == 1 else (nrhs, T, Z, Y, X, 4, 3)
        out = torch.empty(shape, dtype=torch.complex128, device=self.buf.device)
        w.wd_spinor_export(self.handle, packed, self.prec, nrhs, out, stream=stream)
        return out.cpu().numpy()

    def half_spinor(self, nrhs: int = 1) -> torch.Tensor:
        """An uninitialised buffer of nrhs half spinor fields (one parity)."""
        return torch.empty(max(1, w.wd_spinor_eo_bytes(self.dims, self.prec, nrhs)),
                           dtype=torch.uint8, device=self.buf.device)

    def pack_eo(self, psi: np.ndarray | torch.Tensor, parity: int, nrhs: int | None = None,
                stream=None) -> torch.Tensor:
        """Half fields of the sites of one parity of canonical spinor(s) psi."""
        if nrhs is None:
            nrhs = 1 if psi.ndim == 6 else psi.shape[0]
        src = to_device(psi, self.buf.device) if isinstance(psi, np.ndarray) else psi
        dst = self.half_spinor(nrhs)
        w.wd_spinor_import_eo(self.handle, src, self.prec, nrhs, parity, dst, stream=stream)
        return dst

    def unpack_eo(self, packed: torch.Tensor, parity: int, nrhs: int = 1, stream=None) -> np.ndarray:
        """Canonical complex128 copy of half fields (zero on the other parity)."""
        X, Y, Z, T = self.dims
        shape = (T, Z, Y, X, 4, 3) if nrhs == 1 else (nrhs, T, Z, Y, X, 4, 3)
        out = torch.empty(shape, dtype=torch.complex128, device=self.buf.device)
        w.wd_spinor_export_eo(self.handle, packed, self.prec, nrhs, parity, out, stream=stream)
        return out.cpu().numpy()

    def close(self):
        self.handle.close()
