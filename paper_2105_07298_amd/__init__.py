"""fwapsp: blocked Floyd-Warshall all-pairs shortest paths on MI355X (gfx950).

The computation lives in the HIP library libfwapsp.so (C ABI in include/fw_apsp.h);
this package is its Python face:
  * the C entry points under the same names (argument marshalling only), and
  * PyTorch conveniences that allocate device tensors and pass the current stream.
PyTorch provides device memory and streams only; no step of the method runs in it.
"""
from __future__ import annotations

from ._lib import (FW_EHIP, FW_EINVAL, FW_ENOMEM, FW_EUNSUPPORTED, FW_F32, FW_F64, FW_OK,  # noqa: F401
                   FwError, fw_apsp, fw_apsp_backward, fw_apsp_batched, fw_apsp_config, fw_last_error,
                   fw_prof_enable, fw_prof_read, fw_status_string, fw_version, lib)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return FW_F32
    if t.dtype == torch.float64:
        return FW_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _stream_ptr(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def apsp_(D, P=None, block: int = 0, tile: int = 0):
    """In-place APSP of the square device tensor D (float32/float64, contiguous).

    D holds the weight matrix (0 diagonal, +inf = no edge) and is overwritten with
    shortest distances; P (int32, same shape) receives the path matrix if given.
    Runs on the current stream of D's device.
    """
    import torch
    if not (D.is_cuda and D.dim() == 2 and D.shape[0] == D.shape[1] and D.is_contiguous()):
        raise ValueError("D must be a contiguous square device tensor")
    n = D.shape[0]
    pp = None
    if P is not None:
        if not (P.is_cuda and P.dtype == torch.int32 and P.shape == D.shape and P.is_contiguous()):
            raise ValueError("P must be a contiguous int32 device tensor shaped like D")
        pp = P.data_ptr()
    fw_apsp_config(_dtype_code(D), n, D.data_ptr(), pp, block, tile, _stream_ptr(D.device))
    return D, P


def apsp(W, path: bool = True, block: int = 0, tile: int = 0):
    """Return (D, P) for the weight matrix W (device tensor; W is not modified).
    P is None when path=False."""
    import torch
    D = W.contiguous().clone()
    P = torch.empty(D.shape, dtype=torch.int32, device=D.device) if path else None
    return apsp_(D, P, block, tile)
