"""fwapsp: blocked Floyd-Warshall all-pairs shortest paths on MI355X (gfx950).

The computation lives in the HIP library libfwapsp.so (C ABI in include/fw_apsp.h);
this package is its Python face:
  * the C entry points under the same names (argument marshalling only), and
  * PyTorch conveniences that allocate device tensors and pass the current stream.
PyTorch provides device memory and streams only; no step of the method runs in it.
"""
from __future__ import annotations

from ._lib import (FW_EHIP, FW_EINPUT, FW_EINVAL, FW_ENOMEM, FW_EUNSUPPORTED, FW_F16, FW_F32, FW_F64, FW_OK,  # noqa: F401
                   FW_P4_PANELS, FW_P4_WAVEROWS, FW_SCHED_LOOKAHEAD, FW_SCHED_PAIRS, FW_SCHED_PAIRS_LOOKAHEAD, FW_SCHED_SERIAL, FwError, fw_apsp, fw_apsp_backward, fw_apsp_batched,
                   fw_apsp_batched_config, fw_apsp_batched_device, fw_apsp_batched_device_noalloc, fw_apsp_config, fw_apsp_ooc, fw_last_error, fw_list_configs, fw_ooc_superblock,
                   fw_prof_enable,
                   fw_prof_read, fw_query_config, fw_status_string, fw_validate_input, fw_version, lib, lookahead_applies,
                   pairs_applies, pairs_lookahead_applies)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return FW_F32
    if t.dtype == torch.float64:
        return FW_F64
    if t.dtype == torch.float16:
        return FW_F16
    raise TypeError(f"unsupported dtype {t.dtype} (float32, float64 or float16)")


def _stream_ptr(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def apsp_(D, P=None, block: int = 0, tile_m: int = 0, tile_n: int = 0, variant: int = 0, schedule: int = 0):
    """In-place APSP of the square device tensor D (float32/float64/float16, contiguous).

    float16 is the half-width variant: exact for integer weights when every finite
    shortest distance is below 2048.

    D holds the weight matrix (0 diagonal, +inf = no edge) and is overwritten with
    shortest distances; P (int32, same shape) receives the path matrix if given.
    Runs on the current stream of D's device.  block / tile_m / tile_n / variant /
    schedule override the tuned configuration (0 = tuned; variant FW_P4_PANELS or
    FW_P4_WAVEROWS picks the last-phase kernel, schedule FW_SCHED_SERIAL,
    FW_SCHED_LOOKAHEAD, FW_SCHED_PAIRS or FW_SCHED_PAIRS_LOOKAHEAD the round schedule).
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
    fw_apsp_config(_dtype_code(D), n, D.data_ptr(), pp, block, tile_m, tile_n, variant, schedule,
                   _stream_ptr(D.device))
    return D, P


def validate(W):
    """Check the device tensor W against the input contract (0 diagonal, weights
    >= 0 or +inf, no NaN) on the library's kernel; raises FwError (FW_EINPUT)
    naming the first offending entry.  Waits for the current stream."""
    if not (W.is_cuda and W.dim() == 2 and W.shape[0] == W.shape[1] and W.is_contiguous()):
        raise ValueError("W must be a contiguous square device tensor")
    fw_validate_input(_dtype_code(W), W.shape[0], W.data_ptr(), _stream_ptr(W.device))


def apsp(W, path: bool = True, block: int = 0, tile_m: int = 0, tile_n: int = 0, variant: int = 0,
         schedule: int = 0):
    """Return (D, P) for the weight matrix W (device tensor; W is not modified).
    P is None when path=False."""
    import torch
    D = W.contiguous().clone()
    P = torch.empty(D.shape, dtype=torch.int32, device=D.device) if path else None
    return apsp_(D, P, block, tile_m, tile_n, variant, schedule)


def apsp_ooc_(W, P=None, device_bytes: int = 0):
    """In place for a square CPU tensor W (float32/float64, contiguous; pinned
    memory lets transfers overlap the work): W becomes the distances and P (int32
    CPU tensor shaped like W, optional) the path matrix, through at most
    device_bytes of device memory (0: 90% of the free memory).  Work is ordered
    after the current stream; returns when W and P hold the results."""
    import torch
    if W.is_cuda or W.dim() != 2 or W.shape[0] != W.shape[1] or not W.is_contiguous():
        raise ValueError("W must be a contiguous square CPU tensor")
    pp = None
    if P is not None:
        if P.is_cuda or P.dtype != torch.int32 or P.shape != W.shape or not P.is_contiguous():
            raise ValueError("P must be a contiguous int32 CPU tensor shaped like W")
        pp = P.data_ptr()
    fw_apsp_ooc(_dtype_code(W), W.shape[0], W.data_ptr(), pp, device_bytes,
                torch.cuda.current_stream().cuda_stream)
    return W, P


def apsp_batched_(Dcat, ns, offsets, Pcat=None, small_max_n: int = -1, route: int = 0):
    """In-place APSP of many graphs in one persistent launch.

    Dcat: 1-D contiguous device tensor (float32/float64) holding every graph's
    n_b x n_b weight matrix row-major at element offset offsets[b]; overwritten
    with distances.  ns (int32) and offsets (int64) are host sequences of length
    batch.  Pcat (int32, same length as Dcat) receives the path matrices.
    small_max_n: graphs with n <= small_max_n use 32 x 32 tiles, the others 64 x 64
    (-1 = the tuned choice per 32-vertex size class).
    route: graphs solved by fw_apsp instead of the persistent launch (0 = those
    that would hold far more than their share of the batch's work, -1 = none,
    k > 0 = every graph with n >= k).
    """
    import numpy as np
    import torch
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    if ns.shape != offs.shape or ns.ndim != 1:
        raise ValueError("ns and offsets must be 1-D of equal length")
    if not (Dcat.is_cuda and Dcat.dim() == 1 and Dcat.is_contiguous()):
        raise ValueError("Dcat must be a contiguous 1-D device tensor")
    if (offs + ns.astype(np.int64) ** 2).max(initial=0) > Dcat.numel():
        raise ValueError("a graph extends past the end of Dcat")
    pp = None
    if Pcat is not None:
        if not (Pcat.is_cuda and Pcat.dtype == torch.int32 and Pcat.shape == Dcat.shape and Pcat.is_contiguous()):
            raise ValueError("Pcat must be a contiguous int32 device tensor shaped like Dcat")
        pp = Pcat.data_ptr()
    fw_apsp_batched_config(_dtype_code(Dcat), int(ns.size), ns.ctypes.data, offs.ctypes.data, Dcat.data_ptr(), pp,
                           small_max_n, _stream_ptr(Dcat.device), route)
    return Dcat, Pcat


def apsp_batched(Wcat, ns, offsets, path: bool = True, small_max_n: int = -1, route: int = 0):
    """(Dcat, Pcat) for a ragged batch of weight matrices (Wcat is not modified)."""
    import torch
    D = Wcat.contiguous().clone()
    P = torch.empty(D.shape, dtype=torch.int32, device=D.device) if path else None
    return apsp_batched_(D, ns, offsets, P, small_max_n, route)


def apsp_batched_device_(Dcat, n_dev, off_dev, Pcat=None):
    """apsp_batched_ with the vertex counts (int32) and element offsets (int64) as
    1-D device tensors of length batch, read by the library on the device; every
    graph runs in the persistent launch.  Graphs with n outside [1, 4096] or a
    negative offset are skipped on the device (left untouched)."""
    import torch
    if not (n_dev.is_cuda and n_dev.dtype == torch.int32 and n_dev.dim() == 1 and n_dev.is_contiguous()):
        raise ValueError("n_dev must be a contiguous 1-D int32 device tensor")
    if not (off_dev.is_cuda and off_dev.dtype == torch.int64 and off_dev.dim() == 1 and off_dev.is_contiguous()
            and off_dev.numel() >= n_dev.numel()):
        raise ValueError("off_dev must be a contiguous 1-D int64 device tensor with at least batch entries")
    if not (Dcat.is_cuda and Dcat.dim() == 1 and Dcat.is_contiguous()):
        raise ValueError("Dcat must be a contiguous 1-D device tensor")
    pp = None
    if Pcat is not None:
        if not (Pcat.is_cuda and Pcat.dtype == torch.int32 and Pcat.shape == Dcat.shape and Pcat.is_contiguous()):
            raise ValueError("Pcat must be a contiguous int32 device tensor shaped like Dcat")
        pp = Pcat.data_ptr()
    fw_apsp_batched_device(_dtype_code(Dcat), int(n_dev.numel()), n_dev.data_ptr(), off_dev.data_ptr(),
                           Dcat.data_ptr(), pp, _stream_ptr(Dcat.device))
    return Dcat, Pcat


def apsp_backward(D, P, G):
    """dL/dW from forward outputs D, P ([n, n] or [B, n, n]) and G = dL/dD (same
    shape and dtype as D), via the library's subtree-sum kernel."""
    import torch
    if D.shape != G.shape or D.shape != P.shape or D.dtype != G.dtype:
        raise ValueError("D, P and G must have the same shape; D and G the same dtype")
    if D.dim() not in (2, 3) or D.shape[-1] != D.shape[-2]:
        raise ValueError("expected [n, n] or [B, n, n]")
    Dc, Pc, Gc = D.contiguous(), P.contiguous(), G.contiguous()
    gW = torch.empty_like(Dc)
    n = D.shape[-1]
    batch = 1 if D.dim() == 2 else D.shape[0]
    fw_apsp_backward(_dtype_code(Dc), n, batch, Dc.data_ptr(), Pc.data_ptr(), Gc.data_ptr(), gW.data_ptr(),
                     _stream_ptr(D.device))
    return gW


def _forward(W):
    import numpy as np
    import torch
    if W.dim() == 2:
        return apsp(W, path=True)
    B, n = W.shape[0], W.shape[-1]
    offs = np.arange(B, dtype=np.int64) * n * n
    ns = np.full(B, n, dtype=np.int32)
    Dc, Pc = apsp_batched(W.contiguous().reshape(-1), ns, offs, path=True)
    return Dc.view(B, n, n), Pc.view(B, n, n)


def _make_function():
    import torch

    class APSP(torch.autograd.Function):
        """D = APSP(W) for W of shape [n, n] or [B, n, n] (float32/float64, device).

        Forward: fw_apsp (or fw_apsp_batched for a batch), saving D and the path
        matrix P (n^2 each; no per-k record).  Backward: fw_apsp_backward, the
        subgradient along the shortest paths P encodes.
        """

        @staticmethod
        def forward(ctx, W):
            D, P = _forward(W.detach())
            ctx.save_for_backward(D, P)
            ctx.mark_non_differentiable(P)
            return D, P

        @staticmethod
        def backward(ctx, gD, gP):
            D, P = ctx.saved_tensors
            if gD is None:
                return None
            return apsp_backward(D, P, gD)

    return APSP


_APSP = None


def apsp_autograd(W):
    """(D, P) = APSP(W) with autograd support for D (P carries no gradient)."""
    global _APSP
    if _APSP is None:
        _APSP = _make_function()
    return _APSP.apply(W)
