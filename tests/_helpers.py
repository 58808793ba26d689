"""Shared helpers of the GPU parity tests (comparison metrics, device transfer)."""
import numpy as np

import oracle


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def componentwise(got, ref, scale):
    """max |got - ref| / scale over entries with scale > 0 (0 if none)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    err = np.abs(got - ref)
    pos = scale > 0
    if np.any(~pos & (err > 0)):
        return np.inf
    return float(np.max(err[pos] / scale[pos])) if np.any(pos) else 0.0


def gemm_scale(A, B, opA=0, opB=0):
    """(|A| |B|)_ij in float64, the componentwise error scale of a matrix product."""
    return oracle.gemm(np.abs(A), np.abs(B), opA, opB)


def gemm_scale_sampled(A, B, rows, cols):
    return oracle.gemm_sampled(np.abs(A), np.abs(B), rows, cols)


def stencil_scale(img, w, pad):
    return oracle.stencil2d(np.abs(img), np.abs(w), pad)
