"""Helpers for the GPU parity tests: run the library through the C ABI on cuda:0."""

import numpy as np

import paper_2112_00864_amd as bcv


def rel_l2(leaves, u, ref):
    """Relative L2(Omega) error of cell averages u/|w| against ref/|w| (the paper's norm)."""
    vol = np.ldexp(1.0, -3 * np.asarray(leaves)[:, 0].astype(np.int32))
    return float(np.sqrt(np.sum(vol * ((u - ref) / vol) ** 2) / np.sum(vol * (ref / vol) ** 2)))


def gpu_apply(plan, f, parts=None):
    import torch

    fd = torch.tensor(np.asarray(f, dtype=np.float64), device="cuda:0")
    ud = torch.full_like(fd, float("nan"))
    if parts is None:
        bcv.vtv_apply(plan, fd, ud)
    else:
        bcv.vtv_apply_parts(plan, fd, ud, parts)
    torch.cuda.synchronize()
    return ud.cpu().numpy()
