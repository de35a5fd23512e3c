"""Shared helpers for the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    return torch


def dev_factors(factors, dtype=None):
    torch = torch_mod()
    out = []
    for f in factors:
        t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.contiguous())
    return out


def nan_out(rows, rank):
    torch = torch_mod()
    return torch.full((rows, rank), float("nan"), dtype=torch.float32, device="cuda")


def hip_mttkrp(t, mode, dfac, bf16=False, stream=None):
    from paper_2507_15121_amd import api
    torch = torch_mod()
    rank = dfac[0].shape[1]
    out = nan_out(t.dims[mode], rank)
    f = [None if w == mode else x for w, x in enumerate(dfac)]
    if bf16:
        api.mttkrp_bf16(t, mode, f, out=out, stream=stream)
    else:
        api.mttkrp(t, mode, f, out=out, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_mttkrp(idx, val, dims, factors, mode):
    return oracle.mttkrp(idx, np.asarray(val, np.float64), dims,
                         [np.asarray(f, np.float64) for f in factors], mode)


def rel(a, b):
    return oracle.rel_fro(a, b)
