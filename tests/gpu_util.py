"""Helpers for the GPU parity tests: device context, user-order <-> internal-order transfers, and the
error measures the parity bars are stated in (max-norm relative error per output array)."""
import numpy as np

from paper_2603_15920_amd import binding as B


def torch():
    import torch as _t
    return _t


_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = B.Context(0)
    return _CTX


def note(*a):
    print("[gpu]", *a, flush=True)


def dev(a, dtype=None):
    t = torch()
    a = np.ascontiguousarray(a)
    return t.from_numpy(a).to(device="cuda:0", dtype=dtype or t.float64)


def host(t):
    return t.detach().cpu().numpy()


def to_int(M, a, kind, dtype=None):
    """numpy user-order array -> device tensor in internal order"""
    return M.to_internal(dev(a, dtype), kind)


def to_user(M, t, kind):
    return host(M.to_user(t, kind))


def rel_err(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (scale if scale > 0 else 1.0))


def empty(shape, dtype=None):
    t = torch()
    return t.empty(shape, dtype=dtype or t.float64, device="cuda:0")
