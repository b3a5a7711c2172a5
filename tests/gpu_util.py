"""Shared helpers for the GPU parity tests (oracle vs libmbamg on one system)."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_hierarchy(system, **kw):
    from paper_2103_07537_amd import mbamg
    return mbamg.Hierarchy(system.blocks, system.dofs, system.n_vec, **kw)


def oracle_params(**kw):
    from oracle import amg
    keep = {k: v for k, v in kw.items() if k in amg.Params.__dataclass_fields__}
    return amg.Params(**keep)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_close(got, ref, tol, what="vcycle"):
    """Element by element and as a norm: max|got - ref| <= tol max|ref| and
    ||got - ref|| <= tol ||ref||."""
    m = np.max(np.abs(ref))
    ew = np.max(np.abs(got - ref)) / (m if m > 0 else 1.0)
    nw = rel(got, ref)
    log(f"  {what}: element-wise {ew:.2e}, norm-wise {nw:.2e}")
    assert ew <= tol, f"{what}: element-wise {ew:.3e} > {tol:.1e}"
    assert nw <= tol, f"{what}: norm-wise {nw:.3e} > {tol:.1e}"
