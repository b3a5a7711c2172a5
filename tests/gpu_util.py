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
