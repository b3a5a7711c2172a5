"""The allocation-free gradient entry point against the allocating one.

mbamg_mlp_loss_grad_noalloc keeps its partial sums in a static per-device
buffer; with the same grid and summation order as mbamg_mlp_loss_grad its loss
and gradient must be the same bit for bit.  Two calls in a row, the second on
a smaller batch (fewer workgroups: the first call's partial sums stay in the
buffer beyond what the second reads), and a third larger one after it.  Both
are also checked against the bfloat16-emulating oracle."""
import numpy as np
import pytest

from gpu_util import log, rel, torch_dev

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    X = np.random.default_rng(seed).standard_normal((n, 12)).astype(np.float32)
    T = np.stack([np.random.default_rng(seed + 1).uniform(0, 0.8, n),
                  np.random.default_rng(seed + 2).uniform(0.3, 1.3, n)], 1).astype(np.float32)
    return X, T


def test_noalloc_gradient_matches_the_allocating_entry_point():
    import torch
    from oracle import learned
    from paper_2103_07537_amd import mbamg
    th = learned.init_params(7)
    th[4992:5122] = np.random.default_rng(8).standard_normal(130) * 0.3
    th = th.astype(np.float32)
    P = torch_dev(th)
    for n, seed in [(20000, 11), (300, 21), (70000, 31)]:
        X, T = _batch(n, seed)
        Xd, Td = torch_dev(X), torch_dev(T)
        g_ref = torch.zeros(5122, dtype=torch.float32, device="cuda")
        l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
        g_new = torch.full((5122,), float("nan"), dtype=torch.float32, device="cuda")
        l_new = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        log(f"  no-alloc gradient: n={n}")
        mbamg.mlp_loss_grad(P, Xd, Td, g_ref, l_ref)
        mbamg.mlp_loss_grad_noalloc(P, Xd, Td, g_new, l_new)
        torch.cuda.synchronize()
        a, b = g_new.cpu().numpy(), g_ref.cpu().numpy()
        assert np.array_equal(a, b), f"n={n}: max |diff| {np.abs(a - b).max():.3e}"
        assert l_new.item() == l_ref.item()
        L, g = learned.loss_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), emulate=True)
        log(f"    loss {l_new.item():.6e} (oracle {L:.6e}), grad rel {rel(a, g):.2e}")
        assert abs(l_new.item() - L) <= 1e-5 * abs(L)
        assert rel(a, g) <= 1e-4


def test_noalloc_gradient_rejects_an_empty_batch():
    import torch
    from paper_2103_07537_amd import mbamg
    z = torch.zeros(16, dtype=torch.float32, device="cuda")
    code = mbamg.lib().mbamg_mlp_loss_grad_noalloc(z.data_ptr(), z.data_ptr(), z.data_ptr(), 0, z.data_ptr(),
                                                   z.data_ptr(), None)
    assert code == -1 and b"bad argument" in mbamg.lib().mbamg_last_error()
