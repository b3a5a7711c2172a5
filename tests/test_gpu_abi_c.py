"""The C-ABI from a plain HIP program (tests/abi_driver.cpp, built by
__graft_entry__.build()), with no Python or torch in the process: host-resident
blocks, device vectors allocated by the program, aliased V-cycle arguments
rejected, and the V-cycle and the solve equal to the ones the Python binding
gets from the same library, and the V-cycle to the oracle's."""
import os
import subprocess

import numpy as np
import pytest

from gpu_util import assert_close, gpu_hierarchy, log, torch_dev
from paper_2103_07537_amd.inputs import make_system, workload

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "abi_driver")


def _write_system(s, path):
    with open(path, "wb") as f:
        np.array([0x4d42414d, 2, s.dofs[0], s.dofs[1], s.n_vec[0], s.n_vec[1]], dtype=np.int32).tofile(f)
        for fi in range(2):
            for g in range(2):
                B = s.blocks[fi][g]
                nnzb = int(B.col_idx.shape[0])
                np.array([B.n_brows, B.n_bcols, s.dofs[fi], s.dofs[g]], dtype=np.int32).tofile(f)
                np.array([nnzb], dtype=np.int64).tofile(f)
                np.ascontiguousarray(B.row_ptr, dtype=np.int32).tofile(f)
                np.ascontiguousarray(B.col_idx, dtype=np.int32).tofile(f)
                np.ascontiguousarray(B.vals, dtype=np.float64).tofile(f)
        np.array([s.b.shape[0]], dtype=np.int64).tofile(f)
        np.ascontiguousarray(s.b, dtype=np.float64).tofile(f)


CASES = {
    "2d-32": lambda: workload("2d-32", seed=1),
    "3d-11-lognormal": lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal"),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_c_program_matches_the_binding_and_the_oracle(case, precision, tmp_path):
    from oracle import amg
    assert os.path.exists(DRIVER), "tests/_build/abi_driver is missing: run __graft_entry__.build()"
    s = CASES[case]()
    sysf, outf = tmp_path / "system.bin", tmp_path / "out.bin"
    _write_system(s, sysf)
    log(f"case={case} precision={precision}: running the C driver")
    p = subprocess.run([DRIVER, str(sysf), str(outf), str(precision)], capture_output=True, text=True, timeout=120)
    log(f"  driver: {p.stdout.strip()} {p.stderr.strip()}")
    assert p.returncode == 0, p.stderr
    out = np.fromfile(outf, dtype=np.float64)
    n = s.b.shape[0]
    z_c, x_c = out[:n], out[n:]
    its_c = int(p.stdout.split("iterations")[1].split()[0])
    # the same library through the Python binding
    hg = gpu_hierarchy(s, precision=precision)
    z = torch_dev(np.zeros(n))
    hg.vcycle(torch_dev(s.b), z)
    x = torch_dev(np.zeros(n))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    assert its_c == info["iterations"]
    assert_close(z_c, z.cpu().numpy(), 1e-14, "V-cycle, C program against the binding")
    assert_close(x_c, x.cpu().numpy(), 1e-14, "solution, C program against the binding")
    if precision == 0:
        ho = amg.setup(s.blocks, s.dofs, amg.Params(), n_vec=s.n_vec)
        assert_close(z_c, amg.vcycle(ho, s.b), 1e-12, "V-cycle, C program against the oracle")
    res = np.linalg.norm(s.b - s.to_scipy() @ x_c) / np.linalg.norm(s.b)
    assert res <= 1e-8 * (1 + 1e-6)
    hg.close()
