"""The byte model behind the bench's bandwidth figures, checked through the
C-ABI.  The operator apply's bytes against a closed form recomputed from the
finest level's blocks (every nonzero entry and stored block of both block
rows, a 4-byte row entry per node, x_f, x_g and the result); and the
bookkeeping: under per-launch timing one V-cycle's launches add up, level by
level, to `mbamg_level_vcycle_bytes`, the levels to `mbamg_vcycle_bytes`, and
each level's colour passes are one launch per colour and block."""
import numpy as np
import pytest

from gpu_util import gpu_hierarchy, log, torch_dev
from paper_2103_07537_amd.inputs import make_system

pytestmark = pytest.mark.gpu

CASES = {
    "2d-23": lambda: make_system(23, 2, 0.7, seed=3, kappa="lognormal", blk1_scale=2.0, a10_scale=0.5),
    "3d-11": lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal", blk1_scale=0.5, a10_scale=1.5),
}
TK_LEVEL = 16   # level l: TK_LEVEL + 2 l (down), TK_LEVEL + 2 l + 1 (up)


def weights_fn(level, n_agg, F):
    k = np.arange(n_agg)
    return 0.1 + 0.6 * ((k * 37 + level) % 11) / 10.0, 0.5 + 0.5 * ((k * 13 + 3 * level) % 7) / 6.0


def launch_kind(l, k):
    return k if l == 0 else 64 + 8 * l + k


@pytest.mark.parametrize("case", list(CASES))
def test_apply_bytes_follow_the_closed_form(case):
    s = CASES[case]()
    hg = gpu_hierarchy(s, max_coarse=60)
    expected = 0
    for f in range(2):
        n_f, d_f = hg.block_nodes(0, f), s.dofs[f]
        for g in range(2):
            rp, ci, v = hg.level_block(0, f, g)
            nnzb = int(rp[-1])
            expected += 8 * int(np.count_nonzero(v[:nnzb * d_f * s.dofs[g]])) + 4 * nnzb
        expected += 4 * n_f + 3 * n_f * d_f * 8          # row entries; x_f, x_g gathered, result
    x = torch_dev(np.random.default_rng(81).standard_normal(s.n_dofs))
    w = torch_dev(np.zeros(s.n_dofs))
    hg.timing_enable(1)
    hg.apply(x, w)
    st = hg.timing_get(2)
    log(f"  {case}: apply {st['bytes']:.0f} B, closed form {expected} B")
    assert st["launches"] == 1 and st["bytes"] == expected
    hg.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("form", ["fp64", "fp32", "weighted"])
def test_launch_bytes_add_up_to_the_level_and_cycle_model(case, form):
    s = CASES[case]()
    kw = dict(max_coarse=60)
    if form == "fp32":
        kw["precision"] = 1
    if form == "weighted":
        kw.update(weights=weights_fn, judge=0)
    hg = gpu_hierarchy(s, **kw)
    L = hg.num_levels()
    assert L >= 3
    r = torch_dev(np.random.default_rng(82).standard_normal(s.n_dofs))
    z = torch_dev(np.zeros(s.n_dofs))
    hg.timing_enable(1)
    hg.vcycle(r, z)
    total = 0.0
    for l in range(L):
        down, up = hg.level_vcycle_bytes(l)
        total += down + up
        seg_d, seg_u = hg.timing_get(TK_LEVEL + 2 * l), hg.timing_get(TK_LEVEL + 2 * l + 1)
        if l == L - 1:
            assert up == 0.0 and seg_d["bytes"] == down
            continue
        assert seg_d["bytes"] == down and seg_u["bytes"] == up
        got = sum(hg.timing_get(launch_kind(l, k))["bytes"] for k in (0, 1, 3, 5, 6))
        log(f"  {case} {form} level {l}: launches {got:.0f} B, model {down + up:.0f} B")
        assert abs(got - (down + up)) <= 1e-12 * (down + up)
        # one launch per colour and block in each sweep: the pre-smoother's passes
        # start from zero (kind 3), the post-smoother's carry the coupling term (kind 0)
        colours = sum(int(hg.colours(l, f).max()) + 1 for f in range(2))
        assert hg.timing_get(launch_kind(l, 0))["launches"] == colours
        assert hg.timing_get(launch_kind(l, 3))["launches"] == colours
        for k in (1, 5, 6):
            assert hg.timing_get(launch_kind(l, k))["launches"] == 1
    assert abs(hg.vcycle_bytes() - total) <= 1e-12 * total
    hg.close()
