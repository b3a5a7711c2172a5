"""Every kernel form of the setup computes the same sums in the same order, so
hierarchies built under each forced form are bit-identical to the default
choice (which the oracle tests pin):

- smoothed prolongator: one thread per row with the row in registers, the
  generic one-thread form, one wavefront per row;
- numeric Galerkin product: one thread per output block (with 1, 2 or 4 row
  entries' lookups in flight), one lane per entry, one launch for the block
  pairs that share their patterns;
- aggregate member lists: one lane per aggregate, one wavefront per aggregate;
- product pattern: one thread per row (registers), one wavefront per row (LDS
  hash set); a forced thread form falls back where a row overflows.

The solve-phase forms that change the summation order (the row form of the
coarse-level smoother, the restriction's lane-group size) are pinned to the
oracle's V-cycle instead.
"""
import numpy as np
import pytest

from gpu_util import gpu_hierarchy, log
from paper_2103_07537_amd.inputs import make_system

pytestmark = pytest.mark.gpu


def weights_fn(level, n_agg, F):
    k = np.arange(n_agg)
    return 0.1 + 0.6 * ((k * 37 + level) % 11) / 10.0, 0.5 + 0.5 * ((k * 13 + 3 * level) % 7) / 6.0


CASES = {
    "3d-20-lognormal": lambda: make_system(20, 3, 2.0, seed=21, kappa="lognormal"),
    "2d-96-lognormal": lambda: make_system(96, 2, 5.0, seed=22, kappa="lognormal"),
}

FORMS = [("MBAMG_SA_FORM", "thread"), ("MBAMG_SA_FORM", "wave"), ("MBAMG_SA_FORM", "generic"),
         ("MBAMG_SPGEMM_FORM", "block"), ("MBAMG_SPGEMM_FORM", "entry"), ("MBAMG_SPGEMM_FORM", "fused"),
         ("MBAMG_SPGEMM_FORM", "chunk2"), ("MBAMG_SPGEMM_FORM", "chunk4"),
         ("MBAMG_SORT_FORM", "thread"), ("MBAMG_SORT_FORM", "wave"),
         ("MBAMG_SYM_FORM", "thread"), ("MBAMG_SYM_FORM", "wave")]


def _snapshot(h):
    out = []
    L = h.num_levels()
    for l in range(L):
        if l + 1 < L:
            out.append(h.aggregates(l))
        for f in range(2):
            for g in range(2):
                out.extend(h.level_block(l, f, g))
    return out


@pytest.fixture(scope="module", params=list(CASES))
def ref(request):
    s = CASES[request.param]()
    log(f"case={request.param} N={s.N}")
    h = gpu_hierarchy(s, weights=weights_fn, judge=0, max_coarse=60)
    snap = _snapshot(h)
    log(f"  {h.num_levels()} levels")
    h.close()
    return s, snap


@pytest.mark.parametrize("var,form", FORMS)
def test_kernel_form_is_bit_identical(ref, var, form, monkeypatch):
    s, snap = ref
    monkeypatch.setenv(var, form)
    log(f"  {var}={form}")
    h = gpu_hierarchy(s, weights=weights_fn, judge=0, max_coarse=60)
    got = _snapshot(h)
    h.close()
    assert len(got) == len(snap)
    for a, b in zip(got, snap):
        assert a.dtype == b.dtype and a.shape == b.shape
        assert a.tobytes() == b.tobytes()


# The row form (one wavefront per row on coarse levels, or four for long rows)
# sums each row in a different order from the sliced form, so it is pinned to
# the oracle instead: forced onto every coarse level with either split, FP64
# cycles within 1e-12, FP32 within 1e-5.
ROW_CASES = {
    "3d-lognormal-weighted": (lambda: make_system(11, 3, 2.0, seed=5, kappa="lognormal"), True),
    "2d-fixed": (lambda: make_system(40, 2, 0.7, seed=3), False),
}


@pytest.mark.parametrize("case", list(ROW_CASES))
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("split", ["1", "4"])
def test_row_form_matches_oracle(case, precision, split, monkeypatch):
    from oracle import amg
    from gpu_util import assert_close, torch_dev
    make, weighted = ROW_CASES[case]
    s = make()
    kw = dict(weights=weights_fn, judge=0) if weighted else {}
    okw = dict(weights=weights_fn) if weighted else {}
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60, **okw), n_vec=s.n_vec)
    monkeypatch.setenv("MBAMG_ROWS_FORM", "rows")
    monkeypatch.setenv("MBAMG_ROW_SPLIT", split)   # wavefronts per row (4: 4 x 4 blocks only)
    hg = gpu_hierarchy(s, max_coarse=60, precision=precision, **kw)
    log(f"case={case} precision={precision} split={split} levels={hg.num_levels()}")
    assert hg.num_levels() == len(ho.levels) >= 3
    r = np.random.default_rng(7).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5)
    x = torch_dev(np.zeros(s.n_dofs))
    info = hg.solve(torch_dev(s.b), x, rtol=1e-8)
    A = s.to_scipy()
    assert info["converged"]
    assert np.linalg.norm(s.b - A @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(s.b) * (1 + 1e-6)
    hg.close()


# The tentative restriction gives each coarse row a group of 4, 8, 16 or 64
# lanes and adds the group's partial sums in a tree, so each group size sums
# in its own order: every one is pinned to the oracle's V-cycle (FP64, 1e-12),
# including the sizes the test systems' aggregates would not select.
@pytest.mark.parametrize("group", [4, 8, 16, 64])
def test_restriction_groups_match_oracle(group, monkeypatch):
    from oracle import amg
    from gpu_util import assert_close, torch_dev
    s = make_system(11, 3, 2.0, seed=5, kappa="lognormal")
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60), n_vec=s.n_vec)
    monkeypatch.setenv("MBAMG_RESTRICT_GROUP", str(group))
    hg = gpu_hierarchy(s, max_coarse=60)
    log(f"group={group} levels={hg.num_levels()}")
    assert hg.num_levels() == len(ho.levels) >= 3
    r = np.random.default_rng(8).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12)
    hg.close()


# The smoothed restriction runs on P^T sliced over the next level's rows in
# natural order, or, for small next levels, one wavefront per row: the two
# forms sum in different orders, and both are pinned to the oracle's V-cycle,
# on a 3D case (4 x 4 blocks, the 16-byte row reads) and a 2D one (3 x 3).
@pytest.mark.parametrize("form", ["rows", "sliced"])
@pytest.mark.parametrize("case", ["3d", "2d"])
@pytest.mark.parametrize("precision", [0, 1])
def test_smoothed_restriction_forms_match_oracle(form, case, precision, monkeypatch):
    from oracle import amg
    from gpu_util import assert_close, torch_dev
    s = make_system(11, 3, 2.0, seed=5, kappa="lognormal") if case == "3d" else make_system(30, 2, 0.9, seed=4)
    ho = amg.setup(s.blocks, s.dofs, amg.Params(max_coarse=60, weights=weights_fn), n_vec=s.n_vec)
    monkeypatch.setenv("MBAMG_XFER_FORM", form)
    hg = gpu_hierarchy(s, max_coarse=60, precision=precision, weights=weights_fn, judge=0)
    log(f"form={form} case={case} precision={precision} levels={hg.num_levels()}")
    assert hg.num_levels() == len(ho.levels) >= 3
    r = np.random.default_rng(9).standard_normal(s.n_dofs)
    z = torch_dev(np.zeros(s.n_dofs))
    hg.vcycle(torch_dev(r), z)
    assert_close(z.cpu().numpy(), amg.vcycle(ho, r), 1e-12 if precision == 0 else 1e-5)
    hg.close()
