"""The smoother studies run end to end on a small system: every point
converges, and two sweeps of each kind need no more iterations than one
(the parameters themselves are pinned to the oracle in test_gpu_parity)."""
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


def test_omega_study_points_converge():
    from paper_2103_07537_amd import studies
    rows = studies.study("omega", "2d-32", repeats=1, points=(0.6, 0.8, 1.0))
    for r in rows:
        log(f"  omega={r['params']['omega']}: {r['iterations']} its, {r['total_ms']:.1f} ms")
        assert r["converged"] and r["rel_residual"] <= 1e-8 * (1 + 1e-6)
    assert [r["params"]["omega"] for r in rows] == [0.6, 0.8, 1.0]


def test_more_sweeps_need_no_more_iterations():
    from paper_2103_07537_amd import studies
    rows = studies.study("sweeps", "2d-32", repeats=1, points=((1, 1), (2, 1), (2, 2)))
    its = [r["iterations"] for r in rows]
    log(f"  iterations {its}")
    assert all(r["converged"] for r in rows)
    assert its[1] <= its[0] and its[2] <= its[1]
    assert "| parameters |" in studies.table(rows)


def test_smoother_study_compares_both_smoothers():
    from paper_2103_07537_amd import studies
    rows = studies.study("smoother", "2d-32", repeats=1)
    assert [r["params"]["smoother"] for r in rows] == [0, 1]
    for r in rows:
        log(f"  smoother={r['params']['smoother']}: {r['iterations']} its, {r['total_ms']:.1f} ms")
        assert r["converged"] and r["rel_residual"] <= 1e-8 * (1 + 1e-6)
