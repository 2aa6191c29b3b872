"""The FR memory-traffic calculator against §4 Table (mem_usage) and the predicted improvements."""
import os

import pytest

from paper_2003_02633_amd import fr_traffic as T
from tests.conftest import GOLDEN


def _golden():
    rows, avg, imp = {}, None, None
    for line in open(os.path.join(GOLDEN, "mem_usage.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "avg":
            avg = [float(x) for x in f[1:]]
        elif f[0] == "improvement":
            imp = [float(x) for x in f[1:]]
        else:
            rows[int(f[0])] = [float(x) for x in f[1:]]
    return rows, avg, imp


@pytest.mark.parametrize("ki,k", [(0, 3), (1, 4), (2, 5)])
def test_table_mem_usage_as_printed(ki, k):
    rows, avg, imp = _golden()
    got, (tot, gam) = T.table(k, as_printed=True)
    for step, desc, t, g in got:
        assert abs(t - rows[step][2 * ki]) <= 0.006, (k, step, t)
        assert abs(g - rows[step][2 * ki + 1]) <= 0.006, (k, step, g)
    assert abs(tot - avg[2 * ki]) <= 0.03            # the printed total sums the printed rows


@pytest.mark.parametrize("ki,k", [(0, 3), (1, 4), (2, 5)])
def test_weighted_ratio_and_improvement(ki, k):
    """the weighted Gamma and the predicted improvements follow from the listed step data (step 4
    scaling with n_s); with the printed step-4 row they would not (k = 4, 5)"""
    rows, avg, imp = _golden()
    _, (tot, gam) = T.table(k)
    assert abs(gam - avg[2 * ki + 1]) <= 0.005
    assert abs(100 * T.improvement(k) - imp[ki]) <= 0.05
    if k > 3:
        assert abs(100 * T.improvement(k, as_printed=True) - imp[ki]) > 0.3


def test_step4_counts_listed_data():
    """the listed data of step 4 (q^s in, w^s out) scale with n_s; the printed row does not"""
    for k in (3, 4, 5):
        ns = (k + 1) ** 3
        f, c = T.step_bytes(k, 4)
        assert f == c == 2 * ns * 5 * 4
    assert T.step_bytes(3, 4) == T.step_bytes(3, 4, as_printed=True)


def test_step10_is_the_flux_divergence_kernel():
    """step 10 moves exactly what the compressed flux-divergence kernel moves per element"""
    for k in (3, 4, 5):
        ns = (k + 1) ** 3
        f, c = T.step_bytes(k, 10)
        assert f == ns * 5 * 12 + ns * 5 * 4 and c == ns * 5 * 8 + ns * 5 * 4
