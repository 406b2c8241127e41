"""The windowed oracle (used for sampled parity at full size) agrees with the
whole oracle model where both can be built: the estimator's entries depend
on Q only near the core, and a row of Q x only near its node."""
import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import Workload, normals
from window import core_box, estimator_entry, q_row

WL = Workload(name="w", m=30, T=12, range_=0.2, rho=0.9, tau=1.0, sigma=0.5, obs_frac=0.3,
              n_tslabs=3, n_tiles=3, n_l=1, n_k=6, rtol=1e-12, mask_seed=71, z_seed=72)


@pytest.fixture(scope="module")
def full():
    M = O.OracleModel.from_workload(WL)
    lab = O.grid_cores(WL.m, WL.m, WL.T, WL.n_tslabs, WL.n_tiles, WL.n_tiles)
    return M, lab, WL.mask()


def test_core_box_matches_labels(full):
    M, lab, mask = full
    ns = WL.m * WL.m
    for p in range(WL.n_tslabs * WL.n_tiles ** 2):
        (t0, t1), (x0, x1), (y0, y1) = core_box(WL, p)
        idx = np.flatnonzero(lab == p)
        t, r = np.divmod(idx, ns)
        y, x = np.divmod(r, WL.m)
        assert (t.min(), t.max() + 1, x.min(), x.max() + 1, y.min(), y.max() + 1) == \
            (t0, t1, x0, x1, y0, y1)
        assert len(idx) == (t1 - t0) * (x1 - x0) * (y1 - y0)


@pytest.mark.parametrize("t,x,y", [(0, 0, 0), (5, 14, 15), (11, 29, 20)])
def test_window_entry_equals_full_entry(full, t, x, y):
    M, lab, mask = full
    i = t * WL.m * WL.m + y * WL.m + x
    p = int(lab[i])
    xs = normals((WL.n_k, M.n), 5)
    a = M.entry(lab, p, WL.n_l, i, xs)
    b = estimator_entry(WL, mask, p, i, xs)
    np.testing.assert_allclose(b, a, rtol=1e-10)


def test_window_rows_of_operators(full):
    M, lab, mask = full
    xs = normals((3, M.n), 6)
    for which in (O.Q, O.DQ_LOGKAPPA, O.DQ_RHO, O.DQ_LOGSIGMA):
        y = M.apply(which, xs)
        for i in (0, 455, 901, M.n - 1, 5 * 900 + 14 * 30 + 29):
            np.testing.assert_allclose(q_row(WL, mask, which, i, xs), y[:, i], rtol=1e-12,
                                       atol=1e-12 * np.abs(y).max())
