"""The condition bound behind the full-size parity bars (tests/cond_bars.py)
against the exact cond_2(Q_AA) of every subdomain, from dense eigenvalues of
the oracle's Q_AA, on workloads small enough to form Q: the bound holds, is
within a small factor of the truth, and Omega_p* is the product set T_A x R
the bound assumes."""
import numpy as np
import pytest

import oracle as O
from cond_bars import cond_bound, parity_bar, U64, BAR_C
from paper_2309_05435_amd.inputs import WORKLOADS, Workload

CASES = [WORKLOADS["small"],
         Workload(name="tiles", m=20, T=6, range_=0.25, rho=0.95, tau=1.0, sigma=0.5,
                  obs_frac=0.3, n_tslabs=2, n_tiles=3, n_l=1, n_k=0, rtol=1e-12,
                  mask_seed=81, z_seed=82),
         Workload(name="tiles2", m=18, T=8, range_=0.4, rho=0.7, tau=2.0, sigma=0.3,
                  obs_frac=0.5, n_tslabs=3, n_tiles=2, n_l=2, n_k=0, rtol=1e-12,
                  mask_seed=83, z_seed=84)]


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_bound_holds_and_is_tight(wl):
    M = O.OracleModel.from_workload(wl)
    Q = M.csr(O.Q).dense()
    lab = O.grid_cores(wl.m, wl.m, wl.T, wl.n_tslabs, wl.n_tiles, wl.n_tiles)
    ns = wl.m * wl.m
    worst = 0.0
    for p in range(wl.n_tslabs * wl.n_tiles ** 2):
        st = M.subdomain_state(lab, p, wl.n_l)
        A = np.flatnonzero((st == 1) | (st == 2))
        # Omega_p* = T_A x R
        ts, ss = np.unique(A // ns), np.unique(A % ns)
        assert len(A) == len(ts) * len(ss)
        assert np.all(np.diff(ts) == 1)
        ev = np.linalg.eigvalsh(Q[np.ix_(A, A)])
        worst = max(worst, ev[-1] / ev[0])
    K = cond_bound(wl)["K"]
    assert worst <= K * (1 + 1e-10)
    assert K <= 3.0 * worst, (K, worst)  # measured 1.0-1.6x


def test_bars_of_the_full_size_workloads():
    """The bars the full-size parity tests use, 8 u max cond(Q_AA): about
    1e-9 at 64 x 64 x 32, 1e-8 at 256 x 256 x 64, 1.3e-7 at 512 x 512 x 48."""
    for name, lo, hi in [("slab64", 5e-10, 5e-9), ("tile256", 5e-9, 5e-8),
                         ("tile512", 5e-8, 5e-7)]:
        wl = WORKLOADS[name]
        b = parity_bar(wl)
        assert lo < b < hi, (name, b)
        assert b == BAR_C * U64 * cond_bound(wl)["K"]
