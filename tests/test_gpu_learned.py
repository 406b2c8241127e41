"""The learned correction of the block-Jacobi preconditioner (opts.precond =
RBMC_PC_BJ_LEARNED): its convolutions against a plain NumPy implementation of
the same network (BF16-rounded weights, FP64 arithmetic), its training on
pairs from the sampler (the held-out energy error must drop below block
Jacobi's), and flexible PCG with the safeguarded correction converging to the
same samples as the exact solve - also with arbitrary weights."""
import numpy as np
import pytest

import oracle as O
from paper_2309_05435_amd.inputs import Workload, normals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2309_05435_amd import binding as B  # noqa: E402


def say(*a):
    print(*a, flush=True)


def wl_of(m, T, P, tiles, n_l, seed=11):
    return Workload(name="t", m=m, T=T, range_=0.3, rho=0.9, tau=1.0, sigma=0.5, obs_frac=0.3,
                    n_tslabs=P, n_tiles=tiles, n_l=n_l, n_k=0, rtol=1e-10, mask_seed=seed,
                    z_seed=seed + 1)


def bf16(w):
    """round to nearest even BF16, back to float64"""
    u = np.asarray(w, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3d_ref(x, w):
    """x: (cin, T, Y, X), w: (cout, cin, 27) -> (cout, T, Y, X); zero outside."""
    cin, T, Y, X = x.shape
    xp = np.zeros((cin, T + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], T, Y, X))
    for tap in range(27):
        dt, dy, dx = tap // 9, (tap // 3) % 3, tap % 3
        sl = xp[:, dt:dt + T, dy:dy + Y, dx:dx + X]
        out += np.einsum("oc,ctyx->otyx", w[:, :, tap], sl)
    return out


def net_ref(r, u, wvec, T, Y, X):
    h = np.stack([r.reshape(T, Y, X), u.reshape(T, Y, X)])
    off = 0
    for l, (ci, co) in enumerate(B.PC_LAYERS):
        w = bf16(wvec[off:off + ci * co * 27]).reshape(co, ci, 27)
        off += ci * co * 27
        h = conv3d_ref(np.maximum(h, 0.0) if l > 0 else h, w)
    return h.reshape(-1)


def test_learned_network_matches_numpy():
    wl = wl_of(40, 9, 1, 1, 1)   # 40 x 40 x 9: ragged against the 32 x 8 x 4 tiles
    say("learned: network vs numpy")
    gm = B.Model(wl)
    rng = np.random.default_rng(3)
    w = np.concatenate([rng.standard_normal(ci * co * 27) * np.sqrt(2.0 / (ci * 27))
                        for ci, co in B.PC_LAYERS]).astype(np.float32)
    B.rbmc_precond_set_weights(gm.m, w)
    w2 = B.rbmc_precond_get_weights(gm.m)
    info = B.rbmc_precond_info(gm.m)
    assert np.array_equal(w2, w) and info.ready and info.usable and info.val_ratio == -1.0
    r = rng.standard_normal((3, gm.n))
    u = rng.standard_normal((3, gm.n)) * 0.5
    rd = torch.from_numpy(r).cuda()
    ud = torch.from_numpy(u).cuda()
    y = torch.empty_like(rd)
    B.rbmc_precond_apply(gm.m, rd, ud, y, 3)
    y = y.cpu().numpy()
    for k in range(3):
        ref = net_ref(r[k], u[k], w, wl.T, wl.m, wl.m)
        # FP32 activations, 27..432-term FP32 sums: ~1e-6 relative to the magnitude
        np.testing.assert_allclose(y[k], ref, rtol=0, atol=2e-5 * np.abs(ref).max())
    gm.close()


def exact_vs_pcg(gm, M, seed, tag):
    """PCG samples (plain and learned) against the oracle's exact samples."""
    z = normals((6, M.n + M.n_obs), seed)
    x_ref = M.sample(z)
    x = torch.empty((6, gm.n), dtype=torch.float64, device="cuda")
    its = {}
    for pc in (B.RBMC_PC_BJ, B.RBMC_PC_BJ_LEARNED):
        st, rep = B.rbmc_sample(gm.m, B.make_opts(6, 5000, 1e-12, precond=pc),
                                torch.from_numpy(z).cuda(), x)
        err = np.linalg.norm(x.cpu().numpy() - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
        say(f"learned ({tag}): precond {pc}: iterations {rep.pcg_it_max}, max err {err.max():.2e}")
        assert st == B.RBMC_OK and err.max() < 1e-8
        its[pc] = rep.pcg_it_max
    return its


def test_train_and_flexible_pcg():
    wl = wl_of(24, 8, 2, 2, 1)
    say("learned: training")
    gm = B.Model(wl, pc=None)   # block-Jacobi over the 8 cores
    M = O.OracleModel.from_workload(wl)
    zt = torch.from_numpy(normals((8, gm.n + gm.n_obs), 61)).cuda()
    st, loss, rep = B.rbmc_precond_train(gm.m, B.make_opts(4, 5000, 1e-10),
                                         B.make_train_opts(n_pairs=400, epochs=12, batch=8,
                                                           lr=2e-3, seed=5), zt, 8)
    say(f"learned: epoch energy ratios {np.round(loss[:-1], 4)} held-out {loss[-1]:.3f}")
    assert st == B.RBMC_OK and all(np.isfinite(loss))
    assert loss[-2] < loss[0]   # the training loss decreases
    info = B.rbmc_precond_info(gm.m)
    say(f"learned: trial iterations block Jacobi {info.trial_it_bj} ({info.trial_s_bj:.3f} s), "
        f"learned {info.trial_it_learned} ({info.trial_s_learned:.3f} s), usable {info.usable}")
    # one preconditioning step with the correction leaves less energy error
    # than block Jacobi alone on held-out pairs
    assert info.val_ratio == pytest.approx(loss[-1], rel=1e-6) and info.val_ratio < 0.95
    # the acceptance trial ran, and the correction is used only if it won it
    assert info.trial_it_bj > 0 and info.trial_it_learned > 0
    assert bool(info.usable) == (info.trial_it_learned < info.trial_it_bj
                                 and info.trial_s_learned < info.trial_s_bj)
    exact_vs_pcg(gm, M, 62, "trained")
    # on fresh right-hand sides at the trial's tolerance the accepted
    # correction generalizes (15% slack); a rejected one is plain block Jacobi
    z = torch.from_numpy(normals((8, gm.n + gm.n_obs), 64)).cuda()
    x = torch.empty((8, gm.n), dtype=torch.float64, device="cuda")
    its = {}
    for pc in (B.RBMC_PC_BJ, B.RBMC_PC_BJ_LEARNED):
        st, rep = B.rbmc_sample(gm.m, B.make_opts(8, 5000, 1e-10, precond=pc), z, x)
        assert st == B.RBMC_OK
        its[pc] = rep.pcg_it_max
    say(f"learned: fresh right-hand sides at 1e-10: iterations {its}")
    if info.usable:
        assert its[B.RBMC_PC_BJ_LEARNED] <= 1.15 * its[B.RBMC_PC_BJ]
    else:
        assert its[B.RBMC_PC_BJ_LEARNED] == its[B.RBMC_PC_BJ]
    gm.close()


def test_safeguard_with_arbitrary_weights():
    """Untrained, large random weights: the per-column energy-optimal step keeps
    every preconditioning step no worse than block Jacobi, so flexible PCG
    still reaches the exact samples."""
    wl = wl_of(20, 6, 2, 1, 1, seed=13)
    say("learned: arbitrary weights")
    gm = B.Model(wl, pc=None)
    M = O.OracleModel.from_workload(wl)
    rng = np.random.default_rng(8)
    w = np.concatenate([rng.standard_normal(ci * co * 27) * np.sqrt(2.0 / (ci * 27)) * 10.0
                        for ci, co in B.PC_LAYERS]).astype(np.float32)
    B.rbmc_precond_set_weights(gm.m, w)
    exact_vs_pcg(gm, M, 63, "arbitrary")
    gm.close()
