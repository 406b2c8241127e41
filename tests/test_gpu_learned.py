"""The learned correction of the block-Jacobi preconditioner (opts.precond =
RBMC_PC_BJ_LEARNED): its convolutions against a plain NumPy implementation of
the same network (BF16-rounded weights, FP64 arithmetic), its training on
pairs from the sampler, and flexible PCG with it converging to the same
samples as the exact solve."""
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


def net_ref(r, wvec, T, Y, X):
    h = r.reshape(1, T, Y, X)
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
    w2, usable, err = B.rbmc_precond_get_weights(gm.m)
    assert np.array_equal(w2, w) and usable
    r = rng.standard_normal((3, gm.n))
    rd = torch.from_numpy(r).cuda()
    y = torch.empty_like(rd)
    B.rbmc_precond_apply(gm.m, rd, y, 3)
    y = y.cpu().numpy()
    for k in range(3):
        ref = net_ref(r[k], w, wl.T, wl.m, wl.m)
        # FP32 activations, 27..432-term FP32 sums: ~1e-6 relative to the magnitude
        np.testing.assert_allclose(y[k], ref, rtol=0, atol=2e-5 * np.abs(ref).max())
    gm.close()


def test_train_and_flexible_pcg():
    wl = wl_of(24, 8, 2, 2, 1)
    say("learned: training")
    gm = B.Model(wl, pc=None)   # block-Jacobi over the 8 cores
    M = O.OracleModel.from_workload(wl)
    zt = torch.from_numpy(normals((4, gm.n + gm.n_obs), 61)).cuda()
    st, loss, rep = B.rbmc_precond_train(gm.m, B.make_opts(4, 5000, 1e-10),
                                         B.make_train_opts(n_pairs=200, epochs=4, batch=8,
                                                           lr=2e-3, seed=5, crop_t=4,
                                                           crop_xy=12), zt, 4)
    say(f"learned: epoch losses {np.round(loss[:-1], 4)} held-out rel err {loss[-1]:.3f}")
    assert all(np.isfinite(loss))
    assert loss[-2] < loss[0]   # the training loss decreases
    # flexible PCG with the correction reaches the exact samples
    z = normals((6, M.n + M.n_obs), 62)
    x_ref = M.sample(z)
    x = torch.empty((6, gm.n), dtype=torch.float64, device="cuda")
    for pc in (B.RBMC_PC_BJ, B.RBMC_PC_BJ_LEARNED):
        st, rep = B.rbmc_sample(gm.m, B.make_opts(6, 5000, 1e-12, precond=pc), torch.from_numpy(z).cuda(), x)
        err = np.linalg.norm(x.cpu().numpy() - x_ref, axis=1) / np.linalg.norm(x_ref, axis=1)
        say(f"learned: precond {pc}: iterations {rep.pcg_it_max}, max err {err.max():.2e}")
        assert st == B.RBMC_OK and err.max() < 1e-8
    gm.close()
