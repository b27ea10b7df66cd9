"""The allocation-free critic entry point (cyrus_critic_evaluate_noalloc):
its per-row target scratch lives in a static device array instead of the
handle's workspace. Two calls in a row on one GPU, the second with fewer
rows, each checked against cyrus_critic_evaluate on the same inputs (same
kernels, so bit for bit) and against the FP64 oracle; rows beyond the
scratch limit are refused before anything is enqueued."""
import numpy as np
import pytest

import oracle
from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl

pytestmark = pytest.mark.gpu


def _pass(cfg, wseed, bseed, seed, episode):
    import torch
    actor, q, qt = wl.make_critic_weights(cfg, wseed)
    batch = wl.make_critic_batch(cfg, bseed)
    cr = cyrus.Critic(cfg, actor, q, qt)
    dev = cyrus.critic_batch_to_device(batch)
    q0, qh0, l0 = (x.clone() for x in cr.evaluate(dev, seed, episode))
    torch.cuda.synchronize()
    q1, qh1, l1 = cr.evaluate_noalloc(dev, seed, episode)
    torch.cuda.synchronize()
    q0, qh0, l0, q1, qh1, l1 = (x.cpu().numpy() for x in (q0, qh0, l0, q1, qh1, l1))
    print(f"[noalloc] H={cfg.num_samples} M={cfg.num_minislots}: loss {l1} (workspace path {l0})", flush=True)
    assert np.array_equal(q1, q0) and np.array_equal(qh1, qh0) and np.array_equal(l1, l0)
    oq, oqhat, _, oloss = oracle.critic_evaluate(cfg.num_ue, cfg.num_minislots, actor, q, qt, *batch, seed, episode,
                                                 cfg.discount, cfg.entropy_coef)
    assert (np.abs(q1 - oq) / np.maximum(1.0, np.abs(oq))).max() < 1e-4
    assert np.abs(qh1 - oqhat).max() < 1e-3
    assert (np.abs(l1 - oloss) / np.maximum(1e-6, np.abs(oloss))).max() < 1e-3
    cr.close()


def test_noalloc_matches_workspace_path_twice():
    big = wl.CriticConfig(num_ue=8, max_arrival=3, num_minislots=7, num_samples=300, actor_hidden=(256, 256),
                          critic_hidden=(256, 256), discount=0.9, entropy_coef=0.05)
    small = wl.CriticConfig(num_ue=4, max_arrival=2, num_minislots=7, num_samples=37, actor_hidden=(128,),
                            critic_hidden=(256, 128), discount=0.95, entropy_coef=0.1)
    _pass(big, 81, 82, 3, 4)
    _pass(small, 83, 84, 5, 6)


def test_noalloc_refuses_rows_beyond_the_scratch():
    cfg = wl.CriticConfig(num_ue=4, max_arrival=2, num_minislots=7, num_samples=9400, actor_hidden=(128,),
                          critic_hidden=(128,), discount=0.9, entropy_coef=0.1)  # 65,800 rows > 65,536
    actor, q, qt = wl.make_critic_weights(cfg, 1)
    cr = cyrus.Critic(cfg, actor, q, qt)
    dev = cyrus.critic_batch_to_device(wl.make_critic_batch(cfg, 2))
    with pytest.raises(cyrus.CyrusError) as ei:
        cr.evaluate_noalloc(dev, 1, 1)
    assert ei.value.status == -2
    cr.close()
