"""Parity of the Near-RT RIC critic pass (cyrus_critic_*, Sec. IV-B, Eqs. (3)
and (4)) with the FP64 oracle, through the C ABI.

Q values: FP32 MLPs against float64, within 1e-4 (relative to max(1, |Q|)).
Targets: they add the Gaussian draws (FP32 Box-Muller against float64) and the
sum of E log-density terms, each O(10) at most, so 1e-3 absolute. Losses: the
mean of squared differences, within 1e-3 relative. The pass is deterministic
for a given seed and episode, and a new episode gives new targets.
"""
import numpy as np
import pytest

import oracle
from paper_2506_00167_amd import cyrus
from paper_2506_00167_amd import workload as wl

pytestmark = pytest.mark.gpu


def _check(cfg, wseed, bseed, seed, episode):
    import torch
    actor, q, qt = wl.make_critic_weights(cfg, wseed)
    batch = wl.make_critic_batch(cfg, bseed)
    cr = cyrus.Critic(cfg, actor, q, qt)
    dev = cyrus.critic_batch_to_device(batch)
    gq, gqhat, gloss = cr.evaluate(dev, seed, episode)
    torch.cuda.synchronize()
    gq, gqhat, gloss = gq.cpu().numpy(), gqhat.cpu().numpy(), gloss.cpu().numpy()
    oq, oqhat, olp, oloss = oracle.critic_evaluate(cfg.num_ue, cfg.num_minislots, actor, q, qt, *batch, seed, episode,
                                                   cfg.discount, cfg.entropy_coef)
    dq = np.abs(gq - oq) / np.maximum(1.0, np.abs(oq))
    dt = np.abs(gqhat - oqhat)
    dl = np.abs(gloss - oloss) / np.maximum(1e-6, np.abs(oloss))
    print(f"[critic] {cfg}: max dq {dq.max():.2e}, max dqhat {dt.max():.2e}, loss gpu {gloss} oracle {oloss}, "
          f"max |log pi| {np.abs(olp).max():.1f}", flush=True)
    assert dq.max() < 1e-4
    assert dt.max() < 1e-3
    assert dl.max() < 1e-3
    # terminal steps are the rewards, exactly
    assert np.array_equal(gqhat[:, -1], batch[4])
    # deterministic, and the episode drives the draws
    q2, qhat2, loss2 = cr.evaluate(dev, seed, episode)
    torch.cuda.synchronize()
    assert np.array_equal(qhat2.cpu().numpy(), gqhat) and np.array_equal(loss2.cpu().numpy(), gloss)
    _, qhat3, _ = cr.evaluate(dev, seed, episode + 1)
    torch.cuda.synchronize()
    acting = batch[1][:, 1:] > 0
    assert not np.array_equal(qhat3.cpu().numpy()[:, :-1][acting], gqhat[:, :-1][acting])
    cr.close()


def test_critic_small_ragged():
    # 37 samples x 7 steps = 259 rows: whole row tiles and a ragged tail; a
    # single 128-wide actor layer takes the streamed-weight kernel
    cfg = wl.CriticConfig(num_ue=4, max_arrival=2, num_minislots=7, num_samples=37, actor_hidden=(128,),
                          critic_hidden=(256, 128), discount=0.95, entropy_coef=0.1)
    _check(cfg, 61, 62, 5, 9)


@pytest.mark.parametrize("shape", [
    # register-resident kernel with 128-wide layers (one neuron tile per
    # wave), 5E+2 = 17 inputs in two chunks, 41 x 5 = 205 rows (ragged tile)
    dict(num_ue=3, num_minislots=5, num_samples=41, actor_hidden=(128, 128), critic_hidden=(128, 128)),
    # 256-wide layers, 5E+2 = 12 inputs in one chunk, 23 x 7 = 161 rows
    dict(num_ue=2, num_minislots=7, num_samples=23),
    # widths that are multiples of 32 but not of 128 (zero-padded to 128 and
    # 256): the register-resident kernel with 96-wide layers, then the
    # streamed-weight kernel with 160- and 224-wide layers
    dict(num_ue=3, num_minislots=5, num_samples=29, actor_hidden=(96, 96), critic_hidden=(96, 96)),
    dict(num_ue=4, num_minislots=7, num_samples=17, actor_hidden=(160,), critic_hidden=(224, 32)),
])
def test_critic_register_shapes(shape):
    _check(wl.CriticConfig(**shape), 67, 68, 11, 3)


def test_critic_ric_shape():
    # the RIC's update shape: H = 256 samples, M = 7, 2 x 256 critics
    _check(wl.CRITIC_RIC, 63, 64, 0xC0FFEE, 1)


def test_critic_one_step_samples_are_rewards():
    cfg = wl.CriticConfig(num_ue=2, max_arrival=1, num_minislots=1, num_samples=19, actor_hidden=(128,),
                          critic_hidden=(128,))
    import torch
    actor, q, qt = wl.make_critic_weights(cfg, 65)
    batch = wl.make_critic_batch(cfg, 66)
    cr = cyrus.Critic(cfg, actor, q, qt)
    _, gqhat, _ = cr.evaluate(cyrus.critic_batch_to_device(batch), 1, 2)
    torch.cuda.synchronize()
    assert np.array_equal(gqhat.cpu().numpy()[:, 0], batch[4])
    cr.close()
