"""The training entry point that allocates nothing (ldgs_learned_train_noalloc,
fixed per-GPU workspace) against the allocating one (ldgs_learned_train) on
the same inputs, through the C ABI: two calls in a row, the second on a
smaller network and run, so that anything the first call left in the
workspace would show.  The two run the same kernels; the weight gradients
are accumulated with floating-point atomics, whose order varies between
runs, so the comparison allows for rounding."""
import numpy as np
import pytest

from synth.learning import batch_order, bf16_grid_values

pytestmark = pytest.mark.gpu


def _compare(d, p, crop, ncrops, batch, steps, seed):
    import torch
    from paper_1911_05888_amd import learned_train, init_net_params
    print(f"[noalloc] d={d} p={p} crop={crop} ncrops={ncrops} batch={batch} steps={steps}", flush=True)
    nb = (d + 1) * (p + 1) ** d
    chp = (nb + 1 + 7) // 8 * 8
    rng = np.random.Generator(np.random.PCG64(seed))
    _, Fb = bf16_grid_values(rng, (ncrops, (crop + 2) ** d, chp))
    Fb[:, :, nb + 1:] = 0
    _, Tb = bf16_grid_values(rng, (ncrops, crop ** d, nb), scale=0.5)
    feat = torch.tensor(Fb.view(np.int16).ravel(), device="cuda")
    targ = torch.tensor(Tb.view(np.int16).ravel(), device="cuda")
    p0 = init_net_params(d, p, seed)
    order = batch_order(seed + 1, steps, batch, ncrops)
    out = []
    for noalloc in (False, True):
        out.append(learned_train(d, p, crop, ncrops, feat, targ, 0.8, 1.3, p0, order, want_grad0=True,
                                 noalloc=noalloc))
    (pa, la, ga), (pb, lb, gb) = out
    assert np.all(np.isfinite(pb)) and np.all(np.isfinite(lb))
    # losses of every step and the first gradient: rounding of the atomics only
    assert np.allclose(lb, la, rtol=1e-5, atol=0.0), np.abs(lb / la - 1).max()
    assert np.linalg.norm(gb - ga) <= 1e-5 * np.linalg.norm(ga)
    # parameters after the Adam steps (the step is normalised per entry, so
    # entries with nearly vanishing gradients amplify the rounding)
    assert np.linalg.norm(pb - pa) <= 1e-3 * np.linalg.norm(pa - p0)
    assert not np.array_equal(pb, p0)


def test_noalloc_training_matches_allocating_entry_point():
    _compare(d=2, p=3, crop=8, ncrops=12, batch=4, steps=12, seed=11)
    _compare(d=2, p=2, crop=4, ncrops=6, batch=3, steps=5, seed=12)


def test_noalloc_training_rejects_runs_beyond_the_workspace():
    import torch
    from paper_1911_05888_amd import learned_train, init_net_params, TRAIN_WORKSPACE_BYTES
    from paper_1911_05888_amd.ldgs import LdgsError, E_ARG
    d, p, crop, ncrops = 2, 2, 4, 2
    steps, batch = TRAIN_WORKSPACE_BYTES // 4 // 2 + 1, 2      # the batch order alone exceeds the workspace
    feat = torch.zeros(ncrops * (crop + 2) ** d * 32, dtype=torch.int16, device="cuda")
    targ = torch.zeros(ncrops * crop ** d * 27, dtype=torch.int16, device="cuda")
    order = np.zeros((steps, batch), dtype=np.int32)
    with pytest.raises(LdgsError) as ei:
        learned_train(d, p, crop, ncrops, feat, targ, 1.0, 1.0, init_net_params(d, p, 0), order, noalloc=True)
    assert ei.value.status == E_ARG
