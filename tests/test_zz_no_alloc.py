"""swe_trainer_loss_grad_static (the entry point that allocates nothing:
per-block partials in a static device array) against swe_trainer_loss_grad,
which uses the trainer's own workspace: bitwise equal loss and gradient on
two calls in a row, the second with fewer records (fewer blocks, so rows of
the static array left by the first call must not leak into the sum)."""
import numpy as np
import pytest

from gpu_util import lib

pytestmark = pytest.mark.gpu


def records(n_rec, seed, width):
    rng = np.random.default_rng(seed)
    R = np.zeros((n_rec, width), np.float32)
    R[:, :14] = rng.normal(0.0, 1.0, (n_rec, 14))          # features
    R[:, 14:18] = rng.uniform(0.5, 3.0, (n_rec, 4))        # cell values
    R[:, 18:22] = rng.normal(0.0, 0.05, (n_rec, 4))        # central slopes
    R[:, 22] = rng.uniform(1.0, 4.0, n_rec)                # target distance
    R[:, 23:27] = R[:, 14:18] + rng.normal(0.0, 0.05, (n_rec, 4))  # targets
    R[:, 27] = 1.0
    R[:, 32:36] = R[:, 18:22] * rng.uniform(0.2, 1.5, (n_rec, 4))  # backward slopes
    R[:, 36:40] = R[:, 18:22] * rng.uniform(0.2, 1.5, (n_rec, 4))  # forward slopes
    return R


def test_static_loss_grad_equals_trainer():
    import torch
    swe, _ = lib()
    rng = np.random.default_rng(7)
    w = rng.normal(0.0, 0.2, swe.MLP_NPARAM).astype(np.float32)
    wv = np.array([1.0, 1.0, 0.5, 0.5], np.float32)
    tr = swe.Trainer(w)
    params = torch.from_numpy(w).cuda()
    out = torch.full((swe.MLP_NPARAM + 1,), float("nan"), dtype=torch.float32, device="cuda")
    # 40,000 records over 512 blocks, then 3,000 over 47 blocks; the index
    # lists pick a subset with repeats and one out-of-range entry (absent)
    for n_rec, n_idx, seed in ((40000, 50000, 1), (3000, 3000, 2)):
        R = records(n_rec, seed, swe.PAIR_RECORD)
        rec = torch.from_numpy(R.ravel()).cuda()
        idx_np = np.random.default_rng(seed + 10).integers(0, n_rec, n_idx).astype(np.int32)
        idx_np[5] = n_rec + 3
        idx = torch.from_numpy(idx_np).cuda()
        loss_t, g_t = tr.loss_grad(rec, idx, wv)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            swe.trainer_loss_grad_static(params, rec, idx, wv, out, stream=s)
        s.synchronize()
        o = out.cpu().numpy()
        print(n_rec, n_idx, "loss", loss_t, o[-1])
        assert np.isfinite(o).all()
        assert np.array_equal(o[:-1].view(np.uint32), g_t.view(np.uint32))
        assert o[-1] == np.float32(loss_t)
    tr.close()


def test_static_loss_grad_rejects_bad_arguments():
    import torch
    swe, _ = lib()
    params = torch.zeros(swe.MLP_NPARAM, dtype=torch.float32, device="cuda")
    rec = torch.zeros(swe.PAIR_RECORD * 10, dtype=torch.float32, device="cuda")
    idx = torch.zeros(10, dtype=torch.int32, device="cuda")
    out = torch.zeros(swe.MLP_NPARAM + 1, dtype=torch.float32, device="cuda")
    wv = np.ones(4, np.float32)
    with pytest.raises(swe.SweError):
        swe.trainer_loss_grad_static(params, rec, idx, wv, out[:10])
    with pytest.raises(swe.SweError):
        swe.trainer_loss_grad_static(params, rec, idx[:0], wv, out)
