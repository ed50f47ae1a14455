"""Autotuner: workload keys and the cache (CPU), and a GPU tuning run whose
every trial must reproduce the reference results."""

import numpy as np
import pytest

from paper_1509_06004_amd import workload as W


def test_workload_key_and_cache(tmp_path):
    from paper_1509_06004_amd import tune as T
    a = W.config0()
    b = [W.tiny_random(np.random.default_rng(1), 64, 64, 8, L=1)]
    ka, kb = T.workload_key(a, "dev"), T.workload_key(b, "dev")
    assert ka != kb and "K4" in ka and "K8" in kb
    assert T.workload_key(a, "dev") == ka
    p = str(tmp_path / "c.json")
    assert T.load_cache(p) == {}
    T.save_cache({ka: {"options": {"tile_w": 64}}}, p)
    assert T.load_cache(p)[ka]["options"]["tile_w"] == 64


@pytest.mark.gpu
def test_tuner_trials_agree(tmp_path):
    import torch
    from paper_1509_06004_amd import pmf
    from paper_1509_06004_amd import tune as T
    rng = np.random.default_rng(3)
    insts = [W.tiny_random(rng, 70, 50, 4, cmax=200, L=4, p_seed=0.03, lam_max=60),
             W.tiny_random(rng, 40, 90, 8, cmax=200, L=3, p_seed=0.03, lam_max=60)]
    dev = pmf.to_device(insts)
    space = {"tile_w": [32, 64], "inner_iters": [4, 16], "sweeps_per_relabel": [2, 8],
             "local_bfs_iters": [16, 64], "exchange_rounds": [1, 3], "order": [0, 1],
             "lambda_chunk": [1, 3]}
    out = T.tune(dev, repeats=1, space=space)
    assert out["rejected"] == []
    assert len(out["trials"]) >= 6
    assert set(T.KNOBS) <= set(out["options"])
    opts = T.options_for(insts, dev, path=str(tmp_path / "c.json"))
    assert T.options_for(insts, None, path=str(tmp_path / "c.json")) == opts
    torch.cuda.synchronize()
