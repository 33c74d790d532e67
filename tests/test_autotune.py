"""Autotuner: candidate selection and the JSON cache (host logic), and one
real tuning run on the GPU whose tuned handle agrees with the default one."""
import json

import numpy as np
import pytest
import torch

from paper_2108_08845_amd import autotune


def test_choose_and_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    times = {(0, 1): 3.0, (32, 1): 2.5, (64, 1): None, (0, 2): 2.5}
    best, timings = autotune.tune(4096, 64, 8, 4, 1, "fp32", candidates=list(times), path=path,
                                  timer=lambda tr, wg: times[(tr, wg)])
    assert best == (32, 1)                     # fastest; the later tie and the failed candidate lose
    assert timings == times
    rec = json.load(open(path))
    assert len(rec) == 1
    opts = autotune.tuned_options(4096, 64, 8, 4, 1, "fp32", device="timer", path=path)
    assert opts == {"tile_rows": 32, "wg_per_cu": 1}
    # unknown shape -> library defaults
    assert autotune.tuned_options(4096, 64, 9, 4, 1, "fp32", device="timer", path=path) == \
        {"tile_rows": 0, "wg_per_cu": 0}
    with pytest.raises(RuntimeError):
        autotune.tune(1, 1, 1, candidates=[(0, 1)], path=path, timer=lambda tr, wg: None)


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.load_cache(str(path)) == {}
    autotune.tune(8, 8, 1, candidates=[(0, 1)], path=str(path), timer=lambda tr, wg: 1.0)
    assert len(autotune.load_cache(str(path))) == 1


@pytest.mark.gpu
def test_tuned_configuration_matches_default(tmp_path):
    import paper_2108_08845_amd as P
    import synth
    path = str(tmp_path / "tune.json")
    M, N, K, p, q = 1 << 15, 128, 20, 8, 1
    best, timings = autotune.tune(M, N, K, p, q, "fp32", path=path, warmup=1, reps=2)
    assert timings[best] is not None and timings[best] > 0
    opts = autotune.tuned_options(M, N, K, p, q, "fp32", path=path)
    w = synth.scaled(synth.c2_randomized_fp32(), M=M, N=N, batches=3, K=K)
    bs = [b.cuda() for b in synth.planted_stream(w)]
    out = []
    for kw in ({}, opts):
        svd = P.StreamingSVD(M, K, ff=w.ff, oversampling=p, power_iters=q, randomized=True, precision="fp32",
                             seed=3, **kw)
        for b in bs:
            svd.incorporate_data(b.t())
        out.append(svd.singular_values)
    assert np.max(np.abs(out[0] - out[1]) / out[1]) <= 1e-4
