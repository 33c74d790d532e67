"""Autotuner: candidate selection and the JSON cache (host logic), and one
real tuning run on the GPU whose tuned handle (the cached setting applied by
StreamingSVD itself) matches the FP64 oracle."""
import json

import numpy as np
import pytest
import torch

from paper_2108_08845_amd import autotune


def test_choose_and_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    fused = [{"tile_rows": 0, "wg_per_cu": 1, "panel_width": 0}, {"tile_rows": 32, "wg_per_cu": 1, "panel_width": 0},
             {"tile_rows": 64, "wg_per_cu": 1, "panel_width": 0}, {"tile_rows": 0, "wg_per_cu": 2, "panel_width": 0}]
    times = {(0, 1, 0, 0): 3.0, (32, 1, 0, 0): 2.5, (64, 1, 0, 0): None, (0, 2, 0, 0): 2.5,
             (32, 1, 0, 512): 2.6, (32, 1, 0, 2048): 2.4}
    seen = []

    def timer(opts):
        k = tuple(opts[x] for x in autotune.KNOBS)
        seen.append(k)
        return times[k]

    best, timings = autotune.tune(4096, 64, 8, 4, 1, "fp32", fused_candidates=fused, split_candidates=[512, 0, 2048],
                                  path=path, timer=timer)
    # fused family first (fastest; the later tie and the failed candidate lose), then split_m on top of it
    assert best == {"tile_rows": 32, "wg_per_cu": 1, "panel_width": 0, "split_m": 2048}
    assert seen == [(0, 1, 0, 0), (32, 1, 0, 0), (64, 1, 0, 0), (0, 2, 0, 0), (32, 1, 0, 512), (32, 1, 0, 2048)]
    rec = json.load(open(path))
    assert len(rec) == 1
    assert autotune.cached_options(4096, 64, 8, 4, 1, "fp32", device="timer", path=path) == best
    # unknown shape: no cached setting, the library defaults
    assert autotune.cached_options(4096, 64, 9, 4, 1, "fp32", device="timer", path=path) is None
    assert autotune.tuned_options(4096, 64, 9, 4, 1, "fp32", device="timer", path=path) == \
        {"tile_rows": 0, "wg_per_cu": 0, "panel_width": 0, "split_m": 0}
    with pytest.raises(RuntimeError):
        autotune.tune(1, 1, 1, fused_candidates=fused[:1], path=path, timer=lambda opts: None)


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.load_cache(str(path)) == {}
    autotune.tune(8, 8, 1, fused_candidates=[{"tile_rows": 0, "wg_per_cu": 1, "panel_width": 0}],
                  split_candidates=[1024], path=str(path), timer=lambda opts: 1.0)
    assert len(autotune.load_cache(str(path))) == 1


@pytest.mark.gpu
def test_tuned_handle_matches_oracle(tmp_path, monkeypatch):
    import oracle
    import paper_2108_08845_amd as P
    import synth
    from conftest import sigma_rel_err, orth_err
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv("PSVD_TUNE_CACHE", path)
    M, N, K, p, q = 1 << 15, 128, 20, 8, 1
    best, timings = autotune.tune(M, N, K, p, q, "fp32", warmup=1, reps=2)
    assert timings[tuple(best[k] for k in autotune.KNOBS)] > 0
    w = synth.scaled(synth.c2_randomized_fp32(), M=M, N=N, batches=3, K=K, oversampling=p, power_iters=q)
    bs = synth.planted_stream(w)
    svd = P.StreamingSVD(M, K, ff=w.ff, oversampling=p, power_iters=q, randomized=True, precision="fp32", seed=3)
    for b in bs:
        svd.incorporate_data(b.cuda().t())
    assert svd.tuning == best                      # the cached setting was applied
    so = oracle.StreamOracle(M, K, ff=w.ff, oversampling=p, power_iters=q, randomized=True, seed=3,
                             omega_precision=oracle.PREC_F32)
    for b in bs:
        so.incorporate(synth.numpy_cm(b))
    assert sigma_rel_err(svd.singular_values, so.singular_values) <= 1e-4
    assert orth_err(svd.modes.double().cpu().numpy()) <= 1e-5
