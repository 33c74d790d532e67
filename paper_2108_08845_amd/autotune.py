"""Autotuner of the tall-panel passes.

The fused passes (BF16 power pass, FP32 final pass, lift) have two launch
parameters that do not change what is computed, only the order of the
fixed-order partial sums and the speed:

  tile_rows  rows per tile (16, 32, 64; 0 = the library's default plan),
  wg_per_cu  work-groups per compute unit (1 .. 4).

`tune()` times every candidate pair on synthetic batches of the requested
shape (a few streaming updates after a warm-up, HIP events on the stream)
and records the fastest in a JSON cache keyed by the shape, the precision
and the device name.  `tuned_options()` reads that cache; `StreamingSVD`
accepts the two values directly (tile_rows=..., wg_per_cu=...).

Results of different configurations agree to rounding (the partial sums are
grouped differently); each configuration is itself run-to-run deterministic.
"""
import json
import os
import time

DEFAULT_CANDIDATES = [(0, 1), (32, 1), (64, 1), (0, 2), (32, 2)]


def cache_path():
    p = os.environ.get("PSVD_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "psvd_autotune.json")


def _key(M, N, K, oversampling, power_iters, precision, device):
    return f"{device}|M={int(M)}|N={int(N)}|K={int(K)}|p={int(oversampling)}|q={int(power_iters)}|{precision}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data, path=None):
    path = path or cache_path()
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def tuned_options(M, N, K, oversampling=10, power_iters=2, precision="mixed", device=None, path=None):
    """{'tile_rows': .., 'wg_per_cu': ..} from the cache, or the defaults (0, 0)."""
    rec = load_cache(path).get(_key(M, N, K, oversampling, power_iters, precision, device or device_name()))
    if rec:
        return {"tile_rows": int(rec["tile_rows"]), "wg_per_cu": int(rec["wg_per_cu"])}
    return {"tile_rows": 0, "wg_per_cu": 0}


def choose(timings):
    """Fastest candidate of {(tile_rows, wg_per_cu): ms}; ties go to the earlier candidate."""
    best = None
    for cand, ms in timings.items():
        if ms is None:
            continue
        if best is None or ms < timings[best]:
            best = cand
    return best


def _time_candidate(M, N, K, oversampling, power_iters, precision, tile_rows, wg_per_cu, batches, warmup, reps,
                    ff, seed):
    import torch
    from . import StreamingSVD, PsvdError
    try:
        svd = StreamingSVD(M, K, ff=ff, oversampling=oversampling, power_iters=power_iters, randomized=True,
                           precision=precision, seed=seed, async_updates=True, tile_rows=tile_rows,
                           wg_per_cu=wg_per_cu)
    except PsvdError:
        return None
    try:
        for i in range(warmup):
            svd.incorporate_data(batches[i % len(batches)].t())
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for i in range(reps):
            svd.incorporate_data(batches[(warmup + i) % len(batches)].t())
        ev1.record()
        torch.cuda.synchronize()
        svd.singular_values          # surfaces any device error of the timed updates
        return ev0.elapsed_time(ev1) / reps
    except PsvdError:
        return None
    finally:
        svd.close()


def tune(M, N, K, oversampling=10, power_iters=2, precision="mixed", candidates=None, warmup=2, reps=4, ff=0.95,
         seed=0, path=None, timer=None):
    """Time the candidates on synthetic data of this shape and cache the fastest.

    Returns (best (tile_rows, wg_per_cu), {candidate: ms per update}).  `timer`
    replaces the GPU timing (a function of (tile_rows, wg_per_cu) -> ms or
    None), for tests of the selection and caching logic.
    """
    candidates = list(candidates or DEFAULT_CANDIDATES)
    timings = {}
    if timer is None:
        import torch
        g = torch.Generator(device="cuda").manual_seed(int(seed))
        batches = [torch.randn((N, M), generator=g, device="cuda", dtype=torch.float32) for _ in range(2)]
        device = device_name()
        for tr, wg in candidates:
            timings[(tr, wg)] = _time_candidate(M, N, K, oversampling, power_iters, precision, tr, wg, batches,
                                                warmup, reps, ff, seed)
        del batches
    else:
        device = "timer"
        for tr, wg in candidates:
            timings[(tr, wg)] = timer(tr, wg)
    best = choose(timings)
    if best is None:
        raise RuntimeError("no candidate configuration ran")
    data = load_cache(path)
    data[_key(M, N, K, oversampling, power_iters, precision, device)] = {
        "tile_rows": best[0], "wg_per_cu": best[1], "ms_per_update": timings[best],
        "timings": {f"{tr},{wg}": ms for (tr, wg), ms in timings.items()}, "when": time.time(),
    }
    save_cache(data, path)
    return best, timings
