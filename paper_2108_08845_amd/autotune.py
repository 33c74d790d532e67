"""Autotuner of the tall-panel kernels.

Launch parameters that do not change what is computed -- only the grouping of
the fixed-order partial sums and the speed -- per kernel family:

  fused passes (power passes, final pass, lift):
    tile_rows    rows per tile (16, 32, 64; 0 = the library's plan),
    wg_per_cu    work-groups per compute unit (1 .. 4; 0 = 1),
    panel_width  plan the passes for a panel at least this wide (a wider
                 compiled tile width; 0 = the panel's own width);
  generic tall products (the FP64 path, Grams and products of the
  deterministic step, the unfused passes of wide sketches):
    split_m      work items the rows are split into, times output blocks
                 (0 = 1024).

`tune()` times candidates family by family on synthetic batches of the
requested shape (a few streaming updates after a warm-up, HIP events on the
stream): first the fused-pass candidates, then split_m with the best of those.
The fastest setting goes to a JSON cache keyed by the shape, the method, the
precision and the device name.  `StreamingSVD` applies a cached setting by
itself at its first batch (when the batch width is known); `cached_options()`
reads the cache.

Results of different settings agree to rounding (the partial sums are grouped
differently); each setting is itself run-to-run deterministic.
"""
import json
import os
import time

FUSED_CANDIDATES = [
    {"tile_rows": 0, "wg_per_cu": 1, "panel_width": 0},
    {"tile_rows": 32, "wg_per_cu": 1, "panel_width": 0},
    {"tile_rows": 64, "wg_per_cu": 1, "panel_width": 0},
    {"tile_rows": 0, "wg_per_cu": 2, "panel_width": 0},
    {"tile_rows": 32, "wg_per_cu": 2, "panel_width": 0},
]


def default_fused_candidates(N, K):
    """The fused-pass candidates, plus one planned for a panel 64 columns wider
    than the steady-state panel K + N (the next compiled tile width)."""
    return FUSED_CANDIDATES + [{"tile_rows": 0, "wg_per_cu": 1, "panel_width": int(K) + int(N) + 64}]
SPLIT_CANDIDATES = [512, 1024, 2048]
KNOBS = ("tile_rows", "wg_per_cu", "panel_width", "split_m")


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


def cached_options(M, N, K, oversampling=10, power_iters=2, precision="mixed", device=None, path=None):
    """The cached launch parameters of this shape ({knob: value}), or None."""
    rec = load_cache(path).get(_key(M, N, K, oversampling, power_iters, precision, device or device_name()))
    if not rec:
        return None
    try:
        return {k: int(rec.get(k, 0)) for k in KNOBS}
    except (TypeError, ValueError):
        return None


def tuned_options(M, N, K, oversampling=10, power_iters=2, precision="mixed", device=None, path=None):
    """The cached launch parameters, or the library defaults (all 0)."""
    return cached_options(M, N, K, oversampling, power_iters, precision, device, path) or {k: 0 for k in KNOBS}


def choose(timings):
    """Fastest candidate of {candidate: ms}; ties and failed (None) candidates lose to earlier ones."""
    best = None
    for cand, ms in timings.items():
        if ms is None:
            continue
        if best is None or ms < timings[best]:
            best = cand
    return best


def _freeze(opts):
    return tuple(int(opts.get(k, 0)) for k in KNOBS)


def _time_candidate(M, N, K, oversampling, power_iters, precision, opts, batches, warmup, reps, ff, seed):
    import torch
    from . import StreamingSVD, PsvdError
    try:
        svd = StreamingSVD(M, K, ff=ff, oversampling=oversampling, power_iters=power_iters, randomized=True,
                           precision=precision, seed=seed, async_updates=True, autotuned=False, **opts)
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


def tune(M, N, K, oversampling=10, power_iters=2, precision="mixed", fused_candidates=None, split_candidates=None,
         warmup=2, reps=4, ff=0.95, seed=0, path=None, timer=None):
    """Time the candidates on synthetic data of this shape and cache the fastest.

    Returns (best {knob: value}, {candidate tuple (tile_rows, wg_per_cu,
    panel_width, split_m): ms per update}).  `timer` replaces the GPU timing (a
    function of a {knob: value} dict -> ms or None), for tests of the selection
    and caching logic.
    """
    fused = list(fused_candidates or default_fused_candidates(N, K))
    splits = list(split_candidates or SPLIT_CANDIDATES)
    timings = {}
    batches = None
    if timer is None:
        import torch
        g = torch.Generator(device="cuda").manual_seed(int(seed))
        batches = [torch.randn((N, M), generator=g, device="cuda", dtype=torch.float32) for _ in range(2)]
        device = device_name()

        def timer(opts):
            return _time_candidate(M, N, K, oversampling, power_iters, precision, opts, batches, warmup, reps, ff,
                                   seed)
    else:
        device = "timer"
    for c in fused:
        opts = dict(c, split_m=0)
        timings[_freeze(opts)] = timer(opts)
    best = choose(timings)
    if best is None:
        raise RuntimeError("no candidate configuration ran")
    base = dict(zip(KNOBS, best))
    for sm in splits:
        opts = dict(base, split_m=sm)
        key = _freeze(opts)
        if key not in timings:
            timings[key] = timer(opts)
    best = choose(timings)
    del batches
    opts = dict(zip(KNOBS, best))
    data = load_cache(path)
    data[_key(M, N, K, oversampling, power_iters, precision, device)] = dict(
        opts, ms_per_update=timings[best], when=time.time(),
        timings={",".join(str(v) for v in k): ms for k, ms in timings.items()})
    save_cache(data, path)
    return opts, timings
