"""Autotuner of the deposition tile shape and the re-sort threshold.

The fused particle kernel's speed depends on the tile shape: it sets the
LDS region, the halo overhead per particle, the bucket count and the
parallelism. It also depends on how often the particles are re-sorted by
tile. The best choice varies with grid size, particles per cell and drift.
The tuner times a few steps of the actual workload (the same particles,
fresh contexts) for each candidate and keeps the fastest. It tunes the tile
shape first, at the default threshold, then the threshold with that tile.
One setting applies to every run of a context.  Results do not depend on
the setting beyond the order of float sums.
"""

import time

TILES = [(8, 8, 8), (4, 8, 8), (8, 4, 8), (8, 8, 4), (4, 4, 8), (4, 8, 4), (8, 4, 4), (4, 4, 4)]
RESORT_DIVS = [64, 16, 256]


def time_setting(cfgs, inputs, precision, tile, resort_div, steps=20, warmup=5):
    """ms per step of `steps` steps after `warmup` (both from the bound state)."""
    import torch

    from . import galpic as gp

    grids = []
    for c in cfgs:
        t = tuple(min(tile[a], c.shape[a]) for a in range(3))
        grids.append(gp.grid_from_config(c, precision, tile=t, resort_div=resort_div))
    ctx = gp.Context(grids)
    for r, c in enumerate(cfgs):
        ctx.set_v_gal(r, c.v_gal())
    parts = [gp.particles_from_inputs(i, c, precision, with_ids=False)
             for c, i in zip(cfgs, inputs)]
    ctx.bind_particles(parts)
    ctx.run(warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run(steps)
    ctx.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    ctx.close()
    del parts
    torch.cuda.empty_cache()
    return ms


def tune(cfgs, inputs, precision, steps=20, warmup=5, tiles=TILES, resort_divs=RESORT_DIVS,
         log=None):
    """Best (tile, resort_div) for a list of RunConfigs and their inputs;
    returns (best, {setting: ms})."""
    results = {}

    def run(tile, div):
        key = (tuple(tile), int(div))
        if key not in results:
            results[key] = time_setting(cfgs, inputs, precision, tile, div, steps, warmup)
            if log:
                log(f"tile {tile} resort n/{div}: {results[key]:.3f} ms/step")
        return results[key]

    best_tile = min(tiles, key=lambda t: run(t, resort_divs[0]))
    best_div = min(resort_divs, key=lambda d: run(best_tile, d))
    return (tuple(best_tile), int(best_div)), results
