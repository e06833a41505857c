"""Tile-shape autotuner for the stage kernel.

Builds one solver per candidate tile (elements per workgroup) for the same
workload, times a few RK4 steps of each on the GPU with HIP events on the
launch stream, and returns the fastest. Host-side selection logic only:
every candidate runs the library's own kernels, and results do not depend on
the tile (the face exchange is exact either way).
"""
from __future__ import annotations


def autotune_tile(make_solver, candidates=(32, 64), steps=10, warmup=3):
    """make_solver(tile) -> a bound Solver holding the workload's state.

    Returns (best_tile, {tile: microseconds per step}). Candidates the
    library rejects (e.g. LDS too small) are skipped."""
    import torch

    from .mdg import MdgError

    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    timings = {}
    for tile in candidates:
        try:
            s = make_solver(tile)
        except MdgError:
            continue
        try:
            s.step(warmup, sp)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            s.step(steps, sp)
            e1.record(stream)
            torch.cuda.synchronize()
            timings[s.query()["tile_size"]] = e0.elapsed_time(e1) * 1000.0 / steps
        finally:
            s.close()
    if not timings:
        raise RuntimeError("autotune_tile: no candidate tile could be built")
    best = min(timings, key=timings.get)
    return best, timings
