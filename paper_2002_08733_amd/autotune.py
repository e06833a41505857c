"""Launch-shape autotuner for the stage kernel.

Builds one solver per candidate launch shape — elements per workgroup
(`tile`) and grid (`launch`: one workgroup per tile, or only the resident
workgroups looping over tiles) — for the same workload, times a few RK4
steps of each on the GPU with HIP events on the launch stream, and returns
the fastest. Host-side selection logic only: every candidate runs the
library's own kernels, and results do not depend on the shape (the face
exchange is exact either way, the persistent grid visits the same tiles).
"""
from __future__ import annotations


def launch_candidates(precision, order, tiles=(32, 64)):
    """The shapes worth timing: every tile with one workgroup per tile, and
    the persistent grid where the library builds it (FP32, orders 1-3; it
    falls back to one workgroup per tile elsewhere, which would only time
    the same launch twice)."""
    cands = [{"tile": t, "launch": "per_tile"} for t in tiles]
    if precision == "fp32" and order <= 3:
        cands += [{"tile": t, "launch": "persistent"} for t in tiles]
    return cands


def autotune(make_solver, candidates, steps=10, warmup=3):
    """make_solver(**shape) -> a bound Solver holding the workload's state,
    for each shape (a dict of Solver keyword arguments) in candidates.

    Returns (best_shape, {key: microseconds per step}), key "tile/launch"
    with the tile the library actually used. Candidates the library rejects
    (e.g. LDS too small for the tile) are skipped."""
    import torch

    from .mdg import MdgError

    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    timings, shapes = {}, {}
    for shape in candidates:
        try:
            s = make_solver(**shape)
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
            key = f"{s.query()['tile_size']}/{shape.get('launch', 'auto')}"
            timings[key] = e0.elapsed_time(e1) * 1000.0 / steps
            shapes[key] = dict(shape, tile=s.query()["tile_size"])
        finally:
            s.close()
    if not timings:
        raise RuntimeError("autotune: no candidate launch shape could be built")
    best = min(timings, key=timings.get)
    return shapes[best], timings


def autotune_tile(make_solver, candidates=(32, 64), steps=10, warmup=3):
    """make_solver(tile) -> a bound Solver. Returns (best_tile, {tile: us per
    step}) over one-workgroup-per-tile launches."""
    best, timings = autotune(lambda tile, launch: make_solver(tile), [{"tile": t, "launch": "per_tile"}
                                                                       for t in candidates], steps, warmup)
    return best["tile"], {int(k.split("/")[0]): v for k, v in timings.items()}
