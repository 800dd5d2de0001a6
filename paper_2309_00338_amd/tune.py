"""Launch-schedule tuner for the EBIT engines (one grid, batch, pool).

The engines' persistent kernels spread their tiles and marker jobs over a
fixed number of workgroups per compute unit (the ebit_schedule of
include/ebit.h). The best split depends on the GPU and on the workload's size
and interface density, and it never changes a result, so it can be chosen by
measurement. tune() does coordinate descent over the schedule fields: for each
field in turn it times a few steps of the caller's own workload under each
candidate value, the other fields held at their best so far, and keeps the
fastest. Results are cached in a JSON file keyed by the GPU's architecture, the
engine kind and the workload's size bucket; schedule_for() looks a key up.

All timing is on the engine's stream with HIP events; the caller supplies the
step function (advect plus fraction/curvature on its own buffers), so the
tuned work is exactly the work that will run.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Tuple

CANDIDATES: Dict[str, List[float]] = {
    "frac_near_per_cu": [3.0, 4.0, 4.5, 5.0, 5.5, 6.0, 7.0, 8.0],
    "sweep_per_cu": [8, 12, 16],
    "fit_per_cu": [2, 4, 6, 8],
    "sweep_min_chunk": [1, 4, 8, 16, 32],
    "ns_near_per_cu": [3.0, 4.0, 5.0, 6.0, 7.0, 8.0],
}
# fields that matter for the plain step of one grid (the minimum chunk is read
# only with several grids, the consumers' split only by ebit_ns_fields)
ONE_GRID = ("frac_near_per_cu", "sweep_per_cu", "fit_per_cu")
SEVERAL = ("frac_near_per_cu", "sweep_per_cu", "fit_per_cu", "sweep_min_chunk")


def cache_path() -> str:
    return os.environ.get("EBIT_SCHEDULE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ebit_schedule.json"))


def arch() -> str:
    import torch

    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def size_key(kind: str, cells: int, grids: int = 1) -> str:
    """Engine kind, cells rounded to a power of two, grid count to a power of two."""
    return f"{arch()}/{kind}/cells2^{round(math.log2(max(cells, 1)))}/grids2^{round(math.log2(max(grids, 1)))}"


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def schedule_for(key: str, path: Optional[str] = None) -> Optional[dict]:
    return load_cache(path).get(key, {}).get("schedule")


def _time_steps(step: Callable[[], None], stream, steps: int) -> float:
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / steps  # us per step


def tune(engine, step: Callable[[], None], stream, fields: Iterable[str] = ONE_GRID, steps: int = 6,
         reps: int = 2, key: Optional[str] = None, path: Optional[str] = None) -> Tuple[dict, dict]:
    """Coordinate descent over `fields` of `engine`'s schedule (an EbitGrid,
    EbitBatch or EbitPool), timing `steps` calls of `step` per candidate (best
    of `reps`, after one untimed call). Leaves the best schedule set on the
    engine and returns it with the measured table {field: {value: us}}. With
    `key`, the result is stored in the cache."""
    best = engine.get_schedule()
    engine.set_schedule(best)
    step()
    best_us = min(_time_steps(step, stream, steps) for _ in range(reps))
    table = {}
    for f in fields:
        table[f] = {}
        for val in CANDIDATES[f]:
            trial = dict(best, **{f: val})
            engine.set_schedule(trial)
            step()
            us = min(_time_steps(step, stream, steps) for _ in range(reps))
            table[f][str(val)] = us
            if us < best_us:
                best_us, best = us, engine.get_schedule()
        engine.set_schedule(best)
    if key:
        cache = load_cache(path)
        cache[key] = {"schedule": best, "us_per_step": best_us, "table": table}
        save_cache(cache, path)
    return best, {"us_per_step": best_us, "table": table}
