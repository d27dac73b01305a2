"""Launch-shape autotuner and memory-probed state-batch sizing.

* ``tune``: times ``bin + composite`` for every tile shape (16x16, 32x8),
  states-per-group S in {2, 4, 8, 16, 32}, compositing launch (grid or
  persistent) and list entries staged in LDS per batch (128, 256, 512; groups
  of 4 or more states) on the caller's own scene, camera and states, and keeps
  the fastest.  Results are cached in a JSON file keyed by
  the device name and the workload's shape.
* ``probe_state_batch``: the largest number of states whose images and
  workspace fit a memory budget.  Like the paper's probe-based world-batch
  tuner (Sec. 6), it allocates for real, doubles while allocations succeed and
  backs off by halving after an out-of-memory failure.

Timing and allocation are injectable, so the search logic is testable on a
host without a GPU.
"""

from __future__ import annotations

import json
import os
from dataclasses import dataclass
from typing import Callable, Dict, Iterable, Optional, Tuple

TILES = ((16, 16), (32, 8))
GROUP_SIZES = (2, 4, 8, 16, 32)
LAUNCHES = (False, True)  # persistent compositing launch off / on
LDS_BATCHES = (128, 256, 512)  # list entries per LDS batch (variants exist for S >= 4)
DEFAULT_LDS_BATCH = 256


@dataclass
class TuneResult:
    tile: Tuple[int, int]
    states_per_group: int
    persistent: bool
    ms: float
    table: Dict[str, float]
    lds_batch: int = DEFAULT_LDS_BATCH

    def as_dict(self):
        return {"tile": list(self.tile), "states_per_group": self.states_per_group,
                "persistent": self.persistent, "lds_batch": self.lds_batch, "ms": self.ms, "table": self.table}


def _key(device_name: str, n: int, width: int, height: int, num_states: int, packets: int) -> str:
    return f"{device_name}|n={n}|{width}x{height}|W={num_states}|P={packets}"


def search(timer: Callable[[Tuple[int, int], int, bool, int], float], num_states: int,
           tiles: Iterable[Tuple[int, int]] = TILES, group_sizes: Iterable[int] = GROUP_SIZES,
           launches: Iterable[bool] = LAUNCHES, lds_batches: Iterable[int] = LDS_BATCHES) -> TuneResult:
    """Exhaustive search: ``timer(tile, S, persistent, lds_batch)`` returns
    milliseconds (may raise to reject a candidate).  Group sizes above the
    state count add nothing and are skipped; groups of fewer than 4 states have
    only the default LDS batch, so they are timed once."""
    table = {}
    best = None
    cap = 1
    while cap < max(num_states, 1):
        cap *= 2
    group_sizes = tuple(group_sizes)
    lds_batches = tuple(lds_batches)
    for tile in tiles:
        for S in group_sizes:
            if S > cap and S != min(group_sizes):
                continue
            batches = lds_batches if S >= 4 else (DEFAULT_LDS_BATCH,)
            for pers in launches:
                for B in batches:
                    name = f"{tile[0]}x{tile[1]}/S{S}/{'persistent' if pers else 'grid'}/B{B}"
                    try:
                        ms = float(timer(tile, S, pers, B))
                    except Exception as e:  # a candidate that fails (e.g. out of memory) is skipped
                        table[name] = f"failed: {type(e).__name__}"
                        continue
                    table[name] = ms
                    if best is None or ms < best.ms:
                        best = TuneResult(tile, S, bool(pers), ms, table, B)
    if best is None:
        raise RuntimeError("no launch shape could be timed")
    best.table = table
    return best


def probe_state_batch(try_alloc: Callable[[int], object], upper: int, lower: int = 1,
                      is_oom: Callable[[BaseException], bool] = lambda e: isinstance(e, MemoryError)) -> int:
    """Largest batch b in [lower, upper] for which ``try_alloc(b)`` succeeds.
    Doubles from ``lower`` while allocations succeed; after an OOM, bisects
    between the last success and the failure.  Returns 0 if even ``lower``
    fails.  ``try_alloc`` must release what it allocates before returning."""
    def ok(b):
        try:
            try_alloc(b)
            return True
        except BaseException as e:  # noqa: B902
            if is_oom(e):
                return False
            raise

    if not ok(lower):
        return 0
    good, b = lower, lower
    bad = None
    while b < upper:
        nb = min(upper, b * 2)
        if ok(nb):
            good = b = nb
        else:
            bad = nb
            break
    if bad is None:
        return good
    while bad - good > 1:
        mid = (good + bad) // 2
        if ok(mid):
            good = mid
        else:
            bad = mid
    return good


class Autotuner:
    """GPU front end: times the real kernels through a ``Renderer`` factory."""

    def __init__(self, cache_path: Optional[str] = None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def tune(self, scene, camera, codes, basis, background=(0, 0, 0), reps: int = 5,
             tiles=TILES, group_sizes=GROUP_SIZES, launches=LAUNCHES, lds_batches=LDS_BATCHES) -> TuneResult:
        import torch

        from .render import Renderer

        dev = codes.device
        key = _key(torch.cuda.get_device_name(dev), scene.n, camera.width, camera.height,
                   int(codes.shape[0]), scene.num_packets)
        if key in self.cache:
            c = self.cache[key]
            return TuneResult(tuple(c["tile"]), int(c["states_per_group"]), bool(c.get("persistent", False)),
                              float(c["ms"]), c["table"], int(c.get("lds_batch", DEFAULT_LDS_BATCH)))
        W = int(codes.shape[0])
        img = torch.empty((W, camera.height, camera.width, 3), dtype=torch.float32, device=dev)

        def timer(tile, S, persistent, lds_batch):
            r = Renderer(dev, tile=tile, states_per_group=S, persistent=persistent, lds_batch=lds_batch)
            r.plan(scene, camera, basis, W)
            for _ in range(2):
                r.bin(scene, camera, basis)
                r.composite(scene, camera, codes, basis, background, out=img)
            st = torch.cuda.current_stream(dev)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            best = float("inf")
            for _ in range(3):  # the fastest of three timed blocks: a transient stall cannot pick the winner
                e0.record(st)
                for _ in range(reps):
                    r.bin(scene, camera, basis)
                    r.composite(scene, camera, codes, basis, background, out=img)
                e1.record(st)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) / reps)
            r.check()
            del r
            return best

        res = search(timer, W, tiles, group_sizes, launches, lds_batches)
        self.cache[key] = res.as_dict()
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return res

    @staticmethod
    def max_states(scene, camera, renderer, upper: int, budget_bytes: Optional[int] = None) -> int:
        """Largest state batch whose images and workspace fit ``budget_bytes``
        (default: 90% of the device's free memory), probed with real
        allocations."""
        import torch

        dev = renderer.device
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(dev)
            budget_bytes = int(0.9 * free)
        per_state_img = camera.height * camera.width * 3 * 4

        def try_alloc(b):
            ws = renderer.workspace_bytes(scene, camera, b, renderer.capacity)
            if ws + b * per_state_img > budget_bytes:
                raise MemoryError("over budget")
            x = torch.empty(ws + b * per_state_img, dtype=torch.uint8, device=dev)
            del x

        return probe_state_batch(try_alloc, upper,
                                 is_oom=lambda e: isinstance(e, (MemoryError, torch.cuda.OutOfMemoryError)))
