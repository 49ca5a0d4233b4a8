"""Persistent cache of autotuned launch shapes, one JSON file.

``lbm_autotune`` and ``lbm_batch_autotune`` time every candidate shape, which
takes seconds on a large lattice; the shape they pick depends only on the
lattice (or the batch's runs), the storage, the operator, the walls, the step
mode, the kernel code and the GPU.  The cache keys a tuned shape on all of
those and restores it without timing anything when the same configuration
comes back.  The kernel code enters the key through the library's source
digest, so a rebuilt kernel tunes afresh.

File layout (written by this module; any other content is ignored and
rewritten)::

    {"format": "mrt-lbm-tune-cache", "version": 1,
     "entries": {"<key>": {"mode": "split", "tile": [128, 4, 128]}, ...}}

Batch entries hold ``{"mode", "item_nodes", "blocks"}`` instead of a tile.
Writes go to a temporary file that replaces the cache, so a reader never sees
a half-written file; two processes tuning at once keep whichever wrote last.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

FORMAT = "mrt-lbm-tune-cache"
VERSION = 1


def _device_tag() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', '')}:{p.name}:{p.multi_processor_count}cu"


def _code_tag() -> str:
    from paper_1805_08643_amd import build
    return build.source_digest()


def lattice_key(cfg: dict, mode: str, device: str | None = None, code: str | None = None) -> str:
    """Key of a single lattice's tuned tile: sizes, walls, storage, operator,
    step mode, kernel code and device."""
    parts = [f"{cfg['nx']}x{cfg['ny']}x{cfg['nz']}", f"wz{int(cfg.get('wall_z', 0))}",
             f"wx{int(cfg.get('wall_x', 0))}", f"wy{int(cfg.get('wall_y', 0))}", cfg.get("storage", "f32"),
             cfg.get("op", "nonorth"), mode, code if code is not None else _code_tag(),
             device if device is not None else _device_tag()]
    return "lattice|" + "|".join(parts)


def batch_key(cfgs, device: str | None = None, code: str | None = None) -> str:
    """Key of a batch's tuning: the multiset of run sizes (with the shared
    storage and operator), kernel code and device."""
    sizes = sorted(f"{c['nx']}x{c['ny']}x{c['nz']}" for c in cfgs)
    h = hashlib.sha256(",".join(sizes).encode()).hexdigest()[:16]
    c0 = cfgs[0]
    parts = [f"{len(sizes)}runs", h, c0.get("storage", "f32"), c0.get("op", "nonorth"),
             code if code is not None else _code_tag(), device if device is not None else _device_tag()]
    return "batch|" + "|".join(parts)


class TuneCache:
    """device, code: override the device and kernel-code parts of the keys
    (default: the current GPU and the library's source digest)."""

    def __init__(self, path: str, device: str | None = None, code: str | None = None):
        self.path = path
        self.device, self.code = device, code
        self.entries = {}
        self.hits = self.misses = 0
        try:
            with open(path) as fh:
                d = json.load(fh)
            if isinstance(d, dict) and d.get("format") == FORMAT and d.get("version") == VERSION \
                    and isinstance(d.get("entries"), dict):
                self.entries = {k: v for k, v in d["entries"].items() if self._valid(v)}
        except (OSError, ValueError):
            pass  # missing or unreadable: start empty

    @staticmethod
    def _valid(v) -> bool:
        if not isinstance(v, dict) or not isinstance(v.get("mode"), str):
            return False
        if "tile" in v:
            t = v["tile"]
            return isinstance(t, list) and len(t) == 3 and all(isinstance(x, int) and x > 0 for x in t)
        return all(isinstance(v.get(k), int) and v[k] > 0 for k in ("item_nodes", "blocks"))

    def save(self):
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(prefix=".tune-", suffix=".json", dir=d)
        with os.fdopen(fd, "w") as fh:
            json.dump({"format": FORMAT, "version": VERSION, "entries": self.entries}, fh, indent=1,
                      sort_keys=True)
        os.replace(tmp, self.path)

    def tune_lattice(self, lat, trials: int = 3):
        """Restore the lattice's cached tile for its current step mode, or
        autotune it and cache the result.  Returns (tile, hit)."""
        key = lattice_key(lat.cfg, lat.step_mode(), self.device, self.code)
        e = self.entries.get(key)
        if e is not None:
            self.hits += 1
            lat.set_tile(*e["tile"])
            return tuple(e["tile"]), True
        self.misses += 1
        tile = tuple(int(v) for v in lat.autotune(trials))
        self.entries[key] = {"mode": lat.step_mode(), "tile": list(tile)}
        self.save()
        return tile, False

    def tune_batch(self, batch, trials: int = 3):
        """Restore the batch's cached mode, work-item size and grid, or
        autotune them and cache the result.  Returns ((mode, item_nodes,
        blocks), hit)."""
        key = batch_key(batch.cfgs, self.device, self.code)
        e = self.entries.get(key)
        if e is not None:
            self.hits += 1
            batch.set_step_mode(e["mode"])
            batch.set_item_nodes(e["item_nodes"])
            batch.set_blocks(e["blocks"])
            return (e["mode"], e["item_nodes"], e["blocks"]), True
        self.misses += 1
        batch.autotune(trials)
        mode, items, blocks = batch.tuning()
        self.entries[key] = {"mode": mode, "item_nodes": items, "blocks": blocks}
        self.save()
        return (mode, items, blocks), False
