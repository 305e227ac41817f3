"""Tile-shape and path autotuning with a persistent cache.

The library times its candidates itself (``sg_matvec_autotune``: 1, 2 or 4
tiles of 64 rows per work-group of the staged SG matvec; ``ras_autotune``:
the RAS sweep and the dense path with 64 or 32 owned rows per wave).  This
module keys each choice by the workload's shape and the GPU architecture and
keeps it in a JSON file, so a later run on the same shape selects it without
timing (``sg_matvec_select``, ``ras_select``).
"""
from __future__ import annotations

import json
import os
import tempfile
from typing import Optional


def default_path() -> str:
    """``$SGSOLVE_TUNE_CACHE``, else ``$XDG_CACHE_HOME/sgsolve/autotune.json``
    (``~/.cache`` when unset)."""
    env = os.environ.get("SGSOLVE_TUNE_CACHE")
    if env:
        return env
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "sgsolve", "autotune.json")


def make_key(kind: str, arch: str, **shape) -> str:
    """Stable text key: kind, architecture, then the shape fields sorted by name."""
    fields = ",".join(f"{k}={shape[k]}" for k in sorted(shape))
    return f"{kind}|{arch}|{fields}"


class TuneCache:
    """Choices by key, read from and written back to one JSON file.  A missing
    or unreadable file starts an empty cache (the tuner then times again)."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_path()
        self.entries: dict = {}
        try:
            with open(self.path) as f:
                data = json.load(f)
            if isinstance(data, dict) and isinstance(data.get("entries"), dict):
                self.entries = data["entries"]
        except (OSError, ValueError):
            self.entries = {}

    def get(self, key: str):
        return self.entries.get(key)

    def put(self, key: str, value) -> None:
        self.entries[key] = value
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        # write a sibling file, then rename it over the cache (atomic on POSIX)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune.", suffix=".json")
        try:
            with os.fdopen(fd, "w") as f:
                json.dump({"version": 1, "entries": self.entries}, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise
