"""Tuned knob settings kept on disk, keyed by GPU architecture, graph and batch width.

``dawn_autotune`` searches the knobs of one resident graph; this module keeps
what it found between processes, so that a later run on the same graph and
device family loads the settings instead of searching again.  An entry's key
is the GPU architecture name (for example ``gfx950``), a SHA-256 of the
graph's CSR arrays, and the batch width the settings were tuned for (1 for
single-source runs, the number of sources per batch for batched ones).  The
file is JSON; writes replace it atomically.  Nothing here touches a distance.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
import time

import numpy as np

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_params.json")


def graph_signature(row_ptr, col) -> str:
    """SHA-256 (first 16 hex digits) of the int32 CSR: n, row_ptr and col."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    h = hashlib.sha256()
    h.update(np.int64(rp.size - 1).tobytes())
    h.update(rp.tobytes())
    h.update(c.tobytes())
    return h.hexdigest()[:16]


def device_arch(device: int = 0) -> str:
    """The GPU's architecture name without feature suffixes (``gfx950``)."""
    import torch
    name = torch.cuda.get_device_properties(device).gcnArchName
    return name.split(":")[0]


def entry_key(arch: str, signature: str, width: int) -> str:
    return f"{arch}/{signature}/{int(width)}"


def load(path: str | None = None) -> dict:
    try:
        with open(path or DEFAULT_PATH) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def lookup(arch: str, signature: str, width: int, path: str | None = None) -> dict | None:
    """The stored knob settings for the key, or None."""
    e = load(path).get(entry_key(arch, signature, width))
    return dict(e["params"]) if isinstance(e, dict) and "params" in e else None


def store(arch: str, signature: str, width: int, params: dict, path: str | None = None,
          note: str = "") -> None:
    """Record `params` under the key (other entries are kept)."""
    path = path or DEFAULT_PATH
    data = load(path)
    data[entry_key(arch, signature, width)] = {
        "params": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in params.items()},
        "note": note, "time": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime()),
    }
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuned_", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)
