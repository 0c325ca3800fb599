"""JSON cache of autotuned launch configurations.

The fastest launch of an ensemble depends on the device, on the library
build and on what the step kernel is instantiated and sized for: velocity
set, collision, storage, arithmetic, shifting, and the list of lattice sizes.
The key hashes exactly these; the wall geometry, tau, the force and the wall
and EQ values are left out (they change which tiles the step skips and a few
operations per cell, never whether a launch is valid).  An entry holds the
lbm_launch fields that the autotuner chose except graph_steps, which stays
the caller's choice.

The file is one JSON object {key: entry}.  A write reads the file, adds or
replaces one entry and renames a temporary file over it, so readers never see
a partial file; of two processes writing at once, one entry may be lost.  A
file that is missing or not valid JSON reads as empty.

Host logic only: nothing here runs on the device."""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

LAUNCH_FIELDS = ("mode", "block", "cells_per_lane", "persistent")


def ensemble_key(params, device: str, library_id: str) -> str:
    """Hex digest naming one ensemble on one device with one library build.
    `params`: a sequence of LbmParams (or objects with the same fields)."""
    plist = list(params)
    p0 = plist[0]
    desc = {
        "device": device,
        "library": library_id,
        "q": int(p0.q), "collision": int(p0.collision), "storage": int(p0.storage),
        "arith": int(p0.arith), "unshifted": int(p0.unshifted),
        "sizes": [[int(p.nx), int(p.ny), int(p.nz)] for p in plist],
    }
    return hashlib.sha256(json.dumps(desc, sort_keys=True).encode()).hexdigest()


def _read(path: str) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def load(path: str, key: str) -> dict | None:
    """The cached launch fields for `key`, or None."""
    entry = _read(path).get(key)
    if not isinstance(entry, dict):
        return None
    try:
        return {f: int(entry[f]) for f in LAUNCH_FIELDS}
    except (KeyError, TypeError, ValueError):
        return None


def store(path: str, key: str, launch: dict, note: str = "") -> None:
    """Add or replace the entry for `key` (the LAUNCH_FIELDS of `launch`)."""
    data = _read(path)
    entry = {f: int(launch[f]) for f in LAUNCH_FIELDS}
    if note:
        entry["note"] = note
    data[key] = entry
    folder = os.path.dirname(os.path.abspath(path))
    os.makedirs(folder, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".tuning-", suffix=".json", dir=folder)
    try:
        with os.fdopen(fd, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise
