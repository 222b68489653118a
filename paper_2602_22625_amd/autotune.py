"""Autotuner for the raster launch: screen-tile size x launch schedule.

Candidates are tile edges T in {8, 16, 32} (one, four or sixteen 8x8-pixel waves per
workgroup) crossed with the schedules of dbmp_set_schedule: one workgroup per tile in image
order, one workgroup per tile longest list first, or a persistent grid of 2, 4 or 8 workgroups
per compute unit that takes the longest-first tiles in fixed strides or from a device queue, 1
or 16 items per grab. Each candidate is timed over a few steps of the
caller's workload and the fastest is kept in a JSON cache keyed by a bucket of the workload's
shape (image sizes and primitive counts) and by a digest of the built library, so a rebuilt
kernel is tuned again.

The tile list lengths, and so the best choice, follow from the image sizes, the primitive count
and their scales (the cost of a tile is its list length times its pixel count); the bucket
rounds sizes to 128 px and counts to powers of two.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

SCHED_NAMES = {0: "grid", 1: "sorted", 2: "persistent"}


def candidates(tiles=(8, 16, 32), persistent_wgs=(2, 4, 8), grabs=(0, 1, 16)):
    """(tile, schedule, workgroups_per_cu, items_per_grab) tuples."""
    out = []
    for t in tiles:
        out.append((t, 0, 4, 1))
        out.append((t, 1, 4, 1))
        for w in persistent_wgs:
            for g in grabs:
                out.append((t, 2, w, g))
    return out


def cfg_name(c):
    if c[1] == 2:
        return "T%d/persistent/%d/%s" % (c[0], c[2], "stride" if c[3] == 0 else "grab%d" % c[3])
    return "T%d/%s" % (c[0], SCHED_NAMES[c[1]])


def bucket_key(shapes):
    """Key of a workload given as [(H, W, N), ...] (one entry per image of a batch)."""
    def b(h, w, n):
        r = lambda v: max(128, int(round(v / 128.0)) * 128)
        p = 1 << max(0, int(math.floor(math.log2(max(n, 1)))))
        return "%dx%d:%d" % (r(h), r(w), p)
    parts = sorted(b(*s) for s in shapes)
    key = "n%d|" % len(parts) + ",".join(parts)
    if len(key) > 200:
        key = "n%d|sha1:%s" % (len(parts), hashlib.sha1(key.encode()).hexdigest())
    return key


def library_digest():
    from . import capi
    h = hashlib.sha256()
    with open(capi.LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


class Autotuner:
    def __init__(self, path=None, version=None):
        if path is None:
            path = os.environ.get("DBMP_TUNE_CACHE") or os.path.join(
                os.path.expanduser("~"), ".cache", "diffbmp_tune.json")
        self.path = path
        self.version = version
        self._db = None

    def _load(self):
        if self._db is None:
            try:
                with open(self.path) as f:
                    self._db = json.load(f)
            except (OSError, ValueError):
                self._db = {}
        return self._db

    def _save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self._db, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, key):
        e = self._load().get(key)
        if e is None or e.get("version") != self.version:
            return None
        return (e["tile"], e["schedule"], e["workgroups_per_cu"], e["items_per_grab"])

    def tune(self, key, measure, cands=None, force=False):
        """measure(cfg) -> seconds per step for cfg = (tile, schedule, workgroups_per_cu,
        items_per_grab).
        Returns the fastest cfg, from the cache unless `force` or the cache is stale."""
        if not force:
            hit = self.lookup(key)
            if hit is not None:
                return hit
        cands = cands or candidates()
        times = {}
        for cfg in cands:
            times[cfg] = float(measure(cfg))
        best = min(cands, key=lambda c: times[c])
        self._load()[key] = {
            "version": self.version, "tile": best[0], "schedule": best[1],
            "workgroups_per_cu": best[2], "items_per_grab": best[3],
            "seconds_per_step": times[best],
            "all": {cfg_name(c): times[c] for c in cands},
        }
        self._save()
        return best

    def entry(self, key):
        return self._load().get(key)
