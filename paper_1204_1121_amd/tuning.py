"""Launch-shape cache: autotuned (P, o) per table shape and size bucket.

blip_autotune picks the fastest (positions per workgroup P, table elements
per lane o) on the caller's buffers; this module keeps the winners in a JSON
file keyed by architecture, storage dtype, orbital count, grid, path (single
block or batched), outputs (with derivatives, or values only) and the
power-of-two size bucket, and restores them into a table with
blip_set_shape, so a run does not need to re-tune.  Shapes measured for the
acceptance-ratio pass (the ratio epilogue with the values and Laplacian rows)
are kept under their own path and restored into the table's ratio mode, so
they never change the shape of a plain launch.  A table holds one shape per
size bucket and mode, so a caller that uses one table for values only and for
derivatives restores the output mode it runs.
"""
from __future__ import annotations

import json
import os

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def bucket(npos: int) -> int:
    """Lower end of the power-of-two size bucket holding npos."""
    lo = 1
    while lo * 2 <= npos:
        lo *= 2
    return lo


def key(table, npos: int, batched: bool, values_only: bool = False, ratio: bool = False,
        arch: str = "gfx950") -> str:
    n1, n2, n3 = table.n
    path = (("batched" if batched else "block") + ("-values" if values_only else "")
            + ("-ratio" if ratio else ""))
    return f"{arch}/{table.storage}/L{table.norb}/{n1}x{n2}x{n3}/{path}/{bucket(npos)}"


class TuneCache:
    def __init__(self, path: str = DEFAULT_PATH):
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, table, npos: int, batched: bool = False, values_only: bool = False,
            ratio: bool = False):
        return self.entries.get(key(table, npos, batched, values_only, ratio))

    def put(self, table, npos: int, batched: bool, best: dict, note: str = "",
            values_only: bool = False, ratio: bool = False) -> None:
        e = {"tile_pos": int(best["tile_pos"]), "vec": int(best["vec"]),
             "us": float(best["us"])}
        if note:
            e["note"] = note
        self.entries[key(table, npos, batched, values_only, ratio)] = e

    def apply(self, table, npos: int, batched: bool = False, values_only: bool = False,
              ratio: bool = False) -> bool:
        """Set the cached shape on the table; False if none is cached."""
        e = self.get(table, npos, batched, values_only, ratio)
        if e is None:
            return False
        table.set_shape(npos, e["tile_pos"], e["vec"], batched=batched, ratio=ratio)
        return True

    def save(self, path: str | None = None) -> None:
        with open(path or self.path, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
            f.write("\n")
