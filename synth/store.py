"""On-disk index files: plain .npy arrays plus a JSON manifest.

Holds no arithmetic of the method; it only writes and reads arrays, checks
their SHA-256 and regenerates the base vectors and queries from the seeded
generator.  Layout of ``<root>/<workload>/``:

  manifest.json    workload parameters, medoid, array shapes and digests
  codebooks.npy    float32 [m][256][d/m]
  codes.npy        uint8   [n][m]
  adj.npy          uint32  [n][R], 0xFFFFFFFF marks an empty slot
  gt_ids.npy       uint32  [nq][k_gt]   exact nearest neighbours
  gt_dists.npy     float64 [nq][k_gt]

Base vectors and queries are not stored: ``load`` regenerates them from the
workload's seeds and checks them against the digests in the manifest.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os

import numpy as np

from . import Workload, base_and_queries

DEFAULT_ROOT = os.environ.get(
    "BANG_INDEX_DIR",
    os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                 "indexcache"))
ARRAYS = ("codebooks", "codes", "adj", "gt_ids", "gt_dists")
FORMAT_VERSION = 1
# search-time parameters: they do not change the stored index
SEARCH_ONLY = ("Ls", "k")


def _index_params(w) -> dict:
    d = json.loads(json.dumps(dataclasses.asdict(w)))
    for key in SEARCH_ONLY:
        d.pop(key, None)
    return d


def digest(a: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(np.ascontiguousarray(a).data)
    return h.hexdigest()


def path_for(w: Workload, root: str | None = None) -> str:
    return os.path.join(root or DEFAULT_ROOT, w.name)


def save(w: Workload, arrays: dict, medoid: int, extra: dict | None = None,
         base: np.ndarray | None = None, queries: np.ndarray | None = None,
         root: str | None = None) -> str:
    p = path_for(w, root)
    os.makedirs(p, exist_ok=True)
    man = {"format": FORMAT_VERSION, "workload": dataclasses.asdict(w),
           "medoid": int(medoid), "arrays": {}, "extra": extra or {}}
    for name in ARRAYS:
        a = np.ascontiguousarray(arrays[name])
        np.save(os.path.join(p, name + ".npy"), a, allow_pickle=False)
        man["arrays"][name] = {"shape": list(a.shape), "dtype": str(a.dtype),
                               "sha256": digest(a)}
    if base is not None:
        man["base_sha256"] = digest(base)
    if queries is not None:
        man["queries_sha256"] = digest(queries)
    with open(os.path.join(p, "manifest.json.tmp"), "w") as f:
        json.dump(man, f, indent=1)
    os.replace(os.path.join(p, "manifest.json.tmp"),
               os.path.join(p, "manifest.json"))
    return p


def exists(w: Workload, root: str | None = None) -> bool:
    p = path_for(w, root)
    if not os.path.exists(os.path.join(p, "manifest.json")):
        return False
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    stored = dict(man["workload"])
    for key in SEARCH_ONLY:
        stored.pop(key, None)
    return man.get("format") == FORMAT_VERSION and stored == _index_params(w)


def load(w: Workload, root: str | None = None, verify: bool = True,
         with_base: bool = True) -> dict:
    """Return a dict with base, queries, medoid and the stored arrays."""
    p = path_for(w, root)
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    if man.get("format") != FORMAT_VERSION:
        raise ValueError(f"{p}: index format {man.get('format')} is stale")
    stored = dict(man["workload"])
    for key in SEARCH_ONLY:
        stored.pop(key, None)
    if stored != _index_params(w):
        raise ValueError(f"{p}: built for different workload parameters")
    out = {"medoid": int(man["medoid"]), "manifest": man}
    for name in ARRAYS:
        a = np.load(os.path.join(p, name + ".npy"), allow_pickle=False)
        meta = man["arrays"][name]
        if list(a.shape) != meta["shape"] or str(a.dtype) != meta["dtype"]:
            raise ValueError(f"{p}/{name}.npy: shape/dtype mismatch")
        if verify and digest(a) != meta["sha256"]:
            raise ValueError(f"{p}/{name}.npy: content digest mismatch")
        out[name] = a
    if with_base:
        base, queries = base_and_queries(w)
        if verify and man.get("base_sha256") not in (None, digest(base)):
            raise ValueError("regenerated base vectors differ from the index")
        if verify and man.get("queries_sha256") not in (None, digest(queries)):
            raise ValueError("regenerated queries differ from the index")
        out["base"], out["queries"] = base, queries
    return out
