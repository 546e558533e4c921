"""On-disk index files: plain .npy arrays plus a JSON manifest.

Holds no arithmetic of the method; it only writes and reads arrays, checks
their SHA-256 and regenerates the base vectors and queries from the seeded
generator.  Layout of ``<root>/<workload>/``:

  manifest.json    workload parameters, medoid, array shapes and digests
  codebooks.npy    float32 [m][256][d/m]
  codes.npy        uint8   [n][m]
  adj.npy          uint32  [n][R], 0xFFFFFFFF marks an empty slot, or
  adj.bits.npy     the same ids bit-packed (manifest "packed_bits" = w):
                   ids in w = bit_length(n) bits each (an empty slot as n),
                   little-endian within uint64 words
  gt_ids.npy       uint32  [nq][k_gt]   exact nearest neighbours
  gt_dists.npy     float64 [nq][k_gt]
  <name>.npy       optional further arrays (manifest "extra_arrays"), e.g.
                   codebooks_m16 / codes_m16: the same base encoded with
                   another number of subspaces

Base vectors and queries are not stored: ``load`` regenerates them from the
workload's seeds and checks them against the digests in the manifest.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
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


# fields added later, left out of the comparison while they hold their
# default, so indexes written before them stay valid
LATER_DEFAULTS = {"unit": False}


def _index_params(w) -> dict:
    d = json.loads(json.dumps(dataclasses.asdict(w)))
    for key in SEARCH_ONLY:
        d.pop(key, None)
    for key, v in LATER_DEFAULTS.items():
        if d.get(key) == v:
            d.pop(key)
    return d


def _stored_params(man) -> dict:
    d = dict(man["workload"])
    for key in SEARCH_ONLY:
        d.pop(key, None)
    for key, v in LATER_DEFAULTS.items():
        if d.get(key) == v:
            d.pop(key)
    return d


def pack_ids(a: np.ndarray, n: int):
    """uint32 ids (0xFFFFFFFF = empty) in bit_length(n) bits each; returns
    (uint64 words, width)."""
    w = max(1, int(n).bit_length())
    v = a.reshape(-1).astype(np.uint64)
    v[v == 0xFFFFFFFF] = n
    g = 64 // math.gcd(64, w)          # ids per group of whole words
    nw = g * w // 64
    v = np.concatenate([v, np.zeros((-len(v)) % g, np.uint64)]).reshape(-1, g)
    out = np.zeros((v.shape[0], nw), np.uint64)
    for i in range(g):
        word, sh = divmod(i * w, 64)
        out[:, word] |= v[:, i] << np.uint64(sh)
        if sh + w > 64:
            out[:, word + 1] |= v[:, i] >> np.uint64(64 - sh)
    return out.reshape(-1), w


def unpack_ids(words: np.ndarray, shape, n: int, w: int) -> np.ndarray:
    """Inverse of pack_ids."""
    g = 64 // math.gcd(64, w)
    nw = g * w // 64
    count = int(np.prod(shape))
    words = words.reshape(-1, nw)
    out = np.empty((words.shape[0], g), np.uint64)
    mask = np.uint64((1 << w) - 1)
    for i in range(g):
        word, sh = divmod(i * w, 64)
        x = words[:, word] >> np.uint64(sh)
        if sh + w > 64:
            x |= words[:, word + 1] << np.uint64(64 - sh)
        out[:, i] = x & mask
    ids = out.reshape(-1)[:count].astype(np.uint32)
    ids[ids == n] = 0xFFFFFFFF
    return ids.reshape(shape)


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
        man["arrays"][name] = {"shape": list(a.shape), "dtype": str(a.dtype),
                               "sha256": digest(a)}
        if name == "adj":
            words, width = pack_ids(a, w.n)
            np.save(os.path.join(p, "adj.bits.npy"), words, allow_pickle=False)
            man["arrays"][name]["packed_bits"] = width
            stale = os.path.join(p, "adj.npy")
            if os.path.exists(stale):
                os.remove(stale)
        else:
            np.save(os.path.join(p, name + ".npy"), a, allow_pickle=False)
    if base is not None:
        man["base_sha256"] = digest(base)
    if queries is not None:
        man["queries_sha256"] = digest(queries)
    with open(os.path.join(p, "manifest.json.tmp"), "w") as f:
        json.dump(man, f, indent=1)
    os.replace(os.path.join(p, "manifest.json.tmp"),
               os.path.join(p, "manifest.json"))
    return p


def save_extra(w: Workload, arrays: dict, root: str | None = None) -> str:
    """Add arrays beside an existing index (digests in the manifest)."""
    p = path_for(w, root)
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    ex = man.setdefault("extra_arrays", {})
    for name, a in arrays.items():
        if name in ARRAYS or not name.isidentifier():
            raise ValueError(f"bad extra array name {name!r}")
        a = np.ascontiguousarray(a)
        np.save(os.path.join(p, name + ".npy"), a, allow_pickle=False)
        ex[name] = {"shape": list(a.shape), "dtype": str(a.dtype),
                    "sha256": digest(a)}
    with open(os.path.join(p, "manifest.json.tmp"), "w") as f:
        json.dump(man, f, indent=1)
    os.replace(os.path.join(p, "manifest.json.tmp"),
               os.path.join(p, "manifest.json"))
    return p


def extra_names(w: Workload, root: str | None = None) -> list:
    with open(os.path.join(path_for(w, root), "manifest.json")) as f:
        return sorted(json.load(f).get("extra_arrays", {}))


def load_extra(w: Workload, names, root: str | None = None,
               verify: bool = True) -> dict:
    p = path_for(w, root)
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    if _stored_params(man) != _index_params(w):
        raise ValueError(f"{p}: built for different workload parameters")
    out = {}
    for name in names:
        meta = man.get("extra_arrays", {}).get(name)
        if meta is None:
            raise KeyError(f"{p}: no extra array {name!r}")
        a = np.load(os.path.join(p, name + ".npy"), allow_pickle=False)
        if list(a.shape) != meta["shape"] or str(a.dtype) != meta["dtype"]:
            raise ValueError(f"{p}/{name}.npy: shape/dtype mismatch")
        if verify and digest(a) != meta["sha256"]:
            raise ValueError(f"{p}/{name}.npy: content digest mismatch")
        out[name] = a
    return out


def exists(w: Workload, root: str | None = None) -> bool:
    p = path_for(w, root)
    if not os.path.exists(os.path.join(p, "manifest.json")):
        return False
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    return (man.get("format") == FORMAT_VERSION
            and _stored_params(man) == _index_params(w))


def load(w: Workload, root: str | None = None, verify: bool = True,
         with_base: bool = True) -> dict:
    """Return a dict with base, queries, medoid and the stored arrays."""
    p = path_for(w, root)
    with open(os.path.join(p, "manifest.json")) as f:
        man = json.load(f)
    if man.get("format") != FORMAT_VERSION:
        raise ValueError(f"{p}: index format {man.get('format')} is stale")
    if _stored_params(man) != _index_params(w):
        raise ValueError(f"{p}: built for different workload parameters")
    out = {"medoid": int(man["medoid"]), "manifest": man}
    for name in ARRAYS:
        meta = man["arrays"][name]
        if meta.get("packed_bits"):
            words = np.load(os.path.join(p, name + ".bits.npy"),
                            allow_pickle=False)
            a = unpack_ids(words, tuple(meta["shape"]), w.n,
                           int(meta["packed_bits"]))
        else:
            a = np.load(os.path.join(p, name + ".npy"), allow_pickle=False)
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


def repack(w: Workload, root: str | None = None) -> str:
    """Rewrite an index written with a plain adj.npy in the packed form
    (same arrays and digests)."""
    d = load(w, root=root, verify=True, with_base=False)
    man = d["manifest"]
    base_sha, q_sha = man.get("base_sha256"), man.get("queries_sha256")
    p = save(w, {k: d[k] for k in ARRAYS}, d["medoid"], man.get("extra"),
             root=root)
    with open(os.path.join(p, "manifest.json")) as f:
        new = json.load(f)
    new["base_sha256"], new["queries_sha256"] = base_sha, q_sha
    with open(os.path.join(p, "manifest.json.tmp"), "w") as f:
        json.dump(new, f, indent=1)
    os.replace(os.path.join(p, "manifest.json.tmp"),
               os.path.join(p, "manifest.json"))
    return p


if __name__ == "__main__":
    import sys
    from . import WORKLOADS
    if len(sys.argv) == 3 and sys.argv[1] == "repack":
        print(repack(WORKLOADS[sys.argv[2]]))
    else:
        print("usage: python -m synth.store repack <workload>")
