"""Stored oracle results for the full-size workloads, and the fingerprints
the parity checks compare them with.

Each file ``<family>.json`` under this directory is written by
``make_golden.py``, which calls only the CPU oracle (``oracle/``) on inputs
from ``workloads.py``.  A case records the run's parameters (including the
block the library's tuner assigns, ``workloads.tuned_block``), the totals
(events, M, bond sum, lattice digest) and SHA-256 fingerprints of the
per-subdomain arrays: final spins (int8, row-major), event digests (uint64),
committed flips (int64) and carry (j, anchor, acc as int64, one row per
subdomain).  A fingerprint is the hash of the array's little-endian bytes in
that dtype, so any single differing element changes it.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

DTYPES = {"spins": "<i1", "sub_digest": "<u8", "sub_flips": "<i8", "carry": "<i8"}


def sha(a, kind: str) -> str:
    """SHA-256 of the array's bytes in the fixed dtype of `kind`."""
    x = np.ascontiguousarray(np.asarray(a).astype(DTYPES[kind], copy=False))
    return hashlib.sha256(x.tobytes()).hexdigest()


def fingerprints(spins, sub_digest, sub_flips, carry3) -> dict:
    return {"spins": sha(spins, "spins"), "sub_digest": sha(sub_digest, "sub_digest"),
            "sub_flips": sha(sub_flips, "sub_flips"), "carry": sha(carry3, "carry")}


def path(family: str) -> str:
    return os.path.join(HERE, f"{family}.json")


def load(family: str) -> dict:
    """{case id: case record} of one family."""
    with open(path(family)) as f:
        doc = json.load(f)
    return {c["id"]: c for c in doc["cases"]}


def available(family: str) -> bool:
    return os.path.exists(path(family))
