"""Reader for the text fixtures under tests/golden/."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_sections(name: str) -> dict:
    """Parse an INI-like fixture: [section] then `key = values` lines."""
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = out.setdefault(line[1:-1], {})
                continue
            key, _, val = line.partition("=")
            cur[key.strip()] = val.strip()
    return out


def matrix(s: str) -> np.ndarray:
    rows = [[int(x) for x in r.split()] for r in s.split(";")]
    return np.array(rows, dtype=np.int32)


def ints(s: str) -> list:
    return [int(x) for x in s.split()]


def worked_examples() -> dict:
    return read_sections("worked_examples.txt")
