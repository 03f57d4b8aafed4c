import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def read_golden_rows(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, vals = line.split(":", 1)
            rows[key.strip()] = [int(v, 16) for v in vals.split()]
    return rows


def read_labelled_vectors():
    out = []
    with open(os.path.join(GOLDEN, "labelled_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            hexs, exp, label, src = [p.strip() for p in line.split("|")]
            out.append((bytes.fromhex(hexs), int(exp), label, src))
    return out
