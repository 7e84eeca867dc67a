import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (large rasters)")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    """Parse a golden fixture: '#' comments, optional 'tile th tw', then 'dirs'
    and 'A' blocks of whitespace-separated integers."""
    import numpy as np
    blocks, cur, tile = {}, None, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("tile"):
                tile = tuple(int(v) for v in line.split()[1:3])
                continue
            if line in ("dirs", "A"):
                cur = blocks.setdefault(line, [])
                continue
            cur.append([int(v) for v in line.split()])
    return (np.array(blocks["dirs"], dtype=np.uint8), np.array(blocks["A"], dtype=np.uint64), tile)


GOLDEN_FILES = sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
