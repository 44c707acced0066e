import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_golden(name):
    """Parse a tests/golden fixture into (src, dst, t) int arrays."""
    import numpy as np
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if len(parts) == 3:
                s, d, hms = parts
                day = 0
            else:
                s, d, day, hms = parts
            h, m, sec = (int(x) for x in hms.split(":"))
            rows.append((int(s), int(d), int(day) * 86400 + h * 3600 + m * 60 + sec))
    a = np.array(rows, dtype=np.int64)
    return a[:, 0].astype(np.int32), a[:, 1].astype(np.int32), a[:, 2]
