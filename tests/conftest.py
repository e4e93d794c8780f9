import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_handworked():
    """Parse tests/golden/handworked_d2.txt -> (points, eps, minpts, counts, core, labels)."""
    rows = []
    header = None
    with open(os.path.join(GOLDEN, "handworked_d2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if header is None:
                e, m = line.split()
                header = (float(e), int(m))
                continue
            rows.append([int(v) for v in line.split()])
    a = np.array(rows, dtype=np.int64)
    assert (a[:, 0] == np.arange(len(a))).all()
    pts = a[:, 1:3].astype(np.float32)
    return pts, header[0], header[1], a[:, 3], a[:, 4].astype(bool), a[:, 5]


@pytest.fixture(scope="session")
def handworked():
    return load_handworked()
