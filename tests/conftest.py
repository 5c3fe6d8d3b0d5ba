import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests cannot run without a device; skip them loudly rather than fail on import.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def read_golden_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


def read_golden_matrices(name):
    """Parse 'name nrows ncols' headers followed by rows."""
    import numpy as np
    rows = read_golden_table(name)
    out = {}
    i = 0
    while i < len(rows):
        nm, nr, nc = rows[i][0], int(rows[i][1]), int(rows[i][2])
        data = [[float(v) for v in rows[i + 1 + r]] for r in range(nr)]
        out[nm] = np.array(data)
        assert out[nm].shape == (nr, nc)
        i += 1 + nr
    return out
