import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2206_10435_amd.workloads import Query  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU check")


def load_fig1() -> Query:
    """The three tables of Figure 1 as a chain query T1(A,B) - T2(B,C) - T3(C,D)."""
    rows = {"T1": [], "T2": [], "T3": []}
    with open(os.path.join(GOLDEN, "fig1_tables.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t, a, b = line.split()
            rows[t].append((int(a), int(b)))
    tables = []
    for t in ("T1", "T2", "T3"):
        arr = np.array(rows[t], dtype=np.int32)
        tables.append([arr[:, 0].copy(), arr[:, 1].copy()])
    return Query("fig1", tables, [-1, 0, 1], [0, 0, 0], [0, 1, 1])


def load_fig2():
    gfjs = {}
    rows = []
    facts = {}
    with open(os.path.join(GOLDEN, "fig2_gfjs.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "gfjs":
                gfjs.setdefault(p[1], []).append((int(p[2]), int(p[3])))
            elif p[0] == "rows":
                rows.append(tuple(int(x) for x in p[1:]))
            else:
                facts[p[0]] = int(p[1])
    return gfjs, rows, facts


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.build()
    return O
