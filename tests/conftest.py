import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# ---------------------------------------------------------------------------
# The 500 Mbp database of the batched, uneven and served workloads (200
# genomes x 2.5 Mbp, per-genome GC ~ U(0.3, 0.7), seed 1) and the oracle's
# index over it, built once per session for the full-size GPU tests.
# ---------------------------------------------------------------------------

@pytest.fixture(scope="session")
def batched_db():
    import synth
    db = synth.workload_batched_db()
    return dict(db=db, ga=db.ascii())


@pytest.fixture(scope="session")
def batched_oracle(batched_db):
    import oracle
    oracle.set_threads(0)
    return oracle.Index(batched_db["ga"], 21, 11)
