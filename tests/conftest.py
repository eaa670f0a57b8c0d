import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def trained():
    """Both networks trained by the library on its own data, in the full
    configuration the benchmark uses (same seeds, so the same networks):
    {2: message-passing blob, 0: Fig. 2 per-node blob}.  About 10 s of GPU."""
    from paper_2504_14494_amd import train
    data = train.datasets(train.DataConfig())
    out = {}
    for rounds in (2, 0):
        tr, _ = train.train(train.DataConfig(), steps=2000, batch=32, rounds=rounds, data=data)
        out[rounds] = tr.blob
    return out
