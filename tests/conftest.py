import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in one process, in file order; nothing to reorder here.
    pass


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_cylinder_golden():
    """The paper's cylinder results (tests/golden/cylinder_present.txt):
    {"steady": {Re: (Cd, L/R)}, "unsteady": {Re: (Cd, L/R, St)}}."""
    out = {"steady": {}, "unsteady": {}}
    with open(os.path.join(GOLDEN, "cylinder_present.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            kind, re_, vals = line[0], int(line[1]), [None if v == "-" else float(v) for v in line[2:]]
            out[kind][re_] = tuple(v for v in vals if v is not None)
    return out


@pytest.fixture(scope="session")
def paper_cylinder():
    return read_cylinder_golden()
