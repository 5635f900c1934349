import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# Method parameters shared by every test (windows, cuts and fit settings are
# the neighbour-search and fit constants of the reconstruction; both the
# oracle and the GPU library receive them from here).
NB = dict(win_y=2.5, win_z=2.5, cut_y=0.6, cut_z=0.75)
MIN_HITS = 5
FIT = dict(bz=0.5, sigma_y=0.05, sigma_z=0.06, max_sin=0.999, var_sin0=1.0, var_tgl0=1.0,
           var_qpt0=100.0)


@pytest.fixture(scope="session")
def nb_params():
    return dict(NB)


@pytest.fixture(scope="session")
def fit_params():
    return dict(FIT)
