import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running check (full-size workloads, long CPU pins)")


def alm_index(lmax: int, l: int, m: int) -> int:
    return m * (2 * lmax + 1 - m) // 2 + l


def ell_of_index(lmax: int) -> np.ndarray:
    """l for every healpy-ordered entry."""
    return np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])


def m_of_index(lmax: int) -> np.ndarray:
    return np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])


def per_l_rel_err(a, ref, lmax: int) -> np.ndarray:
    """err_l = ||a_l. - ref_l.||_2 / ||ref_l.||_2 over m = 0..l (norm-wise per l)."""
    L = ell_of_index(lmax)
    num = np.bincount(L, weights=np.abs(np.asarray(a) - np.asarray(ref)) ** 2, minlength=lmax + 1)
    den = np.bincount(L, weights=np.abs(np.asarray(ref)) ** 2, minlength=lmax + 1)
    return np.sqrt(num / np.maximum(den, 1e-300))


@pytest.fixture(scope="session")
def oracle():
    from oracle import ref
    ref._load()
    return ref


# Measured figures that tests state (error curves and the like): collected during the run and
# printed in the terminal summary, so they reach the log whatever the verbosity.
_MEASURED = []


@pytest.fixture(scope="session")
def measured():
    return _MEASURED


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if _MEASURED:
        terminalreporter.section("measured")
        for line in _MEASURED:
            terminalreporter.write_line(line)
