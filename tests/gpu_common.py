"""Shared helpers of the GPU tests (context fixture, case printing)."""
import sys

import pytest

from paper_2007_07627_amd import binding as B


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="session")
def ctx():
    h = B.icp_create(0, 16 << 30)
    yield h
    B.icp_destroy(h)
