"""Shared helpers of the GPU tests (context fixture, case printing)."""
import sys

import pytest

from paper_2007_07627_amd import binding as B


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


def torch_first():
    """Initialise torch's GPU runtime (torch carries its own HIP runtime
    library) before the library's first HIP call, the order bench.py uses;
    tests that hand torch tensors to the library need it."""
    import torch
    torch.cuda.init()
    torch.zeros(1, device="cuda:0")


@pytest.fixture(scope="session")
def ctx():
    torch_first()
    h = B.icp_create(0, 16 << 30)
    yield h
    B.icp_destroy(h)
