"""Helpers for the GPU tests: load the HIP library (no fallback) and name
each GPU case on stdout before it runs."""
import sys

import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1911_12954_amd import _lib
    _lib.load()   # raises when libtrg.so is missing: no fallback path exists
    return torch


def announce(*parts):
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()
