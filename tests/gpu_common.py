"""Helpers for the GPU parity tests."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def gpu_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1911_06969_amd import binding
    binding.load_library()
    return torch


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
    # also past pytest's capture, so that a long test shows its progress
    print(*a, file=sys.__stderr__, flush=True)
