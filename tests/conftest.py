"""Shared pytest configuration.

Markers:
  gpu   -- needs an MI355X (runs through the C-ABI library on a real device)
  slow  -- CPU tests that relax fields with the oracle for a minute or more;
           run them with --runslow
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False, help="run the slow oracle relaxations")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU (MI355X); calls the HIP library through the C ABI")
    config.addinivalue_line("markers", "slow: long CPU relaxations with the oracle; needs --runslow")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--runslow"):
        return
    skip = pytest.mark.skip(reason="slow oracle relaxation; pass --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
