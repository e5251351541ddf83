"""Workload descriptions: the synthetic scenes and CEM settings, read from JSON.

This module only reads files and draws nothing: it holds no arithmetic of the
method.  It is the one input source shared by the GPU library's binding and by
the test harness that drives the CPU oracle.
"""
import json
import os

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def names():
    return sorted(f[:-5] for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))


def load(name):
    """Return the workload dict for `name` (a file stem under configs/)."""
    with open(os.path.join(CONFIG_DIR, name + ".json")) as f:
        return json.load(f)
