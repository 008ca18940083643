"""The package's command line: argument handling on the CPU (the `run`
subcommand itself needs a GPU and is exercised by tests/test_gpu_cli.py)."""
import argparse

import numpy as np
import pytest

import workloads
from paper_2604_26423_amd import __main__ as cli


def test_instance_recipe_matches_the_workloads():
    a = argparse.Namespace(weights=None, n=12, seed=0)
    assert np.array_equal(cli._weights(a, np), workloads.complete_graph_tenths(12, 0))


def test_weights_file(tmp_path):
    f = tmp_path / "w.txt"
    f.write_text("1 2 3\n4 5 6\n")
    a = argparse.Namespace(weights=str(f), n=None, seed=0)
    assert list(cli._weights(a, np)) == [1, 2, 3, 4, 5, 6]


def test_run_without_instance_or_gpu_exits():
    with pytest.raises(SystemExit):
        cli.main(["run", "--p", "3"])          # neither --n nor --weights (or no GPU)
    with pytest.raises(SystemExit):
        cli.main(["run", "--p", "3", "--adjoint", "sideways", "--n", "8"])
