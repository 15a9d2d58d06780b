"""The paper's execution-time model (Sec. 4.5) as bench.py evaluates it,
against the bounds the paper prints for its three processors. CPU only."""
import numpy as np
import pytest

import bench
from tests import _witness as W


def test_model_reproduces_the_printed_bounds():
    g = W.load_golden("execution_time_model.txt")
    rates = {int(r[0]): (r[1], r[2]) for r in g["rates"]}
    cases = {int(c[0]): (c[1], c[2:5]) for c in g["cases"]}
    checked = 0
    for proc, case, *times in g["times"]:
        stream, dgemm = rates[int(proc)]
        words, ops = cases[int(case)]
        for order in range(3):
            model = bench.model_bound_ns(words, ops[order], stream, dgemm)
            if int(proc) == 2 and int(case) in (2, 4) and order == 2:
                # the Xeon Phi SSQ prism cells repeat the Xeon SQS values;
                # the model gives 65.3 and 77.7 ns, the values the measured
                # times' percentages of the bound imply
                assert times[order] == pytest.approx(
                    bench.model_bound_ns(words, ops[1], 67, 0.18), abs=0.005)
                assert model == pytest.approx({2: 65.33, 4: 77.66}[int(case)], abs=0.01)
                continue
            assert model == pytest.approx(times[order], abs=0.005), (proc, case, order)
            checked += 1
    assert checked == 34
