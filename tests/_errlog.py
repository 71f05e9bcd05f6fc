"""Measured-error log of the GPU parity tests.

With the environment variable LBM_ERROR_LOG naming a file, record() appends
one JSON line per measured error (test id, quantity, labels, value), which is
how the bounds of the 16-bit storages in these tests were set (a small
multiple of the largest error measured on the GPU).  Without it, record() does
nothing."""
import json
import os


def record(quantity: str, value, **labels):
    path = os.environ.get("LBM_ERROR_LOG")
    if not path:
        return
    test = os.environ.get("PYTEST_CURRENT_TEST", "").rsplit(" ", 1)[0]
    with open(path, "a") as fh:
        fh.write(json.dumps(dict(test=test, quantity=quantity, value=float(value), **labels)) + "\n")
