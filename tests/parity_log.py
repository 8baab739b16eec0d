"""Tolerance checks that can also record the measured error.

parity(what, err, tol) asserts err < tol; when the environment variable TVMC_PARITY_LOG names
a file, every check also appends one JSON line (test, quantity, measured error, tolerance), so
one GPU run documents how much of each tolerance the arithmetic actually uses."""
import json
import os


def parity(what, err, tol):
    path = os.environ.get("TVMC_PARITY_LOG")
    if path:
        test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
        with open(path, "a") as f:
            f.write(json.dumps({"test": test, "what": what, "err": float(err), "tol": float(tol)}) + "\n")
    assert err < tol, (what, err, tol)
