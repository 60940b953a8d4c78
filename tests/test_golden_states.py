"""CPU checks of the stored full-size oracle states (tests/golden/oracle_state_*): the stored
vector is the one the metadata describes (SHA-256), the inputs the seeded generators build
today are the ones the oracle ran on, and the state carries the oracle's own guarantees
(unitarity within its bound, the whole interval covered, the bound within the tolerance)."""

import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("make_oracle_states", os.path.join(GOLDEN, "make_oracle_states.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _stored(name):
    mk = _maker()
    npy, meta_path = mk.state_paths(name)
    if not (os.path.exists(npy) and os.path.exists(meta_path)):
        pytest.skip(f"no stored oracle state for {name}")
    with open(meta_path) as f:
        meta = json.load(f)
    return mk, np.load(npy, allow_pickle=False), meta


@pytest.mark.slow
@pytest.mark.parametrize("name", ["xxz_L20", "bose_K12", "paper_d1565904"])
def test_stored_state_is_consistent(name):
    mk, v, meta = _stored(name)
    spec = W.WORKLOADS[name]
    assert v.dtype == np.complex128 and v.shape == (meta["dim"],)
    assert hashlib.sha256(np.ascontiguousarray(v, dtype="<c16").tobytes()).hexdigest() == meta["state_sha256"]
    assert (meta["kind"], meta["size"], meta["seed"], meta["t"], meta["tol"], meta["m"]) == \
        (spec["kind"], spec["size"], spec["seed"], spec["t"], spec["tol"], spec["m"])
    # the oracle's own guarantees: the interval is covered, the bound obeys the tolerance, the
    # steps add up to t, and the state is unitary to within its bound (plus rounding)
    assert meta["t_reached"] == meta["t"]
    assert meta["err_bound"] <= meta["tol"]
    assert abs(sum(meta["taus"]) - meta["t"]) <= 1e-9 * meta["t"]
    assert len(meta["taus"]) == meta["steps"] and meta["matvecs"] == meta["m"] * meta["steps"]
    assert abs(np.linalg.norm(v) - 1.0) <= meta["err_bound"] + 1e-12
    # the inputs the generators build today are those the oracle ran on
    wl = W.workload(name)
    assert wl.H.dim == meta["dim"] and wl.H.nnz == meta["nnz"]
    assert mk.input_digest(wl.H, wl.v0) == meta["input_sha256"]
