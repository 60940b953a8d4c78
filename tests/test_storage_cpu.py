"""The matrix facts the storage tests rely on, checked on the CPU: how many distinct
(column - row, value) pairs and distinct values the test matrices hold off the diagonal, which
decides the storage kind the library picks (at most 255 / 65535 pairs: 1- / 2-byte pair codes;
else at most 255 / 65535 values: value codes beside the columns; else CSR), and that the
few-valued fixtures are Hermitian with real diagonals."""

import numpy as np
import pytest

import workloads as W
from tests.exact import few_values_hermitian, random_hermitian_csr
from workloads import memory_burden as MB


def distinct(H):
    rows = np.repeat(np.arange(H.dim), np.diff(H.row_ptr)).astype(np.int64)
    off = rows != H.col
    re = H.val.real[off].view(np.int64)
    im = H.val.imag[off].view(np.int64)
    pairs = np.unique(np.stack([H.col[off].astype(np.int64) - rows[off], re, im], 1), axis=0).shape[0]
    values = np.unique(np.stack([re, im], 1), axis=0).shape[0]
    diag = H.val[~off]
    return pairs, values, bool(np.all(diag.imag.view(np.int64) == 0)), int(np.max(np.bincount(rows[~off])))


def kind(H):
    pairs, values, real_diag, max_diag = distinct(H)
    if not real_diag or max_diag > 1:
        return "csr"
    if pairs <= 65535:
        return "packed8" if pairs <= 255 else "packed16"
    if values <= 65535:
        return "coded8" if values <= 255 else "coded16"
    return "csr"


@pytest.mark.parametrize("name,make,want", [
    ("xxz10", lambda: W.xxz_chain(10, seed=1)[0], "packed8"),
    ("bose8_5", lambda: W.bosonic_chain(8, 5, 3)[0], "packed16"),
    ("paper_fig1", lambda: MB.memory_burden_model()[0], "packed8"),
    ("paper_4_4_2_6", lambda: MB.memory_burden_model(K=4, Kp=4, Nm=2, N0=6)[0], "packed8"),
    ("paper_5_5_3_8", lambda: MB.memory_burden_model(K=5, Kp=5, Nm=3, N0=8)[0], "packed16"),
    ("random300", lambda: random_hermitian_csr(300, 0.03, seed=2), "packed16"),
    ("random3000", lambda: random_hermitian_csr(3000, 0.01, seed=3), "csr"),
    ("few40", lambda: few_values_hermitian(3000, 0.01, 5, 40), "coded8"),
    ("few2000", lambda: few_values_hermitian(3000, 0.01, 5, 2000), "coded16"),
    ("few40_s10", lambda: few_values_hermitian(3000, 0.01, 10, 40), "coded8"),
])
def test_storage_kind_of_the_test_matrices(name, make, want):
    H = make()
    assert kind(H) == want, (name, distinct(H))


def test_xxz_ring_has_two_pairs_per_bond():
    for L in (8, 10, 12):
        pairs, _, real_diag, _ = distinct(W.xxz_chain(L, seed=4)[0])
        assert pairs == 2 * L and real_diag


@pytest.mark.parametrize("n_values", [40, 2000])
def test_few_valued_fixture_is_hermitian(n_values):
    F = few_values_hermitian(3000, 0.01, 5, n_values)
    A = F.to_scipy()
    assert abs(A - A.conj().T).max() == 0.0
    assert np.all(A.diagonal().imag == 0.0)
    _, values, _, _ = distinct(F)
    assert values == 2 * n_values  # each table value and its conjugate
