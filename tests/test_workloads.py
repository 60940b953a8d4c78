"""Generator pins: closed-form sizes, Hermiticity, conservation laws, the basis map."""

import json
import os
from math import comb

import numpy as np
import pytest

import workloads as W
from workloads.bosonic import FockIndex
from workloads.xxz import magnon_sector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _check_csr(H):
    rp, col = H.row_ptr.astype(np.int64), H.col.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == H.nnz and np.all(np.diff(rp) >= 1)
    rows = np.repeat(np.arange(H.dim), np.diff(rp))
    # sorted, unique columns inside each row, diagonal present
    key = rows * H.dim + col
    assert np.all(np.diff(key) > 0)
    assert np.count_nonzero(rows == col) == H.dim
    A = H.to_scipy()
    assert abs(A - A.conj().T).max() == 0.0


@pytest.mark.parametrize("L", [3, 4, 5, 8, 11, 12])
def test_xxz_nnz_closed_form_and_hermitian(L):
    H, v0 = W.xxz_chain(L, seed=7)
    assert H.dim == 2 ** L and H.nnz == W.xxz_nnz(L) == 2 ** L * (1 + L / 2)
    _check_csr(H)
    assert abs(np.linalg.norm(v0) - 1) < 1e-14


def test_xxz_named_sizes():
    assert W.xxz_nnz(12) == 28672
    assert W.xxz_nnz(20) == 11534336
    assert W.xxz_nnz(22) == 50331648


def test_xxz_conserves_magnetisation():
    L = 9
    H, _ = W.xxz_chain(L, seed=3)
    rp = H.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(H.dim), np.diff(rp))
    pop = lambda s: sum(((s >> i) & 1) for i in range(L))
    assert np.all(pop(rows) == pop(H.col.astype(np.int64)))
    assert sum(len(magnon_sector(L, n)) for n in range(L + 1)) == 2 ** L


def test_xxz_matrix_elements_match_spin_algebra():
    # Build a 4-site ring from Pauli matrices and compare entry by entry.
    L = 4
    H, _ = W.xxz_chain(L, seed=11, with_v0=False)
    rng = np.random.default_rng(11)
    h = rng.uniform(-1, 1, L)
    phi = rng.uniform(0, 2 * np.pi, L)
    sp_ = np.array([[0, 0], [1, 0]], dtype=complex)  # raises: |down>=0 -> |up>=1 (bit value 1 = up)
    sm = sp_.T.copy()
    sz = np.diag([-0.5, 0.5]).astype(complex)
    I = np.eye(2)

    def site(op, i):
        # bit i of the basis index <-> kron factor (L-1-i) (most significant first)
        mats = [I] * L
        mats[L - 1 - i] = op
        out = mats[0]
        for m in mats[1:]:
            out = np.kron(out, m)
        return out

    ref = np.zeros((16, 16), dtype=complex)
    for i in range(L):
        j = (i + 1) % L
        ref += 0.5 * (np.exp(1j * phi[i]) * site(sp_, i) @ site(sm, j)
                      + np.exp(-1j * phi[i]) * site(sm, i) @ site(sp_, j))
        ref += 0.5 * site(sz, i) @ site(sz, j) + h[i] * site(sz, i)
    assert np.allclose(H.to_scipy().toarray(), ref, atol=1e-15)


@pytest.mark.parametrize("K,N", [(2, 5), (3, 3), (5, 4), (6, 6), (8, 3)])
def test_fock_dimension_and_index_round_trip(K, N):
    basis = W.fock_basis(K, N)
    assert basis.shape == (comb(N + K - 1, K - 1), K)
    assert np.all(basis.sum(axis=1) == N)
    assert tuple(basis[0]) == (N,) + (0,) * (K - 1)
    idx = FockIndex(basis)
    assert np.array_equal(idx.lookup(basis), np.arange(basis.shape[0]))


def test_bosonic_chain_hermitian_and_number_conserving():
    H, v0 = W.bosonic_chain(5, 5, seed=3)
    assert H.dim == W.fock_dim(5, 5) == 126
    _check_csr(H)
    # hopping entries: sqrt((n_k+1) n_{k+1}) |a_k| with |a_k| in [0.5, 1.5]
    A = H.to_scipy().toarray()
    off = np.abs(A - np.diag(np.diag(A)))
    assert off.max() <= 1.5 * 5 + 1e-12
    assert np.allclose(np.diag(A).imag, 0)


def test_bosonic_cfg_size():
    H, _ = W.bosonic_chain(12, 12, seed=3)
    assert H.dim == comb(23, 11) == 1352078
    assert H.nnz == 16871582


def test_paper_dimensions_from_golden():
    gold = json.load(open(GOLDEN))
    for e in gold["dimensions"]:
        assert W.memory_burden_dim(e["N0"], e["K"], e["Kp"], e["Nm"]) == e["dim"]
        # enumerate the qubit sector the way the model does and check the count too
        qubits = W.capped_fock_basis([1] * (e["K"] + e["Kp"]), e["Nm"])
        assert (e["N0"] + 1) * qubits.shape[0] == e["dim"]


def test_memory_burden_model_small():
    H, v0, basis = W.memory_burden_model()
    assert H.dim == 588 == W.memory_burden_dim(20, 4, 4, 2)
    _check_csr(H)
    assert np.count_nonzero(v0) == 1 and v0.max() == 1.0
    # both sector totals are conserved by construction of the basis
    assert np.all(basis[:, :2].sum(axis=1) == 20) and np.all(basis[:, 2:].sum(axis=1) == 2)
    # the mode a_0 carries N_0 quanta in the initial state
    k = int(np.nonzero(v0)[0][0])
    assert basis[k, 0] == 20 and basis[k, 1] == 0 and list(basis[k, 2:4]) == [1, 1]


def test_batch_and_serving_draws_are_deterministic():
    a = W.batch_jobs(8)
    b = W.batch_jobs(8)
    assert [(j.L, j.n_v0, j.t, j.tol) for j in a] == [(j.L, j.n_v0, j.t, j.tol) for j in b]
    assert all(10 <= j.L <= 18 and 1 <= j.n_v0 <= 8 and 1 <= j.t <= 100 for j in a)
    r = W.serving_requests(16, qps=5.0)
    assert all(x.arrival < y.arrival for x, y in zip(r, r[1:]))
    assert all((x.kind == "xxz" and 14 <= x.size <= 22) or (x.kind == "bose" and 10 <= x.size <= 12) for x in r)
