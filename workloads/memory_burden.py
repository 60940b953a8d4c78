"""The paper's exemplary system (Sec. "Exemplary System", eq. fullHamiltonianSimple).

Modes, in this order: a_0 (n_0), b_0 (m_0), memory qubits a_1..a_K, memory
qubits a'_1..a'_K'.  The two sector totals N_0 = n_0 + m_0 and
N_m = sum n_k + sum n'_k' (eq. subsetOccupations) are conserved, so the basis
is the product of the (N_0 + 1) two-mode states and the C(K + K', N_m) qubit
configurations, enumerated in descending lexicographic order:
dimension (N_0 + 1) * C(K + K', N_m)  (588 for the default parameters).

Terms:
  C_0 (a0+ b0 + b0+ a0)
  + eps_m (1 - n_0/N_c) sum_k n_k + eps_m (1 - n_0/(N_c - dN_c)) sum_k' n'_k'
  + C_m [ sum_{k,k'} f_1(k,k') (a_k+ a'_k' + h.c.) + sum_{k<l} f_2(k,l) (a_k+ a_l + h.c.)
          + sum_{k'<l'} f_3(k',l') (a'_k'+ a'_l' + h.c.) ]
with f_i = F_i - 1 if F_i < 0.5 else F_i and
F_i(k,l) = (sqrt(2) (k + dk_i)^3 + sqrt(7) (l + dl_i)^5) mod 1,
dk_1 = dk_2 = 1, dk_3 = K + 1, dl_1 = dl_3 = K + 1, dl_2 = 1.
Initial state (eq. initialStateSimple): |N_0, 0, 1 x N_m, 0, ..., 0>.
"""

from math import comb

import numpy as np

from .bosonic import FockIndex, capped_fock_basis, hopping_triplets
from .csr import from_triplets

DEFAULTS = dict(eps_m=np.sqrt(20.0), N0=20, Nc=20.0, dNc=12.0, K=4, Kp=4, C0=1.0, Cm=1.0, Nm=2)


def memory_burden_dim(N0: int, K: int, Kp: int, Nm: int) -> int:
    return (N0 + 1) * comb(K + Kp, Nm)


def _f(i: int, k: int, l: int, K: int) -> float:
    dk = {1: 1, 2: 1, 3: K + 1}[i]
    dl = {1: K + 1, 2: 1, 3: K + 1}[i]
    F = (np.sqrt(2.0) * float(k + dk) ** 3 + np.sqrt(7.0) * float(l + dl) ** 5) % 1.0
    return F - 1.0 if F < 0.5 else F


def memory_burden_model(**params):
    """Return (CSR, v0, basis) for eq. fullHamiltonianSimple with the initial state
    of eq. initialStateSimple; unspecified parameters take the paper's defaults."""
    p = dict(DEFAULTS)
    p.update(params)
    K, Kp, N0, Nm = int(p["K"]), int(p["Kp"]), int(p["N0"]), int(p["Nm"])
    if not (0 < p["dNc"] < p["Nc"]) or Nm > K:
        raise ValueError("need 0 < dN_c < N_c and N_m <= K")
    sector0 = capped_fock_basis([N0, N0], N0)
    sector1 = capped_fock_basis([1] * (K + Kp), Nm)
    basis = np.hstack([np.repeat(sector0, sector1.shape[0], axis=0),
                       np.tile(sector1, (sector0.shape[0], 1))]).astype(np.uint8)
    d = basis.shape[0]
    caps = [N0, N0] + [1] * (K + Kp)
    index = FockIndex(basis)

    n0 = basis[:, 0].astype(np.float64)
    nk = basis[:, 2:2 + K].sum(axis=1).astype(np.float64)
    nkp = basis[:, 2 + K:].sum(axis=1).astype(np.float64)
    diag = p["eps_m"] * (1.0 - n0 / p["Nc"]) * nk + p["eps_m"] * (1.0 - n0 / (p["Nc"] - p["dNc"])) * nkp

    rows = [np.arange(d, dtype=np.int64)]
    cols = [np.arange(d, dtype=np.int64)]
    vals = [diag.astype(np.complex128)]

    def hop_pair(mode_a, mode_b, amp):
        # amp (a+_{mode_a} a_{mode_b} + h.c.)
        for src, dst in ((mode_b, mode_a), (mode_a, mode_b)):
            t, s, v = hopping_triplets(basis, index, src, dst, amp, caps)
            rows.append(t); cols.append(s); vals.append(v.astype(np.complex128))

    hop_pair(0, 1, p["C0"])
    for k in range(1, K + 1):
        for kp in range(1, Kp + 1):
            hop_pair(1 + k, 1 + K + kp, p["Cm"] * _f(1, k, kp, K))
    for k in range(1, K + 1):
        for l in range(k + 1, K + 1):
            hop_pair(1 + k, 1 + l, p["Cm"] * _f(2, k, l, K))
    for kp in range(1, Kp + 1):
        for lp in range(kp + 1, Kp + 1):
            hop_pair(1 + K + kp, 1 + K + lp, p["Cm"] * _f(3, kp, lp, K))

    csr = from_triplets(d, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals),
                        f"memory_burden_K{K}_Kp{Kp}_N0{N0}_Nm{Nm}")
    start = np.zeros((1, basis.shape[1]), dtype=np.uint8)
    start[0, 0] = N0
    start[0, 2:2 + Nm] = 1
    v0 = np.zeros(d, dtype=np.complex128)
    v0[index.lookup(start)[0]] = 1.0
    return csr, v0, basis
