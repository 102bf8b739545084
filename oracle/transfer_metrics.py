"""Plain FP64 oracle of the transfer-matrix metrics.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's AutoAlign section and its "Transfer matrix analysis parameters"
list name nine properties of the batch transfer matrix and define them in
words only (insertion loss; mode dependent loss, "a.k.a. matrix condition
number"; total diagonal power; diagonal over off-diagonal power, on average,
for the best and the worst batch element, and with coupling inside a
degenerate HG mode group counted as signal). The same section says how the
matrix is built from a batch: combined polarisations give a
batch x (pol x mode) matrix; independent polarisations give a
(batch x pol) x (pol x mode) matrix whose cross-polarisation entries are zero,
so that a missing polarisation drives the mode dependent loss to -inf. It
can also analyse A A* instead of A. The readings taken here (dB scales, which
entries are "diagonal"), with s_k the singular values of A and D = A (or
A A*):

  IL        10 log10(mean_k s_k^2)
  MDL       10 log10(min_k s_k^2 / max_k s_k^2)            (<= 0 dB)
  DIAG      10 log10(mean_i |D_ii|^2),  i < min(rows, cols)
  SNRAVG    10 log10(sum_i |D_ii|^2 / sum_{(i,j) off the diagonal} |D_ij|^2)
  DIAGBEST  10 log10(max_i |D_ii|^2);   DIAGWORST: min
  SNRBEST   10 log10(max_i |D_ii|^2 / sum_{j != i} |D_ij|^2); SNRWORST: min
  SNRMG     as SNRAVG, with every (i, j) whose modes share polarisation and
            HG group m+n counted as signal

Rows i >= min(rows, cols) have no diagonal entry; their power counts as
off-diagonal in SNRAVG and SNRMG. The singular values come from numpy's SVD
(a library routine).
"""
from __future__ import annotations

import math

import numpy as np

from .holo_oracle import mode_list

METRICS = ["IL", "MDL", "DIAG", "SNRAVG", "DIAGBEST", "DIAGWORST", "SNRBEST", "SNRWORST", "SNRMG"]


def _db(x: float) -> float:
    if x <= 0.0:
        return -math.inf
    if math.isinf(x):
        return math.inf
    return 10.0 * math.log10(x)


def transfer_matrix(coefs: np.ndarray, pol_independent: bool) -> np.ndarray:
    """coefs [batch][pol][mode] -> the batch transfer matrix (FP64 complex).
    Combined: row b, column p*M + m. Independent: row p*batch + b, column
    p*M + m, zero where the row's and the column's polarisations differ."""
    c = np.asarray(coefs, dtype=np.complex128)
    b, npol, m = c.shape
    if not pol_independent:
        return c.reshape(b, npol * m)
    a = np.zeros((npol * b, npol * m), dtype=np.complex128)
    for p in range(npol):
        a[p * b:(p + 1) * b, p * m:(p + 1) * m] = c[:, p, :]
    return a


def column_keys(npol: int, group_count: int, groups=None) -> np.ndarray:
    """(pol, mode group) of every column of the transfer matrix, as one
    integer. The groups are the HG groups m + n of `group_count` groups, or
    the given group id of each mode (another basis)."""
    if groups is None:
        groups = [m + n for m, n in mode_list(group_count)]
    groups = np.asarray(groups, dtype=np.int64)
    span = int(groups.max()) + 1 if groups.size else 1
    return np.concatenate([p * span + groups for p in range(npol)])


def transfer_metrics(coefs: np.ndarray, group_count: int, pol_independent: bool = False,
                     mul_conj_trans: bool = False, groups=None) -> dict:
    """The nine metrics of the batch transfer matrix, in dB. `groups`: the
    mode group of each column mode when the coefficients are not HG (an LG
    basis keeps the HG groups; a custom basis gives each mode its own)."""
    c = np.asarray(coefs, dtype=np.complex128)
    npol = c.shape[1]
    a = transfer_matrix(c, pol_independent)
    s2 = np.linalg.svd(a, compute_uv=False) ** 2
    out = {"IL": _db(float(np.mean(s2))), "MDL": _db(float(s2.min() / s2.max())) if s2.max() > 0 else -math.inf}

    d = a @ a.conj().T if mul_conj_trans else a
    p = np.abs(d) ** 2
    nd = min(p.shape)
    diag = np.array([p[i, i] for i in range(nd)])
    total = float(p.sum())
    dsum = float(diag.sum())
    out["DIAG"] = _db(float(diag.mean()))
    out["SNRAVG"] = _db(dsum / (total - dsum)) if total > dsum else math.inf
    out["DIAGBEST"] = _db(float(diag.max()))
    out["DIAGWORST"] = _db(float(diag.min()))
    rows = p[:nd].sum(axis=1)
    snr = np.array([diag[i] / (rows[i] - diag[i]) if rows[i] > diag[i] else math.inf for i in range(nd)])
    out["SNRBEST"] = _db(float(snr.max()))
    out["SNRWORST"] = _db(float(snr.min()))

    # SNRMG: index k (row or column of D) stands for the mode of column k of A
    # (a frame meant to excite that mode); indices past the modes match nothing
    keys = column_keys(npol, group_count, groups)

    def key(n):
        k = np.arange(n)
        return np.where(k < keys.size, np.concatenate([keys, np.zeros(max(0, n - keys.size), np.int64)])[:n],
                        -1 - k)

    same = key(nd)[:, None] == key(p.shape[1])[None, :]
    sig = float(p[:nd][same].sum())
    out["SNRMG"] = _db(sig / (total - sig)) if total > sig else math.inf
    return out
