"""Analysis kernels on the GPU through the C ABI: the eigen step of the MDL
metric on matrices with a planted spectrum."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _planted(n, rank, seed):
    """U diag(lam) U^H with a random unitary U and eigenvalues spread over
    eight decades (zeros past `rank`): the spectrum is known exactly."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q = q * (np.diag(r) / np.abs(np.diag(r)))
    lam = np.zeros(n)
    lam[:rank] = np.logspace(0, -8, rank) if rank > 1 else 1.0
    rng.shuffle(lam)
    a = (q * lam) @ q.conj().T
    return 0.5 * (a + a.conj().T), np.sort(lam)


@pytest.mark.parametrize("n,rank", [(1, 1), (2, 2), (7, 7), (90, 90), (90, 40), (96, 96), (97, 97), (250, 250)])
def test_hermitian_eigenvalues_planted_spectrum(n, rank):
    """Every eigenvalue of a planted Hermitian positive semi-definite matrix,
    in LDS (n <= 96) and in global memory (n > 96), odd and even n, and
    rank-deficient: within 1e-12 of the largest, and the small ones to 1e-5
    relative (what the MDL metric's ratio needs)."""
    _torch()
    import paper_2204_02348_amd as dh
    a, lam = _planted(n, rank, 100 + n + rank)
    _say(f"Jacobi eigenvalues n={n} rank={rank}")
    w = dh.hermitian_eigenvalues(a)
    err = np.abs(w - lam)
    assert err.max() <= 1e-12 * lam.max(), err.max()
    big = lam > 1e-6
    assert np.all(err[big] <= 1e-5 * lam[big])


def test_hermitian_eigenvalues_rejects():
    _torch()
    import paper_2204_02348_amd as dh
    with pytest.raises(dh.DhError) as e:
        dh.hermitian_eigenvalues(np.zeros((2049, 2049), np.complex128))
    assert e.value.code == dh.ERR_INVALIDDIMENSION
