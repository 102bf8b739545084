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
    _say(f"eigenvalues n={n} rank={rank}")
    w = dh.hermitian_eigenvalues(a)
    err = np.abs(w - lam)
    assert err.max() <= 1e-12 * lam.max(), err.max()
    big = lam > 1e-6
    assert np.all(err[big] <= 1e-5 * lam[big])


@pytest.mark.parametrize("n", [5, 90, 130])
def test_hermitian_eigenvalues_use_the_hermitian_part(n):
    """A matrix that is not Hermitian: the eigenvalues are those of its
    Hermitian part (A + A^H) / 2 (numpy's eigvalsh of that part), in the
    LDS form and in the global-memory form."""
    _torch()
    import paper_2204_02348_amd as dh
    rng = np.random.default_rng(500 + n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    _say(f"eigenvalues of the Hermitian part, n={n}")
    w = dh.hermitian_eigenvalues(a)
    ref = np.linalg.eigvalsh(0.5 * (a + a.conj().T))
    assert np.abs(w - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(w - ref).max()


def test_hermitian_eigenvalues_not_finite():
    """Entries that are not finite: DH_ERR_ERROR (the kernel flags the
    tridiagonal as not finite instead of returning numbers)."""
    _torch()
    import paper_2204_02348_amd as dh
    a = np.eye(6, dtype=np.complex128)
    a[2, 3] = np.nan
    a[3, 2] = np.nan
    _say("eigenvalues of a matrix with NaN entries")
    with pytest.raises(dh.DhError) as e:
        dh.hermitian_eigenvalues(a)
    assert e.value.code == dh.ERR_ERROR


def test_hermitian_eigenvalues_rejects():
    _torch()
    import paper_2204_02348_amd as dh
    with pytest.raises(dh.DhError) as e:
        dh.hermitian_eigenvalues(np.zeros((2049, 2049), np.complex128))
    assert e.value.code == dh.ERR_INVALIDDIMENSION


# ---------------------------------------------------------------- batch summary
import dh_synth  # noqa: E402
import oracle  # noqa: E402


def _compare_summary(got, ref, x, y, tol):
    """Continuous parameters within tol (centres relative to the axis span);
    the peak index by value: the reference intensity there is the maximum."""
    span_x, span_y = abs(x[-1] - x[0]) + abs(x[1] - x[0]), abs(y[-1] - y[0]) + abs(y[1] - y[0])
    for k, name in enumerate(oracle.PARAMETERS):
        g, r = got[k], ref[k]
        if name == "MAXABSIDX":
            continue
        if name in ("COMX",):
            err = np.abs(g - r).max() / span_x
        elif name in ("COMY", "COMYWRAP"):
            d = np.abs(g - r)
            if name == "COMYWRAP":
                d = np.minimum(d, span_y - d)      # the same point across the wrap
            err = d.max() / span_y
        else:
            err = (np.abs(g - r) / np.maximum(np.abs(r), 1e-300)).max()
        _say(f"  {name}: max err {err:.2e}")
        assert err <= tol, (name, err)


@pytest.mark.parametrize("mode", [1, 0])
def test_batch_summary_field_plane_vs_oracle(mode):
    """Plane 1 on 5 frames 640x512 (2 pols): the same analysis as the oracle's
    on the GPU's own fields (peak index identical, the rest to rounding), and
    within 1e-5 of the oracle's analysis of its own fields."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(1)
    f, _ = dh_synth.make_frames(cfg, n_frames=5)
    params = dict(cfg["params"], ifft_mode=mode, keep_fields=1)
    _say(f"batch summary, field plane, IFFT mode {mode}")
    plan = dh.Plan(params, max_batch=5)
    plan.process(torch.from_numpy(f).cuda(), 5, None)
    got, tot, x, y = plan.batch_summary(1)
    gf = plan.fields()
    ax, ay = plan.field_axes()
    plan.destroy()
    ox, oy = oracle.field_axes(params)
    assert np.abs(x - ox).max() <= 1e-15 and np.abs(y - oy).max() <= 1e-15
    assert np.array_equal(ax, x) and np.array_equal(ay, y)
    same, same_tot, _, _ = oracle.batch_summary_field(gf, params)
    assert np.array_equal(got[4], same[4])                    # the same argmax on the same values
    _compare_summary(got, same, x, y, 1e-6)
    assert np.linalg.norm(tot - same_tot) <= 1e-6 * np.linalg.norm(same_tot)
    of = np.stack([oracle.process_frame(f[i].astype(np.float64), params)["field"] for i in range(5)])
    ref, ref_tot, _, _ = oracle.batch_summary_field(of, params)
    _compare_summary(got, ref, x, y, 1e-5)
    inten = np.abs(of) ** 2
    for b in range(5):
        for p in range(2):
            k = int(got[4, p, b])
            assert inten[b, p].ravel()[k] >= (1 - 1e-5) * inten[b, p].max()


@pytest.mark.parametrize("idx,cam,n", [(1, 0, 3), (3, 0, 4)])
def test_batch_summary_fourier_plane_vs_oracle(idx, cam, n):
    """Plane 0 (the half Fourier plane of each pol window) of a few frames,
    f32 two-pol and a u16 camera, against the oracle's explicit DFT."""
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(idx, cam)
    f, _ = dh_synth.make_frames(cfg, n_frames=n)
    _say(f"batch summary, Fourier plane, recipe {idx} camera {cam}, {n} frames")
    plan = dh.Plan(cfg["params"], max_batch=n)
    got, tot, x, y = plan.batch_summary(0, torch.from_numpy(f).cuda(), n)
    plan.destroy()
    ref, ref_tot, ox, oy = oracle.batch_summary_fourier(f.astype(np.float64), cfg["params"])
    assert np.abs(x - ox).max() <= 1e-12 and np.abs(y - oy).max() <= 1e-12
    _compare_summary(got, ref, x, y, 1e-5)
    assert np.array_equal(got[4], ref[4])                      # the DC bin
    assert np.linalg.norm(tot - ref_tot) <= 1e-5 * np.linalg.norm(ref_tot)


def test_batch_summary_rejections():
    torch = _torch()
    import paper_2204_02348_amd as dh
    cfg = dh_synth.config(0)
    plan = dh.Plan(cfg["params"], max_batch=1)
    for plane, code in [(2, dh.ERR_INVALIDARGUMENT), (1, dh.ERR_ERROR)]:   # no fields kept
        with pytest.raises(dh.DhError) as e:
            plan.batch_summary(plane, torch.zeros(128 * 128, device="cuda"), 1)
        assert e.value.code == code
    plan.destroy()
