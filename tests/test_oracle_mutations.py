"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch each one: a dropped term, a wrong sign or index, a
transposed operand, a wrong scale, a wrong ordering."""
import math
import os
import types

import numpy as np
import pytest

import dh_synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "holo_oracle.py")

MUTATIONS = {
    "drop_defocus": ('+ np.pi * gp["defocus"] * (xk[None, :] ** 2 + yl[:, None] ** 2) / lam', ''),
    "tilt_sign": ('phi = (2 * np.pi * (gp["ax"]', 'phi = (-2 * np.pi * (gp["ax"]'),
    "other_cross_term": ('((uu + ax) / rx) ** 2', '((uu - ax) / rx) ** 2'),
    "field_pitch": ('px2=nx * p / fx', 'px2=p'),
    "pixel_origin": ('xj = (np.arange(nx) - nx / 2.0) * p', 'xj = (np.arange(nx) - nx / 2.0 + 1) * p'),
    "subpixel_sign": ('* p - gp["dx"]', '* p + gp["dx"]'),
    "hermite_recurrence": ('- math.sqrt(n / (n + 1)) * psi_prev', '+ math.sqrt(n / (n + 1)) * psi_prev'),
    "hg_norm": ("out * (2.0 ** 0.25 / math.sqrt(waist))", "out * (2.0 ** 0.5 / math.sqrt(waist))"),
    "mode_transpose": ('cm[n, m] for (m, n)', 'cm[m, n] for (m, n)'),
    "mode_order": ('for m in range(g, -1, -1):', 'for m in range(0, g + 1):'),
    "ifft_scale": ('@ gx / (nx * ny)', '@ gx'),
    "ifft_sign": ('gx = np.exp(2j', 'gx = np.exp(-2j'),
    "quadrature_weight": ('* (g["px2"] * g["py2"])', '* (g["px2"])'),
    "mask_radius": ('** 2 <= 1.0', '** 2 <= 0.8'),
    "ifft_size_rule": ('need = int(math.floor(2.0 * r_bins)) + 1', 'need = int(math.floor(r_bins)) + 1'),
    "tilt_axis_swap": ('ay = tilt_bins(params["tilt_deg"][pol][1], ny, p, lam)',
                       'ay = tilt_bins(params["tilt_deg"][pol][0], ny, p, lam)'),
    "power_norm": ('c / math.sqrt(pw)', 'c / pw'),
}


def _mutant(name):
    src = open(SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("oracle_mutant_" + name)
    exec(compile(src.replace(old, new), SRC + ":" + name, "exec"), mod.__dict__)
    return mod


def _checks(o):
    """The pins, run against module `o`; returns the names that fail."""
    bad = []
    # closed-form recovery with defocus, tilt differing per axis, sub-pixel
    # centre, two pols and non-square windows
    cfg = dh_synth.config(1)
    truth = dict(cfg["truth"], defocus=[0.2, -0.15], tilt_deg=[[1.45, 1.55], [1.52, 1.47]],
                 beam_centre=[[0.3 * 20e-6, -0.2 * 20e-6], [-0.4 * 20e-6, 0.1 * 20e-6]])
    cfg = dict(cfg, truth=truth)
    f, c = dh_synth.make_frames(cfg, n_frames=1, quantise=False)
    try:
        r = o.process_frame(f[0], truth)
        if not np.abs(r["coefs_norm"] - c[0]).max() < 1e-8:
            bad.append("recovery")
        # raw scale: unit-power coefficients times A = max|S|; ||c|| = A here
        amp = math.sqrt(float(np.sum(np.abs(r["coefs"]) ** 2)))
        ref_amp = _amp(truth, c[0])
        if not abs(amp - ref_amp) < 1e-8 * ref_amp:
            bad.append("scale")
    except Exception:
        bad.append("crash")
    # paper's FFT/IFFT size pairs
    lam, pix = 1565e-9, 20e-6
    wmax_deg = o.w_max_rad(pix, lam) / o.DEG
    for fft, ifft in [(64, 32), (128, 48), (256, 96), (512, 176), (1024, 336)]:
        if o.ifft_size(o.radius_bins(0.32 * wmax_deg, fft, pix, lam)) != ifft:
            bad.append("sizes")
            break
    # mask area equals the window ellipse
    g = o.geometry(truth)
    m = g["pols"][0]["mask"]
    if abs(m.sum() - math.pi * g["rx"] * g["ry"]) > 0.02 * math.pi * g["rx"] * g["ry"]:
        bad.append("mask_area")
    # mode list order printed in the tests
    if o.mode_list(3) != [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]:
        bad.append("order")
    return bad


def _amp(truth, c):
    half = truth["frame_w"] // truth["pol_count"]
    best = 0.0
    modes = [(m, g - m) for g in range(truth["max_mg"]) for m in range(g, -1, -1)]
    for pol in range(truth["pol_count"]):
        x = (np.arange(half) - half // 2) * truth["pixel_size"] - truth["beam_centre"][pol][0]
        y = (np.arange(truth["frame_h"]) - truth["frame_h"] // 2) * truth["pixel_size"] - truth["beam_centre"][pol][1]
        s = sum(c[pol][k] * np.outer(dh_synth.hg_closed_form(n, y, truth["waist"]),
                                     dh_synth.hg_closed_form(m, x, truth["waist"]))
                for k, (m, n) in enumerate(modes))
        best = max(best, float(np.abs(s).max()))
    return best


def test_unmutated_oracle_passes_the_checks():
    from oracle import holo_oracle
    assert _checks(holo_oracle) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    assert _checks(_mutant(name)) != [], name


# ---------------------------------------------------------------- transfer-matrix metrics
TM_SRC = os.path.join(os.path.dirname(SRC), "transfer_metrics.py")

TM_MUTATIONS = {
    "il_sum": ("np.mean(s2)", "np.sum(s2)"),
    "mdl_inverse": ("s2.min() / s2.max())", "s2.max() / s2.min())"),
    "mdl_amplitude": ("np.linalg.svd(a, compute_uv=False) ** 2", "np.linalg.svd(a, compute_uv=False)"),
    "pol_independence_ignored": ("    if not pol_independent:\n", "    if True:\n"),
    "diag_amplitude": ("p = np.abs(d) ** 2", "p = np.abs(d)"),
    "aa_star_transposed": ("a @ a.conj().T if mul_conj_trans", "a.conj().T @ a if mul_conj_trans"),
    "snr_row_total": ("diag[i] / (rows[i] - diag[i])", "diag[i] / rows[i]"),
    "snrmg_ignores_pol": ("p * span + groups", "groups"),
}


def _tm_mutant(name):
    import oracle
    src = open(TM_SRC).read()
    old, new = TM_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace("from .holo_oracle import mode_list\n", "")
    mod = types.ModuleType("tm_mutant_" + name)
    mod.__dict__["mode_list"] = oracle.mode_list
    exec(compile(src, TM_SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(TM_MUTATIONS))
def test_metric_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    mut = _tm_mutant(name)
    monkeypatch.setattr(oracle, "transfer_metrics", mut.transfer_metrics)
    failed = 0
    for t in [pins.test_metrics_identity_and_scaled_unitary,
              pins.test_metrics_il_mdl_closed_form_from_chosen_singular_values,
              pins.test_metrics_diagonal_and_snr_closed_forms,
              pins.test_metrics_mode_group_snr_counts_coupling_inside_a_group,
              pins.test_metrics_missing_polarisation_combined_vs_independent,
              pins.test_metrics_aa_star_of_a_wide_matrix_and_two_pol_groups]:
        try:
            with np.errstate(divide="ignore", invalid="ignore"):
                t()
        except (AssertionError, FloatingPointError, ZeroDivisionError, ValueError):
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- alignment snap
SNAP_SRC = os.path.join(os.path.dirname(SRC), "align_snap.py")

SNAP_MUTATIONS = {
    "defocus_factor": ("* lam / (2.0 * math.pi))", "* lam / math.pi)"),
    "modes_spread": ("ks = 2.0 * (2 * params[\"max_mg\"] + 1)", "ks = (2 * params[\"max_mg\"] + 1)"),
    "k_axes": ("ky * ky * (pw * (vv - mv) ** 2)", "kx * kx * (pw * (vv - mv) ** 2)"),
    "k_not_central": ("(pw * (uu - mu) ** 2)", "(pw * uu ** 2)"),
    "spread_not_central": ("spread = (sxx - sx * sx / s) / s", "spread = sxx / s"),
    "centre_sign": ("cx + sx / s, cy + sy / s", "cx - sx / s, cy - sy / s"),
    "centre_axes_swapped": ("cx + sx / s, cy + sy / s", "cx + sy / s, cy + sx / s"),
    "not_central": ("mxx += sxx - sx * sx / s", "mxx += sxx"),
    "group_factor": ("(2 * g + 1)", "(2 * g - 1)"),
    "grid_origin": ("(np.arange(fx) - fx / 2.0)", "np.arange(fx)"),
    "amplitude_not_intensity": ("i = np.abs(np.asarray(field, dtype=np.complex128)) ** 2",
                                "i = np.abs(np.asarray(field, dtype=np.complex128))"),
    "pol_not_own": ("cx, cy = params[\"beam_centre\"][pol]", "cx, cy = params[\"beam_centre\"][0]"),
}


def _snap_mutant(name):
    import oracle
    src = open(SNAP_SRC).read()
    old, new = SNAP_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace(
        "from .holo_oracle import field_from_window, geometry, spectrum_window, window_pixels\n", "")
    mod = types.ModuleType("snap_mutant_" + name)
    for k in ("field_from_window", "geometry", "spectrum_window", "window_pixels"):
        mod.__dict__[k] = getattr(oracle, k)
    exec(compile(src, SNAP_SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(SNAP_MUTATIONS))
def test_snap_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    mut = _snap_mutant(name)
    monkeypatch.setattr(oracle, "snap_centre_waist", mut.snap_centre_waist)
    monkeypatch.setattr(oracle, "batch_moments", mut.batch_moments)
    monkeypatch.setattr(oracle, "snap_defocus_magnitude", mut.snap_defocus_magnitude)
    failed = 0
    for t in [pins.test_snap_centre_is_the_offset_of_a_shifted_gaussian,
              pins.test_snap_waist_from_every_mode_of_g_groups,
              pins.test_snap_centre_per_polarisation,
              pins.test_snap_defocus_magnitude_of_a_gaussian_beam,
              pins.test_snap_defocus_magnitude_with_every_mode_of_g_groups]:
        try:
            t()
        except AssertionError:
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- alignment snap: tilt from the whole plane
PLANE_SRC = os.path.join(os.path.dirname(SRC), "plane_snap.py")

PLANE_MUTATIONS = {
    "tilt_sign": ("tilts.append([-uc * binx, -vc * biny])", "tilts.append([uc * binx, vc * biny])"),
    "mirror_rule": ("first = d1 < d2 if d1 != d2 else", "first = d1 > d2 if d1 != d2 else"),
    "centroid_not_periodic": ("sv += w * dv", "sv += w * (_signed((cv + dv) % ny, ny) - cv)"),
    "bins_per_degree_axes": ("binx = params[\"wavelength\"] / (nx *", "binx = params[\"wavelength\"] / (ny *"),
    "centroid_axes_swapped": ("uc = cu + (su / sw", "uc = cu + (sv / sw"),
}


def _plane_mutant(name):
    import oracle
    src = open(PLANE_SRC).read()
    old, new = PLANE_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace("from .holo_oracle import geometry\n", "")
    mod = types.ModuleType("plane_mutant_" + name)
    mod.__dict__["geometry"] = oracle.geometry
    exec(compile(src, PLANE_SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(PLANE_MUTATIONS))
def test_plane_snap_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    mut = _plane_mutant(name)
    monkeypatch.setattr(oracle, "snap_tilt_plane", mut.snap_tilt_plane)
    failed = 0
    for t in [pins.test_plane_snap_finds_the_tilt_of_a_gaussian_beam,
              pins.test_plane_snap_takes_the_term_nearer_the_start,
              pins.test_plane_snap_per_polarisation_on_a_rectangular_window,
              pins.test_plane_snap_term_across_the_plane_edge]:
        try:
            t()
        except AssertionError:
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- IFFT mode 0 and the int16 format
M0_MUTATIONS = {
    "mode0_coarse_pitch": ("fx, fy = (wx, wy) if mode == 1 else (nx, ny)", "fx, fy = (wx, wy)"),
    "mode0_pitch_of_window": ("px2=nx * p / fx, py2=ny * p / fy", "px2=nx * p / wx, py2=ny * p / wy"),
    "mode0_grid_origin": ("xk = (np.arange(g[\"fx\"]) - g[\"fx\"] / 2.0) * g[\"px2\"]\n    yl = (np.arange(g[\"fy\"]) - g[\"fy\"] / 2.0) * g[\"py2\"]\n    # every",
                          "xk = np.arange(g[\"fx\"]) * g[\"px2\"]\n    yl = np.arange(g[\"fy\"]) * g[\"py2\"]\n    # every"),
    "int16_scale_from_real_only": ("float(np.abs(im).max(initial=0.0))", "0.0"),
    "int16_truncates": ("np.rint(re * scale)", "np.trunc(re * scale)"),
    "int16_full_scale": ("INT16_FULL = 32767", "INT16_FULL = 32768"),
    "int16_rounds_half_away": ("qr = np.rint(re * scale)", "qr = np.sign(re * scale) * np.floor(np.abs(re * scale) + 0.5)"),
}


@pytest.mark.parametrize("name", sorted(M0_MUTATIONS))
def test_mode0_and_int16_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    old, new = M0_MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mut = types.ModuleType("m0_mutant_" + name)
    exec(compile(src.replace(old, new), SRC + ":" + name, "exec"), mut.__dict__)
    for k in ("geometry", "field_from_window", "spectrum_window", "process_frame", "fields_to_int16", "overlap"):
        monkeypatch.setattr(oracle, k, getattr(mut, k))
    failed = 0
    tests = [pins.test_mode0_field_is_the_full_size_inverse_fft,
             lambda: pins.test_mode0_closed_form_recovery(0, 0),
             pins.test_int16_peak_maps_to_full_scale_and_round_trips,
             pins.test_int16_ties_to_even_and_zero_field]
    for t in tests:
        try:
            with np.errstate(all="ignore"):
                t()
        except (AssertionError, ValueError, IndexError, OverflowError):
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- basis transforms
BASIS_SRC = os.path.join(os.path.dirname(SRC), "basis.py")

BASIS_MUTATIONS = {
    "l_order_reversed": ("for l in range(n, -n - 1, -2):", "for l in range(-n, n + 1, 2):"),
    "no_conjugate": ("return np.conj(lg) @ (ww.ravel() * hg).T", "return lg @ (ww.ravel() * hg).T"),
    "lg_norm": ("math.factorial(p + abs(l))", "math.factorial(p)"),
    "phi_sign": ("np.exp(1j * l * phi)", "np.exp(-1j * l * phi)"),
    "laguerre_argument": ("special.eval_genlaguerre(p, abs(l), 2.0 * r2)", "special.eval_genlaguerre(p, abs(l), r2)"),
    "hg_axes_swapped": ("np.outer(u[n], u[m]).ravel() for m, n", "np.outer(u[m], u[n]).ravel() for m, n"),
    "block_wrong_group": ("hg[start:start + n + 1], group_count + 4", "hg[start + 1:start + n + 2], group_count + 4"),
    "block_no_conjugate_order": ("b, c[..., start:start + k]", "b.T, c[..., start:start + k]"),
    "custom_extra_columns_used": ("k = min(modes, t.shape[1])", "k = t.shape[1]"),
}


def _basis_mutant(name):
    import oracle
    src = open(BASIS_SRC).read()
    old, new = BASIS_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace("from .holo_oracle import hermite_gauss_1d, mode_list\n", "")
    mod = types.ModuleType("basis_mutant_" + name)
    mod.__dict__["hermite_gauss_1d"] = oracle.hermite_gauss_1d
    mod.__dict__["mode_list"] = oracle.mode_list
    exec(compile(src, BASIS_SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(BASIS_MUTATIONS))
def test_basis_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    mut = _basis_mutant(name)
    for k in ("lg_modes", "lg_function", "hg_to_lg", "lg_blocks", "apply_lg_blocks", "custom_transform",
              "apply_basis"):
        monkeypatch.setattr(oracle, k, getattr(mut, k))
    failed = 0
    for t in [pins.test_lg_transform_is_unitary_and_keeps_groups,
              pins.test_lg_low_orders_are_the_textbook_combinations,
              pins.test_lg_transform_matches_the_closed_form,
              pins.test_lg_transform_matches_fine_grid_overlaps,
              pins.test_custom_transform_uses_only_the_plan_modes,
              pins.test_lg_blocks_are_the_full_transform,
              pins.test_lg_blocks_at_100_groups]:           # the costly pin last
        try:
            with np.errstate(all="ignore"):
                t()
        except (AssertionError, ValueError, IndexError):
            failed += 1
            break
    assert failed > 0, name


# ---------------------------------------------------------------- wavelength sweeps and averaging
SWEEP_SRC = os.path.join(os.path.dirname(SRC), "sweep_avg.py")

SWEEP_MUTATIONS = {
    "interlace_stride_inputs": ("frames[o, a] = a * n_out + j", "frames[o, a] = a * n_in + j"),
    "sweep_ignores_repetition": ("frames[o, a] = (i * avg_count + a) * wl_count + w", "frames[o, a] = (i + a) * wl_count + w"),
    "slow_output_is_fast": ("o = i * wl_count + w if out_order == FAST else w * n_in + i",
                            "o = i * wl_count + w"),
    "slow_input_is_fast": ("j = i * wl_count + w if in_order == FAST else w * n_in + i", "j = i * wl_count + w"),
    "phase_not_removed": ("acc += w[a] * np.exp(-1j * ph[a])", "acc += w[a] * np.exp(1j * ph[a])"),
    "sum_not_mean": ("return acc / w.shape[0], ph", "return acc, ph"),
    "centre_wavelength_tilt": ("g = geometry(dict(params, wavelength=lam))", "g = geometry(dict(params))"),
}


def _sweep_mutant(name):
    import oracle
    src = open(SWEEP_SRC).read()
    old, new = SWEEP_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace(
        "from .holo_oracle import field_from_window, geometry, mask_bins, overlap, power_normalise, spectrum_window\n",
        "")
    mod = types.ModuleType("sweep_mutant_" + name)
    for k in ("field_from_window", "geometry", "mask_bins", "overlap", "power_normalise", "spectrum_window"):
        mod.__dict__[k] = getattr(oracle, k)
    exec(compile(src, SWEEP_SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(SWEEP_MUTATIONS))
def test_sweep_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    mut = _sweep_mutant(name)
    for k in ("frame_index_map", "at_wavelength", "average_windows", "process_sweep"):
        monkeypatch.setattr(oracle, k, getattr(mut, k))
    failed = 0
    for t in [pins.test_frame_index_map_follows_the_paper_patterns,
              pins.test_frame_index_map_output_orders,
              pins.test_sweep_frame_is_processed_at_its_wavelength,
              lambda: pins.test_averaging_aligns_the_phase_of_each_repetition(0),
              lambda: pins.test_averaging_aligns_the_phase_of_each_repetition(1)]:
        try:
            t()
        except (AssertionError, ValueError, IndexError):
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- largest window for a tilt
WIN_SRC = os.path.join(os.path.dirname(SRC), "window_fit.py")

WIN_MUTATIONS = {
    "origin_terms_radius_w": ("w = min(math.hypot(tx, ty) / 3.0,", "w = min(math.hypot(tx, ty) / 2.0,"),
    "no_spectrum_edge": ("w_max_deg - abs(tx), w_max_deg - abs(ty))", "math.inf)"),
    "no_periodic_images": ("for kx in range(-2, 3):\n                for ky in range(-2, 3):",
                           "for kx in range(0, 1):\n                for ky in range(0, 1):"),
    "conjugate_gap_w": ("math.hypot(2 * tx - kx * period, 2 * ty - ky * period) / 2.0",
                        "math.hypot(2 * tx - kx * period, 2 * ty - ky * period) / 1.0"),
    "wrap_origin_image_period": ("math.hypot(tx - kx * period, ty - ky * period) / 3.0",
                                 "math.hypot(tx - kx * w_max_deg, ty - ky * w_max_deg) / 3.0"),
}


@pytest.mark.parametrize("name", sorted(WIN_MUTATIONS))
def test_window_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    src = open(WIN_SRC).read()
    old, new = WIN_MUTATIONS[name]
    assert src.count(old) == 1, name
    mod = types.ModuleType("win_mutant_" + name)
    exec(compile(src.replace(old, new), WIN_SRC + ":" + name, "exec"), mod.__dict__)
    monkeypatch.setattr(oracle, "max_window_radius", mod.max_window_radius)
    failed = 0
    for t in [pins.test_largest_window_at_the_papers_tilt, pins.test_largest_wrapped_window,
              lambda: pins.test_largest_window_by_brute_force(False),
              lambda: pins.test_largest_window_by_brute_force(True)]:
        try:
            t()
        except AssertionError:
            failed += 1
    assert failed > 0, name


# ---------------------------------------------------------------- batch summary
SUM_SRC = os.path.join(os.path.dirname(SRC), "batch_summary.py")

SUM_MUTATIONS = {
    "aeff_not_squared": ("out[5] = (s * da) ** 2", "out[5] = (s * da)"),
    "com_over_power": ("out[1] = float(i.sum(axis=0) @ x) / s", "out[1] = float(i.sum(axis=0) @ x) / (s * da)"),
    "total_without_cell": ("out[0] = s * da", "out[0] = s"),
    "maxabs_is_intensity": ("out[3] = math.sqrt(flat[k])", "out[3] = flat[k]"),
    "index_column_major": ("flat = i.ravel()", "flat = i.T.ravel()"),
    "wrap_period_off_by_one": ("period = h * dy", "period = (h - 1) * dy"),
    "fourier_rows_unshifted": ("ky = np.arange(ny) - ny // 2", "ky = np.arange(ny)"),
    "fourier_x_axis_pitch": ("x = np.arange(nx // 2 + 1) * lam / (nx * p) / DEG",
                             "x = np.arange(nx // 2 + 1) * lam / (ny * p) / DEG"),
    "batch_entry_mean": ("total = intensities.sum(axis=0)", "total = intensities.mean(axis=0)"),
}


@pytest.mark.parametrize("name", sorted(SUM_MUTATIONS))
def test_summary_pins_catch_planted_mistake(name, monkeypatch):
    import oracle
    import tests.test_oracle_pins as pins
    src = open(SUM_SRC).read()
    old, new = SUM_MUTATIONS[name]
    assert src.count(old) == 1, name
    src = src.replace(old, new).replace("from .holo_oracle import DEG, geometry, window_pixels\n", "")
    mod = types.ModuleType("sum_mutant_" + name)
    for k in ("DEG", "geometry", "window_pixels"):
        mod.__dict__[k] = getattr(oracle.holo_oracle, k)
    exec(compile(src, SUM_SRC + ":" + name, "exec"), mod.__dict__)
    for f in ("plane_parameters", "fourier_axes", "fourier_plane", "field_axes", "summarise",
              "batch_summary_fourier", "batch_summary_field"):
        monkeypatch.setattr(oracle, f, getattr(mod, f))
    failed = 0
    for t in [pins.test_summary_gaussian_beam_closed_forms, pins.test_summary_wrapped_centre_of_mass,
              pins.test_summary_uniform_patch_and_zero_plane, pins.test_summary_fourier_plane_of_a_tone,
              pins.test_summary_field_plane_of_a_fundamental_mode,
              pins.test_summary_batch_entry_is_the_summed_intensity]:
        try:
            t()
        except (AssertionError, ValueError, IndexError):
            failed += 1
    assert failed > 0, name
