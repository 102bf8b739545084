"""Plain FP64 oracle of the basis transforms applied after the HG overlap.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the GPU
library imports, links or runs this file.

The paper's "Basis types" section: fields are always decomposed in the HG
basis; an LG or custom basis is obtained from the HG coefficients by one
matrix multiplication, c_out = T c_HG. For a custom basis the user gives T
(modeCountOut x modeCountIn; columns past the plan's HG modes are not used).
For LG the paper names the basis only. Readings taken here:

  LG_{p,l}(r, phi) = sqrt(2 p! / (pi (p + |l|)!)) / w * (sqrt2 r / w)^|l|
                     * L_p^|l|(2 r^2 / w^2) * exp(-r^2 / w^2) * exp(i l phi),
  with phi measured from +x towards +y, the same waist as the HG modes and no
  further phase factor. Group N = 2p + |l| holds the same N + 1 modes as HG
  group N = m + n; inside a group the modes run l = N, N - 2, ..., -N.
  T[k][j] = <LG_k | HG_j> (the overlap integral), so that the LG coefficient
  of a field is the sum over HG modes of T times its HG coefficient.

The overlap is evaluated by Gauss-Hermite quadrature: both functions are a
polynomial times exp(-(x^2 + y^2) / w^2), so with x = w s / sqrt2 the
integrand is a polynomial times exp(-s^2 - t^2), which a rule of G + 4
nodes per axis integrates exactly (up to rounding). The Laguerre polynomials
come from scipy, the Gauss-Hermite rule from numpy. For large G (up to the
100 groups the paper names for LG) the transform is taken one mode group at
a time (lg_blocks): the full matrix is pinned block diagonal at small G.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .holo_oracle import hermite_gauss_1d, mode_list


def lg_modes(group_count: int):
    """(p, l) of every LG mode of groups 0 .. G-1, in basis order."""
    out = []
    for n in range(group_count):
        for l in range(n, -n - 1, -2):
            out.append(((n - abs(l)) // 2, l))
    return out


def lg_function(p: int, l: int, x: np.ndarray, y: np.ndarray, waist: float) -> np.ndarray:
    """LG_{p,l} at the points (x, y) (arrays of one shape), unit L2 norm."""
    r2 = (x * x + y * y) / (waist * waist)
    phi = np.arctan2(y, x)
    c = math.sqrt(2.0 * math.factorial(p) / (math.pi * math.factorial(p + abs(l)))) / waist
    rad = (2.0 * r2) ** (abs(l) / 2.0) * special.eval_genlaguerre(p, abs(l), 2.0 * r2) * np.exp(-r2)
    return c * rad * np.exp(1j * l * phi)


def _overlaps(lg_pl, hg_mn, nodes: int) -> np.ndarray:
    """<LG_k | HG_j> for the LG modes lg_pl [(p, l)] (rows) and the HG modes
    hg_mn [(m, n)] (columns), by Gauss-Hermite quadrature with `nodes` nodes
    per axis, at w = 1 (the transform does not depend on the waist: both
    bases scale with it)."""
    w = 1.0
    s, wt = np.polynomial.hermite.hermgauss(nodes)
    x = w * s / math.sqrt(2.0)                    # nodes along each axis
    u = hermite_gauss_1d(max(max(m, n) for m, n in hg_mn) + 1, x, w)     # [n][node]
    xx, yy = np.meshgrid(x, x, indexing="xy")     # [y node][x node]
    # integral f exp(-s^2 - t^2) ds dt ~ sum wt_a wt_b f; f = product * exp(s^2 + t^2)
    ww = np.outer(wt, wt) * np.exp(np.add.outer(s * s, s * s)) * (w * w / 2.0)
    hg = np.array([np.outer(u[n], u[m]).ravel() for m, n in hg_mn])      # [y][x]: u_n(y) u_m(x)
    lg = np.array([lg_function(p, l, xx, yy, w).ravel() for p, l in lg_pl])
    return np.conj(lg) @ (ww.ravel() * hg).T


def hg_to_lg(group_count: int) -> np.ndarray:
    """T (M x M, complex): c_LG = T c_HG, T[k][j] = <LG_k | HG_j>, every LG
    mode against every HG mode (the definition; practical for G up to ~20).
    A rule of G + 4 nodes integrates every product of two modes of groups
    below G exactly (a polynomial of degree < 2G times the Gaussian)."""
    return _overlaps(lg_modes(group_count), mode_list(group_count), group_count + 4)


def lg_blocks(group_count: int) -> list:
    """The transform for large G, one block per mode group: block N is the
    (N+1) x (N+1) matrix <LG_k | HG_j> over the LG and HG modes of group N,
    in basis order, with the same quadrature rule as hg_to_lg. An LG mode of
    group N = 2p + |l| has no overlap with HG modes of other groups (both are
    a polynomial of total degree N times the same Gaussian, and the HG modes
    of a group span exactly the degree-N part), so T is block diagonal."""
    lg, hg = lg_modes(group_count), mode_list(group_count)
    out, start = [], 0
    for n in range(group_count):
        out.append(_overlaps(lg[start:start + n + 1], hg[start:start + n + 1], group_count + 4))
        start += n + 1
    return out


def apply_lg_blocks(coefs: np.ndarray, blocks: list) -> np.ndarray:
    """coefs [..., pol, M] HG -> LG [..., pol, M], each group by its block."""
    c = np.asarray(coefs, dtype=np.complex128)
    out = np.zeros_like(c)
    start = 0
    for b in blocks:
        k = b.shape[0]
        out[..., start:start + k] = np.einsum("km,...m->...k", b, c[..., start:start + k])
        start += k
    return out


def custom_transform(matrix: np.ndarray, modes: int) -> np.ndarray:
    """A user's modeCountOut x modeCountIn matrix cut or zero-padded to the
    plan's `modes` HG columns (columns past them are not used)."""
    t = np.asarray(matrix, dtype=np.complex128)
    out = np.zeros((t.shape[0], modes), dtype=np.complex128)
    k = min(modes, t.shape[1])
    out[:, :k] = t[:, :k]
    return out


def apply_basis(coefs: np.ndarray, t: np.ndarray) -> np.ndarray:
    """coefs [..., pol, M] HG -> [..., pol, M_out], each pol on its own."""
    return np.einsum("km,...m->...k", np.asarray(t, dtype=np.complex128), np.asarray(coefs, dtype=np.complex128))
