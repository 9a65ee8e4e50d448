"""The oracle's pins catch plausible mistakes.

Each case copies oracle/oracle.c, plants one mistake (a transposed operand,
a dropped term, a wrong sign, an off-by-one), builds the copy on the CPU and
runs a compact set of the same pins as test_oracle.py against it.  Every
mutant must fail at least one pin, and the unmodified source must pass all
of them.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "apply_transposed_S": ("num += phiq[c] * Sh[c * d + e];", "num += phiq[c] * Sh[e * d + c];"),
    "apply_no_division": ("orow[e] = num / den;", "orow[e] = num;"),
    "summary_z_counts_tokens": ("zh[c] += p;", "zh[c] += 1.0;"),
    "summary_skips_first_key": ("for (int64_t j = 0; j < N; ++j) {\n        for (int64_t e = 0; e < d; ++e) vrow[e] = elem(&v",
                                "for (int64_t j = 1; j < N; ++j) {\n        for (int64_t e = 0; e < d; ++e) vrow[e] = elem(&v"),
    "phi_drops_one": ("return x > 0.0 ? x + 1.0 : exp(x); }", "return x > 0.0 ? x : exp(x); }"),
    "phi_negated_exponent": ("return x > 0.0 ? x + 1.0 : exp(x); }", "return x > 0.0 ? x + 1.0 : exp(-x); }"),
    "dphi_zero_slope": ("return x > 0.0 ? 1.0 : exp(x); }", "return x > 0.0 ? 0.0 : exp(x); }"),
    "dden_sign": ("dden[i] = -go / den;", "dden[i] = go / den;"),
    "dq_drops_z_term": ("acc += dden[i] * z[c];", ""),
    "dk_drops_dz_term": ("acc += dz[c];", ""),
    "dv_transposed_dS": ("acc += phik[c] * dS[c * d + e];", "acc += phik[c] * dS[e * d + c];"),
    "dq_uses_phi_not_dphi": ("dq[i * d + c] = acc * oracle_dphi(", "dq[i * d + c] = acc * oracle_phi("),
    "dS_uses_raw_gradient": ("dS[c * d + e] += p * dnum[i * d + e];",
                             "dS[c * d + e] += p * elem(g, b, h, i, e);"),
}

GATE_MUTANTS = {
    "gate_weights_swapped": ("out[i] = g * a[i] + (1.0 - g) * elem(&other, b, h, n, c);",
                             "out[i] = (1.0 - g) * a[i] + g * elem(&other, b, h, n, c);"),
    "gate_in_variance": ("return sigma_data / (sigma_data + sigma);",
                         "return sigma_data * sigma_data / (sigma_data * sigma_data + sigma * sigma);"),
    "gate_wrong_batch": ("const double g = oracle_noise_gate(sigma[b], sigma_data);",
                         "const double g = oracle_noise_gate(sigma[0], sigma_data);"),
    "mix_drops_other": ("out[i] = g * a[i] + (1.0 - g) * elem(&other, b, h, n, c);",
                        "out[i] = g * a[i];"),
}

TILE_MUTANTS = {
    "hann_not_squared": ("  return sn * sn;", "  return sn;"),
    "hann_no_half_offset": ("((double)u + 0.5)", "((double)u)"),
    "blend_not_normalised": ("    for (int64_t c = 0; c < C; ++c) out[p * C + c] /= wsum[p];",
                             "    for (int64_t c = 0; c < C; ++c) out[p * C + c] /= 1.0;"),
    "blend_ignores_halo_offset": ("          const int64_t gx = j * core[2] - halo[2] + ux;",
                                  "          const int64_t gx = j * core[2] + ux;"),
    "extract_wrong_row": ("          const int64_t gy = clamp64(i * core[1] - halo[1] + uy, 0, dims[1] - 1);",
                          "          const int64_t gy = clamp64(i * core[1] + uy, 0, dims[1] - 1);"),
}


def phi_np(x):
    return np.where(x > 0, x + 1.0, np.exp(np.minimum(x, 0.0)))


def _pins():
    """Return the names of the pins that fail for the loaded oracle."""
    failed = []
    rng = np.random.default_rng(7)
    q, k, v, g = (rng.standard_normal((1, 2, 40, 4)) for _ in range(4))
    A = np.einsum("bhic,bhjc->bhij", phi_np(q), phi_np(k))
    ref = np.einsum("bhij,bhje->bhie", A, v) / A.sum(-1, keepdims=True)
    o = oracle.forward(q, k, v)
    if not np.allclose(o, ref, rtol=1e-12, atol=1e-12):
        failed.append("quadratic_form")
    dq, dk, dv = oracle.backward(q, k, v, g)
    for name, x, grad in (("q", q, dq), ("k", k, dk), ("v", v, dv)):
        fd = np.empty_like(x)
        for idx in np.ndindex(x.shape):
            x0 = x[idx]
            h = 1e-6 * max(1.0, abs(x0))
            x[idx] = x0 + h
            lp = (oracle.forward(q, k, v) * g).sum()
            x[idx] = x0 - h
            lm = (oracle.forward(q, k, v) * g).sum()
            x[idx] = x0
            fd[idx] = (lp - lm) / (2 * h)
        if not np.allclose(grad, fd, rtol=1e-5, atol=1e-7):
            failed.append("fd_" + name)
    if not np.allclose(dv.sum(2), g.sum(2), rtol=1e-11, atol=1e-11):
        failed.append("dv_column_sums")
    return failed


def _tile_pins():
    """Names of the tile-operation pins that fail for the loaded oracle."""
    import math
    failed = []
    a, b = (2 - math.sqrt(2)) / 4, (2 + math.sqrt(2)) / 4
    tiles = np.array([10.0, 20, 30, 40, 50, 60, 70, 80]).reshape(2, 1, 1, 4, 1)
    out = oracle.tile_blend(tiles, (1, 1, 4), (1, 1, 2), (0, 0, 1)).ravel()
    expect = [20.0, (b * 30 + a * 50) / (a + b), (a * 40 + b * 60) / (a + b), 70.0]
    if not np.allclose(out, expect, rtol=1e-14):
        failed.append("hand_example")
    x = np.random.default_rng(3).standard_normal((2, 5, 7, 2))
    for core, halo in (((1, 2, 3), (1, 1, 2)), ((2, 3, 2), (0, 2, 1))):
        t = oracle.tile_extract(x, core, halo)
        if not np.allclose(oracle.tile_blend(t, x.shape[:3], core, halo), x, atol=1e-13):
            failed.append("round_trip")
    one = oracle.tile_extract(x, (2, 5, 7), (0, 1, 1))
    if not np.array_equal(one[0, :, 1:6, 1:8], x):
        failed.append("extract_inner")
    return failed


def _build(tmp_path, text, name):
    src = tmp_path / (name + ".c")
    src.write_text(text)
    so = tmp_path / ("lib" + name + ".so")
    inc = os.path.dirname(SRC)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-I", inc,
                    "-o", str(so), str(src), "-lm"], check=True)
    return str(so)


def _with_library(path):
    prev = oracle.use_library(path)
    try:
        return _pins()
    finally:
        oracle.restore_library(prev)


def test_unmodified_oracle_passes_compact_pins(tmp_path):
    so = _build(tmp_path, open(SRC).read(), "pristine")
    assert _with_library(so) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not unique: " + name
    so = _build(tmp_path, text.replace(old, new), name)
    failed = _with_library(so)
    assert failed, "no pin caught the planted mistake " + name


def _with_tile_library(path):
    prev = oracle.use_library(path)
    try:
        return _tile_pins()
    finally:
        oracle.restore_library(prev)


def test_unmodified_oracle_passes_tile_pins(tmp_path):
    so = _build(tmp_path, open(SRC).read(), "pristine_tiles")
    assert _with_tile_library(so) == []


@pytest.mark.parametrize("name", sorted(TILE_MUTANTS))
def test_planted_tile_mistake_is_caught(tmp_path, name):
    old, new = TILE_MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not unique: " + name
    so = _build(tmp_path, text.replace(old, new), name)
    assert _with_tile_library(so), "no pin caught the planted mistake " + name


def _gate_pins():
    """Names of the noise-gate pins that fail for the loaded oracle."""
    import math
    failed = []
    special = pytest.importorskip("scipy.special")
    for s in (0.01, 0.3, 2.0, 40.0):
        if abs(oracle.noise_gate(s, 0.5) - special.expit(math.log(0.5 / s))) > 1e-15:
            failed.append("logistic")
            break
    rng = np.random.default_rng(11)
    a = rng.standard_normal((3, 1, 5, 4))
    other = rng.standard_normal((3, 1, 5, 4))
    out = oracle.gated_mix(a, other, [0.0, 0.5, math.inf], 0.5)
    if not (np.array_equal(out[0], a[0]) and np.allclose(out[1], 0.5 * (a[1] + other[1]), rtol=1e-15)
            and np.array_equal(out[2], other[2])):
        failed.append("fixed_points")
    return failed


def _with_gate_library(path):
    prev = oracle.use_library(path)
    try:
        return _gate_pins()
    finally:
        oracle.restore_library(prev)


def test_unmodified_oracle_passes_gate_pins(tmp_path):
    so = _build(tmp_path, open(SRC).read(), "pristine_gate")
    assert _with_gate_library(so) == []


@pytest.mark.parametrize("name", sorted(GATE_MUTANTS))
def test_planted_gate_mistake_is_caught(tmp_path, name):
    old, new = GATE_MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site not unique: " + name
    so = _build(tmp_path, text.replace(old, new), name)
    assert _with_gate_library(so), "no pin caught the planted mistake " + name
