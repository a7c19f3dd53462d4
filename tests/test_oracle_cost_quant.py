"""Pins of the cost model (numbers printed in the paper) and of the low-precision storage rules."""
import json
import os

import numpy as np
import pytest

from oracle import cost, quant

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_per_site_cost():
    g = json.load(open(os.path.join(GOLDEN, "paper_cost_model.json")))
    flops, nbytes = cost.paper_site_cost(naik=False)
    assert flops == g["per_site_flops"]
    assert nbytes == g["per_site_bytes"]


def test_paper_even_sweep_28cubed_96():
    g = json.load(open(os.path.join(GOLDEN, "paper_cost_model.json")))
    flops, nbytes = cost.paper_even_sweep(tuple(g["lattice"]), naik=False)
    assert round(flops / 1e9, 1) == g["even_sweep_flops_printed"] / 1e9      # 0.607e9 -> "0.6 billion"
    assert round(nbytes / 2**30, 1) == g["even_sweep_bytes_printed"] / 1e9    # 1.554 GiB -> "1.6 giga"
    assert nbytes == 1_669_054_464


def test_compulsory_bytes():
    assert cost.compulsory_bytes_per_site("f64", 1) == 2400
    assert cost.compulsory_bytes_per_site("f32", 1) == 1200
    assert cost.compulsory_bytes_per_site("f16", 1) == 616
    assert cost.compulsory_bytes_per_site("f16", 8) == 584 + 32 * 8
    assert cost.flops_per_site(True, 1) == 1146
    assert cost.cg_iteration_bytes_per_site("f64") == 5232


def test_f32_rounding_is_round_to_nearest_even():
    z = np.array([1 + 2 ** -24 + 0j, 1 + 3 * 2 ** -25 + 1j * (1 + 2 ** -25)])
    r = quant.to_f32(z)
    assert r[0].real == 1.0                      # tie at 1 + 2^-24 goes to even (1.0)
    assert r[1].real == 1 + 2 ** -23             # 1 + 1.5 ulp rounds up
    assert r[1].imag == 1.0                      # 1 + 0.5 ulp tie goes to even


def test_f16_spinor_codes_are_nearest_and_bounded():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((2000, 3)) + 1j * rng.standard_normal((2000, 3))
    v[5] = 0.0                                  # an all-zero site keeps zero codes
    codes, s = quant.quantize_spinor_f16(v)
    back = quant.dequantize_spinor_f16(codes, s)
    reals = np.stack([v.real, v.imag], -1).reshape(-1, 6)
    assert np.all(s == np.abs(reals).max(-1).astype(np.float32))
    assert not codes[5].any() and s[5] == 0
    # brute force: each code is the binary16 nearest to the binary32 quotient
    q32 = (reals / np.where(s[:, None] > 0, s[:, None].astype(np.float64), 1)).astype(np.float32)
    lo = np.nextafter(codes, np.float16(-np.inf)).astype(np.float32)
    hi = np.nextafter(codes, np.float16(np.inf)).astype(np.float32)
    c32 = codes.astype(np.float32)
    assert np.all(np.abs(q32 - c32) <= np.abs(q32 - lo)) and np.all(np.abs(q32 - c32) <= np.abs(q32 - hi))
    # error bound per component: half a binary16 spacing at magnitude <= 1 of the scale (+ binary32 slack)
    err = np.abs(np.stack([(back - v).real, (back - v).imag], -1).reshape(-1, 6))
    assert np.all(err <= (2.0 ** -12 + 2.0 ** -23) * s[:, None] * 1.0000001)


def test_f16_exact_values_roundtrip():
    v = np.array([[0.5 + 0.25j, -1.0 + 0.0j, 0.125 - 0.75j]])
    np.testing.assert_array_equal(quant.spinor_f16_roundtrip(v), v)


def test_f16_link_group():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((10, 8, 3, 3)) + 1j * rng.standard_normal((10, 8, 3, 3))
    codes, s = quant.quantize_link_group_f16(U)
    back = quant.dequantize_link_group_f16(codes, s)
    assert codes.shape == (10, 8, 3, 3, 2) and s.shape == (10,)
    rel = np.abs(back - U).max(axis=(1, 2, 3)) / s
    assert np.all(rel <= 2.0 ** -11)
