"""CPU checks of the test-side BF16 model (tests/bf16.py): its rounding
against torch's own float32 -> bfloat16 conversion (nearest even), a few
hand-worked ties, and its error bounds against a direct FP32 evaluation."""
import numpy as np
import pytest

from tests.bf16 import U16, cell_bound, input_rounding_bound, round_bf16

torch = pytest.importorskip("torch")


def test_round_matches_torch_bfloat16():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, -3.0e38, 1e-40, np.inf, -np.inf]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = round_bf16(a)
    assert np.array_equal(got, ref)
    assert np.isnan(round_bf16(np.array([np.nan]))[0])


def test_round_ties_to_even():
    # spacing of BF16 just above 1 is 2^-7
    assert round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0               # tie, even is 1
    assert round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6   # tie, even is 1+2^-6
    assert round_bf16(np.array([1 + 2 ** -8 + 2 ** -20]))[0] == 1 + 2 ** -7
    assert round_bf16(np.array([255.0]))[0] == 255.0                    # small integers exact
    assert round_bf16(np.array([257.0]))[0] == 256.0


def test_cell_bound_covers_fp32_evaluation():
    rng = np.random.default_rng(6)
    for d in (8, 128, 200):
        x = round_bf16(rng.normal(size=(17, d)) * 3)
        y = round_bf16(rng.normal(size=(11, d)) * 3 + 1)
        exact = ((x[:, None] - y[None]) ** 2).sum(-1)
        x32, y32 = x.astype(np.float32), y.astype(np.float32)
        c32 = ((x32 * x32).sum(1)[:, None] + (y32 * y32).sum(1)[None]
               - np.float32(2) * (x32 @ y32.T)).astype(np.float64)
        assert np.all(np.abs(np.maximum(c32, 0) - exact) <= cell_bound(x, y))


def test_input_rounding_bound():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(9, 64)) * 5
    y = rng.normal(size=(13, 64)) * 5 - 2
    c = ((x[:, None] - y[None]) ** 2).sum(-1)
    xr, yr = round_bf16(x), round_bf16(y)
    cr = ((xr[:, None] - yr[None]) ** 2).sum(-1)
    b = input_rounding_bound(x, y)
    assert np.all(np.abs(cr - c) <= b)
    assert np.all(np.abs(xr - x) <= (U16 + 2 ** -23) * np.abs(x))
