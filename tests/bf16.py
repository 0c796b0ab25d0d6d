"""Test-side model of the BF16 cost mode: the rounding of its inputs and the
error bound of its FP32 arithmetic.

Rounding: each coordinate goes FP64 -> FP32 (nearest even) -> BF16 (nearest
even on the top 16 bits of the FP32 word).

Bound: with x, y already rounded, the products x_k y_k and squares x_k^2 are
exact in FP32 (8-bit significands), so the only errors are the FP32 sums
of d terms and the three final operations; for a cell
    |C_fp32 - C_exact| <= gamma_(d+3) * (|x|^2 + |y|^2 + 2 sum_k |x_k y_k|)
                        <= gamma_(d+3) * 2 (|x|^2 + |y|^2),
gamma_m = m u / (1 - m u), u = 2^-24 (clamping at 0 only moves the value
toward the exact, non-negative C).  The transportation LP optimum moves by at
most the largest cell change (the plan has total mass 1), so the same bound,
maximised over the pair's cells, covers D^2.
"""
import numpy as np

U32 = 2.0 ** -24
U16 = 2.0 ** -8          # BF16 unit roundoff (8 significand bits)


def round_bf16(a) -> np.ndarray:
    """FP64 values rounded as the device rounds them, returned as FP64."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x40, r).astype(np.uint32)
    return (r << 16).view(np.float32).astype(np.float64).reshape(np.shape(a))


def gamma(m: int) -> float:
    return m * U32 / (1.0 - m * U32)


def cell_bound(x, y) -> np.ndarray:
    """Bound on |C_bf16 - C_exact(rounded)| for every cell of a pair."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    nx = (x * x).sum(1); ny = (y * y).sum(1)
    return gamma(x.shape[1] + 3) * 2.0 * (nx[:, None] + ny[None, :])


def input_rounding_bound(x, y) -> np.ndarray:
    """Bound on |C_exact(rounded) - C_exact(original)| per cell: with
    e = (U16 + 2 U32)(|x| + |y|) bounding |x~ - x| + |y~ - y|,
    | |x~-y~|^2 - |x-y|^2 | <= e (2 |x-y| + e)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    e = (U16 + 2 * U32) * (np.linalg.norm(x, axis=1)[:, None] + np.linalg.norm(y, axis=1)[None, :])
    dist = np.sqrt(((x[:, None] - y[None]) ** 2).sum(-1))
    return e * (2.0 * dist + e)


def rounded_set(S):
    """The ragged set with every coordinate rounded to BF16 (weights kept)."""
    import synth
    return synth.RaggedSet(S.offsets.copy(), round_bf16(S.points), S.weights.astype(np.float64))
